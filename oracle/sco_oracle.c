/*
 * sco_oracle.c -- plain, serial, FP64 CPU oracle of one stochastic-cutoff (SCO) step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls this
 * file: only tests/, the smoke check and the CPU-baseline leg of bench.py use it.  It
 * shares no code, header, table or constant generator with the HIP library.
 *
 * What it computes (paper: "Parallelized Stochastic Cutoff Method for Long-Range
 * Interacting Systems", Endo, Toga & Sasaki):
 *   - the model: Ising spins s_i = +-1 perpendicular to a 2-D square lattice, i.e.
 *     Eq. (6) with every spin along z so that the (S.r)(S.r) term vanishes:
 *         H = -J sum_<ij> s_i s_j + sum_{i<j} J_ij s_i s_j,  J_ij = D / r_ij^3
 *     (open lattice), or J_ij summed over the periodic images |n_x|,|n_y| <= n_images;
 *   - step (A) / Fig. 1 step (1): stochastic potential switching of every dipolar
 *     bond, Eqs. (1)-(3), with V^max = kappa * J_ij (kappa >= 1);
 *   - Fig. 1 step (2): vertex colouring of the surviving-bond graph (united with the
 *     never-switched nearest-neighbour exchange bonds) by Kuhn-Wattenhofer colour
 *     reduction, each level run as basic colour reduction with the locally-maximal
 *     rule (2)' of Sec. 2.3.2, in synchronous (Jacobi) rounds, Sec. 2.3.1 / 2.3.3;
 *   - step (B) / Fig. 1 step (3): n_sw Metropolis sweeps of the switched
 *     Hamiltonian H' of Eq. (4), colour by colour;
 *   - the observables E (full H), M and the graph statistics of Sec. 3.2.
 *
 * Readings where the paper is silent (full list in the design notes):
 *   - candidate bonds are generated per owner site by a Poisson process over the
 *     cumulative bound rate (geometric skipping), then thinned by (1-P_ij)/pbar_ij;
 *   - kappa == 1 makes a surviving bond "hard" (pseudo-interaction +inf for the
 *     parallel state): both of its spins are frozen for the rest of the step;
 *   - the initial N-colouring of KW is the row-major site index; the new colour of
 *     a recoloured vertex is the smallest colour unused by its same-group neighbours;
 *   - all randomness is Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) keyed by
 *     (seed, chain_id) with counter (step, site, draw, tag).
 *
 * Compiled with -O2 -ffp-contract=off: every floating-point expression is evaluated
 * exactly as written, in the order written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- parameters */
typedef struct {
  int32_t L, periodic, n_images, n_sw;
  double J, D, T, kappa;
  uint32_t seed, chain_id;
  /* colouring of Fig. 1 step (2): 0 KW with rule (2)' on the union graph; 1 the
   * checkerboard product 2 c + ((x + y) mod 2), c a KW colouring of the bonds alone;
   * 2 basic colour reduction with rule (2)' on the whole union graph, no KW groups */
  int32_t coloring;
  /* 0: Ising spins perpendicular to the plane; 1: classical Heisenberg spins with the
   * full dipolar tensor of Eq. (6) (open lattices, V^max = 2 D / r^3 per pair) */
  int32_t model;
} orc_params;

typedef struct {
  double E, E_exchange, E_dipolar;
  int64_t M, n_edges;
  int32_t delta_union, q, colors_used, kw_levels;
  int64_t kw_rounds, accepted, attempts, near_ties;
  int32_t delta_sco, pad; /* maximum degree of the switched graph alone */
  double m_phi;           /* Eq. (7) before the average and modulus (Heisenberg; 0 for Ising) */
} orc_obs;

enum { TAG_INIT = 1, TAG_SW = 2, TAG_TH = 3, TAG_MC = 4, TAG_HP = 5, TAG_HA = 6 };

/* ---------------------------------------------------------------- Philox4x32-10
 * Salmon et al. (SC'11), Sec. 3.2: ten rounds of two 32x32->64 multiplications
 * with a Weyl-sequence key schedule. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform on (0,1): the top 52 bits of (hi:lo) as an integer k, u = (k + 1/2) 2^-52.
 * Every value is exact, the smallest is 2^-53 and the largest 1 - 2^-53. */
double orc_u52(uint32_t lo, uint32_t hi) {
  uint64_t w = ((uint64_t)hi << 32) | (uint64_t)lo;
  double k = (double)(w >> 12);
  return (k + 0.5) * 0x1p-52;
}

static void draw(const orc_params* p, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag,
                 uint32_t out[4]) {
  uint32_t ctr[4] = {c0, c1, c2, tag};
  uint32_t key[2] = {p->seed, p->chain_id};
  orc_philox(ctr, key, out);
}

/* A point uniform on the unit sphere by Marsaglia's method (Ann. Math. Stat. 43, 645
 * (1972)): x1, x2 uniform in (-1, 1) until q = x1^2 + x2^2 < 1, then
 * (2 x1 sqrt(1-q), 2 x2 sqrt(1-q), 1 - 2q).  Try k uses Philox(c0, c1, c2, tag + 256 k);
 * after 64 rejected tries there is no point (returns 0).  Only a square root is
 * involved, so every evaluation that rounds correctly gives the same bits. */
static int sphere_point(const orc_params* p, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag, double out[3]) {
  for (uint32_t k = 0; k < 64; ++k) {
    uint32_t w[4];
    draw(p, c0, c1, c2, tag + (k << 8), w);
    double x1 = 2.0 * orc_u52(w[0], w[1]) - 1.0;
    double x2 = 2.0 * orc_u52(w[2], w[3]) - 1.0;
    double q = x1 * x1 + x2 * x2;
    if (q < 1.0) {
      double t = sqrt(1.0 - q);
      out[0] = 2.0 * x1 * t;
      out[1] = 2.0 * x2 * t;
      out[2] = 1.0 - 2.0 * q;
      return 1;
    }
  }
  return 0;
}

/* Dipolar pair energy of Eq. (6) for in-plane displacement (dx, dy):
 * V = (D / r^3) [S_i . S_j - 3 (S_i . r)(S_j . r) / r^2], with D / r^3 = J_m / 2. */
static double pair_energy(const double* si, const double* sj, int dx, int dy, double Jm) {
  double dot = si[0] * sj[0] + si[1] * sj[1] + si[2] * sj[2];
  double pi = si[0] * (double)dx + si[1] * (double)dy;
  double pj = sj[0] * (double)dx + sj[1] * (double)dy;
  double r2 = (double)dx * (double)dx + (double)dy * (double)dy;
  return (Jm * 0.5) * (dot - 3.0 * (pi * pj) / r2);
}

/* ---------------------------------------------------------------- chain state */
typedef struct {
  orc_params p;
  int L, N, K, hard;
  double beta, inv_rate;
  /* half-displacement table, sorted by (r^2, dy, dx) */
  int32_t *hdx, *hdy;
  double *Jm, *Cm, *theta, *delta;
  int8_t* s;
  double* s3;   /* Heisenberg spins, (x, y, z) per site */
  double* hden; /* Heisenberg: expm1(-2 beta J_m), J_m = V^max of the pair */
  /* switched-bond graph (both directions), rows ascending by neighbour */
  int64_t n_edges, cap;
  int32_t *sv_owner, *sv_nb, *sv_m; /* survivors in draw order */
  int32_t *row_ptr, *col, *attr;
  /* colouring */
  int32_t delta_union, q, M;
  int64_t kw_rounds;
  int32_t* kw_rounds_level; /* [64] */
  int32_t* color;
  /* counters */
  int64_t accepted, attempts, near_ties;
  /* the near-tie decisions since the last switching: kind (1 switching, 2 sweep)
   * and site (the owner, or the swept site); the first 256 are kept */
  int32_t tie_kind[256], tie_site[256];
  int32_t n_tie;
} orc_chain;

static void note_tie(orc_chain* c, int kind, int site) {
  c->near_ties++;
  if (c->n_tie < 256) {
    c->tie_kind[c->n_tie] = kind;
    c->tie_site[c->n_tie] = site;
  }
  c->n_tie++;
}

static int cmp_disp(const void* a, const void* b) {
  const int32_t* u = (const int32_t*)a;
  const int32_t* v = (const int32_t*)b;
  int64_t ru = (int64_t)u[0] * u[0] + (int64_t)u[1] * u[1];
  int64_t rv = (int64_t)v[0] * v[0] + (int64_t)v[1] * v[1];
  if (ru != rv) return ru < rv ? -1 : 1;
  if (u[1] != v[1]) return u[1] < v[1] ? -1 : 1;
  if (u[0] != v[0]) return u[0] < v[0] ? -1 : 1;
  return 0;
}

/* Dipolar coupling of one displacement: D / r^3, summed over the periodic images
 * (nx outer, ny inner, both ascending) when the lattice is periodic. */
static double coupling(const orc_params* p, int dx, int dy) {
  if (!p->periodic) {
    double r2 = (double)dx * (double)dx + (double)dy * (double)dy;
    /* Heisenberg: the bound V^max = 2 D / r^3 of the pair (the largest eigenvalue
     * magnitude of the dipolar tensor (D / r^3)(I - 3 rhat rhat)) */
    double Dc = p->model == 1 ? 2.0 * p->D : p->D;
    return Dc / (r2 * sqrt(r2));
  }
  double acc = 0.0;
  int n = p->n_images, L = p->L;
  for (int nx = -n; nx <= n; ++nx)
    for (int ny = -n; ny <= n; ++ny) {
      double X = (double)(dx + nx * L), Y = (double)(dy + ny * L);
      double r2 = X * X + Y * Y;
      if (r2 == 0.0) continue;
      acc += p->D / (r2 * sqrt(r2));
    }
  return acc;
}

/* Partner of owner i through half-displacement m; returns -1 when the pair is not
 * owned by i (outside an open lattice, or the other half of a self-conjugate
 * displacement of a periodic lattice). */
static int partner(const orc_chain* c, int i, int m) {
  int L = c->L, x = i % L, y = i / L, dx = c->hdx[m], dy = c->hdy[m];
  if (c->p.periodic) {
    int h = L / 2;
    if (dy == 0 && dx == h && x >= h) return -1;
    if (dy == h && (dx == 0 || dx == h) && y >= h) return -1;
    int jx = (x + dx + L) % L, jy = (y + dy) % L;
    return jy * L + jx;
  }
  int jx = x + dx, jy = y + dy;
  if (jx < 0 || jx >= L || jy >= L) return -1;
  return jy * L + jx;
}

/* nearest neighbours in the order +x, -x, +y, -y; returns the count */
static int neighbours(const orc_chain* c, int v, int nb[4]) {
  int L = c->L, x = v % L, y = v / L, n = 0;
  if (c->p.periodic) {
    nb[0] = y * L + (x + 1) % L;
    nb[1] = y * L + (x + L - 1) % L;
    nb[2] = ((y + 1) % L) * L + x;
    nb[3] = ((y + L - 1) % L) * L + x;
    return 4;
  }
  if (x + 1 < L) nb[n++] = v + 1;
  if (x > 0) nb[n++] = v - 1;
  if (y + 1 < L) nb[n++] = v + L;
  if (y > 0) nb[n++] = v - L;
  return n;
}

/* The temperature-dependent columns of the table at beta = 1/T. */
static void temperature_columns(orc_chain* c) {
  const orc_params* p = &c->p;
  if (p->model == 1) {
    /* a candidate of the bound rate 2 beta J_m survives with probability
     * (1 - P_ij) / pbar_m, pbar_m = 1 - exp(-2 beta J_m) = -hden_m (Eqs. 1-2) */
    for (int m = 0; m < c->K; ++m) c->hden[m] = expm1(-c->beta * 2.0 * c->Jm[m]);
    return;
  }
  for (int m = 0; m < c->K; ++m) {
    double Jd = c->Jm[m];
    /* Eq. (2) with V = J s_i s_j and V^max = kappa J:
     *   P(parallel) = exp(-beta (kappa-1) J), P(antiparallel) = exp(-beta (kappa+1) J).
     * A candidate (probability 1-P(antiparallel)) survives with probability
     * (1-P)/(1-P(antiparallel)): 1 for antiparallel, theta for parallel. */
    double em = expm1(-c->beta * (p->kappa + 1.0) * Jd);
    double ep = expm1(-c->beta * (p->kappa - 1.0) * Jd);
    c->theta[m] = c->hard ? 0.0 : ep / em;
    /* Eq. (3): Vbar(s) = J s - T log(1 - P(s)); delta = Vbar(+1) - Vbar(-1). */
    c->delta[m] = c->hard ? INFINITY : 2.0 * Jd + p->T * log(em / ep);
  }
}

/* A new temperature for the steps that follow (the cooling protocol of Sec. 3.1):
 * beta, the bound rate and the columns of Eqs. (2)-(3).  Returns -1 for T <= 0. */
int orc_set_temperature(orc_chain* c, double T) {
  if (!(T > 0.0)) return -1;
  c->p.T = T;
  c->beta = 1.0 / T;
  c->inv_rate = T / (c->p.kappa + 1.0);
  temperature_columns(c);
  return 0;
}

void orc_destroy(orc_chain* c) {
  if (!c) return;
  free(c->hdx); free(c->hdy); free(c->Jm); free(c->Cm); free(c->theta); free(c->delta);
  free(c->s); free(c->s3); free(c->hden); free(c->sv_owner); free(c->sv_nb); free(c->sv_m);
  free(c->row_ptr); free(c->col); free(c->attr); free(c->kw_rounds_level); free(c->color);
  free(c);
}

/* Returns NULL on invalid parameters. */
orc_chain* orc_create(const orc_params* p, const int8_t* init_spins) {
  if (p->L < 2 || p->T <= 0.0 || !(p->kappa >= 1.0) || p->n_sw < 0 || p->n_images < 0) return NULL;
  if (p->periodic && (p->L < 4 || (p->L & 1))) return NULL;
  if (p->model != 0 && p->model != 1) return NULL;
  if (p->model == 1 && (p->periodic || p->kappa != 1.0)) return NULL; /* open, V^max = 2 D / r^3 */
  orc_chain* c = (orc_chain*)calloc(1, sizeof(orc_chain));
  c->p = *p;
  c->L = p->L;
  c->N = p->L * p->L;
  c->hard = (p->kappa == 1.0);
  c->beta = 1.0 / p->T;
  c->inv_rate = p->T / (p->kappa + 1.0);
  int L = c->L, N = c->N;

  /* half-displacement set: each unordered pair of sites is reached from exactly one
   * (owner, displacement) combination that passes partner(). */
  int cap = p->periodic ? (L / 2 + 1) * L : 2 * L * L;
  int32_t* d = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)cap);
  int K = 0;
  if (p->periodic) {
    int h = L / 2;
    for (int dy = 0; dy <= h; ++dy)
      for (int dx = -h + 1; dx <= h; ++dx) {
        int keep;
        if (dy > 0 && dy < h) keep = 1;
        else keep = (dx > 0) || (dy == h && dx == 0); /* dy==0: 0<dx<=h ; dy==h: 0<=dx<=h */
        if (!keep) continue;
        d[2 * K] = dx; d[2 * K + 1] = dy; ++K;
      }
  } else {
    for (int dy = 0; dy < L; ++dy)
      for (int dx = -(L - 1); dx < L; ++dx) {
        if (dy == 0 && dx <= 0) continue;
        d[2 * K] = dx; d[2 * K + 1] = dy; ++K;
      }
  }
  qsort(d, (size_t)K, 2 * sizeof(int32_t), cmp_disp);
  c->K = K;
  c->hdx = (int32_t*)malloc(sizeof(int32_t) * K);
  c->hdy = (int32_t*)malloc(sizeof(int32_t) * K);
  c->Jm = (double*)malloc(sizeof(double) * K);
  c->Cm = (double*)malloc(sizeof(double) * K);
  c->theta = (double*)malloc(sizeof(double) * K);
  c->delta = (double*)malloc(sizeof(double) * K);
  c->hden = (double*)malloc(sizeof(double) * K);
  double acc = 0.0;
  for (int m = 0; m < K; ++m) {
    c->hdx[m] = d[2 * m];
    c->hdy[m] = d[2 * m + 1];
    double Jd = coupling(p, c->hdx[m], c->hdy[m]);
    c->Jm[m] = Jd;
    acc += Jd;
    c->Cm[m] = acc;
  }
  free(d);
  temperature_columns(c);

  c->s = (int8_t*)malloc((size_t)N);
  c->s3 = (double*)calloc(3 * (size_t)N, sizeof(double));
  for (int v = 0; v < N; ++v) {
    if (p->model == 1) { /* uniform on the sphere (never rejected in practice) */
      if (!sphere_point(p, 0u, (uint32_t)v, 0u, TAG_INIT, c->s3 + 3 * (size_t)v)) c->s3[3 * (size_t)v + 2] = 1.0;
      c->s[v] = 1;
      continue;
    }
    if (init_spins) { c->s[v] = init_spins[v] > 0 ? 1 : -1; continue; }
    uint32_t w[4];
    draw(p, 0u, (uint32_t)v, 0u, TAG_INIT, w);
    c->s[v] = (w[0] >> 31) ? -1 : 1;
  }
  c->cap = 1024;
  c->sv_owner = (int32_t*)malloc(sizeof(int32_t) * c->cap);
  c->sv_nb = (int32_t*)malloc(sizeof(int32_t) * c->cap);
  c->sv_m = (int32_t*)malloc(sizeof(int32_t) * c->cap);
  c->row_ptr = (int32_t*)calloc((size_t)N + 1, sizeof(int32_t));
  c->col = (int32_t*)malloc(sizeof(int32_t) * 2 * c->cap);
  c->attr = (int32_t*)malloc(sizeof(int32_t) * 2 * c->cap);
  c->kw_rounds_level = (int32_t*)calloc(64, sizeof(int32_t));
  c->color = (int32_t*)calloc((size_t)N, sizeof(int32_t));
  return c;
}

static void push_survivor(orc_chain* c, int i, int j, int m) {
  if (c->n_edges == c->cap) {
    c->cap *= 2;
    c->sv_owner = (int32_t*)realloc(c->sv_owner, sizeof(int32_t) * c->cap);
    c->sv_nb = (int32_t*)realloc(c->sv_nb, sizeof(int32_t) * c->cap);
    c->sv_m = (int32_t*)realloc(c->sv_m, sizeof(int32_t) * c->cap);
    c->col = (int32_t*)realloc(c->col, sizeof(int32_t) * 2 * c->cap);
    c->attr = (int32_t*)realloc(c->attr, sizeof(int32_t) * 2 * c->cap);
  }
  c->sv_owner[c->n_edges] = i;
  c->sv_nb[c->n_edges] = j;
  c->sv_m[c->n_edges] = m;
  c->n_edges++;
}

static int near(double a, double b) { return fabs(a - b) <= 1e-12 * fabs(b); }

/* ------------------------------------------------------------ step (A): switching
 * Every pair (i, i+d_m) is a candidate with probability pbar_m = 1 - exp(-lambda_m),
 * lambda_m = (kappa+1) beta J_m, independently: the candidates of owner i are the
 * intervals (C_{m-1}, C_m] of the cumulative coupling hit by a Poisson process of
 * rate (kappa+1) beta, scanned from the start of the table.  A candidate then
 * survives with probability (1 - P_ij(s)) / pbar_m, which makes the overall
 * survival probability exactly 1 - P_ij as Eq. (1) requires. */
int orc_switch(orc_chain* c, uint64_t t) {
  c->n_edges = 0;
  c->n_tie = 0;
  const double Ctop = c->Cm[c->K - 1];
  for (int i = 0; i < c->N; ++i) {
    int pos = -1, k = 0;
    double Cpos = 0.0;
    for (; pos < c->K - 1; ++k) { /* no candidate lies beyond the last table entry */
      uint32_t w[4];
      draw(&c->p, (uint32_t)t, (uint32_t)i, (uint32_t)(k >> 1), TAG_SW, w);
      double u1 = (k & 1) ? orc_u52(w[2], w[3]) : orc_u52(w[0], w[1]);
      double target = Cpos + (-log(u1)) * c->inv_rate;
      if (near(target, Ctop)) note_tie(c, 1, i);
      if (target > Ctop) break;
      int lo = pos + 1, hi = c->K - 1; /* smallest m > pos with C_m >= target */
      while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if (c->Cm[mid] >= target) hi = mid; else lo = mid + 1;
      }
      int m = lo;
      if (near(target, c->Cm[m]) || (m - 1 > pos && near(target, c->Cm[m - 1]))) note_tie(c, 1, i);
      int j = partner(c, i, m);
      if (j >= 0 && c->p.model == 1) {
        /* Heisenberg: survive with probability (1 - P_ij) / pbar_m, P_ij of Eq. (2)
         * at the current spins */
        uint32_t w2[4];
        draw(&c->p, (uint32_t)t, (uint32_t)i, (uint32_t)k, TAG_TH, w2);
        double u = orc_u52(w2[0], w2[1]);
        double V = pair_energy(c->s3 + 3 * (size_t)i, c->s3 + 3 * (size_t)j, c->hdx[m], c->hdy[m], c->Jm[m]);
        double ratio = expm1(c->beta * (V - c->Jm[m])) / c->hden[m];
        if (fabs(u - ratio) < 1e-12) note_tie(c, 1, i);
        if (u < ratio) push_survivor(c, i, j, m);
      } else if (j >= 0) {
        int keep = (c->s[i] != c->s[j]);
        if (!keep && !c->hard) {
          uint32_t w2[4];
          draw(&c->p, (uint32_t)t, (uint32_t)i, (uint32_t)k, TAG_TH, w2);
          keep = orc_u52(w2[0], w2[1]) < c->theta[m];
        }
        if (keep) push_survivor(c, i, j, m);
      }
      pos = m;
      Cpos = c->Cm[m];
    }
  }
  /* both directions of every surviving bond, rows ascending by neighbour index */
  int N = c->N;
  memset(c->row_ptr, 0, sizeof(int32_t) * ((size_t)N + 1));
  for (int64_t e = 0; e < c->n_edges; ++e) {
    c->row_ptr[c->sv_owner[e] + 1]++;
    c->row_ptr[c->sv_nb[e] + 1]++;
  }
  for (int v = 0; v < N; ++v) c->row_ptr[v + 1] += c->row_ptr[v];
  int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  memcpy(fill, c->row_ptr, sizeof(int32_t) * (size_t)N);
  for (int64_t e = 0; e < c->n_edges; ++e) {
    int a = c->sv_owner[e], b = c->sv_nb[e], m = c->sv_m[e];
    c->col[fill[a]] = b; c->attr[fill[a]] = m; fill[a]++;
    c->col[fill[b]] = a; c->attr[fill[b]] = m; fill[b]++;
  }
  free(fill);
  for (int v = 0; v < N; ++v) { /* insertion sort of each (short) row */
    for (int x = c->row_ptr[v] + 1; x < c->row_ptr[v + 1]; ++x) {
      int32_t kc = c->col[x], ka = c->attr[x];
      int y = x - 1;
      while (y >= c->row_ptr[v] && c->col[y] > kc) {
        c->col[y + 1] = c->col[y]; c->attr[y + 1] = c->attr[y]; --y;
      }
      c->col[y + 1] = kc; c->attr[y + 1] = ka;
    }
  }
  return 0;
}

/* distinct neighbours of v in the union of the exchange lattice (with_nn) and the
 * surviving bonds; returns the count */
static int graph_neighbours(const orc_chain* c, int v, int32_t* out, int cap, int with_nn) {
  int nb[4], n = with_nn ? neighbours(c, v, nb) : 0, cnt = 0;
  for (int a = 0; a < n; ++a) {
    int dup = 0;
    for (int b = 0; b < cnt; ++b) dup |= (out[b] == nb[a]);
    if (!dup && cnt < cap) out[cnt++] = nb[a];
  }
  for (int x = c->row_ptr[v]; x < c->row_ptr[v + 1]; ++x) {
    int dup = 0;
    for (int b = 0; b < cnt; ++b) dup |= (out[b] == c->col[x]);
    if (!dup && cnt < cap) out[cnt++] = c->col[x];
  }
  return cnt;
}

/* ---------------------------------------------------- Fig. 1 step (2): colouring
 * Sec. 2.3.3: level-0 groups of q = Delta+1 consecutive initial colours (initial
 * colour = site index), so vertex v starts in group v/q with colour v mod q inside
 * it.  Level p unites pairs of groups; the upper half (bit p-1 of v/q set) carries
 * colours q..2q-1 and is reduced back into 0..q-1 by colour-reduction rounds
 * (Sec. 2.3.2).  rule 3 is rule (2)': in a round every pending vertex whose colour
 * exceeds the colour of every pending neighbour of its group takes the smallest colour
 * in 0..q-1 that no neighbour of its group holds.  rule 2 is the basic step (2): round
 * r recolours the vertices of colour alpha = 2q - r (alpha runs from 2q-1 down to q,
 * one colour per round).  All decisions of a round read the colours of the previous
 * round (synchronous communication, Sec. 2.3.1).  The graph is the union of the
 * exchange lattice and the bonds (with_nn) or the bonds alone.  Returns -1 when a
 * palette of q colours does not suffice. */
static int kw_reduce(orc_chain* c, int q, int with_nn, int rule, int32_t* cur, int64_t* total_rounds,
                     int32_t* level_rounds, int* levels) {
  int N = c->N;
  int32_t nbuf[4096];
  /* the graph's adjacency, listed once */
  int32_t* uoff = (int32_t*)malloc(sizeof(int32_t) * ((size_t)N + 1));
  size_t ucap = (size_t)N * 4 + 2 * (size_t)c->n_edges + 1, un = 0;
  int32_t* uadj = (int32_t*)malloc(sizeof(int32_t) * ucap);
  for (int v = 0; v < N; ++v) {
    int d = graph_neighbours(c, v, nbuf, 4096, with_nn);
    uoff[v] = (int32_t)un;
    for (int a = 0; a < d; ++a) uadj[un++] = nbuf[a];
  }
  uoff[N] = (int32_t)un;
  int groups = (N + q - 1) / q, M = 0;
  while ((1 << M) < groups) ++M;
  *levels = M;
  *total_rounds = 0;
  uint8_t* pend = (uint8_t*)calloc((size_t)N, 1);
  int32_t* plist = (int32_t*)malloc(sizeof(int32_t) * (size_t)N); /* pending vertices */
  int32_t* dec_v = (int32_t*)malloc(sizeof(int32_t) * (size_t)N); /* decisions of a round */
  int32_t* dec_c = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  uint8_t* used = (uint8_t*)malloc((size_t)q);
  int fail = 0;
  for (int v = 0; v < N; ++v) cur[v] = v % q;
  for (int p = 1; p <= M && !fail; ++p) {
    int npending = 0;
    for (int v = 0; v < N; ++v) {
      pend[v] = (uint8_t)(((v / q) >> (p - 1)) & 1);
      if (pend[v]) { cur[v] += q; plist[npending++] = v; }
    }
    int rounds = 0;
    /* rule (2)' runs until no vertex is pending; rule (2) runs alpha from 2q-1 down to
     * q, one colour per round, whether or not a colour class is empty */
    while (rule == 2 ? rounds < q : npending > 0) {
      ++rounds;
      /* every decision of the round reads the colours and pending marks left by the
       * previous round; they are applied together afterwards */
      int ndec = 0;
      const int alpha = 2 * q - rounds; /* rule (2): the colour recoloured this round */
      for (int k = 0; k < npending; ++k) {
        int v = plist[k];
        int grp = (v / q) >> p;
        int go = 1;
        memset(used, 0, (size_t)q);
        for (int x = uoff[v]; x < uoff[v + 1]; ++x) {
          int u = uadj[x];
          if (((u / q) >> p) != grp) continue;
          if (rule == 3 && pend[u] && cur[u] > cur[v]) go = 0;
          if (cur[u] < q) used[cur[u]] = 1;
        }
        if (rule == 2) go = (cur[v] == alpha);
        if (!go) continue;
        int nc = 0;
        while (nc < q && used[nc]) ++nc;
        if (nc == q) { fail = 1; break; }
        dec_v[ndec] = v;
        dec_c[ndec] = nc;
        ++ndec;
      }
      if (fail) break;
      for (int k = 0; k < ndec; ++k) {
        cur[dec_v[k]] = dec_c[k];
        pend[dec_v[k]] = 0;
      }
      int keep = 0;
      for (int k = 0; k < npending; ++k)
        if (pend[plist[k]]) plist[keep++] = plist[k];
      npending = keep;
    }
    if (npending > 0) fail = 1; /* cannot happen: every pending colour is some alpha */
    level_rounds[p < 64 ? p : 63] = rounds;
    *total_rounds += rounds;
  }
  free(uoff); free(uadj); free(pend); free(plist); free(dec_v); free(dec_c); free(used);
  return fail ? -1 : 0;
}

/* Basic colour reduction on the whole union graph, no KW groups (Sec. 2.3.2): the
 * initial colour is the site index, the vertices with colours q..N-1 are pending, and
 * in every round each pending vertex whose colour exceeds those of all its pending
 * neighbours takes the smallest colour in 0..q-1 that no neighbour holds (rule (2)');
 * rounds read the previous round's colours.  Returns -1 when q colours do not suffice. */
static int bcr_whole(orc_chain* c, int q, int32_t* cur, int64_t* rounds_out) {
  int N = c->N;
  int32_t nbuf[4096];
  int32_t* uoff = (int32_t*)malloc(sizeof(int32_t) * ((size_t)N + 1));
  size_t ucap = (size_t)N * 4 + 2 * (size_t)c->n_edges + 1, un = 0;
  int32_t* uadj = (int32_t*)malloc(sizeof(int32_t) * ucap);
  for (int v = 0; v < N; ++v) {
    int d = graph_neighbours(c, v, nbuf, 4096, 1);
    uoff[v] = (int32_t)un;
    for (int a = 0; a < d; ++a) uadj[un++] = nbuf[a];
  }
  uoff[N] = (int32_t)un;
  int32_t* plist = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  int32_t* dec_v = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  int32_t* dec_c = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  uint8_t* used = (uint8_t*)malloc((size_t)q);
  int npending = 0, fail = 0;
  int64_t rounds = 0;
  for (int v = 0; v < N; ++v) {
    cur[v] = v;
    if (v >= q) plist[npending++] = v;
  }
  while (npending > 0 && !fail) {
    ++rounds;
    int ndec = 0;
    for (int k = 0; k < npending; ++k) {
      int v = plist[k], localmax = 1;
      memset(used, 0, (size_t)q);
      for (int x = uoff[v]; x < uoff[v + 1]; ++x) {
        int u = uadj[x];
        if (cur[u] >= q && cur[u] > cur[v]) localmax = 0;
        if (cur[u] < q) used[cur[u]] = 1;
      }
      if (!localmax) continue;
      int nc = 0;
      while (nc < q && used[nc]) ++nc;
      if (nc == q) { fail = 1; break; }
      dec_v[ndec] = v;
      dec_c[ndec] = nc;
      ++ndec;
    }
    for (int k = 0; k < ndec; ++k) cur[dec_v[k]] = dec_c[k];
    int keep = 0;
    for (int k = 0; k < npending; ++k)
      if (cur[plist[k]] >= q) plist[keep++] = plist[k];
    npending = keep;
  }
  *rounds_out = rounds;
  free(uoff); free(uadj); free(plist); free(dec_v); free(dec_c); free(used);
  return fail ? -1 : 0;
}

/* maximum degree of the union graph (with_nn) or of the bonds alone */
static int max_degree(const orc_chain* c, int with_nn) {
  int32_t nbuf[4096];
  int maxdeg = 0;
  for (int v = 0; v < c->N; ++v) {
    int d = graph_neighbours(c, v, nbuf, 4096, with_nn);
    if (d > maxdeg) maxdeg = d;
  }
  return maxdeg;
}

int orc_color(orc_chain* c) {
  int N = c->N;
  c->delta_union = max_degree(c, 1);
  memset(c->kw_rounds_level, 0, 64 * sizeof(int32_t));
  int rc = 0;
  if (c->p.coloring == 1) {
    /* checkerboard product: a KW colouring c' of the bonds alone with
     * q = max(Delta_bonds + 1, 2), then colour 2 c' + ((x + y) mod 2): bond partners
     * differ in c', lattice neighbours in the parity */
    int q = max_degree(c, 0) + 1;
    if (q < 2) q = 2;
    c->q = q;
    int M = 0;
    rc = kw_reduce(c, q, 0, 3, c->color, &c->kw_rounds, c->kw_rounds_level, &M);
    c->M = M;
    for (int v = 0; v < N; ++v) c->color[v] = 2 * c->color[v] + ((v % c->L + v / c->L) & 1);
  } else if (c->p.coloring == 2) {
    c->q = c->delta_union + 1;
    c->M = 1;
    rc = bcr_whole(c, c->q, c->color, &c->kw_rounds);
    c->kw_rounds_level[1] = (int32_t)c->kw_rounds;
  } else {
    c->q = c->delta_union + 1;
    int M = 0;
    rc = kw_reduce(c, c->q, 1, 3, c->color, &c->kw_rounds, c->kw_rounds_level, &M);
    c->M = M;
  }
  return rc;
}

/* Test helper: the KW colouring of the union graph with the basic step (2) in every
 * level instead of rule (2)' (colours into out[N], rounds into *rounds). */
int orc_color_rule2(orc_chain* c, int32_t* out, int64_t* rounds) {
  int32_t lv[64];
  int M = 0;
  return kw_reduce(c, max_degree(c, 1) + 1, 1, 2, out, rounds, lv, &M);
}

/* Test helper: basic colour reduction with step (2) on the whole union graph from the
 * N-colouring (N - q rounds; small lattices only). */
int orc_color_whole_rule2(orc_chain* c, int32_t* out, int64_t* rounds) {
  int N = c->N, q = max_degree(c, 1) + 1;
  int32_t nbuf[4096];
  uint8_t* used = (uint8_t*)malloc((size_t)q);
  int32_t* nxt = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  int fail = 0;
  for (int v = 0; v < N; ++v) out[v] = v;
  *rounds = 0;
  for (int alpha = N - 1; alpha >= q && !fail; --alpha) { /* one colour per round */
    ++*rounds;
    memcpy(nxt, out, sizeof(int32_t) * (size_t)N);
    for (int v = 0; v < N; ++v) {
      if (out[v] != alpha) continue;
      int d = graph_neighbours(c, v, nbuf, 4096, 1);
      memset(used, 0, (size_t)q);
      for (int a = 0; a < d; ++a)
        if (out[nbuf[a]] < q) used[out[nbuf[a]]] = 1;
      int nc = 0;
      while (nc < q && used[nc]) ++nc;
      if (nc == q) { fail = 1; break; }
      nxt[v] = nc;
    }
    memcpy(out, nxt, sizeof(int32_t) * (size_t)N);
  }
  free(used); free(nxt);
  return fail ? -1 : 0;
}

/* ------------------------------------------------- step (B): Metropolis on H'
 * One MC step is one trial per spin (Sec. 2.1), taken colour by colour.  Flipping
 * s_v changes H' by s_v h_v, h_v = 2J sum_NN s_u - sum_bonds delta_m s_u, where
 * delta_m = Vbar(+1) - Vbar(-1).  With kappa == 1 a bond's parallel state has
 * infinite pseudo-energy, so a spin carrying a surviving bond never flips. */
/* Pseudo-interaction of Eq. (3) for Heisenberg spins: Vbar = V - T log(1 - P),
 * 1 - P = -expm1(beta (V - V^max)); +inf where 1 - P is not positive. */
static double heis_vbar(const orc_chain* c, const double* si, const double* sj, int m) {
  double V = pair_energy(si, sj, c->hdx[m], c->hdy[m], c->Jm[m]);
  double g = -expm1(c->beta * (V - c->Jm[m]));
  return g > 0.0 ? V - c->p.T * log(g) : INFINITY;
}

/* Heisenberg Metropolis on H' (Eq. 4): spin v proposes S' uniform on the sphere
 * (sphere_point with Philox(t, v, s, TAG_HP + 256 k)) and the local energy is
 * -J S.h + sum over its bonds of Vbar, h the sum of its lattice neighbours (+x, -x,
 * +y, -y), the bonds in row order; dE = E(S') - E(S) is accepted when dE <= 0, else
 * when u < exp(-beta dE), u from Philox(t, v, s, TAG_HA). */
static void heis_sweep(orc_chain* c, uint64_t t, int n_sw) {
  int N = c->N;
  const int np = c->p.coloring == 1 ? 2 * c->q : c->q; /* every colour class */
  for (int s = 0; s < n_sw; ++s)
    for (int col = 0; col < np; ++col)
      for (int v = 0; v < N; ++v) {
        if (c->color[v] != col) continue;
        c->attempts++;
        double* S = c->s3 + 3 * (size_t)v;
        double Sn[3];
        if (!sphere_point(&c->p, (uint32_t)t, (uint32_t)v, (uint32_t)s, TAG_HP, Sn)) continue;
        int nb[4], n = neighbours(c, v, nb);
        double h[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < n; ++a)
          for (int k = 0; k < 3; ++k) h[k] += c->s3[3 * (size_t)nb[a] + k];
        double Eold = (-c->p.J) * (S[0] * h[0] + S[1] * h[1] + S[2] * h[2]);
        double Enew = (-c->p.J) * (Sn[0] * h[0] + Sn[1] * h[1] + Sn[2] * h[2]);
        for (int x = c->row_ptr[v]; x < c->row_ptr[v + 1]; ++x) {
          const double* Sj = c->s3 + 3 * (size_t)c->col[x];
          Eold += heis_vbar(c, S, Sj, c->attr[x]);
          Enew += heis_vbar(c, Sn, Sj, c->attr[x]);
        }
        double dE = Enew - Eold;
        int acc = 1;
        if (!(dE <= 0.0)) {
          uint32_t w[4];
          draw(&c->p, (uint32_t)t, (uint32_t)v, (uint32_t)s, TAG_HA, w);
          double u = orc_u52(w[0], w[1]);
          double pr = exp(-c->beta * dE);
          if (fabs(u - pr) < 1e-12) note_tie(c, 2, v);
          acc = u < pr;
        }
        if (acc) {
          S[0] = Sn[0]; S[1] = Sn[1]; S[2] = Sn[2];
          c->accepted++;
        }
      }
}

int orc_sweep(orc_chain* c, uint64_t t, int n_sw) {
  if (c->p.model == 1) {
    heis_sweep(c, t, n_sw);
    return 0;
  }
  int N = c->N;
  /* every colour class of the palette: q colours, 2 q for the checkerboard product */
  const int np = c->p.coloring == 1 ? 2 * c->q : c->q;
  for (int s = 0; s < n_sw; ++s)
    for (int col = 0; col < np; ++col)
      for (int v = 0; v < N; ++v) {
        if (c->color[v] != col) continue;
        c->attempts++;
        int b0 = c->row_ptr[v], b1 = c->row_ptr[v + 1];
        if (c->hard && b1 > b0) continue;
        int nb[4], n = neighbours(c, v, nb), nn = 0;
        for (int a = 0; a < n; ++a) nn += c->s[nb[a]];
        double h = (2.0 * c->p.J) * (double)nn;
        for (int x = b0; x < b1; ++x) {
          double dm = c->delta[c->attr[x]];
          h = c->s[c->col[x]] > 0 ? h - dm : h + dm;
        }
        double dE = c->s[v] > 0 ? h : -h;
        int acc = 1;
        if (dE > 0.0) {
          uint32_t w[4];
          draw(&c->p, (uint32_t)t, (uint32_t)v, (uint32_t)s, TAG_MC, w);
          double u = orc_u52(w[0], w[1]);
          double pr = exp(-c->beta * dE);
          if (fabs(u - pr) < 1e-12) note_tie(c, 2, v);
          acc = u < pr;
        }
        if (acc) { c->s[v] = (int8_t)-c->s[v]; c->accepted++; }
      }
  return 0;
}

int orc_step(orc_chain* c, uint64_t t) {
  if (orc_switch(c, t)) return -1;
  if (orc_color(c)) return -1;
  return orc_sweep(c, t, c->p.n_sw);
}

/* ------------------------------------------------------------- observables
 * E = -J sum_<ij> s_i s_j + sum_{i<j} J_ij s_i s_j, the second sum taken pair by
 * pair through the owner rule (O(N K): used for small lattices; the Python layer
 * evaluates the same sum from FFT autocorrelations for large ones). */
/* Heisenberg: E_exchange = -J sum over (+x, +y) lattice pairs of S_i . S_j (sites
 * ascending), E_dipolar = sum over m of (sum over owners i ascending of V(S_i, S_i+d_m)),
 * and Eq. (7) before the average: (1/N) sum_i [S_i x (r_i - r_c) / |r_i - r_c|]_z with
 * r_c the centre of the lattice ((L-1)/2, (L-1)/2) (a site at the centre adds 0). */
static void heis_observables(orc_chain* c, orc_obs* o, int with_dipolar) {
  int N = c->N, L = c->L;
  double ex = 0.0, mphi = 0.0;
  for (int v = 0; v < N; ++v) {
    int x = v % L, y = v / L;
    const double* S = c->s3 + 3 * (size_t)v;
    if (x + 1 < L) {
      const double* R = S + 3;
      ex += S[0] * R[0] + S[1] * R[1] + S[2] * R[2];
    }
    if (y + 1 < L) {
      const double* U = S + 3 * (size_t)L;
      ex += S[0] * U[0] + S[1] * U[1] + S[2] * U[2];
    }
    double rx = (double)x - 0.5 * (double)(L - 1), ry = (double)y - 0.5 * (double)(L - 1);
    double d = sqrt(rx * rx + ry * ry);
    if (d > 0.0) mphi += (S[0] * ry - S[1] * rx) / d;
  }
  double Edip = 0.0;
  if (with_dipolar)
    for (int m = 0; m < c->K; ++m) {
      double em = 0.0;
      for (int i = 0; i < N; ++i) {
        int j = partner(c, i, m);
        if (j >= 0) em += pair_energy(c->s3 + 3 * (size_t)i, c->s3 + 3 * (size_t)j, c->hdx[m], c->hdy[m], c->Jm[m]);
      }
      Edip += em;
    }
  o->E_exchange = -c->p.J * ex;
  o->E_dipolar = Edip;
  o->E = o->E_exchange + Edip;
  o->M = 0;
  o->m_phi = mphi / (double)N;
}

void orc_observables(orc_chain* c, orc_obs* o, int with_dipolar) {
  int N = c->N;
  int64_t M = 0, ex = 0;
  o->m_phi = 0.0;
  for (int v = 0; v < N; ++v) {
    M += c->s[v];
    int L = c->L, x = v % L, y = v / L;
    if (c->p.periodic) {
      ex += c->s[v] * c->s[y * L + (x + 1) % L];
      ex += c->s[v] * c->s[((y + 1) % L) * L + x];
    } else {
      if (x + 1 < L) ex += c->s[v] * c->s[v + 1];
      if (y + 1 < L) ex += c->s[v] * c->s[v + L];
    }
  }
  double Edip = 0.0;
  if (with_dipolar && c->p.model == 0) {
    for (int m = 0; m < c->K; ++m) {
      int64_t cm = 0;
      for (int i = 0; i < N; ++i) {
        int j = partner(c, i, m);
        if (j >= 0) cm += c->s[i] * c->s[j];
      }
      Edip += c->Jm[m] * (double)cm;
    }
  }
  int colors_used = 0;
  if (c->q > 0) {
    /* the palette: q colours, 2 q for the checkerboard product */
    const int np = c->p.coloring == 1 ? 2 * c->q : c->q;
    uint8_t* seen = (uint8_t*)calloc((size_t)np, 1);
    for (int v = 0; v < N; ++v) if (c->color[v] >= 0 && c->color[v] < np) seen[c->color[v]] = 1;
    for (int a = 0; a < np; ++a) colors_used += seen[a];
    free(seen);
  }
  o->E_exchange = -c->p.J * (double)ex;
  o->E_dipolar = Edip;
  o->E = o->E_exchange + Edip;
  o->M = M;
  if (c->p.model == 1) heis_observables(c, o, with_dipolar);
  o->n_edges = c->n_edges;
  o->delta_union = c->delta_union;
  o->q = c->q;
  o->colors_used = colors_used;
  o->kw_levels = c->M;
  o->kw_rounds = c->kw_rounds;
  o->accepted = c->accepted;
  o->attempts = c->attempts;
  o->near_ties = c->near_ties;
  int dmax = 0;
  for (int v = 0; v < N; ++v)
    if (c->row_ptr[v + 1] - c->row_ptr[v] > dmax) dmax = c->row_ptr[v + 1] - c->row_ptr[v];
  o->delta_sco = dmax;
  o->pad = 0;
}

/* ----------------------------------------------------------- accessors */
int orc_N(const orc_chain* c) { return c->N; }
int orc_K(const orc_chain* c) { return c->K; }
int64_t orc_n_edges(const orc_chain* c) { return c->n_edges; }
void orc_get_spins(const orc_chain* c, int8_t* out) { memcpy(out, c->s, (size_t)c->N); }
void orc_set_spins(orc_chain* c, const int8_t* in) {
  for (int v = 0; v < c->N; ++v) c->s[v] = in[v] > 0 ? 1 : -1;
}
void orc_get_tables(const orc_chain* c, int32_t* dx, int32_t* dy, double* J, double* C,
                    double* theta, double* delta) {
  size_t K = (size_t)c->K;
  if (dx) memcpy(dx, c->hdx, K * sizeof(int32_t));
  if (dy) memcpy(dy, c->hdy, K * sizeof(int32_t));
  if (J) memcpy(J, c->Jm, K * sizeof(double));
  if (C) memcpy(C, c->Cm, K * sizeof(double));
  if (theta) memcpy(theta, c->theta, K * sizeof(double));
  if (delta) memcpy(delta, c->delta, K * sizeof(double));
}
/* survivors in draw order (owner ascending, then draw order) */
void orc_get_survivors(const orc_chain* c, int32_t* owner, int32_t* nb, int32_t* m) {
  size_t E = (size_t)c->n_edges;
  memcpy(owner, c->sv_owner, E * sizeof(int32_t));
  memcpy(nb, c->sv_nb, E * sizeof(int32_t));
  memcpy(m, c->sv_m, E * sizeof(int32_t));
}
void orc_get_csr(const orc_chain* c, int32_t* row_ptr, int32_t* col, int32_t* attr) {
  memcpy(row_ptr, c->row_ptr, ((size_t)c->N + 1) * sizeof(int32_t));
  memcpy(col, c->col, 2 * (size_t)c->n_edges * sizeof(int32_t));
  memcpy(attr, c->attr, 2 * (size_t)c->n_edges * sizeof(int32_t));
}
void orc_get_colors(const orc_chain* c, int32_t* out) { memcpy(out, c->color, (size_t)c->N * sizeof(int32_t)); }
void orc_get_kw_rounds(const orc_chain* c, int32_t* out64) { memcpy(out64, c->kw_rounds_level, 64 * sizeof(int32_t)); }
int orc_partner(const orc_chain* c, int i, int m) { return partner(c, i, m); }
void orc_get_spins3(const orc_chain* c, double* out) { memcpy(out, c->s3, 3 * (size_t)c->N * sizeof(double)); }
void orc_set_spins3(orc_chain* c, const double* in) { memcpy(c->s3, in, 3 * (size_t)c->N * sizeof(double)); }
double orc_pair_energy(const double* si, const double* sj, int dx, int dy, double Jm) {
  return pair_energy(si, sj, dx, dy, Jm);
}
int orc_sphere_point(const orc_chain* c, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag, double* out) {
  return sphere_point(&c->p, c0, c1, c2, tag, out);
}
void orc_reset_counters(orc_chain* c) { c->accepted = c->attempts = c->near_ties = 0; }

/* The near-tie decisions since the last switching into kinds[] and sites[] (up to
 * cap, at most 256 kept); returns how many there were. */
int orc_ties(const orc_chain* c, int32_t* kinds, int32_t* sites, int cap) {
  int n = c->n_tie < 256 ? c->n_tie : 256;
  for (int k = 0; k < n && k < cap; ++k) {
    kinds[k] = c->tie_kind[k];
    sites[k] = c->tie_site[k];
  }
  return c->n_tie;
}

/* Per-pair survival counts over n_steps switching passes with the spins held fixed
 * (statistical test helper): counts[i*K + m] += 1 for every survivor (i, m). */
void orc_survival_counts(orc_chain* c, uint64_t t0, int n_steps, int32_t* counts) {
  for (int s = 0; s < n_steps; ++s) {
    orc_switch(c, t0 + (uint64_t)s);
    for (int64_t e = 0; e < c->n_edges; ++e)
      counts[(size_t)c->sv_owner[e] * (size_t)c->K + (size_t)c->sv_m[e]]++;
  }
}

/* Runs n_steps SCO steps from step t0 and records (E, M) after every thin-th step,
 * E recomputed from its definition (small lattices only).  Returns the next step
 * index. */
uint64_t orc_run_record(orc_chain* c, uint64_t t0, int n_steps, int thin, double* E_out,
                        int64_t* M_out) {
  uint64_t t = t0;
  int rec = 0;
  for (int s = 0; s < n_steps; ++s, ++t) {
    orc_step(c, t);
    if (thin > 0 && (s + 1) % thin == 0) {
      orc_obs o;
      orc_observables(c, &o, 1);
      E_out[rec] = o.E;
      M_out[rec] = o.M;
      ++rec;
    }
  }
  return t;
}
