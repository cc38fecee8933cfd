// sco_kernels.hip -- gfx950 kernels of the stochastic-cutoff (SCO) step.
//
// One SCO step (Endo, Toga & Sasaki, Sec. 2.1-2.3, Fig. 1):
//   k_switch            step (1): switch every dipolar bond (Eqs. 1-3) by geometric
//                       skipping over the cumulative coupling + thinning; survivors are
//                       appended with one atomic per wavefront (ballot count)
//   k_scan_*            exclusive prefix sums (row offsets, colour-class offsets)
//   k_scatter, k_rowsort both directions of every survivor into a CSR, rows ascending
//   k_kw                step (2): Kuhn-Wattenhofer colour reduction, Sec. 2.3.3
//   k_bucket_*          stable counting sort of the sites by colour
//   k_sweep             step (3): Metropolis on H' (Eq. 4), one colour class at a time
// The kernels that iterate over dependent phases (k_kw, k_sweep) are persistent and
// separate the phases with a device-wide barrier whose waits are bounded: a wait that
// runs out raises SCO_FLAG_TIMEOUT and every wave then leaves the kernel.
//
// Floating point: FP64 with contraction disabled (-ffp-contract=off); every decision
// that the CPU reference also takes is evaluated with the same operations in the
// same order.  Only exp/log of the device math library can differ from the host's
// in the last bit.
#include <hip/hip_runtime.h>

#include "sco_internal.h"

namespace {

constexpr int kBlock = 256;  // == SCO_CHUNK: a block of per-site threads is one chunk

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror & Shaw (SC'11): ten rounds of S-box free multiply/xor with
// the Weyl key schedule (0x9E3779B9, 0xBB67AE85) and multipliers 0xD2511F53,
// 0xCD9E8D57.
struct W4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ W4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return W4{c0, c1, c2, c3};
}

// (0,1) uniform from the top 52 bits of hi:lo, at the midpoints (k + 1/2) 2^-52.
__device__ __forceinline__ double unit52(uint32_t lo, uint32_t hi) {
  const uint64_t w = (static_cast<uint64_t>(hi) << 32) | lo;
  return (static_cast<double>(w >> 12) + 0.5) * 0x1p-52;
}

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int64_t gtid() {
  return static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// exact floor(v / d) for 0 <= v < 2^31, 1 <= d < 2^15, via a double reciprocal:
// (v + 1/2) / d is at least 1/(2d) away from an integer, far above the rounding error.
__device__ __forceinline__ int fdiv(int v, double inv_d) {
  return static_cast<int>((static_cast<double>(v) + 0.5) * inv_d);
}

__device__ __forceinline__ void set_flag(SyncWords* s, uint32_t f) {
  __hip_atomic_fetch_or(&s->flags, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-wide barrier for a grid whose blocks are all resident (cooperative launch).
// Returns false once any block has raised a flag that ends the kernel.
constexpr uint32_t kSpinLimit = 1u << 22;  // ~ seconds; reached only if residency fails

__device__ bool grid_barrier(SyncWords* s) {
  __shared__ uint32_t s_ok;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t nb = gridDim.x;
    const uint32_t gen = __hip_atomic_load(&s->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t arrived =
        __hip_atomic_fetch_add(&s->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (arrived == nb) {
      __hip_atomic_store(&s->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&s->bar_gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t n = 0;
      while (__hip_atomic_load(&s->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(&s->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & SCO_FLAG_TIMEOUT)
          break;
        if (++n > kSpinLimit) {
          set_flag(s, SCO_FLAG_TIMEOUT);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    s_ok = (__hip_atomic_load(&s->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
            SCO_FLAG_TIMEOUT) == 0;
  }
  __syncthreads();
  __threadfence();
  return s_ok != 0;
}

// Sum over a block of kBlock threads (all threads must call).
template <typename T>
__device__ T block_sum(T v) {
  __shared__ T red[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  T t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) t += red[i];
  return t;  // valid in thread 0
}

__device__ __forceinline__ int block_max(int v) {
  __shared__ int red[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  int t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) t = max(t, red[i]);
  return t;
}

// partner of owner (x, y) through half-displacement (dx, dy); -1 when not owned
__device__ __forceinline__ int partner_of(int x, int y, int dx, int dy, int L, int periodic) {
  if (periodic) {
    const int h = L >> 1;
    if (dy == 0 && dx == h && x >= h) return -1;
    if (dy == h && (dx == 0 || dx == h) && y >= h) return -1;
    int jx = x + dx;
    jx += (jx < 0) ? L : 0;
    jx -= (jx >= L) ? L : 0;
    int jy = y + dy;
    jy -= (jy >= L) ? L : 0;
    return jy * L + jx;
  }
  const int jx = x + dx, jy = y + dy;
  if (jx < 0 || jx >= L || jy >= L) return -1;
  return jy * L + jx;
}

// nearest neighbours (+x, -x, +y, -y); returns the count (open lattices: 2..4)
__device__ __forceinline__ int nn_sites(int x, int y, int L, int periodic, int nb[4]) {
  const int v = y * L + x;
  if (periodic) {
    nb[0] = y * L + (x + 1 == L ? 0 : x + 1);
    nb[1] = y * L + (x == 0 ? L - 1 : x - 1);
    nb[2] = (y + 1 == L ? 0 : y + 1) * L + x;
    nb[3] = (y == 0 ? L - 1 : y - 1) * L + x;
    return 4;
  }
  int n = 0;
  if (x + 1 < L) nb[n++] = v + 1;
  if (x > 0) nb[n++] = v - 1;
  if (y + 1 < L) nb[n++] = v + L;
  if (y > 0) nb[n++] = v - L;
  return n;
}

}  // namespace

// =================================================================== tables
// J(d_m) = D / r^3, summed over the images nx, ny in [-n, n] (nx outer, ny inner,
// ascending) on a periodic lattice.
extern "C" __global__ void k_table_j(const uint32_t* __restrict__ hd, int K, int L, int periodic,
                                     int n_images, double D, double* __restrict__ J) {
  const int64_t m = gtid();
  if (m >= K) return;
  const uint32_t p = hd[m];
  const int dx = static_cast<int16_t>(p & 0xFFFFu), dy = static_cast<int16_t>(p >> 16);
  if (!periodic) {
    const double r2 = static_cast<double>(dx) * static_cast<double>(dx) +
                      static_cast<double>(dy) * static_cast<double>(dy);
    J[m] = D / (r2 * sqrt(r2));
    return;
  }
  double acc = 0.0;
  for (int nx = -n_images; nx <= n_images; ++nx)
    for (int ny = -n_images; ny <= n_images; ++ny) {
      const double X = static_cast<double>(dx + nx * L), Y = static_cast<double>(dy + ny * L);
      const double r2 = X * X + Y * Y;
      if (r2 == 0.0) continue;
      acc += D / (r2 * sqrt(r2));
    }
  J[m] = acc;
}

// =================================================================== spins
// Initial spins: sign bit of word 0 of Philox(0, v, 0, INIT), or the caller's spins
// (concatenated without padding in chain order, src_base[c] = first index of chain c).
extern "C" __global__ void __launch_bounds__(kBlock)
    k_init_spins(const ChainDesc* __restrict__ cd, const int32_t* __restrict__ chunk_chain,
                 const int64_t* __restrict__ src_base, const int8_t* __restrict__ src,
                 int8_t* __restrict__ spin, int64_t G) {
  const int64_t g = gtid();
  if (g >= G) return;
  const int c = chunk_chain[g >> SCO_CHUNK_SHIFT];
  const ChainDesc& d = cd[c];
  const int v = static_cast<int>(g - d.vbase);
  if (v >= d.N) {
    spin[g] = 1;
    return;
  }
  if (src) {
    spin[g] = src[src_base[c] + v] > 0 ? int8_t(1) : int8_t(-1);
    return;
  }
  const W4 r = philox10(0u, static_cast<uint32_t>(v), 0u, SCO_TAG_INIT, d.seed, d.chain_id);
  spin[g] = (r.x >> 31) ? int8_t(-1) : int8_t(1);
}



// ------------------------------------------------------------------ scan (3 phases)
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;

__device__ void scan_partials(const int32_t* __restrict__ in, int64_t n, int32_t* __restrict__ part) {
  const int64_t nt = (n + kTile - 1) / kTile;
  for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const int64_t base = t * kTile;
    int32_t s = 0;
    for (int i = 0; i < kItems; ++i) {
      const int64_t idx = base + static_cast<int64_t>(i) * kBlock + threadIdx.x;
      if (idx < n) s += in[idx];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[t] = s;
  }
}

// block 0 only: exclusive scan of part[0..nt) in place, part[nt] = total
__device__ void scan_top(int32_t* __restrict__ part, int64_t n) {
  if (blockIdx.x != 0) return;
  const int nt = static_cast<int>((n + kTile - 1) / kTile);
  __shared__ int32_t sums[kBlock];
  const int per = (nt + kBlock - 1) / kBlock;
  const int b0 = threadIdx.x * per;
  int32_t s = 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nt) s += part[b0 + i];
  sums[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    const int32_t t = threadIdx.x >= static_cast<uint32_t>(o) ? sums[threadIdx.x - o] : 0;
    __syncthreads();
    sums[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = threadIdx.x ? sums[threadIdx.x - 1] : 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nt) {
      const int32_t t = part[b0 + i];
      part[b0 + i] = run;
      run += t;
    }
  if (threadIdx.x == kBlock - 1) part[nt] = sums[kBlock - 1];
  __syncthreads();
}

// out[i] = exclusive prefix (out may alias in); out[n] = total
__device__ void scan_final(const int32_t* in, int64_t n, const int32_t* __restrict__ part,
                           int32_t* out) {
  __shared__ int32_t wsum[kBlock / 64];
  const int64_t nt = (n + kTile - 1) / kTile;
  for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const int64_t base = t * kTile + static_cast<int64_t>(threadIdx.x) * kItems;
    int32_t vals[kItems];
    int32_t s = 0;
    for (int i = 0; i < kItems; ++i) {
      const int64_t idx = base + i;
      vals[i] = idx < n ? in[idx] : 0;
      s += vals[i];
    }
    int32_t incl = s;
    const uint32_t lane = lane_id();
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t x = __shfl_up(incl, o);
      if (lane >= static_cast<uint32_t>(o)) incl += x;
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int32_t woff = 0;
    for (int i = 0; i < w; ++i) woff += wsum[i];
    int32_t run = part[t] + woff + incl - s;
    for (int i = 0; i < kItems; ++i) {
      const int64_t idx = base + i;
      if (idx < n) out[idx] = run;
      run += vals[i];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = part[nt];
}

// ------------------------------------------------------------------ step (1)
// One thread per owner site.  Candidate bonds of owner v: the table intervals
// (C_{m-1}, C_m] hit by a Poisson process of rate (kappa+1) beta run from C = 0,
// found by drawing exponential gaps E = -log(u) and locating C_pos + E T/(kappa+1)
// in the cumulative table (guide-table bracket, then binary search).  A candidate
// survives if its spins are antiparallel or, when kappa > 1, with probability
// theta_m if they are parallel.  Draw k of owner v is half k&1 of
// Philox(step, v, k>>1, SW); the thinning draw of candidate k is Philox(step, v, k, TH).
__device__ void phase_switch(const StepArgs& a) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kBlock; base < a.G; base += stride) {
    const int64_t g = base + threadIdx.x;  // a whole block is one chunk: one chain
    const ChainDesc& d = a.cd[a.chunk_chain[base >> SCO_CHUNK_SHIFT]];
    const int v = static_cast<int>(g - d.vbase);
    bool active = v < d.N;
    const int L = d.L;
    const int y = active ? fdiv(v, 1.0 / L) : 0, x = v - y * L;
    const int8_t si = active ? a.spin[g] : int8_t(0);
    const double* __restrict__ C = d.C;
    const double C_top = d.C_top, inv_rate = d.inv_rate, ginv = d.guide_inv;
    const int K = d.K, NB = d.nguide;
    int pos = -1;
    double Cpos = 0.0;
    uint32_t k = 0;
    W4 r{0, 0, 0, 0};
    while (true) {
      bool found = false;
      int j = -1, m = 0;
      active = active && pos < K - 1;  // no candidate lies beyond the last table entry
      if (active) {
        if ((k & 1u) == 0)
          r = philox10(a.step, static_cast<uint32_t>(v), k >> 1, SCO_TAG_SW, d.seed, d.chain_id);
        const double u1 = (k & 1u) ? unit52(r.z, r.w) : unit52(r.x, r.y);
        const double target = Cpos + (-log(u1)) * inv_rate;
        if (target > C_top) {
          active = false;
        } else {
          int b = static_cast<int>(target * ginv);
          b = b < 0 ? 0 : (b > NB ? NB : b);
          int lo = d.guide[b > 0 ? b - 1 : 0];
          int hi = (b + 2 <= NB) ? d.guide[b + 2] : K - 1;
          lo = lo > pos + 1 ? lo : pos + 1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (C[mid] >= target) hi = mid;
            else lo = mid + 1;
          }
          m = lo;
          const uint32_t p = d.hd[m];
          const int dx = static_cast<int16_t>(p & 0xFFFFu), dy = static_cast<int16_t>(p >> 16);
          j = partner_of(x, y, dx, dy, L, d.periodic);
          if (j >= 0) {
            found = si != a.spin[d.vbase + j];
            if (!found && !d.hard) {
              const W4 t = philox10(a.step, static_cast<uint32_t>(v), k, SCO_TAG_TH, d.seed, d.chain_id);
              found = unit52(t.x, t.y) < d.theta[m];
            }
          }
          pos = m;
          Cpos = C[m];
          ++k;
        }
      }
      // wavefront-aggregated append: one atomic per wave and draw round
      const uint64_t mask = __ballot(found);
      if (mask) {
        const uint32_t lane = lane_id();
        const int leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
        uint32_t eb = 0;
        if (static_cast<int>(lane) == leader)
          eb = atomicAdd(&a.sync->edge_count, static_cast<uint32_t>(__popcll(mask)));
        eb = __shfl(eb, leader);
        if (found) {
          const uint32_t e = eb + static_cast<uint32_t>(__popcll(mask & ((1ull << lane) - 1ull)));
          if (e < a.cap_und) {
            const int32_t gj = static_cast<int32_t>(d.vbase + j);
            a.ea[e] = static_cast<int32_t>(g);
            a.eb[e] = gj;
            a.em[e] = m;
            atomicAdd(&a.deg[g], 1);
            atomicAdd(&a.deg[gj], 1);
          } else {
            set_flag(a.sync, SCO_FLAG_OVERFLOW);
          }
        }
      }
      if (__ballot(active) == 0) break;
    }
  }
}

__device__ void phase_scatter(const StepArgs& a) {
  const uint32_t ne = min(a.sync->edge_count, a.cap_und);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; e < ne; e += stride) {
    const int32_t u = a.ea[e], w = a.eb[e], m = a.em[e];
    const int32_t pu = a.row_ptr[u] + atomicAdd(&a.fill[u], 1);
    a.col[pu] = w;
    a.attr[pu] = m;
    const int32_t pw = a.row_ptr[w] + atomicAdd(&a.fill[w], 1);
    a.col[pw] = u;
    a.attr[pw] = m;
  }
}

// Sorts each row ascending by neighbour; union degree |CSR(v) u NN(v)|; Delta and
// directed bond count per chain.  Block-stride over chunks (one chain each).
__device__ void phase_rowsort(const StepArgs& a) {
  for (int ch = blockIdx.x; ch < a.nchunks; ch += gridDim.x) {
    const int c = a.chunk_chain[ch];
    const ChainDesc& d = a.cd[c];
    const int64_t g = (static_cast<int64_t>(ch) << SCO_CHUNK_SHIFT) + threadIdx.x;
    const int v = static_cast<int>(g - d.vbase);
    int udeg = 0, rowlen = 0;
    if (v < d.N) {
      const int r0 = a.row_ptr[g], r1 = a.row_ptr[g + 1];
      rowlen = r1 - r0;
      int32_t* __restrict__ col = a.col;
      int32_t* __restrict__ attr = a.attr;
      for (int q = r0 + 1; q < r1; ++q) {
        const int32_t kc = col[q], ka = attr[q];
        int b = q - 1;
        while (b >= r0 && col[b] > kc) {
          col[b + 1] = col[b];
          attr[b + 1] = attr[b];
          --b;
        }
        col[b + 1] = kc;
        attr[b + 1] = ka;
      }
      const int y = fdiv(v, 1.0 / d.L), x = v - y * d.L;
      int nb[4];
      const int n = nn_sites(x, y, d.L, d.periodic, nb);
      udeg = rowlen;
      for (int q = 0; q < n; ++q) {
        const int32_t gu = static_cast<int32_t>(d.vbase + nb[q]);
        bool dup = false;
        for (int b = r0; b < r1; ++b) dup |= (col[b] == gu);
        udeg += dup ? 0 : 1;
      }
    }
    const int mx = block_max(udeg);
    const int tot = block_sum(rowlen);
    if (threadIdx.x == 0) {
      atomicMax(&a.st[c].delta_union, mx);
      atomicAdd(&a.st[c].n_edges, static_cast<uint32_t>(tot));  // directed count
    }
  }
}

// ------------------------------------------------------------------ step (2)
__device__ void phase_kw_setup(const StepArgs& a) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  uint32_t qmax = 0, mmax = 0;
  for (int c = 0; c < a.n_chains; ++c) {
    int q = a.st[c].delta_union + 1;
    if (q > SCO_MAXQ) {
      set_flag(a.sync, SCO_FLAG_PALETTE);
      q = SCO_MAXQ;
    }
    const int N = a.cd[c].N;
    const int groups = (N + q - 1) / q;
    int M = 0;
    while ((1 << M) < groups) ++M;
    a.st[c].q = q;
    a.st[c].M = M;
    for (int p = 0; p < SCO_MAXLEVEL; ++p) a.st[c].kw_rounds[p] = 0;
    qmax = max(qmax, static_cast<uint32_t>(q));
    mmax = max(mmax, static_cast<uint32_t>(M));
  }
  a.sync->qmax = qmax;
  a.sync->mmax = mmax;
}

// Kuhn-Wattenhofer colour reduction (Sec. 2.3.3).  Level 0: site v of a chain with
// palette q is in group v/q with colour v mod q.  Level p unites pairs of groups; the
// upper half (bit p-1 of v/q set) is pending and is recoloured into 0..q-1 by rule
// (2)' of Sec. 2.3.2 in synchronous rounds.  The rounds are evaluated in an
// equivalent order: a pending vertex decides exactly when every pending same-group
// neighbour with a larger colour has decided (it is then a local maximum) and it
// sees their new colours, so treating the pending vertices colour class by colour
// class, largest first, yields the same colours.  The round in which v decides is
// rho(v) = 1 + max rho over those larger neighbours; a level takes max rho rounds.
//
// Block b owns the global sites [b*S, (b+1)*S) and keeps its pending sites of the
// level bucketed by colour in plist; grid barriers separate the colour classes.
__device__ bool phase_kw(const StepArgs& a) {
  __shared__ int32_t hist[SCO_MAXQ];
  __shared__ int32_t boff[SCO_MAXQ + 1];
  const int64_t S = ((a.G + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
  const int64_t r0 = min(static_cast<int64_t>(blockIdx.x) * S, a.G);
  const int64_t r1 = min(r0 + S, a.G);
  const int qmax = static_cast<int>(a.sync->qmax);
  const int mmax = static_cast<int>(a.sync->mmax);

  for (int64_t g = r0 + threadIdx.x; g < r1; g += kBlock) {
    const int c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
    const int v = static_cast<int>(g - a.cd[c].vbase);
    if (v >= a.cd[c].N) continue;
    const int q = a.st[c].q;
    const int grp = fdiv(v, 1.0 / q);
    a.g0[g] = grp;
    a.color[g] = static_cast<uint16_t>(v - grp * q);
  }
  if (!grid_barrier(a.sync)) return false;

  for (int p = 1; p <= mmax; ++p) {
    for (int i = threadIdx.x; i < qmax; i += kBlock) hist[i] = 0;
    __syncthreads();
    for (int64_t g = r0 + threadIdx.x; g < r1; g += kBlock) {
      const int c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
      if (static_cast<int>(g - a.cd[c].vbase) >= a.cd[c].N || p > a.st[c].M) continue;
      if ((a.g0[g] >> (p - 1)) & 1) {
        atomicAdd(&hist[a.color[g]], 1);
        a.rho[g] = 0;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t s = 0;
      for (int i = 0; i < qmax; ++i) {
        boff[i] = s;
        s += hist[i];
      }
      boff[qmax] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < qmax; i += kBlock) hist[i] = 0;
    __syncthreads();
    for (int64_t g = r0 + threadIdx.x; g < r1; g += kBlock) {
      const int c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
      if (static_cast<int>(g - a.cd[c].vbase) >= a.cd[c].N || p > a.st[c].M) continue;
      if ((a.g0[g] >> (p - 1)) & 1) {
        const int cc = a.color[g];
        a.plist[r0 + boff[cc] + atomicAdd(&hist[cc], 1)] = static_cast<int32_t>(g);
      }
    }
    if (!grid_barrier(a.sync)) return false;

    for (int cc = qmax - 1; cc >= 0; --cc) {
      for (int i = boff[cc] + threadIdx.x; i < boff[cc + 1]; i += kBlock) {
        const int32_t g = a.plist[r0 + i];
        const int c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
        const ChainDesc& d = a.cd[c];
        const int q = a.st[c].q;
        const int v = static_cast<int>(g - d.vbase);
        const int grp = a.g0[g] >> p;
        const int y = fdiv(v, 1.0 / d.L), x = v - y * d.L;
        int nb[4];
        const int n = nn_sites(x, y, d.L, d.periodic, nb);
        uint64_t taken[4] = {0, 0, 0, 0};
        int rmax = 0;
        const int q0 = a.row_ptr[g], q1 = a.row_ptr[g + 1];
        for (int t = 0; t < n + (q1 - q0); ++t) {
          const int32_t gu = t < n ? static_cast<int32_t>(d.vbase + nb[t]) : a.col[q0 + t - n];
          const int gg = a.g0[gu];
          if ((gg >> p) != grp) continue;  // another group at this level
          if ((gg >> (p - 1)) & 1) {       // pending at this level
            const int ru = a.rho[gu];
            if (ru == 0) continue;         // undecided: a smaller colour, not a constraint
            rmax = max(rmax, ru);
          }
          const int cu = a.color[gu];
          taken[cu >> 6] |= 1ull << (cu & 63);
        }
        int nc = 0;
        while (nc < q && ((taken[nc >> 6] >> (nc & 63)) & 1ull)) ++nc;
        if (nc >= q) {
          set_flag(a.sync, SCO_FLAG_PALETTE);
          nc = q - 1;
        }
        a.color[g] = static_cast<uint16_t>(nc);
        a.rho[g] = static_cast<uint16_t>(rmax + 1);
      }
      if (!grid_barrier(a.sync)) return false;
    }
    // rounds of this level: max rho per chain (S is a multiple of kBlock, so the
    // trip count is uniform and each wave covers 64 sites of one chunk)
    for (int64_t g = r0 + threadIdx.x; g < r0 + S; g += kBlock) {
      int rr = 0;
      int c = 0;
      if (g < r1) {
        c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
        if (static_cast<int>(g - a.cd[c].vbase) < a.cd[c].N && p <= a.st[c].M &&
            ((a.g0[g] >> (p - 1)) & 1))
          rr = a.rho[g];
      }
      for (int o = 32; o > 0; o >>= 1) rr = max(rr, __shfl_xor(rr, o));
      if ((threadIdx.x & 63) == 0 && rr > 0) atomicMax(&a.st[c].kw_rounds[p], rr);
    }
  }
  return true;
}

// Per chunk: histogram of colours -> hist[k * nchunks + chunk] (colour-major, so an
// exclusive scan of the whole array gives every (colour, chunk) its first position in
// one colour-major site list covering all chains).
__device__ void phase_bucket_hist(const StepArgs& a, int qmax) {
  __shared__ int32_t h[SCO_MAXQ];
  for (int ch = blockIdx.x; ch < a.nchunks; ch += gridDim.x) {
    for (int i = threadIdx.x; i < qmax; i += kBlock) h[i] = 0;
    __syncthreads();
    const int c = a.chunk_chain[ch];
    const int64_t g = (static_cast<int64_t>(ch) << SCO_CHUNK_SHIFT) + threadIdx.x;
    if (static_cast<int>(g - a.cd[c].vbase) < a.cd[c].N) atomicAdd(&h[a.color[g]], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < qmax; i += kBlock)
      a.hist[static_cast<int64_t>(i) * a.nchunks + ch] = h[i];
    __syncthreads();
  }
}

// stable scatter: rank among the equal colours of the chunk from wave ballots
__device__ void phase_bucket_scatter(const StepArgs& a, int qmax) {
  __shared__ int32_t wcount[kBlock / 64][SCO_MAXQ];
  for (int ch = blockIdx.x; ch < a.nchunks; ch += gridDim.x) {
    const int c = a.chunk_chain[ch];
    const int64_t g = (static_cast<int64_t>(ch) << SCO_CHUNK_SHIFT) + threadIdx.x;
    const bool ok = static_cast<int>(g - a.cd[c].vbase) < a.cd[c].N;
    const int my = ok ? a.color[g] : -1;
    const uint32_t lane = lane_id();
    const int w = threadIdx.x >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    int rank = 0;
    for (int k = 0; k < qmax; ++k) {
      const uint64_t mask = __ballot(my == k);
      if (lane == 0) wcount[w][k] = __popcll(mask);
      if (my == k) rank = __popcll(mask & lt);
    }
    __syncthreads();
    if (ok) {
      for (int i = 0; i < w; ++i) rank += wcount[i][my];
      a.perm[a.hist[static_cast<int64_t>(my) * a.nchunks + ch] + rank] = static_cast<int32_t>(g);
    }
    __syncthreads();
  }
}

// colour classes holding at least one site, per chain (from the scanned histogram)
__device__ void phase_colors_used(const StepArgs& a, int qmax) {
  for (int c = blockIdx.x; c < a.n_chains; c += gridDim.x) {
    const int ch0 = static_cast<int>(a.cd[c].vbase >> SCO_CHUNK_SHIFT);
    const int ch1 = ch0 + (a.cd[c].N + SCO_CHUNK - 1) / SCO_CHUNK;
    int used = 0;
    for (int k = threadIdx.x; k < qmax; k += kBlock) {
      const int64_t r = static_cast<int64_t>(k) * a.nchunks;
      used += (a.hist[r + ch1] - a.hist[r + ch0]) > 0;
    }
    used = block_sum(used);
    if (threadIdx.x == 0) a.st[c].colors_used = used;
  }
}

// ------------------------------------------------------------------ step (3)
// Colour classes in ascending order; class k of every chain is the run
// perm[hist[k * nchunks] .. hist[(k+1) * nchunks]).  Flipping s_v changes H' by
// s_v h_v, h_v = 2J sum_NN s_u - sum_bonds delta_m s_u (NN first, then the bonds in
// row order); with kappa == 1 a bond is hard and forbids the flip, and the
// exchange-only acceptance is the table pacc.
__device__ bool phase_sweep(const StepArgs& a) {
  const int qmax = static_cast<int>(a.sync->qmax);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int s = 0; s < a.nsw_max; ++s) {
    for (int k = 0; k < qmax; ++k) {
      const int64_t i0 = a.hist[static_cast<int64_t>(k) * a.nchunks];
      const int64_t i1 = a.hist[static_cast<int64_t>(k + 1) * a.nchunks];
      // every thread runs the same number of iterations: the ballots see whole waves
      for (int64_t base = i0 + static_cast<int64_t>(blockIdx.x) * kBlock; base < i1; base += stride) {
        const int64_t i = base + threadIdx.x;
        bool acc = false;
        int c = -1;
        if (i < i1) {
          const int32_t g = a.perm[i];
          c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
          const ChainDesc& d = a.cd[c];
          const int nsw = a.nsw_override >= 0 ? a.nsw_override : d.n_sw;
          if (s < nsw) {
            const int v = static_cast<int>(g - d.vbase);
            const int y = fdiv(v, 1.0 / d.L), x = v - y * d.L;
            int nb[4];
            const int n = nn_sites(x, y, d.L, d.periodic, nb);
            int nn = 0;
            for (int t = 0; t < n; ++t) nn += a.spin[d.vbase + nb[t]];
            const int8_t sv = a.spin[g];
            const int q0 = a.row_ptr[g], q1 = a.row_ptr[g + 1];
            if (d.hard) {
              if (q1 == q0) {
                const double pa = d.pacc[sv * nn + 4];
                if (pa >= 1.0) {
                  acc = true;
                } else {
                  const W4 r = philox10(a.step, static_cast<uint32_t>(v), static_cast<uint32_t>(s),
                                        SCO_TAG_MC, d.seed, d.chain_id);
                  acc = unit52(r.x, r.y) < pa;
                }
              }
            } else {
              double h = d.twoJ * static_cast<double>(nn);
              for (int t = q0; t < q1; ++t) {
                const double dm = d.delta[a.attr[t]];
                h = a.spin[a.col[t]] > 0 ? h - dm : h + dm;
              }
              const double dE = sv > 0 ? h : -h;
              if (dE <= 0.0) {
                acc = true;
              } else {
                const W4 r = philox10(a.step, static_cast<uint32_t>(v), static_cast<uint32_t>(s),
                                      SCO_TAG_MC, d.seed, d.chain_id);
                const double u = unit52(r.x, r.y);
                const double pr = exp(d.neg_beta * dE);
                if (fabs(u - pr) < 1e-12) atomicAdd(&a.st[c].near_ties, 1ull);
                acc = u < pr;
              }
            }
            if (acc) a.spin[g] = static_cast<int8_t>(-sv);
          }
        }
        // accepted flips per chain: one atomic per wave when the wave is one chain
        const int c0 = __shfl(c, 0);
        if (__ballot(c != c0 && c >= 0) == 0) {
          const uint64_t mk = __ballot(acc);
          if (lane_id() == 0 && mk && c0 >= 0)
            atomicAdd(&a.st[c0].accepted, static_cast<unsigned long long>(__popcll(mk)));
        } else if (acc) {
          atomicAdd(&a.st[c].accepted, 1ull);
        }
      }
      if (!grid_barrier(a.sync)) return false;
    }
  }
  if (blockIdx.x == 0)
    for (int c = threadIdx.x; c < a.n_chains; c += kBlock) {
      const int nsw = a.nsw_override >= 0 ? a.nsw_override : a.cd[c].n_sw;
      a.st[c].attempts += static_cast<unsigned long long>(a.cd[c].N) * static_cast<unsigned long long>(nsw);
    }
  return true;
}

// ------------------------------------------------------------------ the step
// Persistent kernel (cooperative launch: every block resident).  `phases` selects
// steps (1) switching + assembly, (2) colouring + bucketing, (3) sweeps.
extern "C" __global__ void __launch_bounds__(kBlock) k_step(StepArgs a, uint32_t phases) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  if (phases & PH_SWITCH) {
    for (int64_t g = gtid(); g < a.G; g += stride) {
      a.deg[g] = 0;
      a.fill[g] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a.sync->edge_count = 0;
    for (int c = gtid(); c < a.n_chains; c += stride) {
      a.st[c].delta_union = 0;
      a.st[c].n_edges = 0;
    }
    if (!grid_barrier(a.sync)) return;
    phase_switch(a);
    if (!grid_barrier(a.sync)) return;
    scan_partials(a.deg, a.G, a.part);
    if (!grid_barrier(a.sync)) return;
    scan_top(a.part, a.G);
    if (!grid_barrier(a.sync)) return;
    scan_final(a.deg, a.G, a.part, a.row_ptr);
    if (!grid_barrier(a.sync)) return;
    phase_scatter(a);
    if (!grid_barrier(a.sync)) return;
    phase_rowsort(a);
    if (!grid_barrier(a.sync)) return;
  }
  if (phases & PH_COLOR) {
    phase_kw_setup(a);
    if (!grid_barrier(a.sync)) return;
    if (!phase_kw(a)) return;
    const int qmax = static_cast<int>(a.sync->qmax);
    phase_bucket_hist(a, qmax);
    if (!grid_barrier(a.sync)) return;
    const int64_t nh = static_cast<int64_t>(qmax) * a.nchunks;
    scan_partials(a.hist, nh, a.part);
    if (!grid_barrier(a.sync)) return;
    scan_top(a.part, nh);
    if (!grid_barrier(a.sync)) return;
    scan_final(a.hist, nh, a.part, a.hist);
    if (!grid_barrier(a.sync)) return;
    phase_bucket_scatter(a, qmax);
    phase_colors_used(a, qmax);
    if (!grid_barrier(a.sync)) return;
  }
  if (phases & PH_SWEEP) {
    if (!phase_sweep(a)) return;
  }
}

// =================================================================== observables
// Per chunk (one chain): sum s and sum over the NN pairs (+x, +y) of s_i s_j.
extern "C" __global__ void __launch_bounds__(kBlock)
    k_obs_basic(const ChainDesc* __restrict__ cd, const int32_t* __restrict__ chunk_chain,
                const int8_t* __restrict__ spin, unsigned long long* __restrict__ out, int64_t G) {
  const int64_t g = gtid();
  const int c = chunk_chain[blockIdx.x];
  const ChainDesc& d = cd[c];
  const int v = static_cast<int>(g - d.vbase);
  long long m = 0, ex = 0;
  if (g < G && v < d.N) {
    const int L = d.L, y = v / L, x = v - y * L;
    const int s = spin[g];
    m = s;
    if (d.periodic) {
      ex += s * spin[d.vbase + y * L + (x + 1 == L ? 0 : x + 1)];
      ex += s * spin[d.vbase + (y + 1 == L ? 0 : y + 1) * L + x];
    } else {
      if (x + 1 < L) ex += s * spin[g + 1];
      if (y + 1 < L) ex += s * spin[g + L];
    }
  }
  m = block_sum(m);
  ex = block_sum(ex);
  if (threadIdx.x == 0) {
    atomicAdd(&out[2 * c], static_cast<unsigned long long>(m));
    atomicAdd(&out[2 * c + 1], static_cast<unsigned long long>(ex));
  }
}

// Spins of one chain as bit rows: bit x of row y set when s(x, y) = -1; W words a row.
extern "C" __global__ void k_obs_pack(const int8_t* __restrict__ spin, int64_t vbase, int L, int W,
                                      uint32_t* __restrict__ bits) {
  const int64_t t = gtid();
  if (t >= static_cast<int64_t>(L) * W) return;
  const int y = static_cast<int>(t / W), w = static_cast<int>(t - static_cast<int64_t>(y) * W);
  uint32_t b = 0;
  for (int i = 0; i < 32; ++i) {
    const int x = w * 32 + i;
    if (x < L && spin[vbase + static_cast<int64_t>(y) * L + x] < 0) b |= 1u << i;
  }
  bits[t] = b;
}

// 32 bits of an L-bit row (L = 32 W) starting at bit `off` >= 0: cyclic, or zero
// beyond the row
__device__ __forceinline__ uint32_t row_word(const uint32_t* __restrict__ row, int W, int off,
                                             bool cyclic) {
  const int w = off >> 5, sh = off & 31;
  uint32_t lo, hi;
  if (cyclic) {
    lo = row[w % W];
    hi = row[(w + 1) % W];
  } else {
    lo = w < W ? row[w] : 0u;
    hi = (w + 1) < W ? row[w + 1] : 0u;
  }
  return sh ? (lo >> sh) | (hi << (32 - sh)) : lo;
}

// Owned-pair correlation C_m = sum over the pairs (i, i + d_m) owned by i of
// s_i s_j, exact (mismatching bits counted by popcount), then prod[m] = J_m C_m.
// Needs L % 32 == 0.
extern "C" __global__ void k_obs_corr_bits(const uint32_t* __restrict__ hd, const double* __restrict__ J,
                                           int K, int L, int periodic,
                                           const uint32_t* __restrict__ bits,
                                           double* __restrict__ prod) {
  const int64_t m = gtid();
  if (m >= K) return;
  const int W = L >> 5;
  const uint32_t p = hd[m];
  const int dx = static_cast<int16_t>(p & 0xFFFFu), dy = static_cast<int16_t>(p >> 16);
  const int h = L >> 1;
  long long mism = 0, pairs = 0;
  if (periodic) {
    int y1 = L, xlim = L;
    if (dy == 0 && dx == h) xlim = h;             // owners x < L/2
    if (dy == h && (dx == 0 || dx == h)) y1 = h;  // owners y < L/2
    const int sx = dx < 0 ? dx + L : dx;
    for (int y = 0; y < y1; ++y) {
      const uint32_t* ra = bits + static_cast<int64_t>(y) * W;
      const int yb = y + dy >= L ? y + dy - L : y + dy;
      const uint32_t* rb = bits + static_cast<int64_t>(yb) * W;
      for (int w = 0; w * 32 < xlim; ++w) {
        uint32_t mask = 0xFFFFFFFFu;
        if (w * 32 + 32 > xlim) mask = (1u << (xlim - w * 32)) - 1u;
        const int off = w * 32 + sx;
        const uint32_t b = row_word(rb, W, off >= L ? off - L : off, true);
        mism += __popc((ra[w] ^ b) & mask);
      }
      pairs += xlim;
    }
  } else {
    const int xa0 = dx < 0 ? -dx : 0, xa1 = dx < 0 ? L : L - dx;  // owners x in [xa0, xa1)
    for (int y = 0; y + dy < L; ++y) {
      const uint32_t* ra = bits + static_cast<int64_t>(y) * W;
      const uint32_t* rb = bits + static_cast<int64_t>(y + dy) * W;
      for (int w = 0; w < W; ++w) {
        const int xb = w * 32;
        if (xb + 32 <= xa0 || xb >= xa1) continue;
        uint32_t mask = 0xFFFFFFFFu;
        if (xb < xa0) mask &= ~((1u << (xa0 - xb)) - 1u);
        if (xb + 32 > xa1) mask &= (1u << (xa1 - xb)) - 1u;
        const int off = xb + dx;  // partner of bit i is bit off + i of row y + dy
        const uint32_t b = off >= 0 ? row_word(rb, W, off, false) : (row_word(rb, W, 0, false) << (-off));
        mism += __popc((ra[w] ^ b) & mask);
      }
      pairs += xa1 - xa0;
    }
  }
  const long long cm = pairs - 2 * mism;
  prod[m] = J[m] * static_cast<double>(cm);
}

// Same quantity for any L, pair by pair (small lattices).
extern "C" __global__ void k_obs_corr_plain(const uint32_t* __restrict__ hd, const double* __restrict__ J,
                                            int K, int L, int periodic, const int8_t* __restrict__ spin,
                                            int64_t vbase, double* __restrict__ prod) {
  const int64_t m = gtid();
  if (m >= K) return;
  const uint32_t p = hd[m];
  const int dx = static_cast<int16_t>(p & 0xFFFFu), dy = static_cast<int16_t>(p >> 16);
  long long cm = 0;
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      const int j = partner_of(x, y, dx, dy, L, periodic);
      if (j >= 0) cm += spin[vbase + y * L + x] * spin[vbase + j];
    }
  prod[m] = J[m] * static_cast<double>(cm);
}

// Deterministic sum of prod[0..K): blocks of 4096 terms (per-thread runs of 16,
// then a fixed tree), then the block partials in order by one thread.
extern "C" __global__ void __launch_bounds__(kBlock)
    k_obs_sum_partials(const double* __restrict__ prod, int K, double* __restrict__ part) {
  __shared__ double buf[kBlock];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * 4096;
  double s = 0.0;
  for (int i = 0; i < 16; ++i) {
    const int64_t idx = base + static_cast<int64_t>(threadIdx.x) * 16 + i;
    if (idx < K) s += prod[idx];
  }
  buf[threadIdx.x] = s;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < static_cast<uint32_t>(o)) buf[threadIdx.x] += buf[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = buf[0];
}

extern "C" __global__ void k_obs_sum_final(const double* __restrict__ part, int nparts,
                                           double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < nparts; ++i) s += part[i];
  *out = s;
}

// =================================================================== host launchers
namespace sco_dev {

hipError_t table_j(hipStream_t s, const uint32_t* hd, int K, int L, int periodic, int n_images,
                   double D, double* J) {
  hipLaunchKernelGGL(k_table_j, dim3((K + kBlock - 1) / kBlock), dim3(kBlock), 0, s, hd, K, L,
                     periodic, n_images, D, J);
  return hipGetLastError();
}

hipError_t init_spins(hipStream_t s, const ChainDesc* cd, const int32_t* chunk_chain,
                      const int64_t* src_base, const int8_t* src, int8_t* spin, int64_t G) {
  hipLaunchKernelGGL(k_init_spins, dim3(static_cast<uint32_t>(G / kBlock)), dim3(kBlock), 0, s, cd,
                     chunk_chain, src_base, src, spin, G);
  return hipGetLastError();
}

int step_max_blocks() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(k_step), kBlock, 0) !=
      hipSuccess)
    return 0;
  return per * cus;
}

hipError_t step(hipStream_t s, const StepArgs& a, uint32_t phases, int blocks) {
  StepArgs copy = a;
  void* args[] = {&copy, &phases};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_step), dim3(blocks), dim3(kBlock),
                                    args, 0, s);
}

hipError_t obs_basic(hipStream_t s, const ChainDesc* cd, const int32_t* chunk_chain, const int8_t* spin,
                     unsigned long long* out, int64_t G) {
  hipLaunchKernelGGL(k_obs_basic, dim3(static_cast<uint32_t>(G / kBlock)), dim3(kBlock), 0, s, cd,
                     chunk_chain, spin, out, G);
  return hipGetLastError();
}

hipError_t obs_dipolar(hipStream_t s, const uint32_t* hd, const double* J, int K, int L, int periodic,
                       const int8_t* spin, int64_t vbase, uint32_t* bits, double* prod, double* part,
                       double* out) {
  if (L % 32 == 0) {
    const int W = L / 32;
    hipLaunchKernelGGL(k_obs_pack, dim3((L * W + kBlock - 1) / kBlock), dim3(kBlock), 0, s, spin, vbase,
                       L, W, bits);
    hipLaunchKernelGGL(k_obs_corr_bits, dim3((K + kBlock - 1) / kBlock), dim3(kBlock), 0, s, hd, J, K, L,
                       periodic, bits, prod);
  } else {
    hipLaunchKernelGGL(k_obs_corr_plain, dim3((K + kBlock - 1) / kBlock), dim3(kBlock), 0, s, hd, J, K,
                       L, periodic, spin, vbase, prod);
  }
  const int nparts = (K + 4095) / 4096;
  hipLaunchKernelGGL(k_obs_sum_partials, dim3(nparts), dim3(kBlock), 0, s, prod, K, part);
  hipLaunchKernelGGL(k_obs_sum_final, dim3(1), dim3(64), 0, s, part, nparts, out);
  return hipGetLastError();
}

}  // namespace sco_dev
