// sco_api.cpp -- host runtime of libsco: parameter checks, workspace layout, the
// displacement tables, launches and read-backs.  See include/sco.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/sco.h"
#include "sco_internal.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int kNB = 1 << SCO_GUIDE_BITS;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int64_t halfset_size(int L, int periodic) {
  return periodic ? static_cast<int64_t>(L) * L / 2 + 1 : 2LL * L * (L - 1);
}

bool valid(const sco_chain_params& p) {
  if (p.L < 2 || p.L > 16384) return false;
  if (p.periodic && (p.L < 4 || (p.L & 1))) return false;
  if (!(p.T > 0.0) || !(p.kappa >= 1.0) || !(p.J > 0.0) || !(p.D > 0.0)) return false;
  if (!std::isfinite(p.T) || !std::isfinite(p.kappa) || !std::isfinite(p.J) || !std::isfinite(p.D)) return false;
  if (p.n_sw < 0 || p.n_images < 0 || p.n_images > 64) return false;
  if (p.precision != 0 && p.precision != 1) return false;
  if (p.edge_factor < 0 || p.edge_factor > 256) return false;
  if (p.model != SCO_MODEL_ISING && p.model != SCO_MODEL_HEIS) return false;
  // Heisenberg spins: open lattices (Sec. 3.1), V^max = 2 D / r^3, FP64 decisions
  if (p.model == SCO_MODEL_HEIS && (p.periodic || p.kappa != 1.0 || p.precision != 0)) return false;
  return true;
}

// the displacement table's coupling constant: J_m = D / r^3 for Ising spins, the bound
// V^max = 2 D / r^3 of the dipolar tensor for Heisenberg spins
double table_d(const sco_chain_params& p) { return p.model == SCO_MODEL_HEIS ? 2.0 * p.D : p.D; }

// ---- exact transform plans for the pair correlations (Ising chains)
bool is_prime32(uint32_t x) {
  if (x < 2) return false;
  for (uint32_t i = 2; static_cast<uint64_t>(i) * i <= x; ++i)
    if (x % i == 0) return false;
  return true;
}
uint32_t pow_mod(uint64_t b, uint64_t e, uint32_t p) {
  uint64_t r = 1;
  b %= p;
  for (; e; e >>= 1, b = b * b % p)
    if (e & 1) r = r * b % p;
  return static_cast<uint32_t>(r);
}
// radices 8, 4, 2, 3, 5, 7 of n (powers of two by 8s, then one 4 or 2); false when n has
// another prime factor
bool ntt_radices(int n, NttPlan& pl) {
  pl.nrad = 0;
  int twos = 0;
  while (n % 2 == 0) {
    n /= 2;
    ++twos;
  }
  for (; twos >= 3; twos -= 3) pl.rad[pl.nrad++] = 8;
  if (twos > 0) pl.rad[pl.nrad++] = 1 << twos;
  for (int r : {3, 5, 7})
    while (n % r == 0) {
      n /= r;
      pl.rad[pl.nrad++] = r;
      if (pl.nrad >= 24) return false;
    }
  return n == 1;
}
// The transform of one chain's lattice: length L (periodic) or the smallest 2^a 3^b
// 5^c 7^d >= 2L - 1 (open, zero-padded so the cyclic correlation is the linear one);
// n = 0 when L has another prime factor or no prime below 2^31 fits.
NttPlan ntt_plan(const sco_chain_params& q) {
  NttPlan pl{};
  if (q.model != SCO_MODEL_ISING) return pl;
  const int64_t L = q.L;
  const uint64_t minp = 2 * static_cast<uint64_t>(L) * static_cast<uint64_t>(L) + 1;  // |C| <= L^2
  if (minp >= (1ull << 30)) return pl;
  int n = 0;
  if (q.periodic) {
    n = static_cast<int>(L);
    if (!ntt_radices(n, pl)) return NttPlan{};
  } else {
    for (n = static_cast<int>(2 * L - 1); n < 8 * L; ++n)
      if (ntt_radices(n, pl)) break;
  }
  if (n < 2 || n > 16384) return NttPlan{};
  uint32_t p = 0;
  for (uint64_t k = ((1ull << 31) - 1) / static_cast<uint64_t>(n); k > 0; --k) {
    const uint64_t c = k * static_cast<uint64_t>(n) + 1;
    if (c <= minp) break;
    if (c < (1ull << 31) && is_prime32(static_cast<uint32_t>(c))) {
      p = static_cast<uint32_t>(c);
      break;
    }
  }
  if (p == 0) return NttPlan{};
  pl.n = n;
  pl.p = p;
  uint32_t inv = p;  // p^-1 mod 2^32 by Newton's iteration (p odd)
  for (int i = 0; i < 5; ++i) inv *= 2u - p * inv;
  pl.pinv = 0u - inv;
  pl.one = static_cast<uint32_t>((1ull << 32) % p);
  const uint32_t ninv = pow_mod(static_cast<uint64_t>(n), p - 2, p);
  pl.ninv2 = static_cast<uint32_t>(static_cast<uint64_t>(ninv) * ninv % p);
  return pl;
}
// The FP64 transforms of a Heisenberg chain's dipolar energy: length the smallest
// 2^a 3^b 5^c 7^d >= 2L - 1 (open lattice, zero-padded); n = 0 (the direct pair sums)
// while N K <= 2e9, where those take at most about a second.
NttPlan fft_plan(const sco_chain_params& q) {
  NttPlan pl{};
  if (q.model != SCO_MODEL_HEIS) return pl;
  const double L = q.L;
  if (L * L * 2.0 * L * (L - 1.0) <= 2e9) return pl;
  int n = 0;
  for (n = 2 * q.L - 1; n < 8 * q.L; ++n)
    if (ntt_radices(n, pl)) break;
  if (n > 16384) return NttPlan{};
  pl.n = n;
  return pl;
}
// (cos, sin)(2 pi e / n), e < n
std::vector<double> fft_twiddles(int n) {
  std::vector<double> tw(2 * static_cast<size_t>(n));
  const double step = 2.0 * 3.14159265358979323846 / static_cast<double>(n);
  for (int e = 0; e < n; ++e) {
    tw[2 * e] = std::cos(step * e);
    tw[2 * e + 1] = std::sin(step * e);
  }
  return tw;
}

// w^e in Montgomery form, e < n, w a primitive n-th root of unity mod p
std::vector<uint32_t> ntt_twiddles(const NttPlan& pl) {
  const uint32_t p = pl.p;
  std::vector<uint32_t> f;  // the prime factors of p - 1
  uint32_t x = p - 1;
  for (uint32_t i = 2; static_cast<uint64_t>(i) * i <= x; ++i)
    if (x % i == 0) {
      f.push_back(i);
      while (x % i == 0) x /= i;
    }
  if (x > 1) f.push_back(x);
  uint32_t g = 2;
  for (;; ++g) {
    bool prim = true;
    for (uint32_t q : f) prim = prim && pow_mod(g, (p - 1) / q, p) != 1;
    if (prim) break;
  }
  const uint32_t w = pow_mod(g, (p - 1) / static_cast<uint32_t>(pl.n), p);
  std::vector<uint32_t> tw(pl.n);
  uint64_t we = 1;
  for (int e = 0; e < pl.n; ++e, we = we * w % p) tw[e] = static_cast<uint32_t>((we << 32) % p);
  return tw;
}

using TableKey = std::tuple<int, int, int, double>;  // L, periodic, n_images, D

struct Layout {
  // per distinct lattice
  std::map<TableKey, int> table_index;
  std::vector<TableKey> tables;
  std::vector<int64_t> table_K;
  std::vector<size_t> off_hd, off_J, off_C, off_guide;
  // per chain
  std::vector<int> chain_table;
  std::vector<int64_t> vbase;
  std::vector<size_t> off_theta, off_delta, off_delta32;
  size_t off_sync = 0, off_cd = 0, off_st = 0, off_chunk = 0, off_srcbase = 0;
  size_t off_spin = 0, off_deg = 0, off_row = 0, off_fill = 0, off_ea = 0, off_eb = 0, off_em = 0, off_er = 0;
  size_t off_col = 0, off_attr = 0, off_color = 0, off_word = 0, off_rec = 0, off_ecount = 0, off_trace = 0;
  size_t off_spin_bak = 0, off_st_bak = 0;
  size_t off_agg = 0, off_obs = 0, off_used = 0, off_bits = 0, off_prod = 0, off_dpart = 0, off_dres = 0;
  size_t off_acc = 0, off_spin3 = 0, off_hpart = 0, off_hres = 0, off_csz = 0;
  size_t off_ntt = 0, off_tw = 0;  // transform buffers (2 n^2) and twiddles (n) of the largest plan
  size_t off_fft = 0, off_ftw = 0;  // Heisenberg: FP64 transform buffers (3 n^2 complex), twiddles
  int64_t G = 0, nchunks = 0, ntiles = 0, maxK = 0;
  uint32_t cap_und = 0;
  size_t bytes = 0;
};

int make_layout(const sco_chain_params* p, int n, Layout& lay) {
  size_t off = 0;
  auto take = [&](size_t nbytes) {
    const size_t o = off;
    off = align_up(off + nbytes);
    return o;
  };
  lay.off_sync = take(sizeof(SyncWords));
  lay.off_cd = take(sizeof(ChainDesc) * n);
  lay.off_st = take(sizeof(ChainState) * n);
  int64_t G = 0, edges = 0;
  for (int c = 0; c < n; ++c) {
    if (p[c].model != p[0].model) return SCO_EINVAL;  // one spin model per context
    const TableKey key{p[c].L, p[c].periodic ? 1 : 0, p[c].periodic ? p[c].n_images : 0, table_d(p[c])};
    auto it = lay.table_index.find(key);
    int t;
    if (it == lay.table_index.end()) {
      t = static_cast<int>(lay.tables.size());
      lay.table_index[key] = t;
      lay.tables.push_back(key);
      lay.table_K.push_back(halfset_size(p[c].L, p[c].periodic));
    } else {
      t = it->second;
    }
    lay.chain_table.push_back(t);
    lay.vbase.push_back(G);
    const int64_t N = static_cast<int64_t>(p[c].L) * p[c].L;
    G += (N + SCO_CHUNK - 1) / SCO_CHUNK * SCO_CHUNK;
    const int ef = p[c].edge_factor ? p[c].edge_factor : 4;
    edges = std::max<int64_t>(edges, static_cast<int64_t>(SCO_CHUNK) * ef / 2);  // per chunk
  }
  lay.G = G;
  lay.nchunks = G / SCO_CHUNK;
  // every chunk gets the same survivor region: the largest edge factor of the chains
  if (G >= (1LL << 31) - SCO_CHUNK || edges * lay.nchunks >= (1LL << 30)) return SCO_EINVAL;
  lay.cap_und = static_cast<uint32_t>(edges * lay.nchunks);
  lay.off_chunk = take(sizeof(int32_t) * lay.nchunks);
  lay.off_srcbase = take(sizeof(int64_t) * n);
  for (size_t t = 0; t < lay.tables.size(); ++t) {
    const int64_t K = lay.table_K[t];
    lay.maxK = std::max(lay.maxK, K);
    lay.off_hd.push_back(take(sizeof(uint32_t) * K));
    lay.off_J.push_back(take(sizeof(double) * K));
    lay.off_C.push_back(take(sizeof(double) * K));
    lay.off_guide.push_back(take(sizeof(int32_t) * (kNB + 1)));
  }
  for (int c = 0; c < n; ++c) {
    const int64_t K = lay.table_K[lay.chain_table[c]];
    const bool hard = p[c].kappa == 1.0;
    const bool heis = p[c].model == SCO_MODEL_HEIS;
    // theta (Ising kappa > 1) or the Heisenberg denominators expm1(-2 beta J_m)
    lay.off_theta.push_back(hard && !heis ? 0 : take(sizeof(double) * K));
    lay.off_delta.push_back(hard ? 0 : take(sizeof(double) * K));
    lay.off_delta32.push_back(hard ? 0 : take(sizeof(float) * K));
  }
  lay.off_spin = take(G);
  lay.off_spin3 = p[0].model == SCO_MODEL_HEIS ? take(sizeof(double) * 3 * G) : 0;
  lay.off_deg = take(sizeof(int32_t) * G);
  lay.off_row = take(sizeof(int32_t) * (G + 1));
  lay.off_fill = take(sizeof(int32_t) * G);
  lay.off_ea = take(sizeof(int32_t) * lay.cap_und);
  lay.off_eb = take(sizeof(int32_t) * lay.cap_und);
  lay.off_em = take(sizeof(int32_t) * lay.cap_und);
  lay.off_er = take(sizeof(int32_t) * lay.cap_und);
  lay.off_col = take(sizeof(int32_t) * 2 * static_cast<size_t>(lay.cap_und));
  lay.off_attr = take(sizeof(int32_t) * 2 * static_cast<size_t>(lay.cap_und));
  lay.off_color = take(sizeof(uint16_t) * G);
  lay.off_word = take(sizeof(uint32_t) * G);
  lay.off_rec = take(sizeof(int4) * G);
  lay.off_ecount = take(sizeof(uint32_t) * lay.nchunks);
  lay.off_trace = take(sizeof(unsigned long long) * SCO_TRACE_SLOTS);
  lay.ntiles = G / (SCO_SCAN_ITEMS * SCO_CHUNK) + 2;  // tiles of the degree scan
  lay.off_agg = take(sizeof(long long) * lay.ntiles);
  lay.off_spin_bak = take(G);  // autotuning trials restore the chain from here
  lay.off_st_bak = take(sizeof(ChainState) * n);
  lay.off_obs = take(sizeof(unsigned long long) * 2 * n);
  lay.off_used = take(sizeof(uint32_t) * SCO_QWORDS * n);
  int maxbits = 0;
  for (int c = 0; c < n; ++c) maxbits = std::max(maxbits, p[c].L * ((p[c].L + 31) / 32));
  lay.off_bits = take(sizeof(uint32_t) * maxbits);
  lay.off_prod = take(sizeof(double) * lay.maxK);
  lay.off_dpart = take(sizeof(double) * (lay.maxK / 4096 + 2));
  lay.off_dres = take(sizeof(double) * n);
  lay.off_acc = take(sizeof(AnnealAcc) * n);
  int64_t maxN = 0;
  for (int c = 0; c < n; ++c) maxN = std::max<int64_t>(maxN, static_cast<int64_t>(p[c].L) * p[c].L);
  lay.off_hpart = take(sizeof(double) * 2 * (maxN / 256 + 2));
  lay.off_hres = take(sizeof(double) * 2);
  lay.off_csz = take(sizeof(unsigned long long) * 256);
  int64_t nmax = 0;
  for (int c = 0; c < n; ++c) nmax = std::max<int64_t>(nmax, ntt_plan(p[c]).n);
  lay.off_ntt = take(sizeof(uint32_t) * 2 * nmax * nmax);
  lay.off_tw = take(sizeof(uint32_t) * nmax);
  int64_t fmax = 0;
  for (int c = 0; c < n; ++c) fmax = std::max<int64_t>(fmax, fft_plan(p[c]).n);
  lay.off_fft = take(2 * sizeof(double) * 3 * fmax * fmax);
  lay.off_ftw = take(2 * sizeof(double) * fmax);
  lay.bytes = off;
  return SCO_OK;
}

// Half-displacement set: each unordered pair of sites is reached from exactly one
// (owner, displacement) that passes the owner rule; sorted by (r^2, dy, dx).
void build_halfset(int L, int periodic, std::vector<uint32_t>& hd) {
  std::vector<std::pair<int, int>> d;
  if (periodic) {
    const int h = L / 2;
    for (int dy = 0; dy <= h; ++dy)
      for (int dx = -h + 1; dx <= h; ++dx) {
        const bool keep = (dy > 0 && dy < h) || dx > 0 || (dy == h && dx == 0);
        if (keep) d.emplace_back(dx, dy);
      }
  } else {
    for (int dy = 0; dy < L; ++dy)
      for (int dx = -(L - 1); dx < L; ++dx)
        if (dy > 0 || dx > 0) d.emplace_back(dx, dy);
  }
  std::sort(d.begin(), d.end(), [](const std::pair<int, int>& a, const std::pair<int, int>& b) {
    const int64_t ra = static_cast<int64_t>(a.first) * a.first + static_cast<int64_t>(a.second) * a.second;
    const int64_t rb = static_cast<int64_t>(b.first) * b.first + static_cast<int64_t>(b.second) * b.second;
    if (ra != rb) return ra < rb;
    if (a.second != b.second) return a.second < b.second;
    return a.first < b.first;
  });
  hd.resize(d.size());
  for (size_t m = 0; m < d.size(); ++m)
    hd[m] = static_cast<uint32_t>(static_cast<uint16_t>(d[m].first)) |
            (static_cast<uint32_t>(static_cast<uint16_t>(d[m].second)) << 16);
}

}  // namespace

struct sco_ctx {
  hipStream_t stream = nullptr;
  int n = 0;
  int model = SCO_MODEL_ISING;
  std::vector<sco_chain_params> params;
  Layout lay;
  char* ws = nullptr;
  std::vector<std::vector<double>> J, C;          // per table (host copies)
  std::vector<std::vector<uint32_t>> hd;           // per table
  std::vector<std::vector<double>> theta, delta;   // per chain (empty when hard)
  std::vector<ChainDesc> cd;                       // host copy of the descriptors
  StepArgs args{};
  int blocks = 0, max_blocks = 0;  // grid of the step kernel (schedule), co-resident limit
  int launched_blocks = 0;         // grid of the last launch (its barrier counters)
  int nsw_max = 0;
  int graph_state = 0;  // 0 no bond graph yet, 1 switched, 2 switched and coloured
  int step_fused = 0;   // a step as one launch of the fused kernel (else three launches)
  bool trace_on = false;
  double wall_mhz = 100.0;
  unsigned long long* pinned = nullptr;            // read-back staging
  size_t pinned_bytes = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  float phase_ms[3] = {0, 0, 0};
  int64_t flags_seen = 0;
  uint32_t last_flags = 0;  // flags of the last flagged launch consumed
  uint32_t flags_host = 0;  // read-back word when there is no pinned staging
  // the step graph of sco_run_graph: n_steps cooperative k_step<7> nodes in a chain,
  // built for one grid size; its nodes' arguments are rewritten for every replay
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<hipGraphNode_t> graph_nodes;
  std::vector<StepArgs> graph_args;
  int graph_blocks = 0;
};

namespace {

template <typename T>
T* at(sco_ctx* c, size_t off) {
  return reinterpret_cast<T*>(c->ws + off);
}

#define HIP_TRY(expr)                     \
  do {                                    \
    if ((expr) != hipSuccess) return SCO_EHIP; \
  } while (0)

int read_flags(sco_ctx* c, uint32_t* flags) {
  const SyncWords* d = at<SyncWords>(c, c->lay.off_sync);
  // the pinned staging word, or (a context that allocates nothing) a host member
  void* dst = c->pinned ? static_cast<void*>(c->pinned) : static_cast<void*>(&c->flags_host);
  HIP_TRY(hipMemcpyAsync(dst, &d->flags, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *flags = *static_cast<const uint32_t*>(dst);
  return SCO_OK;
}

// Clears the flags and the barrier words (a timed-out barrier can leave the count
// non-zero); returns the code that the flags map to.
int consume_flags(sco_ctx* c) {
  uint32_t f = 0;
  int rc = read_flags(c, &f);
  if (rc) return rc;
  if (f == 0) return SCO_OK;
  c->flags_seen |= f;
  c->last_flags = f;
  // a flagged launch stopped at a barrier and later launches did nothing: the bond
  // graph and colouring are not valid any more (the device words are cleared with
  // the rest of the sync block, the halt word included)
  c->graph_state = 0;
  HIP_TRY(hipMemsetAsync(at<SyncWords>(c, c->lay.off_sync), 0, sizeof(SyncWords), c->stream));
  // the partner counts start every switching at zero; a stopped step may have left
  // them anywhere (the scatter clears them only in a step that reached it)
  HIP_TRY(hipMemsetAsync(at<int32_t>(c, c->lay.off_deg), 0, sizeof(int32_t) * c->lay.G, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (f & SCO_FLAG_TIMEOUT) return SCO_ETIMEOUT;
  if (f & SCO_FLAG_OVERFLOW) return SCO_EOVERFLOW;
  if (f & SCO_FLAG_PALETTE) return SCO_EPALETTE;
  return SCO_EINTERNAL;
}

// Launches `phases` for SCO step `step`.
int launch(sco_ctx* c, uint32_t phases, uint64_t step, int nsw_override, bool trace_reset = true) {
  if (step > 0xFFFFFFFFull) return SCO_EINVAL;
  if (c->blocks != c->launched_blocks) {
    // the barrier counters count arrivals in groups sized by the grid: start them
    // afresh for another grid size (stream-ordered: no launch is running)
    HIP_TRY(hipMemsetAsync(at<SyncWords>(c, c->lay.off_sync), 0, offsetof(SyncWords, flags), c->stream));
    c->launched_blocks = c->blocks;
  }
  c->args.step = static_cast<uint32_t>(step);
  if (c->trace_on) {
    c->args.trace = at<unsigned long long>(c, c->lay.off_trace);
    if (trace_reset) HIP_TRY(hipMemsetAsync(c->args.trace, 0, sizeof(unsigned long long), c->stream));
  } else {
    c->args.trace = nullptr;
  }
  c->args.nsw_override = nsw_override;
  c->args.nsw_max = nsw_override >= 0 ? nsw_override : c->nsw_max;
  HIP_TRY(sco_dev::step(c->stream, c->args, phases, c->blocks, c->model));
  return SCO_OK;
}

// Full steps first_step .. first_step + n - 1: one launch of the fused kernel per step,
// or (the default, measured faster: each phase kernel holds only its own registers,
// and the launch boundaries replace two device-wide barriers) the switching,
// colouring and sweep kernels one after another; the last step's phases are timed.
int run_steps(sco_ctx* c, uint64_t first_step, int n) {
  for (int s = 0; s < n; ++s) {
    const uint64_t t = first_step + static_cast<uint64_t>(s);
    const bool last = s + 1 == n && c->ev[0] != nullptr;  // (the allocation-free context has no events)
    if (c->step_fused) {
      const int rc = launch(c, PH_SWITCH | PH_COLOR | PH_SWEEP, t, -1);
      if (rc) return rc;
    } else {
      if (last) HIP_TRY(hipEventRecord(c->ev[0], c->stream));
      int rc = launch(c, PH_SWITCH, t, -1);
      if (last && rc == SCO_OK) HIP_TRY(hipEventRecord(c->ev[1], c->stream));
      if (rc == SCO_OK) rc = launch(c, PH_COLOR, t, -1, false);
      if (last && rc == SCO_OK) HIP_TRY(hipEventRecord(c->ev[2], c->stream));
      if (rc == SCO_OK) rc = launch(c, PH_SWEEP, t, -1, false);
      if (last && rc == SCO_OK) HIP_TRY(hipEventRecord(c->ev[3], c->stream));
      if (rc) return rc;
    }
    c->graph_state = 2;
  }
  return SCO_OK;
}

}  // namespace

extern "C" {

const char* sco_strerror(int code) {
  switch (code) {
    case SCO_OK: return "ok";
    case SCO_EINVAL: return "invalid argument";
    case SCO_EHIP: return "HIP runtime error";
    case SCO_EOVERFLOW: return "surviving bonds exceeded the edge capacity";
    case SCO_EINTERNAL: return "internal invariant failed (colouring or sweep without a valid bond graph, or "
                                  "a CSR row out of range)";
    case SCO_ENOSPC: return "workspace too small";
    case SCO_ETIMEOUT: return "a bounded device wait timed out (not every block of the persistent kernel ran)";
    case SCO_EPALETTE: return "the union graph needs more than 255 colours";
    default: return "unknown error";
  }
}

int sco_workspace_size(const sco_chain_params* params, int n_chains, size_t* bytes) {
  if (!params || n_chains <= 0 || n_chains > SCO_MAXCHAINS || !bytes) return SCO_EINVAL;
  for (int c = 0; c < n_chains; ++c)
    if (!valid(params[c])) return SCO_EINVAL;
  Layout lay;
  const int rc = make_layout(params, n_chains, lay);
  if (rc) return rc;
  *bytes = lay.bytes;
  return SCO_OK;
}

namespace {
// The temperature-dependent part of a chain (Eqs. 2-3 at beta = 1/T): the descriptor's
// beta, rate and exchange-only acceptance, and for kappa > 1 the survival ratio theta
// and the pseudo-interaction difference delta of every displacement, uploaded to the
// workspace (synchronous; the descriptor itself is uploaded by the caller).
int temperature_tables(sco_ctx* c, int ci, double T) {
  const Layout& L = c->lay;
  sco_chain_params& p = c->params[ci];
  p.T = T;
  ChainDesc& d = c->cd[ci];
  const double beta = 1.0 / T;
  d.beta = beta;
  d.neg_beta = -beta;
  d.inv_rate = T / (p.kappa + 1.0);
  d.inv_rate32 = static_cast<float>(d.inv_rate);
  d.neg_beta32 = static_cast<float>(-beta);
  // an FP32 gap decision is at least inv_rate 2^-20 from the compared table value;
  // it may stand only where no near tie (1e-12 relative) of the FP64 gap can hide
  d.fp32_gap = d.inv_rate * 0x1p-20 > 2e-12 * d.C_top ? 1 : 0;
  // An owner's first draw u ends it when (-log u) inv_rate > C_top, a near tie when
  // within 1e-12 C_top.  Below u_first_end the target exceeds C_top (1 + 2e-12) less
  // the roundings of log, the product and this bound (each under 1e-15 relative), so
  // the draw ends its owner with certainty and is no near tie.
  d.u_first_end = std::exp(-(d.C_top * (1.0 + 2e-12)) / d.inv_rate) * (1.0 - 1e-14);
  for (int k = -4; k <= 4; ++k) {
    const double dE = (2.0 * p.J) * static_cast<double>(k);
    d.pacc[k + 4] = dE > 0.0 ? std::exp(-beta * dE) : 2.0;
  }
  d.T = T;
  const int t = L.chain_table[ci];
  const int64_t K = L.table_K[t];
  if (d.model == SCO_MODEL_HEIS) {
    // a candidate of the bound rate 2 beta J_m survives with probability
    // (1 - P_ij) / pbar_m, pbar_m = -expm1(-2 beta J_m) (Eqs. 1-2)
    std::vector<double> hd(K);
    const std::vector<double>& Jt = c->J[t];
    for (int64_t m = 0; m < K; ++m) hd[m] = std::expm1(-beta * 2.0 * Jt[m]);
    HIP_TRY(hipMemcpyAsync(const_cast<double*>(d.hden), hd.data(), sizeof(double) * K, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SCO_OK;
  }
  if (d.hard) return SCO_OK;
  std::vector<double>& th = c->theta[ci];
  std::vector<double>& de = c->delta[ci];
  std::vector<float> de32(K);
  th.resize(K);
  de.resize(K);
  const std::vector<double>& Jt = c->J[t];
  for (int64_t m = 0; m < K; ++m) {
    const double em = std::expm1(-beta * (p.kappa + 1.0) * Jt[m]);
    const double ep = std::expm1(-beta * (p.kappa - 1.0) * Jt[m]);
    th[m] = ep / em;
    de[m] = 2.0 * Jt[m] + T * std::log(em / ep);
    de32[m] = static_cast<float>(de[m]);
  }
  HIP_TRY(hipMemcpyAsync(const_cast<double*>(d.theta), th.data(), sizeof(double) * K, hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(const_cast<double*>(d.delta), de.data(), sizeof(double) * K, hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(const_cast<float*>(d.delta32), de32.data(), sizeof(float) * K, hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return SCO_OK;
}

// st[c].mag of every chain from its spins (after the spins were set from outside)
int refresh_mag(sco_ctx* c) {
  const Layout& L = c->lay;
  unsigned long long* d_obs = at<unsigned long long>(c, L.off_obs);
  HIP_TRY(hipMemsetAsync(d_obs, 0, sizeof(unsigned long long) * 2 * c->n, c->stream));
  HIP_TRY(hipMemsetAsync(at<uint32_t>(c, L.off_used), 0, sizeof(uint32_t) * SCO_QWORDS * c->n, c->stream));
  HIP_TRY(sco_dev::obs_basic(c->stream, at<ChainDesc>(c, L.off_cd), at<int32_t>(c, L.off_chunk),
                             at<int8_t>(c, L.off_spin), at<uint16_t>(c, L.off_color), d_obs,
                             at<uint32_t>(c, L.off_used), L.G));
  HIP_TRY(sco_dev::set_mag(c->stream, at<ChainState>(c, L.off_st), d_obs, c->n));
  return SCO_OK;
}

// noalloc: no pinned staging and no events (the context of sco_run_noalloc, which
// allocates nothing); such a context serves launches, flags and observables only.
int init_impl(sco_ctx** out, const sco_chain_params* params, int n_chains, void* dev_workspace,
              size_t workspace_bytes, const int8_t* dev_init_spins, void* stream, bool noalloc) {
  if (!out || !params || n_chains <= 0 || n_chains > SCO_MAXCHAINS || !dev_workspace) return SCO_EINVAL;
  *out = nullptr;
  if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) return SCO_EINVAL;
  for (int c = 0; c < n_chains; ++c)
    if (!valid(params[c])) return SCO_EINVAL;
  sco_ctx* c = new (std::nothrow) sco_ctx();
  if (!c) return SCO_EINTERNAL;
  int rc = make_layout(params, n_chains, c->lay);
  if (rc) {
    delete c;
    return rc;
  }
  if (workspace_bytes < c->lay.bytes) {
    delete c;
    return SCO_ENOSPC;
  }
  c->stream = static_cast<hipStream_t>(stream);
  c->n = n_chains;
  c->model = params[0].model;
  if (c->model == SCO_MODEL_HEIS && dev_init_spins) {  // Heisenberg chains start from Philox
    delete c;
    return SCO_EINVAL;
  }
  c->params.assign(params, params + n_chains);
  c->ws = static_cast<char*>(dev_workspace);
  const Layout& L = c->lay;
  auto fail = [&](int code) {
    sco_destroy(c);
    return code;
  };
  if (!noalloc) {
    c->pinned_bytes = std::max<size_t>(4096, sizeof(ChainState) * n_chains + 64);
    c->pinned_bytes =
        std::max(c->pinned_bytes, sizeof(unsigned long long) * 2 * n_chains + sizeof(double) * n_chains);
    if (hipHostMalloc(reinterpret_cast<void**>(&c->pinned), c->pinned_bytes, hipHostMallocDefault) != hipSuccess)
      return fail(SCO_EHIP);
    for (auto& e : c->ev)
      if (hipEventCreate(&e) != hipSuccess) return fail(SCO_EHIP);
  }
  if (hipMemsetAsync(at<char>(c, L.off_sync), 0, sizeof(SyncWords), c->stream) != hipSuccess) return fail(SCO_EHIP);
  if (hipMemsetAsync(at<char>(c, L.off_st), 0, sizeof(ChainState) * n_chains, c->stream) != hipSuccess)
    return fail(SCO_EHIP);

  // displacement tables per lattice: J(d) on the GPU, cumulative sums and the guide on
  // the host (sequential FP64 sum in table order)
  const size_t nt = L.tables.size();
  c->hd.resize(nt);
  c->J.resize(nt);
  c->C.resize(nt);
  for (size_t t = 0; t < nt; ++t) {
    const int Lt = std::get<0>(L.tables[t]), per = std::get<1>(L.tables[t]);
    const int nim = std::get<2>(L.tables[t]);
    const double D = std::get<3>(L.tables[t]);  // table_d of the chains
    build_halfset(Lt, per, c->hd[t]);
    const int64_t K = static_cast<int64_t>(c->hd[t].size());
    if (K != L.table_K[t]) return fail(SCO_EINTERNAL);
    uint32_t* d_hd = at<uint32_t>(c, L.off_hd[t]);
    double* d_J = at<double>(c, L.off_J[t]);
    if (hipMemcpyAsync(d_hd, c->hd[t].data(), sizeof(uint32_t) * K, hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return fail(SCO_EHIP);
    if (sco_dev::table_j(c->stream, d_hd, static_cast<int>(K), Lt, per, nim, D, d_J) != hipSuccess)
      return fail(SCO_EHIP);
    c->J[t].resize(K);
    if (hipMemcpyAsync(c->J[t].data(), d_J, sizeof(double) * K, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      return fail(SCO_EHIP);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(SCO_EHIP);
    c->C[t].resize(K);
    double acc = 0.0;
    for (int64_t m = 0; m < K; ++m) {
      acc += c->J[t][m];
      c->C[t][m] = acc;
    }
    const double Ctop = c->C[t][K - 1];
    const double stepb = Ctop / kNB;
    std::vector<int32_t> guide(kNB + 1);
    for (int b = 0; b <= kNB; ++b) {
      const double thr = static_cast<double>(b) * stepb;
      const auto it = std::lower_bound(c->C[t].begin(), c->C[t].end(), thr);
      guide[b] = it == c->C[t].end() ? static_cast<int32_t>(K - 1) : static_cast<int32_t>(it - c->C[t].begin());
    }
    if (hipMemcpyAsync(at<double>(c, L.off_C[t]), c->C[t].data(), sizeof(double) * K, hipMemcpyHostToDevice,
                       c->stream) != hipSuccess ||
        hipMemcpyAsync(at<int32_t>(c, L.off_guide[t]), guide.data(), sizeof(int32_t) * (kNB + 1),
                       hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return fail(SCO_EHIP);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(SCO_EHIP);
  }

  // per-chain switching and pseudo-interaction columns (Eqs. 2-3) and descriptors
  c->theta.resize(n_chains);
  c->delta.resize(n_chains);
  c->cd.resize(n_chains);
  std::vector<int32_t> chunk_chain(L.nchunks, 0);
  std::vector<int64_t> src_base(n_chains, 0);
  int64_t sb = 0;
  for (int ci = 0; ci < n_chains; ++ci) {
    const sco_chain_params& p = params[ci];
    const int t = L.chain_table[ci];
    const int64_t K = L.table_K[t];
    const bool hard = p.kappa == 1.0;
    ChainDesc d{};
    d.L = p.L;
    d.N = p.L * p.L;
    d.K = static_cast<int32_t>(K);
    d.periodic = p.periodic ? 1 : 0;
    d.vbase = L.vbase[ci];
    d.hd = at<uint32_t>(c, L.off_hd[t]);
    d.J = at<double>(c, L.off_J[t]);
    d.C = at<double>(c, L.off_C[t]);
    d.guide = at<int32_t>(c, L.off_guide[t]);
    d.C_top = c->C[t][K - 1];
    d.guide_inv = static_cast<double>(kNB) / d.C_top;
    d.nguide = kNB;
    d.twoJ = 2.0 * p.J;
    d.inv_L = 1.0 / p.L;
    d.twoJ32 = static_cast<float>(d.twoJ);
    d.twoJ32_exact = static_cast<double>(d.twoJ32) == d.twoJ ? 1 : 0;
    d.seed = p.seed;
    d.chain_id = p.chain_id;
    d.model = p.model;
    d.hard = hard && p.model == SCO_MODEL_ISING ? 1 : 0;
    d.precision = p.precision;
    d.n_sw = p.n_sw;
    if (p.model == SCO_MODEL_HEIS) {
      d.hden = at<double>(c, L.off_theta[ci]);
    } else if (!hard) {
      d.theta = at<double>(c, L.off_theta[ci]);
      d.delta = at<double>(c, L.off_delta[ci]);
      d.delta32 = at<float>(c, L.off_delta32[ci]);
    }
    c->cd[ci] = d;
    const int tr = temperature_tables(c, ci, p.T);
    if (tr) return fail(tr);
    const int64_t ch0 = L.vbase[ci] / SCO_CHUNK, chn = (static_cast<int64_t>(d.N) + SCO_CHUNK - 1) / SCO_CHUNK;
    for (int64_t ch = ch0; ch < ch0 + chn; ++ch) chunk_chain[ch] = ci;
    src_base[ci] = sb;
    sb += d.N;
    c->nsw_max = std::max(c->nsw_max, p.n_sw);
  }
  if (hipMemcpyAsync(at<ChainDesc>(c, L.off_cd), c->cd.data(), sizeof(ChainDesc) * n_chains, hipMemcpyHostToDevice,
                     c->stream) != hipSuccess ||
      hipMemcpyAsync(at<int32_t>(c, L.off_chunk), chunk_chain.data(), sizeof(int32_t) * L.nchunks,
                     hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(at<int64_t>(c, L.off_srcbase), src_base.data(), sizeof(int64_t) * n_chains,
                     hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return fail(SCO_EHIP);
  double* spin3 = c->model == SCO_MODEL_HEIS ? at<double>(c, L.off_spin3) : nullptr;
  if (sco_dev::init_spins(c->stream, at<ChainDesc>(c, L.off_cd), at<int32_t>(c, L.off_chunk),
                          at<int64_t>(c, L.off_srcbase), dev_init_spins, at<int8_t>(c, L.off_spin), spin3,
                          L.G) != hipSuccess)
    return fail(SCO_EHIP);
  // an empty graph until the first switching (row offsets of zero length)
  if (hipMemsetAsync(at<int32_t>(c, L.off_row), 0, sizeof(int32_t) * (L.G + 1), c->stream) != hipSuccess ||
      hipMemsetAsync(at<int32_t>(c, L.off_deg), 0, sizeof(int32_t) * L.G, c->stream) != hipSuccess ||
      hipMemsetAsync(at<int32_t>(c, L.off_fill), 0, sizeof(int32_t) * L.G, c->stream) != hipSuccess)
    return fail(SCO_EHIP);

  StepArgs& a = c->args;
  a.cd = at<ChainDesc>(c, L.off_cd);
  a.st = at<ChainState>(c, L.off_st);
  a.sync = at<SyncWords>(c, L.off_sync);
  a.chunk_chain = at<int32_t>(c, L.off_chunk);
  a.spin = at<int8_t>(c, L.off_spin);
  a.spin3 = spin3;
  a.deg = at<int32_t>(c, L.off_deg);
  a.row_ptr = at<int32_t>(c, L.off_row);
  a.fill = at<int32_t>(c, L.off_fill);
  a.own = reinterpret_cast<uint16_t*>(a.fill);
  a.ea = at<int32_t>(c, L.off_ea);
  a.eb = at<int32_t>(c, L.off_eb);
  a.em = at<int32_t>(c, L.off_em);
  a.er = at<int32_t>(c, L.off_er);
  a.col = at<int32_t>(c, L.off_col);
  a.attr = at<int32_t>(c, L.off_attr);
  a.color = at<uint16_t>(c, L.off_color);
  a.kw_word = at<uint32_t>(c, L.off_word);
  a.rec = at<int4>(c, L.off_rec);
  a.ecount = at<uint32_t>(c, L.off_ecount);
  a.trace = nullptr;
  a.scan_agg = at<long long>(c, L.off_agg);
  a.G = L.G;
  a.nchunks = static_cast<int32_t>(L.nchunks);
  a.n_chains = n_chains;
  a.cap_und = L.cap_und;
  a.any_fp32 = 0;
  for (int ci = 0; ci < n_chains; ++ci)
    if (params[ci].precision == 1) a.any_fp32 = 1;
  const int maxb = sco_dev::step_max_blocks();
  if (maxb <= 0) return fail(SCO_EHIP);
  c->max_blocks = std::min(maxb, SCO_MAX_BLOCKS);
  c->blocks = c->max_blocks;
  c->args.tile_limit = SCO_TILE_MAX;
  {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      c->wall_mhz = khz / 1000.0;
  }
  // colouring words start at level 31, which no colouring reaches (they are all
  // rewritten by the tile levels of every colouring before any level reads them)
  if (hipMemsetAsync(at<uint32_t>(c, L.off_word), 0xFF, sizeof(uint32_t) * L.G, c->stream) != hipSuccess)
    return fail(SCO_EHIP);
  if (hipMemsetAsync(at<uint16_t>(c, L.off_color), 0, sizeof(uint16_t) * L.G, c->stream) != hipSuccess)
    return fail(SCO_EHIP);
  {
    const int mr = refresh_mag(c);
    if (mr) return fail(mr);
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(SCO_EHIP);
  *out = c;
  return SCO_OK;
}
}  // namespace

int sco_init(sco_ctx** out, const sco_chain_params* params, int n_chains, void* dev_workspace,
             size_t workspace_bytes, const int8_t* dev_init_spins, void* stream) {
  return init_impl(out, params, n_chains, dev_workspace, workspace_bytes, dev_init_spins, stream, false);
}

int sco_switch(sco_ctx* c, uint64_t step) {
  if (!c) return SCO_EINVAL;
  HIP_TRY(hipEventRecord(c->ev[0], c->stream));
  int rc = launch(c, PH_SWITCH, step, 0);
  HIP_TRY(hipEventRecord(c->ev[1], c->stream));
  if (rc == SCO_OK) c->graph_state = 1;
  return rc;
}

int sco_color(sco_ctx* c) {
  if (!c) return SCO_EINVAL;
  if (c->graph_state < 1) return SCO_EINVAL;  // no bond graph to colour yet
  HIP_TRY(hipEventRecord(c->ev[1], c->stream));
  int rc = launch(c, PH_COLOR, 0, 0);
  HIP_TRY(hipEventRecord(c->ev[2], c->stream));
  if (rc == SCO_OK) c->graph_state = 2;
  return rc;
}

int sco_sweep(sco_ctx* c, uint64_t step, int n_sw) {
  if (!c || n_sw < 0) return SCO_EINVAL;
  if (c->graph_state != 2) return SCO_EINVAL;  // the colouring must match the bond graph
  HIP_TRY(hipEventRecord(c->ev[2], c->stream));
  int rc = launch(c, PH_SWEEP, step, n_sw);
  HIP_TRY(hipEventRecord(c->ev[3], c->stream));
  return rc;
}

int sco_step(sco_ctx* c, uint64_t step) {
  if (!c) return SCO_EINVAL;
  return run_steps(c, step, 1);
}

int sco_run(sco_ctx* c, uint64_t first_step, int n_steps) {
  if (!c || n_steps < 0) return SCO_EINVAL;
  const int rc = run_steps(c, first_step, n_steps);
  if (rc) return rc;
  // a step that raised a flag ended at a barrier and every later launch did nothing
  return n_steps > 0 ? consume_flags(c) : SCO_OK;
}


int sco_run_noalloc(const sco_chain_params* params, int n_chains, const int8_t* dev_spins_in,
                    int8_t* dev_spins_out, uint64_t first_step, int n_steps, sco_obs* host_obs, void* stream) {
  if (!params || n_chains <= 0 || n_chains > SCO_MAXCHAINS || !dev_spins_out || n_steps < 0) return SCO_EINVAL;
  if (params[0].model != SCO_MODEL_ISING) return SCO_EINVAL;  // int8 spins in and out
  size_t need = 0;
  int rc = sco_workspace_size(params, n_chains, &need);
  if (rc) return rc;
  if (need > static_cast<size_t>(SCO_NOALLOC_BYTES)) return SCO_ENOSPC;
  void* scratch = nullptr;  // this GPU's copy of the library's static scratch array
  if (sco_dev::noalloc_scratch(&scratch) != hipSuccess || !scratch) return SCO_EHIP;
  sco_ctx* c = nullptr;
  rc = init_impl(&c, params, n_chains, scratch, SCO_NOALLOC_BYTES, dev_spins_in, stream, true);
  if (rc) return rc;
  rc = sco_run(c, first_step, n_steps);
  if (rc == SCO_OK && host_obs) rc = sco_observables(c, host_obs);
  // the chains' spins, concatenated without padding
  int64_t off = 0;
  for (int ci = 0; ci < n_chains && rc == SCO_OK; ++ci) {
    const ChainDesc& d = c->cd[ci];
    if (hipMemcpyAsync(dev_spins_out + off, at<int8_t>(c, c->lay.off_spin) + d.vbase, d.N, hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess)
      rc = SCO_EHIP;
    off += d.N;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess && rc == SCO_OK) rc = SCO_EHIP;
  sco_destroy(c);
  return rc;
}

namespace {
void graph_release(sco_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
  c->graph_nodes.clear();
  c->graph_args.clear();
}

// A graph of n full-step kernel nodes, each depending on the one before, every node
// a cooperative launch of the schedule's grid.
// the phases of node k of the step graph (one node per step, or three)
uint32_t graph_node_phases(const sco_ctx* c, int k) {
  if (c->step_fused) return PH_SWITCH | PH_COLOR | PH_SWEEP;
  const uint32_t ph[3] = {PH_SWITCH, PH_COLOR, PH_SWEEP};
  return ph[k % 3];
}

int graph_build(sco_ctx* c, int n_steps) {
  graph_release(c);
  if (hipGraphCreate(&c->graph, 0) != hipSuccess) return SCO_EHIP;
  const int n = n_steps * (c->step_fused ? 1 : 3);
  c->graph_nodes.resize(n);
  c->graph_args.assign(n, c->args);
  for (int s = 0; s < n; ++s) {
    void* kargs[] = {&c->graph_args[s]};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(sco_dev::step_kernel_for(graph_node_phases(c, s), c->model));
    kp.gridDim = dim3(c->blocks);
    kp.blockDim = dim3(SCO_CHUNK);
    kp.sharedMemBytes = 0;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    const hipGraphNode_t* dep = s > 0 ? &c->graph_nodes[s - 1] : nullptr;
    if (hipGraphAddKernelNode(&c->graph_nodes[s], c->graph, dep, s > 0 ? 1 : 0, &kp) != hipSuccess) {
      graph_release(c);
      return SCO_EHIP;
    }
    hipKernelNodeAttrValue v{};
    v.cooperative = 1;
    if (hipGraphKernelNodeSetAttribute(c->graph_nodes[s], hipKernelNodeAttributeCooperative, &v) != hipSuccess) {
      graph_release(c);
      return SCO_EHIP;
    }
  }
  if (hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0) != hipSuccess) {
    graph_release(c);
    return SCO_EHIP;
  }
  c->graph_blocks = c->blocks;
  return SCO_OK;
}
}  // namespace

int sco_run_graph(sco_ctx* c, uint64_t first_step, int n_steps) {
  if (!c || n_steps < 0) return SCO_EINVAL;
  if (n_steps == 0) return SCO_OK;
  if (first_step + static_cast<uint64_t>(n_steps) - 1 > 0xFFFFFFFFull) return SCO_EINVAL;
  const int per = c->step_fused ? 1 : 3;
  if (!c->graph_exec || static_cast<int>(c->graph_nodes.size()) != n_steps * per || c->graph_blocks != c->blocks) {
    const int rc = graph_build(c, n_steps);
    if (rc) return rc;
  }
  if (c->blocks != c->launched_blocks) {
    HIP_TRY(hipMemsetAsync(at<SyncWords>(c, c->lay.off_sync), 0, offsetof(SyncWords, flags), c->stream));
    c->launched_blocks = c->blocks;
  }
  // this replay's step indices (and the current tile limit) into the nodes' arguments
  for (int k = 0; k < n_steps * per; ++k) {
    StepArgs& a = c->graph_args[k];
    a = c->args;
    a.trace = nullptr;
    a.nsw_override = -1;
    a.nsw_max = c->nsw_max;
    a.step = static_cast<uint32_t>(first_step + static_cast<uint64_t>(k / per));
    void* kargs[] = {&a};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(sco_dev::step_kernel_for(graph_node_phases(c, k), c->model));
    kp.gridDim = dim3(c->blocks);
    kp.blockDim = dim3(SCO_CHUNK);
    kp.kernelParams = kargs;
    HIP_TRY(hipGraphExecKernelNodeSetParams(c->graph_exec, c->graph_nodes[k], &kp));
  }
  HIP_TRY(hipGraphLaunch(c->graph_exec, c->stream));
  c->graph_state = 2;
  return consume_flags(c);
}

int sco_set_step_form(sco_ctx* c, int fused) {
  if (!c || fused < 0 || fused > 1) return SCO_EINVAL;
  if (c->step_fused != fused) graph_release(c);
  c->step_fused = fused;
  return SCO_OK;
}

int sco_set_temperature(sco_ctx* c, int chain, double T) {
  if (!c || chain < -1 || chain >= c->n || !(T > 0.0) || !std::isfinite(T)) return SCO_EINVAL;
  const int c0 = chain < 0 ? 0 : chain, c1 = chain < 0 ? c->n : chain + 1;
  for (int ci = c0; ci < c1; ++ci) {
    const int rc = temperature_tables(c, ci, T);
    if (rc) return rc;
  }
  HIP_TRY(hipMemcpyAsync(at<ChainDesc>(c, c->lay.off_cd) + c0, c->cd.data() + c0, sizeof(ChainDesc) * (c1 - c0),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return SCO_OK;
}

int sco_anneal(sco_ctx* c, const double* temps, int n_stages, int equil_steps, int meas_steps,
               uint64_t first_step, sco_stage* out) {
  if (!c || !temps || !out || n_stages < 0 || equil_steps < 0 || meas_steps < 0) return SCO_EINVAL;
  for (int64_t i = 0; i < static_cast<int64_t>(n_stages) * c->n; ++i)
    if (!(temps[i] > 0.0) || !std::isfinite(temps[i])) return SCO_EINVAL;
  const Layout& L = c->lay;
  AnnealAcc* acc = at<AnnealAcc>(c, L.off_acc);
  std::vector<AnnealAcc> h(c->n);
  std::vector<ChainState> st0(c->n), st1(c->n);
  uint64_t step = first_step;
  for (int k = 0; k < n_stages; ++k) {
    for (int ci = 0; ci < c->n; ++ci) {
      const int rc = temperature_tables(c, ci, temps[static_cast<int64_t>(k) * c->n + ci]);
      if (rc) return rc;
    }
    HIP_TRY(hipMemcpyAsync(at<ChainDesc>(c, L.off_cd), c->cd.data(), sizeof(ChainDesc) * c->n,
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(st0.data(), at<ChainState>(c, L.off_st), sizeof(ChainState) * c->n,
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    int rc = sco_run(c, step, equil_steps);
    if (rc) return rc;
    step += static_cast<uint64_t>(equil_steps);
    HIP_TRY(hipMemsetAsync(acc, 0, sizeof(AnnealAcc) * c->n, c->stream));
    for (int s = 0; s < meas_steps; ++s, ++step) {
      rc = launch(c, PH_SWITCH | PH_COLOR | PH_SWEEP, step, -1);
      if (rc) return rc;
      HIP_TRY(sco_dev::anneal_acc(c->stream, at<ChainState>(c, L.off_st), acc, c->n));
    }
    c->graph_state = 2;
    rc = consume_flags(c);  // synchronises
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(h.data(), acc, sizeof(AnnealAcc) * c->n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(st1.data(), at<ChainState>(c, L.off_st), sizeof(ChainState) * c->n,
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<sco_obs> obs(c->n);
    rc = sco_observables(c, obs.data());
    if (rc) return rc;
    for (int ci = 0; ci < c->n; ++ci) {
      sco_stage& o = out[static_cast<int64_t>(k) * c->n + ci];
      const double N = static_cast<double>(c->cd[ci].N);
      const double ns = static_cast<double>(h[ci].samples);
      o.T = c->params[ci].T;
      o.E = obs[ci].E;
      o.M = obs[ci].M;
      o.m_phi = obs[ci].m_phi;
      o.samples = static_cast<int64_t>(h[ci].samples);
      const bool ising = c->model == SCO_MODEL_ISING;  // the magnetisation is an Ising sum
      o.abs_m = ising && ns > 0 ? static_cast<double>(h[ci].abs_m) / ns / N : 0.0;
      o.m2 = ising && ns > 0 ? static_cast<double>(h[ci].m2) / ns / (N * N) : 0.0;
      o.k_mean = ns > 0 ? static_cast<double>(h[ci].bonds) / ns / N : 0.0;
      o.delta_sco_mean = ns > 0 ? static_cast<double>(h[ci].delta_sco) / ns : 0.0;
      o.delta_union_mean = ns > 0 ? static_cast<double>(h[ci].delta_union) / ns : 0.0;
      const double att = static_cast<double>(st1[ci].attempts - st0[ci].attempts);
      o.acceptance = att > 0 ? static_cast<double>(st1[ci].accepted - st0[ci].accepted) / att : 0.0;
    }
  }
  return SCO_OK;
}

int sco_set_fenced_sweeps(sco_ctx* c, int on) {
  if (!c || on < 0 || on > 1) return SCO_EINVAL;
  c->args.fenced_classes = on;
  return SCO_OK;
}

int sco_set_round_cap(sco_ctx* c, int cap) {
  if (!c || cap < 0) return SCO_EINVAL;
  c->args.round_cap = cap;
  return SCO_OK;
}

int sco_class_sizes(sco_ctx* c, int chain, int64_t* sizes, int* n_colors) {
  if (!c || chain < 0 || chain >= c->n || !sizes) return SCO_EINVAL;
  const int fr = consume_flags(c);
  if (fr) return fr;
  if (c->graph_state < 2) return SCO_EINVAL;  // no colouring of the current graph
  unsigned long long* d = at<unsigned long long>(c, c->lay.off_csz);
  HIP_TRY(hipMemsetAsync(d, 0, sizeof(unsigned long long) * 256, c->stream));
  const ChainDesc& cd = c->cd[chain];
  HIP_TRY(sco_dev::class_sizes(c->stream, at<uint16_t>(c, c->lay.off_color), cd.vbase, cd.N, d));
  std::vector<unsigned long long> h(256);
  HIP_TRY(hipMemcpyAsync(h.data(), d, sizeof(unsigned long long) * 256, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  int last = 0;
  for (int k = 0; k < 256; ++k) {
    sizes[k] = static_cast<int64_t>(h[k]);
    if (h[k]) last = k + 1;
  }
  if (n_colors) *n_colors = last;
  return SCO_OK;
}

int sco_bond_histogram(sco_ctx* c, int chain, int64_t* counts) {
  if (!c || chain < 0 || chain >= c->n || !counts) return SCO_EINVAL;
  const int fr = consume_flags(c);
  if (fr) return fr;
  if (c->graph_state < 1) return SCO_EINVAL;
  const ChainDesc& cd = c->cd[chain];
  unsigned long long* d = at<unsigned long long>(c, c->lay.off_prod);  // K entries fit (maxK doubles)
  HIP_TRY(hipMemsetAsync(d, 0, sizeof(unsigned long long) * cd.K, c->stream));
  HIP_TRY(sco_dev::bond_hist(c->stream, at<int32_t>(c, c->lay.off_row), at<int32_t>(c, c->lay.off_col),
                             at<int32_t>(c, c->lay.off_attr), cd.vbase, cd.N, d));
  HIP_TRY(hipMemcpyAsync(counts, d, sizeof(int64_t) * cd.K, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return SCO_OK;
}

int sco_survival_by_distance(sco_ctx* c, int chain, double* r, double* p_survive, int max, int* n) {
  if (!c || chain < 0 || chain >= c->n || !n || max < 0) return SCO_EINVAL;
  const ChainDesc& cd = c->cd[chain];
  std::vector<int64_t> counts(cd.K);
  const int rc = sco_bond_histogram(c, chain, counts.data());
  if (rc) return rc;
  const int t = c->lay.chain_table[chain];
  const int L = cd.L, h = L / 2;
  int k = 0;
  int64_t cur_r2 = -1;
  double bonds = 0.0, pairs = 0.0;
  auto emit = [&]() {
    if (cur_r2 >= 0 && pairs > 0) {
      if (k < max) {
        if (r) r[k] = std::sqrt(static_cast<double>(cur_r2));
        if (p_survive) p_survive[k] = bonds / pairs;
      }
      ++k;
    }
  };
  // the table is sorted by r^2: one bin per distance
  for (int64_t m = 0; m < cd.K; ++m) {
    const uint32_t w = c->hd[t][m];
    const int dx = static_cast<int16_t>(w & 0xFFFFu), dy = static_cast<int16_t>(w >> 16);
    const int64_t r2 = static_cast<int64_t>(dx) * dx + static_cast<int64_t>(dy) * dy;
    if (r2 != cur_r2) {
      emit();
      cur_r2 = r2;
      bonds = pairs = 0.0;
    }
    // owned pairs of the displacement (the owner rules of the half set)
    double np;
    if (cd.periodic) {
      const bool sc = (dy == 0 && dx == h) || (dy == h && (dx == 0 || dx == h));
      np = sc ? 0.5 * cd.N : static_cast<double>(cd.N);
    } else {
      np = static_cast<double>(L - std::abs(dx)) * static_cast<double>(L - dy);
    }
    bonds += static_cast<double>(counts[m]);
    pairs += np;
  }
  emit();
  *n = k;
  return SCO_OK;
}

int sco_validate(sco_ctx* c, int chain, int64_t* failed) {
  if (!c || chain < 0 || chain >= c->n) return SCO_EINVAL;
  const int fr = consume_flags(c);
  if (fr) return fr;
  const ChainDesc& d = c->cd[chain];
  const Layout& L = c->lay;
  const int N = d.N, Ls = d.L;
  int64_t bad = 0;
  // spins
  if (c->model == SCO_MODEL_ISING) {
    std::vector<int8_t> s(N);
    std::vector<ChainState> st(c->n);
    HIP_TRY(hipMemcpyAsync(s.data(), at<int8_t>(c, L.off_spin) + d.vbase, N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(st.data(), at<ChainState>(c, L.off_st), sizeof(ChainState) * c->n, hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    long long m = 0;
    for (int v = 0; v < N; ++v) {
      if (s[v] != 1 && s[v] != -1) bad |= 1;
      m += s[v];
    }
    if (m != st[chain].mag) bad |= 2;
  } else {
    std::vector<double> s3(3 * static_cast<size_t>(N));
    HIP_TRY(hipMemcpyAsync(s3.data(), at<double>(c, L.off_spin3) + 3 * d.vbase, sizeof(double) * 3 * N,
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int v = 0; v < N; ++v) {
      const double x = s3[3 * v], y = s3[3 * v + 1], z = s3[3 * v + 2];
      const double n2 = x * x + y * y + z * z;
      if (!std::isfinite(n2) || std::fabs(n2 - 1.0) > 1e-12) bad |= 1;
    }
  }
  if (c->graph_state >= 1) {
    std::vector<int32_t> rp(N + 1);
    HIP_TRY(hipMemcpyAsync(rp.data(), at<int32_t>(c, L.off_row) + d.vbase, sizeof(int32_t) * (N + 1),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const int32_t e0 = rp[0], e1 = rp[N];
    bool rows_ok = e0 >= 0 && e1 >= e0 && static_cast<int64_t>(e1) <= 2 * static_cast<int64_t>(L.cap_und);
    for (int v = 0; v < N && rows_ok; ++v) rows_ok = rp[v + 1] >= rp[v];
    if (!rows_ok) bad |= 4;
    std::vector<int32_t> col, attr;
    if (rows_ok && e1 > e0) {
      col.resize(e1 - e0);
      attr.resize(e1 - e0);
      HIP_TRY(hipMemcpyAsync(col.data(), at<int32_t>(c, L.off_col) + e0, sizeof(int32_t) * (e1 - e0),
                             hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipMemcpyAsync(attr.data(), at<int32_t>(c, L.off_attr) + e0, sizeof(int32_t) * (e1 - e0),
                             hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      for (auto& x : col) x -= static_cast<int32_t>(d.vbase);
      for (int v = 0; v < N; ++v)
        for (int e = rp[v] - e0; e < rp[v + 1] - e0; ++e) {
          const int u = col[e];
          if (u < 0 || u >= N || u == v || attr[e] < 0 || attr[e] >= d.K ||
              (e > rp[v] - e0 && col[e - 1] >= u)) {
            bad |= 8;
            continue;
          }
          // the reverse direction, with the same displacement index
          const int a0 = rp[u] - e0, a1 = rp[u + 1] - e0;
          const auto it = std::lower_bound(col.begin() + a0, col.begin() + a1, v);
          if (it == col.begin() + a1 || *it != v || attr[it - col.begin()] != attr[e]) bad |= 16;
        }
    }
    if (c->graph_state >= 2 && rows_ok) {
      std::vector<uint16_t> cl(N);
      std::vector<ChainState> st(c->n);
      HIP_TRY(hipMemcpyAsync(cl.data(), at<uint16_t>(c, L.off_color) + d.vbase, sizeof(uint16_t) * N,
                             hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipMemcpyAsync(st.data(), at<ChainState>(c, L.off_st), sizeof(ChainState) * c->n, hipMemcpyDeviceToHost,
                             c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      const int palette = c->args.coloring == SCO_COLOR_CHECKER ? 2 * st[chain].q : st[chain].q;
      for (int v = 0; v < N; ++v) {
        if (cl[v] >= palette) bad |= 32;
        const int x = v % Ls, y = v / Ls;
        int nb[4] = {-1, -1, -1, -1};
        if (d.periodic) {
          nb[0] = y * Ls + (x + 1) % Ls;
          nb[2] = ((y + 1) % Ls) * Ls + x;
        } else {
          if (x + 1 < Ls) nb[0] = v + 1;
          if (y + 1 < Ls) nb[2] = v + Ls;
        }
        for (int t = 0; t < 4; ++t)
          if (nb[t] >= 0 && cl[nb[t]] == cl[v]) bad |= 32;
        for (int e = rp[v] - e0; e < rp[v + 1] - e0 && !col.empty(); ++e)
          if (col[e] >= 0 && col[e] < N && cl[col[e]] == cl[v]) bad |= 32;
      }
    }
  }
  if (failed) *failed = bad;
  return bad ? SCO_EINTERNAL : SCO_OK;
}

int sco_get_flags(sco_ctx* c, int64_t* last, int64_t* seen) {
  if (!c) return SCO_EINVAL;
  if (last) *last = c->last_flags;
  if (seen) *seen = c->flags_seen;
  return SCO_OK;
}

int sco_set_schedule(sco_ctx* c, int blocks, int tile_limit) {
  if (!c) return SCO_EINVAL;
  if (blocks == 0) blocks = c->max_blocks;
  if (tile_limit == 0) tile_limit = SCO_TILE_MAX;
  if (blocks < 1 || blocks > c->max_blocks || tile_limit < 64 || tile_limit > SCO_TILE_MAX) return SCO_EINVAL;
  c->blocks = blocks;
  c->args.tile_limit = tile_limit;
  return SCO_OK;
}

int sco_set_coloring(sco_ctx* c, int mode) {
  if (!c || mode < SCO_COLOR_KW || mode > SCO_COLOR_BCR) return SCO_EINVAL;
  c->args.coloring = mode;
  if (c->graph_state == 2) c->graph_state = 1;  // the colouring of the current graph is stale
  return SCO_OK;
}

int sco_get_schedule(sco_ctx* c, int* blocks, int* tile_limit) {
  if (!c) return SCO_EINVAL;
  if (blocks) *blocks = c->blocks;
  if (tile_limit) *tile_limit = c->args.tile_limit;
  return SCO_OK;
}

int sco_autotune(sco_ctx* c, int trial_steps, int* blocks, int* tile_limit, float* ms_per_step) {
  if (!c || trial_steps < 1 || trial_steps > 1000) return SCO_EINVAL;
  const int fr = consume_flags(c);
  if (fr) return fr;
  const Layout& L = c->lay;
  // the chain's state before the trials: spins and counters
  HIP_TRY(hipMemcpyAsync(at<int8_t>(c, L.off_spin_bak), at<int8_t>(c, L.off_spin), L.G, hipMemcpyDeviceToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(at<ChainState>(c, L.off_st_bak), at<ChainState>(c, L.off_st), sizeof(ChainState) * c->n,
                         hipMemcpyDeviceToDevice, c->stream));
  const int cand_blocks[3] = {c->max_blocks, (c->max_blocks * 3) / 4, c->max_blocks / 2};
  const int cand_tiles[3] = {SCO_TILE_MAX, SCO_TILE_MAX / 2, SCO_TILE_MAX / 4};
  float best = -1.0f;
  int best_b = c->blocks, best_t = c->args.tile_limit;
  for (int bi = 0; bi < 3; ++bi)
    for (int ti = 0; ti < 3; ++ti) {
      const int b = cand_blocks[bi];
      if (b < 1 || (bi > 0 && b == cand_blocks[bi - 1])) continue;
      c->blocks = b;
      c->args.tile_limit = cand_tiles[ti];
      // trial steps from the saved state, with step counters no chain uses
      HIP_TRY(hipMemcpyAsync(at<int8_t>(c, L.off_spin), at<int8_t>(c, L.off_spin_bak), L.G,
                             hipMemcpyDeviceToDevice, c->stream));
      int rc = launch(c, PH_SWITCH | PH_COLOR | PH_SWEEP, 0xFFFFFF00u, -1);  // warm-up
      HIP_TRY(hipEventRecord(c->ev[0], c->stream));
      for (int s = 0; s < trial_steps && rc == SCO_OK; ++s)
        rc = launch(c, PH_SWITCH | PH_COLOR | PH_SWEEP, 0xFFFFFF01u + static_cast<uint32_t>(s), -1);
      HIP_TRY(hipEventRecord(c->ev[1], c->stream));
      if (rc) return rc;
      HIP_TRY(hipEventSynchronize(c->ev[1]));
      const int f = consume_flags(c);
      if (f) return f;
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
      ms /= static_cast<float>(trial_steps);
      if (best < 0.f || ms < best) {
        best = ms;
        best_b = b;
        best_t = cand_tiles[ti];
      }
    }
  c->blocks = best_b;
  c->args.tile_limit = best_t;
  HIP_TRY(hipMemcpyAsync(at<int8_t>(c, L.off_spin), at<int8_t>(c, L.off_spin_bak), L.G, hipMemcpyDeviceToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(at<ChainState>(c, L.off_st), at<ChainState>(c, L.off_st_bak), sizeof(ChainState) * c->n,
                         hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  // the trials left their own bond graph: a colouring or sweep needs a new switching
  c->graph_state = 0;
  if (blocks) *blocks = best_b;
  if (tile_limit) *tile_limit = best_t;
  if (ms_per_step) *ms_per_step = best;
  return SCO_OK;
}

int sco_phase_times(sco_ctx* c, float* out3) {
  if (!c || !out3) return SCO_EINVAL;
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int i = 0; i < 3; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]) != hipSuccess) ms = -1.f;
    out3[i] = ms;
  }
  return SCO_OK;
}

int sco_trace(sco_ctx* c, int enable) {
  if (!c) return SCO_EINVAL;
  c->trace_on = enable != 0;
  return SCO_OK;
}

int sco_trace_read(sco_ctx* c, int32_t* ids, double* us, int max, int* n) {
  if (!c || !n || max < 0) return SCO_EINVAL;
  std::vector<unsigned long long> t(SCO_TRACE_SLOTS);
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(t.data(), at<unsigned long long>(c, c->lay.off_trace), sizeof(unsigned long long) * t.size(),
                    hipMemcpyDeviceToHost));
  const int cnt = static_cast<int>(std::min<unsigned long long>(t[0], (SCO_TRACE_SLOTS - 1) / 2));
  *n = cnt;
  for (int i = 0; i < cnt && i < max; ++i) {
    if (ids) ids[i] = static_cast<int32_t>(t[2 * i + 1]);
    if (us)  // marks: microseconds since the first mark; ids >= 900000 carry a raw value
      us[i] = t[2 * i + 1] >= 900000 ? static_cast<double>(t[2 * i + 2])
                                     : static_cast<double>(t[2 * i + 2] - t[2]) / c->wall_mhz;
  }
  return SCO_OK;
}

int sco_reset_counters(sco_ctx* c) {
  if (!c) return SCO_EINVAL;
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::vector<ChainState> st(c->n);
  HIP_TRY(hipMemcpy(st.data(), at<ChainState>(c, c->lay.off_st), sizeof(ChainState) * c->n, hipMemcpyDeviceToHost));
  for (auto& s : st) s.accepted = s.attempts = s.rechecks = s.near_ties = 0;
  HIP_TRY(hipMemcpy(at<ChainState>(c, c->lay.off_st), st.data(), sizeof(ChainState) * c->n, hipMemcpyHostToDevice));
  c->flags_seen = 0;
  c->last_flags = 0;
  return SCO_OK;
}

namespace {
int observables_impl(sco_ctx* c, sco_obs* out, bool dipolar) {
  if (!c || !out) return SCO_EINVAL;
  const int fr = consume_flags(c);
  const Layout& L = c->lay;
  unsigned long long* d_obs = at<unsigned long long>(c, L.off_obs);
  uint32_t* d_used = at<uint32_t>(c, L.off_used);
  HIP_TRY(hipMemsetAsync(d_obs, 0, sizeof(unsigned long long) * 2 * c->n, c->stream));
  HIP_TRY(hipMemsetAsync(d_used, 0, sizeof(uint32_t) * SCO_QWORDS * c->n, c->stream));
  HIP_TRY(sco_dev::obs_basic(c->stream, at<ChainDesc>(c, L.off_cd), at<int32_t>(c, L.off_chunk),
                             at<int8_t>(c, L.off_spin), at<uint16_t>(c, L.off_color), d_obs, d_used, L.G));
  const bool heis = c->model == SCO_MODEL_HEIS;
  std::vector<double> hres(2 * c->n, 0.0);  // Heisenberg: exchange sum, M_phi sum
  for (int ci = 0; ci < c->n && (dipolar || heis); ++ci) {
    const ChainDesc& d = c->cd[ci];
    if (heis) {
      const NttPlan fp = dipolar ? fft_plan(c->params[ci]) : NttPlan{};
      if (fp.n > 0) {
        const std::vector<double> tw = fft_twiddles(fp.n);
        HIP_TRY(hipMemcpyAsync(at<double>(c, L.off_ftw), tw.data(), sizeof(double) * tw.size(), hipMemcpyHostToDevice,
                               c->stream));
      }
      HIP_TRY(sco_dev::obs_heis(c->stream, at<ChainDesc>(c, L.off_cd), ci, d, at<double>(c, L.off_spin3),
                                at<double>(c, L.off_prod), at<double>(c, L.off_dpart), at<double>(c, L.off_dres) + ci,
                                at<double>(c, L.off_hpart), at<double>(c, L.off_hres), dipolar, &fp,
                                at<double2>(c, L.off_fft), at<double2>(c, L.off_ftw)));
      HIP_TRY(hipMemcpyAsync(&hres[2 * ci], at<double>(c, L.off_hres), 2 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      continue;
    }
    const NttPlan plan = ntt_plan(c->params[ci]);
    if (plan.n > 0) {
      const std::vector<uint32_t> tw = ntt_twiddles(plan);
      HIP_TRY(hipMemcpyAsync(at<uint32_t>(c, L.off_tw), tw.data(), sizeof(uint32_t) * tw.size(),
                             hipMemcpyHostToDevice, c->stream));
    }
    HIP_TRY(sco_dev::obs_dipolar(c->stream, d.hd, d.J, d.K, d.L, d.periodic, at<int8_t>(c, L.off_spin), d.vbase,
                                 at<uint32_t>(c, L.off_bits), at<double>(c, L.off_prod), at<double>(c, L.off_dpart),
                                 at<double>(c, L.off_dres) + ci, &plan, at<uint32_t>(c, L.off_ntt),
                                 at<uint32_t>(c, L.off_tw)));
    HIP_TRY(hipStreamSynchronize(c->stream));  // the twiddles of the next chain overwrite these
  }
  std::vector<ChainState> st(c->n);
  std::vector<unsigned long long> sums(2 * c->n);
  std::vector<double> edip(c->n);
  std::vector<uint32_t> used(SCO_QWORDS * c->n);
  HIP_TRY(hipMemcpyAsync(used.data(), d_used, sizeof(uint32_t) * used.size(), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(st.data(), at<ChainState>(c, L.off_st), sizeof(ChainState) * c->n, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(sums.data(), d_obs, sizeof(unsigned long long) * 2 * c->n, hipMemcpyDeviceToHost, c->stream));
  if (dipolar)
    HIP_TRY(hipMemcpyAsync(edip.data(), at<double>(c, L.off_dres), sizeof(double) * c->n, hipMemcpyDeviceToHost,
                           c->stream));
  else
    std::fill(edip.begin(), edip.end(), std::nan(""));
  HIP_TRY(hipStreamSynchronize(c->stream));
  int bad_mag = 0;
  for (int ci = 0; ci < c->n; ++ci) {
    sco_obs& o = out[ci];
    const ChainState& s = st[ci];
    o.M = static_cast<long long>(sums[2 * ci]);
    // the magnetisation the sweeps keep must equal the sum of the spins
    if (!heis && s.mag != o.M) bad_mag = 1;
    o.E_exchange = -c->params[ci].J * static_cast<double>(static_cast<long long>(sums[2 * ci + 1]));
    o.E_dipolar = edip[ci];
    o.E = o.E_exchange + o.E_dipolar;
    o.n_edges = s.n_edges / 2;
    o.delta_union = s.delta_union;
    o.q = s.q;
    int cu = 0;
    for (int w = 0; w < SCO_QWORDS; ++w) cu += __builtin_popcount(used[ci * SCO_QWORDS + w]);
    o.colors_used = c->graph_state == 2 ? cu : 0;
    o.kw_levels = s.M;
    int64_t r = 0;
    for (int p = 0; p < SCO_MAXLEVEL; ++p) r += s.kw_rounds[p];
    o.kw_rounds = r;
    o.accepted = static_cast<int64_t>(s.accepted);
    o.attempts = static_cast<int64_t>(s.attempts);
    o.rechecks = static_cast<int64_t>(s.rechecks);
    o.flags = c->flags_seen;
    o.near_ties = static_cast<int64_t>(s.near_ties);
    o.delta_sco = s.delta_sco;
    o.m_phi = 0.0;
    if (heis) {  // Eq. (6) with Heisenberg spins and Eq. (7) before its average
      o.M = 0;
      o.E_exchange = -c->params[ci].J * hres[2 * ci];
      o.E_dipolar = dipolar ? edip[ci] : std::nan("");
      o.E = o.E_exchange + o.E_dipolar;
      o.m_phi = hres[2 * ci + 1] / static_cast<double>(c->cd[ci].N);
    }
  }
  if (fr == SCO_OK && bad_mag) return SCO_EINTERNAL;
  return fr;
}
}  // namespace

int sco_observables(sco_ctx* c, sco_obs* out) { return observables_impl(c, out, true); }

int sco_counters(sco_ctx* c, sco_obs* out) { return observables_impl(c, out, false); }

int sco_get_spins3(sco_ctx* c, int chain, double* host_out) {
  if (!c || chain < 0 || chain >= c->n || !host_out || c->model != SCO_MODEL_HEIS) return SCO_EINVAL;
  const ChainDesc& d = c->cd[chain];
  HIP_TRY(hipMemcpyAsync(host_out, at<double>(c, c->lay.off_spin3) + 3 * d.vbase, sizeof(double) * 3 * d.N,
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return SCO_OK;
}

int sco_set_spins3(sco_ctx* c, int chain, const double* host_in) {
  if (!c || chain < 0 || chain >= c->n || !host_in || c->model != SCO_MODEL_HEIS) return SCO_EINVAL;
  const ChainDesc& d = c->cd[chain];
  for (int64_t i = 0; i < 3 * static_cast<int64_t>(d.N); ++i)
    if (!std::isfinite(host_in[i])) return SCO_EINVAL;
  HIP_TRY(hipMemcpyAsync(at<double>(c, c->lay.off_spin3) + 3 * d.vbase, host_in, sizeof(double) * 3 * d.N,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return SCO_OK;
}

int sco_get_spins(sco_ctx* c, int chain, int8_t* host_out) {
  if (!c || chain < 0 || chain >= c->n || !host_out || c->model != SCO_MODEL_ISING) return SCO_EINVAL;
  const ChainDesc& d = c->cd[chain];
  HIP_TRY(hipMemcpyAsync(host_out, at<int8_t>(c, c->lay.off_spin) + d.vbase, d.N, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return SCO_OK;
}

int sco_set_spins(sco_ctx* c, int chain, const int8_t* host_in) {
  if (!c || chain < 0 || chain >= c->n || !host_in || c->model != SCO_MODEL_ISING) return SCO_EINVAL;
  const ChainDesc& d = c->cd[chain];
  std::vector<int8_t> s(d.N);
  for (int v = 0; v < d.N; ++v) s[v] = host_in[v] > 0 ? 1 : -1;
  HIP_TRY(hipMemcpyAsync(at<int8_t>(c, c->lay.off_spin) + d.vbase, s.data(), d.N, hipMemcpyHostToDevice, c->stream));
  const int mr = refresh_mag(c);
  if (mr) return mr;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return SCO_OK;
}

int sco_get_graph(sco_ctx* c, int chain, int32_t* row_ptr, int32_t* col, int32_t* attr, int32_t* colors,
                  int64_t* n_dir) {
  if (!c || chain < 0 || chain >= c->n) return SCO_EINVAL;
  const int fr = consume_flags(c);
  if (fr != SCO_OK) return fr;  // the graph of a flagged launch is not usable
  if (c->graph_state < 1) return SCO_EINVAL;
  const ChainDesc& d = c->cd[chain];
  const Layout& L = c->lay;
  std::vector<int32_t> rp(d.N + 1);
  HIP_TRY(hipMemcpyAsync(rp.data(), at<int32_t>(c, L.off_row) + d.vbase, sizeof(int32_t) * (d.N + 1),
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const int32_t e0 = rp[0], e1 = rp[d.N];
  if (e0 < 0 || e1 < e0 || static_cast<int64_t>(e1) > 2 * static_cast<int64_t>(L.cap_und)) return SCO_EINTERNAL;
  if (n_dir) *n_dir = e1 - e0;
  if (row_ptr)
    for (int v = 0; v <= d.N; ++v) row_ptr[v] = rp[v] - e0;
  if ((col || attr) && e1 > e0) {
    std::vector<int32_t> cl(e1 - e0);
    HIP_TRY(hipMemcpy(cl.data(), at<int32_t>(c, L.off_col) + e0, sizeof(int32_t) * (e1 - e0), hipMemcpyDeviceToHost));
    if (col)
      for (int32_t i = 0; i < e1 - e0; ++i) col[i] = cl[i] - static_cast<int32_t>(d.vbase);
    if (attr)
      HIP_TRY(hipMemcpy(attr, at<int32_t>(c, L.off_attr) + e0, sizeof(int32_t) * (e1 - e0), hipMemcpyDeviceToHost));
  }
  if (colors) {
    std::vector<uint16_t> cc(d.N);
    HIP_TRY(hipMemcpy(cc.data(), at<uint16_t>(c, L.off_color) + d.vbase, sizeof(uint16_t) * d.N,
                      hipMemcpyDeviceToHost));
    for (int v = 0; v < d.N; ++v) colors[v] = cc[v];
  }
  return fr;
}

int sco_get_tables(sco_ctx* c, int chain, int32_t* K, int32_t* dx, int32_t* dy, double* J, double* C,
                   double* theta, double* delta) {
  if (!c || chain < 0 || chain >= c->n) return SCO_EINVAL;
  const int t = c->lay.chain_table[chain];
  const int64_t n = c->lay.table_K[t];
  if (K) *K = static_cast<int32_t>(n);
  for (int64_t m = 0; m < n; ++m) {
    const uint32_t p = c->hd[t][m];
    if (dx) dx[m] = static_cast<int16_t>(p & 0xFFFFu);
    if (dy) dy[m] = static_cast<int16_t>(p >> 16);
    if (J) J[m] = c->J[t][m];
    if (C) C[m] = c->C[t][m];
    if (theta) theta[m] = c->theta[chain].empty() ? 0.0 : c->theta[chain][m];
    if (delta) delta[m] = c->delta[chain].empty() ? INFINITY : c->delta[chain][m];
  }
  return SCO_OK;
}

int sco_destroy(sco_ctx* c) {
  if (!c) return SCO_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  graph_release(c);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
  return SCO_OK;
}

}  // extern "C"
