// sco_kernels.hip -- gfx950 kernels of the stochastic-cutoff (SCO) step.
//
// One SCO step (Endo, Toga & Sasaki, Sec. 2.1-2.3, Fig. 1) runs as one persistent
// kernel k_step<phases> whose blocks are all resident (cooperative launch, one
// 1024-thread block per CU):
//   step (1)  phase_switch    switch every dipolar bond (Eqs. 1-3): geometric skipping
//                             over the cumulative coupling, then thinning; survivors
//                             appended with one atomic per wavefront (ballot count)
//             scan_lookback   single-pass prefix sum of the degrees (row offsets)
//             phase_scatter   both directions of every survivor into the CSR
//             phase_rowsort   rows ascending by neighbour, union degree, Delta
//   step (2)  phase_kw_local  Kuhn-Wattenhofer levels whose groups fit in one LDS tile
//             phase_kw_global the remaining levels, colour class by colour class
//   step (3)  phase_sweep     Metropolis on H' (Eq. 4), one colour class at a time
// Device-wide barriers separate dependent phases; every wait in them is bounded and a
// wait that runs out raises SCO_FLAG_TIMEOUT, after which every wave leaves the kernel.
//
// Floating point: FP64 with contraction disabled (-ffp-contract=off); every decision
// that the CPU reference also takes is evaluated with the same operations in the
// same order.  Only exp/log of the device math library can differ from the host's in
// the last bit.
#include <hip/hip_runtime.h>

#include "sco_internal.h"

namespace {

constexpr int kBlock = SCO_CHUNK;  // a block of per-site threads is one chunk
constexpr int kWaves = kBlock / 64;

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror & Shaw (SC'11): ten rounds of multiply/xor with the Weyl key
// schedule (0x9E3779B9, 0xBB67AE85) and multipliers 0xD2511F53, 0xCD9E8D57.
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

template <typename T>
__device__ __forceinline__ T ld_relaxed(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_relaxed(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Coherent read for polling: a read-modify-write at device scope is performed where
// all XCDs see the same value, while a plain load (even device-scope) has been seen to
// keep returning a stale line on one XCD.
template <typename T>
__device__ __forceinline__ T ld_poll(T* p) {
  return __hip_atomic_fetch_or(p, T(0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_flag(SyncWords* s, uint32_t f) {
  __hip_atomic_fetch_or(&s->flags, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool timed_out(SyncWords* s) {
  return (ld_relaxed(&s->flags) & SCO_FLAG_TIMEOUT) != 0;
}

constexpr uint32_t kSpinLimit = 1u << 22;  // ~ seconds; reached only if residency fails

// Device-wide barrier (all blocks resident).  Arrival is counted in SCO_BAR_GROUPS
// groups, then by group; counters only grow, so nothing is reset between barriers.
// One wave per block fences: a release before arriving and an acquire after the
// generation word moved, which makes every write of the block before the barrier
// visible to every read after it.  Returns false once a wait has timed out.
__device__ bool grid_barrier(SyncWords* s) {
  __shared__ uint32_t s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t nb = gridDim.x;
    const uint32_t ng = nb < SCO_BAR_GROUPS ? nb : SCO_BAR_GROUPS;
    const uint32_t grp = blockIdx.x % ng;
    const uint32_t members = nb / ng + (grp < nb % ng ? 1u : 0u);
    const uint32_t gen = ld_relaxed(&s->gen);
    bool last = false;
    const unsigned long long a =
        __hip_atomic_fetch_add(&s->grp[grp * 16], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1ull;
    if (a % members == 0) {
      const unsigned long long t =
          __hip_atomic_fetch_add(&s->top, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1ull;
      last = (t % ng == 0);
    }
    if (last) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(&s->gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t n = 0;
      while (ld_poll(&s->gen) == gen) {
        if (timed_out(s)) break;
        if (++n > kSpinLimit) {
          set_flag(s, SCO_FLAG_TIMEOUT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = timed_out(s) ? 0u : 1u;
  }
  __syncthreads();
  return s_ok != 0;
}

// Sum / max over a block (all threads must call); result valid in every thread.
template <typename T>
__device__ T block_sum(T v) {
  __shared__ T red[kWaves];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T t = 0;
  for (int i = 0; i < kWaves; ++i) t += red[i];
  return t;
}

__device__ int block_max(int v) {
  __shared__ int red[kWaves];
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
  for (int i = 0; i < kWaves; ++i) t = max(t, red[i]);
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

// max over the wave (all lanes must call)
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// atomicMax of per-lane values into a per-chain LDS array; one atomic per wave when
// the lanes with a value share the chain (all lanes must call; c < 0: no value)
__device__ __forceinline__ void wave_max_to(int* per_chain, int c, int val) {
  const int c0 = __shfl(c, __ffsll(static_cast<unsigned long long>(__ballot(c >= 0))) - 1);
  if (__ballot(c >= 0) == 0) return;
  if (__ballot(c >= 0 && c != c0) == 0) {
    const int m = wave_max(c >= 0 ? val : 0);
    if (lane_id() == 0) atomicMax(&per_chain[c0], m);
  } else if (c >= 0) {
    atomicMax(&per_chain[c], val);
  }
}

// 256-bit colour set without dynamic register indexing
struct ColorSet {
  uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
  __device__ __forceinline__ void add(int c) {
    const uint64_t b = 1ull << (c & 63);
    if (c < 64) w0 |= b;
    else if (c < 128) w1 |= b;
    else if (c < 192) w2 |= b;
    else w3 |= b;
  }
  // smallest colour not in the set (256 when all are taken)
  __device__ __forceinline__ int first_free() const {
    if (~w0) return __ffsll(static_cast<unsigned long long>(~w0)) - 1;
    if (~w1) return 64 + __ffsll(static_cast<unsigned long long>(~w1)) - 1;
    if (~w2) return 128 + __ffsll(static_cast<unsigned long long>(~w2)) - 1;
    if (~w3) return 192 + __ffsll(static_cast<unsigned long long>(~w3)) - 1;
    return 256;
  }
};

// Phase marks of block 0 (wall clock), for attributing the time of the persistent
// kernel: trace[0] = count, then (id, time) pairs.
__device__ __forceinline__ void mark(unsigned long long* trace, uint32_t id) {
  if (trace == nullptr || blockIdx.x != 0 || threadIdx.x != 0) return;
  const unsigned long long n = atomicAdd(&trace[0], 1ull);
  if (2 * n + 2 < SCO_TRACE_SLOTS) {
    trace[2 * n + 1] = id;
    trace[2 * n + 2] = static_cast<unsigned long long>(wall_clock64());
  }
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

// =================================================================== step (1)
// One thread per owner site.  Candidate bonds of owner v: the table intervals
// (C_{m-1}, C_m] hit by a Poisson process of rate (kappa+1) beta run from C = 0,
// found by drawing exponential gaps E = -log(u) and locating C_pos + E T/(kappa+1)
// in the cumulative table (guide-table bracket, then binary search).  A candidate
// survives if its spins are antiparallel or, when kappa > 1, with probability
// theta_m if they are parallel.  Draw k of owner v is half k&1 of
// Philox(step, v, k>>1, SW); the thinning draw of candidate k is Philox(step, v, k, TH).
__device__ void phase_switch(const StepArgs& a) {
  __shared__ uint32_t s_count;
  const uint32_t cap_chunk = a.cap_und / static_cast<uint32_t>(a.nchunks);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kBlock; base < a.G; base += stride) {
    const int64_t g = base + threadIdx.x;  // a block-iteration is one chunk: one chain
    const int64_t chunk = base >> SCO_CHUNK_SHIFT;
    const uint32_t e_base = static_cast<uint32_t>(chunk) * cap_chunk;
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();
    const ChainDesc& d = a.cd[a.chunk_chain[base >> SCO_CHUNK_SHIFT]];
    const int v = static_cast<int>(g - d.vbase);
    bool active = v < d.N;
    const int L = d.L;
    const int y = active ? fdiv(v, d.inv_L) : 0, x = v - y * L;
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
      // wavefront-aggregated append into the block's region: one LDS atomic per wave
      // and draw round
      const uint64_t mask = __ballot(found);
      if (mask) {
        const uint32_t lane = lane_id();
        const int leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
        uint32_t e0 = 0;
        if (static_cast<int>(lane) == leader) e0 = atomicAdd(&s_count, static_cast<uint32_t>(__popcll(mask)));
        e0 = __shfl(e0, leader);
        if (found) {
          const uint32_t eo = e0 + static_cast<uint32_t>(__popcll(mask & ((1ull << lane) - 1ull)));
          const uint32_t e = e_base + eo;
          if (eo < cap_chunk) {
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
    __syncthreads();
    if (threadIdx.x == 0) a.ecount[chunk] = min(s_count, cap_chunk);
    __syncthreads();
  }
}

// ------------------------------------------------------------------ prefix sum
// Single-pass exclusive scan (decoupled look-back) of n int32 values: tile t
// publishes its aggregate, then its inclusive prefix, in one 64-bit word
// (epoch:24 | state:8 | value:32) so that one relaxed atomic carries both.  Tiles are
// taken in increasing order by every block, so the tile a block waits on is owned by
// a block that is not waiting on it.  out[n] = total.  out may alias in.
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;

__device__ bool scan_lookback(const int32_t* in, int64_t n, int32_t* out, unsigned long long* ts,
                              uint32_t epoch, SyncWords* sync) {
  __shared__ int32_t wsum[kWaves];
  __shared__ int32_t s_excl;
  const int64_t nt = (n + kTile - 1) / kTile;
  const unsigned long long tag = static_cast<unsigned long long>(epoch & 0xFFFFFFu) << 40;
  bool ok = true;
  for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const int64_t base = t * kTile + static_cast<int64_t>(threadIdx.x) * kItems;
    int32_t vals[kItems];
    int32_t s = 0;
#pragma unroll
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
    int32_t woff = 0, agg = 0;
    for (int i = 0; i < kWaves; ++i) {
      woff += i < w ? wsum[i] : 0;
      agg += wsum[i];
    }
    if (threadIdx.x == 0) {
      int32_t excl = 0;
      if (t == 0) {
        st_relaxed(&ts[t], tag | (2ull << 32) | static_cast<uint32_t>(agg));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      } else {
        st_relaxed(&ts[t], tag | (1ull << 32) | static_cast<uint32_t>(agg));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        int64_t jdx = t - 1;
        uint32_t spins = 0;
        while (jdx >= 0) {
          const unsigned long long wv = spins ? ld_poll(&ts[jdx]) : ld_relaxed(&ts[jdx]);
          uint32_t state = static_cast<uint32_t>((wv >> 32) & 0xFFu);
          if ((wv >> 40) != (tag >> 40) || state > 2u) state = 0;  // another launch's word
          if (state == 0) {
            if (timed_out(sync) || ++spins > kSpinLimit) {
              set_flag(sync, SCO_FLAG_TIMEOUT);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          excl += static_cast<int32_t>(wv & 0xFFFFFFFFu);
          if (state == 2) break;
          --jdx;
        }
        st_relaxed(&ts[t], tag | (2ull << 32) | static_cast<uint32_t>(excl + agg));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      }
      s_excl = excl;
    }
    __syncthreads();
    if (timed_out(sync)) ok = false;
    int32_t run = s_excl + woff + incl - s;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const int64_t idx = base + i;
      if (idx < n) out[idx] = run;
      run += vals[i];
    }
    if (t == nt - 1 && threadIdx.x == kBlock - 1) out[n] = run;
    __syncthreads();
  }
  return ok;
}

// both directions of every survivor into the CSR
__device__ void phase_scatter(const StepArgs& a) {
  const uint32_t cap_chunk = a.cap_und / static_cast<uint32_t>(a.nchunks);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int ch = blockIdx.x; ch < a.nchunks; ch += gridDim.x) {
    const uint32_t e0 = static_cast<uint32_t>(ch) * cap_chunk, e1 = e0 + a.ecount[ch];
    const int64_t cap2 = 2 * static_cast<int64_t>(a.cap_und);
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
      const int32_t u = a.ea[e], w = a.eb[e], m = a.em[e];
      const int64_t pu = a.row_ptr[u] + atomicAdd(&a.fill[u], 1);
      const int64_t pw = a.row_ptr[w] + atomicAdd(&a.fill[w], 1);
      if (pu < 0 || pu >= cap2 || pw < 0 || pw >= cap2) {  // cannot happen: degrees sum to 2 e
        set_flag(a.sync, SCO_FLAG_OVERFLOW);
        continue;
      }
      a.col[pu] = w;
      a.attr[pu] = m;
      a.col[pw] = u;
      a.attr[pw] = m;
    }
  }
  (void)stride;
}

// Sorts each row ascending by neighbour; union degree |CSR(v) u NN(v)|; Delta and
// directed bond count per chain.
__device__ void phase_rowsort(const StepArgs& a) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kBlock; base < a.G; base += stride) {
    const int c = a.chunk_chain[base >> SCO_CHUNK_SHIFT];
    const ChainDesc& d = a.cd[c];
    const int64_t g = base + threadIdx.x;
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
      const int y = fdiv(v, d.inv_L), x = v - y * d.L;
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
      atomicAdd(&a.st[c].n_edges, static_cast<uint32_t>(tot));
    }
  }
}

// =================================================================== step (2)
// Kuhn-Wattenhofer colour reduction (Sec. 2.3.3).  Level 0: site v of a chain with
// palette q is in group v/q with colour v mod q.  Level p unites pairs of groups; the
// upper half (bit p-1 of v/q set) is pending and is recoloured into 0..q-1 by rule
// (2)' of Sec. 2.3.2 in synchronous rounds.  The rounds are evaluated in an
// equivalent order: a pending vertex decides exactly when every pending same-group
// neighbour with a larger colour has decided (it is then a local maximum), and it
// sees their new colours; so treating the pending vertices colour class by colour
// class, largest first, yields the same colours.  The round in which v decides is
// rho(v) = 1 + max rho over those larger neighbours; a level takes max rho rounds.
//
// Per chain: P = the levels whose groups (q 2^p sites, aligned) fit in one LDS tile
// of T = q 2^P <= SCO_TILE_MAX sites; those run tile by tile entirely in LDS.  The
// levels above P run over the whole site space with device-wide barriers between
// colour classes.
struct KwChain {
  int q, M, P, tile0;  // tile0: first global tile of the chain
};

__device__ int kw_setup(const StepArgs& a, KwChain* kc, int* s_tiles) {
  // every block computes the same per-chain parameters (Delta is final here)
  for (int c = threadIdx.x; c < a.n_chains; c += kBlock) {
    int q = a.st[c].delta_union + 1;
    if (q > SCO_MAXQ) {
      set_flag(a.sync, SCO_FLAG_PALETTE);
      q = SCO_MAXQ;
    }
    const int N = a.cd[c].N;
    const int groups = (N + q - 1) / q;
    int M = 0;
    while ((1 << M) < groups) ++M;
    int P = 0;
    while (P < M && (q << (P + 1)) <= SCO_TILE_MAX) ++P;
    kc[c].q = q;
    kc[c].M = M;
    kc[c].P = P;
    if (blockIdx.x == 0) {
      a.st[c].q = q;
      a.st[c].M = M;
      a.st[c].P = P;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    uint32_t qmax = 0, mmax = 0;
    for (int c = 0; c < a.n_chains; ++c) {
      kc[c].tile0 = t;
      const int T = kc[c].q << kc[c].P;
      t += (a.cd[c].N + T - 1) / T;
      qmax = max(qmax, static_cast<uint32_t>(kc[c].q));
      mmax = max(mmax, static_cast<uint32_t>(kc[c].M));
    }
    *s_tiles = t;
    if (blockIdx.x == 0) {
      a.sync->qmax = qmax;
      a.sync->mmax = mmax;
    }
  }
  __syncthreads();
  return *s_tiles;
}

// Levels 1..P of every tile, in LDS.  Groups up to level P are aligned to the tile,
// so the same-group neighbours of a tile site are inside the tile.
__device__ void phase_kw_local(const StepArgs& a, const KwChain* kc, int ntiles) {
  __shared__ uint16_t t_col[SCO_TILE_MAX];
  __shared__ uint16_t t_rho[SCO_TILE_MAX];
  __shared__ uint16_t t_list[SCO_TILE_MAX];
  __shared__ int32_t t_off[SCO_MAXQ + 1];
  __shared__ int32_t t_fill[SCO_MAXQ];
  __shared__ int32_t t_rounds;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    int c = 0;
    while (c + 1 < a.n_chains && kc[c + 1].tile0 <= tile) ++c;
    const int L = a.cd[c].L, periodic = a.cd[c].periodic, N = a.cd[c].N;
    const int64_t vbase = a.cd[c].vbase;
    const double inv_L = a.cd[c].inv_L;
    const int q = kc[c].q, P = kc[c].P, T = q << P;
    const double invq = 1.0 / q;
    const int v0 = (tile - kc[c].tile0) * T;
    const int n = min(T, N - v0);
    for (int i = threadIdx.x; i < n; i += kBlock) t_col[i] = static_cast<uint16_t>(i - fdiv(i, invq) * q);
    __syncthreads();
    for (int p = 1; p <= P; ++p) {
      for (int k = threadIdx.x; k <= q; k += kBlock) t_off[k] = 0;
      if (threadIdx.x == 0) t_rounds = 0;
      __syncthreads();
      for (int i = threadIdx.x; i < n; i += kBlock)
        if ((fdiv(i, invq) >> (p - 1)) & 1) atomicAdd(&t_off[t_col[i] + 1], 1);
      __syncthreads();
      if (threadIdx.x == 0)
        for (int k = 0; k < q; ++k) t_off[k + 1] += t_off[k];
      __syncthreads();
      for (int k = threadIdx.x; k < q; k += kBlock) t_fill[k] = 0;
      __syncthreads();
      for (int i = threadIdx.x; i < n; i += kBlock)
        if ((fdiv(i, invq) >> (p - 1)) & 1) {
          const int cc = t_col[i];
          t_list[t_off[cc] + atomicAdd(&t_fill[cc], 1)] = static_cast<uint16_t>(i);
          t_rho[i] = 0;
        }
      __syncthreads();
      for (int cc = q - 1; cc >= 0; --cc) {
        int tmax = 0;
        for (int k = t_off[cc] + threadIdx.x; k < t_off[cc + 1]; k += kBlock) {
          const int i = t_list[k];
          const int v = v0 + i;
          const int grp = fdiv(i, invq) >> p;
          const int y = fdiv(v, inv_L), x = v - y * L;
          int nb[4];
          const int nn = nn_sites(x, y, L, periodic, nb);
          const int64_t g = vbase + v;
          const int r0 = a.row_ptr[g], r1 = a.row_ptr[g + 1];
          ColorSet taken;
          int rmax = 0;
          for (int t = 0; t < nn + (r1 - r0); ++t) {
            const int u = t < nn ? nb[t] : static_cast<int>(a.col[r0 + t - nn] - vbase);
            const int j = u - v0;
            if (j < 0 || j >= n) continue;  // outside the tile: another group
            const int gj = fdiv(j, invq);
            if ((gj >> p) != grp) continue;
            if ((gj >> (p - 1)) & 1) {
              const int rj = t_rho[j];
              if (rj == 0) continue;  // pending, undecided: a smaller colour
              rmax = max(rmax, rj);
            }
            taken.add(t_col[j]);
          }
          int nc = taken.first_free();
          if (nc >= q) {
            set_flag(a.sync, SCO_FLAG_PALETTE);
            nc = q - 1;
          }
          t_col[i] = static_cast<uint16_t>(nc);
          t_rho[i] = static_cast<uint16_t>(rmax + 1);
          tmax = max(tmax, rmax + 1);
        }
        tmax = wave_max(tmax);
        if (lane_id() == 0 && tmax > 0) atomicMax(&t_rounds, tmax);
        __syncthreads();
      }
      if (threadIdx.x == 0 && t_rounds > 0) atomicMax(&a.st[c].kw_rounds[p], t_rounds);
    }
    const uint32_t tag = static_cast<uint32_t>(P) << 18;
    for (int i = threadIdx.x; i < n; i += kBlock) {
      const int64_t g = vbase + v0 + i;
      a.color[g] = t_col[i];
      a.kw_word[g] = tag | t_col[i];
    }
    __syncthreads();
  }
}

// Levels P+1..M over the whole site space.  Block b owns the sites [b S, (b+1) S)
// and buckets its pending sites of the level by colour into plist; device-wide
// barriers separate the colour classes, so every read sees the writes of the classes
// before it.  kw_word[g] holds (level << 18) | (round << 9) | colour of the last
// level that decided g, so "decided at this level" needs no clearing pass.  A colour
// read from memory is checked against the palette before it is used as an index.
__device__ bool phase_kw_global(const StepArgs& a, const KwChain* kc) {
  __shared__ int32_t boff[SCO_MAXQ + 1];
  __shared__ int32_t bfill[SCO_MAXQ];
  __shared__ int32_t brounds[SCO_MAXCHAINS];
  const int64_t S = ((a.G + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
  const int64_t r0 = min(static_cast<int64_t>(blockIdx.x) * S, a.G);
  const int64_t r1 = min(r0 + S, a.G);
  const int qmax = static_cast<int>(a.sync->qmax);
  const int mmax = static_cast<int>(a.sync->mmax);
  int pmin = SCO_MAXLEVEL;
  for (int c = 0; c < a.n_chains; ++c) pmin = min(pmin, kc[c].P);

  for (int p = pmin + 1; p <= mmax; ++p) {
    for (int k = threadIdx.x; k <= qmax; k += kBlock) boff[k] = 0;
    for (int c = threadIdx.x; c < a.n_chains; c += kBlock) brounds[c] = 0;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int64_t g = r0 + threadIdx.x; g < r1; g += kBlock) {
        const int c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
        const int v = static_cast<int>(g - a.cd[c].vbase);
        if (v >= a.cd[c].N || p <= kc[c].P || p > kc[c].M) continue;
        const int gg = fdiv(v, 1.0 / kc[c].q);
        if (((gg >> (p - 1)) & 1) == 0) continue;
        const int cc = a.color[g];
        if (cc >= kc[c].q) {  // cannot happen after a complete colouring
          set_flag(a.sync, SCO_FLAG_PALETTE);
          continue;
        }
        if (pass == 0) atomicAdd(&boff[cc + 1], 1);
        else a.plist[r0 + boff[cc] + atomicAdd(&bfill[cc], 1)] = static_cast<int32_t>(g);
      }
      __syncthreads();
      if (pass == 0) {
        if (threadIdx.x == 0)
          for (int k = 0; k < qmax; ++k) boff[k + 1] += boff[k];
        for (int k = threadIdx.x; k < qmax; k += kBlock) bfill[k] = 0;
        __syncthreads();
      }
    }
    for (int cc = qmax - 1; cc >= 0; --cc) {
      // every thread of the block runs the same number of iterations
      for (int kb = boff[cc]; kb < boff[cc + 1]; kb += kBlock) {
        const int k = kb + static_cast<int>(threadIdx.x);
        int cdone = -1, rdone = 0;
        if (k < boff[cc + 1]) {
        const int32_t g = a.plist[r0 + k];
        const int c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
        const int L = a.cd[c].L, periodic = a.cd[c].periodic;
        const int64_t vbase = a.cd[c].vbase;
        const int q = kc[c].q;
        const double invq = 1.0 / q;
        const int v = static_cast<int>(g - vbase);
        const int grp = fdiv(v, invq) >> p;
        const int y = fdiv(v, a.cd[c].inv_L), x = v - y * L;
        int nb[4];
        const int nn = nn_sites(x, y, L, periodic, nb);
        ColorSet taken;
        int rmax = 0;
        const int r0e = a.row_ptr[g], r1e = a.row_ptr[g + 1];
        for (int t = 0; t < nn + (r1e - r0e); ++t) {
          const int u = t < nn ? nb[t] : static_cast<int>(a.col[r0e + t - nn] - vbase);
          const int gu = fdiv(u, invq);
          if ((gu >> p) != grp) continue;  // another group at this level
          if ((gu >> (p - 1)) & 1) {       // pending at this level
            const uint32_t w = a.kw_word[vbase + u];
            if (static_cast<int>((w >> 18) & 0x1Fu) != p) continue;  // undecided: a smaller colour
            rmax = max(rmax, static_cast<int>((w >> 9) & 0x1FFu));
          }
          taken.add(a.color[vbase + u]);
        }
        int nc = taken.first_free();
        if (nc >= q) {
          set_flag(a.sync, SCO_FLAG_PALETTE);
          nc = q - 1;
        }
        a.color[g] = static_cast<uint16_t>(nc);
        a.kw_word[g] = (static_cast<uint32_t>(p) << 18) | (static_cast<uint32_t>(rmax + 1) << 9) |
                       static_cast<uint32_t>(nc);
        cdone = c;
        rdone = rmax + 1;
        }
        wave_max_to(brounds, cdone, rdone);
      }
      if (!grid_barrier(a.sync)) return false;
    }
    for (int c = threadIdx.x; c < a.n_chains; c += kBlock)
      if (brounds[c] > 0) atomicMax(&a.st[c].kw_rounds[p], brounds[c]);
    mark(a.trace, 100 + p);
  }
  return true;
}

// =================================================================== step (3)
// Block b buckets its own sites [b S, (b+1) S) by colour, then the colour classes are
// swept in ascending order with device-wide barriers between them.  Flipping s_v
// changes H' by s_v h_v, h_v = 2J sum_NN s_u - sum_bonds delta_m s_u (NN first, then
// the bonds in row order); with kappa == 1 a bond is hard and forbids the flip, and
// the exchange-only acceptance is the table pacc.
__device__ bool phase_sweep(const StepArgs& a) {
  __shared__ int32_t boff[SCO_MAXQ + 1];
  __shared__ int32_t bfill[SCO_MAXQ];
  __shared__ unsigned long long bacc[SCO_MAXCHAINS];  // accepted flips of the block per chain
  const int qmax = static_cast<int>(a.sync->qmax);
  const int64_t S = ((a.G + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
  const int64_t r0 = min(static_cast<int64_t>(blockIdx.x) * S, a.G);
  const int64_t r1 = min(r0 + S, a.G);
  for (int k = threadIdx.x; k <= qmax; k += kBlock) boff[k] = 0;
  for (int c = threadIdx.x; c < a.n_chains; c += kBlock) bacc[c] = 0;
  __syncthreads();
  for (int64_t g = r0 + threadIdx.x; g < r1; g += kBlock) {
    const int c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
    if (static_cast<int>(g - a.cd[c].vbase) < a.cd[c].N) {
      const int cc = a.color[g];
      if (cc < qmax) atomicAdd(&boff[cc + 1], 1);
      else set_flag(a.sync, SCO_FLAG_PALETTE);  // cannot happen after a complete colouring
    }
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < qmax; ++k) boff[k + 1] += boff[k];
  for (int k = threadIdx.x; k < qmax; k += kBlock) bfill[k] = 0;
  __syncthreads();
  for (int64_t g = r0 + threadIdx.x; g < r1; g += kBlock) {
    const int c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
    if (static_cast<int>(g - a.cd[c].vbase) < a.cd[c].N) {
      const int cc = a.color[g];
      if (cc < qmax) a.plist[r0 + boff[cc] + atomicAdd(&bfill[cc], 1)] = static_cast<int32_t>(g);
    }
  }
  __syncthreads();
  mark(a.trace, 22);

  for (int s = 0; s < a.nsw_max; ++s) {
    for (int cc = 0; cc < qmax; ++cc) {
      const int k0 = boff[cc], k1 = boff[cc + 1];
      // every thread of the block runs the same number of iterations
      for (int kb = k0; kb < k1; kb += kBlock) {
        const int k = kb + static_cast<int>(threadIdx.x);
        bool acc = false;
        int c = -1;
        if (k < k1) {
          const int32_t g = a.plist[r0 + k];
          c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
          const ChainDesc& d = a.cd[c];
          const int nsw = a.nsw_override >= 0 ? a.nsw_override : d.n_sw;
          if (s < nsw) {
            const int v = static_cast<int>(g - d.vbase);
            const int y = fdiv(v, d.inv_L), x = v - y * d.L;
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
        // accepted flips per chain into LDS: one atomic per wave when the wave is one chain
        const int c0 = __shfl(c, 0);
        if (__ballot(c != c0 && c >= 0) == 0) {
          const uint64_t mk = __ballot(acc);
          if (lane_id() == 0 && mk && c0 >= 0) atomicAdd(&bacc[c0], static_cast<unsigned long long>(__popcll(mk)));
        } else if (acc) {
          atomicAdd(&bacc[c], 1ull);
        }
      }
      if (!grid_barrier(a.sync)) return false;
      mark(a.trace, 1000 + cc);
    }
  }
  for (int c = threadIdx.x; c < a.n_chains; c += kBlock)
    if (bacc[c]) atomicAdd(&a.st[c].accepted, bacc[c]);
  if (blockIdx.x == 0)
    for (int c = threadIdx.x; c < a.n_chains; c += kBlock) {
      const int nsw = a.nsw_override >= 0 ? a.nsw_override : a.cd[c].n_sw;
      a.st[c].attempts += static_cast<unsigned long long>(a.cd[c].N) * static_cast<unsigned long long>(nsw);
    }
  return true;
}

// ------------------------------------------------------------------ the step
// Persistent kernel (cooperative launch: every block resident).  `phases` selects
// steps (1) switching + assembly, (2) colouring, (3) sweeps.  The switching part
// starts by clearing the degree and cursor arrays and the per-chain counters of the
// graph; a launch without it checks that the words left by the earlier launches say
// a complete graph (and colouring) is there.
template <uint32_t phases>
__global__ void __launch_bounds__(kBlock) k_step(StepArgs a) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if constexpr ((phases & PH_SWITCH) != 0) {
    // the degree and cursor arrays start from zero whatever an earlier launch left
    if (lead) {
      a.sync->graph_valid = 0;
      a.sync->color_valid = 0;
    }
    for (int c = gtid(); c < a.n_chains; c += stride) {
      a.st[c].delta_union = 0;
      a.st[c].n_edges = 0;
      for (int p = 0; p < SCO_MAXLEVEL; ++p) a.st[c].kw_rounds[p] = 0;
    }
    for (int64_t g = gtid(); g < a.G; g += stride) {
      a.deg[g] = 0;
      a.fill[g] = 0;
    }
    if (!grid_barrier(a.sync)) return;
    mark(a.trace, 1);
    phase_switch(a);
    mark(a.trace, 2);
    if (!grid_barrier(a.sync)) return;
    mark(a.trace, 3);
    if (!scan_lookback(a.deg, a.G, a.row_ptr, a.scan_ts, a.epoch, a.sync)) return;
    if (!grid_barrier(a.sync)) return;
    mark(a.trace, 4);
    phase_scatter(a);
    if (!grid_barrier(a.sync)) return;
    mark(a.trace, 5);
    phase_rowsort(a);
    if (!grid_barrier(a.sync)) return;
    mark(a.trace, 6);
    if (lead) a.sync->graph_valid = 1;
  }
  if constexpr ((phases & PH_COLOR) != 0) {
    __shared__ KwChain kc[SCO_MAXCHAINS];
    __shared__ int s_tiles;
    if constexpr ((phases & PH_SWITCH) == 0) {
      // a separate colouring needs a completed switching (every block reads the
      // same word, written by an earlier launch)
      if (a.sync->graph_valid != 1) {
        if (lead) set_flag(a.sync, SCO_FLAG_STATE);
        return;
      }
      if (lead) a.sync->color_valid = 0;
    }
    mark(a.trace, 10);
    const int ntiles = kw_setup(a, kc, &s_tiles);
    phase_kw_local(a, kc, ntiles);
    mark(a.trace, 11);
    if (!grid_barrier(a.sync)) return;
    if (!phase_kw_global(a, kc)) return;
    mark(a.trace, 12);
    if (!grid_barrier(a.sync)) return;
    mark(a.trace, 13);
    if (lead) a.sync->color_valid = 1;
  }
  if constexpr ((phases & PH_SWEEP) != 0) {
    if constexpr ((phases & PH_COLOR) == 0) {
      if (a.sync->color_valid != 1) {
        if (lead) set_flag(a.sync, SCO_FLAG_STATE);
        return;
      }
    }
    mark(a.trace, 20);
    if (!phase_sweep(a)) return;
    mark(a.trace, 21);
  }
}

// =================================================================== observables
// Per chunk (one chain): sum s, sum over the NN pairs (+x, +y) of s_i s_j, and the
// set of colours in use.
extern "C" __global__ void __launch_bounds__(kBlock)
    k_obs_basic(const ChainDesc* __restrict__ cd, const int32_t* __restrict__ chunk_chain,
                const int8_t* __restrict__ spin, const uint16_t* __restrict__ color,
                unsigned long long* __restrict__ out, unsigned* __restrict__ used, int64_t G) {
  __shared__ unsigned s_used[SCO_MAXQ / 32];
  if (threadIdx.x < SCO_MAXQ / 32) s_used[threadIdx.x] = 0;
  __syncthreads();
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
    const int k = color[g];
    if (k < SCO_MAXQ) atomicOr(&s_used[k >> 5], 1u << (k & 31));
  }
  m = block_sum(m);
  ex = block_sum(ex);
  if (threadIdx.x == 0) {
    atomicAdd(&out[2 * c], static_cast<unsigned long long>(m));
    atomicAdd(&out[2 * c + 1], static_cast<unsigned long long>(ex));
  }
  if (threadIdx.x < SCO_MAXQ / 32 && s_used[threadIdx.x])
    atomicOr(&used[c * (SCO_MAXQ / 32) + threadIdx.x], s_used[threadIdx.x]);
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

// Deterministic sum of prod[0..K): blocks of 4096 terms (per-thread runs of 16, then
// a fixed tree), then the block partials in order by one thread.
extern "C" __global__ void __launch_bounds__(256)
    k_obs_sum_partials(const double* __restrict__ prod, int K, double* __restrict__ part) {
  __shared__ double buf[256];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * 4096;
  double s = 0.0;
  for (int i = 0; i < 16; ++i) {
    const int64_t idx = base + static_cast<int64_t>(threadIdx.x) * 16 + i;
    if (idx < K) s += prod[idx];
  }
  buf[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
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
  hipLaunchKernelGGL(k_table_j, dim3((K + 255) / 256), dim3(256), 0, s, hd, K, L, periodic, n_images, D, J);
  return hipGetLastError();
}

hipError_t init_spins(hipStream_t s, const ChainDesc* cd, const int32_t* chunk_chain,
                      const int64_t* src_base, const int8_t* src, int8_t* spin, int64_t G) {
  hipLaunchKernelGGL(k_init_spins, dim3(static_cast<uint32_t>(G / kBlock)), dim3(kBlock), 0, s, cd,
                     chunk_chain, src_base, src, spin, G);
  return hipGetLastError();
}

template <uint32_t P>
const void* step_kernel() {
  return reinterpret_cast<const void*>(&k_step<P>);
}

const void* step_kernel_for(uint32_t phases) {
  switch (phases) {
    case PH_SWITCH: return step_kernel<PH_SWITCH>();
    case PH_COLOR: return step_kernel<PH_COLOR>();
    case PH_SWEEP: return step_kernel<PH_SWEEP>();
    default: return step_kernel<PH_SWITCH | PH_COLOR | PH_SWEEP>();
  }
}

// co-resident blocks of the step kernels (the smallest over the variants)
int step_max_blocks() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  int best = 1 << 30;
  const uint32_t variants[4] = {PH_SWITCH, PH_COLOR, PH_SWEEP, PH_SWITCH | PH_COLOR | PH_SWEEP};
  for (uint32_t ph : variants) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, step_kernel_for(ph), kBlock, 0) != hipSuccess) return 0;
    best = per < best ? per : best;
  }
  return best * cus;
}

hipError_t step(hipStream_t s, const StepArgs& a, uint32_t phases, int blocks) {
  StepArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(step_kernel_for(phases), dim3(blocks), dim3(kBlock), args, 0, s);
}

hipError_t obs_basic(hipStream_t s, const ChainDesc* cd, const int32_t* chunk_chain, const int8_t* spin,
                     const uint16_t* color, unsigned long long* out, unsigned* used, int64_t G) {
  hipLaunchKernelGGL(k_obs_basic, dim3(static_cast<uint32_t>(G / kBlock)), dim3(kBlock), 0, s, cd,
                     chunk_chain, spin, color, out, used, G);
  return hipGetLastError();
}

hipError_t obs_dipolar(hipStream_t s, const uint32_t* hd, const double* J, int K, int L, int periodic,
                       const int8_t* spin, int64_t vbase, uint32_t* bits, double* prod, double* part,
                       double* out) {
  if (L % 32 == 0) {
    const int W = L / 32;
    hipLaunchKernelGGL(k_obs_pack, dim3((L * W + 255) / 256), dim3(256), 0, s, spin, vbase, L, W, bits);
    hipLaunchKernelGGL(k_obs_corr_bits, dim3((K + 255) / 256), dim3(256), 0, s, hd, J, K, L, periodic, bits,
                       prod);
  } else {
    hipLaunchKernelGGL(k_obs_corr_plain, dim3((K + 255) / 256), dim3(256), 0, s, hd, J, K, L, periodic, spin,
                       vbase, prod);
  }
  const int nparts = (K + 4095) / 4096;
  hipLaunchKernelGGL(k_obs_sum_partials, dim3(nparts), dim3(256), 0, s, prod, K, part);
  hipLaunchKernelGGL(k_obs_sum_final, dim3(1), dim3(64), 0, s, part, nparts, out);
  return hipGetLastError();
}

}  // namespace sco_dev
