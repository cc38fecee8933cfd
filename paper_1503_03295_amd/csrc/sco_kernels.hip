// sco_kernels.hip -- gfx950 kernels of the stochastic-cutoff (SCO) step.
//
// One SCO step (Endo, Toga & Sasaki, Sec. 2.1-2.3, Fig. 1) runs as one persistent
// kernel k_step<phases, model> whose blocks are all resident (cooperative launch, one
// 1024-thread block per CU); model selects Ising spins or the Heisenberg spins of
// Eq. (6):
//   step (1)  phase_switch    switch every dipolar bond (Eqs. 1-3): geometric skipping
//                             over the cumulative coupling, then thinning; survivors
//                             appended with one atomic per wavefront (ballot count)
//             scan_two_pass   prefix sum of the degrees (row offsets): tile sums, one
//                             device barrier, then every tile scanned in LDS
//             phase_scatter   both directions of every survivor into the CSR, at
//                             slots fixed in the switching (no atomics)
//             phase_rowsort   rows ascending by neighbour, union degree, Delta
//   step (2)  phase_kw_local  Kuhn-Wattenhofer levels whose groups fit in one LDS tile
//             phase_kw_global the remaining levels, colour class by colour class
//             (phase_color_bcr: whole-graph colour reduction, a colouring variant)
//   step (3)  phase_sweep     Metropolis on H' (Eq. 4), one colour class at a time
//             (phase_sweep_heis for Heisenberg spins)
// Device-wide barriers separate dependent phases; every wait in them is bounded and a
// wait that runs out raises SCO_FLAG_TIMEOUT, after which every wave leaves the kernel.
// The observables (energies, M_phi, graph statistics) are separate kernels.
//
// Floating point: FP64 with contraction disabled (-ffp-contract=off); every decision
// that the CPU reference also takes is evaluated with the same operations in the
// same order.  Only exp/log of the device math library can differ from the host's in
// the last bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "sco_internal.h"

namespace {

constexpr int kBlock = SCO_CHUNK;  // a block of per-site threads is one chunk
constexpr int kWaves = kBlock / 64;
// Items per thread whose loads are issued together: in colour classes (kBatch) and in
// scans over sites or survivors (kScan).
constexpr int kBatch = 3;
constexpr int kScan = 4;
constexpr int kOwners = 2;  // owners in flight per thread in the switching
constexpr int kStage = 8;   // tile sites per thread whose rows are read together when staging bonds
// Sites per thread whose colours stay in registers while a block buckets them: a
// device-wide level's share and a sweep range of a 2304^2 lattice over 256 blocks.
constexpr int kHeldKW = 12;
constexpr int kHeldSw = 21;
// Spin words (4 sites each) per thread when a block stages its own sweep range in LDS,
// and halo bytes per thread (two rows of up to 2560 sites).
constexpr int kStageSw = 6;
constexpr int kHaloSw = 5;

template <bool B>
struct Flag {
  static constexpr bool value = B;
};

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

// The same generator with each 32 x 32 -> 64-bit product taken whole (one
// multiply-add instruction instead of a low and a high multiply).
__device__ __forceinline__ W4 philox10_wide(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = static_cast<uint32_t>(p1);
    c2 = n2;
    c3 = static_cast<uint32_t>(p0);
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

// A point uniform on the unit sphere by Marsaglia's method (Ann. Math. Stat. 43, 645
// (1972)): x1, x2 uniform in (-1, 1) until q = x1^2 + x2^2 < 1, then
// (2 x1 sqrt(1-q), 2 x2 sqrt(1-q), 1 - 2q).  Try k draws Philox(c0, c1, c2, tag + 256 k);
// false after 64 rejected tries.  Only a correctly rounded square root is involved.
__device__ __forceinline__ bool sphere_point(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag, uint32_t k0,
                                             uint32_t k1, double& ox, double& oy, double& oz) {
  for (uint32_t k = 0; k < 64; ++k) {
    const W4 w = philox10(c0, c1, c2, tag + (k << 8), k0, k1);
    const double x1 = 2.0 * unit52(w.x, w.y) - 1.0;
    const double x2 = 2.0 * unit52(w.z, w.w) - 1.0;
    const double q = x1 * x1 + x2 * x2;
    if (q < 1.0) {
      const double t = sqrt(1.0 - q);
      ox = 2.0 * x1 * t;
      oy = 2.0 * x2 * t;
      oz = 1.0 - 2.0 * q;
      return true;
    }
  }
  return false;
}

// Dipolar pair energy of Eq. (6) for in-plane displacement (dx, dy):
// (D / r^3) [S_i . S_j - 3 (S_i . r)(S_j . r) / r^2], D / r^3 = J_m / 2 (J_m = V^max).
__device__ __forceinline__ double heis_pair(double ax, double ay, double az, double bx, double by, double bz, int dx,
                                            int dy, double Jm) {
  const double dot = ax * bx + ay * by + az * bz;
  const double pi = ax * static_cast<double>(dx) + ay * static_cast<double>(dy);
  const double pj = bx * static_cast<double>(dx) + by * static_cast<double>(dy);
  const double r2 = static_cast<double>(dx) * static_cast<double>(dx) + static_cast<double>(dy) * static_cast<double>(dy);
  return (Jm * 0.5) * (dot - 3.0 * (pi * pj) / r2);
}

// ------------------------------------------------------------------ helpers
// |a - b| <= 1e-12 |b|: a decision this close may differ from a host evaluation whose
// exp / log differ in the last bit; such decisions are counted (near ties).
__device__ __forceinline__ bool near_tie(double a, double b) { return fabs(a - b) <= 1e-12 * fabs(b); }

__device__ __forceinline__ int64_t gtid() {
  return static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// exact floor(v / d) for 0 <= v < 2^31, 1 <= d < 2^20, via a double reciprocal:
// (v + 1/2) / d is at least 1/(2d) away from an integer, while the two roundings
// move the product by at most 2^31 2^-52 = 2^-21.
__device__ __forceinline__ int idiv_fp(int v, double inv_d) {
  return static_cast<int>((static_cast<double>(v) + 0.5) * inv_d);
}

// exact floor(i / d) for 0 <= i < 2^16 and 2 <= d < 2^16 with m = ceil(2^32 / d):
// i m / 2^32 exceeds i / d by less than i / 2^32 < 2^-16 < 1/d.
__device__ __forceinline__ uint32_t magic16(uint32_t d) {
  return static_cast<uint32_t>((0x100000000ull + d - 1u) / d);
}
__device__ __forceinline__ int div16(int i, uint32_t m) {
  return static_cast<int>(__umulhi(static_cast<uint32_t>(i), m));
}

// A read through a pointer known to address global memory (tables whose pointers
// are themselves read from memory would otherwise be read with flat instructions).
template <typename T>
__device__ __forceinline__ T ld_global(const T* p) {
  return *(const __attribute__((address_space(1))) T*)(p);
}

template <typename T>
__device__ __forceinline__ T ld_relaxed(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_relaxed(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Coherent read for polling: a read-modify-write at device scope is performed at the
// one point where every XCD's atomics to the address are ordered, so it returns the
// latest value in the address's modification order.  (A plain load, even an
// agent-scope one, may be served from a line that this XCD's L2 still holds.)
template <typename T>
__device__ __forceinline__ T ld_poll(T* p) {
  return __hip_atomic_fetch_or(p, T(0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publishing store for a word that other blocks poll: an atomic exchange, performed
// at the same point as the polls' read-modify-writes (no returned value is waited for).
template <typename T>
__device__ __forceinline__ void st_publish(T* p, T v) {
  (void)__hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_flag(SyncWords* s, uint32_t f) {
  __hip_atomic_fetch_or(&s->flags, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool timed_out(SyncWords* s) {
  return (ld_poll(&s->flags) & SCO_FLAG_TIMEOUT) != 0;
}

constexpr uint32_t kSpinLimit = 1u << 22;  // ~ seconds; reached only if residency fails

// Device-wide barriers (all blocks resident).  Arrival is counted in SCO_BAR_GROUPS
// groups, then by group, on counters that only grow between host resets (the host
// clears gen, stop, top and grp together).  A block's ticket a in its group (members
// blocks arrive there per barrier) names the barrier instance b = (a - 1) / members,
// counted from the reset; the block that completes the last group publishes the
// generation b + 1, and every other block waits until gen has reached b + 1.  No
// block reads gen before it arrives, so neither a stale copy of gen nor a load
// performed after the arrival can make it wait for the wrong generation.  Every
// access to gen, stop and the counters is a device-scope read-modify-write, so all
// of them are ordered at one point per word.
//
// `full`: the release/acquire sequence of the documented agent-scope memory model
// carries every write before the barrier to every read after it:
//   member   fence release; arrival RMW on its group counter
//   group completer: fence acq_rel after its group RMW (acquires its members'
//            release sequences, releases them on), then the RMW on the top counter
//   last arriver: fence acq_rel after the top RMW, then the exchange that publishes
//   waiter   RMW polls of gen until it reaches the target; fence acquire
// (fences at agent scope: L2 write-back / invalidation on each XCD).  The last
// arriver also copies the verdict of the raised flags into `stop`, so that every block
// takes the same decision to end the launch at the same barrier.
//
// Without `full` (colour classes of a sweep) only the control is ordered; the data
// the classes exchange (spins) is written and read with agent-scope atomics and the
// barrier adds no cache maintenance.
struct BarTicket {
  uint32_t target;
  bool last;
};

__device__ __forceinline__ BarTicket bar_arrive(SyncWords* s, bool full) {
  const uint32_t nb = gridDim.x;
  const uint32_t ng = nb < SCO_BAR_GROUPS ? nb : SCO_BAR_GROUPS;
  const uint32_t grp = blockIdx.x % ng;
  const uint32_t members = nb / ng + (grp < nb % ng ? 1u : 0u);
  const unsigned long long a =
      __hip_atomic_fetch_add(&s->grp[grp * 16], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1ull;
  const unsigned long long b = (a - 1ull) / members;
  BarTicket t{static_cast<uint32_t>(b + 1ull), false};
  if (a % members == 0) {  // this block completes its group for instance b
    if (full) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
    const unsigned long long k =
        __hip_atomic_fetch_add(&s->top, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1ull;
    t.last = (k % ng == 0);
  }
  return t;
}

// Waits for generation `target`; false once a wait has timed out.
__device__ __forceinline__ bool bar_wait(SyncWords* s, uint32_t target) {
  uint32_t n = 0;
  while (static_cast<int32_t>(ld_poll(&s->gen) - target) < 0) {
    if ((n & 63u) == 63u && timed_out(s)) return false;
    if (++n > kSpinLimit) {
      set_flag(s, SCO_FLAG_TIMEOUT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// Full device-wide barrier between dependent phases.  Returns false when the launch
// must end: a wait timed out, or a flag (edge overflow, palette, state) was raised
// before the barrier; every block then returns false at the same barrier.
__device__ __forceinline__ bool grid_barrier(SyncWords* s) {
  __shared__ uint32_t s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const BarTicket t = bar_arrive(s, true);
    bool ok = true;
    if (t.last) {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      if (ld_poll(&s->flags) != 0) {
        st_publish(&s->stop, t.target);
        st_publish(&s->halt, 1u);
      }
      st_publish(&s->gen, t.target);
    } else {
      ok = bar_wait(s, t.target);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // stop is written only by last arrivers; the next one can write it only after
    // this block has arrived at the next barrier, so this read sees this barrier's
    // verdict
    if (ok && ld_poll(&s->stop) == t.target) ok = false;
    s_ok = ok ? 1u : 0u;
  }
  __syncthreads();
  return s_ok != 0;
}

// Device-wide barrier between the colour classes of one sweep phase, for data that is
// written and read only with device-coherent (agent-scope) accesses: every wave waits
// until its own stores have completed, then the same arrival and bounded wait as
// grid_barrier, without the L2 write-back and invalidation of the agent-scope fences,
// so data that no class writes stays cached.  Returns false once a wait has timed out.
//
// Rule for its use (measured on gfx950): an XCD's own coherent store leaves the line
// valid in that XCD's L2, and its later coherent loads are served from there.  So
// between two full barriers every coherently written word must be written by blocks of
// one XCD only (here: by the one block that owns the site for the whole phase), or a
// former writer reads its own stale copy.  The barrier words themselves are written
// by whichever block arrives last; they are therefore touched only by
// read-modify-writes, which this rule does not concern.
__device__ __forceinline__ bool class_barrier(SyncWords* s) {
  __shared__ uint32_t s_ok;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    const BarTicket t = bar_arrive(s, false);
    bool ok = true;
    if (t.last) st_publish(&s->gen, t.target);
    else ok = bar_wait(s, t.target);
    s_ok = ok ? 1u : 0u;
  }
  __syncthreads();
  return s_ok != 0;
}

// Sum over a block (all threads must call); result valid in every thread.
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

// nearest neighbours in the slots (+x, -x, +y, -y); -1 where an open lattice ends
// (fixed slots keep the array in registers)
__device__ __forceinline__ void nn_sites(int x, int y, int L, int periodic, int nb[4]) {
  const int v = y * L + x;
  if (periodic) {
    nb[0] = y * L + (x + 1 == L ? 0 : x + 1);
    nb[1] = y * L + (x == 0 ? L - 1 : x - 1);
    nb[2] = (y + 1 == L ? 0 : y + 1) * L + x;
    nb[3] = (y == 0 ? L - 1 : y - 1) * L + x;
    return;
  }
  nb[0] = x + 1 < L ? v + 1 : -1;
  nb[1] = x > 0 ? v - 1 : -1;
  nb[2] = y + 1 < L ? v + L : -1;
  nb[3] = y > 0 ? v - L : -1;
}

// max over the wave (all lanes must call)
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// atomicMax of per-lane values into a per-chain LDS array; one atomic per wave when
// the lanes with a value share the chain (all lanes must call; c < 0: no value)
__device__ __forceinline__ void wave_max_to(int* per_chain, int c, int val) {
  const uint64_t has = __ballot(c >= 0);
  if (has == 0) return;
  const int c0 = __shfl(c, __ffsll(static_cast<unsigned long long>(has)) - 1);
  if (__ballot(c >= 0 && c != c0) == 0) {
    const int m = wave_max(c >= 0 ? val : 0);
    if (lane_id() == 0) atomicMax(&per_chain[c0], m);
  } else if (c >= 0) {
    atomicMax(&per_chain[c], val);
  }
}

// A CSR row [r0, r1) inside the edge arrays.  Anything else, which only a launch
// that broke off could leave, raises SCO_FLAG_STATE and reads as an empty row.
__device__ __forceinline__ void row_checked(const StepArgs& a, int& r0, int& r1) {
  const int cap2 = 2 * static_cast<int>(a.cap_und);
  if (r0 < 0 || r1 < r0 || r1 > cap2) {
    set_flag(a.sync, SCO_FLAG_STATE);
    r0 = r1 = 0;
  }
}

// atomicAdd of per-lane values into a per-chain LDS array; one atomic per wave when
// the lanes with a value share the chain (all lanes must call; c < 0: no value)
__device__ __forceinline__ void wave_sum_to(int* per_chain, int c, int val) {
  const uint64_t has = __ballot(c >= 0);
  if (has == 0) return;
  const int c0 = __shfl(c, __ffsll(static_cast<unsigned long long>(has)) - 1);
  if (__ballot(c >= 0 && c != c0) == 0) {
    int t = c >= 0 ? val : 0;
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if (lane_id() == 0 && t != 0) atomicAdd(&per_chain[c0], t);
  } else if (c >= 0 && val != 0) {
    atomicAdd(&per_chain[c], val);
  }
}

// Exclusive offsets of the q <= 255 class counts cnt[1..q] into off[0..q], taken by
// one wave (four counts per lane).  Every wave of a block may run it: they write the
// same values, so each can use the offsets at once, with no barrier after it.
__device__ __forceinline__ void wave_class_offsets(const int32_t* cnt, int32_t* off, int q) {
  const int lane = static_cast<int>(lane_id());
  int c4[4], s = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int idx = 1 + 4 * lane + r;
    c4[r] = idx <= q ? cnt[idx] : 0;
    s += c4[r];
  }
  int incl = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int x = __shfl_up(incl, o);
    if (lane >= o) incl += x;
  }
  int run = incl - s;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int idx = 1 + 4 * lane + r;
    run += c4[r];
    if (idx <= q) off[idx] = run;
  }
  if (lane == 0) off[0] = 0;
}

// 256-bit colour set without dynamic register indexing
struct ColorSet {
  uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
  __device__ __forceinline__ void add(int c) {
    const uint64_t b = 1ull << (c & 63);
    const int h = (c >> 6) & 3;
    w0 |= h == 0 ? b : 0ull;
    w1 |= h == 1 ? b : 0ull;
    w2 |= h == 2 ? b : 0ull;
    w3 |= h == 3 ? b : 0ull;
  }
  // adds c when `on` (no branch)
  __device__ __forceinline__ void add_if(bool on, int c) {
    const uint64_t b = on ? 1ull << (c & 63) : 0ull;
    const int h = (c >> 6) & 3;
    w0 |= h == 0 ? b : 0ull;
    w1 |= h == 1 ? b : 0ull;
    w2 |= h == 2 ? b : 0ull;
    w3 |= h == 3 ? b : 0ull;
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

// The same for palettes of at most 64 colours (every colour stored is below q).
struct ColorSet32 {
  uint32_t w = 0;
  __device__ __forceinline__ void add(int c) { w |= 1u << (c & 31); }
  __device__ __forceinline__ void add_if(bool on, int c) { w |= on ? 1u << (c & 31) : 0u; }
  __device__ __forceinline__ int first_free() const { return ~w ? __ffs(~w) - 1 : 32; }
};

struct ColorSet64 {
  uint64_t w = 0;
  __device__ __forceinline__ void add(int c) { w |= 1ull << (c & 63); }
  __device__ __forceinline__ void add_if(bool on, int c) { w |= on ? 1ull << (c & 63) : 0ull; }
  __device__ __forceinline__ int first_free() const {
    return ~w ? __ffsll(static_cast<unsigned long long>(~w)) - 1 : 64;
  }
};

// Rare-event counts of a phase (FP32 decisions recomputed in FP64, near ties): kept
// per thread for the first chain c0 of the block's range and added to its chain state
// once per block by flush (every thread calls it); other chains take one device atomic
// per event.
struct Tally {
  int c0;
  uint32_t rechecks = 0u, ties = 0u;
  __device__ __forceinline__ explicit Tally(int first) : c0(first) {}
  __device__ __forceinline__ void recheck(const StepArgs& a, int c) {
    if (c == c0) ++rechecks;
    else atomicAdd(&a.st[c].rechecks, 1ull);
  }
  __device__ __forceinline__ void tie(const StepArgs& a, int c) {
    if (c == c0) ++ties;
    else atomicAdd(&a.st[c].near_ties, 1ull);
  }
  __device__ __forceinline__ void flush(const StepArgs& a) {
    const unsigned long long r = block_sum(static_cast<unsigned long long>(rechecks));
    const unsigned long long t = block_sum(static_cast<unsigned long long>(ties));
    if (threadIdx.x == 0 && c0 < a.n_chains) {
      if (r) atomicAdd(&a.st[c0].rechecks, r);
      if (t) atomicAdd(&a.st[c0].near_ties, t);
    }
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
                 int8_t* __restrict__ spin, double* __restrict__ spin3, int64_t G) {
  const int64_t g = gtid();
  if (g >= G) return;
  const int c = chunk_chain[g >> SCO_CHUNK_SHIFT];
  const ChainDesc& d = cd[c];
  const int v = static_cast<int>(g - d.vbase);
  if (d.model == SCO_MODEL_HEIS) {  // uniform on the sphere, Philox(0, v, 0, INIT + 256 k)
    double x = 0.0, y = 0.0, z = 1.0;
    if (v < d.N && !sphere_point(0u, static_cast<uint32_t>(v), 0u, SCO_TAG_INIT, d.seed, d.chain_id, x, y, z)) {
      x = y = 0.0;
      z = 1.0;
    }
    spin3[3 * g] = x;
    spin3[3 * g + 1] = y;
    spin3[3 * g + 2] = z;
    spin[g] = 1;
    return;
  }
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
// One owner's scan over the displacement table: the state of an in-flight site.
struct Owner {
  int64_t g;       // global site
  int v, x, y, c;  // chain-local site, its coordinates, its chain
  int pos;         // table index of the last candidate (-1 before the first draw)
  uint32_t k;      // draws made
  double Cpos;     // C at pos
  uint32_t slo, shi;  // second half of the last Philox output: the next (odd) draw
  int si;          // the owner's spin
  double sx, sy, sz;  // the owner's Heisenberg spin
  int ns;          // survivors of the owner stored so far
  bool live;
};

// The fields of owner o at global site g of chain c that follow from the site alone.
template <bool Heis>
__device__ __forceinline__ void owner_load(const StepArgs& a, const ChainDesc& d, Owner& o, int64_t g, int c) {
  o.g = g;
  o.v = static_cast<int>(g - d.vbase);
  o.c = c;
  o.y = idiv_fp(o.v, d.inv_L);
  o.x = o.v - o.y * d.L;
  if constexpr (Heis) {
    o.sx = a.spin3[3 * g];
    o.sy = a.spin3[3 * g + 1];
    o.sz = a.spin3[3 * g + 2];
  } else {
    o.si = a.spin[g];
  }
}

// In-tile bond lists held in LDS: for at most kBondedCap sites with in-tile bonds and
// kAdjCap entries; a site beyond either reads its row from global memory instead.
constexpr int kBondedCap = 8192;
constexpr int kAdjCap = 10240;

// LDS of the colouring and sweep phases: the tile arrays of the local levels, or the
// bucket list of a block (block-local offsets) in the global levels and the sweeps.
struct TileLds {
  uint16_t cr[SCO_TILE_MAX];          // current colour | round of the decision << 8 (0: undecided)
  uint16_t list[SCO_TILE_MAX / 2];    // pending sites bucketed by colour
  uint32_t bmask[SCO_TILE_MAX / 32];  // bit i: site i has in-tile bonds
  uint16_t brank[SCO_TILE_MAX / 32];  // sites with in-tile bonds before word w
  uint16_t boff[kBondedCap + 1];      // the r-th such site's partners: adj[boff[r], boff[r+1])
  uint16_t adj[kAdjCap];
};
constexpr int kListCap = static_cast<int>(sizeof(TileLds) / sizeof(int32_t));
union alignas(16) PhaseLds {
  TileLds tile;
  int32_t list[kListCap];
};

// The first kSwC entries of a chain's cumulative couplings C and displacements hd,
// and a guide of kSwGuide buckets, staged in LDS for the switching of a block whose
// chunks all belong to that chain; nearly every candidate falls among them.  KL = 0:
// everything is read from global memory.
constexpr int kSwC = 5120;
constexpr int kSwGuide = 1 << 12;
// the switching's list of owners with a candidate, after its table head or alone
constexpr int kSwHeadBytes =
    kSwC * static_cast<int>(sizeof(double) + sizeof(uint32_t)) + (kSwGuide + 1) * static_cast<int>(sizeof(int32_t));
constexpr uint32_t kSwListCap = static_cast<uint32_t>((static_cast<int>(sizeof(int32_t)) * kListCap - kSwHeadBytes) / 2);
constexpr uint32_t kSwListCapAll =
    static_cast<uint32_t>(static_cast<int>(sizeof(int32_t)) * kListCap / 2) < 65536u
        ? static_cast<uint32_t>(static_cast<int>(sizeof(int32_t)) * kListCap / 2)
        : 65536u;
static_assert(kSwListCap >= static_cast<uint32_t>(kBlock), "the switching lists owners after its table head");
struct SwitchTables {
  const double* C;       // C_0 .. C_{KL-1}
  const uint32_t* hd;    // hd_0 .. hd_{KL-1}
  const int32_t* guide;  // guide[b] = first m with C_m >= b C_top / kSwGuide, b = 0..kSwGuide
  int KL;
  double guide_inv;      // kSwGuide / C_top
  int klast;             // K - 1 (the bracket's end above the last guide bucket)
  __device__ __forceinline__ double c_at(const ChainDesc& d, int m) const { return m < KL ? C[m] : ld_global(&d.C[m]); }
  __device__ __forceinline__ uint32_t hd_at(const ChainDesc& d, int m) const {
    return m < KL ? hd[m] : ld_global(&d.hd[m]);
  }
  // whether the LDS bracket of `target` lies inside the staged entries
  __device__ __forceinline__ bool in_head(double target) const {
    if (KL <= 0) return false;
    int b = static_cast<int>(target * guide_inv);
    b = b < 0 ? 0 : (b > kSwGuide ? kSwGuide : b);
    return ((b + 2 <= kSwGuide) ? guide[b + 2] : klast) < KL;
  }
};

// First table index m > pos with C_m >= target (guide-table bracket, then binary
// search over the FP64 cumulative couplings).  The LDS bracket is used when it lies
// inside the staged entries; both brackets contain the answer, so the result is the
// same either way.
__device__ __forceinline__ int table_search(const ChainDesc& d, const SwitchTables& tb, double target, int pos) {
  if (tb.KL > 0) {
    int b = static_cast<int>(target * tb.guide_inv);
    b = b < 0 ? 0 : (b > kSwGuide ? kSwGuide : b);
    const int hi0 = (b + 2 <= kSwGuide) ? tb.guide[b + 2] : d.K - 1;
    if (hi0 < tb.KL) {
      int lo = tb.guide[b > 0 ? b - 1 : 0], hi = hi0;
      lo = lo > pos + 1 ? lo : pos + 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tb.C[mid] >= target) hi = mid;
        else lo = mid + 1;
      }
      return lo;
    }
  }
  const double* __restrict__ C = d.C;
  const int K = d.K, NB = d.nguide;
  int b = static_cast<int>(target * d.guide_inv);
  b = b < 0 ? 0 : (b > NB ? NB : b);
  int lo = ld_global(&d.guide[b > 0 ? b - 1 : 0]);
  int hi = (b + 2 <= NB) ? ld_global(&d.guide[b + 2]) : K - 1;
  lo = lo > pos + 1 ? lo : pos + 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ld_global(&C[mid]) >= target) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// One draw of a live owner: the next candidate (table entry m, partner j, -1 when the
// displacement leaves an open lattice, and the draw index kc); false when the owner
// ends instead (the target passes C_top or the table is exhausted).  With precision
// 1 the exponential gap is computed in FP32; the FP64 outcome is certain unless the
// target lies within `tol` of C_top or of the table values it was compared with, and
// then the gap is recomputed in FP64 (counted in `rechecks`).  With may_park, a draw
// that would search the table in global memory (its target beyond the entries staged
// in LDS: a long bond, about one candidate in a hundred) or recompute in FP64 is not
// taken: `park` is set and the owner is resumed at the same draw later, so that the
// wave running it is not held by one lane's chain of dependent global loads.
template <class Desc>
__device__ __forceinline__ bool owner_candidate(const StepArgs& a, const Desc& desc_of, const SwitchTables& tb,
                                                uint32_t step, Owner& o, int& j, int& m, uint32_t& kc,
                                                Tally& tally, int& ddx, int& ddy, bool may_park, bool& park) {
  const ChainDesc& d = desc_of(o.c);
  const int K = d.K;
  if (o.pos >= K - 1) {  // no candidate lies beyond the last table entry
    o.live = false;
    return false;
  }
  uint32_t wlo, whi;
  if ((o.k & 1u) == 0) {
    const W4 r = philox10(step, static_cast<uint32_t>(o.v), o.k >> 1, SCO_TAG_SW, d.seed, d.chain_id);
    wlo = r.x;
    whi = r.y;
    o.slo = r.z;
    o.shi = r.w;
  } else {
    wlo = o.slo;
    whi = o.shi;
  }
  const double u1 = unit52(wlo, whi);
  bool done = false;
  if (d.precision == 1 && d.fp32_gap && may_park) {
    // -log u rounded through FP32 (u to float: 2^-24 relative; logf: about one ulp;
    // the product: two roundings) stays within inv_rate (2^-24 + 2^-22 E) of the exact
    // gap; tol takes four times that, plus the rounding of the FP64 sums.  fp32_gap
    // holds when inv_rate 2^-20 > 2e-12 C_top: a decision taken here is then far from
    // any near tie of the FP64 evaluation.
    const float E = -logf(static_cast<float>(u1));
    const double target = o.Cpos + static_cast<double>(E * d.inv_rate32);
    const double tol = static_cast<double>(d.inv_rate32) * (static_cast<double>(E) + 1.0) * 0x1p-20 + target * 0x1p-50;
    if (target - tol > d.C_top) {
      o.live = false;
      return false;
    }
    if (target + tol <= d.C_top) {
      if (tb.KL > 0 && !tb.in_head(target + tol)) {  // a long bond: searched later
        park = true;
        return false;
      }
      m = table_search(d, tb, target, o.pos);
      done = tb.c_at(d, m) >= target + tol && (m == o.pos + 1 || tb.c_at(d, m - 1) < target - tol);
    }
    if (!done) {
      // the owner is parked and finishes its scan in FP64 after the block's pool
      // (the draw is not consumed)
      tally.recheck(a, o.c);
      park = true;
      return false;
    }
  }
  if (!done) {
    const double target = o.Cpos + (-log(u1)) * d.inv_rate;
    if (may_park && target <= d.C_top && tb.KL > 0 && !tb.in_head(target)) {  // searched later
      park = true;
      return false;
    }
    if (near_tie(target, d.C_top)) tally.tie(a, o.c);
    if (target > d.C_top) {
      o.live = false;
      return false;
    }
    m = table_search(d, tb, target, o.pos);
    if (near_tie(target, tb.c_at(d, m)) || (m - 1 > o.pos && near_tie(target, tb.c_at(d, m - 1))))
      tally.tie(a, o.c);
  }
  const uint32_t p = tb.hd_at(d, m);
  const int dx = static_cast<int16_t>(p & 0xFFFFu), dy = static_cast<int16_t>(p >> 16);
  j = partner_of(o.x, o.y, dx, dy, d.L, d.periodic);
  ddx = dx;
  ddy = dy;
  kc = o.k;
  o.pos = m;
  o.Cpos = tb.c_at(d, m);
  ++o.k;
  return true;
}

// Whether candidate (j, m, kc) of owner o survives, given the partner's spin sj:
// antiparallel spins always, parallel ones (kappa > 1) with probability theta_m.
// Heisenberg: the candidate survives with probability (1 - P_ij) / pbar_m =
// expm1(beta (V_ij - V^max)) / expm1(-2 beta J_m) at the current spins (Eqs. 1-2).
template <class Desc>
__device__ __forceinline__ bool owner_survives_heis(const StepArgs& a, const Desc& desc_of, uint32_t step,
                                                    const Owner& o, int j, int m, uint32_t kc, int dx, int dy,
                                                    double bx, double by, double bz, Tally& tally) {
  if (j < 0) return false;
  const ChainDesc& d = desc_of(o.c);
  const W4 t = philox10(step, static_cast<uint32_t>(o.v), kc, SCO_TAG_TH, d.seed, d.chain_id);
  const double u = unit52(t.x, t.y);
  const double Jm = ld_global(&d.J[m]);
  const double V = heis_pair(o.sx, o.sy, o.sz, bx, by, bz, dx, dy, Jm);
  const double ratio = expm1(d.beta * (V - Jm)) / ld_global(&d.hden[m]);
  if (fabs(u - ratio) < 1e-12) tally.tie(a, o.c);
  return u < ratio;
}

template <class Desc>
__device__ __forceinline__ bool owner_survives(const Desc& desc_of, uint32_t step, const Owner& o, int j, int m,
                                               uint32_t kc, int sj) {
  if (j < 0) return false;
  const ChainDesc& d = desc_of(o.c);
  if (o.si != sj) return true;
  if (d.hard) return false;
  const W4 t = philox10(step, static_cast<uint32_t>(o.v), kc, SCO_TAG_TH, d.seed, d.chain_id);
  return unit52(t.x, t.y) < ld_global(&d.theta[m]);
}


// One thread per owner site.  Candidate bonds of owner v: the table intervals
// (C_{m-1}, C_m] hit by a Poisson process of rate (kappa+1) beta run from C = 0,
// found by drawing exponential gaps E = -log(u) and locating C_pos + E T/(kappa+1)
// in the cumulative table (guide-table bracket, then binary search).  A candidate
// survives if its spins are antiparallel or, when kappa > 1, with probability
// theta_m if they are parallel.  Draw k of owner v is half k&1 of
// Philox(step, v, k>>1, SW); the thinning draw of candidate k is Philox(step, v, k, TH).
//
// Block b owns a contiguous range of chunks; each thread keeps two owners of that
// range in flight and takes the next from the block's pool as soon as one ends, so a
// wave is held neither by its slowest owner nor by its busiest lane.  Survivors go to the block's region (one LDS atomic per wave
// and append); its count is written to the entry of the range's first chunk.
template <bool Heis>
__device__ __forceinline__ void phase_switch(const StepArgs& a, uint32_t step, int32_t* lds_raw) {
  __shared__ uint32_t s_count, s_next, s_park, s_ptake, s_nlist;
  const uint32_t cap_chunk = a.cap_und / static_cast<uint32_t>(a.nchunks);
  const int cpb = (a.nchunks + static_cast<int>(gridDim.x) - 1) / static_cast<int>(gridDim.x);
  const int ch0 = min(static_cast<int>(blockIdx.x) * cpb, a.nchunks), ch1 = min(ch0 + cpb, a.nchunks);
  const uint32_t e_base = static_cast<uint32_t>(ch0) * cap_chunk;
  const uint32_t cap_blk = static_cast<uint32_t>(ch1 - ch0) * cap_chunk;
  if (threadIdx.x == 0) s_count = s_next = s_park = s_ptake = 0;
  __syncthreads();
  const uint32_t lane = lane_id();
  // parked owners (three int4 each, in the block's share of the bucket records, which
  // the switching does not use)
  int4* const parked = a.rec + (static_cast<int64_t>(ch0) << SCO_CHUNK_SHIFT);
  const uint32_t park_cap = (static_cast<uint32_t>(ch1 - ch0) << SCO_CHUNK_SHIFT) / 3u;
  // returns the owner's count of stored survivors after this append
  auto append = [&](bool f, int64_t g, int v, int j, int m, int ns) -> int {
    const uint64_t mask = __ballot(f);
    if (mask == 0) return ns;
    const int leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
    uint32_t e0 = 0;
    if (static_cast<int>(lane) == leader) e0 = atomicAdd(&s_count, static_cast<uint32_t>(__popcll(mask)));
    e0 = __shfl(e0, leader);
    if (f) {
      const uint32_t eo = e0 + static_cast<uint32_t>(__popcll(mask & ((1ull << lane) - 1ull)));
      if (eo < cap_blk) {
        const uint32_t e = e_base + eo;
        const int32_t gj = static_cast<int32_t>(g - v + j);  // the chain's base is g - v
        a.ea[e] = static_cast<int32_t>(g);
        a.eb[e] = gj;
        a.em[e] = m;
        a.er[e] = ns++;
      } else {
        set_flag(a.sync, SCO_FLAG_OVERFLOW);
      }
    }
    return ns;
  };
  Tally tally(ch0 < ch1 ? a.chunk_chain[ch0] : 0);
  // lst: LDS room for lcap (>= kBlock) owner indices of a segment of the block's owners
  auto run = [&](const auto& desc_of, const SwitchTables& tb, int c_uni, uint16_t* lst, uint32_t lcap) {
  const uint32_t total = static_cast<uint32_t>(ch1 - ch0) << SCO_CHUNK_SHIFT;
  // phase 0, segment by segment: every owner's first draw is taken by one lane each
  // (a convergent pass); an owner whose uniform lies below u_first_end has no
  // candidate and is done (about half of them), the others are listed and dealt to
  // the lanes, which run their draws (FP32 where the chain allows);
  // phase 1: the parked owners (a long bond's table search, or an FP32 draw that
  // needs FP64), every draw in FP64, the lanes' global searches in flight together
  for (int phase = 0; phase < 2; ++phase) {
   uint32_t s0 = 0;
   do {
    const bool may_park = phase == 0;
    uint32_t np = 0, s1 = total;
    if (phase == 1) {
      __syncthreads();
      mark(a.trace, 503);
      np = min(s_park, park_cap);
      if (np == 0) break;  // block-uniform
    } else {
      s1 = min(s0 + lcap, total);
      __syncthreads();  // the previous segment's list is dealt
      if (threadIdx.x == 0) s_nlist = s_next = 0;
      __syncthreads();
      for (uint32_t i0 = s0; i0 < s1; i0 += kBlock) {
        const uint32_t idx = i0 + threadIdx.x;
        bool keep = false;
        if (idx < s1) {
          const int64_t g = (static_cast<int64_t>(ch0) << SCO_CHUNK_SHIFT) + idx;
          const int c = c_uni >= 0 ? c_uni : a.chunk_chain[g >> SCO_CHUNK_SHIFT];
          const ChainDesc& d = desc_of(c);
          const int v = static_cast<int>(g - d.vbase);
          if (v < d.N) {  // else chunk padding
            const W4 r = philox10(step, static_cast<uint32_t>(v), 0u, SCO_TAG_SW, d.seed, d.chain_id);
            keep = !(unit52(r.x, r.y) < d.u_first_end);
          }
          if (!keep) a.own[g] = 0;  // an owner with no survivor (or padding)
        }
        const uint64_t m = __ballot(keep);
        if (m != 0) {
          const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
          uint32_t base = 0;
          if (static_cast<int>(lane) == leader) base = atomicAdd(&s_nlist, static_cast<uint32_t>(__popcll(m)));
          base = __shfl(base, leader);
          if (keep) lst[base + __popcll(m & ((1ull << lane) - 1ull))] = static_cast<uint16_t>(idx - s0);
        }
      }
      __syncthreads();
      if (s0 == 0) mark(a.trace, 502);
    }
    const uint32_t nlist = s_nlist;
    bool pool = true;
    Owner O[kOwners];
    // the next parked owner for each lane that asks (one LDS atomic per wave)
    auto take_parked = [&](Owner& o, bool need) {
      const uint64_t m = __ballot(need);
      if (m == 0) return;
      const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
      uint32_t base = 0;
      if (static_cast<int>(lane) == leader) base = atomicAdd(&s_ptake, static_cast<uint32_t>(__popcll(m)));
      base = __shfl(base, leader);
      if (!need) return;
      const uint32_t idx = base + static_cast<uint32_t>(__popcll(m & ((1ull << lane) - 1ull)));
      if (idx >= np) {
        o.live = false;
        pool = false;
        return;
      }
      const int4 e0 = parked[3 * idx], e1 = parked[3 * idx + 1], e2 = parked[3 * idx + 2];
      owner_load<Heis>(a, desc_of(e0.y), o, e0.x, e0.y);
      o.pos = e0.z;
      o.k = static_cast<uint32_t>(e0.w);
      o.Cpos = __hiloint2double(e1.y, e1.x);
      o.slo = static_cast<uint32_t>(e1.z);
      o.shi = static_cast<uint32_t>(e1.w);
      o.ns = e2.x;
      o.live = true;
    };
    // the next listed owner for each lane that asks (one LDS atomic per wave): lanes
    // that finish early take more, so a wave is not held by its busiest lane
    auto take_listed = [&](Owner& o, bool need) {
      const uint64_t m = __ballot(need);
      if (m == 0) return;
      const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
      uint32_t base = 0;
      if (static_cast<int>(lane) == leader) base = atomicAdd(&s_next, static_cast<uint32_t>(__popcll(m)));
      base = __shfl(base, leader);
      if (!need) return;
      const uint32_t j = base + static_cast<uint32_t>(__popcll(m & ((1ull << lane) - 1ull)));
      if (j >= nlist) {
        o.live = false;
        pool = false;
        return;
      }
      const int64_t g = (static_cast<int64_t>(ch0) << SCO_CHUNK_SHIFT) + s0 + lst[j];
      const int c = c_uni >= 0 ? c_uni : a.chunk_chain[g >> SCO_CHUNK_SHIFT];
      owner_load<Heis>(a, desc_of(c), o, g, c);
      o.pos = -1;
      o.k = 0;
      o.Cpos = 0.0;
      o.ns = 0;
      o.live = true;
    };
    auto take = [&](Owner& o, bool need) {
      if (phase == 0) take_listed(o, need);
      else take_parked(o, need);
    };
#pragma unroll
    for (int u = 0; u < kOwners; ++u) {
      O[u].ns = 0;
      O[u].live = false;
      take(O[u], pool);
    }
    auto any_live = [&]() {
      bool l = false;
#pragma unroll
      for (int u = 0; u < kOwners; ++u) l = l || O[u].live;
      return l;
    };
    while (__ballot(any_live()) != 0) {
      // every owner's candidate first, then all partner spins in flight together
      int jc[kOwners], mc[kOwners], sc[kOwners], xc[kOwners], yc[kOwners];
      double bx[kOwners], by[kOwners], bz[kOwners];
      uint32_t kc[kOwners];
      bool cc[kOwners], fin[kOwners];
#pragma unroll
      for (int u = 0; u < kOwners; ++u) {
        jc[u] = -1;
        mc[u] = 0;
        kc[u] = 0;
        xc[u] = yc[u] = 0;
        const bool was_live = O[u].live;
        bool park = false;
        cc[u] = O[u].live &&
                owner_candidate(a, desc_of, tb, step, O[u], jc[u], mc[u], kc[u], tally, xc[u], yc[u], may_park, park);
        if (park) {
          const uint32_t idx = atomicAdd(&s_park, 1u);
          if (idx < park_cap) {  // saved: the lane takes another owner
            const Owner& o = O[u];
            parked[3 * idx] = make_int4(static_cast<int32_t>(o.g), o.c, o.pos, static_cast<int32_t>(o.k));
            parked[3 * idx + 1] = make_int4(__double2loint(o.Cpos), __double2hiint(o.Cpos), static_cast<int32_t>(o.slo),
                                            static_cast<int32_t>(o.shi));
            parked[3 * idx + 2] = make_int4(o.ns, 0, 0, 0);
            O[u].live = false;
            O[u].ns = 0;
            fin[u] = false;  // not ended: resumed in the second pass
            continue;
          } else {  // no room: this draw in FP64 now
            bool again = false;
            cc[u] = owner_candidate(a, desc_of, tb, step, O[u], jc[u], mc[u], kc[u], tally, xc[u], yc[u], false, again);
          }
        }
        fin[u] = was_live && !O[u].live;
      }
#pragma unroll
      for (int u = 0; u < kOwners; ++u) {
        if constexpr (Heis) {
          bx[u] = by[u] = bz[u] = 0.0;
          if (cc[u] && jc[u] >= 0) {
            const double* B = a.spin3 + 3 * (desc_of(O[u].c).vbase + jc[u]);
            bx[u] = B[0];
            by[u] = B[1];
            bz[u] = B[2];
          }
        } else {
          sc[u] = cc[u] && jc[u] >= 0 ? a.spin[desc_of(O[u].c).vbase + jc[u]] : 0;
        }
      }
#pragma unroll
      for (int u = 0; u < kOwners; ++u) {
        bool f;
        if constexpr (Heis)
          f = cc[u] && owner_survives_heis(a, desc_of, step, O[u], jc[u], mc[u], kc[u], xc[u], yc[u], bx[u], by[u],
                                           bz[u], tally);
        else
          f = cc[u] && owner_survives(desc_of, step, O[u], jc[u], mc[u], kc[u], sc[u]);
        O[u].ns = append(f, O[u].g, O[u].v, jc[u], mc[u], O[u].ns);
      }
      // an ended owner's survivor count: the front of its row
#pragma unroll
      for (int u = 0; u < kOwners; ++u) {
        if (fin[u]) {
          if (O[u].ns > 0xFFFF) set_flag(a.sync, SCO_FLAG_OVERFLOW);
          a.own[O[u].g] = static_cast<uint16_t>(O[u].ns);
          O[u].ns = 0;
        }
        take(O[u], !O[u].live && pool);
      }
    }
    s0 = s1;
   } while (phase == 0 && s0 < total);
  }
  };
  if (ch0 < ch1) {
    // the chunks of a block usually belong to one chain: its descriptor is then
    // block-uniform and read with scalar loads
    const int c_lo = a.chunk_chain[ch0], c_hi = a.chunk_chain[ch1 - 1];
    if (c_lo == c_hi) {
      const ChainDesc& d0 = a.cd[c_lo];
      // the chain's table head in LDS (the guide every nguide / kSwGuide-th bucket)
      double* lC = reinterpret_cast<double*>(lds_raw);
      uint32_t* lhd = reinterpret_cast<uint32_t*>(lC + kSwC);
      int32_t* lg = reinterpret_cast<int32_t*>(lhd + kSwC);
      const int gs = d0.nguide / kSwGuide;
      const int KL = (gs >= 1 && gs * kSwGuide == d0.nguide) ? min(d0.K, kSwC) : 0;
      for (int i = threadIdx.x; i < KL; i += kBlock) {
        lC[i] = ld_global(&d0.C[i]);
        lhd[i] = ld_global(&d0.hd[i]);
      }
      if (KL > 0)
        for (int b = threadIdx.x; b <= kSwGuide; b += kBlock) lg[b] = ld_global(&d0.guide[b * gs]);
      __syncthreads();
      mark(a.trace, 501);
      const SwitchTables tb{lC, lhd, lg, KL, d0.guide_inv / gs, d0.K - 1};
      uint16_t* lst = reinterpret_cast<uint16_t*>(lg + kSwGuide + 1);
      run([&](int) -> const ChainDesc& { return d0; }, tb, c_lo, lst, kSwListCap);
    } else {
      const SwitchTables tb{nullptr, nullptr, nullptr, 0, 0.0, 0};
      run([&](int c) -> const ChainDesc& { return a.cd[c]; }, tb, -1, reinterpret_cast<uint16_t*>(lds_raw),
          kSwListCapAll);
    }
  }
  __syncthreads();
  mark(a.trace, 504);
  // The partners' counts, from the block's survivor list (issued after the draws, so
  // no load of the draw loop waits behind them).  The count before a survivor's
  // increment is its slot among its partner's incoming survivors, kept beside its rank
  // (er: rank | place << 16 | in-range bit << 31).  A partner inside the block's own
  // range (most: the bonds are short) is counted in LDS, then added to its owner
  // count; one outside it, with a device atomic on deg.  A row holds the owner's
  // survivors first, by rank, then the in-range incoming ones (place: the owner count
  // plus the slot), and the others from the row's end (place: the slot).
  const uint32_t ne = min(s_count, cap_blk);
  uint32_t* const er = reinterpret_cast<uint32_t*>(a.er) + e_base;
  const int64_t glo = static_cast<int64_t>(ch0) << SCO_CHUNK_SHIFT;
  const uint32_t nloc = static_cast<uint32_t>(ch1 - ch0) << SCO_CHUNK_SHIFT;
  const bool local = nloc / 2u <= static_cast<uint32_t>(kListCap);  // block-uniform
  uint32_t* const lcnt = reinterpret_cast<uint32_t*>(lds_raw);       // two u16 counts per word
  if (local) {
    for (uint32_t k = threadIdx.x; k < nloc / 2u; k += kBlock) lcnt[k] = 0u;
    __syncthreads();
  }
  for (uint32_t e0 = 0; e0 < ne; e0 += kScan * kBlock) {
    int32_t pj[kScan];
    uint32_t rk[kScan];
#pragma unroll
    for (int r = 0; r < kScan; ++r) {
      const uint32_t e = e0 + r * kBlock + threadIdx.x;
      pj[r] = -1;
      rk[r] = 0;
      if (e < ne) {
        pj[r] = a.eb[e_base + e];
        rk[r] = er[e];
      }
    }
    uint32_t sl[kScan], ow[kScan];
    bool in[kScan];
#pragma unroll
    for (int r = 0; r < kScan; ++r) {
      const uint32_t li = static_cast<uint32_t>(pj[r] - glo);
      in[r] = local && pj[r] >= 0 && li < nloc;
      sl[r] = ow[r] = 0u;
      if (in[r]) {
        ow[r] = a.own[pj[r]];  // written by this block's owners
        const uint32_t sh = 16u * (li & 1u);
        sl[r] = (atomicAdd(&lcnt[li >> 1], 1u << sh) >> sh) & 0xFFFFu;
      } else if (pj[r] >= 0) {
        sl[r] = static_cast<uint32_t>(atomicAdd(&a.deg[pj[r]], 1));
      }
    }
#pragma unroll
    for (int r = 0; r < kScan; ++r) sl[r] += ow[r];
#pragma unroll
    for (int r = 0; r < kScan; ++r) {
      const uint32_t e = e0 + r * kBlock + threadIdx.x;
      if (pj[r] < 0) continue;
      // an in-range count reaching 2^16 carries into its neighbour: flagged either way
      if (sl[r] >= 0x7FFFu || rk[r] > 0xFFFFu) set_flag(a.sync, SCO_FLAG_OVERFLOW);
      er[e] = (rk[r] & 0xFFFFu) | ((sl[r] & 0x7FFFu) << 16) | (in[r] ? 0x80000000u : 0u);
    }
  }
  if (local) {
    // the in-range counts join the owner counts (this block alone wrote them)
    __syncthreads();
    uint32_t* const own2 = reinterpret_cast<uint32_t*>(a.own + glo);
    for (uint32_t k = threadIdx.x; k < nloc / 2u; k += kBlock) {
      const uint32_t c = lcnt[k];
      if (c == 0u) continue;
      const uint32_t o = own2[k];
      const uint32_t lo = (o & 0xFFFFu) + (c & 0xFFFFu), hi = (o >> 16) + (c >> 16);
      if (lo > 0xFFFFu || hi > 0xFFFFu) set_flag(a.sync, SCO_FLAG_OVERFLOW);
      own2[k] = (lo & 0xFFFFu) | (hi << 16);
    }
  }
  if (threadIdx.x == 0)
    for (int ch = ch0; ch < ch1; ++ch) a.ecount[ch] = ch == ch0 ? ne : 0u;
  tally.flush(a);  // its block sums also order the block's work before the return
  mark(a.trace, 505);
}

// ------------------------------------------------------------------ prefix sum
// Exclusive scan of the n sums in[i] + in2[i] in tiles of kTile: (1) every block sums its tiles
// into agg[t]; (2) a device-wide barrier; (3) each block adds the sums of the tiles
// before each of its tiles and scans the tile.  Global memory is read and written in
// coalesced rows (item k * kBlock + thread); the scan order goes through LDS, padded
// one word in 32 against bank conflicts.  When no block has more than one tile, a
// thread keeps its values in registers from (1) to (3) instead of reading them twice.
// out[n] = total.  out may alias in.
constexpr int kItems = SCO_SCAN_ITEMS;  // one tile per block at L = 2304 on 256 blocks
constexpr int kTile = kBlock * kItems;
constexpr int kScanLds = kTile + kTile / 32;  // words of the padded tile in LDS

__device__ __forceinline__ bool scan_two_pass(const int32_t* in, const uint16_t* in2, int64_t n64, int32_t* out,
                                              long long* agg, int32_t* lds, SyncWords* sync) {
  __shared__ int32_t wsum[kWaves];
  const int n = static_cast<int>(n64);  // G < 2^31
  const int nt = (n + kTile - 1) / kTile;
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  const int tid = static_cast<int>(threadIdx.x);
  // padded LDS addresses (one word in 32: index x at x + x / 32): row item k of this
  // thread at rowb + k kRow, scan item i at pad(cb + i)
  const int rowb = tid + (tid >> 5), cb = tid * kItems;
  constexpr int kRow = kBlock + kBlock / 32;
  auto pad = [](int x) { return x + (x >> 5); };
  const bool one = nt <= static_cast<int>(gridDim.x);
  int32_t kept[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) kept[k] = 0;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const int tb = t * kTile + tid;
    long long s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int idx = tb + k * kBlock;
      const int32_t v = idx < n ? in[idx] + static_cast<int32_t>(in2[idx]) : 0;
      kept[k] = v;
      s += v;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) agg[t] = s;
  }
  if (!grid_barrier(sync)) return false;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const int tb = t * kTile + tid;
    // coalesced rows into LDS
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int idx = tb + k * kBlock;
      lds[rowb + k * kRow] = one ? kept[k] : (idx < n ? in[idx] + static_cast<int32_t>(in2[idx]) : 0);
    }
    // sum of the tiles before t
    long long pre = 0;
    for (int k = tid; k < t; k += kBlock) pre += agg[k];
    pre = block_sum(pre);  // in every thread; its barriers also order the LDS stores
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) s += lds[pad(cb + i)];
    int32_t incl = s;
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t x = __shfl_up(incl, o);
      if (lane >= static_cast<uint32_t>(o)) incl += x;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int32_t woff = 0;
    for (int i = 0; i < w; ++i) woff += wsum[i];
    int32_t run = static_cast<int32_t>(pre) + woff + incl - s;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const int32_t v = lds[pad(cb + i)];
      lds[pad(cb + i)] = run;
      run += v;
    }
    if (t == nt - 1 && threadIdx.x == kBlock - 1) out[n] = run;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int idx = tb + k * kBlock;
      if (idx < n) out[idx] = lds[rowb + k * kRow];
    }
    __syncthreads();
  }
  return true;
}

// both directions of every survivor into the CSR; the partner counts of the block's
// chunks back to zero for the next step's switching (the scan has read them, and
// nothing later in the step does)
__device__ __forceinline__ void phase_scatter(const StepArgs& a) {
  const uint32_t cap_chunk = a.cap_und / static_cast<uint32_t>(a.nchunks);
  const int cpb = (a.nchunks + static_cast<int>(gridDim.x) - 1) / static_cast<int>(gridDim.x);
  const int ch0 = min(static_cast<int>(blockIdx.x) * cpb, a.nchunks), ch1 = min(ch0 + cpb, a.nchunks);
  const int64_t cap2 = 2 * static_cast<int64_t>(a.cap_und);
  for (int64_t g = (static_cast<int64_t>(ch0) << SCO_CHUNK_SHIFT) + threadIdx.x;
       g < (static_cast<int64_t>(ch1) << SCO_CHUNK_SHIFT); g += kBlock)
    a.deg[g] = 0;
  // the switching stored the block's survivors from its first chunk's region on (the
  // same grid runs both), and the count there; one read, not one per chunk
  if (ch0 < ch1) {
    const int ch = ch0;
    const uint32_t e0 = static_cast<uint32_t>(ch) * cap_chunk, e1 = e0 + a.ecount[ch];
    // kScan survivors per thread and iteration, their loads issued together
    for (uint32_t eb = e0; eb < e1; eb += kScan * kBlock) {
      int32_t u[kScan], w[kScan], m[kScan], rk[kScan];
      bool ok[kScan];
#pragma unroll
      for (int r = 0; r < kScan; ++r) {
        const uint32_t e = eb + r * kBlock + threadIdx.x;
        ok[r] = e < e1;
        u[r] = w[r] = m[r] = rk[r] = 0;
        if (ok[r]) {
          u[r] = a.ea[e];
          w[r] = a.eb[e];
          m[r] = a.em[e];
          rk[r] = a.er[e];
        }
      }
      // the owner's entries at the front of its row, at their rank; the partner's
      // entry at its place: from the front when its owner's block holds the partner
      // (after the partner's own entries), else from the back
      int64_t pu[kScan], pw[kScan];
#pragma unroll
      for (int r = 0; r < kScan; ++r) {
        pu[r] = pw[r] = -1;
        if (ok[r]) {
          const uint32_t rs = static_cast<uint32_t>(rk[r]);
          const int64_t place = (rs >> 16) & 0x7FFFu;
          pu[r] = static_cast<int64_t>(a.row_ptr[u[r]]) + (rs & 0xFFFFu);
          pw[r] = (rs >> 31) ? a.row_ptr[w[r]] + place : a.row_ptr[w[r] + 1] - 1 - place;
        }
      }
#pragma unroll
      for (int r = 0; r < kScan; ++r) {
        if (!ok[r]) continue;
        if (pu[r] < 0 || pu[r] >= cap2 || pw[r] < 0 || pw[r] >= cap2) {  // cannot happen: degrees sum to 2 e
          set_flag(a.sync, SCO_FLAG_OVERFLOW);
          continue;
        }
        a.col[pu[r]] = w[r];
        a.attr[pu[r]] = m[r];
        a.col[pw[r]] = u[r];
        a.attr[pw[r]] = m[r];
      }
    }
  }
}

// Sorts each row ascending by neighbour; union degree |CSR(v) u NN(v)|; Delta and
// directed bond count per chain.  Block b takes a contiguous range of chunks.  When
// every site of the range fits the LDS queue (q_cap entries), a first pass reads only the row
// offsets (kScanRow chunks per iteration): an empty row, the usual case, has its
// lattice neighbour count as union degree, and the sites with bonds are queued; a
// second pass reads, sorts and checks the queued rows.  Otherwise each site takes the
// full path, kScan chunks per iteration.  When the block's range is one chain (the
// usual case) its descriptor is block-uniform and the maxima and sum are kept per
// thread and reduced once at the end; otherwise they gather in LDS per row (one atomic
// per wave when the wave is one chain).  Either way they reach the chain states once
// per block.
constexpr int kScanRow = 8;
__device__ __forceinline__ void phase_rowsort(const StepArgs& a, int32_t* lds_q, int q_cap) {
  __shared__ int32_t rmax[SCO_MAXCHAINS];  // union degree
  __shared__ int32_t rsum[SCO_MAXCHAINS];  // bonds
  __shared__ int32_t rbmx[SCO_MAXCHAINS];  // bond degree
  __shared__ int32_t s_nq;
  const int cpb = (a.nchunks + static_cast<int>(gridDim.x) - 1) / static_cast<int>(gridDim.x);
  const int ch0 = min(static_cast<int>(blockIdx.x) * cpb, a.nchunks), ch1 = min(ch0 + cpb, a.nchunks);
  for (int c = threadIdx.x; c < a.n_chains; c += kBlock) rmax[c] = rsum[c] = rbmx[c] = 0;
  if (threadIdx.x == 0) s_nq = 0;
  __syncthreads();
  const int c_uni = ch0 < ch1 && a.chunk_chain[ch0] == a.chunk_chain[ch1 - 1] ? a.chunk_chain[ch0] : -1;
  // per-thread maximum union degree, maximum and sum of bond degrees (c_uni >= 0)
  int t_umax = 0, t_bmax = 0, t_bsum = 0;
  auto tally_row = [&](int c, int udeg, int rowlen, bool bonds) __attribute__((always_inline)) {
    if (c_uni >= 0) {
      if (c >= 0) {
        t_umax = max(t_umax, udeg);
        t_bmax = max(t_bmax, rowlen);
        t_bsum += rowlen;
      }
    } else {
      wave_max_to(rmax, c, udeg);
      if (bonds) {
        wave_max_to(rbmx, c, rowlen);
        wave_sum_to(rsum, c, rowlen);
      }
    }
  };
  // the full path for up to kScan sites per thread (g < 0: none): row read in one
  // round, sorted in registers when short (nearly all), union degree against the
  // lattice neighbours
  auto full_rows = [&](const int64_t (&gs)[kScan]) __attribute__((always_inline)) {
    int cs[kScan], r0[kScan], r1[kScan];
    bool ok[kScan];
#pragma unroll
    for (int r = 0; r < kScan; ++r) {
      ok[r] = false;
      cs[r] = -1;
      r0[r] = r1[r] = 0;
      if (gs[r] >= 0) {
        cs[r] = c_uni >= 0 ? c_uni : a.chunk_chain[gs[r] >> SCO_CHUNK_SHIFT];
        ok[r] = static_cast<int>(gs[r] - a.cd[cs[r]].vbase) < a.cd[cs[r]].N;
        if (ok[r]) {
          r0[r] = a.row_ptr[gs[r]];
          r1[r] = a.row_ptr[gs[r] + 1];
        }
      }
    }
    // rows of up to kRowReg entries (nearly all) are read in one round for all kScan
    // rows, sorted in registers and written back; longer ones are sorted in place
    constexpr int kRowReg = 4;
    int kc[kScan][kRowReg], ka[kScan][kRowReg];
#pragma unroll
    for (int r = 0; r < kScan; ++r) {
      row_checked(a, r0[r], r1[r]);
      const int len = r1[r] - r0[r];
#pragma unroll
      for (int i = 0; i < kRowReg; ++i) {
        const bool in = len <= kRowReg && i < len;
        kc[r][i] = in ? a.col[r0[r] + i] : INT32_MAX;
        ka[r][i] = in ? a.attr[r0[r] + i] : 0;
      }
    }
#pragma unroll
    for (int r = 0; r < kScan; ++r) {
      int udeg = 0, rowlen = 0;
      if (ok[r]) {
        const ChainDesc& d = a.cd[cs[r]];
        const int v = static_cast<int>(gs[r] - d.vbase);
        const int q0 = r0[r], q1 = r1[r];
        rowlen = q1 - q0;
        const int y = idiv_fp(v, d.inv_L), x = v - y * d.L;
        int nb[4];
        nn_sites(x, y, d.L, d.periodic, nb);
        udeg = rowlen;
        if (rowlen <= kRowReg) {
          // adjacent exchanges on strictly greater keys: a stable sort (padding last)
          auto cx = [&](int i) {
            const bool sw = kc[r][i] > kc[r][i + 1];
            const int c0 = kc[r][i], a0 = ka[r][i];
            kc[r][i] = sw ? kc[r][i + 1] : c0;
            ka[r][i] = sw ? ka[r][i + 1] : a0;
            kc[r][i + 1] = sw ? c0 : kc[r][i + 1];
            ka[r][i + 1] = sw ? a0 : ka[r][i + 1];
          };
          cx(0); cx(1); cx(2); cx(0); cx(1); cx(0);
          if (rowlen > 1)
#pragma unroll
            for (int i = 0; i < kRowReg; ++i)
              if (i < rowlen) {
                a.col[q0 + i] = kc[r][i];
                a.attr[q0 + i] = ka[r][i];
              }
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            if (nb[t] < 0) continue;
            const int32_t gu = static_cast<int32_t>(d.vbase + nb[t]);
            bool dup = false;
#pragma unroll
            for (int i = 0; i < kRowReg; ++i) dup |= (kc[r][i] == gu);
            udeg += dup ? 0 : 1;
          }
        } else {
          int32_t* __restrict__ col = a.col;
          int32_t* __restrict__ attr = a.attr;
          for (int q = q0 + 1; q < q1; ++q) {
            const int32_t kq = col[q], aq = attr[q];
            int b = q - 1;
            while (b >= q0 && col[b] > kq) {
              col[b + 1] = col[b];
              attr[b + 1] = attr[b];
              --b;
            }
            col[b + 1] = kq;
            attr[b + 1] = aq;
          }
          bool dup[4] = {false, false, false, false};
          for (int b = q0; b < q1; ++b) {
            const int32_t cb = col[b];
#pragma unroll
            for (int t = 0; t < 4; ++t) dup[t] |= nb[t] >= 0 && cb == static_cast<int32_t>(d.vbase + nb[t]);
          }
#pragma unroll
          for (int t = 0; t < 4; ++t) udeg += (nb[t] >= 0 && !dup[t]) ? 1 : 0;
        }
      }
      tally_row(ok[r] ? cs[r] : -1, udeg, rowlen, true);
    }
  };
  const bool queued = static_cast<int64_t>(ch1 - ch0) * kBlock <= q_cap;
  if (queued) {
    const uint32_t lane = lane_id();
    for (int chb = ch0; chb < ch1; chb += kScanRow) {
      int cs[kScanRow], r0[kScanRow], r1[kScanRow];
      bool ok[kScanRow];
#pragma unroll
      for (int r = 0; r < kScanRow; ++r) {
        const int ch = chb + r;
        ok[r] = false;
        cs[r] = -1;
        r0[r] = r1[r] = 0;
        if (ch < ch1) {
          cs[r] = c_uni >= 0 ? c_uni : a.chunk_chain[ch];
          const int64_t g = (static_cast<int64_t>(ch) << SCO_CHUNK_SHIFT) + threadIdx.x;
          ok[r] = static_cast<int>(g - a.cd[cs[r]].vbase) < a.cd[cs[r]].N;
          if (ok[r]) {
            r0[r] = a.row_ptr[g];
            r1[r] = a.row_ptr[g + 1];
          }
        }
      }
#pragma unroll
      for (int r = 0; r < kScanRow; ++r) {
        const int64_t g = (static_cast<int64_t>(chb + r) << SCO_CHUNK_SHIFT) + threadIdx.x;
        if (ok[r]) row_checked(a, r0[r], r1[r]);
        const bool push = ok[r] && r1[r] > r0[r];
        const uint64_t pm = __ballot(push);
        if (pm != 0) {
          const int leader = __ffsll(static_cast<unsigned long long>(pm)) - 1;
          int base = 0;
          if (static_cast<int>(lane) == leader) base = atomicAdd(&s_nq, __popcll(pm));
          base = __shfl(base, leader);
          if (push) lds_q[base + __popcll(pm & ((1ull << lane) - 1ull))] = static_cast<int32_t>(g);
        }
        // an empty row: the union degree is the number of lattice neighbours
        int udeg = 0;
        if (ok[r] && !push) {
          const ChainDesc& d = a.cd[cs[r]];
          if (d.periodic) {
            udeg = 4;
          } else {
            const int v = static_cast<int>(g - d.vbase);
            const int y = idiv_fp(v, d.inv_L), x = v - y * d.L;
            udeg = (x + 1 < d.L) + (x > 0) + (y + 1 < d.L) + (y > 0);
          }
        }
        tally_row(ok[r] && !push ? cs[r] : -1, udeg, 0, false);
      }
    }
    __syncthreads();
    const int nq = s_nq;
    for (int qb = 0; qb < nq; qb += kScan * kBlock) {
      int64_t gs[kScan];
#pragma unroll
      for (int r = 0; r < kScan; ++r) {
        const int k = qb + r * kBlock + static_cast<int>(threadIdx.x);
        gs[r] = k < nq ? static_cast<int64_t>(lds_q[k]) : -1;
      }
      full_rows(gs);
    }
  } else {
    for (int chb = ch0; chb < ch1; chb += kScan) {
      int64_t gs[kScan];
#pragma unroll
      for (int r = 0; r < kScan; ++r)
        gs[r] = chb + r < ch1 ? (static_cast<int64_t>(chb + r) << SCO_CHUNK_SHIFT) + threadIdx.x : -1;
      full_rows(gs);
    }
  }
  if (c_uni >= 0) {
    wave_max_to(rmax, c_uni, t_umax);
    wave_max_to(rbmx, c_uni, t_bmax);
    wave_sum_to(rsum, c_uni, t_bsum);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < a.n_chains; c += kBlock) {
    if (rmax[c] > 0) atomicMax(&a.st[c].delta_union, rmax[c]);
    if (rbmx[c] > 0) atomicMax(&a.st[c].delta_sco, rbmx[c]);
    if (rsum[c] > 0) atomicAdd(&a.st[c].n_edges, static_cast<uint32_t>(rsum[c]));
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
// of T = q 2^P <= tile_limit (at most SCO_TILE_MAX) sites; those run tile by tile
// entirely in LDS.  The
// levels above P run over the whole site space with device-wide barriers between
// colour classes, their pending sites spread evenly over the blocks.
struct KwChain {
  int q, M, P, tile0;  // palette, levels, levels inside a tile, first global tile
  int L, N, periodic, pad;
  int64_t vbase;
  double inv_L, inv_q;
};

struct KwShared {
  KwChain kc[SCO_MAXCHAINS];
  int ntiles, qmax, mmax, pmin;
};

__device__ __forceinline__ void kw_setup(const StepArgs& a, KwShared& ks) {
  // every block computes the same per-chain parameters (Delta is final here)
  for (int c = threadIdx.x; c < a.n_chains; c += kBlock) {
    const ChainDesc& d = a.cd[c];
    // every site has a nearest neighbour, so q >= 2 (the tile divisions rely on it);
    // the checkerboard product colours the bonds alone (palette of at least 2) and
    // doubles the colours, which must still fit a byte
    const bool checker = a.coloring == SCO_COLOR_CHECKER;
    int q = max((checker ? a.st[c].delta_sco : a.st[c].delta_union) + 1, 2);
    const int qlim = checker ? (SCO_MAXQ + 1) / 2 : SCO_MAXQ;
    if (q > qlim) {
      set_flag(a.sync, SCO_FLAG_PALETTE);
      q = qlim;
    }
    const int groups = (d.N + q - 1) / q;
    int M = 0;
    while ((1 << M) < groups) ++M;
    int P = 0;
    while (P < M && (q << (P + 1)) <= a.tile_limit) ++P;
    KwChain& k = ks.kc[c];
    k.q = q;
    k.M = M;
    k.P = P;
    k.L = d.L;
    k.N = d.N;
    k.periodic = d.periodic;
    k.vbase = d.vbase;
    k.inv_L = d.inv_L;
    k.inv_q = 1.0 / q;
    if (blockIdx.x == 0) {
      a.st[c].q = q;
      a.st[c].M = a.coloring == SCO_COLOR_BCR ? 1 : M;  // one whole-graph reduction
      a.st[c].P = a.coloring == SCO_COLOR_BCR ? 0 : P;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0, qmax = 0, mmax = 0, pmin = SCO_MAXLEVEL;
    for (int c = 0; c < a.n_chains; ++c) {
      KwChain& k = ks.kc[c];
      k.tile0 = t;
      const int T = k.q << k.P;
      t += (k.N + T - 1) / T;
      qmax = max(qmax, k.q);
      mmax = max(mmax, k.M);
      pmin = min(pmin, k.P);
    }
    ks.ntiles = t;
    ks.qmax = qmax;
    ks.mmax = mmax;
    ks.pmin = pmin;
    if (blockIdx.x == 0) {
      // the sweep's colour classes
      a.sync->qmax = static_cast<uint32_t>(a.coloring == SCO_COLOR_CHECKER ? 2 * qmax : qmax);
      a.sync->mmax = static_cast<uint32_t>(mmax);
    }
  }
  __syncthreads();
}

// pending sites of a chain of N sites at a level with half-group size h: the upper
// halves [(2j+1) h, (2j+2) h) clipped to N
__device__ __forceinline__ int64_t pending_count(int N, int64_t h) {
  const int64_t full = N / (2 * h), rem = N - full * 2 * h;
  return full * h + (rem > h ? rem - h : 0);
}


static_assert(kListCap >= kScanLds, "the scan stages a padded tile in the phase LDS");

// Levels 1..P of every tile, in LDS.  Groups up to level P are aligned to the tile,
// so the same-group neighbours of a tile site are inside the tile; the tile's
// in-tile bonds are staged once, so a level touches global memory only at its end.
__device__ __forceinline__ void phase_kw_local(const StepArgs& a, const KwShared& ks, TileLds& tl) {
  uint16_t* const t_cr = tl.cr;
  uint16_t* const t_list = tl.list;
  uint32_t* const t_bmask = tl.bmask;
  uint16_t* const t_brank = tl.brank;
  uint16_t* const t_boff = tl.boff;
  uint16_t* const t_adj = tl.adj;
  __shared__ int32_t t_off[SCO_MAXQ + 1];  // class offsets of the level's list
  __shared__ int32_t t_cnt[SCO_MAXQ + 1];  // class c counted at c + 1; zero between levels
  __shared__ int32_t t_fill[SCO_MAXQ];     // zero between levels
  __shared__ int32_t t_wsum[kWaves];
  __shared__ int32_t t_rounds, t_nbonded;
  const uint32_t lane = lane_id();
  const int wave = threadIdx.x >> 6;
  const int tid = static_cast<int>(threadIdx.x);
  const bool checker = a.coloring == SCO_COLOR_CHECKER;
  // rank of a site with in-tile bonds among those of the tile
  auto bond_rank = [&](int i) {
    return static_cast<int>(t_brank[i >> 5]) + __popc(t_bmask[i >> 5] & ((1u << (i & 31)) - 1u));
  };
  for (int tile = blockIdx.x; tile < ks.ntiles; tile += gridDim.x) {
    int c = 0;
    while (c + 1 < a.n_chains && ks.kc[c + 1].tile0 <= tile) ++c;
    const KwChain& K = ks.kc[c];
    const int q = K.q, P = K.P, T = q << P, L = K.L, periodic = K.periodic;
    const int64_t vbase = K.vbase;
    const int v0 = (tile - K.tile0) * T;
    const int n = min(T, K.N - v0);
    const int32_t gt0 = static_cast<int32_t>(vbase + v0);  // first global site of the tile
    // tile indices and x0 + i are below 2^16, so the divisions by q, L and the
    // half-group sizes are exact multiply-highs
    const uint32_t mq = magic16(static_cast<uint32_t>(q)), mL = magic16(static_cast<uint32_t>(L));
    const int y0 = idiv_fp(v0, K.inv_L), x0 = v0 - y0 * L;
    const int nw = (n + 31) >> 5;
    if (P > 0) {
      // 1. row lengths (held in cr until the colours start) and the mask of sites with
      //    bonds, one ballot per 64 consecutive sites; kStage sites per thread and
      //    iteration, their row offsets read together.  A partner outside the tile is
      //    kept in the lists as a mark the visits skip.
      for (int ib = 0; ib < n; ib += kStage * kBlock) {
        int r0[kStage], r1[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
          const int i = ib + u * kBlock + tid;
          r0[u] = r1[u] = 0;
          if (i < n) {
            r0[u] = a.row_ptr[gt0 + i];
            r1[u] = a.row_ptr[gt0 + i + 1];
          }
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
          const int i = ib + u * kBlock + tid;
          row_checked(a, r0[u], r1[u]);
          const int k = min(r1[u] - r0[u], 65535);
          if (i < n) t_cr[i] = static_cast<uint16_t>(k);
          const uint64_t m = __ballot(k > 0);
          const int w0 = (ib + u * kBlock + wave * 64) >> 5;
          if (lane == 0 && w0 < nw) t_bmask[w0] = static_cast<uint32_t>(m);
          if (lane == 0 && w0 + 1 < nw) t_bmask[w0 + 1] = static_cast<uint32_t>(m >> 32);
        }
      }
      __syncthreads();
      // 2. ranks: exclusive prefix of the word popcounts (nw <= 1024 words)
      {
        const int cnt = tid < nw ? __popc(t_bmask[tid]) : 0;
        int incl = cnt;
        for (int o = 1; o < 64; o <<= 1) {
          const int x = __shfl_up(incl, o);
          if (lane >= static_cast<uint32_t>(o)) incl += x;
        }
        if (lane == 63) t_wsum[wave] = incl;
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wave; ++w) off += t_wsum[w];
        if (tid < nw) t_brank[tid] = static_cast<uint16_t>(off + incl - cnt);
        if (tid == kBlock - 1) t_nbonded = off + incl;
      }
      __syncthreads();
      // 3. list offsets of the first kBondedCap such sites (block scan, saturating)
      const int nb = min(t_nbonded, kBondedCap);
      for (int i = tid; i < n; i += kBlock)
        if ((t_bmask[i >> 5] >> (i & 31)) & 1u) {
          const int r = bond_rank(i);
          if (r < kBondedCap) {
            t_boff[r + 1] = t_cr[i];
            t_list[r] = static_cast<uint16_t>(i);  // the r-th bonded site (list unused until the levels)
          }
        }
      __syncthreads();
      {
        constexpr int kPer = (kBondedCap + kBlock - 1) / kBlock;
        const int b0 = 1 + tid * kPer;
        int s = 0;
        for (int k = 0; k < kPer; ++k)
          if (b0 + k <= nb) s += t_boff[b0 + k];
        int incl = s;
        for (int o = 1; o < 64; o <<= 1) {
          const int x = __shfl_up(incl, o);
          if (lane >= static_cast<uint32_t>(o)) incl += x;
        }
        if (lane == 63) t_wsum[wave] = incl;
        __syncthreads();
        int run = incl - s;
        for (int w = 0; w < wave; ++w) run += t_wsum[w];
        for (int k = 0; k < kPer; ++k)
          if (b0 + k <= nb) {
            run += t_boff[b0 + k];
            t_boff[b0 + k] = static_cast<uint16_t>(min(run, 65535));
          }
        if (tid == 0) t_boff[0] = 0;
      }
      __syncthreads();
      // 4. the partners, in row order, of the bonded sites by rank (kStage per thread
      //    and iteration, their rows read together); 0xFFFF marks one outside the tile
      for (int rb = 0; rb < nb; rb += kStage * kBlock) {
        int r0[kStage], r1[kStage], wp[kStage], we[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
          const int r = rb + u * kBlock + tid;
          r0[u] = r1[u] = wp[u] = 0;
          we[u] = -1;
          // rows past the LDS capacity are read from global memory when needed
          if (r < nb && t_boff[r + 1] <= kAdjCap) {
            const int i = t_list[r];
            wp[u] = t_boff[r];
            we[u] = t_boff[r + 1];
            r0[u] = a.row_ptr[gt0 + i];
            r1[u] = a.row_ptr[gt0 + i + 1];
          }
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
          if (we[u] < 0) continue;
          row_checked(a, r0[u], r1[u]);
          int w = wp[u];
          for (int e = r0[u]; e < r1[u] && w < we[u]; ++e) {
            const int j = a.col[e] - gt0;
            t_adj[w++] = (j >= 0 && j < n) ? static_cast<uint16_t>(j) : static_cast<uint16_t>(0xFFFF);
          }
        }
      }
      __syncthreads();
    }
    // level 0: colour i mod q (cr held the partner counts until here)
    for (int i = tid; i < n; i += kBlock) t_cr[i] = static_cast<uint16_t>(i - div16(i, mq) * q);
    for (int k = tid; k <= q; k += kBlock) t_cnt[k] = 0;
    for (int k = tid; k < q; k += kBlock) t_fill[k] = 0;
    if (tid == 0) t_rounds = 0;
    __syncthreads();
    if (tile == static_cast<int>(blockIdx.x)) mark(a.trace, 30);
    for (int p = 1; p <= P; ++p) {
      // pending sites: k -> (2 (k / H) + 1) H + k mod H, H = q 2^(p-1) the half-group
      const int H = q << (p - 1);
      const uint32_t mH = magic16(static_cast<uint32_t>(H));
      const int npend = static_cast<int>(pending_count(n, H));
      // t_cnt, t_fill and t_rounds are zero here (cleared before the barrier that ends
      // the level before)
      // classes 0 and 1 (most pending sites) are counted per wave by ballot, the others
      // with one LDS atomic per site
      for (int kb = 0; kb < npend; kb += kBlock) {
        const int k = kb + tid;
        int cc = -1;
        if (k < npend) {
          const int j = div16(k, mH);
          cc = t_cr[(2 * j + 1) * H + (k - j * H)] & 0xFF;
        }
        const uint64_t m0 = __ballot(cc == 0), m1 = __ballot(cc == 1);
        if (lane == 0) {
          if (m0) atomicAdd(&t_cnt[1], __popcll(m0));
          if (m1) atomicAdd(&t_cnt[2], __popcll(m1));
        }
        if (cc >= 2) atomicAdd(&t_cnt[cc + 1], 1);
      }
      __syncthreads();
      wave_class_offsets(t_cnt, t_off, q);  // in every wave: no barrier before bucketing
      if (tile == static_cast<int>(blockIdx.x)) mark(a.trace, 60 + p);
      for (int kb = 0; kb < npend; kb += kBlock) {
        const int k = kb + tid;
        int cc = -1, i = 0;
        if (k < npend) {
          const int j = div16(k, mH);
          i = (2 * j + 1) * H + (k - j * H);
          cc = t_cr[i] & 0xFF;
        }
        // classes 0 and 1: one LDS atomic per wave, the lanes ranked by ballot
        const uint64_t m0 = __ballot(cc == 0), m1 = __ballot(cc == 1);
        int b0 = 0, b1 = 0;
        if (lane == 0) {
          if (m0) b0 = atomicAdd(&t_fill[0], __popcll(m0));
          if (m1) b1 = atomicAdd(&t_fill[1], __popcll(m1));
        }
        b0 = __shfl(b0, 0);
        b1 = __shfl(b1, 0);
        if (cc >= 0) {
          const uint64_t below = (1ull << lane) - 1ull;
          const int slot = cc == 0   ? t_off[0] + b0 + __popcll(m0 & below)
                           : cc == 1 ? t_off[1] + b1 + __popcll(m1 & below)
                                     : t_off[cc] + atomicAdd(&t_fill[cc], 1);
          t_list[slot] = static_cast<uint16_t>(i);
          t_cr[i] = static_cast<uint16_t>(cc);  // undecided at this level
        }
      }
      __syncthreads();
      if (tile == static_cast<int>(blockIdx.x)) mark(a.trace, 80 + p);
      // The classes run from the top down, a block barrier after each: when a class
      // runs, every pending same-group neighbour of a higher class has decided (its
      // word carries a round) and those of lower classes have not, so no site waits.
      // Most pending sites sit in the two lowest classes (rule (2)' leaves most sites
      // of a lattice with colours 0 and 1), which are throughput-bound: the visit is
      // kept short and free of branches on the neighbours, and each thread takes two
      // sites of a class at a time, their LDS reads in flight together.
      auto run_classes = [&](auto set_tag) {
        using Set = decltype(set_tag);
        const int NL = L * L;
        const int gsz2 = 2 * H;
        int tmax = 0;
        // the decision of the site at list position kx
        auto decide = [&](int kx) {
          const int i = t_list[kx];
          const int glo = static_cast<int>(__umul24(div16(i, mq) >> p, gsz2));
          const int gmid = glo + H;
          const uint32_t gsz = static_cast<uint32_t>(min(glo + gsz2, n) - glo);
          const int t = x0 + i, dy = div16(t, mL);
          const int x = t - dy * L, y = y0 + dy;
          // tile indices of the lattice neighbours (+x, -x, +y, -y); -1 for none (open
          // lattice ends; the checkerboard product colours the bonds alone)
          int jn[4];
          jn[0] = x + 1 < L ? i + 1 : (periodic ? i + 1 - L : -1);
          jn[1] = x > 0 ? i - 1 : (periodic ? i - 1 + L : -1);
          jn[2] = y + 1 < L ? i + L : (periodic ? i + L - NL : -1);
          jn[3] = y > 0 ? i - L : (periodic ? i - L + NL : -1);
          Set taken;
          int rmax = 0;
          // a neighbour counts when in the group and not pending, or pending and
          // decided at this level (its colour then is the new one)
          auto visit = [&](int j, int w) {
            const bool same = static_cast<uint32_t>(j - glo) < gsz;
            const bool pend = j >= gmid;
            const int rj = w >> 8;
            const bool on = same && (!pend || rj != 0);
            rmax = max(rmax, on && pend ? rj : 0);
            taken.add_if(on, w & 0xFF);
          };
          int w[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (checker) jn[u] = -1;
            w[u] = t_cr[static_cast<uint32_t>(jn[u] - glo) < gsz ? jn[u] : i];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) visit(jn[u], w[u]);
          const uint32_t mw = t_bmask[i >> 5];
          if (P > 0 && ((mw >> (i & 31)) & 1u)) {  // the site has in-tile bonds
            const int r = static_cast<int>(t_brank[i >> 5]) + __popc(mw & ((1u << (i & 31)) - 1u));
            const int eb = r < kBondedCap ? t_boff[r + 1] : kAdjCap + 1;
            if (eb <= kAdjCap) {
              for (int e = t_boff[r]; e < eb; ++e) {
                const int j = t_adj[e];  // 0xFFFF: a partner outside the tile
                visit(j, t_cr[j < n ? j : i]);
              }
            } else {  // the row did not fit the LDS lists: read from global memory
              int g0 = a.row_ptr[gt0 + i], g1 = a.row_ptr[gt0 + i + 1];
              row_checked(a, g0, g1);
              for (int e = g0; e < g1; ++e) {
                const int j = a.col[e] - gt0;
                visit(j, t_cr[j >= 0 && j < n ? j : i]);
              }
            }
          }
          int nc = taken.first_free();
          if (nc >= q) {
            set_flag(a.sync, SCO_FLAG_PALETTE);
            nc = q - 1;
          }
          return static_cast<uint32_t>(nc | ((rmax + 1) << 8)) | (static_cast<uint32_t>(i) << 16);
        };
        for (int cl = q - 1; cl >= 0; --cl) {
          const int k0 = t_off[cl], k1 = t_off[cl + 1];
          for (int kx = k0 + tid; kx < k1; kx += 2 * kBlock) {
            const uint32_t d0 = decide(kx);
            const bool two = kx + kBlock < k1;
            const uint32_t d1 = two ? decide(kx + kBlock) : 0u;
            t_cr[d0 >> 16] = static_cast<uint16_t>(d0 & 0xFFFFu);
            tmax = max(tmax, static_cast<int>((d0 >> 8) & 0xFFu));
            if (two) {
              t_cr[d1 >> 16] = static_cast<uint16_t>(d1 & 0xFFFFu);
              tmax = max(tmax, static_cast<int>((d1 >> 8) & 0xFFu));
            }
          }
          __syncthreads();
        }
        tmax = wave_max(tmax);
        if (lane == 0 && tmax > 0) atomicMax(&t_rounds, tmax);
      };
      if (q <= 32) run_classes(ColorSet32{});
      else if (q <= 64) run_classes(ColorSet64{});
      else run_classes(ColorSet{});
      // the counts for the next level start from zero (the last class pass has read
      // its offsets)
      for (int k = tid; k <= q; k += kBlock) t_cnt[k] = 0;
      for (int k = tid; k < q; k += kBlock) t_fill[k] = 0;
      __syncthreads();
      if (threadIdx.x == 0) {
        const int rounds = t_rounds;
        t_rounds = 0;  // written next after the next level's bucketing barrier
        if (rounds > 0) atomicMax(&a.st[c].kw_rounds[p], rounds);
        // Eq. (5): a level takes at most q rounds (or the cap the host set)
        if (rounds > (a.round_cap > 0 ? a.round_cap : q)) set_flag(a.sync, SCO_FLAG_ROUNDS);
      }
      if (tile == static_cast<int>(blockIdx.x)) mark(a.trace, 40 + p);
    }
    const uint32_t tag = static_cast<uint32_t>(P) << 18;
    for (int i = threadIdx.x; i < n; i += kBlock) {
      const uint32_t col = t_cr[i] & 0xFFu;
      uint32_t out = col;
      if (checker) {  // 2 c + ((x + y) mod 2)
        const int t = x0 + i, dy = div16(t, mL);
        out = 2u * col + static_cast<uint32_t>((t - dy * L + y0 + dy) & 1);
      }
      a.color[gt0 + i] = static_cast<uint16_t>(out);
      a.kw_word[gt0 + i] = tag | col;
    }
    __syncthreads();
  }
}

// Levels P+1..M over the whole site space.  The pending sites of a level, numbered
// chain by chain, are split evenly over the blocks; a block buckets its share by
// colour into a list of block-local offsets (in LDS when it fits), then the colour
// classes run largest first with a device-wide barrier after each, so every read sees
// the decisions of the classes before it.  kw_word[g] holds (level << 18) |
// (round << 9) | colour of the last level that decided g, so "decided at this level"
// needs no clearing pass.  A colour read from memory is checked against the palette
// before it is used as an index.
__device__ __forceinline__ bool phase_kw_global(const StepArgs& a, const KwShared& ks, int32_t* lds_list) {
  __shared__ int32_t boff[SCO_MAXQ + 1];
  __shared__ int32_t bcnt[SCO_MAXQ + 1];  // class c counted at c + 1
  __shared__ int32_t bfill[SCO_MAXQ];
  __shared__ int32_t brounds[SCO_MAXCHAINS];
  __shared__ long long cpre[SCO_MAXCHAINS + 1];
  __shared__ long long wtot[kWaves];
  __shared__ int32_t s_pos;  // next list position to deal at the current level
  const uint32_t lane = lane_id();
  const int wave = threadIdx.x >> 6;
  const int tid = static_cast<int>(threadIdx.x);
  const int nch = a.n_chains, qmax = ks.qmax;

  for (int p = ks.pmin + 1; p <= ks.mmax; ++p) {
    // pending counts per chain, exclusive prefix over the chains
    {
      long long np = 0;
      const int c = tid;
      if (c < nch) {
        const KwChain& K = ks.kc[c];
        if (p > K.P && p <= K.M) np = pending_count(K.N, static_cast<int64_t>(K.q) << (p - 1));
      }
      long long incl = np;
      for (int o = 1; o < 64; o <<= 1) {
        const long long x = __shfl_up(incl, o);
        if (lane >= static_cast<uint32_t>(o)) incl += x;
      }
      if (lane == 63) wtot[wave] = incl;
      __syncthreads();
      long long off = 0;
      for (int w = 0; w < wave; ++w) off += wtot[w];
      if (c < nch) cpre[c] = off + incl - np;
      if (c == nch - 1) cpre[nch] = off + incl;
      for (int k = tid; k <= qmax; k += kBlock) bcnt[k] = 0;
      for (int k = tid; k < qmax; k += kBlock) bfill[k] = 0;
      for (int k = tid; k < nch; k += kBlock) brounds[k] = 0;
      if (tid == 0) s_pos = 0;
      __syncthreads();
    }
    const long long tot = cpre[nch];
    const long long k0 = tot * blockIdx.x / gridDim.x, k1 = tot * (blockIdx.x + 1) / gridDim.x;
    // the block's list: LDS when its share fits, else its own range of the records
    // the block's list: LDS when its share fits, else its own range of the records; the
    // two cases are separate inlined copies, so LDS accesses stay LDS instructions
    const bool in_lds = k1 - k0 <= kListCap;
    int32_t* const lst_mem = reinterpret_cast<int32_t*>(a.rec) + k0;
    // pending index -> chain and chain-local site
    auto site_of = [&](long long k, int& c, int& v) {
      int lo = 0, hi = nch - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cpre[mid] <= k) lo = mid;
        else hi = mid - 1;
      }
      c = lo;
      const uint32_t kk = static_cast<uint32_t>(k - cpre[c]);
      const uint32_t h = static_cast<uint32_t>(ks.kc[c].q) << (p - 1);
      // kk / h = (kk / 2^(p-1)) / q, exact through the double reciprocal of q
      const uint32_t j = static_cast<uint32_t>(idiv_fp(static_cast<int>(kk >> (p - 1)), ks.kc[c].inv_q));
      v = static_cast<int>((2u * j + 1u) * h + (kk - j * h));
    };
    auto site_chain = [&](long long k) {
      int c, v;
      site_of(k, c, v);
      return c;
    };
    auto bucket = [&](int32_t* lst) __attribute__((always_inline)) {
      for (int pass = 0; pass < 2; ++pass) {
        // kScan sites per thread and iteration, their loads issued together
        for (long long kb = k0; kb < k1; kb += kScan * kBlock) {
          int cs[kScan], col[kScan];
          bool ok[kScan];
#pragma unroll
          for (int r = 0; r < kScan; ++r) {
            const long long k = kb + r * kBlock + tid;
            ok[r] = k < k1;
            cs[r] = 0;
            col[r] = 0;
            if (ok[r]) {
              int v;
              site_of(k, cs[r], v);
              col[r] = static_cast<int>(a.kw_word[ks.kc[cs[r]].vbase + v] & 0x1FFu);
            }
          }
#pragma unroll
          for (int r = 0; r < kScan; ++r) {
            if (!ok[r]) continue;
            const int cc = col[r];
            if (cc >= ks.kc[cs[r]].q) {  // cannot happen after a complete colouring
              set_flag(a.sync, SCO_FLAG_PALETTE);
              continue;
            }
            if (pass == 0) atomicAdd(&bcnt[cc + 1], 1);
            else lst[boff[cc] + atomicAdd(&bfill[cc], 1)] = static_cast<int32_t>(kb + r * kBlock + tid - k0);
          }
        }
        __syncthreads();
        if (pass == 0) wave_class_offsets(bcnt, boff, qmax);  // in every wave
      }
    };
    // a share of at most kHeldKW sites per thread: every colour loaded at once and kept
    // in registers between the count and the scatter
    auto bucket_held = [&](int32_t* lst) __attribute__((always_inline)) {
      // the word of each site, or ~0 for none; the palette check goes by the chain's q
      uint32_t wd[kHeldKW];
#pragma unroll
      for (int r = 0; r < kHeldKW; ++r) {
        const long long k = k0 + r * kBlock + tid;
        wd[r] = ~0u;
        if (k < k1) {
          int c, v;
          site_of(k, c, v);
          wd[r] = ld_global(&a.kw_word[ks.kc[c].vbase + v]) & 0x1FFu;
        }
      }
#pragma unroll
      for (int r = 0; r < kHeldKW; ++r) {
        if (wd[r] == ~0u) continue;
        const int cc = static_cast<int>(wd[r]);
        if (cc >= qmax || (nch > 1 && cc >= ks.kc[site_chain(k0 + r * kBlock + tid)].q)) {
          set_flag(a.sync, SCO_FLAG_PALETTE);  // cannot happen after a complete colouring
          wd[r] = ~0u;
          continue;
        }
        atomicAdd(&bcnt[cc + 1], 1);
      }
      __syncthreads();
      wave_class_offsets(bcnt, boff, qmax);  // in every wave: no barrier before the scatter
#pragma unroll
      for (int r = 0; r < kHeldKW; ++r)
        if (wd[r] != ~0u) lst[boff[wd[r]] + atomicAdd(&bfill[wd[r]], 1)] = r * kBlock + tid;
      __syncthreads();
    };
    if (k1 - k0 <= static_cast<long long>(kHeldKW) * kBlock) {
      if (in_lds) bucket_held(lds_list);
      else bucket_held(lst_mem);
    } else if (in_lds) {
      bucket(lds_list);
    } else {
      bucket(lst_mem);
    }
    mark(a.trace, 200 + p);
    // The classes run without a barrier between them.  A pending site of class cc
    // reads the colours its same-group pending neighbours of higher classes take at
    // this level and ignores the lower ones (those wait for it), so it decides as soon
    // as every such word carries this level, and the decision does not depend on when
    // the words arrived.  List positions (top class first) are dealt to the lanes from
    // a block-wide counter, so each lane's positions increase; a lane holds one site
    // at a time, re-reads its words while it waits, and takes the next position once
    // it has decided, so a waiting lane holds up neither its wave nor its block.
    // Every wait is on a higher class: the highest undecided class is always ready
    // wherever it is held, and an untaken site of it can only be behind held sites of
    // that same class, so by induction every wait ends (all blocks are resident).
    const int nl = boff[qmax];
    auto run_level = [&](auto set_tag, int32_t* lst) __attribute__((always_inline)) {
      using Set = decltype(set_tag);
      const uint32_t lane = lane_id();
      int cls = qmax - 1;  // class of the lane's current position (only decreases)
      bool have = false, more = true;
      int kx = 0, cl = 0, c = 0, rb = 0, re = 0, pb = -1;
      int32_t g = 0;
      int nbs[4] = {-1, -1, -1, -1};
      uint32_t wn[4] = {0u, 0u, 0u, 0u}, wb = 0u;
      int cloc = -1, rloc = 0;
      for (uint32_t spin = 0;; ++spin) {
        // lanes without a site take the next positions: one LDS atomic per wave
        const bool need = !have && more;
        const uint64_t nm = __ballot(need);
        bool fresh = false;
        if (nm != 0) {
          const int leader = __ffsll(static_cast<unsigned long long>(nm)) - 1;
          int base = 0;
          if (static_cast<int>(lane) == leader) base = atomicAdd(&s_pos, __popcll(nm));
          base = __shfl(base, leader);
          if (need) {
            const int j = base + __popcll(nm & ((1ull << lane) - 1ull));
            if (j >= nl) {
              more = false;
            } else {
              kx = nl - 1 - j;
              while (kx < boff[cls]) --cls;
              cl = cls;
              int v;
              site_of(k0 + lst[kx], c, v);
              const KwChain& K = ks.kc[c];
              const int32_t vb = static_cast<int32_t>(K.vbase);
              g = vb + v;
              const int y = idiv_fp(v, K.inv_L), x = v - y * K.L;
              nn_sites(x, y, K.L, K.periodic, nbs);
              if (a.coloring == SCO_COLOR_CHECKER) nbs[0] = nbs[1] = nbs[2] = nbs[3] = -1;
              // a first read may return an older value of a word (a copy this XCD's L2
              // still holds): an older value shows a higher-class neighbour as
              // undecided, so the site only waits and re-reads with read-modify-writes;
              // a word decided at this level does not change again within it
#pragma unroll
              for (int t = 0; t < 4; ++t) wn[t] = nbs[t] >= 0 ? ld_relaxed(&a.kw_word[vb + nbs[t]]) : 0u;
              rb = a.row_ptr[g];
              re = a.row_ptr[g + 1];
              row_checked(a, rb, re);
              pb = re > rb ? a.col[rb] - vb : -1;
              wb = pb >= 0 ? ld_relaxed(&a.kw_word[vb + pb]) : 0u;
              have = true;
              fresh = true;
            }
          }
        }
        if (__ballot(have || more) == 0) break;
        if (have && !fresh) {
          // still waiting: re-read the words where every XCD sees one value
          const int32_t vb = static_cast<int32_t>(ks.kc[c].vbase);
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (nbs[t] >= 0) wn[t] = ld_poll(&a.kw_word[vb + nbs[t]]);
          if (pb >= 0) wb = ld_poll(&a.kw_word[vb + pb]);
        }
        bool waiting = false;
        if (have) {
          const KwChain& K = ks.kc[c];
          const int q = K.q;
          const int32_t vb = static_cast<int32_t>(K.vbase);
          const int grp = idiv_fp(g - vb, K.inv_q) >> p;
          Set taken;
          int rmax = 0;
          bool ready = true;
          // neighbour u (chain-local) with word w: same group only; a pending one
          // counts once decided at this level, and one of a higher class must be
          auto visit = [&](int u, uint32_t w) {
            const int gu = idiv_fp(u, K.inv_q);
            if ((gu >> p) != grp) return;  // another group at this level
            if ((gu >> (p - 1)) & 1) {     // pending at this level
              if (static_cast<int>((w >> 18) & 0x1Fu) != p) {
                const int cu = static_cast<int>(w & 0x1FFu);
                if (cu > cl && cu < q) ready = false;  // not yet decided
                return;  // a lower class: decides after this site
              }
              rmax = max(rmax, static_cast<int>((w >> 9) & 0x1FFu));
            }
            taken.add(static_cast<int>(w & 0x1FFu));
          };
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (nbs[t] >= 0) visit(nbs[t], wn[t]);
          if (pb >= 0) visit(pb, wb);
          for (int e = rb + 1; e < re; ++e) {
            const int u = a.col[e] - vb;
            visit(u, fresh ? ld_relaxed(&a.kw_word[vb + u]) : ld_poll(&a.kw_word[vb + u]));
          }
          if (ready) {
            int nc = taken.first_free();
            if (nc >= q) {
              set_flag(a.sync, SCO_FLAG_PALETTE);
              nc = q - 1;
            }
            // published where the waiting neighbours' read-modify-write polls read
            st_publish(&a.kw_word[g], (static_cast<uint32_t>(p) << 18) | (static_cast<uint32_t>(rmax + 1) << 9) |
                                          static_cast<uint32_t>(nc));
            if (c != cloc) {
              if (cloc >= 0) atomicMax(&brounds[cloc], rloc);
              cloc = c;
              rloc = 0;
            }
            rloc = max(rloc, rmax + 1);
            have = false;
          } else {
            waiting = true;
          }
        }
        // pause only when no lane of the wave took new work
        if (__ballot(waiting) != 0 && nm == 0) {
          if (spin > kSpinLimit) set_flag(a.sync, SCO_FLAG_TIMEOUT);
          if ((spin & 255u) == 255u && timed_out(a.sync)) break;
          __builtin_amdgcn_s_sleep(1);
        }
      }
      wave_max_to(brounds, cloc, rloc);
    };
    if (!in_lds) run_level(ColorSet{}, lst_mem);
    else if (qmax <= 64) run_level(ColorSet64{}, lds_list);
    else run_level(ColorSet{}, lds_list);
    // the level ends with a full barrier that also publishes the colours
    if (!grid_barrier(a.sync)) return false;
    for (int c = tid; c < nch; c += kBlock) {
      if (brounds[c] > 0) atomicMax(&a.st[c].kw_rounds[p], brounds[c]);
      // Eq. (5): a level takes at most q rounds (or the cap the host set)
      if (brounds[c] > (a.round_cap > 0 ? a.round_cap : ks.kc[c].q)) set_flag(a.sync, SCO_FLAG_ROUNDS);
    }
    mark(a.trace, 100 + p);
  }
  return true;
}

// The levels over the whole site space record their decisions only in kw_word; the
// colours of a block's sweep range are copied out of the words in one coalesced pass
// (after the full barrier that ends the last level), by the block that sweeps them.
__device__ __forceinline__ void phase_colour_fill(const StepArgs& a) {
  const int64_t S = ((a.G + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
  const int64_t r0 = min(static_cast<int64_t>(blockIdx.x) * S, a.G);
  const int64_t r1 = min(r0 + S, a.G);
  if (a.coloring == SCO_COLOR_CHECKER) {  // 2 c + ((x + y) mod 2)
    for (int64_t g = r0 + threadIdx.x; g < r1; g += kBlock) {
      const ChainDesc& d = a.cd[a.chunk_chain[g >> SCO_CHUNK_SHIFT]];
      const int v = static_cast<int>(g - d.vbase);
      const int y = idiv_fp(v, d.inv_L), x = v - y * d.L;
      a.color[g] = static_cast<uint16_t>(2u * (a.kw_word[g] & 0x1FFu) + static_cast<uint32_t>((x + y) & 1));
    }
  } else {
    for (int64_t g = r0 + threadIdx.x; g < r1; g += kBlock) a.color[g] = static_cast<uint16_t>(a.kw_word[g] & 0x1FFu);
  }
  __syncthreads();
}

// Basic colour reduction with rule (2)' on the whole union graph (no KW groups,
// Sec. 2.3.2): the initial colour of a site is its index v, the sites v >= q of every
// chain are pending, and a pending site recolours once every pending neighbour of larger
// colour (index) has, taking the smallest colour in 0..q-1 that no neighbour holds.
// The synchronous rounds are run level by level of that dependence: dep[v] counts the
// pending neighbours above v; the sites at zero form round 1, and every decision
// decrements the counts of its pending neighbours below it, queueing those that reach
// zero for the next round.  A site decides in round 1 + max over its pending
// neighbours above it, the round of the Jacobi iteration, and sees exactly their new
// colours, so the colours are those of the rounds.  dep lives in `fill`, the two
// rotating frontier lists in `rec`, their sizes in sync->fcount.  Returns false when
// the launch must end.
__device__ __forceinline__ bool phase_color_bcr(const StepArgs& a, const KwShared& ks, int32_t* lds) {
  const int tid = static_cast<int>(threadIdx.x);
  const uint32_t lane = lane_id();
  int32_t* const dep = a.fill;
  int32_t* const lists = reinterpret_cast<int32_t*>(a.rec);  // [0, G) and [G, 2 G)
  int32_t* const rnd = lds;  // per chain: the last round in which one of its sites decided
  for (int c = tid; c < a.n_chains; c += kBlock) rnd[c] = 0;
  // the union neighbours of global site g (chain c, local v): the lattice neighbours,
  // then the bond partners that are not among them; f(u) for each
  auto for_union = [&](int c, int v, int64_t g, auto&& f) __attribute__((always_inline)) {
    const KwChain& K = ks.kc[c];
    const int y = idiv_fp(v, K.inv_L), x = v - y * K.L;
    int nb[4];
    nn_sites(x, y, K.L, K.periodic, nb);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (nb[t] >= 0) f(nb[t]);
    int r0 = a.row_ptr[g], r1 = a.row_ptr[g + 1];
    row_checked(a, r0, r1);
    for (int e = r0; e < r1; ++e) {
      const int u = a.col[e] - static_cast<int32_t>(K.vbase);
      if (u != nb[0] && u != nb[1] && u != nb[2] && u != nb[3]) f(u);
    }
  };
  // appends site g to list `lst` (one atomic per wave); every lane of the wave calls it
  auto append = [&](bool on, int32_t g, int32_t* lst, uint32_t* cnt) {
    const uint64_t m = __ballot(on);
    if (m == 0) return;
    const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
    uint32_t base = 0;
    if (static_cast<int>(lane) == leader)
      base = __hip_atomic_fetch_add(cnt, static_cast<uint32_t>(__popcll(m)), __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    base = __shfl(base, leader);
    if (on) lst[base + __popcll(m & ((1ull << lane) - 1ull))] = g;
  };
  if (blockIdx.x == 0 && tid < 3) a.sync->fcount[tid] = 0u;
  if (!grid_barrier(a.sync)) return false;
  // initial colours and dependence counts; the sites without a pending neighbour above
  // them form the first frontier (list 1, size fcount[1])
  for (int64_t gb = static_cast<int64_t>(blockIdx.x) * kBlock; gb < a.G; gb += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t g = gb + tid;
    const int c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
    const KwChain& K = ks.kc[c];
    const int v = static_cast<int>(g - K.vbase);
    bool ready = false;
    if (v < K.N) {
      if (v < K.q) {
        a.color[g] = static_cast<uint16_t>(v);
      } else {
        a.color[g] = 0xFFFFu;
        int n_up = 0;
        for_union(c, v, g, [&](int u) { n_up += (u > v) ? 1 : 0; });
        dep[g] = n_up;
        ready = n_up == 0;
      }
    }
    append(ready, static_cast<int32_t>(g), lists + a.G, &a.sync->fcount[1]);
  }
  for (int r = 1;; ++r) {
    if (!grid_barrier(a.sync)) return false;
    const uint32_t nf = ld_poll(&a.sync->fcount[r % 3]);
    if (nf == 0) break;
    if (blockIdx.x == 0 && tid == 0) a.sync->fcount[(r + 2) % 3] = 0u;  // round r-1's, read by nobody now
    const int32_t* cur = lists + ((r & 1) ? a.G : 0);
    int32_t* nxt = lists + ((r & 1) ? 0 : a.G);
    uint32_t* ncnt = &a.sync->fcount[(r + 1) % 3];
    const uint32_t k0 = static_cast<uint32_t>(static_cast<uint64_t>(nf) * blockIdx.x / gridDim.x);
    const uint32_t k1 = static_cast<uint32_t>(static_cast<uint64_t>(nf) * (blockIdx.x + 1) / gridDim.x);
    for (uint32_t kb = k0; kb < k1; kb += kBlock) {
      const uint32_t k = kb + static_cast<uint32_t>(tid);
      const bool have = k < k1;
      int c = 0, v = 0;
      int64_t g = 0;
      if (have) {
        g = cur[k];
        c = a.chunk_chain[g >> SCO_CHUNK_SHIFT];
        v = static_cast<int>(g - ks.kc[c].vbase);
        const int q = ks.kc[c].q;
        ColorSet taken;
        for_union(c, v, g, [&](int u) {
          const int cu = a.color[ks.kc[c].vbase + u];
          if (cu < q) taken.add(cu);
        });
        int nc = taken.first_free();
        if (nc >= q) {
          set_flag(a.sync, SCO_FLAG_PALETTE);
          nc = q - 1;
        }
        a.color[g] = static_cast<uint16_t>(nc);
        atomicMax(&rnd[c], r);
      }
      // release the pending neighbours below: those whose count reaches zero join the
      // next round (at most 4 + the row's bonds per site; one wave-wide append each)
      int deg = 0;
      if (have) for_union(c, v, g, [&](int) { ++deg; });
      const int dmax = wave_max(deg);
      for (int e = 0; e < dmax; ++e) {
        int u = -1;
        if (have && e < deg) {
          int i = 0;
          for_union(c, v, g, [&](int w) {
            if (i++ == e) u = w;
          });
        }
        bool ready = false;
        int64_t gu = 0;
        if (u >= 0 && u < v && u >= ks.kc[c].q) {
          gu = ks.kc[c].vbase + u;
          ready = atomicSub(&dep[gu], 1) == 1;
        }
        append(ready, static_cast<int32_t>(gu), nxt, ncnt);
      }
    }
  }
  __syncthreads();
  for (int c = tid; c < a.n_chains; c += kBlock)
    if (rnd[c] > 0) atomicMax(&a.st[c].kw_rounds[1], rnd[c]);
  return true;
}

// =================================================================== step (3)
// Block b buckets its own sites [b S, (b+1) S) by colour into a list of block-local
// offsets (in LDS when it fits), then the colour classes are swept in ascending order
// with device-wide barriers between them.  Flipping s_v changes H' by s_v h_v,
// h_v = 2J sum_NN s_u - sum_bonds delta_m s_u (NN first, then the bonds in row
// order); with kappa == 1 a bond is hard and forbids the flip, and the exchange-only
// acceptance is the table pacc.
constexpr int kLocalChains = 4;  // chain descriptors of a block's range held in LDS

__device__ __forceinline__ bool phase_sweep(const StepArgs& a, uint32_t step, int32_t* lds_list) {
  __shared__ int32_t boff[SCO_MAXQ + 1];
  __shared__ int32_t bcnt[SCO_MAXQ + 1];  // class c counted at c + 1
  __shared__ int32_t bfill[SCO_MAXQ];
  // accepted flips of the block per chain: up -> down in the low 32 bits, down -> up in
  // the high 32 bits (the magnetisation moves by 2 (high - low))
  __shared__ unsigned long long bacc[SCO_MAXCHAINS];
  __shared__ ChainDesc lcd[kLocalChains];
  const int qmax = static_cast<int>(a.sync->qmax);
  const int64_t S = ((a.G + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
  const int64_t r0 = min(static_cast<int64_t>(blockIdx.x) * S, a.G);
  const int64_t r1 = min(r0 + S, a.G);
  const int tid = static_cast<int>(threadIdx.x);
  int32_t* const lst_mem = reinterpret_cast<int32_t*>(a.rec) + r0;
  // the chains of the block's range are a contiguous run [c_lo, c_hi]
  const int c_lo = r0 < r1 ? a.chunk_chain[r0 >> SCO_CHUNK_SHIFT] : 0;
  const int c_hi = r0 < r1 ? a.chunk_chain[(r1 - 1) >> SCO_CHUNK_SHIFT] : 0;
  const bool local_cd = c_hi - c_lo < kLocalChains;
  Tally tally(c_lo);
  // FP32 decisions that need FP64 are queued (list positions) and taken after the
  // class's main pass, where they run in dense waves: deciding them in line would make
  // nearly every wave run both paths.  The queue lives in the block's share of the
  // survivor-rank array, which the sweeps do not use.
  __shared__ uint32_t s_rq;
  const uint32_t rq_cap = a.cap_und / gridDim.x;
  int32_t* const rq = a.er + static_cast<int64_t>(blockIdx.x) * rq_cap;
  if (tid == 0) s_rq = 0u;
  // the block's flip counts into the chain states (accepted flips, magnetisation)
  auto flush_flips = [&]() {
    __syncthreads();
    for (int c = tid; c < a.n_chains; c += kBlock) {
      const unsigned long long f = bacc[c];
      if (f) {
        const unsigned long long lo = f & 0xFFFFFFFFull, hi = f >> 32;
        atomicAdd(&a.st[c].accepted, lo + hi);
        atomicAdd(reinterpret_cast<unsigned long long*>(&a.st[c].mag), 2ull * (hi - lo));  // two's complement
        bacc[c] = 0;
      }
    }
    __syncthreads();
  };
  const bool flush_each_sweep = static_cast<int64_t>(a.nsw_max) * (r1 - r0) >= (1ll << 31);
  if (local_cd)
    for (int i = tid; i <= c_hi - c_lo; i += kBlock) lcd[i] = a.cd[c_lo + i];
  for (int k = tid; k <= qmax; k += kBlock) bcnt[k] = 0;
  for (int k = tid; k < qmax; k += kBlock) bfill[k] = 0;
  for (int c = tid; c < a.n_chains; c += kBlock) bacc[c] = 0;
  __syncthreads();
  // The list in LDS and the chain descriptors in LDS (the usual case), or both in
  // global memory: two inlined copies, so LDS accesses stay LDS instructions.
  // staged: the block's range is one chain, and its spins with one lattice row on
  // either side are held in LDS after the list (bit 0: spin up; bit 1: the site has
  // bonds).  A class reads its lattice neighbours there; only the two halo rows,
  // which other blocks update, are read again from global memory before each class.
  auto body = [&](int32_t* lst, const auto& desc, auto staged_tag) __attribute__((always_inline)) -> bool {
    constexpr bool staged = decltype(staged_tag)::value;
    // colour buckets of the block's sites: count, offsets, list.  A range of at most
    // kHeldSw sites per thread loads every colour at once and keeps them in registers;
    // a longer one takes two passes of kScan sites per thread and iteration.
    if (r1 - r0 <= static_cast<int64_t>(kHeldSw) * kBlock) {
      int col[kHeldSw];
#pragma unroll
      for (int r = 0; r < kHeldSw; ++r) {
        const int64_t g = r0 + r * kBlock + tid;
        col[r] = -1;  // no site
        if (g < r1) {
          const int c = c_lo == c_hi ? c_lo : a.chunk_chain[g >> SCO_CHUNK_SHIFT];
          const ChainDesc& d = desc(c);
          if (static_cast<int>(g - d.vbase) < d.N) col[r] = a.color[g];
        }
      }
#pragma unroll
      for (int r = 0; r < kHeldSw; ++r) {
        if (col[r] < 0) continue;
        if (col[r] >= qmax) {  // cannot happen after a complete colouring
          set_flag(a.sync, SCO_FLAG_PALETTE);
          col[r] = -1;
          continue;
        }
        atomicAdd(&bcnt[col[r] + 1], 1);
      }
      __syncthreads();
      wave_class_offsets(bcnt, boff, qmax);  // in every wave: no barrier before the scatter
#pragma unroll
      for (int r = 0; r < kHeldSw; ++r)
        if (col[r] >= 0) lst[boff[col[r]] + atomicAdd(&bfill[col[r]], 1)] = r * kBlock + tid;
      __syncthreads();
    } else
    for (int pass = 0; pass < 2; ++pass) {
      for (int64_t gb = r0; gb < r1; gb += kScan * kBlock) {
        int col[kScan];
        bool ok[kScan];
#pragma unroll
        for (int r = 0; r < kScan; ++r) {
          const int64_t g = gb + r * kBlock + tid;
          ok[r] = false;
          col[r] = 0;
          if (g < r1) {
            const int c = c_lo == c_hi ? c_lo : a.chunk_chain[g >> SCO_CHUNK_SHIFT];
            const ChainDesc& d = desc(c);
            ok[r] = static_cast<int>(g - d.vbase) < d.N;
            if (ok[r]) col[r] = a.color[g];
          }
        }
#pragma unroll
        for (int r = 0; r < kScan; ++r) {
          if (!ok[r]) continue;
          const int cc = col[r];
          if (cc >= qmax) {  // cannot happen after a complete colouring
            if (pass == 0) set_flag(a.sync, SCO_FLAG_PALETTE);
            continue;
          }
          if (pass == 0) atomicAdd(&bcnt[cc + 1], 1);
          else lst[boff[cc] + atomicAdd(&bfill[cc], 1)] = static_cast<int32_t>(gb + r * kBlock + tid - r0);
        }
      }
      __syncthreads();
      if (pass == 0) wave_class_offsets(bcnt, boff, qmax);  // in every wave
    }
    mark(a.trace, 22);

    // tile slot t holds chain-local site tl_base + t (wrapped on a periodic lattice);
    // the own range is slots [L, L + n_own)
    int8_t* const tile = reinterpret_cast<int8_t*>(lst + (r1 - r0));
    const int n_own = static_cast<int>(r1 - r0);
    const int tl_L = staged ? desc(c_lo).L : 0;
    const int tl_N = staged ? desc(c_lo).N : 0;
    const int64_t tl_vb = staged ? desc(c_lo).vbase : 0;
    const int tl_base = static_cast<int>(r0 - tl_vb) - tl_L;
    const bool tl_per = staged && desc(c_lo).periodic != 0;
    // the two halo rows, one coherent byte read per site
    auto load_halo = [&]() __attribute__((always_inline)) {
      int hv[kHaloSw];
#pragma unroll
      for (int r = 0; r < kHaloSw; ++r) {
        const int t = r * kBlock + tid;
        hv[r] = -1;
        if (t < 2 * tl_L) {
          int u = tl_base + (t < tl_L ? t : t + n_own);
          if (tl_per) u = u < 0 ? u + tl_N : (u >= tl_N ? u - tl_N : u);
          if (u >= 0 && u < tl_N) hv[r] = ld_relaxed(&a.spin[tl_vb + u]);
        }
      }
#pragma unroll
      for (int r = 0; r < kHaloSw; ++r) {
        const int t = r * kBlock + tid;
        if (t < 2 * tl_L) tile[t < tl_L ? t : t + n_own] = static_cast<int8_t>(hv[r] > 0 ? 1 : 0);
      }
    };
    if constexpr (staged) {
      // own range, four sites per word read (the range and the chain start on chunk
      // bounds); a site has bonds when its row is not empty
      uint32_t sw[kStageSw];
      int4 dg[kStageSw];
      int32_t rn[kStageSw];
#pragma unroll
      for (int r = 0; r < kStageSw; ++r) {
        const int w = r * kBlock + tid;
        sw[r] = 0u;
        dg[r] = make_int4(0, 0, 0, 0);
        rn[r] = 0;
        if (4 * w < n_own) {
          sw[r] = ld_relaxed(reinterpret_cast<const uint32_t*>(a.spin + r0) + w);
          dg[r] = reinterpret_cast<const int4*>(a.row_ptr + r0)[w];
          rn[r] = a.row_ptr[r0 + 4 * w + 4];
        }
      }
      load_halo();
#pragma unroll
      for (int r = 0; r < kStageSw; ++r) {
        const int w = r * kBlock + tid;
        if (4 * w < n_own) {
          const int dd[4] = {dg[r].y - dg[r].x, dg[r].z - dg[r].y, dg[r].w - dg[r].z, rn[r] - dg[r].w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int8_t sp = static_cast<int8_t>((sw[r] >> (8 * i)) & 0xFFu);
            tile[tl_L + 4 * w + i] = static_cast<int8_t>((sp > 0 ? 1 : 0) | (dd[i] != 0 ? 2 : 0));
          }
        }
      }
      __syncthreads();
    }

    // the FP64 decision of one soft-bond site (local field NN first, then the bonds in
    // row order), also the recheck of the FP32 form
    auto fp64_decision = [&](const ChainDesc& d, int c, int v, int ns, int svv, int b0, int b1,
                             uint32_t sweep) -> bool {
      double h = d.twoJ * static_cast<double>(ns);
      for (int t = b0; t < b1; ++t) {
        const double dm = ld_global(&d.delta[a.attr[t]]);
        h = ld_relaxed(&a.spin[a.col[t]]) > 0 ? h - dm : h + dm;
      }
      const double dE = svv > 0 ? h : -h;
      if (dE <= 0.0) return true;
      const W4 w = philox10_wide(step, static_cast<uint32_t>(v), sweep, SCO_TAG_MC, d.seed, d.chain_id);
      const double u = unit52(w.x, w.y);
      const double pr = exp(d.neg_beta * dE);
      if (fabs(u - pr) < 1e-12) tally.tie(a, c);
      return u < pr;
    };
    // the decision inputs of one site: the lattice neighbours' spin sum, its spin, its row
    auto site_inputs = [&](int64_t g, const ChainDesc& d, int& ns, int& svv, int& b0, int& b1) {
      const int v = static_cast<int>(g - d.vbase);
      const int y = idiv_fp(v, d.inv_L), x = v - y * d.L;
      int nb[4];
      nn_sites(x, y, d.L, d.periodic, nb);
      ns = 0;
      if constexpr (staged) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (nb[t] >= 0) {
            int dv = nb[t] - v;
            dv = dv > tl_N / 2 ? dv - tl_N : (dv < -(tl_N / 2) ? dv + tl_N : dv);
            ns += (tile[v + dv - tl_base] & 1) ? 1 : -1;
          }
        svv = (tile[v - tl_base] & 1) ? 1 : -1;
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (nb[t] >= 0) ns += ld_relaxed(&a.spin[d.vbase + nb[t]]);
        svv = ld_relaxed(&a.spin[g]);
      }
      b0 = a.row_ptr[g];
      b1 = a.row_ptr[g + 1];
      row_checked(a, b0, b1);
    };
    for (int s = 0; s < a.nsw_max; ++s) {
      for (int cc = 0; cc < qmax; ++cc) {
        const int k0 = boff[cc], k1 = boff[cc + 1];
        if constexpr (staged) {
          // the halo rows as the previous class left them (the first class of the
          // first sweep has them from the staging)
          if (s > 0 || cc > 0) {
            load_halo();
            __syncthreads();
          }
        }
        // every thread of the block runs the same number of iterations; each takes
        // kBatch sites of the class and loads their neighbour spins before deciding
        // (sites of one class are not coupled)
        for (int kb = k0; kb < k1; kb += kBatch * kBlock) {
          int64_t gs[kBatch];
          int cs[kBatch], nsum[kBatch], sv[kBatch], q0[kBatch], q1[kBatch];
          bool live[kBatch];
#pragma unroll
          for (int r = 0; r < kBatch; ++r) {
            const int k = kb + r * kBlock + tid;
            live[r] = false;
            gs[r] = 0;
            cs[r] = 0;
            nsum[r] = sv[r] = q0[r] = q1[r] = 0;
            if (k < k1) {
              gs[r] = r0 + lst[k];
              cs[r] = c_lo == c_hi ? c_lo : a.chunk_chain[gs[r] >> SCO_CHUNK_SHIFT];
              const ChainDesc& d = desc(cs[r]);
              const int nsw = a.nsw_override >= 0 ? a.nsw_override : d.n_sw;
              live[r] = s < nsw;
              if (live[r]) {
                const int v = static_cast<int>(gs[r] - d.vbase);
                const int y = idiv_fp(v, d.inv_L), x = v - y * d.L;
                int nb[4];
                nn_sites(x, y, d.L, d.periodic, nb);
                if constexpr (staged) {
                  // a neighbour's slot: its offset from v taken the short way round
#pragma unroll
                  for (int t = 0; t < 4; ++t)
                    if (nb[t] >= 0) {
                      int dv = nb[t] - v;
                      dv = dv > tl_N / 2 ? dv - tl_N : (dv < -(tl_N / 2) ? dv + tl_N : dv);
                      nsum[r] += (tile[v + dv - tl_base] & 1) ? 1 : -1;
                    }
                  const int b = tile[v - tl_base];
                  sv[r] = (b & 1) ? 1 : -1;
                  if (b & 2) {
                    if (d.hard) {
                      q1[r] = 1;  // any bond is hard: the flip is refused without its row
                    } else {
                      q0[r] = a.row_ptr[gs[r]];
                      q1[r] = a.row_ptr[gs[r] + 1];
                      row_checked(a, q0[r], q1[r]);
                    }
                  }
                } else {
#pragma unroll
                  for (int t = 0; t < 4; ++t)
                    if (nb[t] >= 0) nsum[r] += ld_relaxed(&a.spin[d.vbase + nb[t]]);
                  sv[r] = ld_relaxed(&a.spin[gs[r]]);
                  q0[r] = a.row_ptr[gs[r]];
                  q1[r] = a.row_ptr[gs[r] + 1];
                  row_checked(a, q0[r], q1[r]);
                }
              }
            }
          }
          bool acc[kBatch];
#pragma unroll
          for (int r = 0; r < kBatch; ++r) {
            acc[r] = false;
            if (!live[r]) continue;
            const int64_t g = gs[r];
            const int c = cs[r];
            const ChainDesc& d = desc(c);
            const int v = static_cast<int>(g - d.vbase);
            if (d.hard) {
              if (q1[r] == q0[r]) {
                const double pa = d.pacc[sv[r] * nsum[r] + 4];
                if (pa >= 1.0) {
                  acc[r] = true;
                } else {
                  const W4 w = philox10_wide(step, static_cast<uint32_t>(v), static_cast<uint32_t>(s), SCO_TAG_MC,
                                        d.seed, d.chain_id);
                  const double u = unit52(w.x, w.y);
                  if (fabs(u - pa) < 1e-12) tally.tie(a, c);
                  acc[r] = u < pa;
                }
              }
            } else {
              bool done = false, deferred = false;
              if (d.precision == 1) {
                // FP32 local field.  Each term carries the rounding of delta to FP32 and
                // each addition one more, so |dE32 - dE| <= 2 (n + 1) 2^-24 sum|terms|;
                // errE takes twice that.  A decision within errE of dE = 0, or with u
                // within errP of p, is recomputed in FP64 (counted in `rechecks`).
                float h = d.twoJ32 * static_cast<float>(nsum[r]);
                float mag = fabsf(h);
                for (int t = q0[r]; t < q1[r]; ++t) {
                  const float dm = ld_global(&d.delta32[a.attr[t]]);
                  h = ld_relaxed(&a.spin[a.col[t]]) > 0 ? h - dm : h + dm;
                  mag += fabsf(dm);
                }
                const float dE = sv[r] > 0 ? h : -h;
                // a bond-free field 2J nn is exact when 2J is (|nn| <= 4)
                const float errE = (q1[r] == q0[r] && d.twoJ32_exact)
                                       ? 0.0f
                                       : mag * static_cast<float>(q1[r] - q0[r] + 3) * 0x1p-22f;
                if (dE <= -errE) {
                  acc[r] = done = true;
                } else if (dE > errE) {
                  const W4 w = philox10_wide(step, static_cast<uint32_t>(v), static_cast<uint32_t>(s), SCO_TAG_MC,
                                        d.seed, d.chain_id);
                  const double u = unit52(w.x, w.y);
                  const float x = d.neg_beta32 * dE;
                  const float pr = expf(x);
                  // expf: about one ulp; beta and the product: one rounding each; the
                  // field: errE
                  const double errP =
                      static_cast<double>(pr) * (static_cast<double>(-d.neg_beta32) * errE * 1.01 + fabs(x) * 0x1p-21 + 0x1p-21) +
                      0x1p-126;
                  // beyond errP + 1e-12 the FP64 decision is the same and no near tie
                  if (fabs(u - static_cast<double>(pr)) > errP + 1e-12) {
                    acc[r] = u < static_cast<double>(pr);
                    done = true;
                  }
                }
                if (!done) {
                  tally.recheck(a, c);
                  const uint32_t qi = atomicAdd(&s_rq, 1u);
                  if (qi < rq_cap) {
                    rq[qi] = kb + r * kBlock + tid;
                    deferred = true;
                  }
                }
              }
              if (!done && !deferred)
                acc[r] = fp64_decision(d, c, v, nsum[r], sv[r], q0[r], q1[r], static_cast<uint32_t>(s));
            }
            if (acc[r]) {
              st_relaxed(&a.spin[g], static_cast<int8_t>(-sv[r]));
              if constexpr (staged) tile[v - tl_base] ^= 1;
            }
          }
          // accepted flips per chain into LDS: one atomic per wave when the wave is one chain
#pragma unroll
          for (int r = 0; r < kBatch; ++r) {
            const int c = live[r] ? cs[r] : -1;
            const int c0 = __shfl(c, 0);
            if (__ballot(c != c0 && c >= 0) == 0) {
              const uint64_t md = __ballot(acc[r] && sv[r] > 0), mu = __ballot(acc[r] && sv[r] < 0);
              if (lane_id() == 0 && (md | mu) && c0 >= 0)
                atomicAdd(&bacc[c0], static_cast<unsigned long long>(__popcll(md)) |
                                         (static_cast<unsigned long long>(__popcll(mu)) << 32));
            } else if (acc[r]) {
              atomicAdd(&bacc[c], sv[r] > 0 ? 1ull : 1ull << 32);
            }
          }
        }
        if (a.any_fp32) {
          // the queued FP64 rechecks of the class (their neighbours are in other classes,
          // so the order of the decisions does not matter)
          __syncthreads();
          const uint32_t nq = min(s_rq, rq_cap);
          for (uint32_t i = tid; i < nq; i += kBlock) {
            const int k = rq[i];
            const int64_t g = r0 + lst[k];
            const int c = c_lo == c_hi ? c_lo : a.chunk_chain[g >> SCO_CHUNK_SHIFT];
            const ChainDesc& d = desc(c);
            int ns, svv, b0, b1;
            site_inputs(g, d, ns, svv, b0, b1);
            const int v = static_cast<int>(g - d.vbase);
            if (fp64_decision(d, c, v, ns, svv, b0, b1, static_cast<uint32_t>(s))) {
              st_relaxed(&a.spin[g], static_cast<int8_t>(-svv));
              if constexpr (staged) tile[v - tl_base] ^= 1;
              atomicAdd(&bacc[c], svv > 0 ? 1ull : 1ull << 32);
            }
          }
          __syncthreads();
          if (tid == 0) s_rq = 0u;
        }
        // between the classes only the spins change (coherent accesses); the phase ends
        // with a full barrier, and so does every class when the caller asks for the
        // fenced form
        const bool last = s + 1 == a.nsw_max && cc + 1 == qmax;
        if (!(last || a.fenced_classes ? grid_barrier(a.sync) : class_barrier(a.sync))) return false;
        mark(a.trace, 1000 + cc);
      }
      // each half of a block's count stays below 2^32 (flushed every sweep when the
      // whole phase could reach it)
      if (flush_each_sweep && s + 1 < a.nsw_max) flush_flips();
    }
    return true;
  };
  auto ldesc = [&](int c) -> const ChainDesc& { return lcd[c - c_lo]; };
  // staging needs one chain and a range that ends inside it (a wrapped neighbour of
  // the last row is then a halo slot, never a padding site), a lattice of at least
  // 8 x 8, the halo rows within kHaloSw bytes per thread, the range within kStageSw
  // words per thread, and room for list and tile
  const bool staged_ok =
      local_cd && c_lo == c_hi && r0 < r1 && r1 - lcd[0].vbase <= lcd[0].N && lcd[0].L >= 8 &&
      2 * lcd[0].L <= kHaloSw * kBlock &&
      (r1 - r0) % 4 == 0 && r1 - r0 <= 4 * kStageSw * kBlock &&
      4 * (r1 - r0) + (r1 - r0) + 2 * lcd[0].L <= static_cast<int64_t>(sizeof(int32_t)) * kListCap;
  bool ok;
  if (staged_ok) ok = body(lds_list, ldesc, Flag<true>{});
  else if (local_cd && r1 - r0 <= kListCap) ok = body(lds_list, ldesc, Flag<false>{});
  else ok = body(lst_mem, [&](int c) -> const ChainDesc& { return a.cd[c]; }, Flag<false>{});
  if (!ok) return false;
  tally.flush(a);
  flush_flips();
  if (blockIdx.x == 0)
    for (int c = tid; c < a.n_chains; c += kBlock) {
      const int nsw = a.nsw_override >= 0 ? a.nsw_override : a.cd[c].n_sw;
      a.st[c].attempts += static_cast<unsigned long long>(a.cd[c].N) * static_cast<unsigned long long>(nsw);
    }
  return true;
}

// Metropolis on H' (Eq. 4) for Heisenberg spins, colour class by colour class with a
// full device barrier between classes (plain loads and stores of the spins).  Site v
// proposes S' uniform on the sphere (Marsaglia, Philox(step, v, s, HP + 256 k)); its
// local energy is -J S . h + the sum of Vbar over its bonds in row order, h the sum of
// its lattice neighbours (+x, -x, +y, -y), Vbar = V - T log(1 - P) with
// 1 - P = -expm1(beta (V - V^max)) (+inf where that is not positive); dE = E(S') - E(S)
// is accepted when dE <= 0, else when u < exp(-beta dE), u from Philox(step, v, s, HA).
// Out of line: inlined twice per bond, its FP64 expm1 and log pushed the Heisenberg
// sweep past its register budget into spills (measured: a call is 42% faster).
__device__ __noinline__ double heis_vbar(const ChainDesc& d, double ax, double ay, double az, double bx,
                                         double by, double bz, int dx, int dy, double Jm) {
  const double V = heis_pair(ax, ay, az, bx, by, bz, dx, dy, Jm);
  const double g = -expm1(d.beta * (V - Jm));
  return g > 0.0 ? V - d.T * log(g) : static_cast<double>(INFINITY);
}

__device__ __forceinline__ bool phase_sweep_heis(const StepArgs& a, uint32_t step, int32_t* lds_list) {
  __shared__ int32_t hoff[SCO_MAXQ + 1];
  __shared__ int32_t hfill[SCO_MAXQ];
  const int qmax = static_cast<int>(a.sync->qmax);
  const int64_t S = ((a.G + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
  const int64_t r0 = min(static_cast<int64_t>(blockIdx.x) * S, a.G);
  const int64_t r1 = min(r0 + S, a.G);
  const int tid = static_cast<int>(threadIdx.x);
  int32_t* const lst = r1 - r0 <= kListCap ? lds_list : reinterpret_cast<int32_t*>(a.rec) + r0;
  Tally tally(r0 < r1 ? a.chunk_chain[r0 >> SCO_CHUNK_SHIFT] : 0);
  uint32_t acc0 = 0u;  // accepted flips of the block's first chain (tally.c0)
  for (int k = tid; k <= qmax; k += kBlock) hoff[k] = 0;
  __syncthreads();
  // colour buckets of the block's sites (block-local offsets)
  for (int pass = 0; pass < 2; ++pass) {
    for (int64_t g = r0 + tid; g < r1; g += kBlock) {
      const ChainDesc& d = a.cd[a.chunk_chain[g >> SCO_CHUNK_SHIFT]];
      if (static_cast<int>(g - d.vbase) >= d.N) continue;
      const int col = a.color[g];
      if (col >= qmax) {  // cannot happen after a complete colouring
        if (pass == 0) set_flag(a.sync, SCO_FLAG_PALETTE);
        continue;
      }
      if (pass == 0) atomicAdd(&hoff[col + 1], 1);
      else lst[hoff[col] + atomicAdd(&hfill[col], 1)] = static_cast<int32_t>(g - r0);
    }
    __syncthreads();
    if (pass == 0) {
      if (tid == 0)
        for (int k = 0; k < qmax; ++k) hoff[k + 1] += hoff[k];
      for (int k = tid; k < qmax; k += kBlock) hfill[k] = 0;
      __syncthreads();
    }
  }
  // the sweeps, in two inlined copies: the block's range in one chain (the usual case;
  // its descriptor block-uniform, read with scalar loads) or in several
  auto sweeps = [&](const auto& chain_of) __attribute__((always_inline)) -> bool {
  for (int s = 0; s < a.nsw_max; ++s) {
    for (int cc = 0; cc < qmax; ++cc) {
      for (int k = hoff[cc] + tid; k < hoff[cc + 1]; k += kBlock) {
        const int64_t g = r0 + lst[k];
        const int c = chain_of(g);
        const ChainDesc& d = a.cd[c];
        const int nsw = a.nsw_override >= 0 ? a.nsw_override : d.n_sw;
        if (s >= nsw) continue;
        const int v = static_cast<int>(g - d.vbase);
        double px, py, pz;
        if (!sphere_point(step, static_cast<uint32_t>(v), static_cast<uint32_t>(s), SCO_TAG_HP, d.seed, d.chain_id,
                          px, py, pz))
          continue;
        const int y = idiv_fp(v, d.inv_L), x = v - y * d.L;
        int nb[4];
        nn_sites(x, y, d.L, d.periodic, nb);
        double hx = 0.0, hy = 0.0, hz = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (nb[t] >= 0) {
            const double* B = a.spin3 + 3 * (d.vbase + nb[t]);
            hx += B[0];
            hy += B[1];
            hz += B[2];
          }
        double* Sp = a.spin3 + 3 * g;
        const double sx = Sp[0], sy = Sp[1], sz = Sp[2];
        const double mJ = -(d.twoJ * 0.5);
        double Eold = mJ * (sx * hx + sy * hy + sz * hz);
        double Enew = mJ * (px * hx + py * hy + pz * hz);
        int b0 = a.row_ptr[g], b1 = a.row_ptr[g + 1];
        row_checked(a, b0, b1);
        for (int e = b0; e < b1; ++e) {
          const int m = a.attr[e];
          const double* B = a.spin3 + 3 * static_cast<int64_t>(a.col[e]);
          const uint32_t hp = ld_global(&d.hd[m]);
          const int dx = static_cast<int16_t>(hp & 0xFFFFu), dy = static_cast<int16_t>(hp >> 16);
          const double Jm = ld_global(&d.J[m]);
          const double bx = B[0], by = B[1], bz = B[2];
          Eold += heis_vbar(d, sx, sy, sz, bx, by, bz, dx, dy, Jm);
          Enew += heis_vbar(d, px, py, pz, bx, by, bz, dx, dy, Jm);
        }
        const double dE = Enew - Eold;
        bool acc = true;
        if (!(dE <= 0.0)) {
          const W4 w = philox10(step, static_cast<uint32_t>(v), static_cast<uint32_t>(s), SCO_TAG_HA, d.seed,
                                d.chain_id);
          const double u = unit52(w.x, w.y);
          const double pr = exp(-d.beta * dE);
          if (fabs(u - pr) < 1e-12) tally.tie(a, c);
          acc = u < pr;
        }
        if (acc) {
          Sp[0] = px;
          Sp[1] = py;
          Sp[2] = pz;
          if (c == tally.c0) ++acc0;
          else atomicAdd(&a.st[c].accepted, 1ull);
        }
      }
      if (!grid_barrier(a.sync)) return false;
    }
  }
  return true;
  };
  const int c_lo = r0 < r1 ? a.chunk_chain[r0 >> SCO_CHUNK_SHIFT] : 0;
  const int c_hi = r0 < r1 ? a.chunk_chain[(r1 - 1) >> SCO_CHUNK_SHIFT] : 0;
  const bool ok = c_lo == c_hi ? sweeps([&](int64_t) { return c_lo; })
                               : sweeps([&](int64_t g) { return a.chunk_chain[g >> SCO_CHUNK_SHIFT]; });
  if (!ok) return false;
  tally.flush(a);
  const unsigned long long ta = block_sum(static_cast<unsigned long long>(acc0));
  if (tid == 0 && ta && tally.c0 < a.n_chains) atomicAdd(&a.st[tally.c0].accepted, ta);
  if (blockIdx.x == 0)
    for (int c = tid; c < a.n_chains; c += kBlock) {
      const int nsw = a.nsw_override >= 0 ? a.nsw_override : a.cd[c].n_sw;
      a.st[c].attempts += static_cast<unsigned long long>(a.cd[c].N) * static_cast<unsigned long long>(nsw);
    }
  return true;
}

// ------------------------------------------------------------------ the step
// Persistent kernel (cooperative launch: every block resident).  `phases` selects
// steps (1) switching + assembly, (2) colouring, (3) sweeps.  The switching part
// starts by clearing the per-chain counters of the graph; a launch without it checks
// that the words left by the earlier launches say a complete graph (and colouring) is
// there.
template <uint32_t phases, int model>
__device__ __forceinline__ bool step_body(const StepArgs& a, uint32_t step, PhaseLds& lds, KwShared& ks) {
  constexpr bool heis = model == SCO_MODEL_HEIS;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  {
    // A launch after one that ended on a raised flag does nothing until the host has
    // consumed the flags: the spins stay as the failed step found them.  halt is
    // written only by the last arriver of a barrier, which every block of this launch
    // reaches after this check; a timeout needs seconds of waiting inside a launch.
    __shared__ uint32_t s_halt;
    if (threadIdx.x == 0) {
      const uint32_t h = ld_poll(&a.sync->halt), f = ld_poll(&a.sync->flags);  // both in flight
      s_halt = (h != 0 || (f & SCO_FLAG_TIMEOUT) != 0) ? 1u : 0u;
    }
    __syncthreads();
    if (s_halt != 0) return false;
  }
  if constexpr ((phases & PH_SWITCH) != 0) {
    // The partner counts are zero here: the scatter of the step before cleared them
    // once the scan had read them (the host clears them at set-up and after a step
    // that raised a flag, which may have stopped anywhere); the owner counts are
    // written for every site by the switching.  The graph counters of the chain
    // states are next written by the row sort, four device barriers on.
    if (lead) {
      a.sync->graph_valid = 0;
      a.sync->color_valid = 0;
    }
    for (int c = gtid(); c < a.n_chains; c += stride) {
      a.st[c].delta_union = 0;
      a.st[c].delta_sco = 0;
      a.st[c].n_edges = 0;
      for (int p = 0; p < SCO_MAXLEVEL; ++p) a.st[c].kw_rounds[p] = 0;
    }
    mark(a.trace, 1);
    phase_switch<heis>(a, step, lds.list);
    mark(a.trace, 2);
    if (!grid_barrier(a.sync)) return false;
    mark(a.trace, 3);
    if (!scan_two_pass(a.deg, a.own, a.G, a.row_ptr, a.scan_agg, lds.list, a.sync))
      return false;
    if (!grid_barrier(a.sync)) return false;
    mark(a.trace, 4);
    phase_scatter(a);
    if (!grid_barrier(a.sync)) return false;
    mark(a.trace, 5);
    phase_rowsort(a, lds.list, kListCap);
    if (!grid_barrier(a.sync)) return false;
    mark(a.trace, 6);
    if (lead) a.sync->graph_valid = 1;
  }
  if constexpr ((phases & PH_COLOR) != 0) {
    if constexpr ((phases & PH_SWITCH) == 0) {
      // a separate colouring needs a completed switching (every block reads the
      // same word, written by an earlier launch)
      if (a.sync->graph_valid != 1) {
        if (lead) set_flag(a.sync, SCO_FLAG_STATE);
        return false;
      }
      if (lead) a.sync->color_valid = 0;
    }
    mark(a.trace, 10);
    kw_setup(a, ks);
    if (a.coloring == SCO_COLOR_BCR) {
      // ends with the barrier that finds the last frontier empty
      if (!phase_color_bcr(a, ks, lds.list)) return false;
    } else {
      phase_kw_local(a, ks, lds.tile);
      mark(a.trace, 11);
      if (!grid_barrier(a.sync)) return false;
      // the global levels end with a full barrier (none when every level ran in tiles)
      if (!phase_kw_global(a, ks, lds.list)) return false;
      if (ks.mmax > ks.pmin) phase_colour_fill(a);
    }
    mark(a.trace, 12);
    if (lead) a.sync->color_valid = 1;
  }
  if constexpr ((phases & PH_SWEEP) != 0) {
    if constexpr ((phases & PH_COLOR) == 0) {
      if (a.sync->color_valid != 1) {
        if (lead) set_flag(a.sync, SCO_FLAG_STATE);
        return false;
      }
    }
    mark(a.trace, 20);
    // the sweeps end with a full barrier, so the next step sees every spin
    if constexpr (heis) {
      if (!phase_sweep_heis(a, step, lds.list)) return false;
    } else {
      if (!phase_sweep(a, step, lds.list)) return false;
    }
    mark(a.trace, 21);
  }
  return true;
}

// Persistent kernel (cooperative launch: every block resident), one step of every
// chain.  `phases` selects steps (1) switching + assembly, (2) colouring, (3) sweeps.
// The switching part starts by clearing the per-chain counters of the graph; a
// launch without it checks that the words left by the earlier launches say a complete
// graph (and colouring) is there.  (Looping over
// several steps inside one launch was measured to push the fused kernel past its
// register budget into spills, for a saving of a few microseconds per step.)
template <uint32_t phases, int model>
__global__ void __launch_bounds__(kBlock) k_step(const StepArgs a) {
  __shared__ PhaseLds lds;
  __shared__ KwShared ks;
  step_body<phases, model>(a, a.step, lds, ks);
}

// =================================================================== observables
// Per chunk (one chain): sum s, sum over the NN pairs (+x, +y) of s_i s_j, and the
// set of colours in use.
extern "C" __global__ void __launch_bounds__(kBlock)
    k_obs_basic(const ChainDesc* __restrict__ cd, const int32_t* __restrict__ chunk_chain,
                const int8_t* __restrict__ spin, const uint16_t* __restrict__ color,
                unsigned long long* __restrict__ out, unsigned* __restrict__ used, int64_t G) {
  __shared__ unsigned s_used[SCO_QWORDS];
  if (threadIdx.x < SCO_QWORDS) s_used[threadIdx.x] = 0;
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
  if (threadIdx.x < SCO_QWORDS && s_used[threadIdx.x])
    atomicOr(&used[c * SCO_QWORDS + threadIdx.x], s_used[threadIdx.x]);
}

// Colour class sizes of one chain: per-block LDS histogram, one atomic per bin.
extern "C" __global__ void __launch_bounds__(256)
    k_class_sizes(const uint16_t* __restrict__ color, int64_t vbase, int N, unsigned long long* __restrict__ out) {
  __shared__ unsigned int h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  for (int v = static_cast<int>(blockIdx.x * 256 + threadIdx.x); v < N; v += static_cast<int>(gridDim.x * 256)) {
    const int k = color[vbase + v];
    if (k < 256) atomicAdd(&h[k], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&out[threadIdx.x], static_cast<unsigned long long>(h[threadIdx.x]));
}

// Surviving bonds per displacement index of one chain: each undirected bond once, from
// the row of its smaller site.
extern "C" __global__ void k_bond_hist(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                       const int32_t* __restrict__ attr, int64_t vbase, int N,
                                       unsigned long long* __restrict__ counts) {
  const int64_t v = gtid();
  if (v >= N) return;
  const int64_t g = vbase + v;
  for (int e = row_ptr[g]; e < row_ptr[g + 1]; ++e)
    if (col[e] > g) atomicAdd(&counts[attr[e]], 1ull);
}

// st[c].mag from the spin sums of k_obs_basic (after the spins were set from outside).
extern "C" __global__ void k_set_mag(ChainState* __restrict__ st, const unsigned long long* __restrict__ out,
                                     int n) {
  const int c = static_cast<int>(gtid());
  if (c < n) st[c].mag = static_cast<long long>(out[2 * c]);
}

// One measured step of an annealing stage: per chain |M|, M^2, the directed bonds and
// the two maximum degrees of the step's graph, summed exactly.
extern "C" __global__ void k_anneal_acc(const ChainState* __restrict__ st, AnnealAcc* __restrict__ acc, int n) {
  const int c = static_cast<int>(gtid());
  if (c >= n) return;
  const long long m = st[c].mag;
  const unsigned long long am = static_cast<unsigned long long>(m < 0 ? -m : m);
  AnnealAcc& x = acc[c];
  x.samples += 1ull;
  x.abs_m += am;
  x.m2 += am * am;
  x.bonds += st[c].n_edges;
  x.delta_sco += static_cast<unsigned long long>(st[c].delta_sco);
  x.delta_union += static_cast<unsigned long long>(st[c].delta_union);
}

// Heisenberg, open lattice: prod[m] = sum over the owners i ascending of the pair
// energy of displacement m (the order of the reference's sum, so each prod[m] is the
// same number).
extern "C" __global__ void k_obs_heis_pairs(const uint32_t* __restrict__ hd, const double* __restrict__ J, int K,
                                            int L, const double* __restrict__ s3, double* __restrict__ prod) {
  const int64_t m = gtid();
  if (m >= K) return;
  const uint32_t p = hd[m];
  const int dx = static_cast<int16_t>(p & 0xFFFFu), dy = static_cast<int16_t>(p >> 16);
  const double Jm = J[m];
  double em = 0.0;
  for (int y = 0; y + dy < L; ++y)
    for (int x = 0; x < L; ++x) {
      const int jx = x + dx;
      if (jx < 0 || jx >= L) continue;
      const double* A = s3 + 3 * (static_cast<int64_t>(y) * L + x);
      const double* B = s3 + 3 * (static_cast<int64_t>(y + dy) * L + jx);
      em += heis_pair(A[0], A[1], A[2], B[0], B[1], B[2], dx, dy, Jm);
    }
  prod[m] = em;
}

// Heisenberg, per block of 256 sites: the exchange sum over the (+x, +y) pairs and the
// Eq. (7) sum of [S x (r - r_c) / |r - r_c|]_z, r_c = ((L-1)/2, (L-1)/2); fixed tree order.
extern "C" __global__ void __launch_bounds__(256)
    k_obs_heis_site(const double* __restrict__ s3, int L, double* __restrict__ part2) {
  __shared__ double be[256], bm[256];
  const int N = L * L;
  const int v = static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
  double ex = 0.0, mp = 0.0;
  if (v < N) {
    const int y = v / L, x = v - y * L;
    const double* S = s3 + 3 * static_cast<int64_t>(v);
    if (x + 1 < L) ex += S[0] * S[3] + S[1] * S[4] + S[2] * S[5];
    if (y + 1 < L) {
      const double* U = S + 3 * static_cast<int64_t>(L);
      ex += S[0] * U[0] + S[1] * U[1] + S[2] * U[2];
    }
    const double rx = static_cast<double>(x) - 0.5 * static_cast<double>(L - 1);
    const double ry = static_cast<double>(y) - 0.5 * static_cast<double>(L - 1);
    const double d = sqrt(rx * rx + ry * ry);
    if (d > 0.0) mp = (S[0] * ry - S[1] * rx) / d;
  }
  be[threadIdx.x] = ex;
  bm[threadIdx.x] = mp;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < static_cast<uint32_t>(o)) {
      be[threadIdx.x] += be[threadIdx.x + o];
      bm[threadIdx.x] += bm[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part2[2 * blockIdx.x] = be[0];
    part2[2 * blockIdx.x + 1] = bm[0];
  }
}

extern "C" __global__ void k_obs_heis_site_final(const double* __restrict__ part2, int nparts,
                                                 double* __restrict__ out2) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double e = 0.0, m = 0.0;
  for (int i = 0; i < nparts; ++i) {
    e += part2[2 * i];
    m += part2[2 * i + 1];
  }
  out2[0] = e;
  out2[1] = m;
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

// ------------------------------------------------ pair correlations by an exact transform
// The same owned-pair correlations C_m from a number-theoretic transform of the spins:
// arithmetic modulo a prime p < 2^31 with n | p - 1 (chosen on the host, with a
// primitive n-th root of unity w), values in Montgomery form (R = 2^32).  The 2-D
// transform S(k) of the spins on an n x n array (the lattice, zero-padded to
// n >= 2L - 1 when it is open), the product S(k) S(-k), and the inverse transform
// give n^2 C(d), C(d) = sum_x s(x) s(x + d) cyclic over n, exactly as integers mod p
// (|C| < p / 2).  Every 1-D transform runs as Stockham passes of radix 2..8 along the
// rows, then along the columns.

__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t b, uint32_t p, uint32_t pinv) {
  const uint64_t t = static_cast<uint64_t>(a) * b;  // < p^2 < 2^62
  const uint32_t m = static_cast<uint32_t>(t) * pinv;
  const uint64_t u = (t + static_cast<uint64_t>(m) * p) >> 32;  // < 2 p
  return u >= p ? static_cast<uint32_t>(u - p) : static_cast<uint32_t>(u);
}
__device__ __forceinline__ uint32_t mod_add(uint32_t a, uint32_t b, uint32_t p) {
  const uint32_t s = a + b;  // < 2^32 for a, b < p < 2^31
  return s >= p ? s - p : s;
}

// spins (one chain, row-major L x L) into the n x n array: R mod p for +1, p - (R mod
// p) for -1, 0 in the padding
extern "C" __global__ void k_ntt_load(const int8_t* __restrict__ spin, int64_t vbase, int L, int n,
                                      uint32_t one, uint32_t p, uint32_t* __restrict__ out) {
  const int64_t t = gtid();
  if (t >= static_cast<int64_t>(n) * n) return;
  const int y = static_cast<int>(t / n), x = static_cast<int>(t - static_cast<int64_t>(y) * n);
  uint32_t v = 0;
  if (x < L && y < L) v = spin[vbase + static_cast<int64_t>(y) * L + x] > 0 ? one : p - one;
  out[t] = v;
}

// One Stockham pass of radix R over every row (dim 0) or column (dim 1): the pass
// joins R transforms of length Ns into transforms of length Ns R; tw[e] = w^e
// (Montgomery form), e < n; inv: the inverse transform (w^-1), unscaled.
template <int R>
__global__ void k_ntt_pass(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int n, int Ns, int dim,
                           const uint32_t* __restrict__ tw, uint32_t p, uint32_t pinv, int inv) {
  const int64_t t = gtid();
  const int m = n / R;
  if (t >= static_cast<int64_t>(n) * m) return;
  int line, j;
  if (dim == 0) {  // consecutive threads along a row
    line = static_cast<int>(t / m);
    j = static_cast<int>(t - static_cast<int64_t>(line) * m);
  } else {  // consecutive threads across the columns
    j = static_cast<int>(t / n);
    line = static_cast<int>(t - static_cast<int64_t>(j) * n);
  }
  auto at = [&](int x) -> int64_t {
    return dim == 0 ? static_cast<int64_t>(line) * n + x : static_cast<int64_t>(x) * n + line;
  };
  const int k = j % Ns;
  const int step = n / (Ns * R);  // the pass's twiddles are w_{Ns R}^{k q} = w^{step k q}, step k q < n
  uint32_t a[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const uint32_t v = in[at(j + q * m)];
    const int e = step * k * q;
    a[q] = q == 0 ? v : mont_mul(v, tw[inv && e ? n - e : e], p, pinv);
  }
  const int base = (j / Ns) * Ns * R + k;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    uint32_t acc = a[0];
#pragma unroll
    for (int q = 1; q < R; ++q) {
      const int e = static_cast<int>((static_cast<int64_t>(m) * q * u) % n);  // w_R^{q u}
      acc = mod_add(acc, mont_mul(a[q], tw[inv && e ? n - e : e], p, pinv), p);
    }
    out[at(base + u * Ns)] = acc;
  }
}

// S(k) S(-k) of the forward transform
extern "C" __global__ void k_ntt_square(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int n,
                                        uint32_t p, uint32_t pinv) {
  const int64_t t = gtid();
  if (t >= static_cast<int64_t>(n) * n) return;
  const int ky = static_cast<int>(t / n), kx = static_cast<int>(t - static_cast<int64_t>(ky) * n);
  const int64_t tm = static_cast<int64_t>(ky ? n - ky : 0) * n + (kx ? n - kx : 0);
  out[t] = mont_mul(in[t], in[tm], p, pinv);
}

// prod[m] = J_m C_m from the inverse transform (n^2 C(d) in Montgomery form, times
// n^-2 mod p): the owned pairs of displacement d_m are C(d_m), halved for the
// self-conjugate displacements of a periodic lattice, whose pairs C counts twice
extern "C" __global__ void k_ntt_gather(const uint32_t* __restrict__ cn, int n, int L, int periodic,
                                        const uint32_t* __restrict__ hd, const double* __restrict__ J, int K,
                                        uint32_t ninv2, uint32_t p, uint32_t pinv, double* __restrict__ prod) {
  const int64_t m = gtid();
  if (m >= K) return;
  const uint32_t hp = hd[m];
  const int dx = static_cast<int16_t>(hp & 0xFFFFu), dy = static_cast<int16_t>(hp >> 16);
  const int ix = dx < 0 ? dx + n : dx, iy = dy < 0 ? dy + n : dy;
  const uint32_t v = mont_mul(cn[static_cast<int64_t>(iy) * n + ix], ninv2, p, pinv);
  long long c = v > (p >> 1) ? static_cast<long long>(v) - static_cast<long long>(p) : static_cast<long long>(v);
  const int h = L >> 1;
  if (periodic && ((dy == 0 && dx == h) || (dy == h && (dx == 0 || dx == h)))) c /= 2;
  prod[m] = J[m] * static_cast<double>(c);
}

// ------------------------------------------- Heisenberg dipolar energy by FP64 FFTs
// E_dip = sum over the owned pairs of (J_m / 2) [S_i . S_j - 3 (S_i . d)(S_j . d) / r^2]
// (Eq. 6, J_m = 2 D / r^3) needs, per displacement d, the correlations
// C_ab(d) = sum_i S_i^a S_{i+d}^b of the spin components: S . S = C_xx + C_yy + C_zz
// and (S_i . d)(S_j . d) = dx^2 C_xx + dx dy (C_xy + C_yx) + dy^2 C_yy.  They come from
// complex FP64 transforms of the zero-padded n x n component arrays (n >= 2L - 1, so
// the cyclic correlations are the open lattice's): Z1 = FFT(S^x + i S^y), Z2 = FFT(S^z);
// F_x, F_y separate by the symmetry of real inputs, and the real, even spectra
// |F_x|^2 + |F_y|^2 + |F_z|^2, |F_x|^2, |F_y|^2, 2 Re(conj F_x F_y) go back two per
// inverse transform (real and imaginary parts).  Stockham passes as for the exact
// transform; tw[e] = (cos, sin)(2 pi e / n).

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// spins (one chain, 3 doubles per site) into Z1 = S^x + i S^y and Z2 = S^z, zero-padded
extern "C" __global__ void k_fft_load3(const double* __restrict__ s3, int L, int n, double2* __restrict__ z1,
                                       double2* __restrict__ z2) {
  const int64_t t = gtid();
  if (t >= static_cast<int64_t>(n) * n) return;
  const int y = static_cast<int>(t / n), x = static_cast<int>(t - static_cast<int64_t>(y) * n);
  double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
  if (x < L && y < L) {
    const double* S = s3 + 3 * (static_cast<int64_t>(y) * L + x);
    a = make_double2(S[0], S[1]);
    b.x = S[2];
  }
  z1[t] = a;
  z2[t] = b;
}

// One Stockham pass of radix R (forward: e^{-2 pi i / n}; inv: e^{+2 pi i / n}, unscaled)
template <int R>
__global__ void k_fft_pass(const double2* __restrict__ in, double2* __restrict__ out, int n, int Ns, int dim,
                           const double2* __restrict__ tw, int inv) {
  const int64_t t = gtid();
  const int m = n / R;
  if (t >= static_cast<int64_t>(n) * m) return;
  int line, j;
  if (dim == 0) {
    line = static_cast<int>(t / m);
    j = static_cast<int>(t - static_cast<int64_t>(line) * m);
  } else {
    j = static_cast<int>(t / n);
    line = static_cast<int>(t - static_cast<int64_t>(j) * n);
  }
  auto at = [&](int x) -> int64_t {
    return dim == 0 ? static_cast<int64_t>(line) * n + x : static_cast<int64_t>(x) * n + line;
  };
  auto w = [&](int e) {  // w^e of the transform's direction
    const double2 c = tw[e];
    return inv ? c : make_double2(c.x, -c.y);
  };
  const int k = j % Ns;
  const int step = n / (Ns * R);
  double2 a[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const double2 v = in[at(j + q * m)];
    a[q] = q == 0 ? v : cmul(v, w(step * k * q));
  }
  const int base = (j / Ns) * Ns * R + k;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    double2 acc = a[0];
#pragma unroll
    for (int q = 1; q < R; ++q) {
      const double2 c = cmul(a[q], w(static_cast<int>((static_cast<int64_t>(m) * q * u) % n)));
      acc.x += c.x;
      acc.y += c.y;
    }
    out[at(base + u * Ns)] = acc;
  }
}

// The four spectra from Z1, Z2, in place, one thread per pair {k, -k}:
// Z1 <- |F_x|^2 + |F_y|^2 + |F_z|^2 + i |F_x|^2,  Z2 <- |F_y|^2 + i 2 Re(conj F_x F_y),
// F_x(k) = (Z1(k) + conj Z1(-k)) / 2, F_y(k) = (Z1(k) - conj Z1(-k)) / 2i
extern "C" __global__ void k_fft_spectra(double2* __restrict__ z1, double2* __restrict__ z2, int n) {
  const int64_t t = gtid();
  const int64_t nn = static_cast<int64_t>(n) * n;
  if (t >= nn) return;
  const int ky = static_cast<int>(t / n), kx = static_cast<int>(t - static_cast<int64_t>(ky) * n);
  const int64_t tm = static_cast<int64_t>(ky ? n - ky : 0) * n + (kx ? n - kx : 0);
  if (tm < t) return;  // the pair's other member does both
  auto spectra = [](double2 zk, double2 zmk, double2 z2k, double2& o1, double2& o2) {
    const double fxr = 0.5 * (zk.x + zmk.x), fxi = 0.5 * (zk.y - zmk.y);
    const double fyr = 0.5 * (zk.y + zmk.y), fyi = -0.5 * (zk.x - zmk.x);
    const double pxx = fxr * fxr + fxi * fxi, pyy = fyr * fyr + fyi * fyi;
    const double pzz = z2k.x * z2k.x + z2k.y * z2k.y;
    o1 = make_double2(pxx + pyy + pzz, pxx);
    o2 = make_double2(pyy, 2.0 * (fxr * fyr + fxi * fyi));
  };
  const double2 a = z1[t], b = z1[tm], ca = z2[t], cb = z2[tm];
  double2 o1, o2, p1, p2;
  spectra(a, b, ca, o1, o2);
  spectra(b, a, cb, p1, p2);
  z1[t] = o1;
  z2[t] = o2;
  if (tm != t) {
    z1[tm] = p1;
    z2[tm] = p2;
  }
}

// prod[m] = (J_m / 2) [S(d) - 3 (dx^2 C_xx + dx dy (C_xy + C_yx) + dy^2 C_yy) / r^2] from
// the inverse transforms (n^2 times the correlations)
extern "C" __global__ void k_fft_gather_heis(const double2* __restrict__ w1, const double2* __restrict__ w2,
                                             int n, const uint32_t* __restrict__ hd, const double* __restrict__ J,
                                             int K, double* __restrict__ prod) {
  const int64_t m = gtid();
  if (m >= K) return;
  const uint32_t hp = hd[m];
  const int dx = static_cast<int16_t>(hp & 0xFFFFu), dy = static_cast<int16_t>(hp >> 16);
  const int64_t idx = static_cast<int64_t>(dy < 0 ? dy + n : dy) * n + (dx < 0 ? dx + n : dx);
  const double inv = 1.0 / (static_cast<double>(n) * static_cast<double>(n));
  const double2 a = w1[idx], b = w2[idx];
  const double sdot = a.x * inv, cxx = a.y * inv, cyy = b.x * inv, cxy = b.y * inv;
  const double fx = static_cast<double>(dx), fy = static_cast<double>(dy);
  const double r2 = fx * fx + fy * fy;
  prod[m] = (J[m] * 0.5) * (sdot - 3.0 * (fx * fx * cxx + fx * fy * cxy + fy * fy * cyy) / r2);
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

// =================================================================== static scratch
// Device memory of the entry point that allocates nothing (sco_run_noalloc): the
// workspace of its chains lives here.  Every GPU that loads the library holds one copy
// until the process ends; calls on one GPU share it (and must not overlap).  In host
// code `scratch` names only a host-side handle: kernels are given the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[SCO_NOALLOC_BYTES];

// =================================================================== host launchers
namespace sco_dev {

hipError_t noalloc_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (addr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // with device `dev` current
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t table_j(hipStream_t s, const uint32_t* hd, int K, int L, int periodic, int n_images,
                   double D, double* J) {
  hipLaunchKernelGGL(k_table_j, dim3((K + 255) / 256), dim3(256), 0, s, hd, K, L, periodic, n_images, D, J);
  return hipGetLastError();
}

hipError_t init_spins(hipStream_t s, const ChainDesc* cd, const int32_t* chunk_chain,
                      const int64_t* src_base, const int8_t* src, int8_t* spin, double* spin3, int64_t G) {
  hipLaunchKernelGGL(k_init_spins, dim3(static_cast<uint32_t>(G / kBlock)), dim3(kBlock), 0, s, cd,
                     chunk_chain, src_base, src, spin, spin3, G);
  return hipGetLastError();
}

template <uint32_t P, int M>
const void* step_kernel() {
  return reinterpret_cast<const void*>(&k_step<P, M>);
}

template <int M>
const void* step_kernel_of(uint32_t phases) {
  switch (phases) {
    case PH_SWITCH: return step_kernel<PH_SWITCH, M>();
    case PH_COLOR: return step_kernel<PH_COLOR, M>();
    case PH_SWEEP: return step_kernel<PH_SWEEP, M>();
    default: return step_kernel<PH_SWITCH | PH_COLOR | PH_SWEEP, M>();
  }
}

const void* step_kernel_for(uint32_t phases, int model) {
  return model == SCO_MODEL_HEIS ? step_kernel_of<SCO_MODEL_HEIS>(phases) : step_kernel_of<SCO_MODEL_ISING>(phases);
}

// co-resident blocks of the step kernels (the smallest over the variants)
int step_max_blocks() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  int best = 1 << 30;
  const uint32_t variants[4] = {PH_SWITCH, PH_COLOR, PH_SWEEP, PH_SWITCH | PH_COLOR | PH_SWEEP};
  for (int model : {SCO_MODEL_ISING, SCO_MODEL_HEIS})
    for (uint32_t ph : variants) {
      int per = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, step_kernel_for(ph, model), kBlock, 0) != hipSuccess)
        return 0;
      best = per < best ? per : best;
    }
  return best * cus;
}

const void* step_kernel_full(int model) { return step_kernel_for(PH_SWITCH | PH_COLOR | PH_SWEEP, model); }

hipError_t step(hipStream_t s, const StepArgs& a, uint32_t phases, int blocks, int model) {
  StepArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(step_kernel_for(phases, model), dim3(blocks), dim3(kBlock), args, 0, s);
}

hipError_t obs_basic(hipStream_t s, const ChainDesc* cd, const int32_t* chunk_chain, const int8_t* spin,
                     const uint16_t* color, unsigned long long* out, unsigned* used, int64_t G) {
  hipLaunchKernelGGL(k_obs_basic, dim3(static_cast<uint32_t>(G / kBlock)), dim3(kBlock), 0, s, cd,
                     chunk_chain, spin, color, out, used, G);
  return hipGetLastError();
}

hipError_t obs_heis(hipStream_t s, const ChainDesc* cd, int chain, const ChainDesc& h, const double* spin3,
                    double* prod, double* part, double* out, double* part2, double* out2, bool dipolar,
                    const NttPlan* fft, double2* fbuf, const double2* ftw) {
  (void)cd;
  (void)chain;
  const double* s3 = spin3 + 3 * h.vbase;
  if (!dipolar) {
    // the site sums only (exchange, M_phi)
  } else if (fft && fft->n > 0) {
    const int n = fft->n;
    const int64_t nn = static_cast<int64_t>(n) * n;
    const dim3 g1(static_cast<uint32_t>((nn + 255) / 256));
    double2* buf[3] = {fbuf, fbuf + nn, fbuf + 2 * nn};  // Z1, Z2, scratch
    hipLaunchKernelGGL(k_fft_load3, g1, dim3(256), 0, s, s3, h.L, n, buf[0], buf[1]);
    // a 2-D transform of buf[which], ping-ponging with the scratch; the result ends in buf[which]
    auto transform = [&](int which, int inv) {
      double2* A = buf[which];
      double2* B = buf[2];
      for (int dim = 0; dim < 2; ++dim) {
        int Ns = 1;
        for (int i = 0; i < fft->nrad; ++i) {
          const int r = fft->rad[i];
          const dim3 g(static_cast<uint32_t>((nn / r + 255) / 256));
          switch (r) {
            case 2: hipLaunchKernelGGL(k_fft_pass<2>, g, dim3(256), 0, s, A, B, n, Ns, dim, ftw, inv); break;
            case 3: hipLaunchKernelGGL(k_fft_pass<3>, g, dim3(256), 0, s, A, B, n, Ns, dim, ftw, inv); break;
            case 4: hipLaunchKernelGGL(k_fft_pass<4>, g, dim3(256), 0, s, A, B, n, Ns, dim, ftw, inv); break;
            case 5: hipLaunchKernelGGL(k_fft_pass<5>, g, dim3(256), 0, s, A, B, n, Ns, dim, ftw, inv); break;
            case 7: hipLaunchKernelGGL(k_fft_pass<7>, g, dim3(256), 0, s, A, B, n, Ns, dim, ftw, inv); break;
            default: hipLaunchKernelGGL(k_fft_pass<8>, g, dim3(256), 0, s, A, B, n, Ns, dim, ftw, inv); break;
          }
          Ns *= r;
          double2* x = A;
          A = B;
          B = x;
        }
      }
      if (A != buf[which]) {  // an odd number of passes: the result is in the scratch
        buf[2] = buf[which];
        buf[which] = A;
      }
    };
    transform(0, 0);
    transform(1, 0);
    hipLaunchKernelGGL(k_fft_spectra, g1, dim3(256), 0, s, buf[0], buf[1], n);
    transform(0, 1);
    transform(1, 1);
    hipLaunchKernelGGL(k_fft_gather_heis, dim3((h.K + 255) / 256), dim3(256), 0, s, buf[0], buf[1], n, h.hd, h.J,
                       h.K, prod);
  } else {
    hipLaunchKernelGGL(k_obs_heis_pairs, dim3((h.K + 255) / 256), dim3(256), 0, s, h.hd, h.J, h.K, h.L, s3, prod);
  }
  if (dipolar) {
    const int nparts = (h.K + 4095) / 4096;
    hipLaunchKernelGGL(k_obs_sum_partials, dim3(nparts), dim3(256), 0, s, prod, h.K, part);
    hipLaunchKernelGGL(k_obs_sum_final, dim3(1), dim3(64), 0, s, part, nparts, out);
  }
  const int nb = (h.N + 255) / 256;
  hipLaunchKernelGGL(k_obs_heis_site, dim3(nb), dim3(256), 0, s, s3, h.L, part2);
  hipLaunchKernelGGL(k_obs_heis_site_final, dim3(1), dim3(64), 0, s, part2, nb, out2);
  return hipGetLastError();
}

hipError_t class_sizes(hipStream_t s, const uint16_t* color, int64_t vbase, int N, unsigned long long* out) {
  const int nb = std::min(1024, (N + 255) / 256);
  hipLaunchKernelGGL(k_class_sizes, dim3(nb), dim3(256), 0, s, color, vbase, N, out);
  return hipGetLastError();
}

hipError_t bond_hist(hipStream_t s, const int32_t* row_ptr, const int32_t* col, const int32_t* attr, int64_t vbase,
                     int N, unsigned long long* counts) {
  hipLaunchKernelGGL(k_bond_hist, dim3((N + 255) / 256), dim3(256), 0, s, row_ptr, col, attr, vbase, N, counts);
  return hipGetLastError();
}

hipError_t set_mag(hipStream_t s, ChainState* st, const unsigned long long* out, int n) {
  hipLaunchKernelGGL(k_set_mag, dim3((n + 255) / 256), dim3(256), 0, s, st, out, n);
  return hipGetLastError();
}

hipError_t anneal_acc(hipStream_t s, const ChainState* st, AnnealAcc* acc, int n) {
  hipLaunchKernelGGL(k_anneal_acc, dim3((n + 255) / 256), dim3(256), 0, s, st, acc, n);
  return hipGetLastError();
}

hipError_t obs_dipolar(hipStream_t s, const uint32_t* hd, const double* J, int K, int L, int periodic,
                       const int8_t* spin, int64_t vbase, uint32_t* bits, double* prod, double* part,
                       double* out, const NttPlan* plan, uint32_t* nbuf, uint32_t* tw) {
  if (plan && plan->n > 0) {
    const int n = plan->n;
    const int64_t nn = static_cast<int64_t>(n) * n;
    const dim3 g1(static_cast<uint32_t>((nn + 255) / 256));
    uint32_t* A = nbuf;
    uint32_t* B = nbuf + nn;
    hipLaunchKernelGGL(k_ntt_load, g1, dim3(256), 0, s, spin, vbase, L, n, plan->one, plan->p, A);
    auto passes = [&](int inv) {
      for (int dim = 0; dim < 2; ++dim) {
        int Ns = 1;
        for (int i = 0; i < plan->nrad; ++i) {
          const int r = plan->rad[i];
          const dim3 g(static_cast<uint32_t>((nn / r + 255) / 256));
          switch (r) {
            case 2: hipLaunchKernelGGL(k_ntt_pass<2>, g, dim3(256), 0, s, A, B, n, Ns, dim, tw, plan->p, plan->pinv, inv); break;
            case 3: hipLaunchKernelGGL(k_ntt_pass<3>, g, dim3(256), 0, s, A, B, n, Ns, dim, tw, plan->p, plan->pinv, inv); break;
            case 4: hipLaunchKernelGGL(k_ntt_pass<4>, g, dim3(256), 0, s, A, B, n, Ns, dim, tw, plan->p, plan->pinv, inv); break;
            case 5: hipLaunchKernelGGL(k_ntt_pass<5>, g, dim3(256), 0, s, A, B, n, Ns, dim, tw, plan->p, plan->pinv, inv); break;
            case 7: hipLaunchKernelGGL(k_ntt_pass<7>, g, dim3(256), 0, s, A, B, n, Ns, dim, tw, plan->p, plan->pinv, inv); break;
            default: hipLaunchKernelGGL(k_ntt_pass<8>, g, dim3(256), 0, s, A, B, n, Ns, dim, tw, plan->p, plan->pinv, inv); break;
          }
          Ns *= r;
          uint32_t* x = A;
          A = B;
          B = x;
        }
      }
    };
    passes(0);
    hipLaunchKernelGGL(k_ntt_square, g1, dim3(256), 0, s, A, B, n, plan->p, plan->pinv);
    {
      uint32_t* x = A;
      A = B;
      B = x;
    }
    passes(1);
    hipLaunchKernelGGL(k_ntt_gather, dim3((K + 255) / 256), dim3(256), 0, s, A, n, L, periodic, hd, J, K,
                       plan->ninv2, plan->p, plan->pinv, prod);
  } else if (L % 32 == 0) {
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
