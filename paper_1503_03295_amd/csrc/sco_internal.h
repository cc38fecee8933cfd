// sco_internal.h -- layouts shared by the host runtime and the gfx950 kernels of libsco.
//
// Global site space: the chains' sites are concatenated, each chain starting at a
// multiple of SCO_CHUNK so that a chunk of global sites belongs to one chain
// (chunk_chain[g >> SCO_CHUNK_SHIFT]).  Padding sites (local index >= N) are never
// touched by the method.  A chunk is exactly one block of the step kernel.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

#define SCO_CHUNK 1024          // sites per chunk == threads per block
#define SCO_CHUNK_SHIFT 10
#define SCO_MAXQ 255            // largest palette (Delta + 1) handled: colours fit a byte
#define SCO_QWORDS 8            // 32-bit words of a colour bitmask
#define SCO_MAXLEVEL 32         // KW levels are at most ceil(log2(N)) <= 31
#define SCO_MAXCHAINS 256
#define SCO_TILE_MAX 28672      // sites of a KW tile held in LDS (local levels): 7 * 2^12
#define SCO_SCAN_ITEMS 21       // values per thread of a degree-scan tile (21504-value tiles)
#define SCO_GUIDE_BITS 14       // guide table of the cumulative couplings: 2^14 buckets
#define SCO_BAR_GROUPS 32       // first-level arrival groups of the grid barrier
#define SCO_NOALLOC_BYTES (64u << 20)  // static scratch of the entry point that allocates nothing

enum { SCO_TAG_INIT = 1, SCO_TAG_SW = 2, SCO_TAG_TH = 3, SCO_TAG_MC = 4, SCO_TAG_HP = 5, SCO_TAG_HA = 6 };

// spin model of a context: perpendicular Ising spins, or classical Heisenberg spins with
// the full dipolar tensor (open lattices)
enum { SCO_MODEL_ISING = 0, SCO_MODEL_HEIS = 1 };

enum { SCO_FLAG_OVERFLOW = 1, SCO_FLAG_TIMEOUT = 2, SCO_FLAG_PALETTE = 4, SCO_FLAG_STATE = 8, SCO_FLAG_ROUNDS = 16 };

// colouring of step (2): KW with rule (2)' on the union graph; the checkerboard product
// 2 c + ((x + y) mod 2) of a KW colouring c of the bonds alone; basic colour reduction
// with rule (2)' on the whole union graph (no KW groups)
enum { SCO_COLOR_KW = 0, SCO_COLOR_CHECKER = 1, SCO_COLOR_BCR = 2 };

// Immutable per-chain description (device copy written once by sco_init).
struct ChainDesc {
  int32_t L, N, K, periodic;
  int64_t vbase;           // first global site
  const uint32_t* hd;      // packed half-displacements: (uint16)dx | (uint16)dy << 16
  const double* J;         // J(d_m)
  const double* C;         // cumulative sum of J in table order
  const int32_t* guide;    // guide[b] = first m with C_m >= b * C_top / NB, b = 0..NB
  const double* theta;     // survival ratio of a parallel candidate (nullptr when hard)
  const double* delta;     // Vbar(+1) - Vbar(-1) per m (nullptr when hard)
  const float* delta32;    // delta rounded to FP32 (precision 1)
  double C_top, guide_inv; // C_{K-1}, NB / C_top
  double twoJ, beta, inv_rate, neg_beta, inv_L;
  double pacc[9];          // exchange-only flips: index s_v * nn + 4; >= 1 means always accept
  float inv_rate32, neg_beta32, twoJ32;  // FP32 copies (precision 1)
  int32_t twoJ32_exact;                   // 2J is exact in FP32: bond-free fields are exact
  int32_t fp32_gap;                       // precision 1 may decide switching gaps in FP32
  int32_t model;                          // SCO_MODEL_*
  double T;                               // temperature (Heisenberg pseudo-interactions)
  double u_first_end;                     // a first draw's uniform below this ends its owner
                                          // (no candidate and no near tie)
  const double* hden;                     // Heisenberg: expm1(-2 beta J_m) per m (J_m = V^max)
  uint32_t seed, chain_id;
  int32_t hard, precision, n_sw, nguide;
};

// Mutable per-chain state written by the kernels.
struct ChainState {
  int32_t delta_union, q, M, P;  // palette, KW levels, levels run inside one LDS tile
  uint32_t n_edges;              // directed surviving bonds of the last switching
  int32_t delta_sco;             // maximum degree of the switched (bond) graph alone
  unsigned long long accepted, attempts, rechecks, near_ties;
  long long mag;                 // sum of the spins, kept current by the sweeps' flips
  int32_t kw_rounds[SCO_MAXLEVEL];
};

// Per-chain sums over the measured steps of an annealing stage (exact integers).
struct AnnealAcc {
  unsigned long long samples, abs_m, m2, bonds, delta_sco, delta_union;
};

// Device-wide synchronisation words (each counter on its own 128-byte line).
// gen, stop, top and grp are cleared together by the host (barrier counters).
struct SyncWords {
  uint32_t gen, pad0[31];   // barrier instances completed since the counters were cleared
  uint32_t stop, padS[31];  // generation of the last barrier that found a flag raised
  unsigned long long top, pad1[15];
  unsigned long long grp[SCO_BAR_GROUPS * 16];
  uint32_t flags;        // SCO_FLAG_* raised since the host last consumed them
  uint32_t halt;         // 1 once a barrier ended a launch on a raised flag: later launches do nothing
  uint32_t qmax, mmax;
  uint32_t graph_valid;  // 1 once a switching phase completed (0 while one runs)
  uint32_t color_valid;  // 1 once a colouring of the current graph completed
  uint32_t fcount[3];    // frontier sizes of the whole-graph colour reduction (rotating)
  uint32_t pad2[23];
};

// Arguments of the persistent step kernel (all device pointers into the workspace).
struct StepArgs {
  const ChainDesc* cd;
  ChainState* st;
  SyncWords* sync;
  const int32_t* chunk_chain;
  int8_t* spin;
  double* spin3;          // [3 G] Heisenberg spins (x, y, z per site), nullptr for Ising
  int32_t* deg;           // [G] survivors with the site as partner whose owner's block does
                          // not hold the site (zero at every switching: cleared by the
                          // scatter for the next step, by the host at set-up and after a flag)
  int32_t* row_ptr;       // [G + 1]
  int32_t* fill;          // [G] the whole-graph colour reduction's dependence counts
  uint16_t* own;          // [G] survivors with the site as owner, plus those with the site as
                          // partner whose owner's block holds the site (every site written
                          // by the switching; aliases fill, which the colouring alone uses)
  int32_t *ea, *eb, *em;  // survivors: owner, partner (global sites), displacement index
  int32_t* er;            // survivor's rank among its owner's survivors | its place in its
                          // partner's row << 16 (from the front when the owner's block holds
                          // the partner, else from the back) | that case << 31 (as uint32_t)
  int32_t* col;           // [2 * cap] neighbour (global site)
  int32_t* attr;          // [2 * cap] displacement index
  uint16_t* color;        // [G]
  uint32_t* kw_word;      // [G] colouring state: level:5 | round:9 | colour:9
  int4* rec;              // [G] per-block bucket lists: {site, row start, row end, chain}
  uint32_t* ecount;       // [nchunks] survivors of the block whose range starts at the chunk,
                          // stored from that chunk's region on (0 for the block's other chunks)
  long long* scan_agg;    // per-tile sums of the degree scan
  unsigned long long* trace;    // [SCO_TRACE_SLOTS] phase marks of block 0
  int64_t G;
  int32_t nchunks, n_chains;
  uint32_t cap_und;       // undirected survivor capacity (split evenly over the chunks)
  int32_t nsw_override;   // >= 0: sweeps for every chain; < 0: each chain's n_sw
  int32_t nsw_max;
  uint32_t step;
  int32_t tile_limit;     // sites of a KW tile, <= SCO_TILE_MAX (a schedule choice)
  int32_t coloring;       // SCO_COLOR_KW, SCO_COLOR_CHECKER or SCO_COLOR_BCR
  int32_t round_cap;      // KW rounds allowed per level: 0 = the palette size q (Eq. 5)
  int32_t any_fp32;       // some chain decides in FP32 with FP64 recheck (precision 1)
  int32_t fenced_classes; // the sweep's colour classes end with the full (fenced) barrier
};

#define SCO_TRACE_SLOTS 512
#define SCO_MAX_BLOCKS 4096

enum : uint32_t { PH_SWITCH = 1u, PH_COLOR = 2u, PH_SWEEP = 4u };

// Host-side launchers of the kernels (defined next to the kernels).
// An exact transform of one lattice's spins for the pair correlations (host-chosen).
struct NttPlan {
  int32_t n;        // transform length per dimension (0: no plan, the direct kernels run)
  int32_t nrad;     // radices of the Stockham passes, in order
  int32_t rad[24];
  uint32_t p;       // prime, n | p - 1, 2 L^2 + 1 < p < 2^31
  uint32_t pinv;    // -p^-1 mod 2^32
  uint32_t one;     // 2^32 mod p (1 in Montgomery form)
  uint32_t ninv2;   // n^-2 mod p
};

namespace sco_dev {
hipError_t table_j(hipStream_t s, const uint32_t* hd, int K, int L, int periodic, int n_images,
                   double D, double* J);
hipError_t init_spins(hipStream_t s, const ChainDesc* cd, const int32_t* chunk_chain,
                      const int64_t* src_base, const int8_t* src, int8_t* spin, double* spin3, int64_t G);
int step_max_blocks();
hipError_t step(hipStream_t s, const StepArgs& a, uint32_t phases, int blocks, int model);
// The full step kernel of a model, for graph kernel nodes.
const void* step_kernel_full(int model);
const void* step_kernel_for(uint32_t phases, int model);
// Heisenberg observables: prod[m] = sum over owners of the pair energy of displacement
// m; part2[b] = per-block (exchange sum, M_phi sum); out2 = their totals
hipError_t obs_heis(hipStream_t s, const ChainDesc* cd, int chain, const ChainDesc& h, const double* spin3,
                    double* prod, double* part, double* out, double* part2, double* out2, bool dipolar,
                    const NttPlan* fft, double2* fbuf, const double2* ftw);
hipError_t obs_basic(hipStream_t s, const ChainDesc* cd, const int32_t* chunk_chain,
                     const int8_t* spin, const uint16_t* color, unsigned long long* out,
                     unsigned* used, int64_t G);
// st[c].mag = out[2 c] (the spin sums of obs_basic) for every chain
hipError_t set_mag(hipStream_t s, ChainState* st, const unsigned long long* out, int n);
// colour class sizes of one chain into out[256] (added to)
hipError_t class_sizes(hipStream_t s, const uint16_t* color, int64_t vbase, int N, unsigned long long* out);
// surviving bonds per displacement index of one chain into counts[K] (added to)
hipError_t bond_hist(hipStream_t s, const int32_t* row_ptr, const int32_t* col, const int32_t* attr, int64_t vbase,
                     int N, unsigned long long* counts);
// acc[c] += this step's |M|, M^2, directed bonds and maximum degrees
hipError_t anneal_acc(hipStream_t s, const ChainState* st, AnnealAcc* acc, int n);

hipError_t obs_dipolar(hipStream_t s, const uint32_t* hd, const double* J, int K, int L,
                       int periodic, const int8_t* spin, int64_t vbase, uint32_t* bits,
                       double* prod, double* part, double* out, const NttPlan* plan, uint32_t* nbuf,
                       uint32_t* tw);
// Device address of the current GPU's copy of the static scratch array
// (SCO_NOALLOC_BYTES, 256-byte aligned).
hipError_t noalloc_scratch(void** ptr);
}  // namespace sco_dev
