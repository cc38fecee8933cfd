// sco_internal.h -- layouts shared by the host runtime and the gfx950 kernels of libsco.
//
// Global site space: the chains' sites are concatenated, each chain starting at a
// multiple of CHUNK so that a CHUNK-aligned run of global sites belongs to one chain
// (chunk_chain[g / CHUNK]).  Padding sites (local index >= N) are never touched by
// the method.
#pragma once
#include <stdint.h>

#define SCO_CHUNK 256           // sites per chunk; a power of two
#define SCO_CHUNK_SHIFT 8
#define SCO_MAXQ 256            // largest palette (Delta + 1) handled
#define SCO_MAXLEVEL 64         // KW levels are at most ceil(log2(N)) <= 31
#define SCO_GUIDE_BITS 14       // guide table of the cumulative couplings: 2^14 buckets

enum { SCO_TAG_INIT = 1, SCO_TAG_SW = 2, SCO_TAG_TH = 3, SCO_TAG_MC = 4 };

enum { SCO_FLAG_OVERFLOW = 1, SCO_FLAG_TIMEOUT = 2, SCO_FLAG_PALETTE = 4 };

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
  double twoJ, beta, inv_rate, neg_beta;
  double pacc[9];          // exchange-only flips: index s_v * nn + 4; >= 1 means always accept
  uint32_t seed, chain_id;
  int32_t hard, precision, n_sw, nguide;
};

// Mutable per-chain state written by the kernels.
struct ChainState {
  int32_t delta_union, q, M, colors_used;
  uint32_t n_edges;        // undirected surviving bonds of the last switching
  int32_t pad0;
  unsigned long long accepted, attempts, rechecks, near_ties;
  int32_t kw_rounds[SCO_MAXLEVEL];
};

// Device-wide barrier words and flags.
struct SyncWords {
  uint32_t bar_count, bar_gen, flags, edge_count;
  uint32_t qmax, mmax, pad[2];
};

// Arguments of the persistent step kernel (all device pointers into the workspace).
struct StepArgs {
  const ChainDesc* cd;
  ChainState* st;
  SyncWords* sync;
  const int32_t* chunk_chain;
  int8_t* spin;
  int32_t* deg;      // [G] degree, then the exclusive scan is written to row_ptr
  int32_t* row_ptr;  // [G + 1]
  int32_t* fill;     // [G] scatter cursors
  int32_t *ea, *eb, *em;  // survivors: owner, partner (global sites), displacement index
  int32_t* col;      // [2 * cap] neighbour (global site)
  int32_t* attr;     // [2 * cap] displacement index
  uint16_t* color;   // [G]
  uint16_t* rho;     // [G] KW decision round of the current level
  int32_t* g0;       // [G] level-0 group v / q
  int32_t* plist;    // [G] per-block pending lists
  int32_t* perm;     // [G] sites bucketed by colour (colour-major over all chains)
  int32_t* hist;     // [SCO_MAXQ * nchunks + 1] colour histogram, scanned in place
  int32_t* part;     // scan tile partials
  int64_t G;
  int32_t nchunks, n_chains;
  uint32_t cap_und;  // undirected survivor capacity
  int32_t nsw_override;  // >= 0: sweeps for every chain; < 0: each chain's n_sw
  int32_t nsw_max;
  uint32_t step;
};

enum : uint32_t { PH_SWITCH = 1u, PH_COLOR = 2u, PH_SWEEP = 4u };

#include <hip/hip_runtime_api.h>

// Host-side launchers of the kernels (defined next to the kernels).
namespace sco_dev {
hipError_t table_j(hipStream_t s, const uint32_t* hd, int K, int L, int periodic, int n_images,
                   double D, double* J);
hipError_t init_spins(hipStream_t s, const ChainDesc* cd, const int32_t* chunk_chain,
                      const int64_t* src_base, const int8_t* src, int8_t* spin, int64_t G);
int step_max_blocks();
hipError_t step(hipStream_t s, const StepArgs& a, uint32_t phases, int blocks);
hipError_t obs_basic(hipStream_t s, const ChainDesc* cd, const int32_t* chunk_chain,
                     const int8_t* spin, unsigned long long* out, int64_t G);
hipError_t obs_dipolar(hipStream_t s, const uint32_t* hd, const double* J, int K, int L,
                       int periodic, const int8_t* spin, int64_t vbase, uint32_t* bits,
                       double* prod, double* part, double* out);
}  // namespace sco_dev
