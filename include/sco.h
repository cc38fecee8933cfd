/*
 * sco.h -- C-ABI of libsco, the MI355X (gfx950) stochastic-cutoff Monte-Carlo step.
 *
 * Method: Endo, Toga & Sasaki, "Parallelized Stochastic Cutoff Method for
 * Long-Range Interacting Systems".  One SCO step of a chain is
 *   (1) switching of every dipolar bond to 0 or to its pseudo-interaction
 *       (Sec. 2.1, Eqs. 1-3; Fig. 1 step (1)),
 *   (2) Kuhn-Wattenhofer colouring of the graph of surviving bonds united with
 *       the never-switched nearest-neighbour exchange bonds (Sec. 2.3, Eq. 5;
 *       Fig. 1 step (2)),
 *   (3) n_sw Metropolis sweeps of the switched Hamiltonian H' (Eq. 4), one
 *       colour class at a time (Fig. 1 step (3)).
 * Two models of Eq. (6):
 *   - Ising spins perpendicular to the plane (model 0):
 *       H = -J sum_<ij> s_i s_j + sum_{i<j} J_ij s_i s_j,  s_i = +-1,
 *     with J_ij = D / r_ij^3 on an open L x L lattice, or J_ij summed over the
 *     periodic images |n_x|, |n_y| <= n_images of a periodic one;
 *   - classical Heisenberg spins (model 1, open lattices, the paper's Sec. 3.1):
 *       H = -J sum_<ij> S_i . S_j + D sum_{i<j} [S_i . S_j / r^3 - 3 (S_i . r)(S_j . r) / r^5],
 *     switched with the pair bound V^max = 2 D / r^3 (the largest eigenvalue magnitude
 *     of the dipolar tensor); proposals uniform on the sphere.
 *
 * Conventions shared by every call
 *   - All device memory belongs to the caller: one workspace of
 *     sco_workspace_size() bytes (256-byte aligned) handed to sco_init.  The
 *     library never allocates device memory after sco_init and never frees the
 *     caller's memory.  sco_init allocates a small pinned host staging buffer.
 *   - Every call is ordered on the HIP stream given to sco_init (`stream` is a
 *     hipStream_t passed as void*; NULL is the default stream).  Only
 *     sco_observables, sco_get_* , sco_set_spins and sco_init synchronise it.
 *   - A context is used by one host thread at a time.  Several contexts may
 *     coexist; they share nothing.
 *   - Return value: SCO_OK (0) or a negative SCO_E* code; sco_strerror() names it.
 *     Device-side conditions (edge capacity exceeded, a bounded wait that timed
 *     out, palette overflow, a broken graph state) are raised as flags.  The launch
 *     that raises one ends at its next device-wide barrier, before its step moves any
 *     spin, and later launches do nothing until the next synchronising call reports
 *     the flag (SCO_EOVERFLOW, SCO_ETIMEOUT, SCO_EPALETTE, SCO_EINTERNAL) and clears it.
 *   - Sites are numbered row-major, v = y * L + x; spins are int8 +1 / -1.
 *   - Randomness: Philox4x32-10 (Salmon et al., SC'11), key (seed, chain_id),
 *     counter (step, site, draw, tag).  A chain is a pure function of its
 *     parameters, its initial spins and the step indices it was given.
 */
#ifndef SCO_H
#define SCO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCO_OK 0
#define SCO_EINVAL (-1)    /* invalid argument or parameter */
#define SCO_EHIP (-2)      /* a HIP runtime call failed */
#define SCO_EOVERFLOW (-3) /* surviving bonds exceeded the edge capacity: the step is invalid */
#define SCO_EINTERNAL (-4) /* an invariant failed: a colouring or sweep launched without a valid
                              bond graph, a CSR row outside the edge arrays, a KW level above its
                              round cap, or a check of sco_validate */
#define SCO_ENOSPC (-5)    /* the workspace is smaller than sco_workspace_size() */
#define SCO_ETIMEOUT (-6)  /* a bounded device wait ran out (the persistent kernel's blocks were
                              not all resident); the chain state is that before the failed step */
#define SCO_EPALETTE (-7)  /* the union graph needs more than 255 colours (Delta + 1 > 255) */

/* Parameters of one Markov chain. */
typedef struct {
  int32_t L;          /* linear size; periodic lattices need even L >= 4, open L >= 2 */
  int32_t periodic;   /* 1: periodic boundaries with image-summed couplings; 0: open */
  int32_t n_images;   /* periodic image box half-width (8 in the reference workloads) */
  int32_t n_sw;       /* Metropolis sweeps per SCO step (Sec. 2.1 step (B)); >= 0 */
  double J;           /* nearest-neighbour exchange constant (> 0 ferromagnetic) */
  double D;           /* dipolar constant, J_ij = D / r^3 */
  double T;           /* temperature, beta = 1 / T; > 0 */
  double kappa;       /* V^max = kappa * J_ij (Eq. 2 needs V^max >= max V); >= 1 */
  uint32_t seed;      /* Philox key word 0 */
  uint32_t chain_id;  /* Philox key word 1 */
  int32_t precision;  /* 0: FP64 decisions; 1: FP32 accumulation + FP64 recheck (same chain) */
  int32_t edge_factor;/* directed-bond capacity per site, 0 .. 256 (0: default 4) */
  int32_t model;      /* 0: perpendicular Ising; 1: Heisenberg (open, kappa 1, precision 0);
                         every chain of a context has the same model */
  int32_t pad;
} sco_chain_params;

/* Per-chain observables and counters, FP64 / exact integers. */
typedef struct {
  double E;           /* full Hamiltonian of the current spins */
  double E_exchange;  /* -J sum_<ij> s_i s_j (an exact integer times J) */
  double E_dipolar;   /* sum_{i<j} J_ij s_i s_j */
  int64_t M;          /* sum_i s_i */
  int64_t n_edges;    /* surviving bonds of the last switching (undirected) */
  int32_t delta_union;/* maximum degree of the union graph coloured last */
  int32_t q;          /* palette size delta_union + 1 */
  int32_t colors_used;/* colours holding at least one site */
  int32_t kw_levels;  /* KW levels M = ceil(log2(ceil(N / q))) */
  int64_t kw_rounds;  /* synchronous rounds of rule (2)' summed over the levels */
  int64_t accepted;   /* accepted flips since sco_init (or the last counter reset) */
  int64_t attempts;   /* Metropolis trials since sco_init */
  int64_t rechecks;   /* FP32 decisions recomputed in FP64 (precision 1) */
  int64_t flags;      /* device flags seen since the last counter reset: bit 0 edge
                         overflow, bit 1 wait timeout, bit 2 palette overflow,
                         bit 3 colouring or sweep launched without a valid graph,
                         bit 4 a KW level above its round cap */
  int64_t near_ties;  /* decisions whose two compared FP64 numbers lay within 1e-12 of each
                         other: switching targets within 1e-12 relative of C_top or of a
                         bracketing cumulative coupling, Metropolis draws |u - p| < 1e-12
                         (the only decisions a host evaluation may take differently) */
  int32_t delta_sco;  /* maximum degree of the switched graph alone (Table 1's Delta) */
  int32_t pad;
  double m_phi;       /* Heisenberg: Eq. (7) before its thermal average and modulus,
                         (1/N) sum_i [S_i x (r_i - r_c) / |r_i - r_c|]_z with r_c the centre
                         ((L-1)/2, (L-1)/2); 0 for Ising.  (Heisenberg: M = 0, E_exchange =
                         -J sum S_i . S_j over lattice pairs.) */
} sco_obs;

/* Statistics of one chain over one stage of an annealing schedule (sco_anneal). */
typedef struct {
  double T;                /* the stage's temperature */
  double E;                /* full energy at the end of the stage */
  int64_t M;               /* magnetisation at the end of the stage */
  int64_t samples;         /* measured steps of the stage */
  double abs_m, m2;        /* <|M|> / N and <M^2> / N^2 over the measured steps */
  double k_mean;           /* <2 n_edges / N>: mean degree of the switched graph (Table 1's <k>) */
  double delta_sco_mean;   /* mean of its maximum degree (Table 1's <Delta>) */
  double delta_union_mean; /* mean maximum degree of the coloured union graph */
  double acceptance;       /* accepted / attempted flips over the whole stage */
  double m_phi;            /* Heisenberg: M_phi of Eq. (7) (before the modulus) at the end of the
                              stage; abs_m and m2 are 0 for Heisenberg chains */
} sco_stage;

typedef struct sco_ctx sco_ctx;

/* Bytes of device workspace needed for n_chains chains (host-only computation).
 * Returns SCO_EINVAL on invalid parameters. */
int sco_workspace_size(const sco_chain_params* params, int n_chains, size_t* bytes);

/* Creates a context over the caller's workspace.  Builds, per distinct lattice,
 * the half-displacement table sorted by (r^2, dy, dx), the couplings J(d)
 * (image sums on the GPU), the cumulative couplings and, per chain, the switching
 * and pseudo-interaction columns (Eqs. 2-3); then the initial spins: copied from
 * dev_init_spins (int8, the chains' sites concatenated in chain order, may be
 * NULL) or drawn from Philox.  Synchronises `stream`. */
int sco_init(sco_ctx** out, const sco_chain_params* params, int n_chains, void* dev_workspace,
             size_t workspace_bytes, const int8_t* dev_init_spins, void* stream);

/* Step (1) for every chain: switch all dipolar bonds for SCO step `step` and
 * assemble the symmetric CSR of the survivors (rows ascending by neighbour). */
int sco_switch(sco_ctx* ctx, uint64_t step);

/* Step (2): KW colouring of the union graph, then bucketing of the sites by colour. */
int sco_color(sco_ctx* ctx);

/* Step (3): n_sw colour-ordered Metropolis sweeps with the RNG counters of `step`. */
int sco_sweep(sco_ctx* ctx, uint64_t step, int n_sw);

/* Steps (1)-(3) with each chain's own n_sw. */
int sco_step(sco_ctx* ctx, uint64_t step);

/* Runs steps first_step .. first_step + n_steps - 1 back to back, then synchronises
 * and reports any device flag raised by them (a step that raises one ends at its next
 * device-wide barrier and the launches after it do nothing, so the spins are those
 * before the failed step). */
int sco_run(sco_ctx* ctx, uint64_t first_step, int n_steps);

/* How sco_step, sco_run and sco_run_graph launch a step (Sec. 2.1 steps (A)-(C)):
 * 0 (the default) the switching, colouring and sweep kernels one after another,
 * 1 one launch of the fused kernel.  Same results; the three launches are faster
 * (each phase kernel holds only its own registers, and the launch boundaries replace
 * two device-wide barriers), and sco_phase_times then times the last step's phases.
 * SCO_EINVAL for other values. */
int sco_set_step_form(sco_ctx* ctx, int fused);

/* For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid allocation): sco_init + sco_run + sco_get_spins
 * (+ sco_observables) of n_chains chains in one call that allocates nothing.  Their
 * whole workspace lives in a static device array of the library, 64 MiB per GPU
 * (held from the library's first use on that GPU until the process ends), so
 * sco_workspace_size(params) must be at most 64 MiB (L up to about 512 periodic),
 * else SCO_ENOSPC and nothing runs.
 *   dev_spins_in   int8 +-1, the chains' sites concatenated in chain order (row-major,
 *                  no padding); NULL draws the initial spins from Philox
 *   dev_spins_out  the spins after steps first_step .. first_step + n_steps - 1, same
 *                  layout (may equal dev_spins_in)
 *   host_obs       NULL, or n_chains observables after the steps
 * Ising chains only (SCO_EINVAL for Heisenberg parameters).
 * Returns SCO_OK or an error code as sco_init / sco_run; synchronises `stream`.  Every
 * call on one GPU uses that GPU's one array and re-initialises it: calls that overlap
 * on one GPU (other host threads, other streams) race and must be serialised by the
 * caller. */
int sco_run_noalloc(const sco_chain_params* params, int n_chains, const int8_t* dev_spins_in,
                    int8_t* dev_spins_out, uint64_t first_step, int n_steps, sco_obs* host_obs,
                    void* stream);

/* sco_run as one replay of a HIP graph: the steps' cooperative kernel launches (three
 * per step in the default step form, one in the fused form), each node depending on
 * the one before.  The graph is built on the first call
 * with this n_steps (and schedule) and kept in the context; later calls rewrite the
 * nodes' step indices and replay it.  The graph holds kernel nodes only.  Same results
 * as sco_run; synchronises and reports the steps' flags. */
int sco_run_graph(sco_ctx* ctx, uint64_t first_step, int n_steps);

/* Sets the temperature of one chain (chain = -1: every chain) for the steps that follow:
 * beta, the bound rate (kappa + 1) beta J_m of the switching, the survival ratio and the
 * pseudo-interactions of Eqs. (2)-(3) and the exchange-only acceptance are rebuilt
 * (O(K) host work per chain).  Synchronises.  SCO_EINVAL for T <= 0 or not finite. */
int sco_set_temperature(sco_ctx* ctx, int chain, double T);

/* Annealing driver (the cooling protocol of Sec. 3.1): for each stage k = 0 .. n_stages-1,
 * every chain c is set to temperature temps[k * n_chains + c], runs equil_steps SCO
 * steps, then meas_steps steps whose magnetisation and graph statistics are summed
 * exactly on the device; out[k * n_chains + c] receives the stage's statistics.  Stage k
 * uses the step indices first_step + k (equil_steps + meas_steps) onwards, so the run
 * equals sco_set_temperature + sco_run stage by stage.  Synchronises after each stage. */
int sco_anneal(sco_ctx* ctx, const double* temps, int n_stages, int equil_steps, int meas_steps,
               uint64_t first_step, sco_stage* out);

/* Graph statistics of one chain (Sec. 3.2-3.3), synchronising:
 *   sco_class_sizes      sites per colour of the current colouring into sizes[256]
 *                        (the per-class work whose imbalance Eq. (9) measures); *n_colors
 *                        receives 1 + the largest colour in use;
 *   sco_bond_histogram   surviving bonds of the last switching per half-displacement
 *                        index, counts[K] (K of sco_get_tables);
 *   sco_survival_by_distance
 *                        P_survive(r) of Fig. 5: surviving bonds over owned pairs for each
 *                        distance r of the table (ascending), into r[], p_survive[] (up to
 *                        max entries; *n receives the number of distances).
 * SCO_EINVAL when there is no graph (colouring) yet. */
int sco_class_sizes(sco_ctx* ctx, int chain, int64_t* sizes, int* n_colors);
int sco_bond_histogram(sco_ctx* ctx, int chain, int64_t* counts);
int sco_survival_by_distance(sco_ctx* ctx, int chain, double* r, double* p_survive, int max, int* n);

/* Barrier between the colour classes of an Ising sweep (Fig. 1 step (3): a class reads
 * the spins the classes before it wrote).  0 (the default): a light barrier that orders
 * only the control; the spins are read and written with agent-scope atomics, each by
 * the one block owning its site, and each wave's stores complete before its block
 * arrives, with no cache write-back or invalidation.  1: the full barrier with the
 * agent-scope release/acquire fences of the documented memory model after every class
 * (slower: the L2 write-back and invalidation run per class).  Same results either way.
 * Takes effect at the next launch; SCO_EINVAL for other values. */
int sco_set_fenced_sweeps(sco_ctx* ctx, int on);

/* Cap on the synchronous rounds of one KW level (Eq. 5 bounds them by q = Delta + 1):
 * 0 (the default) checks that bound on every level; a positive cap checks that instead
 * (a cap below q is a fault injection).  A level above it raises a flag that the next
 * synchronising call reports as SCO_EINTERNAL (flag bit 4). */
int sco_set_round_cap(sco_ctx* ctx, int cap);

/* Host check of one chain's invariants (reads the state back; synchronises): bit 0 a
 * spin not +-1 (Heisenberg: not a finite unit vector), bit 1 the tracked magnetisation
 * differs from the sum of the spins, bit 2 CSR row offsets out of order or range, bit 3
 * a row not strictly ascending or with a self or foreign bond, bit 4 a bond without its
 * reverse (same displacement index), bit 5 a colouring that is not proper on the union
 * graph or a colour outside the palette.  *failed receives the bits; SCO_EINTERNAL when
 * any is set. */
int sco_validate(sco_ctx* ctx, int chain, int64_t* failed);

/* Device flags (SCO_FLAG bits as in sco_obs.flags) of the last flagged launch that a
 * synchronising call consumed, and all flags seen since the last counter reset. */
int sco_get_flags(sco_ctx* ctx, int64_t* last, int64_t* seen);

/* Observables of every chain into host_out[n_chains]; synchronises.  E_exchange and M
 * follow Eq. (6) restricted to perpendicular spins; E_dipolar = sum_m J_m C_m with the
 * exact integer pair correlation C_m of each half-displacement, from a number-theoretic
 * transform of the spins (O(N log N); lattice sizes with a prime factor above 7 take a
 * direct O(N K / 32) count); Heisenberg chains: E_exchange, E_dipolar (the full tensor
 * of Eq. 6: direct pair sums while N K <= 2e9, above that FP64 FFT correlations of the
 * spin components, O(N log N)) and m_phi of Eq. (7).  n_edges, delta_union, q and the colours are
 * the graph statistics of Sec. 3.2 (mean degree 2 n_edges / N) for the last switching
 * and colouring. */
int sco_observables(sco_ctx* ctx, sco_obs* host_out);

/* The same without the dipolar energy (E and E_dipolar are NaN): integer observables,
 * graph statistics and counters only, in O(N).  Synchronises. */
int sco_counters(sco_ctx* ctx, sco_obs* host_out);

/* Checkpoint / resume: spins of one chain (N int8 values) to / from host memory
 * (Ising contexts; SCO_EINVAL for Heisenberg). */
int sco_get_spins(sco_ctx* ctx, int chain, int8_t* host_out);
int sco_set_spins(sco_ctx* ctx, int chain, const int8_t* host_in);

/* The same for Heisenberg spins: 3 N doubles, (x, y, z) per site, row-major sites
 * (SCO_EINVAL for Ising contexts or a non-finite component). */
int sco_get_spins3(sco_ctx* ctx, int chain, double* host_out);
int sco_set_spins3(sco_ctx* ctx, int chain, const double* host_in);

/* The last switched graph of one chain, in site numbers local to the chain:
 * row_ptr[N+1], col[n_dir], attr[n_dir] (half-displacement index of the bond),
 * colors[N]; any pointer may be NULL; *n_dir receives 2 * n_edges. */
int sco_get_graph(sco_ctx* ctx, int chain, int32_t* row_ptr, int32_t* col, int32_t* attr,
                  int32_t* colors, int64_t* n_dir);

/* The displacement table of one chain: K entries of dx, dy, J, C (cumulative J),
 * theta (survival ratio of a parallel candidate) and delta (Vbar(+1) - Vbar(-1));
 * any pointer may be NULL; *K receives the table length. */
int sco_get_tables(sco_ctx* ctx, int chain, int32_t* K, int32_t* dx, int32_t* dy, double* J,
                   double* C, double* theta, double* delta);

/* Device time of the phases, in ms: of the last sco_switch, sco_color and sco_sweep
 * calls, or of the last step of sco_step / sco_run in the three-launch form.
 * out[0] switching + assembly, out[1] colouring, out[2] sweeps (events on the stream). */
int sco_phase_times(sco_ctx* ctx, float* out3);

/* Phase trace of the persistent step kernel: while enabled, block 0 records a mark
 * (an id and the wall clock) at each phase boundary of every launch.  sco_trace_read
 * returns the marks of the last launch (ids, microseconds since its first mark) and
 * their count in *n; it synchronises.  Ids: 1-6 switching (draws, scan, scatter,
 * row sort), 10-13 colouring (30 bonds of block 0's first tile staged, 60+p and
 * 80+p its tile level p counted and bucketed, 40+p that level done, 200+p global
 * level p bucketed, 100+p global level p done),
 * 20-22 sweeps (1000+k colour class k).  Diagnostic only; costs a small copy per
 * launch. */
int sco_trace(sco_ctx* ctx, int enable);
int sco_trace_read(sco_ctx* ctx, int32_t* ids, double* us, int max, int* n);

/* Schedule of the persistent step kernel: the number of co-resident blocks of its
 * cooperative launch and the largest KW tile (sites) whose levels run in LDS.
 * Neither changes any result: every chain is a function of its parameters, spins and
 * step indices only.  sco_set_schedule: 0 selects the default (all co-resident
 * blocks, 28672-site tiles); blocks must be 1 .. that limit and tile_limit 64 .. 28672,
 * else SCO_EINVAL. */
int sco_set_schedule(sco_ctx* ctx, int blocks, int tile_limit);

/* Colouring of step (2) for the steps that follow (every chain of the context; each
 * colouring changes the sweep order and so the chain, and the oracle takes the same
 * mode):
 *   0  Kuhn-Wattenhofer colour reduction of the union graph, rule (2)' in every level
 *      (Sec. 2.3.2-2.3.3; the default);
 *   1  the checkerboard product 2 c + ((x + y) mod 2), c a KW colouring of the bonds
 *      alone with q = max(Delta_bonds + 1, 2) (2 q colours; SCO_EPALETTE above 128);
 *   2  basic colour reduction with rule (2)' on the whole union graph, without KW groups
 *      (Sec. 2.3.2): first-fit in decreasing site order, one round per level of the
 *      increasing-index dependence (kw_levels 1, kw_rounds the rounds).
 * Rule (2) in place of (2)' gives the same colours in (Delta + 1) M rounds (Eq. 5), or
 * N - Delta - 1 without KW.  SCO_EINVAL for another mode. */
int sco_set_coloring(sco_ctx* ctx, int mode);
int sco_get_schedule(sco_ctx* ctx, int* blocks, int* tile_limit);

/* Autotuner: times trial_steps (1 .. 1000) full steps for each candidate schedule
 * (grid sizes of 1, 3/4 and 1/2 of the co-resident limit x tile limits 28672, 14336,
 * 7168), starting every trial from the chain's current spins, and keeps the fastest.
 * Afterwards the spins and counters are those from before the call; the bond graph
 * is not, so the next call that needs one must be sco_switch, sco_step or sco_run.
 * The chosen schedule and its time per step are returned through the non-NULL
 * pointers.  Synchronises. */
int sco_autotune(sco_ctx* ctx, int trial_steps, int* blocks, int* tile_limit, float* ms_per_step);

/* Sets counters (accepted, attempts, rechecks, flags) of every chain to zero. */
int sco_reset_counters(sco_ctx* ctx);

int sco_destroy(sco_ctx* ctx);
const char* sco_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* SCO_H */
