/*
 * fciqmc.h -- C ABI of the MI355X FCIQMC library (libfciqmc.so).
 *
 * One imaginary-time step of Full Configuration Interaction Quantum Monte
 * Carlo (Guther et al., J. Chem. Phys. 153, 034107 (2020), "NECI"):
 * the projector of Eq. (projector), psi(tau+dtau) = (1 - dtau (H - S)) psi(tau),
 * applied stochastically as the spawn / death / annihilation split of
 * Eq. (fciqmc_dyn), with the initiator rule (Sec. I), the shift S and the
 * reference-projected energy of Eq. (proje) (Sec. IV).
 *
 * Conventions used throughout this header:
 *   - N spatial orbitals, n_alpha + n_beta electrons, 2N spin orbitals;
 *     a determinant is handed over as two uint64 spatial-orbital masks,
 *     alpha first then beta (bit p set = orbital p occupied).
 *   - Integrals are FP64 in chemists' notation: h1 is N*N row-major and
 *     symmetric; (pq|rs) is 8-fold packed with P = p(p+1)/2 + q (p >= q) and
 *     element index P(P+1)/2 + Q (P >= Q).
 *   - Every entry point returns 0 on success or a negative FCIQMC_E* code;
 *     fciqmc_last_error() then describes the failure.  No C++ exception
 *     crosses this boundary.
 *   - Pointers marked "host" are read or written by the call and may be
 *     reused by the caller as soon as it returns.  All device memory is
 *     allocated and owned by the library and released by the free calls.
 *   - A run borrows its system: free every run before its system.  Calls on
 *     one run are serialised by the caller; different runs may be stepped
 *     from different host threads on different streams.
 */
#ifndef FCIQMC_H
#define FCIQMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FCIQMC_OK 0
#define FCIQMC_EINVAL (-1)    /* invalid argument or inconsistent input       */
#define FCIQMC_ENOMEM (-2)    /* device allocation failed or over HBM budget  */
#define FCIQMC_EOVERFLOW (-3) /* capacity could not grow; state is unchanged  */
#define FCIQMC_EDEVICE (-4)   /* HIP runtime error                            */
#define FCIQMC_ESTATE (-5)    /* call out of order, or the run is unusable:   */
                              /* a call that failed with ENOMEM after         */
                              /* releasing buffers it had to regrow leaves    */
                              /* the run without its population; every later  */
                              /* step, batch step, pair step or walker access  */
                              /* on it returns ESTATE (free it)               */

#define FCIQMC_MODE_INTEGER 0 /* signed integer walker numbers                */
#define FCIQMC_MODE_REAL 1    /* real coefficients compressed at c_min        */

#define FCIQMC_GEN_UNIFORM 0  /* uniform singles and doubles (Appendix A.1)   */
#define FCIQMC_GEN_LATTICE 1  /* real-space lattice hopping (Sec. II)         */
#define FCIQMC_GEN_PCHB 2     /* pre-computed heat-bath doubles (App. A.3)    */
/* On-the-fly generators of Appendix A.2 (no tables beyond N x N):
 * weighted singles (hole drawn with weight |H|), electron pair from a uniform
 * first electron and a CPF over |(ii|kk)| biased by p_opp, holes from CPFs
 * over sqrt((ia|ia)) and, for the second hole, either the Cauchy-Schwarz
 * bound (CS) or the exact sqrt(|<ij||ab>|) (Part-Exact).  O(nN) work per
 * draw. */
#define FCIQMC_GEN_CS 3       /* Cauchy-Schwarz (App. A.2)                    */
#define FCIQMC_GEN_PE 4       /* Part-Exact refinement of CS (App. A.2)       */

typedef struct fciqmc_system fciqmc_system;
typedef struct fciqmc_run fciqmc_run;
typedef struct fciqmc_batch fciqmc_batch;
typedef struct fciqmc_server fciqmc_server;
typedef struct fciqmc_pair fciqmc_pair;

/* Parameters of one walker population.  fciqmc_params_default() fills every
 * field; callers then override what they need. */
typedef struct fciqmc_params {
    double tau;             /* time step dtau; must satisfy dtau < 2/W (Sec. I)           */
    double walker_target;   /* N_w at which the shift starts to vary                      */
    double n_initial;       /* walkers placed on the reference determinant at init        */
    double initiator_na;    /* initiator threshold n_a (|C_i| > n_a); < 0 switches it off */
    int mode;               /* FCIQMC_MODE_*                                              */
    double c_min;           /* real mode: compression threshold C_min (Sec. I)           */
    int excitgen;           /* FCIQMC_GEN_*                                               */
    double p_single;        /* probability of a single excitation; < 0: nN/(nN + n^2N^2)  */
    double p_opp;           /* PCHB: prob. of an opposite-spin pair; CS/PE: weight factor */
                            /* of opposite-spin pairs (1 - p_opp for equal spins);       */
                            /* < 0: n_a n_b/C(n,2)                                       */
    uint64_t seed;          /* Philox key word 0                                          */
    uint64_t replica_id;    /* Philox key word 1                                          */
    double shift_damping;   /* zeta of the shift update                                   */
    double shift_restore;   /* xi: pull of S towards the target N_w; < 0: zeta^2/4        */
    int shift_interval;     /* A: steps between shift updates                             */
    uint64_t ref_alpha;     /* reference determinant masks; both 0 = aufbau               */
    uint64_t ref_beta;
    int64_t max_dets;       /* capacity hint for occupied determinants (0 = from target)  */
    int64_t max_spawns;     /* capacity hint for spawn records per step (0 = from target) */
    int64_t hbm_budget_bytes; /* device memory this run may hold (0 = no limit)           */
    int buckets_log2;       /* hash-partition count 2^k of the walker store (0 = auto: from
                               the target, doubled whenever a step leaves more than 600
                               occupied determinants per bucket on average; k > 0 fixes it
                               except where a bucket overflows)                             */
    int det_words;          /* 1 (N <= 32) or 2 (N <= 63) uint64 per determinant; 0 auto  */
    double conv_tol;        /* energy agreement tolerance for the report (Hartree)        */
    int equil_steps;        /* steps after the shift starts varying that the report drops */
    int adaptive_shift;     /* 1: non-initiators die with the local shift f_i S of
                               Sec. "Adaptive Shift" (f_i: accepted share of the weights
                               |H_ij|/|H_jj - E_0| of their spawns this step, E_0 the shift;
                               f_i = 1 without spawns); runs with it step alone (no
                               batch) and take no deterministic space                      */
    int ref_rechoose;       /* 1: ceil(1/tau) steps after the shift starts varying, the most
                               populated determinant (ties: ascending alpha, then beta)
                               becomes the reference of the projected energy (Sec. IV: an
                               appropriate reference determinant) and the determinant that
                               always counts as an initiator, for the following steps (the
                               energy report uses only those); H_00 of ref_alpha/ref_beta
                               stays the energy zero of the diagonal and the shift.  Not with
                               replica pairs (EINVAL at fciqmc_pair_create)                   */
} fciqmc_params;

/* Per-step diagnostics (after the step). */
typedef struct fciqmc_step_stats {
    int64_t iter;           /* number of completed steps                                  */
    double nw;              /* walker number N_w = sum |C_i|                              */
    double nref;            /* C_ref, the reference coefficient                           */
    double enum_;           /* sum_{j != P} H_Pj C_j (P: see e_proj)                      */
    double shift;           /* S after this step's update (relative to H_00)              */
    double e_proj;          /* H_PP + e_core + enum_/nref (absolute; P the reference of the
                               projected energy, the initial reference unless re-chosen)   */
    int64_t ndets;          /* occupied determinants                                      */
    int64_t attempts;       /* spawn attempts made in this step                           */
    int64_t spawns;         /* spawn records emitted in this step                         */
    int vary_shift;         /* 1 once the shift varies                                    */
    int retries;            /* capacity growths this step needed (trajectory unchanged)   */
} fciqmc_step_stats;

/* Energy report from the recorded steps (Flyvbjerg-Petersen blocking). */
typedef struct fciqmc_energy_report {
    double e_proj, e_proj_err;   /* absolute projected energy and its error            */
    double shift, shift_err;     /* absolute shift H_00 + e_core + <S> and its error   */
    double e_ref;                /* H_00 + e_core                                      */
    int64_t n_samples;           /* steps used                                         */
    int64_t first_step;          /* first step used                                    */
    int64_t steps_done;          /* all completed steps                                */
    int converged;               /* |shift - e_proj| < conv_tol and both errors < tol  */
} fciqmc_energy_report;

/* Walker-state scalars that, with the walker list, form a full checkpoint. */
typedef struct fciqmc_checkpoint {
    int64_t iter;
    double shift;
    int vary_shift;
    int64_t last_update_iter;
    double last_update_nw;
} fciqmc_checkpoint;

void fciqmc_params_default(fciqmc_params *p);

/* Load integrals (Sec. XIV, "Interfacing NECI": the method consumes one- and
 * two-electron integrals).  h1: host, n_orb*n_orb; eri_packed: host,
 * eri_len = M(M+1)/2 with M = n_orb(n_orb+1)/2.  Copies both to the device
 * and derives the tables the generators need.  EINVAL if h1 is not
 * symmetric, lengths disagree, n_orb > 63, n_alpha or n_beta > n_orb, or the
 * determinant space holds a single determinant. */
int fciqmc_load_integrals(int n_orb, int n_alpha, int n_beta, double e_core,
                          const double *h1, const double *eri_packed, int64_t eri_len,
                          fciqmc_system **out);

/* Create a walker population: n_initial walkers on the reference (the
 * starting determinant fixes the m_s sector of the walk, Sec. "Symmetries
 * and spin-adapted FCIQMC"; Reading: the paper gives no initial state
 * beyond that, so the reference carries the first walkers and the
 * population grows until the shift controls it, Sec. I).  stream: a
 * hipStream_t to launch on (e.g.
 * torch.cuda.current_stream().cuda_stream), NULL for a library-owned stream.
 * Builds PCHB tables on first use.  EINVAL for a non-positive tau or
 * n_initial, an unknown mode or generator, a reference that is not a
 * determinant of the system, a lattice generator on a system with
 * off-site two-electron integrals, or a layout too narrow for n_orb;
 * ENOMEM if the initial store does not fit hbm_budget_bytes. */
int fciqmc_init(const fciqmc_system *sys, const fciqmc_params *p, void *stream,
                fciqmc_run **out);

/* Advance n_steps imaginary-time steps (Eq. fciqmc_dyn: spawn, death,
 * annihilation with the initiator rule, Sec. I; then estimators and shift).  stats:
 * host array of n_steps entries or NULL.  Capacity overflows grow the
 * buffers and replay the step, which reproduces it exactly. */
int fciqmc_step(fciqmc_run *run, int n_steps, fciqmc_step_stats *stats);

/* Energies from the recorded per-step estimators (host only): the shift
 * (Sec. I) and the projected energy of Eq. (proje) (Sec. IV) as a ratio of
 * means over the steps after the shift started varying, less an
 * equilibration of max(equil_steps or ceil(1/tau), 20 % of them).  Reading:
 * the paper prints results with error bars without the analysis; errors
 * are Flyvbjerg-Petersen blocking estimates (delta method for the ratio),
 * taken at the plateau of the blocking curve. */
int fciqmc_energy(const fciqmc_run *run, fciqmc_energy_report *out);

/* Diagnostics / checkpoint.  dets: host, 2 uint64 per determinant (alpha,
 * beta masks); vals: host.  get: at most cap entries, *n receives the count
 * (ENOMEM-free: returns EOVERFLOW with *n set when cap is too small). */
int fciqmc_get_walkers(const fciqmc_run *run, uint64_t *dets, double *vals, int64_t cap,
                       int64_t *n);
/* Replace the population (values must be non-zero; integer mode: integers).
 * Drops the deterministic space, if any. */
int fciqmc_set_walkers(fciqmc_run *run, const uint64_t *dets, const double *vals, int64_t n);

/* Semi-stochastic projection (Sec. "Semi-stochastic FCIQMC"): make the
 * n_core determinants of largest |C| in the current population (ties:
 * ascending alpha, then beta mask) the deterministic space D.  From the
 * next step on, the projector's elements between determinants of D are
 * applied exactly (a sparse product with H^D, built here on the device from
 * removal keys: two determinants are connected exactly when taking one or
 * two electrons out of each leaves the same strings, so pairs are found by
 * hashing those keys, in time linear in |D|) and only the rest is sampled
 * (the paper builds H^D with the fast scheme it cites): spawns from D into D are
 * dropped, the determinants of D have no stochastic death, are never
 * compressed to C_min, stay in the population at any value (zero included)
 * and count as initiators.  Calling it again re-selects D from the current
 * population; n_core = 0 removes it.  Real mode only (EINVAL otherwise);
 * 0 <= n_core <= 8388608 (EINVAL; the device memory budget may bind first:
 * ENOMEM); a run in a batch: ESTATE, and a run with
 * a deterministic space cannot join a batch.  *n_out (may be NULL)
 * receives |D| = min(n_core, determinants). */
int fciqmc_set_core(fciqmc_run *run, int64_t n_core, int64_t *n_out);

/* The deterministic space: *n_out = |D|, *nnz_out = off-diagonal nonzeros
 * of H^D (either may be NULL); dets (host, may be NULL) receives up to
 * capacity determinants as (alpha, beta) mask pairs, ascending. */
int fciqmc_get_core(const fciqmc_run *run, uint64_t *dets, int64_t capacity, int64_t *n_out,
                    int64_t *nnz_out);
/* Row k of H^D (0 <= k < |D|, determinants in the order fciqmc_get_core
 * gives), for parity checks: *n_out (may be NULL) = its off-diagonal
 * nonzeros; cols and vals (host, may be NULL) receive up to cap of them,
 * the column's index in D and H_kj = <D_k|H|D_j>, in no particular order.
 * EINVAL for k out of range. */
int fciqmc_get_core_row(const fciqmc_run *run, int64_t k, int32_t *cols, double *vals, int64_t cap,
                        int64_t *n_out);
/* The current reference of the projected energy (alpha, beta masks) and its
 * H_PP + e_core (any output may be NULL). */
int fciqmc_get_reference(const fciqmc_run *run, uint64_t *alpha, uint64_t *beta, double *e_ref);
int fciqmc_get_checkpoint(const fciqmc_run *run, fciqmc_checkpoint *out);
int fciqmc_set_checkpoint(fciqmc_run *run, const fciqmc_checkpoint *in);

/* Device Slater-Condon matrix elements <D_j|H|D_i> for n host pairs
 * (dets_i, dets_j: 2 uint64 each; out: host), for parity checks. */
int fciqmc_matrix_elements(const fciqmc_system *sys, const uint64_t *dets_i,
                           const uint64_t *dets_j, int64_t n, double *out);

/* One row of the pre-computed heat-bath alias tables (Appendix A.3, Eq.
 * (hbs)), copied back for parity checks.  opp != 0: the opposite-spin row
 * of electrons (I alpha, J beta), row = I*N + J, over the N*N hole columns
 * A*N + B; opp == 0: the same-spin row of the orbital pair I < J (pairs in
 * lexicographic order), over the N(N-1)/2 hole pairs A < B.  prob, alias,
 * weight (host, one entry per column) receive the alias threshold, the
 * alias column and the column's weight w_ab; *sum the row sum of the
 * weights.  Builds the tables on first use; EINVAL for a row out of range. */
int fciqmc_pchb_row(const fciqmc_system *sys, int opp, int64_t row, double *prob, int32_t *alias,
                    double *weight, double *sum);

/* fciqmc_matrix_elements for callers that cannot allocate device memory
 * (serving loops, allocation-free harnesses): the same values, computed by
 * the same kernel, with the pairs and results staged in a fixed device
 * array of the library instead of buffers allocated per call.  It calls no
 * hipMalloc or hipFree.  At most 65536 pairs per call (EINVAL above that);
 * the array holds about 2.5 MB on each device the library runs on, kept
 * until the process ends.  Calls are serialised within the process by a
 * lock; the array keeps the last call's contents, and calls from several
 * processes on one device use separate copies.  Synchronous (returns when
 * out is written); not for use under stream capture. */
int fciqmc_matrix_elements_noalloc(const fciqmc_system *sys, const uint64_t *dets_i,
                                   const uint64_t *dets_j, int64_t n, double *out);

/* Device memory currently held by a run (bytes). */
int64_t fciqmc_run_device_bytes(const fciqmc_run *run);

/* Per-kernel timing.  enable != 0 starts recording HIP events around each
 * kernel of every 16th later step (steps whose number is a multiple of 16;
 * on the run's stream).  ms: host, 3 entries receive the accumulated
 * milliseconds of the spawn, annihilation and post kernels over the timed
 * steps; *steps the number of steps timed.
 * layout: host, 2 entries receive the bucket count of the walker store and
 * the spawn-record capacity (either output may be NULL). */
int fciqmc_profile(fciqmc_run *run, int enable, double *ms, int64_t *steps, int64_t *layout);

/* ---- Batches: many populations advanced by shared launches ------------
 *
 * A batch steps its member runs together: per step one spawn launch per
 * excitation generator, one annihilation launch and one post launch (or, in
 * the persistent form, one cooperative launch) for all members of the same
 * determinant width and value type, and a single read-back and
 * synchronisation for the whole batch.  The members
 * may hold different systems (orbital counts, integrals), parameters and
 * population sizes.  Each member's arithmetic is exactly that of stepping
 * it alone (Eq. fciqmc_dyn applied per population; the populations never
 * interact), so in integer mode every member's trajectory is bit-identical
 * to its solo trajectory; a member whose step overflows a capacity replays
 * that step alone before the batch step returns.
 *
 * While a run is a member, its own stream is not used (the batch's is),
 * fciqmc_step on it returns ESTATE, and fciqmc_free_run removes it first.
 * fciqmc_energy, get/set_walkers and the checkpoint calls stay valid. */

/* stream: as for fciqmc_init (NULL = library-owned stream). */
int fciqmc_batch_create(void *stream, fciqmc_batch **out);
/* Add a run (EINVAL if it already belongs to a batch); remove it again
 * (EINVAL if it is not a member).  Members keep their order of addition. */
int fciqmc_batch_add(fciqmc_batch *batch, fciqmc_run *run);
int fciqmc_batch_remove(fciqmc_batch *batch, fciqmc_run *run);
int fciqmc_batch_size(const fciqmc_batch *batch);
/* Advance every member n_steps.  stats: host array of n_steps * size
 * entries or NULL; entry [s * size + m] is member m after step s.  On an
 * error the failing member has not recorded that step; the others have. */
int fciqmc_batch_step(fciqmc_batch *batch, int n_steps, fciqmc_step_stats *stats);

/* Autotuner report (see fciqmc_batch_tune). */
typedef struct fciqmc_tune_report {
    int persistent;        /* chosen launch form: 1 one cooperative launch per step          */
    int dets_per_bucket;   /* chosen walker-store occupancy; 0 = partition left as found    */
    int grid_spawn;        /* chosen spawn workgroups per launch; 0 = one per 256 attempts */
    int grid_annihilate;   /* chosen annihilation workgroups; 0 = one per bucket            */
    int trials;            /* configurations timed                                          */
    int64_t steps;         /* steps the tuning advanced every member                        */
    double rate_initial;   /* spawn attempts/s of the configuration found                   */
    double rate_best;      /* spawn attempts/s of the configuration chosen                  */
} fciqmc_tune_report;

/* Time trial_steps real steps under each candidate launch shape -- the
 * launch form (persistent or per phase), walker-store occupancy
 * (determinants per bucket, which sets each member's bucket count), spawn
 * grid and annihilation grid, one coordinate at a time -- and keep the
 * fastest.  None of these changes any trajectory; the tuning steps are
 * ordinary steps of every member.  out: host, may be NULL. */
int fciqmc_batch_tune(fciqmc_batch *batch, int trial_steps, fciqmc_tune_report *out);
/* Launch form of a batch step (default off; fciqmc_batch_tune times both
 * and keeps the faster): on, each group of members
 * with the same determinant width and value type advances through spawn,
 * annihilation, new diagonals and post work in ONE cooperative launch whose
 * workgroups all stay resident, the phases separated by a grid-wide barrier
 * (a bounded wait: a barrier that does not complete fails the step with
 * EDEVICE instead of hanging); off, one launch per phase and generator.
 * Work items and arithmetic are those of the per-phase launches, so every
 * member's trajectory is the same either way. */
int fciqmc_batch_set_persistent(fciqmc_batch *batch, int on);
/* Per-kernel timing of the batch's launches, as fciqmc_profile (ms: spawn,
 * annihilation, post launches of all members; *steps: batch steps timed). */
int fciqmc_batch_profile(fciqmc_batch *batch, int enable, double *ms, int64_t *steps);
/* Remove every member (they keep their state) and release the batch. */
void fciqmc_batch_free(fciqmc_batch *batch);

/* ---- Request server: continuous batching of solves --------------------
 *
 * A solve is a run from n_initial walkers until its energy report (the
 * blocking analysis of fciqmc_energy, with the run's conv_tol and
 * equil_steps) says converged, checked every check_interval of its own
 * steps, or until max_steps.  Requests wait in arrival order; each poll
 * step admits the head of the queue while its device-memory reservation
 * (fciqmc_estimate_bytes) fits the server's budget and fewer than
 * max_running solves run, then advances every running solve by one step in
 * one batch (see the batch calls) and retires those that finished, which
 * frees their memory and slot for the next admission.  A solve's
 * trajectory, step count and energy report are those of the same run
 * stepped alone.  Each admitted run is limited to its reservation
 * (hbm_budget_bytes): outgrowing it fails that request with ENOMEM. */

#define FCIQMC_REQ_QUEUED 0
#define FCIQMC_REQ_RUNNING 1
#define FCIQMC_REQ_DONE 2
#define FCIQMC_REQ_FAILED 3

typedef struct fciqmc_request_info {
    int state;                  /* FCIQMC_REQ_*                                            */
    int error;                  /* FAILED: the FCIQMC_E* code of the failure               */
    int converged;              /* DONE: 1 if the energy criterion ended it, 0 if max_steps */
    int64_t steps;              /* steps taken                                             */
    int64_t attempts;           /* spawn attempts made                                     */
    int64_t reserved_bytes;     /* device memory reserved for it                           */
    double t_arrival;           /* server clock (seconds since creation)                   */
    double t_admit, t_done;     /* server clock; -1 until reached                          */
    fciqmc_energy_report energy; /* at the last check (fields -1 before the first)         */
} fciqmc_request_info;

/* Device bytes a run with these parameters reserves: a walker store of one
 * bucket (1024 entries) per 256 target walkers and at least twice the
 * initial buckets, spawn slabs for six records per target walker (a growing
 * population overshoots its target), and an import staging buffer for three
 * times the target.  Negative FCIQMC_E* on bad arguments. */
int64_t fciqmc_estimate_bytes(const fciqmc_system *sys, const fciqmc_params *p);
/* hbm_budget_bytes: device memory the running solves may reserve together;
 * max_running: largest batch; stream as for fciqmc_init. */
int fciqmc_server_create(int64_t hbm_budget_bytes, int max_running, void *stream,
                         fciqmc_server **out);
/* Queue a solve.  sys is borrowed and must outlive the request; p is copied.
 * t_arrival: the request's arrival on the server clock (< 0: now), from
 * which its latency t_done - t_arrival counts.  *ticket identifies it. */
int fciqmc_server_submit(fciqmc_server *srv, const fciqmc_system *sys, const fciqmc_params *p,
                         int check_interval, int64_t max_steps, double t_arrival,
                         int64_t *ticket);
/* Admit what fits and advance the running solves by up to n_steps batch
 * steps (fewer when none runs); n_running, n_queued (may be NULL) receive
 * the counts afterwards. */
int fciqmc_server_poll(fciqmc_server *srv, int n_steps, int *n_running, int *n_queued);
int fciqmc_server_info(const fciqmc_server *srv, int64_t ticket, fciqmc_request_info *out);
double fciqmc_server_clock(const fciqmc_server *srv);
/* Release every running solve and the server (systems stay the caller's). */
void fciqmc_server_free(fciqmc_server *srv);

/* ---- Replica pairs and the PT2 correction (Sec. "Perturbative correction",
 * Eq. (pt2_correction)) ----
 * Two runs of one system with independent random streams (different
 * replica_id or seed), the same time step, determinant layout and reference,
 * stepped in lockstep.  In each step a run records its discarded spawns: the
 * non-initiator spawns onto determinants unoccupied at tau that no initiator
 * spawn reached.  Over the determinants both replicas discarded,
 *   dE2 = 1/dtau^2 sum_j S_j^1 S_j^2 / (E_0 - H_jj),
 * S_j^r the weight replica r spawned onto j, E_0 the mean of the two shifts
 * used in that step, divided by the replica overlap sum_i C_i^1 C_i^2 of
 * the populations the step began from (the printed equation holds for a
 * normalised wave function; averaged over steps as a ratio of means).  The
 * correction applies to a variational energy of the initiator
 * approximation (not computed here).  Creating a pair gives both
 * runs the same bucket count and fixes it; a store that still outgrows it
 * during a step is read in its own layout for that step's sums (bucket
 * counts are powers of two, so each bucket of the finer layout lies inside
 * one bucket of the coarser), and both are re-bucketed to the larger count
 * afterwards, so every step is evaluated.  A run in a pair cannot
 * join a batch or another pair, is stepped through fciqmc_pair_step only,
 * and freeing it detaches it (the pair then returns ESTATE).
 * fciqmc_pair_step: n_steps lockstep steps; stats1/stats2 (host, n_steps
 * entries) and de2 (host, n_steps doubles) may be NULL.  The per-bucket sums
 * run in as many passes over disjoint hash ranges as a bucket's discarded
 * spawns need (no capacity limit).  If a step fails, the steps before it
 * keep their values (de2, and the pair's record used by fciqmc_pair_pt2),
 * de2 is NaN from the failed step on, and the replicas may stand a step
 * apart: free the pair.
 * fciqmc_pair_pt2: dE2 over the pair's steps from number `skip` on (NaN
 * steps left out) as the ratio of the mean numerator to the mean overlap,
 * with its blocked error; *n receives the steps used. */
int fciqmc_pair_create(fciqmc_run *r1, fciqmc_run *r2, fciqmc_pair **out);
int fciqmc_pair_step(fciqmc_pair *pair, int n_steps, fciqmc_step_stats *stats1,
                     fciqmc_step_stats *stats2, double *de2);
int fciqmc_pair_pt2(const fciqmc_pair *pair, int64_t skip, double *mean, double *err, int64_t *n);

/* ---- Replica 2-RDM and the variational energy (Sec. "Density matrix
 * sampling and pure expectation values", Eq. (FCI2RDM); Sec. "Perturbative
 * correction": the energy the PT2 correction corrects) ----
 * Gamma_{kl,mn} = sum_{i,j} C_i^1 C_j^2 <D_i| a+_k a+_l a_n a_m |D_j> over
 * spin orbitals (canonical index: alpha orbital p -> p, beta p -> N + p),
 * kept for k < l, m < n: pair index P(k,l) = k(2K-k-1)/2 + l-k-1 of the
 * M = K(K-1)/2 pairs (K = 2N), matrix element [P(k,l) M + P(m,n)].
 * fciqmc_pair_rdm_enable(pair, 1) clears the accumulator and samples every
 * later paired step: the diagonal terms C_i^1 C_i^2 exactly over the
 * determinants occupied in both populations a step starts from, and each
 * excitation D_i -> D_j a replica draws in that step (accepted or not)
 * with weight C_i / (m_i p_gen) times the other replica's C_j, halved
 * between the replicas (an unbiased estimate of the replica product; the
 * replica trick removes the bias of a squared amplitude).  Readings: every
 * non-null draw counts; the sum is made hermitian and normalised only when
 * reported.  Excitations the generator can never draw (zero weight) are
 * absent; their Hamiltonian elements vanish.  enable(pair, 0) stops
 * sampling and keeps the sum.  While sampling, a replica's next spawn is
 * not queued ahead of its step.
 * fciqmc_pair_rdm: the accumulated matrix made hermitian, (G + G^T)/2
 * (gamma: host, capacity >= M*M entries, or NULL), *dim = M, the
 * variational energy
 *   E_var = [sum_pq h_pq gamma_pq + sum_{k<l,m<n} Gamma_{kl,mn} <kl||mn>] / norm + E_core,
 *   gamma_pq = sum_r Gamma_{pr,qr} / (n-1),  norm = trace / (n(n-1)/2),
 * the norm (the summed replica overlap) and the steps sampled (any output
 * may be NULL).  ESTATE if sampling was never enabled. */
int fciqmc_pair_rdm_enable(fciqmc_pair *pair, int on);
int fciqmc_pair_rdm(const fciqmc_pair *pair, double *gamma, int64_t capacity, int64_t *dim, double *e_var,
                    double *norm, int64_t *steps);
void fciqmc_pair_free(fciqmc_pair *pair);

void fciqmc_free_run(fciqmc_run *run);
void fciqmc_free_system(fciqmc_system *sys);
const char *fciqmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FCIQMC_H */
