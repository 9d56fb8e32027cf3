/*
 * mbmd.h -- C ABI of libmbmd: write-conflict-free force evaluation for
 * many-body potentials (Tersoff, Stillinger-Weber) on one MI355X (gfx950).
 *
 * Method: Fan, Chen, Vierimaa, Harju, "Efficient molecular dynamics
 * simulations with many-body potentials on graphics processing units".
 * The force on atom i is the sum of explicit pairwise forces
 * F_ij = dU_i/dr_ij - dU_j/dr_ji (Section 2.3, general form Section 2.4); the
 * per-atom virial W_i = -1/2 sum_j r_ij (x) F_ij and the per-atom heat current
 * J_i = sum_j r_ij (dU_j/dr_ji . v_i) (Section 2.3) are accumulated by the
 * thread that owns atom i, so no result is written by two threads and no
 * atomic operation touches a result.
 *
 * Conventions for every call:
 *  - Units: Angstrom, eV, amu, fs.  W_i is in eV (not divided by a volume),
 *    J_i in eV*Angstrom/fs.
 *  - r_ij = r_j - r_i under the minimum-image convention (Section 2.1).
 *  - Device arrays are structure-of-arrays, FP64, caller-owned: positions and
 *    velocities [3][n], forces [3][n], heat current [3][n], energy [n],
 *    virial [9][n] with component 3*alpha + beta holding
 *    W^{alpha beta} = -1/2 sum_j r_ij^alpha F_ij^beta.
 *  - Boxes are orthorhombic and periodic in all three directions; box[3]
 *    is a HOST array of edge lengths, each at least 2 * (cutoff + skin).
 *  - Positions may be given unwrapped; positions returned are wrapped into
 *    [0, L).
 *  - types (device int32 [n]) may be NULL (every atom type 0); otherwise
 *    every entry must lie in [0, ntypes) of the potential: 1 for SW and the
 *    single-element Tersoff, ntypes of mbmd_set_tersoff_multi (else
 *    MBMD_EINVAL).
 *  - Every call enqueues its work on the context's stream and returns after
 *    synchronising that stream, with the device status folded into the
 *    return code.  Outputs are unspecified when a call fails.
 *  - A context is not thread-safe; use one context per host thread and
 *    stream.  The library never frees caller memory.
 *  - Results are bitwise reproducible from run to run (fixed summation
 *    orders, sorted neighbour lists).
 */
#ifndef MBMD_H
#define MBMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MBMD_OK = 0,
    MBMD_EINVAL = 1,      /* invalid argument (null pointer, bad size, type != 0) */
    MBMD_ENOMEM = 2,      /* device allocation failed or bound workspace too small */
    MBMD_EDEVICE = 3,     /* HIP runtime error or internal consistency failure */
    MBMD_EBOX = 4,        /* a box edge is shorter than 2 (cutoff + skin) or not finite */
    MBMD_ENEIGH = 5,      /* a neighbour list needed more than max_neighbors slots */
    MBMD_ESKIN = 6,       /* serving batch: an atom of the structure moved more than
                             skin/2 from its position at a list build before the
                             next scheduled build (reported by mbmd_batch_retire;
                             single runs handle this through the rebuild policy) */
    MBMD_ENONFINITE = 7,  /* a non-finite position */
    MBMD_ENOPOT = 8,      /* no potential set on the context */
    MBMD_EBUSY = 9        /* serving batch: no room now, or structure not finished */
} mbmd_status;

typedef enum {
    MBMD_FP64 = 0,        /* all arithmetic in FP64 */
    MBMD_MIXED = 1        /* bond-order and force arithmetic in FP32; positions,
                             integrator and the per-atom U, F, W, J accumulators
                             in FP64 */
} mbmd_precision;

/* Tersoff potential in the single-element form of Section 2.1: U = 1/2 sum
 * U_ij, U_ij = f_C (f_R - b_ij f_A), b_ij = (1 + beta^n zeta_ij^n)^(-1/(2n)),
 * zeta_ij = sum_k f_C(r_ik) g_ijk, g = 1 + c^2/d^2 - c^2/(d^2 + (h - cos)^2),
 * with f_R = A exp(-lambda r), f_A = B exp(-mu r) and
 * f_C = 1 (r < R), 1/2 + 1/2 cos(pi (r - R)/(S - R)) (R <= r < S), 0 beyond. */
typedef struct {
    double A, B, lambda, mu, beta, n, c, d, h, R, S;
} mbmd_tersoff_params;

/* Stillinger-Weber potential (the paper's second many-body potential,
 * Section 2.4): U_i = 1/2 sum_j phi2(r_ij) + sum_{j<k} h_ijk with
 * phi2 = epsilon A (B (sigma/r)^p - (sigma/r)^q) exp(sigma/(r - a sigma)),
 * h_ijk = epsilon lambda exp(gamma sigma/(r_ij - a sigma)
 *         + gamma sigma/(r_ik - a sigma)) (cos theta_jik + 1/3)^2, cutoff a sigma. */
typedef struct {
    double epsilon, sigma, a, lambda, gamma, A, B, p, q;
} mbmd_sw_params;

/* When nve_run rebuilds the neighbour list (the paper builds it once or on a
 * fixed schedule; Section 3). */
typedef enum {
    MBMD_REBUILD_FIXED = 0,    /* every rebuild_every steps, nothing else; no
                                  displacement is tracked, so the caller picks
                                  rebuild_every short enough that no pair
                                  closes in by more than skin between builds */
    MBMD_REBUILD_ON_SKIN = 1   /* also before any step whose positions moved
                                  more than skin/2 from the last build
                                  (default) */
} mbmd_rebuild_policy;

/* Statistics of the last mbmd_nve_run on a context. */
typedef struct {
    int64_t steps;             /* steps integrated */
    int64_t rebuilds;          /* list builds, the initial one included */
    int64_t rollbacks;         /* chunks replayed to insert an early rebuild */
    double max_displacement;   /* largest distance (A) any atom moved from its
                                  position at the build of the list it was
                                  evaluated with; -1 under MBMD_REBUILD_FIXED */
} mbmd_run_stats;

/* Accumulated device time of one class of kernel launches (profiling). */
typedef struct {
    const char *name;          /* static string owned by the library */
    int64_t launches;
    double total_ms;
} mbmd_kernel_time;

typedef struct mbmd_ctx mbmd_ctx;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL means the default stream).  The stream is borrowed,
 * not owned.  *out receives the context.  The context starts with no
 * potential, skin 0.5 A and an automatic list capacity. */
mbmd_status mbmd_create(mbmd_ctx **out, int device, void *hip_stream);

/* Destroy a context and free the device memory it allocated itself. */
void mbmd_destroy(mbmd_ctx *ctx);

/* Text of the last error on this context (owned by the context; valid until
 * the next call on it). */
const char *mbmd_last_error(const mbmd_ctx *ctx);

/* Select the Tersoff potential with parameters *p (copied): one element,
 * every atom type 0. */
mbmd_status mbmd_set_tersoff(mbmd_ctx *ctx, const mbmd_tersoff_params *p);

/* Select Tersoff's multicomponent form (Tersoff 1989, the potential the
 * paper cites; Section 2.1 states that the method covers several atom
 * types) for ntypes (1..4) elements: elem[ntypes] (copied) with the mixing
 * rules A_ij = sqrt(A_i A_j), B_ij = sqrt(B_i B_j), lambda_ij = (lambda_i +
 * lambda_j)/2, mu_ij = (mu_i + mu_j)/2, R_ij = sqrt(R_i R_j), S_ij =
 * sqrt(S_i S_j) for the bond terms f_C, f_R, f_A of a pair, and atom i's
 * beta, n, c, d, h in b_ij and g_ijk; b_ij is multiplied by chi[ti][tj]
 * (chi: [ntypes][ntypes], symmetric, positive; NULL: all 1).  Atom types come
 * from the types arrays of mbmd_compute/nve_run/npt_run (NULL: all 0) and
 * must lie in [0, ntypes) (else MBMD_EINVAL).  The serving batch treats every
 * atom as type 0. */
mbmd_status mbmd_set_tersoff_multi(mbmd_ctx *ctx, int ntypes, const mbmd_tersoff_params *elem,
                                   const double *chi);

/* Per-type masses (amu) used by mbmd_nve_run and mbmd_npt_run when their
 * mass_amu is 0: mass_amu[ntypes] (copied), ntypes in 1..4; ntypes = 0
 * clears them.  A run with mass 0 needs a mass for every atom type of the
 * potential (MBMD_EINVAL otherwise). */
mbmd_status mbmd_set_type_masses(mbmd_ctx *ctx, int ntypes, const double *mass_amu);

/* Select the Stillinger-Weber potential with parameters *p (copied). */
mbmd_status mbmd_set_sw(mbmd_ctx *ctx, const mbmd_sw_params *p);

/* Neighbour-list settings (Section 2.1: Verlet list built with a cell list).
 * The list radius is the potential cutoff plus `skin` (>= 0); under a
 * multi-element Tersoff potential each pair of types has its own cutoff
 * S_ab = sqrt(S_a S_b), so its own radius S_ab + skin.
 * `max_neighbors` is the list capacity per atom, 1..64, or 0 for the default
 * (16 for Tersoff, 32 for Stillinger-Weber). */
mbmd_status mbmd_set_neighbor(mbmd_ctx *ctx, double skin, int max_neighbors);

/* Rebuild policy of mbmd_nve_run (default MBMD_REBUILD_ON_SKIN). */
mbmd_status mbmd_set_rebuild_policy(mbmd_ctx *ctx, mbmd_rebuild_policy policy);

/* Statistics of the last mbmd_nve_run on this context, copied to *out. */
mbmd_status mbmd_get_run_stats(const mbmd_ctx *ctx, mbmd_run_stats *out);

/* Profiling: with enable != 0 every later call records a pair of HIP events
 * on the context's stream around each kernel launch class and accumulates
 * the elapsed device time (adds a little launch overhead). */
mbmd_status mbmd_set_profiling(mbmd_ctx *ctx, int enable);

/* Zero the accumulated profile. */
mbmd_status mbmd_reset_profile(mbmd_ctx *ctx);

/* Copy up to `capacity` entries of the profile to out[] and store the number
 * of kernel classes in *count (stage_positions, neighbor_build,
 * site_partials, site_partials_overflow, pair_gather, thermo_reduce). */
mbmd_status mbmd_get_profile(const mbmd_ctx *ctx, mbmd_kernel_time *out, int capacity,
                             int *count);

/* Current list capacity per atom (resolved default) in *out. */
mbmd_status mbmd_get_max_neighbors(const mbmd_ctx *ctx, int *out);

/* Device bytes of workspace needed for up to n_atoms atoms with the current
 * potential and neighbour settings. */
mbmd_status mbmd_workspace_size(const mbmd_ctx *ctx, int64_t n_atoms, size_t *bytes);

/* Use caller-owned device memory [dev_ptr, dev_ptr + bytes) as workspace
 * (256-byte aligned).  The caller keeps ownership and must keep it alive
 * while the context uses it; NULL unbinds.  Without a bound workspace the
 * context allocates (and grows) its own. */
mbmd_status mbmd_bind_workspace(mbmd_ctx *ctx, void *dev_ptr, size_t bytes);

/* Build the neighbour list of n atoms at device positions pos[3][n] and copy
 * it out: nn[n] (device, true count per atom) and nl[max_neighbors][n]
 * (device, slot-major; unused slots are left untouched).  Atom j is listed
 * for atom i iff j != i and the minimum-image squared distance, evaluated in
 * FP64 as (dx*dx + dy*dy) + dz*dz with d <- d - L rint(d/L) and no fused
 * multiply-add, is below (cutoff + skin)^2 (the Verlet list over a cell list
 * of Section 2.1).  The cutoff is the pair's: SW's a*sigma, Tersoff's S, and
 * under a multi-element Tersoff potential S_ab = sqrt(S_a S_b) for types a
 * and b (types as in every call taking them: NULL for type 0 everywhere,
 * else each in [0, ntypes)); the run and compute calls build the same
 * lists.  Each list holds the neighbours inside the pair's cutoff first,
 * then the others, each group by ascending atom index: a deterministic
 * order, so every per-atom sum over the list is reproducible.  When a list
 * needs more than max_neighbors slots the call returns MBMD_ENEIGH and still
 * writes both arrays: nn the true counts, nl the first max_neighbors entries
 * of each list in that order. */
mbmd_status mbmd_neighbors(mbmd_ctx *ctx, int64_t n, const double box[3], const double *pos,
                           const int32_t *types, int32_t *nn, int32_t *nl);

/* Single point (the force-evaluation kernel of Section 2.3 with the
 * bond-order precompute for Tersoff): per-atom energy U[n], force F[3][n],
 * virial W[9][n] and heat current J[3][n] (all device, caller-owned) for
 * positions pos[3][n] and velocities vel[3][n] (vel may be NULL: J = 0). */
mbmd_status mbmd_compute(mbmd_ctx *ctx, mbmd_precision prec, int64_t n, const double box[3],
                         const double *pos, const double *vel, const int32_t *types,
                         double *U, double *F, double *W, double *J);

/* mbmd_compute for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results (bit for bit) as mbmd_compute, but the
 * call's whole workspace lies in a static device array of the library
 * (64 MiB on each device the library runs on, held until the process ends)
 * instead of the context's workspace, and the call makes no hipMalloc,
 * hipFree, pinned-memory or other allocating call; profiling is off for it.
 * The array holds the workspace of 74,712 Tersoff atoms at 16 list slots
 * (the need grows with max_neighbors: 47,794 SW atoms at 32);
 * a larger n is refused with MBMD_ENOMEM.  Every call on one device shares
 * that device's array and leaves its contents there (the call clears what
 * it needs cleared), so calls that overlap on one device, from any contexts
 * or streams, race: serialise them.  Like every call it ends by
 * synchronising the context's stream. */
mbmd_status mbmd_compute_noalloc(mbmd_ctx *ctx, mbmd_precision prec, int64_t n,
                                 const double box[3], const double *pos, const double *vel,
                                 const int32_t *types, double *U, double *F, double *W,
                                 double *J);

/* n_steps of NVE velocity-Verlet integration (the integrator of Section 3,
 * without thermostat or barostat) at time step dt_fs for atoms of mass
 * mass_amu.  pos[3][n] and vel[3][n] (device) are advanced in place.  The
 * forces are evaluated at the start (step 0) and after every drift; the list
 * is built before step 0 and rebuilt before step s when s - (step of the last
 * build) == rebuild_every, or, under MBMD_REBUILD_ON_SKIN, when the
 * positions of step s moved more than skin/2 from those of the last build.
 * U, F, W, J receive the last step's values, J_i formed with the full-step
 * velocity.  thermo (device, or NULL) receives [n_steps + 1][16] rows:
 * 0 E_pot, 1 E_kin, 2..10 total W, 11..13 total J, 14 E_pot + E_kin,
 * 15 kinetic temperature with 3n - 3 degrees of freedom. */
mbmd_status mbmd_nve_run(mbmd_ctx *ctx, mbmd_precision prec, int64_t n, const double box[3],
                         double mass_amu, double *pos, double *vel, const int32_t *types,
                         double dt_fs, int n_steps, int rebuild_every, double *U, double *F,
                         double *W, double *J, double *thermo);

/* n_steps more steps of the run that the last call on this context (an
 * mbmd_nve_run or mbmd_nve_continue that completed) took, from the state it
 * left: the positions and velocities in pos and vel, the forces of its last
 * step in F, and, in the context's workspace, its neighbour list, the
 * positions of its last list build and its place in the rebuild schedule.
 * The steps are those the original run would have taken next, bit for bit:
 * the first half-kick and drift that its last step left out, then
 * n_steps - 1 ordinary steps and a last one, with list builds where its
 * schedule (or policy) puts them.  So a run of s1 + s2 steps equals a run
 * of s1 steps continued by s2, and an MD program continues a run without
 * the force evaluation and list build a new run starts with (velocity-Verlet
 * of Section 3).  Arguments as for mbmd_nve_run: n, box, mass, dt,
 * rebuild_every, precision, the rebuild policy and the pos, vel, types and F
 * buffers must be those of the run continued, whose contents the caller has
 * left unchanged (MBMD_EINVAL otherwise, or if no such run precedes: any
 * other call that uses the workspace, or changes the potential, the list
 * settings or the policy, ends the chance to continue).  thermo (device
 * [n_steps + 1][16] or NULL) receives the continued run's rows, row 0 being
 * the state it starts from (the previous run's last row; that run must have
 * had a thermo array).  U, F, W, J receive the last step's values. */
mbmd_status mbmd_nve_continue(mbmd_ctx *ctx, mbmd_precision prec, int64_t n, const double box[3],
                              double mass_amu, double *pos, double *vel, const int32_t *types,
                              double dt_fs, int n_steps, int rebuild_every, double *U,
                              double *F, double *W, double *J, double *thermo);

/* Berendsen weak coupling (Berendsen et al. 1984): the NPT ensemble, at
 * 300 K and 0 Pa, in which the paper times its runs (Section 3).  The paper
 * prints no coupling formula or constants; the isotropic form below is
 * Berendsen's.  A tau <= 0 switches that coupling off. */
typedef struct {
    double T0_K;           /* target temperature (K), >= 0 */
    double tau_T_fs;       /* thermostat time constant (fs); >= dt when on */
    double P0_GPa;         /* target pressure (GPa) */
    double tau_P_fs;       /* barostat time constant (fs) */
    double beta_per_GPa;   /* isothermal compressibility (1/GPa), >= 0 */
} mbmd_berendsen;

/* n_steps of velocity-Verlet with Berendsen weak coupling, otherwise as
 * mbmd_nve_run under MBMD_REBUILD_FIXED (whatever the context's policy).
 * After the second half-kick of step s (s < n_steps) the thermo row gives
 * the kinetic temperature T and the pressure P = (2 E_kin + tr W) / (3 V)
 * from the per-atom virials; velocities are scaled by
 * lambda = sqrt(1 + dt/tau_T (T0/T - 1)) (1 when T = 0) and positions and
 * the three box edges by mu = (1 - beta dt/tau_P (P0 - P))^(1/3) before the
 * first half-kick of step s + 1.  box[3] (host) gives the initial box and
 * receives the final one; the list is rebuilt on the current box every
 * rebuild_every steps, and MBMD_EBOX is returned if an edge has shrunk
 * below 2 (cutoff + skin) by then.  thermo (device, required) receives the
 * [n_steps + 1][16] rows of mbmd_nve_run; box_traj (device, or NULL) the
 * [n_steps + 1][3] box edges each row was evaluated in.  MBMD_EINVAL for
 * out-of-range coupling constants, or if 1 - beta dt/tau_P (P0 - P) <= 0
 * at some step (that step's mu is taken as 1 and the run completes). */
mbmd_status mbmd_npt_run(mbmd_ctx *ctx, mbmd_precision prec, int64_t n, double box[3],
                         double mass_amu, double *pos, double *vel, const int32_t *types,
                         double dt_fs, int n_steps, int rebuild_every,
                         const mbmd_berendsen *coupling, double *U, double *F, double *W,
                         double *J, double *thermo, double *box_traj);

/* Green-Kubo analysis of the total heat current J = sum_i J_i (the
 * potential part of Section 2.3, whose purpose is thermal-conductivity
 * calculations; the Green-Kubo relation itself is the textbook one).
 * thermo (device, [n_rows][16], as written by mbmd_nve_run or mbmd_npt_run,
 * one row per dt_fs) is sampled at rows 0, e, 2e, ... (e = sample_every),
 * S = (n_rows - 1)/e + 1 samples.  hac (device, [max_lag][3]) receives
 * C_a(k) = 1/(S - k) sum_{t=0}^{S-k-1} J_a(t) J_a(t + k) for k < max_lag
 * and a = x, y, z (every time origin used), in (eV A/fs)^2; kappa (device,
 * [max_lag][3], or NULL) the running conductivity in W/(m K),
 * kappa_a(K) = e dt / (k_B T^2 V) [C_a(0)/2 + C_a(1) + ... + C_a(K)/2]
 * (trapezoid rule, kappa_a(0) = 0), with V = volume_A3 and T = T_K.
 * Needs 1 <= max_lag <= S; MBMD_EINVAL otherwise.  The context allocates
 * (and keeps) a scratch of 8 (3 S + min(64, ceil(S/1024)) 3 max_lag) bytes.
 * Synchronous; the result bits do not depend on the run. */
mbmd_status mbmd_green_kubo(mbmd_ctx *ctx, const double *thermo, int64_t n_rows,
                            int sample_every, int max_lag, double dt_fs, double volume_A3,
                            double T_K, double *hac, double *kappa);

/* Wait for everything this context enqueued on its stream and report (and
 * clear) the device status word: MBMD_ENONFINITE, MBMD_ENEIGH or
 * MBMD_EINVAL (atom type) for a condition raised since the last report,
 * MBMD_EDEVICE if the stream failed.  mbmd_compute and mbmd_nve_run already
 * end with this; it is the completion point of the asynchronous batch calls. */
mbmd_status mbmd_sync(mbmd_ctx *ctx);

/* ---- serving batch ------------------------------------------------------
 *
 * Continuous batching of independent structures (the serving form of the
 * path): a batch keeps every admitted structure's positions, velocities and
 * outputs on the device and advances all unfinished structures together, one
 * step per mbmd_batch_step, in single launches whose blocks map to
 * (structure, atom range) through a segment table with per-structure boxes,
 * cell grids, offsets and time steps.  Structures can be admitted whenever
 * an atom range and a slot are free, also while others are mid-run.  A
 * structure's results do not depend on what else shares the batch: every
 * per-atom sum runs over its own sorted list, and every per-structure sum
 * over its own blocks in a fixed order, so they equal, bit for bit, those of
 * the same structure alone.  While a batch is open the context accepts only
 * batch calls.  Lists are rebuilt for all running structures together,
 * every rebuild_every batch steps; an admitted structure starts at the next
 * such step (at once if no structure is running, else at most rebuild_every
 * - 1 batch steps later), so its lists are rebuilt at its own steps 0,
 * rebuild_every, 2 rebuild_every, ... as in a run alone. */

/* Open a batch of at most max_atoms atoms in at most max_structures
 * structures (the workspace is sized for that; see
 * mbmd_batch_workspace_size; a small pinned host buffer for table uploads is
 * allocated too).  Uses the context's potential, skin and list capacity.
 * MBMD_ENOMEM if the workspace or the pinned buffer cannot be had,
 * MBMD_EINVAL if a batch is already open or a size is out of range. */
mbmd_status mbmd_batch_open(mbmd_ctx *ctx, int64_t max_atoms, int max_structures,
                            int rebuild_every);

/* Device bytes of workspace a batch of this capacity needs. */
mbmd_status mbmd_batch_workspace_size(const mbmd_ctx *ctx, int64_t max_atoms,
                                      int max_structures, size_t *bytes);

/* Free atoms, free structure slots and the largest contiguous free atom
 * range of the open batch (a structure needs a contiguous range). */
mbmd_status mbmd_batch_capacity(const mbmd_ctx *ctx, int64_t *free_atoms, int *free_slots,
                                int64_t *largest_range);

/* Admit a structure: n atoms at device positions pos[3][n] with velocities
 * vel[3][n] (copied on the context's stream: the caller may overwrite them
 * with work enqueued after this call on that stream), periodic box (host),
 * mass, time step, and n_steps NVE steps (0: one force evaluation).
 * thermo (device [n_steps + 1][16] or NULL; it must stay allocated until the
 * structure is retired) receives its thermo rows as it runs, in the layout
 * of mbmd_nve_run.  *handle identifies it.  MBMD_EBUSY when no slot or no
 * contiguous atom range of n atoms is free; MBMD_EBOX, MBMD_EINVAL as for
 * mbmd_nve_run.  A non-finite position is reported by the retire call. */
mbmd_status mbmd_batch_add(mbmd_ctx *ctx, int64_t n, const double box[3], const double *pos,
                           const double *vel, double mass_amu, double dt_fs, int n_steps,
                           double *thermo, int *handle);

/* One step of every started, unfinished structure (its force evaluation,
 * and the integration unless it is at its last step).  *n_active receives
 * the number of structures that took part (admitted structures waiting for
 * the next rebuild step do not).  Asynchronous: returns once the work is
 * enqueued. */
mbmd_status mbmd_batch_step(mbmd_ctx *ctx, mbmd_precision prec, int *n_active);

/* Handles of finished, not yet retired structures (up to capacity; *count
 * receives the total).  Finished means that its last step has been
 * enqueued; the retire call waits for it. */
mbmd_status mbmd_batch_finished(const mbmd_ctx *ctx, int *handles, int capacity, int *count);

/* Enqueue the copy of a finished structure's final positions (wrapped),
 * velocities and per-atom U, F, W, J into caller device buffers of its n
 * atoms (layouts of mbmd_nve_run; any may be NULL) and free its slot and
 * atom range at once (a later admission is ordered after the copy on the
 * stream).  status (device int32, or NULL) receives the structure's own
 * status as an mbmd_status value: MBMD_OK; MBMD_ENONFINITE for a non-finite
 * admitted position; MBMD_ENEIGH if one of its list builds overflowed the
 * list capacity; MBMD_ESKIN if, between two of the batch's scheduled list
 * builds, one of its atoms moved more than skin/2 from its position at the
 * last build, so that its lists (of radius cutoff + skin) may have missed a
 * pair (the results are then not those of a complete list; rerun it with
 * rebuilds on the skin, or with a shorter rebuild_every).  The first of
 * these in that order is reported.  Asynchronous: the buffers hold the
 * results once the stream has reached this point (mbmd_batch_sync).
 * MBMD_EBUSY if it has not finished, MBMD_EINVAL for an unknown handle.
 * Its thermo array is complete at the same point. */
mbmd_status mbmd_batch_retire(mbmd_ctx *ctx, int handle, double *pos, double *vel, double *U,
                              double *F, double *W, double *J, int32_t *status);

/* Wait for everything enqueued on the context's stream and report the
 * batch's status: MBMD_ENONFINITE if an admitted structure had a non-finite
 * position, MBMD_ENEIGH if a list build overflowed the list capacity (the
 * results of that build's structures are then wrong).  The status covers
 * the whole batch since the previous sync and is cleared by the call.  Skin
 * violations are reported per structure only (mbmd_batch_retire). */
mbmd_status mbmd_batch_sync(mbmd_ctx *ctx);

/* Close the batch (device memory stays with the context). */
mbmd_status mbmd_batch_close(mbmd_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MBMD_H */
