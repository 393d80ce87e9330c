/*
 * tcm.h -- C ABI of libtcm, an MI355X (gfx950) implementation of the two-centre multipole
 * (TCM) method: per-molecule multipole moments (eq. 8 of Solov'yov et al., "Two center
 * multipole expansion method: application to macromolecular systems") and their two-centre
 * contraction into the Coulomb interaction energy of two well separated molecules (eq. 9,
 * square truncation l1, l2 <= L as stated in the text after eq. 9).
 *
 * Conventions shared by every entry point
 *   - All functions return an int status (TCM_OK or a negative TCM_E* code) and never
 *     throw.  Outputs are written only when the call returns TCM_OK; batch calls report a
 *     status per item and write NaN for failed items.
 *   - Host pointers are read during the call only; the caller owns them and may reuse them
 *     as soon as the call returns.  Device pointers passed to tcm_mol_register_device are
 *     borrowed: they must stay valid until the molecule is released.
 *   - Coordinates: FP64, array of structures [n][3] (x, y, z) unless stated otherwise.
 *     Charges: FP64 [n].  Units are the caller's; eq. 1 has no prefactor, so energies come
 *     out in charge^2 / length (multiply by 332.0637 for kcal/mol with e and Angstrom).
 *   - Moment tables are real-packed, (L+1)^2 FP64 values for order L:
 *       index l*l          : Q_l0 (real)
 *       index l*l + 2m - 1 : Re Q_lm,  index l*l + 2m : Im Q_lm   (1 <= m <= l)
 *     Q_{l,-m} = (-1)^m conj(Q_lm) is implied.  Q_lm follows eq. 8:
 *       Q_lm = sum_i q_i r_i^l sqrt(4 pi / (2l+1)) Y_lm(theta_i, phi_i),
 *     with Condon-Shortley phase and r_i = R_i - centre.  A table of order L' >= L may be
 *     passed where order L is needed (its prefix is the order-L table).
 *   - The centre of a molecule is "any suitable point" (section II); when the caller gives
 *     none, the unweighted centroid of the atoms is used.  The radius of a molecule is
 *     a = max_i |R_i - centre|, the quantity eq. 2 constrains.
 *   - eq. 2 (the expansion converges only if |R0| > a_A + a_B): pair energies with
 *     |R0| <= a_A + a_B are rejected with TCM_EDOMAIN unless TCM_UNCHECKED is set.
 *   - Precision: TCM_F64 computes the moment pass in FP64; TCM_F32C computes it in FP32
 *     on centred coordinates scaled by a bound on the radius, summing each thread's atoms
 *     in FP32 and merging every partial sum above that with compensated (TwoSum,
 *     double-float) additions.  Geometric factors, rotation and the energy contraction
 *     are always FP64.
 *   - A context is externally synchronised: do not call into one context from two
 *     threads at once (the serving loop runs its own thread and locks internally).
 */
#ifndef TCM_H
#define TCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TCM_OK          0
#define TCM_EINVAL     -1   /* null pointer, n < 0, L outside [0, TCM_LMAX], non-finite input */
#define TCM_EDOMAIN    -2   /* |R0| <= a_A + a_B: eq. 2 violated                             */
#define TCM_ENOMEM     -3   /* device allocation failed or the HBM budget is exceeded        */
#define TCM_EDEVICE    -4   /* HIP runtime error                                             */
#define TCM_EAGAIN     -5   /* serving queue full; retry later                               */
#define TCM_ENOTFOUND  -6   /* unknown molecule id or ticket                                 */

#define TCM_LMAX 32         /* largest multipole order accepted */

/* precision of the moment pass */
#define TCM_F64   0
#define TCM_F32C  1

/* per-request flags */
#define TCM_UNCHECKED  1    /* skip the eq. 2 separation test (parity tests only)            */
#define TCM_REUSE      2    /* use the molecule's resident moments if their order is >= L    */
#define TCM_DEVICE_IO  16   /* tcm_scan_translations: R, U_out, status_out are device         */
                            /* pointers and the call is asynchronous on the context's stream  */
#define TCM_TRIANGULAR 32   /* truncate eq. 9 to the blocks l1 + l2 <= L (the other reading   */
                            /* of its garbled limits) instead of the square l1, l2 <= L:      */
                            /* energies, batches, scans, all pairs, adaptive truncation and   */
                            /* serving; the force entry points reject it (TCM_EINVAL)         */

typedef struct tcm_ctx tcm_ctx;
typedef struct tcm_plan tcm_plan;
typedef int64_t tcm_mol_id;

/* Human-readable text for a status code (static storage). */
const char *tcm_strerror(int status);

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the device memory the
 * context may hold for resident molecules and workspace (0 = no bound).  flags: reserved,
 * pass 0.  Builds the FP64 coefficient tables on the device.  Errors: TCM_EINVAL (null
 * ctx), TCM_EDEVICE (no such device), TCM_ENOMEM. */
int tcm_create(tcm_ctx **ctx, int device, size_t hbm_budget_bytes, int flags);

/* Release every device buffer of the context (resident molecules included). */
void tcm_destroy(tcm_ctx *ctx);

/* Run the context's work on this HIP stream (hipStream_t passed as void*; NULL = the
 * context's own stream).  The stream must have default priority. */
int tcm_set_stream(tcm_ctx *ctx, void *hip_stream);
void *tcm_get_stream(tcm_ctx *ctx);

/* Device bytes the context currently holds (tables, workspaces, resident molecules, the
 * serving cache) and its HBM budget; tcm_set_budget changes the budget (0 = unbounded) for
 * later allocations. */
int tcm_mem_info(tcm_ctx *ctx, size_t *used_out, size_t *budget_out);
int tcm_set_budget(tcm_ctx *ctx, size_t hbm_budget_bytes);

/* eq. 8 for one molecule.  coords [n][3], charges [n] (host FP64); centre FP64[3] or NULL
 * (centroid); 0 <= L <= TCM_LMAX; precision TCM_F64 or TCM_F32C.  Q_out: (L+1)^2 FP64
 * (packed layout above).  radius_out (a = max |R_i - centre|) and centre_out (FP64[3])
 * may be NULL.  n = 0 is allowed (all moments zero; centre = the given one or the origin).
 * Synchronous. */
int tcm_moments(tcm_ctx *ctx, const double *coords, const double *charges, int64_t n,
                const double *centre, int L, int precision, double *Q_out, double *radius_out,
                double *centre_out);

/* eq. 9 with square truncation l1, l2 <= L (or l1 + l2 <= L with TCM_TRIANGULAR) for one
 * pair, from host moment tables.
 * QA, QB: packed FP64 tables of order >= L.  aA, aB: the molecules' radii (eq. 2 test).
 * R: FP64[3], c_B - c_A.  quat_b: FP64[4] unit quaternion (w, x, y, z) rotating B actively
 * about its centre before the contraction, or NULL for none; QB are B's moments in its
 * unrotated frame.  flags: TCM_UNCHECKED, TCM_TRIANGULAR or 0.  U_out: the energy.
 * Synchronous. */
int tcm_pair_energy(tcm_ctx *ctx, const double *QA, double aA, const double *QB, double aB,
                    const double *R, const double *quat_b, int L, int flags, double *U_out);

/* The moment pass of tcm_moments without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that forbid the
 * allocator).  d_x, d_y, d_z, d_q: the molecule's atoms on the device (FP64 structure of
 * arrays, n each; the caller's, read by the kernels).  centre: host FP64[3] or NULL
 * (centroid).  d_Q: device FP64[(L+1)^2] receiving the packed moments; d_meta: device FP64[8]
 * receiving [0..2] the centre, [3] the radius a, [4] the internal coordinate scale ([5..7]
 * unspecified).  Same tiling and kernels as tcm_moments: the results are the same bit for bit.
 * Every scratch byte lives in one static 32 MiB array per device, held until the process
 * ends; a molecule whose plan does not fit it (roughly: more than ~3800 tiles at L = 32,
 * ~14000 at L = 16, a tile being 256 kper atoms) returns TCM_ENOMEM before anything is
 * launched; TCM_EINVAL as tcm_moments (null pointers, n < 0, L or precision out of range,
 * non-finite centre).  Asynchronous: the kernels are queued on the context's stream and the
 * outputs are ready when that stream is.  All calls on one device share the array: calls that
 * overlap on a device (two contexts' streams, or threads) race; issue them in stream order. */
int tcm_moments_noalloc(tcm_ctx *ctx, const double *d_x, const double *d_y, const double *d_z,
                        const double *d_q, int64_t n, const double *centre, int L, int precision,
                        double *d_Q, double *d_meta);

/* ---- device-resident molecules ---------------------------------------------------- */

/* Copy a molecule's atoms (host AoS FP64) to the device, in the library's resident layout
 * (FP64 structure of arrays): the charges q_i at R_i of eq. 1, whose eq. 8 moments about the
 * centre later calls compute on demand.  centre: FP64[3] or NULL (centroid; the paper leaves
 * the centre free, section II).  precision: the moment pass used for this molecule.  Its
 * resident moment table (33^2 FP64, every order the library accepts) is allocated here too,
 * so later computations on it allocate nothing for it.  The id stays valid until
 * tcm_mol_release / tcm_destroy.  TCM_EINVAL for null pointers, n < 0 or non-finite input,
 * TCM_ENOMEM beyond the context's budget. */
int tcm_mol_upload(tcm_ctx *ctx, const double *coords, const double *charges, int64_t n,
                   const double *centre, int precision, tcm_mol_id *id_out);

/* Register atoms already on the device (FP64 structure of arrays x[n], y[n], z[n], q[n],
 * borrowed, not copied). */
int tcm_mol_register_device(tcm_ctx *ctx, const double *d_x, const double *d_y,
                            const double *d_z, const double *d_q, int64_t n,
                            const double *centre, int precision, tcm_mol_id *id_out);

/* Free the molecule's atoms (if uploaded) and resident moments.  TCM_EAGAIN while a live plan
 * (tcm_plan_create) names the molecule: its launches address these buffers, so release it
 * after tcm_plan_destroy. */
int tcm_mol_release(tcm_ctx *ctx, tcm_mol_id id);

/* Compute (or, with TCM_REUSE in flags, reuse) the molecule's order-L moments on the device
 * and copy them to the host.  Q_out (L+1)^2 FP64; radius_out, centre_out may be NULL. */
int tcm_mol_moments(tcm_ctx *ctx, tcm_mol_id id, int L, int flags, double *Q_out,
                    double *radius_out, double *centre_out);

/* ---- batches ----------------------------------------------------------------------- */

/* One pair-energy request: molecules a and b (resident ids), R0 = c_b - c_a, optional pose
 * of b (unit quaternion (w, x, y, z); (1, 0, 0, 0) = none), order L, flags. */
typedef struct {
    tcm_mol_id a;
    tcm_mol_id b;
    double R[3];
    double quat_b[4];
    int32_t L;
    int32_t flags;
} tcm_pair_req;

/* Energies of npairs requests in one batched run: the eq. 8 moments of every molecule the
 * batch names are computed on the device (or reused, per TCM_REUSE) with the molecules of each
 * (precision, L) group in one launch, then every pair's eq. 9 (square truncation, or
 * triangular with TCM_TRIANGULAR) is evaluated after the eq. 2 test (|R0| > a_A + a_B, else
 * TCM_EDOMAIN for that item).  U_out[npairs], status_out[npairs] (host).  Returns TCM_OK if
 * every item succeeded, else the first failing item's code.  Synchronous. */
int tcm_batch_energy(tcm_ctx *ctx, const tcm_pair_req *reqs, int64_t npairs, double *U_out,
                     int32_t *status_out);

/* Plan a batch once.  Its launches: one statistics launch for the whole batch, centre/scale,
 * the tile launch of each (precision, L) group, moment finalisation, pairs.  use_graph != 0:
 * they are captured in a HIP graph in that serial order and tcm_plan_run replays the graph;
 * use_graph == 0: tcm_plan_run issues them directly, the groups' tile launches spread over
 * the context's stream and one forked stream (balanced by work) so that their workgroups
 * interleave.  Either way the run is asynchronous on the context's stream (outputs stay on
 * the device until tcm_plan_results), every moment the batch needs is recomputed (no
 * TCM_REUSE), and the results are identical bit for bit.  The moments a plan computes count as
 * resident (for later TCM_REUSE calls on the same stream) once a run has been issued, at the
 * plan's order; until then a reuse recomputes them.  A live plan pins the molecules it names
 * (tcm_mol_release returns TCM_EAGAIN).  Destroy plans before their
 * context: their device memory is returned to its budget. */
int tcm_plan_create(tcm_ctx *ctx, const tcm_pair_req *reqs, int64_t npairs, int use_graph,
                    tcm_plan **plan_out);
/* A plan whose contractions take adaptive truncation (the rule of tcm_batch_energy_adaptive,
 * each request's L its maximum order, tol > 0): every run recomputes the moments, then chooses
 * each pair's order on the device from the requested one, lists the pairs again by chosen
 * order and contracts them -- the same launches, the same bits and the same orders as
 * tcm_batch_energy_adaptive on the same requests and moments.  sum |q| of each molecule is
 * computed when the plan is created (once per molecule, as there).  Runs, results and
 * destruction as for tcm_plan_create; tcm_plan_orders reads the chosen orders and bounds. */
int tcm_plan_create_adaptive(tcm_ctx *ctx, const tcm_pair_req *reqs, int64_t npairs, double tol,
                             int use_graph, tcm_plan **plan_out);
int tcm_plan_run(tcm_ctx *ctx, tcm_plan *plan);
/* The serial-order launches issued directly (no graph); results are identical bit for
 * bit. */
int tcm_plan_run_phased(tcm_ctx *ctx, tcm_plan *plan);
/* One synchronous run with HIP events recorded on the launch stream between its steps;
 * ms_out[4] receives the elapsed milliseconds of (statistics + centre/scale), (moment
 * tiles), (moment finalisation), (pair rotation + contraction). */
int tcm_plan_run_timed(tcm_ctx *ctx, tcm_plan *plan, double *ms_out);
/* Wait for the last run and copy U/status to the host (either may be NULL). */
int tcm_plan_results(tcm_ctx *ctx, tcm_plan *plan, double *U_out, int32_t *status_out);
/* Adaptive plans: wait for the last run and copy each pair's chosen order and its bound (as
 * tcm_batch_energy_adaptive reports them; either may be NULL).  TCM_EINVAL for other plans. */
int tcm_plan_orders(tcm_ctx *ctx, tcm_plan *plan, int32_t *L_out, double *bound_out);
/* Device addresses of the plan's outputs (FP64 U[npairs], int32 status[npairs]). */
int tcm_plan_device_outputs(tcm_plan *plan, double **d_U, int32_t **d_status);
/* Work counts of the plan: atoms, moment flops (algorithmic convention 6(L+1)(L+2) per
 * atom), tile items, pair items. */
int tcm_plan_info(tcm_plan *plan, int64_t *atoms, double *moment_flops, int64_t *tiles,
                  int64_t *pairs);
void tcm_plan_destroy(tcm_plan *plan);

/* ---- translation scan ------------------------------------------------------------ */

/* Energies of molecule B at nR positions relative to A (the scan of the paper's section IV,
 * in any directions), B keeping one orientation: quat_b (w, x, y, z), NULL = identity, as in
 * tcm_pair_req.  R: FP64 [nR][3], each c_B - c_A.  Eq. (9) with l1, l2 <= L (l1 + l2 <= L with
 * TCM_TRIANGULAR in flags) regrouped by L' = l1 + l2: the pair tensor G_{L'M} = sum over
 * l1 + l2 = L', m1 + m2 = M of
 * (-1)^{l2} Q^A_{l1 m1} Q^B_{l2 m2} (with the factorial normalisation) is built once from the
 * moments (computed, or reused with TCM_REUSE in flags), and each position then costs
 * O(L^2) instead of the O(L^4) of a full contraction.  U_out[nR], status_out[nR]:
 * TCM_EDOMAIN (and NaN) where |R| <= a_A + a_B unless TCM_UNCHECKED, TCM_EINVAL where R is
 * zero or not finite.  With TCM_DEVICE_IO, R / U_out / status_out are device pointers and the
 * call returns once the launches are queued on the context's stream (R must be complete on
 * the device before that stream reaches the launches); otherwise they are host arrays and the
 * call is synchronous.  Returns TCM_ENOTFOUND for an unknown id, TCM_EINVAL
 * for bad arguments. */
int tcm_scan_translations(tcm_ctx *ctx, tcm_mol_id a, tcm_mol_id b, int L, const double *quat_b,
                          int flags, const double *R, int64_t nR, double *U_out,
                          int32_t *status_out);

/* Adaptive truncation: each request's L is its maximum order; the pair is contracted at the
 * smallest order L' <= L whose rigorous truncation bound
 *   S_A S_B / (R (1 - alpha - beta)) [(alpha/(1-beta))^{L'+1} + (beta/(1-alpha))^{L'+1}]
 * (alpha = a_A/R, beta = a_B/R, S = sum |q|; it bounds |eq. (1) - eq. (9) at L'|; with
 * TCM_TRIANGULAR in the request's flags the bound of that truncation,
 * S_A S_B t^{L'+1} / (R (1 - t)), t = alpha + beta) is <= tol,
 * or at L when none is.  The moments are computed (or reused with TCM_REUSE) at L and stay
 * resident; sum |q| is computed once per molecule and cached with its moments.  U_out,
 * status_out: as tcm_batch_energy; L_out (may be NULL): the order used (-1 on error);
 * bound_out (may be NULL): the bound at that order (above tol when L was not enough; NaN on
 * error).  The bound covers truncation only, not the rounding of the moment pass.  tol > 0. */
int tcm_batch_energy_adaptive(tcm_ctx *ctx, const tcm_pair_req *reqs, int64_t npairs, double tol,
                              double *U_out, int32_t *L_out, double *bound_out, int32_t *status_out);

/* Forces and torques of the truncated energy of one pair (the paper names forces between the
 * fragments as the other use of its final expression; the derivatives are those of eq. (9)
 * as truncated, l1, l2 <= L).  Request fields as in tcm_pair_req; flags: TCM_REUSE,
 * TCM_UNCHECKED, TCM_DEVICE_IO.  out[10] (host): U, F_B[3] = -grad_R U (the force on B's
 * centre for a rigid translation of B; F_A = -F_B), tau_A[3] and tau_B[3] (torques about
 * each centre for a rigid rotation, tau = -dU/dtheta; tau_A + tau_B + R x F_B = 0).
 * forces_A / forces_B (may be NULL): FP64 [n][3] forces on each atom at fixed centres,
 * F_i = -dU/dx_i through eq. (8), B's in the posed frame (atoms at c_B + Rot(quat_b)(x - c_B));
 * host arrays, or device pointers with TCM_DEVICE_IO.  Per-atom forces are zero at L = 0.
 * Returns the pair's status: TCM_EDOMAIN when |R| <= a_A + a_B (out and host force arrays
 * NaN, device force arrays undefined), TCM_ENOTFOUND, TCM_EINVAL. */
int tcm_pair_forces(tcm_ctx *ctx, tcm_mol_id a, tcm_mol_id b, const double R[3], const double quat_b[4],
                    int L, int flags, double out[10], double *forces_A, double *forces_B);
/* tcm_pair_forces' out[10] for a batch of requests (no per-atom forces): out[npairs][10],
 * status_out[npairs]; failed items NaN.  Returns the first per-item error. */
int tcm_batch_forces(tcm_ctx *ctx, const tcm_pair_req *reqs, int64_t npairs, double *out,
                     int32_t *status_out);

/* Interaction energies of every pair of K resident fragments in place (the many-fragment
 * use of eq. (9) that the paper's outlook names): each fragment's moments once at order L
 * (reused with TCM_REUSE in flags), then the K(K-1)/2 contractions with R = c_j - c_i (no
 * pose; the centres are those of the moment pass, given or centroid).  U_out and
 * status_out: host arrays of K(K-1)/2 in row-major upper-triangle order, pair (i, j), i < j,
 * at index i*K - i*(i+1)/2 + (j - i - 1).  Pairs closer than a_i + a_j return TCM_EDOMAIN
 * (NaN) unless TCM_UNCHECKED; their interaction is outside the expansion's domain (eq. 2)
 * and left to the caller.  The system's inter-fragment energy is the sum of the valid
 * entries.  K <= 11585 (K(K-1)/2 <= 2^26).  Returns the first per-pair error, TCM_ENOTFOUND
 * for an unknown id, TCM_EINVAL for bad arguments. */
int tcm_all_pairs(tcm_ctx *ctx, const tcm_mol_id *ids, int64_t K, int L, int flags,
                  double *U_out, int32_t *status_out);

/* ---- tuning ------------------------------------------------------------------------ */

/* Sustained rate of plain (non-packed) vector FMA instructions on the context's device, in
 * TFLOP/s (an FMA counts two): 16 independent chains per thread on 32 workgroups of 256
 * threads per compute unit, five timed launches.  precision: TCM_F32C (FP32) or TCM_F64.
 * The ceiling against which the ALU-bound kernels are read (the datasheet FP32 figure
 * assumes packed FP32, which this library does not use). */
int tcm_alu_calibrate(tcm_ctx *ctx, int precision, double *tflops_out);

/* Atoms per thread per tile used for (precision, L, n); the tile is 256 * kper atoms.  For
 * TCM_F32C the value used is min(kper, the context's FP32 run cap, tcm_set_fp32_run).
 * tcm_tune_set returns TCM_EAGAIN while a server runs (a fragment's tiling, and so every
 * rounding of its moments, stays fixed while it is served). */
int tcm_tune_get(tcm_ctx *ctx, int precision, int L, int64_t n, int *kper_out);
int tcm_tune_set(tcm_ctx *ctx, int precision, int L, int64_t n, int kper);
/* Cap on the run of atoms one thread sums in plain FP32 in the TCM_F32C moment pass (its kper;
 * every sum above that is compensated).  The cap is part of that path's error bound: each
 * moment is within (8 (l+1) + 2 kmax + 64) 2^-24 of its absolute sum
 * sum_i |q_i| |r_i^l sqrt(4 pi/(2l+1)) Y_lm| (eq. 8), and a shorter run lowers the typical error
 * at the cost of more compensated merges.  1 <= kmax <= 1024; default 64.  The autotuners
 * only try FP32 tilings within the cap.  TCM_EAGAIN while a server runs. */
int tcm_set_fp32_run(tcm_ctx *ctx, int kmax);
/* Autotuner: time the moment-tile kernels for every candidate kper (8..256, powers of two,
 * FP32 within the run cap)
 * on a synthetic batch of copies of an n-atom molecule (at least 64M atoms, or 4096 copies)
 * so that every candidate runs many waves of items, and keep the fastest for (precision, L,
 * n's power-of-two size bucket).  best_ms_out (may be NULL): the winner's tile time per
 * molecule, in ms.  Device memory for the synthetic batch comes from the context's budget. */
int tcm_autotune(tcm_ctx *ctx, int precision, int L, int64_t n, int *best_kper_out,
                 double *best_ms_out);
/* Batch-aware autotuner: for each (precision, L) group of the molecules the requests name,
 * time that group's moment-tile launch on the batch itself for kper in 16..256 (one value
 * for all of the group's size buckets) and keep the fastest for every size bucket of the
 * group's molecules -- the tiling that fills the device for this batch's mix of sizes.
 * Requests are validated as by tcm_batch_energy (invalid ones are skipped); the molecules'
 * resident moments are invalidated (the next batch recomputes them).  best_ms_out (may be
 * NULL): the sum of the groups' best tile times, in ms.  A tiling is still a function of
 * (precision, L, n), so results stay identical alone and in any mix. */
int tcm_autotune_batch(tcm_ctx *ctx, const tcm_pair_req *reqs, int64_t npairs, double *best_ms_out);
/* Persist / restore the tuning table (text file). */
int tcm_tune_save(tcm_ctx *ctx, const char *path);
int tcm_tune_load(tcm_ctx *ctx, const char *path);

/* ---- serving ----------------------------------------------------------------------- */

/* A served pair-energy request.  Fragments are named by caller-chosen keys.  A fragment the
 * server already holds (moments resident in its cache) is reused: its moments are computed
 * once per order and kept for later poses and partners.  A fragment that is not resident must
 * come with its atoms (FP64 structure of arrays x, y, z, q; device pointers, or host pointers
 * with TCM_HOST_ATOMS), which the server copies into memory it owns, so the caller may reuse
 * the arrays once the request completes (or, with TCM_BORROW_ATOMS, references in place).
 * New fragments become resident under an LRU policy bounded by the context's HBM budget:
 * under pressure the atoms of idle fragments are evicted first while their moment tables
 * (fixed-size slots of a device arena, 8.7 KB each) stay, so a fragment is served at any order
 * it already holds after its atoms are gone; a higher order then needs its atoms again (a
 * request that names them; else TCM_ENOTFOUND). */
#define TCM_HOST_ATOMS   4  /* request flag: atoms_a / atoms_b are host pointers (copied)    */
#define TCM_BORROW_ATOMS 8  /* request flag: device atoms are referenced, not copied; they   */
                            /* must stay valid while the fragment is resident (until it is  */
                            /* evicted or the server stops)                                 */

typedef struct {
    int64_t key_a;
    int64_t key_b;
    const double *atoms_a[4];      /* x, y, z, q of fragment a when not resident, else NULL */
    int64_t n_a;
    const double *atoms_b[4];
    int64_t n_b;
    double R[3];                   /* c_b - c_a (centres are the fragments' centroids)       */
    double quat_b[4];              /* pose of b, unit quaternion (w, x, y, z)                */
    int32_t L;
    int32_t flags;                 /* TCM_UNCHECKED, TCM_HOST_ATOMS                          */
    int32_t precision;             /* moment pass of new fragments (TCM_F32C or TCM_F64)     */
    int32_t pad;
} tcm_request;

typedef struct {
    int32_t max_inflight_batches;  /* launches in flight at once, each on its own stream      */
    int32_t max_batch_pairs;       /* requests admitted into one launch                       */
    int32_t queue_capacity;        /* pending requests before tcm_submit returns TCM_EAGAIN   */
    int32_t pad;
} tcm_server_cfg;

/* Start the serving thread (one per context).  Requests that arrive while launches are in
 * flight are admitted into the next launch as soon as a launch slot and memory are free, so
 * the work of several batches overlaps on the device.  A request whose fragment is still
 * being computed by an in-flight launch waits for it and then reuses the result. */
int tcm_server_start(tcm_ctx *ctx, const tcm_server_cfg *cfg);
/* Enqueue a request; returns a ticket.  TCM_EAGAIN when the queue is full, TCM_EINVAL for a
 * malformed request.  Thread-safe with respect to tcm_poll and other submitters. */
int tcm_submit(tcm_ctx *ctx, const tcm_request *req, uint64_t *ticket_out);
/* Non-blocking: TCM_EAGAIN while pending; on completion writes U (NaN on failure), the item
 * status and the latency (seconds from submit to completion observed by the server) and
 * forgets the ticket.  TCM_ENOTFOUND for an unknown ticket. */
int tcm_poll(tcm_ctx *ctx, uint64_t ticket, double *U_out, int32_t *status_out,
             double *latency_s_out);
/* Stop accepting requests, finish the ones admitted or pending, join the serving thread and
 * free the server's cache. */
int tcm_server_stop(tcm_ctx *ctx);
/* Counters since start: completed requests, launches, fragment cache hits / misses,
 * requests that had to wait at least once (memory, or a fragment still in flight), atom
 * evictions (a fragment's atoms freed to make room; its moment table stays resident, so the
 * fragment is still served at any order up to the one it holds), fragments dropped whole
 * (moment table included: the moment arena could not grow), and requests that failed with
 * TCM_ENOTFOUND because they needed an order above the resident one of a fragment whose atoms
 * had been evicted and did not bring them again.  A request is admitted with both of its
 * fragments or waits without fetching either.  Any pointer may be NULL. */
int tcm_server_stats(tcm_ctx *ctx, int64_t *completed, int64_t *launches, int64_t *cache_hits,
                     int64_t *cache_misses, int64_t *deferred, int64_t *evictions, int64_t *dropped,
                     int64_t *evicted_misses);

#ifdef __cplusplus
}
#endif

#endif /* TCM_H */
