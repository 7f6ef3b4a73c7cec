/*
 * mirve.h -- C ABI of the MI355X FFT phase-field-fracture toughness solver.
 *
 * The library computes the effective fracture toughness of a periodic voxel
 * RVE following Aranda & Segurado, "Effective toughness estimation by FFT
 * based phase field fracture" (arXiv 2508.07424):
 *   - degraded elastic law sigma = g(phi) C^r : eps with g = (1-phi)^2 + k
 *     (Sec. 2.1 Eq. 2, Sec. 2.2 Eq. 12-13),
 *   - Fourier-Galerkin equilibrium with the compatible-strain projection
 *     (Sec. 4.1 Eq. 24 R1, Eq. 26),
 *   - AT2 damage balance with history (Eq. 10b, 11, 16b, 38),
 *   - dissipation control: the macroscopic strain E_M = f E (Eq. 9) is the
 *     unknown that makes D(phi) = tau (Eq. 10c / 16c),
 *   - crack-tip enrichment of the initial notch (Sec. 4.3 Eq. 35, 37a, 38),
 *   - G_eff = V (T^f - 1/2 Sigma^f E^f) / A_g (Sec. 4.2 Eq. 32-33).
 *
 * Conventions
 *   - Every function returns RVE_OK (0) or a negative RVE_E* code; the text
 *     of the last error of a handle is available from rve_last_error().
 *   - Grids: n[0] = n_x, n[1] = n_y, n[2] = n_z (n_z = 1 in 2D).  Host
 *     arrays of voxel data are C-ordered with x fastest:
 *     index = (z * n_y + y) * n_x + x.  Multi-component fields put the
 *     component slowest: [c][z][y][x].
 *   - Symmetric tensors are Mandel vectors: 2D plane strain
 *     [xx, yy, sqrt2 xy] (s = 3); 3D [xx, yy, zz, sqrt2 yz, sqrt2 xz,
 *     sqrt2 xy] (s = 6).
 *   - The library never allocates device memory.  The caller passes a
 *     device workspace of at least rve_query_workspace() bytes and a HIP
 *     stream (hipStream_t, or NULL for the default stream); both must
 *     outlive the handle.  Host input arrays are copied during the call.
 *   - A handle is not thread-safe.  Distinct handles may run concurrently
 *     on distinct streams.
 *   - Steps are transactional: a step that fails leaves the committed state
 *     (phi, history, E, curve) as it was when the step began.  A step whose
 *     solve fails (any iteration limit, a stalled stagger or a breakdown) is
 *     first redone as two steps of half the increment, recursively, down to
 *     cfg.max_halvings levels; dissipation control allows any subdivision of
 *     the increment (Sec. 4.1).
 *   - A handle holds cfg.batch RVE slots of the same grid, each with its own
 *     microstructure, state and convergence.  Kernel launches cover the
 *     slots that are in the same phase of their step; a slot that finishes a
 *     step goes on with its next one while others still iterate.  The
 *     functions without a slot argument address slot 0
 *     (rve_step_dissipation needs batch = 1).
 */
#ifndef MIRVE_H
#define MIRVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define RVE_OK        0
#define RVE_EINVAL   -1   /* invalid argument or configuration            */
#define RVE_ENOSPC   -2   /* workspace smaller than rve_query_workspace() */
#define RVE_EDEVICE  -3   /* HIP runtime error                            */
#define RVE_ENOCONV  -4   /* an iteration hit its limit (state unchanged) */
#define RVE_ENUMERIC -5   /* NaN / Inf met in a reduction                 */
#define RVE_ESTATE   -6   /* call out of order (e.g. step before set_microstructure) */
#define RVE_ENOTDONE -7   /* no fracture point reached yet                */

/* why a step failed (rve_step_info.reason) */
#define RVE_WHY_NONE      0
#define RVE_WHY_STAGGER   1  /* staggered fixed point: max_stagger reached, or stalled
                                (its error not halved within stall_window iterations) */
#define RVE_WHY_CG        2  /* mechanics CG reached max_cg                         */
#define RVE_WHY_PCG       3  /* damage PCG reached max_pcg                          */
#define RVE_WHY_ARCLENGTH 4  /* the dissipation constraint's root finder reached
                                its iteration limit                                */
#define RVE_WHY_SPLIT     5  /* the split law's Newton loop reached its limit       */
#define RVE_WHY_BREAKDOWN 6  /* Krylov breakdown or a non-finite reduction          */
#define RVE_WHY_ANDERSON  7  /* singular or non-finite Anderson system              */
#define RVE_WHY_GMRES     8  /* Newton step: GMRES reached max_cycles restarts      */
#define RVE_WHY_NEWTON    9  /* Newton step: max_newton iterations without Eq. 30   */

/* flags of rve_run_slots and rve_run_budget */
#define RVE_RUN_STOP_AT_FRACTURE 1  /* a slot stops after the step that reaches its
                                       fracture point (and takes none once there)   */
#define RVE_RUN_KEEP             2  /* rve_run_budget only: see there                 */

/* precision modes */
#define RVE_PREC_FP64  0  /* every field and transform in FP64                        */
#define RVE_PREC_MIXED 1  /* fields, FFTs, constitutive and Krylov updates in FP32;
                             reductions, the arc-length solve and curve in FP64; the
                             damage solution of the arc-length solve is held in FP64
                             and refined to tol_pcg (FP64 residual, FP32 corrections);
                             the stagger also ends when its error is within 10 tol and
                             has not halved for 20 iterations (the noise floor that
                             the FP32 mechanics solve leaves)                      */

/* tension / compression split of the elastic energy */
#define RVE_SPLIT_NONE   0 /* the paper's model: sigma = g C:eps, psi = 1/2 eps:C:eps  */
#define RVE_SPLIT_VOLDEV 1 /* volumetric split: only K<tr eps>_+^2 and the deviatoric
                              energy are degraded and drive damage                  */

/* preconditioner of the damage solve (Eq. 16b) */
#define RVE_PRECOND_FFT    0 /* diag^-1/2 F^-1 [1 / (abar + bbar |d(xi)|^2)] F diag^-1/2, with
                                abar = mean(Gc/l + 2H), bbar = mean(Gc) l and d the
                                forward-difference symbols (the default)                */
#define RVE_PRECOND_JACOBI 1 /* the inverse diagonal of the damage operator          */

/* phase kinds */
#define RVE_PHASE_ISO   0  /* isotropic: E, nu                                */
#define RVE_PHASE_CUBIC 1  /* cubic: C11, C12, C44 in lattice axes; rotated by
                              the per-voxel in-plane angle theta (Eq. 13)     */

/* fields for rve_get_field / rve_set_field (host arrays of doubles) */
#define RVE_FIELD_PHI     0  /* damage phi (committed)                 N values   */
#define RVE_FIELD_HIST    1  /* history H^n (committed)                N          */
#define RVE_FIELD_PSI_INI 2  /* initial-crack energy psi_ini (Eq. 37a)  N          */
#define RVE_FIELD_EPS1    3  /* unit-load strain f + eps~_1             s * N      */
#define RVE_FIELD_SIG1    4  /* unit-load stress g C:eps_1              s * N      */
#define RVE_FIELD_PSI1    5  /* unit-load energy density psi_o1         N          */
#define RVE_FIELD_PHI_INI 6  /* enriched initial damage (Eq. 35)        N          */

typedef struct rve_handle_s* rve_handle;

typedef struct {
    int    dim;            /* 2 (plane strain) or 3                                  */
    int    n[3];           /* grid; each n_i in [2, 1024]; n[2] = 1 when dim = 2     */
    double h;              /* voxel size (> 0)                                       */
    double ell;            /* phase-field length l (> 0)                             */
    double k_res;          /* residual stiffness k in g = (1-phi)^2 + k (> 0)        */
    double f[6];           /* Mandel load direction f of E_M = f E (first s used)    */
    int    split;          /* RVE_SPLIT_*                                            */
    int    history;        /* 1: H = max(psi_o + psi_ini, H^n) (Eq. 38); 0: no max   */
    int    precision;      /* RVE_PREC_*                                             */
    /* tolerances; 0 takes the default of the precision mode:
       FP64  tol 1e-8, tol_cg 1e-10, tol_pcg 1e-12, tol_al 1e-10;
       MIXED tol 1e-5, tol_cg 1e-6,  tol_pcg 1e-10, tol_al 1e-6                       */
    double tol;            /* stagger tolerance on the relative change of phi and E  */
    double tol_cg;         /* mechanics CG: ||r|| <= tol_cg ||b||                    */
    double tol_pcg;        /* damage PCG: ||r|| <= tol_pcg ||rhs||                   */
    double tol_al;         /* dissipation constraint: |D - tau| <= tol_al tau        */
    int    max_stagger;    /* stagger iteration limit per step attempt               */
    int    max_halvings;   /* a failed step attempt is redone as two of half the
                              increment, at most this many levels deep (0-12)       */
    int    stall_window;   /* an attempt whose stagger error has not halved within
                              this many iterations counts as failed (0, the
                              default: off)                                       */
    int    max_cg;         /* CG iteration limit per mechanics solve                 */
    int    max_pcg;        /* PCG iteration limit per damage solve                   */
    int    anderson_depth; /* Anderson acceleration depth of the stagger (0 = off)   */
    double frac_threshold; /* phi at which a voxel counts as broken (0.95)           */
    double A_g;            /* reference crack area; 0 = lines along the load axis
                              without a notch voxel, times h^(dim-1) (Eq. 32)        */
    int    max_materials;  /* capacity of the per-material table: distinct
                              (phase, theta, notch) combinations, <= 65536          */
    int    batch;          /* RVE slots of this handle (same grid, own microstructure
                              and state), advanced together by every launch; 1-1024  */
    int    damage_precond; /* RVE_PRECOND_* of the damage solve                      */
    int    graphs;         /* 1 (default): run the Krylov iterations as replays of
                              captured HIP graphs (chunks of 8 iterations) when the
                              handle has a stream of its own; 0: launch them       */
    int    streaming;      /* cache policy of the Krylov x passes' r, p, x: -1
                              (default) chosen from the batch's footprint and by
                              rve_autotune; 0 cached loads and stores; 1
                              non-temporal ones (arithmetic is the same)          */
} rve_config;

typedef struct {
    int    kind;           /* RVE_PHASE_ISO or RVE_PHASE_CUBIC */
    double E, nu;          /* isotropic constants              */
    double C11, C12, C44;  /* cubic constants (lattice axes)   */
    double Gc;             /* critical energy release rate     */
    double beta;           /* cleavage anisotropy A_f = I + beta (I - n (x) n) of the
                              crack-surface density (Sec. 2.2, Eq. 14-17, 36-37b):
                              the damage gradient term becomes Gc l/2 grad phi . A
                              grad phi in D, the damage operator and the enrichment;
                              0 = isotropic; must be finite and > -1               */
    double n[3];           /* weak-plane normal in lattice axes (beta != 0), rotated
                              with the voxel's theta about z; in 2D its projection on
                              the plane is used, normalised (along z: A = (1+beta) I);
                              in 3D it must be non-zero                            */
} rve_phase;

typedef struct {
    double E;              /* macroscopic strain scalar of the step (Eq. 9)          */
    double Sigma;          /* <sigma>:f                                              */
    double D;              /* dissipation functional D(phi) (Eq. 3)                  */
    double Gamma;          /* crack surface Gamma(phi) (Eq. 4)                       */
    double tau;            /* imposed dissipation tau^{n+1}                          */
    double T;              /* trapezoid of Sigma dE up to this step (Eq. 33)         */
    int    n_stagger;      /* stagger iterations                                     */
    int    n_cg;           /* mechanics CG iterations                                */
    int    n_pcg;          /* damage PCG iterations                                  */
    int    n_greenop;      /* Green-operator applications                            */
    double res_R1;         /* ||P[sigma]|| / ||sigma|| at the committed state        */
    double res_R2;         /* ||damage residual|| / ||2H|| at the committed state    */
    double res_R3;         /* |D - tau| / tau                                        */
    int    fractured;      /* 1 once every line along the load axis is broken        */
    int    step;           /* index of the committed step (1, 2, ...)                */
    int    n_steps;        /* steps committed by the call                            */
    int    n_substeps;     /* committed sub-steps (a step split by halving has > 1;
                              those of a step that then failed count, though the
                              failure rolled them back)                            */
    int    reason;         /* RVE_WHY_* of a failed step, else RVE_WHY_NONE          */
    double G_inst;         /* instantaneous energy release rate of the step (Sec. 4.2,
                              Eq. 34): V [(T - 1/2 Sigma E)^n - (T - 1/2 Sigma E)^(n-1)]
                              / (Gamma^n - Gamma^(n-1)), the dissipated part of the
                              curve over the growth of the crack surface; NaN when
                              Gamma did not grow or no step was committed        */
} rve_step_info;
/* E .. step describe the last step the call committed (the committed state
 * when it committed none).  The counters n_stagger, n_cg, n_pcg, n_greenop
 * sum all the work of the call, failed attempts included. */

/* Fill cfg with defaults (tolerances, limits, FP64, no split, history on). */
int rve_default_config(rve_config* cfg);

/* Bytes of device workspace a handle of this configuration needs (its HBM
 * footprint; used for admission by a serving loop). */
int rve_query_workspace(const rve_config* cfg, size_t* bytes);

/* Create a handle bound to a caller-owned device workspace and stream.
 * Computes the plan (FFT factors, twiddles, launch shapes).  No compute. */
int rve_create(const rve_config* cfg, void* dev_workspace, size_t workspace_bytes,
               void* hip_stream, rve_handle* out);

int rve_destroy(rve_handle h);

/* Microstructure and initial crack (Sec. 2, 4.3).
 *   phase_id  N uint16, index into phases[0 .. nphases-1]
 *   phases    nphases phase descriptions (copied)
 *   theta     N doubles, in-plane lattice angle per voxel, or NULL (= 0);
 *             cubic stiffness is rotated by it about z (Eq. 13)
 *   void_mask N uint8 or NULL: notch voxels (stiffness k C, no driving force)
 *   phi_disc  N uint8 or NULL: sharp enrichment points of Eq. 35
 *   phi_M     maximum of the enriched initial damage (Eq. 35), in (0, 1)
 * Computes phi_ini, psi_ini, H^0 = psi_ini and tau^0 = D(phi_ini) on the
 * device and resets the loading curve.  Synchronises the stream. */
int rve_set_microstructure(rve_handle h, const uint16_t* phase_id, const rve_phase* phases,
                           int nphases, const double* theta, const uint8_t* void_mask,
                           const uint8_t* phi_disc, double phi_M);

/* Same for one slot of a batched handle; slot in [0, batch). */
int rve_set_microstructure_slot(rve_handle h, int slot, const uint16_t* phase_id,
                                const rve_phase* phases, int nphases, const double* theta,
                                const uint8_t* void_mask, const uint8_t* phi_disc, double phi_M);

/* Same with three Euler angles per voxel in place of theta (Sec. 5.3: grain
 * orientations drawn in three dimensions, stiffness and cleavage normal
 * rotated accordingly): euler[3 i + 0..2] = (a1, a2, a3) of voxel i, the
 * lattice-to-sample rotation R = R_z(a1) R_x(a2) R_z(a3) (z-x-z), so that
 * (a1, 0, 0) is the in-plane angle a1 of rve_set_microstructure.  A
 * one-voxel plate of the paper is the 3D grid with n_z = 2 and a
 * microstructure that does not vary along z: the solution is then
 * z-independent and, per unit thickness, the plate's; its damage gradients
 * lie in the plane, so the cleavage tensor acts through its in-plane block
 * (the projection of the rotated normal on the cross section).  Errors as
 * rve_set_microstructure; RVE_EINVAL for a null euler or a non-finite
 * angle. */
int rve_set_microstructure_euler(rve_handle h, int slot, const uint16_t* phase_id,
                                 const rve_phase* phases, int nphases, const double* euler,
                                 const uint8_t* void_mask, const uint8_t* phi_disc, double phi_M);

/* One dissipation-controlled step tau^{n+1} = tau^n + dtau (Eq. 16): the
 * staggered fixed point of equilibrium, damage and the constraint, then
 * commit and the fracture test.  out may be NULL.  Needs batch = 1. */
int rve_step_dissipation(rve_handle h, double dtau, rve_step_info* out);

/* One step of every slot b with dtau[b] > 0 (dtau[b] = 0: the slot idles).
 * dtau, info (may be NULL) and status (may be NULL) have `batch` entries;
 * each slot's step is transactional on its own.  Returns RVE_OK if every
 * stepped slot succeeded, else the first failure code. */
int rve_step_dissipation_slots(rve_handle h, const double* dtau, rve_step_info* info,
                               int* status);

/* Up to max_steps[b] steps of dtau[b] for every slot b with max_steps[b] > 0
 * and dtau[b] > 0, each slot at its own pace (Eq. 16; the batched form): a
 * slot that commits a step starts its next one while other slots are still
 * iterating theirs.  A slot stops at its first failed step (status[b] then
 * holds its code and info[b].reason the cause; the steps before it stay
 * committed) or, with RVE_RUN_STOP_AT_FRACTURE, after the step that reaches
 * its fracture point.  info and status may be NULL.  Returns RVE_OK if no
 * slot failed, else the first failure code. */
int rve_run_slots(rve_handle h, const double* dtau, const int* max_steps, int flags,
                  rve_step_info* info, int* status);

/* The batched form under a step budget (Eq. 16 per slot): every slot b with
 * dtau[b] > 0 takes steps of dtau[b] at its own pace, at most max_steps[b]
 * (max_steps may be NULL: no limit), until the slots together have
 * committed total_steps steps; the call then ends at the end of that round.
 * Slots that finish early keep the batch busy instead of waiting for the
 * slowest one.  A slot in the middle of a step at the end:
 *   - without RVE_RUN_KEEP returns to the state the step began from (its
 *     step does not happen) and its work counters drop that step's work;
 *   - with RVE_RUN_KEEP keeps the step in flight on the handle (its working
 *     fields stay on the device; the committed state and the scalars are
 *     those before the step).  The next rve_run_budget call with
 *     RVE_RUN_KEEP, max_steps[b] > 0 and the same dtau[b] resumes it where it
 *     stopped, bit for bit as if the calls had been one; the counters of each
 *     call cover the work that call did.  Any other call that reads or
 *     changes the slot (rve_get_*, rve_set_*, checkpoints, the stage-level
 *     forms, rve_step_*, rve_run_slots, a budget run without the flag or
 *     with another dtau, rve_release_slot, rve_effective_toughness*,
 *     rve_profile_pass, rve_autotune) first returns it to the step's start,
 *     as without the flag.
 * A slot stops at a failed step as in rve_run_slots, and with
 * RVE_RUN_STOP_AT_FRACTURE at its fracture point.  info (n_steps per slot)
 * and status as in rve_run_slots.  rve_run_stats reports the call's
 * occupancy.  Returns RVE_EINVAL for total_steps < 0 or unknown flags. */
int rve_run_budget(rve_handle h, const double* dtau, const int* max_steps, long long total_steps,
                   int flags, rve_step_info* info, int* status);

/* Occupancy of the handle's last rve_run_slots or rve_run_budget call: out2[0] = rounds (each
 * round is one launch sequence - a mechanics solve, then one stagger
 * iteration or commit - over the slots that are in that phase of their
 * step), out2[1] = the mean fraction of the batch's slots those rounds
 * covered (1 when every slot was busy in every round; lower while slots
 * that finished wait for others). */
int rve_run_stats(rve_handle h, double* out2);

/* Number of slots of the handle. */
int rve_batch_size(rve_handle h);

/* Forget a slot's microstructure and state (the slot can be set again). */
int rve_release_slot(rve_handle h, int slot);

/* Advance several independent handles by one step each, overlapping their
 * device work (each handle must have its own stream). info may be NULL;
 * status[i] receives each handle's return code. Returns RVE_OK if all did. */
int rve_step_dissipation_batch(rve_handle* hs, int count, const double* dtau,
                               rve_step_info* info, int* status);

/* G_eff = V (T^F - 1/2 Sigma^F E^F) / A_g at the fracture point F
 * (Eq. 32-33).  RVE_ENOTDONE before F. */
int rve_effective_toughness(rve_handle h, double* G_eff);
int rve_effective_toughness_slot(rve_handle h, int slot, double* G_eff);

/* Copy a field (RVE_FIELD_*) to / from a host array of doubles in the host
 * layout above.  count must equal the field's size.  Setting PHI or HIST
 * replaces the committed state (used for checkpoints and tests). */
int rve_get_field(rve_handle h, int which, double* host, size_t count);
int rve_set_field(rve_handle h, int which, const double* host, size_t count);
int rve_get_field_slot(rve_handle h, int slot, int which, double* host, size_t count);
int rve_set_field_slot(rve_handle h, int slot, int which, const double* host, size_t count);

/* Checkpoint of one slot's committed state (phi, history H^n, the committed
 * strain fluctuation, the warm start of the arc-length tangent, and the
 * scalars E, Sigma, T, tau, tau0, Gamma, step, fractured) as an opaque host blob of
 * rve_state_bytes() bytes.  rve_load_state needs a handle of the same grid
 * and precision whose slot already holds the same microstructure
 * (rve_set_microstructure_slot); stepping on from a loaded state gives the
 * same results, bit for bit, as stepping on from the saved one. */
int rve_state_bytes(rve_handle h, size_t* bytes);
int rve_save_state(rve_handle h, int slot, void* host, size_t bytes);
int rve_load_state(rve_handle h, int slot, const void* host, size_t bytes);

/* Scalars of the committed state: out[0..5] = {E, Sigma, T, tau, tau0, step}.
 * The slot form also returns out[6] = fractured and out[7] = A_g (8 values). */
int rve_get_scalars(rve_handle h, double* out6);
int rve_set_scalars(rve_handle h, const double* in6);
int rve_get_scalars_slot(rve_handle h, int slot, double* out8);
int rve_set_scalars_slot(rve_handle h, int slot, const double* in6);

/* Green operator (Eq. 24 R1): out = F^-1{ P : F[ g(phi) C : eps ] } at the
 * committed phi, for eps given as s*N host doubles.  Used for parity. */
int rve_apply_green_op(rve_handle h, const double* eps_host, double* out_host);

/* Device-resident variant for benchmarking: eps and out are device arrays
 * of batch*s*N elements of the handle's bulk type (double, or float in MIXED
 * mode), one block of s*N per slot; `repeat` applications over every slot
 * with a microstructure are enqueued on the handle's stream. */
int rve_apply_green_op_device(rve_handle h, const void* eps_dev, void* out_dev, int repeat);

/* Size of the static device array behind rve_apply_green_op_device_noalloc
 * (one array per device the library runs on, held until the process ends). */
#define RVE_NOALLOC_SCRATCH_BYTES (64u << 20)

/* Allocation-free form of rve_apply_green_op_device, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same operation, arguments, layout and
 * result as rve_apply_green_op_device; the intermediate spectrum and the
 * per-block partial sums of its passes live in the library's static device
 * array of RVE_NOALLOC_SCRATCH_BYTES bytes instead of the handle's
 * workspace.  The call allocates nothing (no hipMalloc, hipFree or other
 * allocating routine) and enqueues its work on the handle's stream.
 *   Limit: the handle needs 16 (FP64) or 8 (MIXED) bytes x s x (n_x/2+1) x
 *   n_y x n_z x batch of spectrum plus 8 bytes per x-pass block and slot;
 *   a larger handle is refused with RVE_ENOSPC before any work.
 *   Sharing: every call on one device uses the same array and leaves its
 *   contents behind (nothing in it needs to start cleared).  Calls ordered
 *   on one stream are safe; calls that overlap in time on one device (other
 *   streams, other host threads) race on the array and give wrong results.
 *   Errors: RVE_EINVAL for a null handle or pointer or repeat < 0;
 *   RVE_EDEVICE if the array's address could not be obtained when the
 *   handle was created. */
int rve_apply_green_op_device_noalloc(rve_handle h, const void* eps_dev, void* out_dev, int repeat);

/* ---- the paper's monolithic per-step solver (Sec. 4.1, Eq. 22-31) ----
 * One dissipation-controlled step of slot `slot` by Newton-Raphson on
 * q = (x, phi, E): the residual R = (R1, R2, R3) of Eq. 24 (equilibrium
 * Gamma[g C (x + E f)], the damage balance with H = max(psi0 + psi_ini,
 * H^n) of Eq. 38, and D(phi) - tau^(n+1)), the Jacobian J1-J3 of Eq. 25
 * applied matrix-free (J1 through the Green operator, J2 through the damage
 * stencil, J3 as a reduction), each Newton system J dq = -R solved by
 * restarted GMRES, the relaxation of Eq. 31 and the convergence test of
 * Eq. 30.  It reaches the fixed point of the staggered step (rve_step_*),
 * which it can replace step for step on the same handle; the commit (Eq. 33,
 * 38, fracture test, Eq. 34) is the same.
 * FP64 handles without a split law only (RVE_EINVAL otherwise).
 * Readings: the relaxation factor of Eq. 31 is
 * alpha = max(theta, Sigma^n / max_(j<n) Sigma^j), 1 for the first two
 * steps; dH/deps = sigma0 where psi0 + psi_ini >= H^n and psi0 > 0 (not on
 * notch voxels); from the unloaded state (E = 0, where J is singular) Newton
 * starts from the elastic unit-load solution scaled to
 * E = sqrt(min G_c / (l max psi_o1)).  The paper names BiCGSTAB for the
 * Newton systems; GMRES is used (BiCGSTAB diverged on them).
 * workspace: caller-owned device memory of at least rve_newton_workspace
 * bytes for opts->restart, not shared with a call in flight; opts may be
 * NULL (defaults).  A failed step (RVE_ENOCONV, RVE_ENUMERIC) leaves the
 * committed state unchanged and sets info->reason.  In info, n_stagger is
 * the Newton iteration count, n_cg the GMRES iterations (all systems),
 * n_greenop the Green-operator applications. */
typedef struct rve_newton_opts {
    double tol;          /* Eq. 30 tolerance; <= 0: the handle's tol               */
    double krylov_tol;   /* relative residual of each GMRES solve (1e-12); a restart
                            cycle that no longer halves the residual ends the solve
                            once it is below sqrt(krylov_tol) (rounding floor near
                            Newton's solution)                                    */
    double theta;        /* lower bound of the relaxation factor (0.3)              */
    int    restart;      /* GMRES restart length, 1..1000 (200)                     */
    int    max_cycles;   /* GMRES restart cycles per Newton system (100)            */
    int    max_newton;   /* Newton iterations (50)                                  */
    int    relax;        /* 1: relaxation of Eq. 31; 0: full Newton steps (1)       */
} rve_newton_opts;
void rve_newton_default_opts(rve_newton_opts* opts);
int rve_newton_workspace(rve_handle h, int restart, size_t* bytes);
int rve_step_newton(rve_handle h, int slot, double dtau, const rve_newton_opts* opts,
                    void* workspace, size_t workspace_bytes, rve_step_info* info);

/* Equilibrium for the unit load at the committed phi (Eq. 16a): updates
 * EPS1/SIG1/PSI1 and returns the CG iteration count and Sigma_1. */
int rve_solve_mechanics(rve_handle h, int* iterations, double* Sigma1);

/* Damage balance at load E with the current unit energy PSI1 and the
 * committed history (Eq. 16b, 38): returns D(phi(E)) and the PCG count;
 * phi(E) is left in the field returned by RVE_FIELD_PHI only if commit_phi. */
int rve_solve_damage(rve_handle h, double E, double* D, int* iterations, int commit_phi);

/* Dissipation D(phi) and crack surface Gamma(phi) of the committed phi. */
int rve_dissipation(rve_handle h, double* D, double* Gamma);

/* Benchmark helper: enqueue `repeat` launches of one kind of FFT pass of the
 * Green operator on the handle's stream (asynchronous) and report the
 * compulsory HBM bytes of one launch (every input read once, every output
 * written once).  pass: 0 x-forward with the constitutive law, 1 the axis
 * pass carrying the projection, 2 x-inverse (store), 3 x-forward with the CG
 * direction update, 4 x-inverse with the CG update, 5 the forward y pass of
 * a 3D operator (2D: as 1).  Works on scratch buffers; the committed state is
 * not changed. */
int rve_profile_pass(rve_handle h, int pass, int repeat, double* bytes_per_launch);

/* Autotuner of the launch shapes of the Green operator's passes (rows per
 * block of the x passes, lines per block of the y pass or, for 2D grids
 * with 256- or 512-point y lines, the one-wave y pass (one line position
 * per wave, every component; no block barrier), y columns per tile of the
 * 3D z pass) and, when the config's streaming is -1, of the streaming
 * policy of the Krylov x passes (non-temporal loads and stores of r, p, x,
 * which leave the last-level cache to the spectrum when the batch's vectors
 * do not fit it): times every
 * feasible choice's CG-mode passes `repeat` times on the handle's own slots
 * (at least one slot must be set) and keeps the fastest for the handle.  The
 * choice is cached for the process per (grid, batch, precision): later
 * handles of the same kind take it without timing.  shape_out (may be NULL)
 * receives four values: rows, lines (0 for the one-wave y pass), columns,
 * and 1 if the vectors are streamed non-temporally (else 0).  Results of the solver do not depend on
 * the choice beyond the summation order of the per-block partial sums. */
int rve_autotune(rve_handle h, int repeat, int* shape_out);

/* Message of the last error of h (or of the calling thread when h is NULL,
 * e.g. after a failed rve_create / rve_query_workspace). */
const char* rve_last_error(rve_handle h);
const char* rve_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MIRVE_H */
