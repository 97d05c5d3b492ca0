/*
 * tplbm.h -- C ABI of the MI355X (gfx950) thermal pseudopotential lattice
 * Boltzmann library.
 *
 * The method is the per-step lattice update of Czelusniak, Cabezas Gomez and
 * Wagner, arXiv 2301.12869, Sec. III ("Pseudopotential lattice Boltzmann
 * method"): the lattice Boltzmann equation (Eq. LBE) with the MRT collision
 * (Eqs. OperatorMRT, MatrixMRT, RelaxationMatrix), Li's forcing scheme
 * (Eq. LiFS), the force-corrected velocity (Eqs. Density, Momentum), the
 * second-order equilibrium (Eq. EquilibriumDistribution), the Shan-Chen
 * nearest-neighbour force (Eq. ShanChenForce) on the Yuan-Schaefer
 * pseudopotential (Eq. InteractionPotential) of the Carnahan-Starling EOS
 * (Eq. EOS), the gravity forms of Sec. II (Eqs. Gravity_1, Gravity_2, Gravity_3),
 * Zou-He no-slip wet-node walls with zero interaction force at the wall, and
 * the energy equation (Eq. Energy_Equation) with isotropic second-order
 * differences and a two-stage Runge-Kutta step.
 *
 * Conventions shared by every entry point
 *  - Status: every int-returning call returns TPLBM_OK (0) or one of the
 *    TPLBM_E* codes below; no call aborts the process or throws.  After a
 *    failure tplbm_last_error() gives a message.
 *  - Memory: the library never allocates device memory.  The caller passes
 *    one device workspace (size from the *_workspace_bytes call), keeps it
 *    alive until the matching destroy, and owns it.  Host arrays passed in
 *    are read or written during the call only and stay owned by the caller.
 *  - Streams: all device work is enqueued on the HIP stream given at create
 *    time (NULL = the legacy default stream).  Calls documented as
 *    synchronous wait for that stream before returning.
 *  - Layout (structure of arrays, x fastest): D2Q9 node (x, y) has linear
 *    index y*nx + x; D3Q19 node (x, y, z) has (z*ny + y)*nx + x; a D1Q3
 *    column node y has index y.  The wall-normal axis (walls at its first
 *    and last layer) is y in 2-D, z in 3-D and the column axis in 1-D; the
 *    other axes are periodic.  Gravity g > 0 points toward the first layer
 *    ("down").
 *  - Units: lattice units throughout; temperatures are absolute (multiply a
 *    reduced T/T_c by tplbm_eos_critical()'s T_c).
 */
#ifndef TPLBM_H
#define TPLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define TPLBM_OK 0
#define TPLBM_EINVAL 1          /* bad argument or parameter value */
#define TPLBM_ESHAPE 2          /* sizes do not fit the lattice or buffer */
#define TPLBM_EUNSUPPORTED 3    /* valid but not implemented (e.g. tau != 1 on D3Q19) */
#define TPLBM_EHIP 4            /* a HIP runtime call failed */
#define TPLBM_EUNPHYSICAL 5     /* NaN, rho <= 0, eta >= 1 or negative psi radicand seen */
#define TPLBM_ENOTCONVERGED 6   /* a host solve did not converge */
#define TPLBM_ENOSOLUTION 7     /* per-column theory status: the configuration cannot exist */

/* ---- enumerations ---- */
#define TPLBM_D1Q3 1
#define TPLBM_D2Q9 2
#define TPLBM_D3Q19 3

#define TPLBM_FP64 0            /* populations stored in FP64 */
#define TPLBM_FP32_DEV 1        /* populations stored in FP32 as f_i - w_i rho_ref(layer) */

/* state between steps (tplbm_params.state).  With every relaxation time 1
 * the post-collision populations are a closed function of the node's density,
 * force-corrected velocity and force (Eq. LiFS with Eq. OperatorMRT at
 * Lambda = I), so an FP64 lattice can carry its moments instead of the
 * populations: rho and j (D2Q9, 3 planes instead of 9; D3Q19, 4 planes
 * and a fifth that a readout fills with psi, instead of 19), plus T; the
 * same arithmetic as the population state, equal to rounding.  MOMENTS
 * carries the moments (FP64, every tau = 1 only: TPLBM_EINVAL otherwise);
 * POPULATIONS always stores populations; AUTO takes the moments wherever they
 * apply (they are the faster state on both lattices). */
#define TPLBM_STATE_AUTO 0
#define TPLBM_STATE_POPULATIONS 1
#define TPLBM_STATE_MOMENTS 2

#define TPLBM_EOS_CARNAHAN_STARLING 0
#define TPLBM_EOS_IDEAL_LATTICE 1 /* p = rho/3, psi = 0: for tests of the closed forms */

/* fields for tplbm_read / tplbm_read_device */
#define TPLBM_RHO 0
#define TPLBM_UX 1
#define TPLBM_UY 2
#define TPLBM_UZ 3
#define TPLBM_T 4
#define TPLBM_P_EOS 5
#define TPLBM_P_NN 6            /* normal pressure: wall-normal diagonal of Eq. GeneralPressureTensor */

/* unphysical-state flags (tplbm_diag.flags) */
#define TPLBM_FLAG_NAN 1u
#define TPLBM_FLAG_RHO 2u       /* rho <= 0 */
#define TPLBM_FLAG_ETA 4u       /* b rho / 4 >= 1 (EOS pole) */
#define TPLBM_FLAG_PSI 8u       /* 2 (p_EOS - rho/3)/G < 0: psi undefined */

/*
 * Lattice parameters.  Paper values (Sec. IV.B): a = 0.5, b = 4, R = 1,
 * sigma = 1.385, every tau = 1, c_v = 5, kappa = 0.02; G = -1 (the sign that
 * makes psi real for this EOS; |G| enters only through the sigma term).
 */
typedef struct tplbm_params {
    int32_t lattice;        /* TPLBM_D2Q9 or TPLBM_D3Q19 (columns: tplbm_batch_*) */
    int32_t nx, ny, nz;     /* nodes per axis; nz ignored for D2Q9 */
    int32_t walls;          /* 1: wet-node walls on the wall-normal axis; 0: periodic */
    int32_t precision;      /* TPLBM_FP64 or TPLBM_FP32_DEV */
    int32_t eos;            /* TPLBM_EOS_* */
    int32_t gravity_form;   /* 1: F_g = rho g (Eq. Gravity_1); 2: (rho - <rho>) g (Eq. Gravity_2);
                               3: (rho - rho_v) g (Eq. Gravity_3) */
    double a, b, R;         /* Carnahan-Starling constants (Eq. EOS) */
    double G;               /* Eq. InteractionPotential, c = 1; must be < 0 for C-S */
    double sigma;           /* Eq. LiFS */
    double tau[6];          /* tau_rho, tau_e, tau_varsigma, tau_j, tau_q, tau_nu (> 1/2) */
    double cv, kappa;       /* Eq. Energy_Equation */
    double g;               /* gravity magnitude along -(wall-normal axis) */
    double rho_ref;         /* FP32_DEV with ref_interval < 0: the one reference density */
    int32_t state;          /* TPLBM_STATE_*: what a lattice stores between steps */
    int32_t ref_interval;   /* FP32_DEV reference densities (ignored for FP64):
                               > 0: one per wall-normal layer (row in 2-D, plane in 3-D),
                                    the layer's mean of the initial density, re-centred
                                    on the layer's current mean density every
                                    ref_interval steps (the stored deviations are
                                    re-encoded; the populations change by at most one
                                    FP32 rounding of the new deviation);
                               0:   the same with TPLBM_REF_INTERVAL_DEFAULT steps;
                               < 0: rho_ref for every layer, never re-centred */
    double rho_v;           /* gravity form 3: the vapour density subtracted (finite) */
} tplbm_params;

#define TPLBM_REF_INTERVAL_DEFAULT 256

/* Diagnostics of the time level `step` (the level the last step started from). */
typedef struct tplbm_diag {
    int64_t step;           /* number of completed steps */
    int64_t first_bad_step; /* level at which a flag was first raised, -1 if none */
    double mass;            /* sum of rho over all nodes at level `step` */
    double mean_rho;        /* <rho> at level `step` (wall nodes included) */
    double max_u;           /* max |u| at level step-1 (the last step's velocity) */
    double min_rho;         /* min rho at level step-1 */
    uint32_t flags;         /* OR of TPLBM_FLAG_* over every step since set_state */
    uint32_t pad;
} tplbm_diag;

typedef struct tplbm_ctx tplbm_ctx;

/* Bytes of device workspace for a lattice with these parameters (pure). */
int tplbm_workspace_bytes(const tplbm_params *p, size_t *bytes);

/* Validate p, bind the workspace and stream, compute host constants.
 * dev_workspace must be at least tplbm_workspace_bytes() bytes, 256-byte
 * aligned.  *out receives a host handle owned by the library.
 * Errors: EINVAL (parameters), ESHAPE (sizes), EUNSUPPORTED, EHIP. */
int tplbm_create(const tplbm_params *p, void *dev_workspace, size_t bytes, void *hip_stream,
                 tplbm_ctx **out);

/* Set the state at level 0 from host arrays of N doubles each (N = node
 * count): populations at rest, f_i = w_i rho0 (reading of the paper's
 * unstated initial condition), and T0.  T0 on the wall layers is kept fixed
 * as Dirichlet data (the paper's T_bot / T_top, Sec. IV).  Synchronous.
 * Errors: EINVAL on NULL, EHIP. */
int tplbm_set_state(tplbm_ctx *ctx, const double *rho0, const double *T0);

/* Advance nsteps >= 0 steps (one fused kernel launch per step), then wait
 * and check the flags: returns TPLBM_EUNPHYSICAL if any step raised one
 * (tplbm_diagnostics gives the first such level).  Synchronous. */
int tplbm_step(tplbm_ctx *ctx, int64_t nsteps);

/* Same, without waiting or checking (for timing and capture by callers). */
int tplbm_step_async(tplbm_ctx *ctx, int64_t nsteps);

/* Macroscopic field of the current level into a host array of N doubles
 * (TPLBM_RHO, TPLBM_UX/UY/UZ: force-corrected velocity of Eq. Momentum,
 * TPLBM_T, TPLBM_P_EOS, TPLBM_P_NN: normal pressure with plain central
 * differences, interior nodes only; wall nodes report p_EOS).  Synchronous.
 * Errors: EINVAL (field), EHIP. */
int tplbm_read(tplbm_ctx *ctx, int field, double *host_out);

/* Same into a device array of N doubles, enqueued on the stream (async). */
int tplbm_read_device(tplbm_ctx *ctx, int field, double *dev_out);

/* Diagnostics of the last completed step.  Synchronous. */
int tplbm_diagnostics(tplbm_ctx *ctx, tplbm_diag *out);

/* Exact checkpoint of the state (populations or moments, temperature,
 * <rho>, step count) to a host blob of tplbm_state_bytes() bytes and back.
 * The blob starts with a 64-byte header naming the lattice, its sizes, the
 * stored precision, the walls and the number of state planes.  load_state
 * takes the blob's length in `bytes` and rejects (ESHAPE, nothing read past
 * the header) a blob whose length or header does not match this lattice;
 * EINVAL for a blob this library did not write.  Synchronous.  Restoring and
 * stepping reproduces an uninterrupted run bit for bit. */
int tplbm_state_bytes(const tplbm_ctx *ctx, size_t *bytes);
int tplbm_save_state(tplbm_ctx *ctx, void *host_blob);
int tplbm_load_state(tplbm_ctx *ctx, const void *host_blob, size_t bytes);

/* Release the host handle (the workspace stays the caller's). NULL is a no-op. */
void tplbm_destroy(tplbm_ctx *ctx);

/* Message of the last failure on ctx, or of the last failed call made with
 * no context when ctx is NULL.  Never NULL. */
const char *tplbm_last_error(const tplbm_ctx *ctx);

/* Copy `bytes` bytes between two 16-byte aligned device buffers with 16-byte
 * vector loads and stores (asynchronous on hip_stream).  A measurement
 * utility: the HBM streaming rate a bandwidth-bound kernel can reach on this
 * GPU, which the benchmark reports beside the lattice kernels' rates.
 * Errors: EINVAL (NULL or misaligned pointer), EHIP. */
int tplbm_stream_copy(const void *dev_src, void *dev_dst, size_t bytes, void *hip_stream);

/* ---- host FP64 equation-of-state utilities (Eq. EOS, Eq. MaxwellRule) ---- */

/* Critical point of Carnahan-Starling with constants a, b, R (the point
 * where dp/drho = d2p/drho2 = 0): out3 = {rho_c, T_c, p_c}. */
int tplbm_eos_critical(double a, double b, double R, double *out3);

/* Coexistence at absolute temperature T by the equal-area rule
 * (Eq. MaxwellRule): out3 = {rho_v, rho_l, p_sat}.  EINVAL at or above T_c. */
int tplbm_eos_coexistence(double a, double b, double R, double T, double *out3);

/* Spinodal densities at T (local extrema of p_EOS, Sec. V):
 * out2 = {vapour spinodal, liquid spinodal}.  EINVAL at or above T_c. */
int tplbm_eos_spinodal(double a, double b, double R, double T, double *out2);

/* ======================================================================
 * Sharp-interface theory of a column (Sec. IV A; its numerical procedure in
 * the appendix; configurations of Sec. VI).  Host only, FP64.
 *
 * At rest the column obeys dp/dy = F_g,y(rho) (Eq. Momentum_Balance_TS) and
 * its temperature is linear between the walls (Eq. Temp_Profile).  An
 * interface at height h joins the Maxwell coexistence states of T(h)
 * (Eq. MaxwellRule); elsewhere the pressure advances by explicit Euler steps
 * and the density is the inverse EOS (Eq. Inverse_EOS) on the phase's stable
 * or metastable branch (Eqs. Numerical_Vapor_Region,
 * Numerical_Liquid_Region).  A branch driven past its spinodal, or a vapour
 * driven to zero pressure, means the configuration cannot exist.  The
 * interface height is searched until the mean density is the given one.
 *
 * Geometry as in a batch column: nodes y = 0 .. height-1, walls on the first
 * and last node, T(y) = T_bot + (T_top - T_bot) y / (height - 1), g > 0
 * pointing to node 0, F = -rho g (form 1), -(rho - mean_rho) g (form 2) or
 * -(rho - rho_v) g (form 3).
 * Discretisation: each node interval is split into `substeps` Euler steps
 * (the interval holding an interface is split there first, each part into
 * `substeps`); a V-L-V configuration is integrated as V-L until p - p_sat(T)
 * changes sign inside the liquid, where a second interface (linearly
 * interpolated inside that Euler step) starts a vapour at the coexistence
 * state.  The mean density is the integral of the sharp profile over the node
 * cells [-1/2, height - 1/2] divided by height (trapezoids over the Euler
 * steps, plus half a cell at each wall holding the wall value): it equals the
 * node mean of a smooth profile and is continuous in h.  Search: h is tried
 * on every node from 0 up; the first pair of neighbouring placements that
 * both exist and bracket mean_rho is bisected to a width of 1e-12.
 * A node exactly on an interface takes the lower phase's value.
 * ====================================================================== */

#define TPLBM_THEORY_LV 0       /* liquid below vapour */
#define TPLBM_THEORY_VL 1       /* vapour below liquid */
#define TPLBM_THEORY_VLV 2      /* vapour, liquid, vapour */

/* reasons a configuration cannot exist (tplbm_theory_result.reasons: the OR
 * over every interface placement the search tried) */
#define TPLBM_THEORY_NO_LIQUID 1u               /* a liquid passed its spinodal (boiling, cavitation) */
#define TPLBM_THEORY_NO_VAPOUR 2u               /* a vapour passed its spinodal (condensation) */
#define TPLBM_THEORY_ZERO_PRESSURE 4u           /* a vapour's pressure fell to zero */
#define TPLBM_THEORY_SUPERCRITICAL_INTERFACE 8u /* interface tried where T >= T_c */
#define TPLBM_THEORY_NO_SECOND_INTERFACE 16u    /* V-L-V: the liquid never met p_sat */
#define TPLBM_THEORY_NO_MATCH 32u               /* no two neighbouring placements bracket mean_rho */
#define TPLBM_THEORY_BROKEN_BRACKET 64u         /* a placement inside the bracket cannot exist */
#define TPLBM_THEORY_SOLVE_FAILED 128u          /* a spinodal or coexistence solve failed (T near T_c) */

typedef struct tplbm_theory_column {
    int32_t height;        /* nodes including both wall nodes, 3 .. 2^24 */
    int32_t gravity_form;  /* 1, 2 or 3 */
    int32_t config;        /* TPLBM_THEORY_LV, _VL or _VLV */
    int32_t substeps;      /* Euler steps per node interval, 1 .. 4096 */
    double T_bot, T_top;   /* absolute wall temperatures (nodes 0 and height-1), > 0 */
    double g;              /* signed; > 0 points to node 0 */
    double mean_rho;       /* mean density, 0 < mean_rho < 4/b */
    double rho_v;          /* form 3: the vapour density subtracted (finite) */
} tplbm_theory_column;

typedef struct tplbm_theory_result {
    int32_t status;        /* TPLBM_OK or TPLBM_ENOSOLUTION */
    int32_t n_interfaces;  /* 1 (L-V, V-L) or 2 (V-L-V); 0 without a solution */
    uint32_t reasons;      /* TPLBM_THEORY_* bits when status is TPLBM_ENOSOLUTION */
    uint32_t pad;
    double interface[2];   /* interface heights (node units from node 0); NaN if absent */
    double mean_rho;       /* mean density of the returned profile */
} tplbm_theory_result;

/* Solve ncols independent columns with the EOS constants a, b, R on up to
 * nthreads host threads (<= 0: one per hardware thread).  rho (and p, which
 * may be NULL) receive the node densities and pressures, column after column
 * (column k at sum_{j<k} height_j); a column without a solution is filled
 * with NaN.  out[k] receives each column's status.  Returns TPLBM_OK once
 * every column has been tried, whatever their statuses; EINVAL or ESHAPE (and
 * nothing written) for a bad column, EOS constant or NULL pointer.
 * Thread-safe; host memory only. */
int tplbm_theory_solve(double a, double b, double R, int32_t ncols, const tplbm_theory_column *cols,
                       double *rho, double *p, tplbm_theory_result *out, int32_t nthreads);

/* Message of the calling thread's last failed tplbm_theory_solve.  Never NULL. */
const char *tplbm_theory_last_error(void);

/* ======================================================================
 * Batched column sweep (one persistent launch runs many independent 1-D
 * columns to steady state).  A column is the paper's minimal 1-D system
 * (Sec. IV): wet-node walls at both ends, liquid/vapour, gravity along the
 * column (Eqs. Gravity_1 / Gravity_2 per column), the temperature of its two
 * end nodes held fixed.  Columns use D1Q3, which at tau = 1 is the exact
 * x-uniform reduction of the D2Q9 update (every relaxation time is 1 here;
 * the paper uses tau = 1 throughout, Sec. IV.B).
 * ====================================================================== */

#define TPLBM_COL_CONVERGED 0   /* max |u| < tol at a check level */
#define TPLBM_COL_DIVERGED 1    /* an unphysical-state flag was seen */
#define TPLBM_COL_MAX_STEPS 2   /* step budget reached first */

typedef struct tplbm_column {
    int32_t height;        /* nodes including both wall nodes, 3 .. 2048 */
    int32_t gravity_form;  /* 1, 2 or 3 (Eqs. Gravity_1, Gravity_2, Gravity_3) */
    double g;              /* signed gravity: > 0 points to node 0, < 0 away from it */
    double rho_v;          /* form 3: the vapour density subtracted (finite; ignored otherwise) */
} tplbm_column;

typedef struct tplbm_batch_params {
    double a, b, R, G, sigma;  /* as in tplbm_params */
    double cv, kappa;
    int32_t eos;               /* TPLBM_EOS_* */
    int32_t pad;
} tplbm_batch_params;

typedef struct tplbm_col_result {
    int64_t steps;     /* level at which the column stopped */
    int32_t status;    /* TPLBM_COL_* */
    int32_t pad;
    double mass;       /* sum of rho at that level */
    double max_u;      /* max |u| at that level */
} tplbm_col_result;

typedef struct tplbm_batch_tuning {
    int32_t shape;         /* kernel shape index (threads x nodes per thread) */
    int32_t threads;       /* threads per column */
    int32_t nodes_per_thread;
    int32_t check_every;   /* steps between steady-state checks */
    int32_t grid;          /* resident workgroups of the persistent launch */
    int32_t pad;
    double node_steps_per_s; /* throughput measured for the choice */
} tplbm_batch_tuning;

typedef struct tplbm_batch tplbm_batch;

/* Device workspace bytes for ncols columns (pure). */
int tplbm_batch_workspace_bytes(const tplbm_batch_params *p, int32_t ncols,
                                const tplbm_column *cols, size_t *bytes);

/* Bind a workspace and stream; columns are copied.  Errors: EINVAL, ESHAPE
 * (a height outside 3..2048), EHIP. */
int tplbm_batch_create(const tplbm_batch_params *p, int32_t ncols, const tplbm_column *cols,
                       void *dev_workspace, size_t bytes, void *hip_stream, tplbm_batch **out);

/* Initial densities and temperatures, concatenated column after column
 * (column k occupies sum_{j<k} height_j .. + height_k).  Populations start at
 * rest (f_i = w_i rho0).  The end nodes' temperatures are the Dirichlet data.
 * Synchronous. */
int tplbm_batch_set_state(tplbm_batch *b, const double *rho_concat, const double *T_concat);

/* Run every column from its initial state until max |u^n| < tol at a level n
 * that is a multiple of the check interval, until a flag is raised, or until
 * n = max_steps; one persistent launch.  out[k] receives column k's result
 * (caller array of ncols; levels count from this run's start).  The final
 * levels are kept for tplbm_batch_read and tplbm_batch_resume.  Never aborts
 * the batch for one bad column.  Synchronous. */
int tplbm_batch_run(tplbm_batch *b, double tol, int64_t max_steps, tplbm_col_result *out);

/* Arm the next tplbm_batch_run to continue every column from the level the
 * last run ended at (its populations and temperatures, bit for bit, as if the
 * run had gone on) instead of from tplbm_batch_set_state's state, with the
 * wall temperatures replaced by T_bot[k] (node 0) and T_top[k] (last node)
 * for column k -- a change of the boundary conditions in the middle of a run,
 * as in the phase-change protocol of Sec. V A.  T_bot or T_top may be NULL to
 * keep those walls.  One-shot: a later run starts from set_state's state
 * again unless resume is called again.  Errors: EINVAL if no run has ended
 * since the last set_state or autotune (whose trial launches overwrite the
 * end state), or a wall temperature is not finite and > 0; EHIP.
 * Synchronous. */
int tplbm_batch_resume(tplbm_batch *b, const double *T_bot, const double *T_top);

/* Final densities (TPLBM_RHO) or temperatures (TPLBM_T), concatenated. */
int tplbm_batch_read(tplbm_batch *b, int field, double *host_out);

/* Pick the kernel shape and the check interval by timing short trial sweeps
 * of the batch (at most about budget_ms of GPU time); the choice is kept for
 * later runs and returned in *out (may be NULL).  Inputs are not modified. */
int tplbm_batch_autotune(tplbm_batch *b, double budget_ms, tplbm_batch_tuning *out);

/* Set the shape and check interval explicitly (shape -1 keeps the current). */
int tplbm_batch_set_tuning(tplbm_batch *b, int32_t shape, int32_t check_every);

void tplbm_batch_destroy(tplbm_batch *b);
const char *tplbm_batch_last_error(const tplbm_batch *b);

/* Allocation-free variant of tplbm_batch_create + tplbm_batch_set_state +
 * tplbm_batch_run, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * It allocates nothing and takes no workspace: it runs the same column
 * kernel as tplbm_batch_run.
 *   cols[ncols]      host column descriptions (read during the call)
 *   dev_rho0, dev_T0 device arrays: initial densities and temperatures,
 *                    concatenated as in tplbm_batch_set_state (populations
 *                    start at rest, f_i = w_i rho0; the end nodes'
 *                    temperatures are the Dirichlet data)
 *   dev_rho_out, dev_T_out  device arrays of the same length: the densities
 *                    and temperatures of each column's end level (they may
 *                    alias dev_rho0 and dev_T0)
 *   dev_results      device array of ncols records, as tplbm_batch_run's out
 *   tol, max_steps   as in tplbm_batch_run; check_every >= 1 is the
 *                    steady-state check interval
 * Columns run in index order on the 256 x 8 kernel shape (no autotuning; a
 * caller that sorts its columns by decreasing height balances the launch).
 * The column descriptions, their node offsets, the processing order and the
 * work-queue counter live in a fixed device array of about 480 KiB per GPU
 * that the library holds until the process ends; ncols is at most 8192
 * (ESHAPE beyond).  Every call on a GPU shares that array, so calls that
 * overlap on one GPU (another stream or another host thread) race: the
 * caller serialises them.  The stream must belong to the current device.
 * Synchronous.  Errors (tplbm_batch_last_error(NULL)): EINVAL, ESHAPE, EHIP. */
int tplbm_batch_run_noalloc(const tplbm_batch_params *p, int32_t ncols, const tplbm_column *cols,
                            const double *dev_rho0, const double *dev_T0, double *dev_rho_out,
                            double *dev_T_out, tplbm_col_result *dev_results, double tol,
                            int64_t max_steps, int32_t check_every, void *hip_stream);

/* ------------------------------------------------------------------------
 * Learned warm start for the column sweep.
 *
 * A 1-D convolutional network maps a column's parameters to its steady
 * density and temperature profiles; its prediction seeds tplbm_batch_* runs,
 * which decide the steady state.  The paper starts its runs
 * from liquid below vapour (Sec. V, example of phase formation) and notes
 * that a run may instead start from the theoretical profile (Sec. IV B);
 * the network is a learned stand-in for that profile, trained on steady
 * profiles that the column sweep itself produced.
 *
 * Network: six width-5 convolutions 8 -> 64 -> 64 -> 64 -> 64 -> 64 -> 2
 * along the column, zero padding at the two ends of each column (columns in
 * a batch never see each other), ReLU after the first five.  Input channels
 * at node y of a column of height H: (y + 1/2)/H - 1/2, T/T_c - 0.8,
 * log10 g + 5, gravity_form - 3/2, <rho>/rho_c - 1.3, H/2048 - 1/2, and
 * clip(d/32, -4, 4)/4, clip(d/4, -4, 4)/4 with d = y + 1/2 - lever_height.
 * Output channels: rho/rho_c - <rho>/rho_c and T/T_c - T_wall/T_c.  Loss:
 * mean over nodes and both channels of the squared error.
 *
 * Arithmetic: FP32 master parameters and Adam moments (beta1 0.9, beta2
 * 0.999, eps 1e-8); every product runs on the BF16 matrix cores (inputs,
 * weights and back-propagated gradients rounded to BF16, nearest-even) with
 * FP32 accumulation; biases, losses and reductions in FP32.
 *
 * Parameter vector (FP32): for each layer l in order, W_l with shape
 * (C_out, 5, C_in) row-major (tap t reads node y + t - 2), then b_l (C_out).
 * ---------------------------------------------------------------------- */

typedef struct tplbm_net_column {
    int32_t height;        /* nodes including both wall nodes, 3 .. 2048 */
    int32_t gravity_form;  /* 1 or 2 */
    double t_reduced;      /* T / T_c of the isothermal column (also its wall value) */
    double g;              /* gravity magnitude, > 0 */
    double mean_reduced;   /* <rho> / rho_c, the column's mean density */
    double lever_height;   /* H (<rho> - rho_v)/(rho_l - rho_v) in nodes, with the
                              Maxwell coexistence densities at T (tplbm_eos_coexistence):
                              where a flat interface would sit without gravity */
} tplbm_net_column;

typedef struct tplbm_net_config {
    double rho_c, T_c;       /* critical density and temperature of the EOS */
    int32_t max_cols;        /* columns per call (minibatch or prediction) */
    int32_t dataset_cols;    /* training columns held on the device (0: none) */
    int64_t max_nodes;       /* sum of heights per call, at most about 2^25 */
    int64_t dataset_nodes;   /* sum of heights of the training columns */
} tplbm_net_config;

typedef struct tplbm_net tplbm_net;

/* Number of parameters (85 442). */
int tplbm_net_num_params(int64_t *n);

/* Device workspace bytes for a configuration (pure). */
int tplbm_net_workspace_bytes(const tplbm_net_config *c, size_t *bytes);

/* Bind a caller-owned device workspace (256-byte aligned, kept alive until
 * destroy) and a HIP stream.  Errors: EINVAL, ESHAPE. */
int tplbm_net_create(const tplbm_net_config *c, void *dev_workspace, size_t bytes, void *hip_stream,
                     tplbm_net **out);

/* Load the FP32 parameter vector from host memory (the layout above) and
 * reset the Adam moments and step count.  Errors: EINVAL (non-finite). */
int tplbm_net_set_params(tplbm_net *n, const float *theta);
int tplbm_net_get_params(tplbm_net *n, float *theta);

/* Initialise the parameters (and reset Adam) with He-uniform weights, bound
 * sqrt(6 / (5 C_in)), and zero biases.  Weight k, counted over the layers in
 * the parameter layout's order, is 2 u_k - 1 times the bound, where u_k takes
 * the top 53 bits of the SplitMix64 finaliser of
 * seed + (k + 1) * 0x9E3779B97F4A7C15 (mod 2^64), rounded to FP32.  The
 * network is an addition to the paper's method: its initialisation follows
 * no passage of the paper. */
int tplbm_net_init(tplbm_net *n, uint64_t seed);

/* Copy a training set to the device: ncols column descriptions and their
 * steady profiles rho and T (host, concatenated column after column).
 * Errors: EINVAL, ESHAPE (more than the workspace holds). */
int tplbm_net_set_dataset(tplbm_net *n, int32_t ncols, const tplbm_net_column *cols, const double *rho,
                          const double *T);

/* Loss of the dataset columns idx[0..nbatch) and its gradient with respect
 * to the parameters (host, may be NULL).  Parameters are not changed.
 * Synchronous. */
int tplbm_net_loss_grad(tplbm_net *n, int32_t nbatch, const int32_t *idx, double *loss, float *grad);

/* One Adam step with learning rate lr on the minibatch idx[0..nbatch);
 * *loss (may be NULL) receives the loss before the step. */
int tplbm_net_train_step(tplbm_net *n, int32_t nbatch, const int32_t *idx, float lr, double *loss);

/* Raw network outputs for caller columns: out[2 (offset_k + y) + c] for
 * channel c at node y of column k (offset_k = sum of earlier heights);
 * host array of 2 * sum(height) floats.  Synchronous. */
int tplbm_net_forward(tplbm_net *n, int32_t ncols, const tplbm_net_column *cols, float *out);

/* Warm-start profiles (host, concatenated, FP64): rho = rho_c (out_0 +
 * <rho>/rho_c) shifted by one constant per column so that its mean is
 * exactly <rho>; T = T_c (T/T_c + out_1) inside and T_c t_reduced at the two
 * wall nodes (the Dirichlet data).  Pass them to tplbm_batch_set_state. */
int tplbm_net_predict(tplbm_net *n, int32_t ncols, const tplbm_net_column *cols, double *rho, double *T);

/* The same profiles into device arrays (caller-owned, sum(height) doubles
 * each), enqueued on the network's stream without waiting: a warm start can
 * then seed tplbm_batch_run_noalloc without a round trip through the host. */
int tplbm_net_predict_device(tplbm_net *n, int32_t ncols, const tplbm_net_column *cols, double *dev_rho,
                             double *dev_T);

/* One v_mfma_f32_32x32x16_bf16 on host operands: a and b hold 64 lanes x 8
 * bf16 values each (lane-major), d receives 64 lanes x 16 FP32 results.  For
 * checking the matrix-core lane layout the kernels assume. */
int tplbm_net_mfma_check(tplbm_net *n, const uint16_t *a, const uint16_t *b, float *d);

void tplbm_net_destroy(tplbm_net *n);
const char *tplbm_net_last_error(const tplbm_net *n);

#ifdef __cplusplus
}
#endif
#endif /* TPLBM_H */
