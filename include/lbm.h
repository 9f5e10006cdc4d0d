/*
 * lbm.h -- C ABI of the MI355X (gfx950) implementation of the coupled
 * density / total-energy D2Q9 MRT lattice Boltzmann step of
 * R. Huang, H. Wu, N. A. Adams, "Lattice Boltzmann model with self-tuning
 * equation of state for coupled thermo-hydrodynamic flows" (arXiv:1809.08683).
 *
 * One time step (lbm_step) is the fused streaming + collision of both DFs:
 *   - density DF f: eq. LBE.u (Sec. 2.1): MRT collision with the self-tuning
 *     EOS (eta from p_EOS), force moments F_m, non-diagonal S and the cubic
 *     corrections R, T.grad(rho), X.grad(p);
 *   - total-energy DF g: eq. LBE.T (Sec. 2.2, App. C): MRT collision with
 *     the modified L and the density-DF coupling Y((m + mbar)/2 - m^eq);
 *   - walls (Sec. 3, App. B): bounce-back temporaries for the wall macros,
 *     then every DF of a wall node rebuilt from equilibrium, force and the
 *     extrapolated tilde non-equilibrium parts.
 *
 * Conventions
 *   - Lattice units: dx = dt = c = 1, c_s^2 = 1/3.
 *   - Grid: nx * ny nodes, node (x, y) at host index y*nx + x (x fastest).
 *     Walls sit on the boundary nodes (Sec. 3.1): a wall side's nodes are
 *     the first/last column or row.  Sides: 0 = {x = 0}, 1 = {x = nx-1},
 *     2 = {y = 0}, 3 = {y = ny-1}; opposite sides are both walls or both
 *     periodic.  A walled axis needs at least 5 nodes.
 *   - Host arrays are caller-owned, FP64, nx*ny long; the library never keeps
 *     a caller pointer.  A NULL output pointer means "skip".
 *   - Device memory is owned by the context (hipMalloc), or supplied by the
 *     caller through lbm_create_ex (it must stay valid until lbm_destroy).
 *   - Time: lbm_init sets t = 0; lbm_step(n) advances t by n.  lbm_macros,
 *     lbm_nusselt and lbm_totals report the pre-collision macroscopic state
 *     at the current t (wall nodes report their prescribed/derived values).
 *   - Every call returns an lbm_status; lbm_last_error gives details.
 *     LBM_EDIVERGED (non-finite or non-positive rho or T seen at the end of
 *     a step call) leaves the state readable.
 *   - One context per host thread; calls on one context are not reentrant.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument; nothing changed */
    LBM_ENOMEM = -2,     /* device allocation failed / workspace too small */
    LBM_EDEVICE = -3,    /* HIP runtime error */
    LBM_EDIVERGED = -4,  /* state contains non-finite or non-positive rho/T */
    LBM_ESTATE = -5      /* call out of order (e.g. step before init) */
} lbm_status;

/* Equations of state (Sec. 4, eqs. EOSs; van der Waals added):
 *   DECOUPLED p = rho R T0, IDEAL p = rho R T,
 *   VDW p = rho R T / (1 - b rho) - a rho^2,
 *   CS  p = Z rho R T, Z = (1 + y + y^2 - y^3)/(1 - y)^3, y = b rho / 4,
 *       b <= 0 selecting sqrt(2) pi / (3 rho0).
 * R <= 0 selects the R for which dp/drho at (rho0, T0) equals c_s^2
 * (eq. cs). */
typedef enum { LBM_EOS_DECOUPLED = 0, LBM_EOS_IDEAL = 1, LBM_EOS_VDW = 2, LBM_EOS_CS = 3 } lbm_eos_kind;
typedef struct {
    int kind;            /* lbm_eos_kind */
    double R, rho0, T0, a, b;
} lbm_eos;

/* Viscosity law mu(T): constant, mu0 T/T0, or Sutherland's law referred to
 * (T0, mu0) with constant S (in units of T0) (Sec. 4.3). */
typedef enum { LBM_VISC_CONST = 0, LBM_VISC_LINEAR = 1, LBM_VISC_SUTHERLAND = 2 } lbm_visc_law;

/* Relaxation (Sec. 4): the local rates follow from
 *   nu = mu(T)/rho = c_s^2 (1/s_p - 1/2),  (1/s_p - 1/2)(1/s_q - 1/2) = 1/12,
 *   bulk viscosity varpi c_s^2 (1/s_e - 1/2) = bulk_ratio * nu, s_eps = s_e,
 *   s_0 = s_j = 1;  lambda = C_p mu / Pr = kappa rho0 C_p (1/sigma_j - 1/2),
 *   (1/sigma_j - 1/2)(1/sigma_e - 1/2) = 1/4, sigma_eps = sigma_p = sigma_e,
 *   sigma_q = sigma_j, sigma_0 = 1;  varpi = 1/6, gamma1 = -2, gamma2 = 2. */
typedef struct {
    double nu0;          /* mu0 / rho0 at T0; tau0 = 3 nu0 + 1/2 */
    double bulk_ratio;   /* bulk / kinematic viscosity (Table 1: 1, 2 or 4) */
    int law;             /* lbm_visc_law */
    double sutherland_S; /* S / T0 */
} lbm_relax;

typedef struct {
    int wall;            /* 1: wall side, 0: periodic */
    double ux, uy;       /* wall velocity (no-slip value, Sec. 3.1) */
    int adiabatic;       /* 1: zero heat flux, 0: Dirichlet temperature T */
    double T;
} lbm_side;

typedef struct {
    lbm_side side[4];
    int extrap_order;    /* 1 or 2 (eq. neq.extrapolation) */
} lbm_boundary;

/* Storage precision of the DFs (always stored as offsets from the
 * rest-state equilibrium):
 *   FP64   - FP64 storage and arithmetic;
 *   FP32   - FP32 storage and arithmetic, temperature recovered in FP64;
 *   FP16S  - FP16 storage of f and g, FP32 arithmetic, temperature in FP64;
 *   F32G16 - FP32 storage of the density DFs f, FP16 storage of the
 *            energy DFs g, FP32 arithmetic, temperature in FP64.
 * The 16-bit rows are rounded stochastically (unbiased; the random operand
 * of a value depends only on where it is stored, its DF row and the step,
 * so results are bitwise reproducible), and with an ideal gas between two
 * Dirichlet x-walls the g rows store offsets from the conduction state
 * between them instead of the global rest state.  On a cavity with
 * eps = 0.6 the mean Nusselt number then stays within 0.2 % (F32G16) and
 * 0.5 % (FP16S; 0.6 % early in a 1024^2 transient) of FP64 up to 2048^2;
 * FP32 within 6e-4. */
typedef enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16S = 2, LBM_F32G16 = 3 } lbm_precision;

typedef struct {
    double fx, fy;       /* force per unit volume, or per unit mass if per_mass */
    int per_mass;        /* 1: F = rho (fx, fy) (gravity) */
    int prec;            /* lbm_precision */
    int cubic;           /* 0: no R, T, X; 1: R only; 2: R, T and X (default) */
    double cp;           /* <= 0: C_p = 3.5 c_s^2 / T0 (eq. Cp) */
    int cv_rule;         /* 0: C_v = C_p / gamma; 1: C_v = C_p - p(rho0,T0)/(rho0 T0) */
    int seg_rows;        /* rows per interior work item (0: automatic) */
    void* hip_stream;    /* hipStream_t to launch on; NULL: context-owned stream */
} lbm_options;

/* Create a context.  Validates the parameters (positive sizes, walled axes
 * >= 5 nodes, rho0, T0, Pr, gamma, nu0 > 0, 0 < s_p, sigma_j < 2 at the
 * reference state) and allocates device memory. */
lbm_status lbm_create(int nx, int ny, const lbm_eos* eos, double Pr, double gamma,
                      const lbm_relax* relax, const lbm_boundary* bc,
                      const lbm_options* opt, lbm_ctx** out);

/* Device bytes lbm_create_ex needs for one case. */
size_t lbm_workspace_bytes(int nx, int ny, int prec);

/* As lbm_create, but places all per-case device arrays in the caller's
 * device allocation [dev_workspace, dev_workspace + bytes) (e.g. a torch
 * tensor); LBM_ENOMEM if bytes < lbm_workspace_bytes(nx, ny, prec). */
lbm_status lbm_create_ex(int nx, int ny, const lbm_eos* eos, double Pr, double gamma,
                         const lbm_relax* relax, const lbm_boundary* bc,
                         const lbm_options* opt, void* dev_workspace, size_t bytes,
                         lbm_ctx** out);

/* Initial state (t = 0) from host macroscopic fields: at every node, walls
 * included, the decomposition of eq. decompose (Sec. 3.2) with a zero
 * non-equilibrium part, m = m^eq - F_m/2 and n = n^eq - Q_m/2, with
 * E = C_v T + |u|^2/2 (Sec. 2.2); the runs of Secs. 4.1-4.3 start from rest
 * at rho0, T0, which NULL fields give (rho0, 0, 0, T0).  Wall velocities and
 * temperatures act from t = 1 (Sec. 4.3: walls changed abruptly).  Layout
 * [ny][nx], caller-owned.  LBM_EINVAL for non-finite values or rho, T <= 0.
 * Synchronises the stream. */
lbm_status lbm_init(lbm_ctx* ctx, const double* rho, const double* ux,
                    const double* uy, const double* T);

/* Advance n >= 0 time steps (one kernel launch per step, on the context
 * stream), then check the state for divergence (synchronises). */
lbm_status lbm_step(lbm_ctx* ctx, long long n);

/* As lbm_step, and report the elapsed device time of the n steps measured
 * with HIP events on the context stream (milliseconds). */
lbm_status lbm_step_timed(lbm_ctx* ctx, long long n, double* ms);

/* As lbm_step, with options (flags, or-ed):
 *   LBM_STEP_GRAPH captures the n steps into a HIP graph on first use (one
 *     graph per n, start buffer and kind, kept until the launch
 *     configuration changes or the context is destroyed) and replays it,
 *     which removes the per-launch host overhead;
 *   LBM_STEP_PERSISTENT runs the n steps in one launch of a persistent
 *     kernel: every wavefront keeps its work item, and a per-case step
 *     barrier (device-scope counters) replaces the launch boundary, so the
 *     cases of a batch advance independently.  It needs every block of the
 *     launch resident at once (LBM_EINVAL otherwise, with the reason in
 *     lbm_last_error); each barrier wait gives up after a bounded number of
 *     polls (lbm_set_persistent_spin_limit), and then the call returns
 *     LBM_EDEVICE and every case must be initialised or loaded again.
 *     With LBM_STEP_GRAPH the counter reset and the persistent launch are
 *     captured together.
 * ms != NULL receives the device time of the n steps (HIP events on the
 * context stream).  Results are bitwise those of lbm_step. */
#define LBM_STEP_GRAPH 1
#define LBM_STEP_PERSISTENT 2
lbm_status lbm_step_ex(lbm_ctx* ctx, long long n, int flags, double* ms);

/* Polls of a persistent step barrier before it gives up (default 2^24,
 * about a second; each poll sleeps about 128 cycles).  For callers that
 * bound the time a stalled launch may take, and for tests of that path. */
lbm_status lbm_set_persistent_spin_limit(lbm_ctx* ctx, unsigned polls);

/* Time level t at the end of the step call that first found case case_id
 * diverged (the flag is checked once per call, so the divergence happened
 * within that call's steps), or -1; reset by lbm_init / lbm_load. */
long long lbm_case_diverged_at(const lbm_ctx* ctx, int case_id);

/* Launch configuration of the step: compiled kernel variant (0: the
 * hand-tuned one; 1: wave priority by progress flipped; 2: LDS parking of
 * the row ahead flipped; 3: the other block size, 4 <-> 8 wavefronts; 4:
 * lockstep march flipped),
 * scale of the modelled cost of an edge-strip row, and row bands per XCD of
 * the work list.  The physics does not depend on it: results are bitwise
 * equal for every configuration. */
lbm_status lbm_set_launch_config(lbm_ctx* ctx, int variant, double xw_scale, int bands_per_xcd);

/* Autotuner of the launch configuration.  If cache_path names a file that
 * holds an entry for this context's key (device architecture, storage
 * format, grid and wall signature of its cases), that entry is applied and
 * no trial runs.  Otherwise every configuration (5 kernel variants x 3
 * edge-cost scales when a case has x-walls x 4 band counts: 4, 1, 8, 16
 * per XCD) is timed over
 * trial_steps steps (0: about 2e7 node updates) from the current state,
 * best of three after a warm-up, the state being restored after each trial
 * (t, buffers, macros and flags are unchanged on return); the fastest is
 * applied if it beats the default configuration (0, 1.0, 4) by more than
 * 1 %, else the default is kept; the choice is written to cache_path if it
 * is not NULL (JSON, one entry per line).  Allocates a device copy of the
 * state while it runs. */
typedef struct {
    int variant;
    double xw_scale;
    int bands_per_xcd;
    double ms_per_step;          /* of the chosen configuration */
    double default_ms_per_step;  /* of configuration (0, 1.0, 4) */
    int trials;                  /* configurations timed (0: from the cache) */
    int from_cache;
} lbm_tune_result;
lbm_status lbm_autotune(lbm_ctx* ctx, int trial_steps, const char* cache_path, lbm_tune_result* out);

/* Macroscopic fields at the current time (FP64 host arrays, nx*ny, layout
 * [ny][nx]): rho and u from eq. rho.u (Sec. 2.1, with the half force), T
 * from eq. E and T = (E - |u|^2/2)/C_v (Sec. 2.2), p = p_EOS(rho, T)
 * (eqs. EOSs); wall nodes report their prescribed u_b and Dirichlet T_b
 * (Sec. 3.1).  Written on the last step of each step call.  Synchronises. */
lbm_status lbm_macros(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* T, double* p);

/* Mean Nusselt number through Dirichlet side `side` (Sec. 4.3):
 * Nu = (1/(lambda0 (T_lo - T_hi))) * sum_j w_j (-lambda(T) dT/dn),
 * n the side's axis (+x or +y), T_lo/T_hi the Dirichlet values of the two
 * sides of that axis, a second-order one-sided dT/dn, trapezoid weights w_j.
 * FP64 on the device.  LBM_EINVAL if the side or its opposite is not a
 * Dirichlet wall or T_lo == T_hi. */
lbm_status lbm_nusselt(lbm_ctx* ctx, int side, double* nu);

/* Sums over all nodes of rho, rho ux, rho uy and rho E (FP64 on the device,
 * fixed reduction order): the quantities whose local conservation the
 * collisions (Secs. 2.1, 2.2) and the wall treatment (Sec. 3.2) keep, so a
 * closed cavity keeps its mass to rounding. */
lbm_status lbm_totals(lbm_ctx* ctx, double* mass, double* momx, double* momy, double* energy);

/* Checkpoint: a format tag, t, the case count, a record per case (nx, ny,
 * precision, row pitch, buffer sizes), then the raw DF state and macros;
 * bytes = lbm_state_bytes(ctx).  lbm_load returns LBM_EINVAL, leaving the
 * context unchanged, if the tag, the case count or any case record differs
 * from the context's own. */
size_t     lbm_state_bytes(const lbm_ctx* ctx);
lbm_status lbm_save(lbm_ctx* ctx, void* host, size_t bytes);
lbm_status lbm_load(lbm_ctx* ctx, const void* host, size_t bytes);

long long   lbm_time(const lbm_ctx* ctx);
const char* lbm_last_error(const lbm_ctx* ctx);
void        lbm_destroy(lbm_ctx* ctx);

/* ---- batches of independent cases stepped by one launch per step ----
 * Every pointer argument is an array of ncases entries; all cases share
 * opt[0].prec and opt[0].hip_stream. */
lbm_status lbm_batch_create(int ncases, const int* nx, const int* ny, const lbm_eos* eos,
                            const double* Pr, const double* gamma, const lbm_relax* relax,
                            const lbm_boundary* bc, const lbm_options* opt, lbm_ctx** out);
int        lbm_batch_size(const lbm_ctx* ctx);
/* Per-case variants of lbm_init / lbm_macros / lbm_nusselt / lbm_totals. */
lbm_status lbm_case_init(lbm_ctx* ctx, int case_id, const double* rho, const double* ux,
                         const double* uy, const double* T);
lbm_status lbm_case_macros(lbm_ctx* ctx, int case_id, double* rho, double* ux, double* uy,
                           double* T, double* p);
lbm_status lbm_case_nusselt(lbm_ctx* ctx, int case_id, int side, double* nu);
lbm_status lbm_case_totals(lbm_ctx* ctx, int case_id, double* mass, double* momx, double* momy,
                           double* energy);
/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid hipMalloc): as lbm_case_init,
 * but the four host fields are staged in a library-owned static device
 * array instead of a per-call allocation.  The array holds 4 x 2^20 doubles
 * (32 MiB), one copy per GPU, kept until the process ends; grids of more
 * than 2^20 nodes are rejected with LBM_EINVAL (use lbm_case_init).  Calls no
 * hipMalloc/hipFree.  Every call on one GPU shares that array: calls that
 * overlap in time on one GPU (from several threads) race.  Synchronises the
 * context stream before returning. */
lbm_status lbm_case_init_static(lbm_ctx* ctx, int case_id, const double* rho, const double* ux,
                                const double* uy, const double* T);

/* The batch calls in the survey's form: lbm_batch_step advances every case
 * n steps and, unlike lbm_step, returns LBM_OK when cases diverged (their
 * flags are reported per case); lbm_batch_nusselt writes, for every case,
 * its divergence flag (1: diverged) and its mean Nusselt number through
 * Dirichlet side `side` as lbm_case_nusselt computes it (NaN for a case
 * that diverged, is not initialised, or has no Dirichlet pair with a
 * temperature difference on that axis).  nu and diverged are caller-owned
 * arrays of lbm_batch_size(ctx) entries.  LBM_EINVAL for side outside 0-3. */
lbm_status lbm_batch_step(lbm_ctx* ctx, long long n);
lbm_status lbm_batch_nusselt(lbm_ctx* ctx, int side, double* nu, int* diverged);

/* Divergence flag of each case (1: diverged) after the last step call. */
lbm_status lbm_batch_flags(lbm_ctx* ctx, int* diverged);

/* Number of work items one step launches (for roofline accounting). */
long long  lbm_work_items(const lbm_ctx* ctx);

/* Plain device copy of `bytes` (multiple of 16) repeated `iters` times on
 * `hip_stream` (NULL: default stream) with library-owned buffers; reports
 * the copy bandwidth 2 * bytes / time (GB/s) and the time per copy (ms).
 * Used as the measured-bandwidth reference of the roofline and to calibrate
 * hardware byte counters. */
lbm_status lbm_copy_bandwidth(size_t bytes, int iters, void* hip_stream, double* gbps, double* ms_per_copy);

/* Stochastic rounding of the 16-bit formats (diagnostics and tests).
 * lbm_rounding_operand: the 32-bit random operand with which DF row q (0-8
 * f, 9-17 g) of node (x, y) is rounded when stored in step t under storage
 * precision prec, computed on the host with the kernels' code; 0 for rows
 * that the precision does not store in 16 bits, for prec outside
 * lbm_precision and for q outside 0-17.
 * lbm_round_half_stochastic: the library's host model of the device's
 * rounding (v_cvt_sr_f16_f32): the FP16 value that v (|v| < 65504) is
 * stored as with operand r.
 * lbm_round_half_device: the same on the device with the store codec's
 * code, for n values; v, r and out are device pointers of n elements,
 * hip_stream NULL for the default stream; waits for the result.  LBM_EINVAL
 * for n < 0 or a NULL pointer with n > 0, LBM_EDEVICE on a HIP error. */
unsigned   lbm_rounding_operand(int prec, int x, int y, unsigned t, int q);
double     lbm_round_half_stochastic(float v, unsigned r);
lbm_status lbm_round_half_device(const float* v, const unsigned* r, float* out, long long n, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
