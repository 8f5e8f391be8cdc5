/*
 * dlrtrt -- SN-like dynamic low-rank (DLR) gray thermal radiative transfer on
 * 2D structured meshes, HIP library for AMD Instinct MI355X (gfx950).
 *
 * Method: Haut, Loffeld, Einkemmer, Guthrey, Brunner, Schill, "Efficient SN-like
 * and PN-like Dynamic Low Rank methods for Thermal Radiative Transfer",
 * arXiv 2601.18705.  One call of dlr_step advances the state by one backward-
 * Euler step of Algorithm 1 (Sec. 4.3): Newton-linearised emission (Sec. 2.2),
 * DEIM angle selection on the angular basis W (Sec. 4.2), source iteration with
 * upwind sweeps over the r selected directions (eq. "steady state collocation"),
 * Gram-Schmidt of the swept columns into X, the Galerkin L-step for every
 * ordinate (eq. "L step"), orthonormalisation L = S W, an SVD of S that orders
 * the angular modes, and the temperature update (eq. "temperature update").
 *
 * Discretisation (the lowest-order member of the upwind DG family of Sec. 4.4):
 * nx x ny uniform cells, cell e = j*nx + i, one value per cell and ordinate.
 * Ordinates: product of n_polar Gauss-Legendre polar cosines on (0,1) (upper
 * hemisphere, xy symmetry) and n_azim azimuths (2k-1) pi / n_azim; weights sum to
 * 4 pi; ordinate index q = p*n_azim + k.  Planck function B(T) = a c T^4 / (4 pi).
 *
 * Conventions for every call:
 *  - No C++ exception crosses this interface; every call returns dlr_status and
 *    leaves a human-readable detail in dlr_last_error() (thread-local).
 *  - All host pointers are caller-owned; the library copies what it keeps.
 *  - Device work runs on the HIP stream given at creation.  Calls on one handle
 *    must be serialised by the caller; distinct handles are independent.
 *  - Arrays are row-major; per-cell arrays follow e = j*nx + i.
 */
#ifndef DLRTRT_H
#define DLRTRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DLR_ABI_VERSION 3

typedef enum {
    DLR_OK = 0,
    DLR_ERR_ARG = -1,            /* invalid argument or shape */
    DLR_ERR_OOM = -2,            /* device memory exhausted (batch: retry later) */
    DLR_ERR_HIP = -3,            /* a HIP runtime call failed */
    DLR_ERR_NOT_CONVERGED = -4,  /* source iteration reached si_max_iter */
    DLR_ERR_NONFINITE = -5,      /* NaN/Inf in the mean intensity or temperature */
    DLR_ERR_STATE = -6,          /* handle poisoned by an earlier device error */
    DLR_ERR_UNSUPPORTED = -7,    /* option not available on the GPU path */
    DLR_ERR_NUMERIC = -8,        /* numerical breakdown: rank-deficient factor with no completion
                                  * vector, singular L-step system, SVD without convergence */
    DLR_ERR_TIMEOUT = -9         /* a bounded wait between workgroups on the device (sweep hand-off,
                                  * DEIM exchange) exceeded its spin limit; the handle is poisoned */
} dlr_status;

enum { DLR_BC_VACUUM = 0, DLR_BC_INFLOW = 1, DLR_BC_REFLECT = 2 };

/* Arithmetic of the step.  Selection (DEIM), QR, SVD, the L-step solves, the
 * temperature update and all conservation sums are FP64 in every mode. */
enum {
    DLR_FP64 = 0,                 /* sweeps and projections in FP64 */
    DLR_FP32_SWEEP = 1,           /* FP32 sweeps and scalar-flux sums; projections on FP32 matrix
                                   * cores (FP32 accumulation per block, FP64 across blocks) */
    DLR_FP32_SWEEP_BF16_PROJ = 2  /* FP32 sweeps; projections on BF16 matrix cores with each operand
                                   * split as hi + lo (three products), FP32 accumulation per block */
};

/*
 * Problem statement (Sec. 2.1-2.2 of the paper, gray TRT):
 *   (1/c) d psi/dt + Omega . grad psi + sigma psi = sigma B(T) + q_ext/(4 pi)
 *   rho c_v dT/dt = sigma (phi - 4 pi B(T)),  phi = int psi dOmega
 * with opacity and heat capacity frozen at their given values.
 *  sigma_a, rho_cv, T_init: [ny*nx], required, sigma_a > 0, rho_cv > 0, T_init >= 0.
 *  q_ext: [ny*nx] or NULL (zero); an isotropic source integrated over angle.
 *  bc[side], side = 0 left, 1 right, 2 bottom, 3 top: DLR_BC_VACUUM or
 *  DLR_BC_INFLOW (isotropic inflow B(T_b[side])).  DLR_BC_REFLECT is
 *  rejected with DLR_ERR_UNSUPPORTED (reference checks only).
 *  rank: 1 <= rank <= min(n_polar*n_azim, nx*ny, 64).  n_azim % 4 == 0.
 *  si_tol: relative 2-norm change of phi that ends source iteration.
 *  deim_tie_tol: DEIM picks among |R| >= (1 - tol) max|R| go to the smallest index.
 * Initial state: psi = B(T_init) isotropic (rank one), completed by graded
 * monomials in space (cell centres mapped to [-1,1]^2) and angle (mu, eta).
 */
typedef struct {
    int32_t abi_version;          /* must be DLR_ABI_VERSION */
    int32_t nx, ny;
    double x0, x1, y0, y1;
    int32_t n_polar, n_azim, rank;
    double dt, c, a;
    const double *sigma_a, *rho_cv, *q_ext, *T_init;
    int32_t bc[4];
    double T_b[4];
    int32_t precision;            /* DLR_FP64 / DLR_FP32_SWEEP / DLR_FP32_SWEEP_BF16_PROJ */
    double si_tol;
    int32_t si_max_iter;
    double deim_tie_tol;
} dlr_problem;

typedef struct dlr_instance *dlr_handle;

/* Device memory of the library.  By default instances, batch slots and tables, and Q1
 * operators take their device memory from hipMalloc and return it with hipFree.  A caller
 * that owns device memory (for example PyTorch's caching allocator) can route every later
 * allocation through its own pair of functions:
 *   alloc(bytes, stream, user): a device pointer aligned to at least 256 bytes, or NULL (the
 *     creating call then fails with DLR_ERR_OOM); stream is the hipStream_t the memory will be
 *     used on (NULL = the default stream);
 *   release(ptr, stream, user): takes it back; the library calls it only after every piece of
 *     work it queued on that memory has completed.
 * An allocation is always released through the pair that made it, so the hook may be replaced
 * at any time; alloc = release = NULL restores hipMalloc / hipFree.  The setting is
 * process-wide and must not race with calls that create or destroy objects.
 * Errors: DLR_ERR_ARG when exactly one of alloc, release is NULL. */
dlr_status dlr_set_allocator(void *(*alloc)(size_t bytes, void *stream, void *user),
                             void (*release)(void *ptr, void *stream, void *user), void *user);

/* Per-step diagnostics of the most recent step (FP64). */
typedef struct {
    int64_t steps_done;           /* steps completed since create / load */
    int32_t si_iters;             /* source iterations of the last step */
    int32_t rank;
    double si_residual;           /* last relative ||phi_k+1 - phi_k||_2 / ||phi_k+1||_2 */
    double deim_min_margin;       /* smallest relative margin of a DEIM pick (1 = no competitor) */
    double sum_abs_cw_over_4pi;   /* sum |c_d| / (4 pi) of the DEIM quadrature weights */
    double energy;                /* sum over cells of area * (rho c_v T + phi / c) */
    double sweep_ms;              /* device time in the sweep kernels of the last step */
    double step_ms;               /* device time of the whole last step; from the second step on from the
                                     previous step's statistics, behind which this step's linearisation and
                                     angle selection were queued */
    int32_t svd_sweeps;           /* Jacobi sweeps of the last step's SVD of S (0 for plain SN) */
    int32_t reserved;
    /* Energy balance of the step (Sec. 2 time-discrete balance, Algorithm 1 step 9).  Powers
     * through the sides of the domain: each face contributes w_q |Omega_q . n| psi times its
     * length, the leaving part from the end-of-step intensity of the wall cell (for DLR the
     * new factors X S W^T), the entering part from the isotropic inflow B(T_b).  For plain
     * SN and full-rank DLR, energy(n+1) - energy(n) = dt (source + inflow - outflow) up to the
     * source-iteration tolerance; at reduced rank the difference is the method's own drift. */
    double inflow;                /* power entering through DLR_BC_INFLOW sides */
    double outflow;               /* power leaving through all sides */
    double source;                /* sum over cells of area * q_ext */
    double si_ms;                 /* device time of the last step's source iterations: the sweeps and the
                                     scalar-flux passes (Algorithm 1 step 4); 0 for batch slots */
} dlr_step_stats;

/* Create an instance: validates the problem, copies fields to the device and
 * builds the initial factors.  hip_stream: a hipStream_t or NULL (default
 * stream).  Errors: DLR_ERR_ARG (shape/values), DLR_ERR_UNSUPPORTED
 * (reflecting walls), DLR_ERR_OOM, DLR_ERR_HIP.  *out is NULL on error. */
dlr_status dlr_create(const dlr_problem *prob, void *hip_stream, dlr_handle *out);

/* Create an instance of the augmented-basis variant of the SN-like step.  Each
 * step orthonormalises the r swept columns together with the old spatial basis
 * X0, so the Galerkin space of the L-step has 2r columns and holds the old
 * solution exactly; the L-step, the angular QR and the SVD of S run at rank 2r,
 * and the SVD result is truncated back to its r largest singular values (the
 * rank-2r representation of Sec. 3 rounded back to rank r, applied to the
 * SN-like step).  After a step the state is X = Xa Q, S = R, W = Wq V_r, where
 * Xa is the 2r-column basis, Wq S^T its angular factor, S = U Sigma V^T, and
 * (U Sigma)_r = Q R (Q with orthonormal columns; a column of a zero singular
 * value is completed with the unit vector of largest remainder, R_kk = 0).  The
 * temperature update, the energy and the outflow use the truncated state.
 * The handle takes every call of dlr_create's handles except batch admission;
 * dlr_read_factors returns rank-r factors as usual.  Requires 2 rank <= min(64,
 * n_polar * n_azim, nx * ny).  Device memory: the spatial bases take 4r planes
 * of cells (against 2r), the per-ordinate L-step matrices (2r)^2 doubles per
 * ordinate.  Errors as dlr_create; DLR_ERR_ARG when the rank condition fails. */
dlr_status dlr_create_augmented(const dlr_problem *prob, void *hip_stream, dlr_handle *out);

/* Create a plain discrete-ordinates (SN) instance of the same problem: the
 * full-rank method the DLR step approximates (Sec. 2: backward Euler with the
 * linearised emission, source iteration on the scalar flux, every ordinate of
 * the n_polar x n_azim quadrature swept each iteration, the intensity of all
 * ordinates kept between steps).  rank and deim_tie_tol are ignored; precision
 * selects FP64 or FP32 sweeps (modes 1 and 2 behave alike: there are no
 * projections).  The handle takes dlr_step, dlr_sync, dlr_read_fields,
 * dlr_read_stats (rank reports the number of ordinates) and dlr_destroy;
 * dlr_read_factors, dlr_load_factors and dlr_force_selection return
 * DLR_ERR_UNSUPPORTED.  Device memory holds two [ordinates][cells] arrays of
 * the sweep precision.  Errors as dlr_create. */
dlr_status dlr_sn_create(const dlr_problem *prob, void *hip_stream, dlr_handle *out);

/* Advance n_steps >= 0 time steps (Algorithm 1).  Errors detected on the
 * device (non-convergence, non-finite values, rank breakdown) poison the
 * handle: this call and every later one except reads of the last good state
 * return the error or DLR_ERR_STATE. */
dlr_status dlr_step(dlr_handle h, int32_t n_steps);

/* Wait for all work queued on the handle's stream. */
dlr_status dlr_sync(dlr_handle h);

/* Radiation energy density E_r = phi / c and material temperature T, [ny*nx]
 * each (caller-allocated; either may be NULL).  Synchronises the stream. */
dlr_status dlr_read_fields(dlr_handle h, double *E_r, double *T);

/* Low-rank factors psi = X S W^T with <X_i, X_j> = delta_ij (cell-area
 * weighted), sum_q w_q W_qi W_qj = delta_ij and S = diag(sigma) descending:
 * X [ny*nx][rank], S [rank][rank], W [n_polar*n_azim][rank], sel [rank] = the
 * DEIM ordinates of the last step (-1 before the first step).  Any pointer may be NULL. */
dlr_status dlr_read_factors(dlr_handle h, double *X, double *S, double *W, int32_t *sel);

/* Replace the state (same layouts as dlr_read_factors; S may be any r x r
 * matrix); resets steps_done.  For checkpoint/resume. */
dlr_status dlr_load_factors(dlr_handle h, const double *X, const double *S, const double *W,
                            const double *T);

/* Diagnostics of the last step. */
dlr_status dlr_read_stats(dlr_handle h, dlr_step_stats *out);

/* Replay hook for parity checks: the next dlr_step uses these rank ordinate
 * indices instead of its own DEIM picks (one step only).  sel: [rank] distinct
 * indices in [0, n_polar*n_azim); NULL clears a pending override. */
dlr_status dlr_force_selection(dlr_handle h, const int32_t *sel);

/* Diffusion synthetic acceleration of the source iteration (Sec. 4, "Diffusion Synthetic
 * Acceleration (DSA) for SN-like DLR method", and its appendix derivation), for DLR and plain SN
 * handles.  After every sweep that has not met si_tol, the swept mean intensity phi_half is
 * corrected to phi_half + delta, where delta solves the consistent diffusion system of the
 * degree-0 cells
 *   [(1/3) sum_j F_j^T M_t^{-1} F_j + F_0 + M_a] delta = M_s (phi_half - phi_old)
 * (F_j: central face operators; F_0: jump penalty with kappa = sum_d c_d |Omega_d . n|, c the
 * collocation weights, or the quadrature weights for SN; M_t, M_s, M_a: cell-area masses of
 * sigma_t, the pseudo-scattering sigma_s and sigma_t - sigma_s; zero exterior values).  The
 * system is solved by Jacobi-preconditioned conjugate gradients in FP64 on the device to the
 * relative residual cg_tol (at most cg_max_iter iterations).  The converged step is the same fixed
 * point as without acceleration; in optically thick, strongly scattering media it takes far fewer
 * source iterations.  enable = 0 turns it off.  The first enable allocates a workspace of 7 FP64
 * cell fields (through the allocator hook if set).
 * Errors: DLR_ERR_ARG (cg_tol outside (0, 1), cg_max_iter outside [1, 100000]), DLR_ERR_OOM,
 * DLR_ERR_STATE (poisoned handle), DLR_ERR_HIP. */
dlr_status dlr_set_dsa(dlr_handle h, int32_t enable, double cg_tol, int32_t cg_max_iter);

/* Launch shape of the instance's transport sweeps (Algorithm 1 step 4): *prefetch = chunks of
 * loads each compute wavefront keeps in flight (2, 4 or 8), *grid_blocks = persistent
 * workgroups; both 0 before the first sweep.  Unless set below, the shape is chosen at the first
 * sweep by timing the candidates (prefetch 2, 4 and, with FP32 sweeps, 8; 256, 512 or 1024
 * workgroups) on the instance's own data, and kept for the life of the process per grid, number
 * of swept directions and sweep precision.  The shape changes no arithmetic: results are bitwise
 * the same for every shape.  Errors: DLR_ERR_ARG (NULL argument). */
dlr_status dlr_sweep_shape(dlr_handle h, int32_t *prefetch, int32_t *grid_blocks);

/* Fix the launch shape (prefetch 2 or 4, or 8 with FP32 sweeps; 1 <= grid_blocks <= 65535), or
 * (0, 0): back to the tuner's choice.  Errors: DLR_ERR_ARG (other values). */
dlr_status dlr_set_sweep_shape(dlr_handle h, int32_t prefetch, int32_t grid_blocks);

/* Free everything.  NULL-safe. */
dlr_status dlr_destroy(dlr_handle h);

/* ------------------------------------------------------------------------------------------
 * Batches and serving: many independent problems of uneven size and rank, resident on the
 * device, advanced together.  A batch owns an HBM budget; a problem is admitted into a slot
 * while its footprint fits (otherwise DLR_ERR_OOM: retry after a release) and keeps its
 * factors on the device until the slot is released.  Each dlr_batch_advance moves every active
 * slot one DLR step: the phases of all slots are issued on per-slot streams so their work
 * overlaps on the device, and every source iteration sweeps the directions of all unconverged
 * slots in one persistent launch.  Slots do not interact: a slot's results are bitwise those
 * of the same problem stepped alone with dlr_step.  The same stepping rules (Algorithm 1) and
 * error semantics apply per slot; a failed slot is finished with its error status and the
 * others go on.  Calls on one batch must be serialised by the caller. */
typedef struct dlr_batch_s *dlr_batch;

/* Device bytes a problem occupies once admitted (validates the problem like dlr_create). */
dlr_status dlr_batch_footprint(const dlr_problem *prob, size_t *bytes);

/* hbm_budget: bytes the batch may hold at once (0 = free device memory minus 1 GiB).
 * hip_stream: stream that orders the batch's shared sweep launches (NULL = default stream). */
dlr_status dlr_batch_create(size_t hbm_budget, void *hip_stream, dlr_batch *out);

/* Admit a problem for n_steps >= 1 steps.  *slot receives its id (increasing, never reused).
 * DLR_ERR_OOM: the footprint does not fit in what the budget has left; nothing was admitted. */
dlr_status dlr_batch_admit(dlr_batch b, const dlr_problem *prob, int32_t n_steps, int64_t *slot);

/* One DLR step of every active slot (slots that still have steps to take).  When the active
 * slots are the same as at the previous advance, the step runs from HIP graphs recorded for that
 * composition (every slot's kernels and the shared sweep launches, kernel nodes only; both
 * parities of the ping-pong buffers; re-recorded when the composition or the number of source
 * iterations changes): the source iteration is then decided on the device -- the scalar-flux
 * kernel of each slot counts the iteration and raises a stop flag at convergence (or a
 * non-finite change norm, or si_max_iter), and every later kernel of that slot's iteration,
 * including its units of the shared sweep, returns at once.  A slot that needs more iterations
 * than were recorded continues on the host's decision.  The arithmetic is the same on both paths
 * (the per-slot results stay bitwise those of dlr_step).  The allocator hook serves the recorded
 * tables; nothing is allocated while replaying. */
dlr_status dlr_batch_advance(dlr_batch b);

/* enable = 0: no recorded-graph steps for this batch; 1 (the default): recorded steps with up to
 * 8 source iterations recorded per step; 2..64: that many at most.  Any change drops the recorded
 * graphs.  Results do not depend on the setting.  Errors: DLR_ERR_ARG (enable outside [0, 64]). */
dlr_status dlr_batch_set_graphs(dlr_batch b, int32_t enable);

/* Steps advanced from recorded graphs since the batch was created (a diagnostic). */
dlr_status dlr_batch_graph_steps(dlr_batch b, int64_t *steps);

/* Slots that finished (all steps taken, or failed) since the last poll, oldest first:
 * up to cap ids in done[], their number in *n. */
dlr_status dlr_batch_poll(dlr_batch b, int64_t *done, int32_t cap, int32_t *n);

/* Fields of a slot (as dlr_read_fields); returns the slot's failure status if it failed. */
dlr_status dlr_batch_read(dlr_batch b, int64_t slot, double *E_r, double *T);

/* Statistics of the slot's most recent step (as dlr_read_stats). */
dlr_status dlr_batch_read_stats(dlr_batch b, int64_t slot, dlr_step_stats *out);

/* Free the slot and return its bytes to the budget. */
dlr_status dlr_batch_release(dlr_batch b, int64_t slot);

/* Active slots and bytes in use. */
dlr_status dlr_batch_usage(dlr_batch b, int32_t *active_slots, size_t *bytes_in_use);

/* Release every slot and free the batch.  NULL-safe. */
dlr_status dlr_batch_destroy(dlr_batch b);

/* ------------------------------------------------------------------------------------------
 * Bilinear (Q1) DG sweep: the transport solve of the paper's spatial discretisation
 * (Sec. 4.4, volume matrices G_j, face matrix F_d with central flux plus half the jump
 * penalty -- which is the upwind flux --, mass matrices) with the degree-1 tensor element
 * on each cell, 4 nodal values per cell and direction.  For every direction d and cell K it
 * solves, cells in upwind order,
 *   -int_K (Omega_d . grad v) psi + sum_{outflow faces} int (Omega_d . n) psi v + int_K sigma_t psi v
 *     = int_K s v + sum_{inflow faces} int |Omega_d . n| psi_upwind v      for all bilinear v on K,
 * psi_upwind being the neighbour's trace, or the inflow data on the domain boundary.
 *
 * Layouts (row-major, element type double for DLR_FP64, float for DLR_FP32_SWEEP):
 *   cell e = j*nx + i, node a = ix + 2*iy at the cell corners (ix = 0 left, 1 right;
 *   iy = 0 bottom, 1 top);
 *   sigma_t  [ny*nx]          total opacity per cell (>= 0);
 *   src      [n_dir][ny*nx][4] nodal values of the source (its bilinear interpolant enters
 *                             as M s);
 *   inflow_x [n_dir][ny][2]   row j's x-inflow face (left if mu > 0, else right), nodes iy;
 *   inflow_y [n_dir][nx][2]   column i's y-inflow face (bottom if eta > 0, else top), nodes ix;
 *   psi      [n_dir][ny*nx][4] output.
 * Arrays are device pointers owned by the caller; src and psi must be aligned to 4
 * elements, inflow arrays to 2.  Each call runs on the stream given at creation. */
typedef struct dlr_q1_s *dlr_q1;

/* Create a sweep operator for an nx x ny grid of hx x hy cells (nx, ny <= 2^20, nx * ny <=
 * 2^28) and n_dir directions (host arrays mu, eta; finite, not both zero; copied).  precision: DLR_FP64 or
 * DLR_FP32_SWEEP (all arithmetic in that type).  Device memory: the direction cosines and one
 * [n_dir][ceil(nx/128)][ny][2] edge buffer.  Errors: DLR_ERR_ARG, DLR_ERR_OOM, DLR_ERR_HIP. */
dlr_status dlr_q1_create(int32_t nx, int32_t ny, double hx, double hy, int32_t n_dir, const double *mu,
                         const double *eta, int32_t precision, void *hip_stream, dlr_q1 *out);

/* Queue one sweep of every direction (asynchronous).  A cell with sigma_t = 0 is fine; the
 * local systems are nonsingular for any sigma_t >= 0.  Errors: DLR_ERR_ARG (NULL or
 * misaligned array), DLR_ERR_HIP (launch), DLR_ERR_STATE (poisoned handle). */
dlr_status dlr_q1_sweep(dlr_q1 h, const void *sigma_t, const void *src, const void *inflow_x,
                        const void *inflow_y, void *psi);

/* Wait for the queued sweeps and check the device status: a cross-workgroup wait that
 * exceeded its spin limit returns DLR_ERR_TIMEOUT and poisons the handle. */
dlr_status dlr_q1_sync(dlr_q1 h);

/* Run reps >= 1 sweeps between two events on the handle's stream, synchronise, check the
 * status as dlr_q1_sync, and return the mean device time of one sweep in milliseconds. */
dlr_status dlr_q1_time(dlr_q1 h, const void *sigma_t, const void *src, const void *inflow_x,
                       const void *inflow_y, void *psi, int32_t reps, double *ms_per_sweep);

/* Free the operator (waits for its stream first).  NULL-safe. */
dlr_status dlr_q1_destroy(dlr_q1 h);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops
 * or harnesses that forbid hipMalloc): one sweep as dlr_q1_sweep, without an operator handle.
 * The arguments are those of dlr_q1_create and dlr_q1_sweep, except that mu and eta are DEVICE
 * arrays [n_dir] (finite, not both zero in a direction; not checked) and the stream must belong
 * to the current device.  status: device int32 owned by the caller, who clears it; the call ORs a
 * nonzero code into it when a cross-workgroup wait of the sweep exceeded its spin limit (what
 * dlr_q1_sync reports as DLR_ERR_TIMEOUT).  The call is asynchronous and allocates nothing: the
 * sweep's hand-off state (unit ticket, progress words, edge values) lives in a static device
 * array of 16 MiB per GPU, held until the process ends; it needs
 * 256 + 8 n_dir ceil(nx / 128) (rounded up to 256) + 2 n_dir ceil(nx / 128) ny * element bytes,
 * and larger problems are rejected with DLR_ERR_ARG before any work is queued.  Every call on a
 * GPU shares that array: calls that overlap on one GPU (different streams, or threads) race and
 * must be serialised by the caller; calls queued one after another on one stream are fine.
 * Errors: DLR_ERR_ARG (shape, NULL or misaligned array, scratch too small, stream of another
 * device), DLR_ERR_HIP (symbol lookup or launch), DLR_ERR_UNSUPPORTED (device index >= 64). */
dlr_status dlr_q1_sweep_noalloc(int32_t nx, int32_t ny, double hx, double hy, int32_t n_dir, const double *mu,
                                const double *eta, int32_t precision, void *hip_stream, const void *sigma_t,
                                const void *src, const void *inflow_x, const void *inflow_y, void *psi,
                                int32_t *status);

/* Static description of a status code. */
const char *dlr_status_string(dlr_status s);

/* Detail of the most recent error on the calling thread ("" if none). */
const char *dlr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DLRTRT_H */
