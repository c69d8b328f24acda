/*
 * gdw.h -- C ABI of the MI355X (gfx950) energy-based DG / Galerkin-difference
 * wave solver.
 *
 * Method: Zhang, Appelo, Hagstrom, "Energy-based discontinuous Galerkin
 * difference methods for second-order wave equations" (arXiv:2105.01722).
 * The library advances the semi-discretisation DG1 + DG1_extra, DG2 (Sec. 2.2)
 * of u_t = v, v_t = div(c^2 grad u) (Sec. 2, eqs. eq:wave_1, eq:wave_2) on a
 * periodic grid of nx x ny tensor-product elements, each carrying an (N+1)^2
 * Galerkin-difference basis of odd degree p with the extrapolation closure
 * (Sec. 2.1), with the numerical fluxes of Sec. 2.2.1 and classical RK4
 * (Sec. 3.3, Sec. 6).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Element e = ey*nx + ex covers [x0 + ex*Hx, x0 + (ex+1)*Hx] x [y0 + ey*Hy, ...],
 *    Hx = Lx/nx, Hy = Ly/ny.  Node (ix, iy), 0 <= ix, iy <= N, of element e sits at
 *    (x0 + ex*Hx + ix*Hx/N, y0 + ey*Hy + iy*Hy/N) and is stored at flat offset
 *    e*(N+1)^2 + iy*(N+1) + ix.  Face nodes are duplicated per element (DG).
 *  - 3D (desc.dim = 3): element e = (ez*ny + ey)*nx + ex adds [z0 + ez*Hz, ...] and node
 *    (ix, iy, iz) is stored at e*(N+1)^3 + (iz*(N+1) + iy)*(N+1) + ix; faces T / B are the
 *    z = R / z = L sides; the path is the constant-coefficient Cartesian one only.
 *  - Every nodal array passed in or out is a contiguous FP64 array of
 *    nx*ny*(N+1)^2 (3D: nx*ny*nz*(N+1)^3) entries in DEVICE memory (hipMalloc'd or a torch CUDA tensor's
 *    data_ptr), whatever the precision mode.  The library copies inputs into its own
 *    workspaces and never keeps a caller pointer.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Every call
 *    is asynchronous on that stream except gdw_energy and gdw_get_stats, which
 *    synchronise it.
 *  - Every call returns a gdw_status; on error a text is available from
 *    gdw_last_error() (per thread) and the context stays valid (it can be destroyed).
 *    No call aborts or exits the process.
 */
#ifndef GDW_H
#define GDW_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GDW_OK = 0,
  GDW_EINVAL = -1,        /* invalid argument or descriptor                      */
  GDW_ENOMEM = -2,        /* device allocation failed                            */
  GDW_EHIP = -3,          /* a HIP runtime call failed                           */
  GDW_ENOCONV = -4,       /* an element solve did not converge (PCG path)        */
  GDW_ENONFINITE = -5,    /* NaN or Inf found in the state after a run            */
  GDW_EUNSUPPORTED = -6   /* a valid request the library does not implement      */
} gdw_status;

/* Numerical flux (Sec. 2.2.1): central alpha = 1/2, beta = tau = 0; upwind
 * alpha = 1/2, beta = xi/2, tau = 1/(2 xi); alternating alpha = 1, beta = tau = 0 with
 * one orientation per face (the printed alpha = 1 with superscript 1 the inside would be
 * two-valued): v* is the value of the element on the low-coordinate side (smaller x or
 * y) and (grad u)* the gradient of the element on the high side, so an element takes
 * alpha = 1 on its E and N faces and alpha = 0 on its W and S faces.  Wall faces take
 * alpha = 1/2 for every flux (with beta = tau = 0 the mirror state then gives v* = 0 on a
 * Dirichlet wall and n . (grad u)* = 0 on a Neumann wall). */
typedef enum { GDW_FLUX_CENTRAL = 0, GDW_FLUX_UPWIND = 1, GDW_FLUX_ALTERNATING = 2 } gdw_flux;

/* Arithmetic of the time loop.  GDW_FP64: state, tables and arithmetic in FP64.
 * GDW_MIXED_FP32, constant-coefficient path: every stage right-hand side (fluxes, lifts,
 * diagonal solve, traces) is evaluated in FP32 from FP32 stage values and tables; the RK4
 * stage registers hold FP32 increments Y - y (so their rounding scales with dt |k|, not
 * |y|) and the step is accumulated into y in FP64; the eigenbasis is built, and the
 * energy, get_state and the non-finite check read y, in FP64.  GDW_MIXED_FP32, PCG
 * path: the state stays FP64; the element operator is split into FP32 parts
 * hi = fl32(A), lo = fl32(A - hi); the inner PCG iterations use hi, and every solve is
 * refined with FP64 residuals b - (hi + lo) x until the FP64 residual meets pcg_rtol
 * (requires N + 1 in {9, 13, 17}; else EUNSUPPORTED).  GDW_MIXED_PC32, PCG path only: the
 * tensor-product preconditioner's four transforms (Sec. 7.1) run in FP32 on the matrix
 * cores inside the FP64 recurrence; operator products, residuals, the stop test and the
 * state stay FP64, so the solves meet pcg_rtol as in GDW_FP64 (requires N + 1 in {9, 13}
 * with p in {5, 7}, or N + 1 = 13 with p = 3; else EUNSUPPORTED). */
typedef enum { GDW_FP64 = 0, GDW_MIXED_FP32 = 1, GDW_MIXED_PC32 = 2 } gdw_precision;

/* Local solve.  FDM: simultaneous diagonalisation (Sec. 3.2), constant c^2 on
 * Cartesian elements only.  PCG: preconditioned conjugate gradients per element
 * (Sec. 7.1) with the tensor-product preconditioner built from element averages;
 * required for variable c^2 or mapped elements.  AUTO picks FDM when it applies. */
typedef enum { GDW_SOLVE_AUTO = 0, GDW_SOLVE_FDM = 1, GDW_SOLVE_PCG = 2 } gdw_solver;

/* Kind of one side of the rectangle.  The paper states no boundary flux (its 2D
 * Dirichlet experiment, Sec. 6, has homogeneous data), so a wall face uses the interior
 * flux of Sec. 2.2.1 with a mirror exterior state built from the element's own traces:
 * DIRICHLET (u = 0): v_ext = -v, a_ext = -a (a = outward normal derivative);
 * NEUMANN (du/dn = 0): v_ext = v, a_ext = a.  On the GD grid this equals the periodic
 * scheme on the rectangle mirrored across the wall with odd (even) data.  A direction
 * is periodic on both of its sides or on neither.  On the PCG path (mapped elements) the
 * mirror is taken at the face quadrature points of the wall face. */
typedef enum { GDW_BC_PERIODIC = 0, GDW_BC_DIRICHLET = 1, GDW_BC_NEUMANN = 2 } gdw_bc;

typedef struct {
  int nx, ny;          /* elements per direction (the paper's n)                     Sec. 2   */
  int N;               /* cells per element per direction, N >= p                    Sec. 2   */
  int p;               /* odd GD degree                                              Sec. 2   */
  double x0, y0;       /* lower-left corner of the rectangle                                   */
  double Lx, Ly;       /* its side lengths (> 0)                                               */
  double c2;           /* constant c^2 > 0 (used when coeff_variable = 0)                      */
  int flux;            /* gdw_flux                                                   Sec. 2.2.1 */
  double xi;           /* upwind splitting speed xi > 0 (paper: xi = c)              Sec. 2.2.1 */
  int precision;       /* gdw_precision                                                       */
  int solver;          /* gdw_solver                                                          */
  int coeff_variable;  /* 1: c^2 given at the nodes by gdw_set_coeff (PCG path)      Sec. 7.1 */
  int mapped;          /* 1: element node coordinates given by gdw_set_coeff (PCG path)        */
  double pcg_rtol;     /* PCG stop: ||r||_2 <= pcg_rtol ||b||_2, r the CG recurrence
                          residual (r_0 = b - A x_0); <= 0: 1e-12                     Sec. 7.1 */
  int pcg_maxit;       /* PCG iteration limit per element solve (<= 0: 200)                   */
  int bc[4];           /* gdw_bc of the sides x = x0 + Lx (E), x = x0 (W), y = y0 + Ly (N),
                          y = y0 (S); all zero: periodic in x and y                            */
  int dim;             /* 2 (or 0) or 3: box elements nx x ny x nz (Sec. 2.2 with d = 3)       */
  int nz;              /* 3D: elements in z                                                    */
  double z0, Lz;       /* 3D: the box's z range [z0, z0 + Lz]                                  */
  int bcz[2];          /* 3D: gdw_bc of the sides z = z0 + Lz (T), z = z0 (B)                  */
} gdw_desc;

typedef struct gdw_ctx gdw_ctx;   /* opaque; owns every device workspace */

/* Library version string (static storage). */
const char* gdw_version(void);

/* Text of the last error raised on the calling thread ("" if none). */
const char* gdw_last_error(void);

/* Validate `desc` and build the element tables: 1D GD mass / stiffness / face
 * vectors (Sec. 3.1, Sec. 3.2) on the host, the generalised eigenbasis
 * S_j psi = lambda M_j psi with psi^T M_j psi = 1 (Sec. 3.2) in FP64 on the device.
 * Errors: EINVAL for a NULL pointer, p even or < 1, N < p, N + 1 > 32, nx or ny < 1, a
 * non-positive length, c2 or xi, an unknown enum, solver FDM with a variable
 * coefficient or a mapped mesh, a direction periodic on one side only, dim not 0, 2 or
 * 3, or in 3D nz < 1 or Lz <= 0; EUNSUPPORTED in 3D for (N + 1)^3 > 1024 (one thread per
 * modal index of an element) or anything but the constant-coefficient Cartesian path, and
 * for the PCG path with p > 7 or, outside the FP64 families whose solves keep no operator
 * in LDS (N + 1 = 9, 13 with p = 3, 5, 7; N + 1 = 17 with p = 3, 5, 7), an element operator
 * that does not fit the 160 KiB of LDS of a workgroup, for the PCG path in
 * GDW_MIXED_FP32 with N + 1 outside {9, 13, 17}, and for GDW_MIXED_PC32 on the
 * constant-coefficient path or outside the PCG families that offer it; ENOMEM / EHIP from
 * the device.  Uses the current HIP device;
 * synchronous. */
gdw_status gdw_create(const gdw_desc* desc, gdw_ctx** out);

/* PCG path only: element geometry and coefficient, then assembly (Sec. 7.1).
 * c2_nodal: c^2 at every node (device FP64, layout above), NULL = desc.c2 everywhere;
 * X_nodal, Y_nodal: physical coordinates of every node, NULL = the Cartesian node
 * positions of the descriptor.  Both copies of a face node must carry the same
 * coordinates and c^2 (a conforming mesh); every element map must have a positive
 * Jacobian (not checked).  Each element is the isoparametric GD image of the
 * reference square; S_K, M_J, w and the face metric are integrated with (p+1)^2
 * Gauss points per cell and p+1 per face cell.  Must precede gdw_set_state.
 * Errors: EINVAL on the FDM path, on NULL ctx, or when only one of X, Y is given. */
gdw_status gdw_set_coeff(gdw_ctx* ctx, const double* c2_nodal, const double* X_nodal,
                         const double* Y_nodal, void* stream);

/* Load the state (u, v) from nodal values U, V (device FP64, layout above).  On the
 * FDM path the state is kept in the simultaneously diagonalised basis of Sec. 3.2
 * (U = Psi Ubar), so this call applies Psi^{-1} = Psi^T M per element; on the PCG path
 * it is kept nodal and the PCG warm starts are reset to zero.  Either way the face
 * traces of the new state are computed.  Errors: EINVAL on NULL arguments, or on the
 * PCG path before gdw_set_coeff. */
gdw_status gdw_set_state(gdw_ctx* ctx, const double* U, const double* V, void* stream);

/* Source term of the PDE (Sec. 2: u_tt = div(c^2 grad u) + f):
 * f(x, y, t) = sum_k sin(omega[k] t + phase[k]) g_k(x, y), k < nterms <= 4, with t the time
 * advanced by gdw_run since the last gdw_set_state.  g_nodal holds the nterms fields
 * back to back, each at every node (device FP64, layout above); each g_k is represented
 * by its GD interpolant, like the initial data, so its load vector is M g_k (M_J g_k on
 * mapped elements) and it adds sum_k s_k(t) g_k to dv/dt (on the FDM path as the modal
 * coefficients of Sec. 3.2, computed here once).  2D only (EUNSUPPORTED in 3D).  RK4 evaluates the weights s_k at the
 * stage times t, t + dt/2, t + dt/2, t + dt: before each step a one-lane kernel computes
 * the step's weights from a device clock and advances it (also inside a batch's captured
 * step).
 * g_k is given at the nodes' physical positions.  omega, phase: host arrays of nterms
 * values.  nterms = 0 removes the term.  The library copies g; the call synchronises
 * `stream`.  Errors: EINVAL for a NULL ctx, nterms outside 0..4, a NULL array with
 * nterms > 0 or a non-finite omega / phase.  A batch rebuilds its captured step after
 * a member's source term changes. */
gdw_status gdw_set_forcing(gdw_ctx* ctx, int nterms, const double* g_nodal, const double* omega,
                           const double* phase, void* stream);

/* Advance `steps` classical RK4 steps of size dt (> 0) on `stream` (asynchronous).
 * Each stage evaluates DG1 + DG1_extra, DG2 element by element with the face
 * fluxes and the local solves (Sec. 3.2 FDM, or Sec. 7.1 PCG warm-started from the
 * previous stage), fused in one kernel per stage.  A PCG solve that reaches
 * pcg_maxit is reported by gdw_get_stats (ENOCONV), not here.
 * steps = 0 is a no-op.  Errors: EINVAL for dt <= 0 or not finite, steps < 0. */
gdw_status gdw_run(gdw_ctx* ctx, double dt, int steps, void* stream);

/* Write the nodal values of the current state to U, V (device FP64). */
gdw_status gdw_get_state(gdw_ctx* ctx, double* U, double* V, void* stream);

/* Discrete energy sum_k 1/2 V^T M V + 1/2 U^T S_{c^2} U (Sec. 2.2; conserved by the
 * central flux), accumulated in FP64 in a fixed order (deterministic).  Synchronises
 * `stream`; *E_host receives the value.  Returns ENONFINITE if it is not finite. */
gdw_status gdw_energy(gdw_ctx* ctx, double* E_host, void* stream);

typedef struct {
  long long steps_taken;     /* RK4 steps advanced since gdw_create                */
  long long dof_updates;     /* steps_taken * nx * ny * (N+1)^2                    */
  int n1;                    /* N + 1                                              */
  int precision;             /* gdw_precision in use                               */
  int solver;                /* gdw_solver in use (FDM or PCG)                     */
  int fail_elem;             /* first element whose PCG hit pcg_maxit, -1 if none  */
  double mean_it_S;          /* PCG: mean iterations per S_hat solve (dU/dt)        */
  double mean_it_M;          /* PCG: mean iterations per M_J solve (dV/dt)          */
  int max_it_S, max_it_M;    /* PCG: largest single-solve counts                   */
  long long solves;          /* PCG: element solves of each kind since set_state   */
  double mean_refine;        /* PCG, GDW_MIXED_FP32: mean FP64 refinement sweeps per
                                solve (residual evaluations after the first)         */
} gdw_stats;

/* Counters of the context.  Synchronises `stream`.  Returns ENOCONV (with
 * fail_elem set) if a PCG solve reached pcg_maxit, ENONFINITE if the state holds
 * NaN or Inf; *out is filled in either case. */
gdw_status gdw_get_stats(gdw_ctx* ctx, gdw_stats* out, void* stream);

/* Free every device workspace of the context (NULL is ignored).  Synchronises the
 * device first so that no queued kernel still uses the context. */
void gdw_destroy(gdw_ctx* ctx);

/* ---------------------------------------------------------------------------------
 * Learned correction of the PCG preconditioner (an addition to the paper's method).
 *
 * The tensor-product preconditioner of the S_hat solve has the modal diagonal
 * D_(ky,kx) = kbar_rr lam_kx + kbar_ss lam_ky (Sec. 3.2 eigenbasis, element averages).  A
 * correction multiplies every entry but (0,0) by exp(o_k).  o comes either from a
 * caller-given array or from a small network (64 -> H -> H -> (N+1)^2 - 1, ReLU) applied
 * to the element's standardised coefficient samples ((c^2 - 1)/0.5 at the centres of an
 * 8 x 8 subdivision of the reference square).  The network runs on the matrix cores:
 * FP16 weights with FP32 accumulation forward, FP32 backward, Adam with FP32 master
 * weights.  Non-finite o is replaced by 0 and |o| is clipped at 8, so the corrected
 * preconditioner stays symmetric positive definite; a learned S_hat solve that reaches
 * pcg_maxit is repeated with the plain preconditioner.
 * ------------------------------------------------------------------------------- */
typedef struct gdw_mlp gdw_mlp;

/* Network with n_in inputs, two hidden layers of `hidden` units and n_out outputs; He
 * initialisation from `seed` (std::mt19937_64, Box-Muller), zero biases.  Workspaces
 * are sized for minibatches of up to max_batch rows.  Errors: EINVAL for non-positive
 * sizes or NULL out. */
gdw_status gdw_mlp_create(int n_in, int hidden, int n_out, unsigned long long seed, int max_batch,
                          gdw_mlp** out);

/* Number of parameters; flat layout W1[hidden][n_in], b1[hidden], W2[hidden][hidden],
 * b2[hidden], W3[n_out][hidden], b3[n_out]. */
gdw_status gdw_mlp_num_params(const gdw_mlp* mlp, long long* n);

/* Copy the FP32 master parameters to / from host memory (synchronous); set also resets
 * the Adam state. */
gdw_status gdw_mlp_get_params(gdw_mlp* mlp, float* host);
gdw_status gdw_mlp_set_params(gdw_mlp* mlp, const float* host);

/* out[n][n_out] = network(x[n][n_in]); device FP32 arrays; any n >= 0 (chunked). */
gdw_status gdw_mlp_forward(gdw_mlp* mlp, const float* x, int n, float* out, void* stream);

/* Gradient (device FP32, flat layout) of mean((network(x) - y)^2) over one minibatch of
 * n <= max_batch rows, and that loss in *loss_host (synchronises `stream`). */
gdw_status gdw_mlp_grad(gdw_mlp* mlp, const float* x, const float* y, int n, float* grad,
                        double* loss_host, void* stream);

/* The gradient of gdw_mlp_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): same arguments and
 * results, except that the loss goes to device memory (*loss, one FP64 value) and the call
 * does not synchronise.  It calls no allocator: the minibatch's activations and partial
 * sums live in a fixed 8 MiB device array of the library (one per device, held until the
 * process ends), so n (the number of rows) is limited by 4 n (6 hidden + 2 n_out) + 512 <= 8 MiB
 * (n <= 1899 for 64 -> 128 -> 128 -> 168); larger n returns EINVAL.  grad: device FP32,
 * num_params entries; x, y as for gdw_mlp_grad.  Every call on one device shares that
 * array and overwrites it: calls that overlap on one device (other streams or threads)
 * race, so serialise them. */
gdw_status gdw_mlp_grad_noalloc(gdw_mlp* mlp, const float* x, const float* y, int n, float* grad,
                                double* loss, void* stream);

/* Adam training (lr, b1 = 0.9, b2 = 0.999, eps = 1e-8) over `epochs` passes of contiguous
 * minibatches of `batch` rows (the last one shorter) of (x, y), device FP32 arrays.
 * loss_host[epoch] receives the mean minibatch loss of each epoch (synchronises). */
gdw_status gdw_mlp_train(gdw_mlp* mlp, const float* x, const float* y, int n, int epochs, int batch,
                         float lr, double* loss_host, void* stream);

void gdw_mlp_destroy(gdw_mlp* mlp);

/* PCG path: training data from the assembled operators of the context (after
 * gdw_set_coeff): samples[n_el][64] (standardised coefficient samples) and
 * targets[n_el][(N+1)^2 - 1] = log(d_k / D_k), d = diag(Psi_2^T S_hat Psi_2) (the exact
 * modal diagonal).  Device FP32 arrays; either may be NULL.  Errors: EINVAL on the FDM
 * path or before gdw_set_coeff. */
gdw_status gdw_precond_data(gdw_ctx* ctx, float* samples, float* targets, void* stream);

/* PCG path: o = network(samples of every element) becomes the preconditioner correction.
 * Errors: EINVAL if the network is not 64 -> ... -> (N+1)^2 - 1 or before gdw_set_coeff. */
gdw_status gdw_set_precond_mlp(gdw_ctx* ctx, gdw_mlp* mlp, void* stream);

/* PCG path: o given directly: device FP32, contiguous [n_el][(N+1)^2 - 1] with
 * n_el = nx * ny, read in full on the given stream (the caller keeps it alive until that
 * read has run); NULL restores the plain preconditioner.  The length cannot be checked
 * here: a shorter buffer is an out-of-bounds device read. */
gdw_status gdw_set_precond_log(gdw_ctx* ctx, const float* log_scale, void* stream);

/* IC(0) baseline (Sec. 7.1: the paper inverts the element matrices by PCG with an
 * incomplete Cholesky preconditioner).  2D PCG path, after gdw_set_coeff.  For every
 * element e: factor the element matrix by zero-fill incomplete Cholesky on the GD stencil
 * (|jx - ix| <= p, |jy - iy| <= p; op 0 takes S_hat's entries on that stencil, the
 * rank-one mean term being dense), then solve S_hat x_e = b_e (op 0, the dU/dt system) or
 * M_J x_e = b_e (op 1, the dV/dt system) by CG with that preconditioner from x_e = 0,
 * stopping when ||r||_2 <= rtol ||b_e||_2 (r the CG recurrence residual) or after maxit
 * iterations.  b, x: device FP64 [n_el][(N+1)^2] (element e = ey * nx + ex, node
 * iy * (N+1) + ix), its: device int [n_el] iteration counts; the caller owns all three.
 * A baseline beside the time loop's tensor-product preconditioner, not part of gdw_run:
 * the first call allocates two operator-sized workspaces (2 n_el nst doubles, nst the
 * upper-half stencil size), kept until gdw_destroy; every call synchronises the stream.
 * Errors: EINVAL (FDM path, 3D, before gdw_set_coeff, op not 0/1, maxit < 1),
 * ENOCONV (a non-positive pivot, or maxit reached; gdw_last_error names the element),
 * ENOMEM. */
gdw_status gdw_ic0_solve(gdw_ctx* ctx, int op, const double* b, double* x, double rtol,
                         int maxit, int* its, void* stream);

/* ---------------------------------------------------------------------------------
 * Batches of independent problems (an addition for throughput on one GPU).
 *
 * A batch owns nprob contexts, created as by gdw_create from descs[i] (any mix of
 * solvers, precisions, N and p).  Each RK stage of all problems runs as one grouped,
 * persistent launch per kernel class (constant-coefficient problems grouped by
 * precision and N+1, PCG problems by N+1), and the four stages of one step are captured
 * once into a HIP graph that gdw_batch_run launches once per step.  Launch shapes
 * (elements per workgroup, block size, grid size) are chosen per class by timing the
 * candidates on the problems' own data (gdw_batch_tune) and kept for the life of the
 * process, keyed by the device architecture, path, arithmetic, kernel family and member
 * sizes: a later class with the same key takes the stored shape untimed.  Every problem
 * advances exactly as gdw_run would advance it alone.
 * --------------------------------------------------------------------------------- */
typedef struct gdw_batch gdw_batch;

/* Create the batch; 1 <= nprob <= 4096.  Errors: those of gdw_create for a problem
 * (the message names it), EUNSUPPORTED for a 3D problem; nothing is left allocated on
 * error. */
gdw_status gdw_batch_create(int nprob, const gdw_desc* descs, gdw_batch** out);

/* Context of problem i, owned by the batch: set its coefficients and state, read its
 * state, energy and counters with the single-problem calls.  Do not destroy it. */
gdw_status gdw_batch_ctx(gdw_batch* batch, int i, gdw_ctx** ctx);

/* Choose the launch shape of every class by timing candidates (stage 1 of the class's
 * own problems, with scratch copies of the PCG warm starts), for the per-problem steps
 * dt[nprob] (host array).  The problems' states are unchanged.  Synchronises `stream`.
 * Every problem must have a state.  gdw_batch_run tunes on first use if this was not
 * called. */
gdw_status gdw_batch_tune(gdw_batch* batch, const double* dt, void* stream);

/* Advance every problem i by `steps` RK4 steps of dt[i] (host array): one graph launch
 * per step, asynchronous on `stream`.  The graph is rebuilt when dt changes. */
gdw_status gdw_batch_run(gdw_batch* batch, const double* dt, int steps, void* stream);

/* Durations (ms) of the n = steps steps of the last gdw_batch_run, from events recorded
 * between the graph launches (synchronises on the last one). */
gdw_status gdw_batch_step_times(gdw_batch* batch, float* ms, int n);

/* Text: the chosen launch shape of every class and the timed candidates (empty before
 * tuning).  Valid until the next tuning or gdw_batch_destroy. */
const char* gdw_batch_plan(gdw_batch* batch);

/* Destroy the batch and every context it owns (synchronises the device; NULL ignored). */
void gdw_batch_destroy(gdw_batch* batch);

#ifdef __cplusplus
}
#endif
#endif /* GDW_H */
