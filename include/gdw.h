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
 *  - Every nodal array passed in or out is a contiguous FP64 array of
 *    nx*ny*(N+1)^2 entries in DEVICE memory (hipMalloc'd or a torch CUDA tensor's
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
  GDW_EUNSUPPORTED = -6   /* a valid request this build does not implement        */
} gdw_status;

/* Numerical flux (Sec. 2.2.1): central alpha = 1/2, beta = tau = 0; upwind
 * alpha = 1/2, beta = xi/2, tau = 1/(2 xi).  The alternating flux is not offered. */
typedef enum { GDW_FLUX_CENTRAL = 0, GDW_FLUX_UPWIND = 1 } gdw_flux;

/* Arithmetic of the time loop.  GDW_FP64: state, tables and arithmetic in FP64.
 * GDW_MIXED_FP32: state and tables stored and computed in FP32; the eigenbasis is
 * built and the energy is accumulated in FP64. */
typedef enum { GDW_FP64 = 0, GDW_MIXED_FP32 = 1 } gdw_precision;

/* Local solve.  FDM: simultaneous diagonalisation (Sec. 3.2), constant c^2 on
 * Cartesian elements only.  AUTO picks FDM when it applies. */
typedef enum { GDW_SOLVE_AUTO = 0, GDW_SOLVE_FDM = 1, GDW_SOLVE_PCG = 2 } gdw_solver;

typedef struct {
  int nx, ny;          /* elements per direction (the paper's n)                     Sec. 2   */
  int N;               /* cells per element per direction, N >= p                    Sec. 2   */
  int p;               /* odd GD degree                                              Sec. 2   */
  double x0, y0;       /* lower-left corner of the periodic rectangle                          */
  double Lx, Ly;       /* its side lengths (> 0)                                               */
  double c2;           /* constant c^2 > 0 (variable c^2 is not offered by this build)          */
  int flux;            /* gdw_flux                                                   Sec. 2.2.1 */
  double xi;           /* upwind splitting speed xi > 0 (paper: xi = c)              Sec. 2.2.1 */
  int precision;       /* gdw_precision                                                       */
  int solver;          /* gdw_solver                                                          */
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
 * non-positive length, c2 or xi, an unknown enum; EUNSUPPORTED for solver PCG;
 * ENOMEM / EHIP from the device.  Uses the current HIP device; synchronous. */
gdw_status gdw_create(const gdw_desc* desc, gdw_ctx** out);

/* Load the state (u, v) from nodal values U, V (device FP64, layout above).  The
 * state is kept in the simultaneously diagonalised basis of Sec. 3.2
 * (U = Psi Ubar), so this call applies Psi^{-1} = Psi^T M per element and computes
 * the face traces of the new state.  Errors: EINVAL on NULL arguments. */
gdw_status gdw_set_state(gdw_ctx* ctx, const double* U, const double* V, void* stream);

/* Advance `steps` classical RK4 steps of size dt (> 0) on `stream` (asynchronous).
 * Each stage evaluates DG1 + DG1_extra, DG2 element by element with the face
 * fluxes and the local solves of Sec. 3.2, fused in one kernel per stage.
 * steps = 0 is a no-op.  Errors: EINVAL for dt <= 0 or not finite, steps < 0. */
gdw_status gdw_run(gdw_ctx* ctx, double dt, int steps, void* stream);

/* Write the nodal values of the current state to U, V (device FP64). */
gdw_status gdw_get_state(gdw_ctx* ctx, double* U, double* V, void* stream);

/* Discrete energy sum_k 1/2 V^T M V + 1/2 c^2 U^T S U (Sec. 2.2; conserved by the
 * central flux), accumulated in FP64 in a fixed order (deterministic).  Synchronises
 * `stream`; *E_host receives the value.  Returns ENONFINITE if it is not finite. */
gdw_status gdw_energy(gdw_ctx* ctx, double* E_host, void* stream);

typedef struct {
  long long steps_taken;     /* RK4 steps advanced since gdw_create                */
  long long dof_updates;     /* steps_taken * nx * ny * (N+1)^2                    */
  int n1;                    /* N + 1                                              */
  int precision;             /* gdw_precision in use                               */
  int solver;                /* gdw_solver in use (FDM or PCG)                     */
  int fail_elem;             /* first element with a failure, -1 if none           */
} gdw_stats;

/* Counters of the context.  Synchronises `stream`. */
gdw_status gdw_get_stats(gdw_ctx* ctx, gdw_stats* out, void* stream);

/* Free every device workspace of the context (NULL is ignored).  Synchronises the
 * device first so that no queued kernel still uses the context. */
void gdw_destroy(gdw_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* GDW_H */
