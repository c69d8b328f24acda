// Constant-coefficient Cartesian path: the energy-DG right-hand side of
// DG1 + DG1_extra, DG2 (Sec. 2.2) fused with the local solves by simultaneous
// diagonalisation (Sec. 3.2) and the classical RK4 stage update, one kernel per
// RK stage.
//
// State representation (Sec. 3.2): U = Psi Ubar, V = Psi Vbar with
// Psi = Psi_x (x) Psi_y, S_j psi = lambda M_j psi, psi^T M_j psi = 1.  In that basis
//   dUbar/dt = Vbar + Lambda_hat^{-1} Psi^T F_u      (DG1_sparse; mode (0,0) from DG1_extra)
//   dVbar/dt = -c^2 Lambda Ubar + Psi^T F_v          (DG2_sparse)
// with Lambda = lambda_x (+) lambda_y.  The face terms are rank one per face
// (Sec. 3.2, B/C/D/E-tilde): on the east face F_u = c^2 dR_x (x) M_y sigma_u, so
// Psi^T F_u = c^2 (Psi_x^T dR_x) (x) (Psi_y^T M_y sigma_u); and because every trace along
// the face is a GD function in the face coordinate, Psi_y^T M_y sigma_u is the same
// combination of the modal face coefficients of the traces (Psi_y^T M_y Psi_y = I).
// So a stage needs, per element, only 8 modal trace vectors of length N+1 of
// itself and of its neighbours, which the previous stage wrote.
//
// Arithmetic per DOF and stage: 8 MACs of lifts + the diagonal solve, plus 8 (N+1)
// MACs per element row for the traces of the new state: the kernel is bound by
// HBM bandwidth.
//
// Layout in HBM: modal arrays are element-major, [e][ky][kx] (kx fastest), one
// array per field.  Traces: [e][8][N+1], slot f2 = 0 aE, 1 vE, 2 aW, 3 vW, 4 aN,
// 5 vN, 6 aS, 7 vS, where a = outward normal derivative and v = value on the face.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "fdm.h"

namespace gdw {

// ---------------------------------------------------------------------------------
// Double-double helpers (error-free transformations: Knuth's TwoSum and the fma-based
// TwoProduct) for the residuals of the eigenpair refinement below.
// ---------------------------------------------------------------------------------
struct dd { double hi, lo; };

__device__ inline dd dd_two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}

// x + a*b with a, b doubles
__device__ inline dd dd_fma(dd x, double a, double b) {
  const double p = a * b;
  const double pe = fma(a, b, -p);
  dd s = dd_two_sum(x.hi, p);
  s.lo += x.lo + pe;
  return dd_two_sum(s.hi, s.lo);
}

// x + a*y with y double-double
__device__ inline dd dd_fma_dd(dd x, double a, dd y) {
  x = dd_fma(x, a, y.hi);
  x.lo += a * y.lo;
  return dd_two_sum(x.hi, x.lo);
}

// One refinement sweep of the eigenpairs of S x = lambda M x (Ogita and Aishima's
// iteration for symmetric eigenproblems, in its M-orthonormal form): with
// R = I - X^T M X and T = X^T S X evaluated in double-double,
// lambda_i = T_ii / (1 - R_ii), E_ii = R_ii / 2 and, for i != j,
// E_ij = (T_ij + lambda_j R_ij) / (lambda_j - lambda_i); X <- X + X E.
// Pairs closer than 1e-3 max|lambda| are treated as a cluster, E_ij = R_ij / 2 (the
// method's rule for close eigenvalues): the GD pencils have close pairs at the top of the
// spectrum (relative gap 6e-4 at N = 16, p = 5, 2e-7 at N = 31, p = 7), and dividing by
// such a gap amplifies the rounding of the FP64 update (X^T M X drifted from I by 1e-13
// at N = 31).  Inside a cluster the rotation keeps Jacobi's accuracy, eps / gap <= 1e-13,
// which changes X Lambda X^T by about 1e-16 relative.
// X = Psi [n][n] (column k = eigenvector k), lam [n]; R, T [n][n] and col [4n] scratch.
__device__ void eig_refine_sweep(const double* M, const double* S, int n, double* X, double* lam,
                                 double* R, double* T, double* col, bool update) {
  for (int j = 0; j < n; ++j) {
    dd* mx = reinterpret_cast<dd*>(col);          // (M X)_{:, j}
    dd* sx = mx + n;                              // (S X)_{:, j}
    for (int i = 0; i < n; ++i) {
      dd a = {0.0, 0.0}, b = {0.0, 0.0};
      for (int k = 0; k < n; ++k) {
        a = dd_fma(a, M[i * n + k], X[k * n + j]);
        b = dd_fma(b, S[i * n + k], X[k * n + j]);
      }
      mx[i] = a;
      sx[i] = b;
    }
    for (int i = 0; i < n; ++i) {
      dd a = {0.0, 0.0}, b = {0.0, 0.0};
      for (int k = 0; k < n; ++k) {
        a = dd_fma_dd(a, X[k * n + i], mx[k]);
        b = dd_fma_dd(b, X[k * n + i], sx[k]);
      }
      const dd r = dd_two_sum((i == j ? 1.0 : 0.0) - a.hi, -a.lo);
      R[i * n + j] = r.hi + r.lo;
      T[i * n + j] = b.hi + b.lo;
    }
  }
  for (int i = 0; i < n; ++i) lam[i] = T[i * n + i] / (1.0 - R[i * n + i]);
  if (!update) return;
  double lmax = 0.0;
  for (int i = 0; i < n; ++i) lmax = fmax(lmax, fabs(lam[i]));
  // E overwrites T
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      const double gap = lam[j] - lam[i];
      T[i * n + j] = (fabs(gap) > 1e-3 * lmax) ? (T[i * n + j] + lam[j] * R[i * n + j]) / gap
                                               : 0.5 * R[i * n + j];
    }
  for (int i = 0; i < n; ++i) T[i * n + i] = 0.5 * R[i * n + i];
  // X <- X + X E, row by row
  for (int r = 0; r < n; ++r) {
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s = fma(X[r * n + k], T[k * n + j], s);
      col[j] = s;
    }
    for (int j = 0; j < n; ++j) X[r * n + j] += col[j];
  }
}

// ---------------------------------------------------------------------------------
// FP64 generalised symmetric eigensolver S psi = lambda M psi for one (N+1)^2 pencil:
// Cholesky M = L L^T, C = L^{-1} S L^{-T}, cyclic Jacobi on C, Psi = L^{-T} Q, then two
// refinement sweeps with double-double residuals, which bring the eigenbasis to FP64
// rounding of the exact one (the FDM solve represents the element operator through
// Psi and lambda, so their backward error is the solver's).
// Runs on a single lane; setup only.  work: 3 n^2 + 5 n doubles; info: 1 + n ints.
// ---------------------------------------------------------------------------------
__global__ void k_eig_pencil(const double* __restrict__ M, const double* __restrict__ S, int n,
                             double* __restrict__ work, double* __restrict__ Psi,
                             double* __restrict__ lam, int* __restrict__ info) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double* L = work;
  double* C = work + n * n;
  double* Q = work + 2 * n * n;
  int ok = 1;
  // Cholesky (lower)
  for (int j = 0; j < n; ++j) {
    double d = M[j * n + j];
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 0.0)) { ok = 0; d = 1.0; }
    const double ljj = sqrt(d);
    L[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double s = M[i * n + j];
      for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = s / ljj;
    }
    for (int i = 0; i < j; ++i) L[i * n + j] = 0.0;
  }
  // Q <- L^{-1} S   (column by column forward substitution)
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double s = S[i * n + c];
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * Q[k * n + c];
      Q[i * n + c] = s / L[i * n + i];
    }
  // C <- L^{-1} Q^T  (= L^{-1} S L^{-T} as S is symmetric)
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double s = Q[c * n + i];
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * C[k * n + c];
      C[i * n + c] = s / L[i * n + i];
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double a = 0.5 * (C[i * n + j] + C[j * n + i]);
      C[i * n + j] = C[j * n + i] = a;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Q[i * n + j] = (i == j) ? 1.0 : 0.0;
  // cyclic Jacobi
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += C[i * n + i] * C[i * n + i];
      for (int j = i + 1; j < n; ++j) off += C[i * n + j] * C[i * n + j];
    }
    if (off <= 1e-34 * diag) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = C[p * n + q];
        if (apq == 0.0) continue;
        const double theta = (C[q * n + q] - C[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double ckp = C[k * n + p], ckq = C[k * n + q];
          C[k * n + p] = c * ckp - s * ckq;
          C[k * n + q] = s * ckp + c * ckq;
        }
        for (int k = 0; k < n; ++k) {
          const double cpk = C[p * n + k], cqk = C[q * n + k];
          C[p * n + k] = c * cpk - s * cqk;
          C[q * n + k] = s * cpk + c * cqk;
        }
        C[p * n + q] = C[q * n + p] = 0.0;
        for (int k = 0; k < n; ++k) {
          const double qkp = Q[k * n + p], qkq = Q[k * n + q];
          Q[k * n + p] = c * qkp - s * qkq;
          Q[k * n + q] = s * qkp + c * qkq;
        }
      }
  }
  // eigenvalues = diagonal of the converged C
  double* D = work + 3 * n * n;
  for (int i = 0; i < n; ++i) D[i] = C[i * n + i];
  // Psi <- L^{-T} Q (back substitution), unsorted, into C's storage
  for (int c = 0; c < n; ++c)
    for (int i = n - 1; i >= 0; --i) {
      double s = Q[i * n + c];
      for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * C[k * n + c];
      C[i * n + c] = s / L[i * n + i];
    }
  // sort ascending (selection); Psi[i*n + k] = psi_k(i); sign: largest entry positive
  int* used = info + 1;
  for (int k = 0; k < n; ++k) used[k] = 0;
  for (int k = 0; k < n; ++k) {
    int best = -1;
    for (int j = 0; j < n; ++j)
      if (!used[j] && (best < 0 || D[j] < D[best])) best = j;
    used[best] = 1;
    int imax = 0;
    double vmax = 0.0;
    for (int i = 0; i < n; ++i)
      if (fabs(C[i * n + best]) > vmax * (1.0 + 1e-12)) { vmax = fabs(C[i * n + best]); imax = i; }
    const double sg = C[imax * n + best] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < n; ++i) Psi[i * n + k] = sg * C[i * n + best];
    lam[k] = D[best];
  }
  // refinement (L, C, Q and D are free now): R = work, T = work + n^2, col = work + 2 n^2
  if (ok) {
    for (int it = 0; it < 2; ++it)
      eig_refine_sweep(M, S, n, Psi, lam, work, work + n * n, work + 2 * n * n, true);
    eig_refine_sweep(M, S, n, Psi, lam, work, work + n * n, work + 2 * n * n, false);
  }
  lam[0] = 0.0;   // the constant mode has lambda = 0 exactly
  info[0] = ok;
}

// ---------------------------------------------------------------------------------
// nodal (FP64) -> modal (T):  Ubar[ky][kx] = sum Py[ky][iy] Px[kx][ix] U[iy][ix],
// P = Psi^T M = Psi^{-1}.  One workgroup per element.
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void k_to_modal(const double* __restrict__ U, T* __restrict__ Ub,
                           const double* __restrict__ Px, const double* __restrict__ Py,
                           int n1, long nel) {
  extern __shared__ double sh[];
  const int nn = n1 * n1;
  double* u = sh;
  double* tmp = sh + nn;
  const long e = blockIdx.x;
  if (e >= nel) return;
  for (int i = threadIdx.x; i < nn; i += blockDim.x) u[i] = U[e * nn + i];
  __syncthreads();
  for (int i = threadIdx.x; i < nn; i += blockDim.x) {
    const int iy = i / n1, kx = i - iy * n1;
    double s = 0.0;
    for (int ix = 0; ix < n1; ++ix) s += Px[kx * n1 + ix] * u[iy * n1 + ix];
    tmp[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nn; i += blockDim.x) {
    const int ky = i / n1, kx = i - ky * n1;
    double s = 0.0;
    for (int iy = 0; iy < n1; ++iy) s += Py[ky * n1 + iy] * tmp[iy * n1 + kx];
    Ub[e * nn + i] = (T)s;
  }
}

// modal (T) -> nodal (FP64):  U[iy][ix] = sum Psi_y[iy][ky] Psi_x[ix][kx] Ubar[ky][kx]
template <typename T>
__global__ void k_to_nodal(const T* __restrict__ Ub, double* __restrict__ U,
                           const double* __restrict__ Psx, const double* __restrict__ Psy,
                           int n1, long nel) {
  extern __shared__ double sh[];
  const int nn = n1 * n1;
  double* u = sh;
  double* tmp = sh + nn;
  const long e = blockIdx.x;
  if (e >= nel) return;
  for (int i = threadIdx.x; i < nn; i += blockDim.x) u[i] = (double)Ub[e * nn + i];
  __syncthreads();
  for (int i = threadIdx.x; i < nn; i += blockDim.x) {
    const int ky = i / n1, ix = i - ky * n1;
    double s = 0.0;
    for (int kx = 0; kx < n1; ++kx) s += Psx[ix * n1 + kx] * u[ky * n1 + kx];
    tmp[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nn; i += blockDim.x) {
    const int iy = i / n1, ix = i - iy * n1;
    double s = 0.0;
    for (int ky = 0; ky < n1; ++ky) s += Psy[iy * n1 + ky] * tmp[ky * n1 + ix];
    U[e * nn + i] = s;
  }
}

// ---------------------------------------------------------------------------------
// Modal face traces of a state (used once after set_state; every stage kernel
// writes the traces of its output itself).
// ---------------------------------------------------------------------------------
template <typename S, typename T>
__global__ void k_traces(const S* __restrict__ Ub, const S* __restrict__ Vb,
                         const double* __restrict__ gh, T* __restrict__ tr, int n1, long nel) {
  const int nn = n1 * n1;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nel * 8 * n1) return;
  const long e = i / (8 * n1);
  const int r = (int)(i - e * 8 * n1);
  const int f2 = r / n1, j = r - f2 * n1;
  const S* F = ((f2 & 1) ? Vb : Ub) + e * nn;
  const double* g = gh + f2 * n1;
  double acc = 0;
  if (f2 < 4)
    for (int k = 0; k < n1; ++k) acc += g[k] * (double)F[j * n1 + k];
  else
    for (int k = 0; k < n1; ++k) acc += g[k] * (double)F[k * n1 + j];
  tr[i] = (T)acc;
}

// sum_k g[k] F[j][k] (contraction along kx) and sum_k g[k] F[k][j] (along ky)
template <typename T, int N1C>
__device__ inline T dot_row(const T* g, const T* F, int j, int n1) {
  T acc = 0;
  if constexpr (N1C > 0) {
#pragma unroll
    for (int k = 0; k < N1C; ++k) acc += g[k] * F[j * N1C + k];
  } else {
    for (int k = 0; k < n1; ++k) acc += g[k] * F[j * n1 + k];
  }
  return acc;
}

template <typename T, int N1C>
__device__ inline T dot_col(const T* g, const T* F, int j, int n1) {
  T acc = 0;
  if constexpr (N1C > 0) {
#pragma unroll
    for (int k = 0; k < N1C; ++k) acc += g[k] * F[k * N1C + j];
  } else {
    for (int k = 0; k < n1; ++k) acc += g[k] * F[k * n1 + j];
  }
  return acc;
}

// ---------------------------------------------------------------------------------
// The fused RK stage.
// FP64 (T = double):
//   STAGE 1: in = y;      out = Y  <- y + dt/2 k1
//   STAGE 2: in = Y, y;   out = Y  <- y + dt/2 k2 (in place),  Tacc <- Yin + 2 Ynew - y
//   STAGE 3: in = Y, y;   out = Y  <- y + dt k3 (in place)
//   STAGE 4: in = Y, Tacc; out = y <- (Tacc + Yin)/3 + dt/6 k4
// Classical RK4 (y_{n+1} = y + dt/6 (k1 + 2k2 + 2k3 + k4)) with Y2 = y + dt/2 k1,
// Y3 = y + dt/2 k2, Y4 = y + dt k3, because
// (Y2 + 2 Y3 + Y4 - y)/3 = y + dt/6 k1 + dt/3 k2 + dt/3 k3.  12 field accesses per
// DOF per step instead of the 16 of the textbook three-register form.
//
// FP32 storage (T = float): the same scheme in increments.  y lives in FP64 (y64); the
// stage registers hold FP32 increments dY_s = Y_s - y and A = dY2 + 2 dY3, so their
// rounding scales with dt |k| instead of |y|, and y accumulates the step in FP64:
//   STAGE 1: in = y64;           out = dY2 <- dt/2 k(y)
//   STAGE 2: in = dY2, y64;      out = dY3 <- dt/2 k(y + dY2) (in place), A <- dY2 + 2 dY3
//   STAGE 3: in = dY3, y64;      out = dY4 <- dt k(y + dY3) (in place)
//   STAGE 4: in = dY4, A, y64;   y64 <- y + (A + dY4)/3 + dt/6 k(y + dY4)
// (y_{n+1} = y + (dY2 + 2 dY3 + dY4)/3 + dt/6 k4 is the form above with Y_s = y + dY_s.)
// The right-hand side stays FP64 arithmetic: in the modal v-equation,
// dVbar/dt = c^2 (lifts - Lambda Ubar) cancels terms of size Lambda |Ubar| down to about
// omega^2 |Ubar| (the lifts carry the boundary terms of the high modes).  A variant that
// evaluated it in FP32 from an FP32 copy of y measured, after 100 steps of the
// 256 x 256, N = 16 workload, 2e-7 relative l2 and 1.0e-6 relative max error in v (u:
// 8e-10); the kernel is bound by HBM bandwidth, so the FP64 arithmetic costs nothing.
// Traces are stored in FP32.
// Bytes per DOF, field and step:
//   stage 1: y r (8 B), dY w (4)     stage 2: y, dY r, dY, A w (20)
//   stage 3: y, dY r, dY w (16)      stage 4: y, dY, A r, y w (24)
// = 72 B against 96 B in FP64.
// ---------------------------------------------------------------------------------
// Thread map: one workgroup of (N+1)^2 threads handles EPB consecutive elements;
// thread t owns the modal index (kx, ky) = (t mod (N+1), t div (N+1)) in every one of
// them.  So the per-index tables (the diagonal solve and the face vectors at kx and
// ky) sit in registers for the whole kernel, and the element loop is uniform across
// the workgroup: state addresses are a scalar element base plus the thread's fixed
// offset.
// One tile (EPB consecutive elements, tile index `tile`) of one problem.
// Streaming access to the per-element state.  Each state word is read once and
// written once per stage, so FP64 words bypass the cache hierarchy's normal
// allocation (nontemporal): measured at the 256x256, N = 16 workload this saves about
// 3% per stage.  FP32 words are half as large and run faster with ordinary accesses.
template <typename T>
__device__ __forceinline__ T ld_state(const T* p) {
  if constexpr (sizeof(T) == 8) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename T>
__device__ __forceinline__ void st_state(T* p, T v) {
  if constexpr (sizeof(T) == 8) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// The RK stage update of one modal coefficient g (both register schemes above): stores
// what the stage writes and returns the new stage value (su, sv), whose traces go to the
// next stage.  (ru, rv, xu, xv): the loaded in / aux words; (yu, yv): y in FP64 (FP32
// storage only); (ub, vb): the stage value the right-hand side (ku, kv) was evaluated at.
template <typename T, int STAGE>
__device__ __forceinline__ void rk_stage_store(const StageArgs<T>& a, long g, T ru, T rv, T xu,
                                               T xv, double yu, double yv, double ub, double vb,
                                               double ku, double kv, double& su, double& sv) {
  constexpr bool MIX = sizeof(T) == 4;
  using R = double;
  const R dt = a.dt;
  if constexpr (MIX) {
    if (STAGE == 4) {          // ru = dY4, xu = A
      const R h6 = dt * (1.0 / 6.0);
      su = yu + ((R)xu + (R)ru) * (1.0 / 3.0) + h6 * ku;
      sv = yv + ((R)xv + (R)rv) * (1.0 / 3.0) + h6 * kv;
      st_state(&a.y64_u[g], su);
      st_state(&a.y64_v[g], sv);
    } else {
      const R w = STAGE == 3 ? dt : R(0.5) * dt;
      const T nu = (T)(w * ku), nv = (T)(w * kv);     // the stored increment
      st_state(&a.out_u[g], nu);
      st_state(&a.out_v[g], nv);
      if (STAGE == 2) {        // ru = dY2
        st_state(&a.acc_u[g], (T)((R)ru + R(2) * (R)nu));
        st_state(&a.acc_v[g], (T)((R)rv + R(2) * (R)nv));
      }
      su = yu + (R)nu;
      sv = yv + (R)nv;
    }
  } else {
    if (STAGE == 1) {          // the input is y itself
      su = ub + R(0.5) * dt * ku;
      sv = vb + R(0.5) * dt * kv;
    } else if (STAGE == 2) {   // xu, xv = y
      su = (R)xu + R(0.5) * dt * ku;
      sv = (R)xv + R(0.5) * dt * kv;
      st_state(&a.acc_u[g], (T)(ub + R(2) * su - (R)xu));
      st_state(&a.acc_v[g], (T)(vb + R(2) * sv - (R)xv));
    } else if (STAGE == 3) {   // xu, xv = y
      su = (R)xu + dt * ku;
      sv = (R)xv + dt * kv;
    } else {                   // xu, xv = accumulator
      su = ((R)xu + ub) * R(1.0 / 3.0) + dt * R(1.0 / 6.0) * ku;
      sv = ((R)xv + vb) * R(1.0 / 3.0) + dt * R(1.0 / 6.0) * kv;
    }
    st_state(&a.out_u[g], (T)su);
    st_state(&a.out_v[g], (T)sv);
  }
}

// FRC: the source term is present (a.nf > 0); without it the kernel is compiled as
// if it did not exist.
template <typename T, int STAGE, int N1C, int EPB, bool FRC = false>
__device__ __forceinline__ void stage_tile(const StageArgs<T>& a, long tile) {
  // FP32 storage runs the increment form around the FP64 register y
  constexpr bool MIX = sizeof(T) == 4;
  using R = double;                              // arithmetic
  const int n1 = N1C > 0 ? N1C : a.n1;
  const int nn = n1 * n1;
  const int tid = threadIdx.x;                   // blockDim.x == nn
  const int ky = tid / n1, kx = tid - ky * n1;
  extern __shared__ unsigned char smem_raw[];
  R* sgh = reinterpret_cast<R*>(smem_raw);       // [8][n1] face tables
  R* sig = sgh + 8 * n1;                         // [EPB][8][n1] modal face fluxes
  R* snew = sig + EPB * 8 * n1;                  // [EPB][2][nn] new stage values
  const long e0 = tile * EPB;
  const int ne = (int)min((long)EPB, a.nel - e0);

  // Issue the state loads of all EPB elements first, so that their HBM latency
  // overlaps the trace loads and the flux computation.  An element's state is read
  // and written only by this workgroup, so loading it all before the (in-place)
  // stores is safe.
  // FP64 storage: ru = in, xu = aux.  FP32 storage: yu = y, ru = the stage increment
  // (stages 2-4), xu = A (stage 4).
  // (loaded values stay in their storage type until use: fewer registers in FP32)
  T ru[EPB], rv[EPB], xu[EPB], xv[EPB];
  R yu[EPB], yv[EPB];
#pragma unroll
  for (int l = 0; l < EPB; ++l) {
    ru[l] = rv[l] = xu[l] = xv[l] = T(0);
    yu[l] = yv[l] = R(0);
    if (l < ne) {
      const long g = (e0 + l) * nn + tid;
      if constexpr (MIX) {
        yu[l] = ld_state(&a.y64_u[g]);
        yv[l] = ld_state(&a.y64_v[g]);
        if (STAGE > 1) {
          ru[l] = ld_state(&a.in_u[g]);
          rv[l] = ld_state(&a.in_v[g]);
        }
        if (STAGE == 4) {
          xu[l] = ld_state(&a.aux_u[g]);
          xv[l] = ld_state(&a.aux_v[g]);
        }
      } else {
        ru[l] = ld_state(&a.in_u[g]);
        rv[l] = ld_state(&a.in_v[g]);
        if (STAGE > 1) {
          xu[l] = ld_state(&a.aux_u[g]);
          xv[l] = ld_state(&a.aux_v[g]);
        }
      }
    }
  }
  const R il = a.invL[tid], lm = a.lam[tid];
  const R gEk = a.gh[0 * n1 + kx], hEk = a.gh[1 * n1 + kx];
  const R gWk = a.gh[2 * n1 + kx], hWk = a.gh[3 * n1 + kx];
  const R gNk = a.gh[4 * n1 + ky], hNk = a.gh[5 * n1 + ky];
  const R gSk = a.gh[6 * n1 + ky], hSk = a.gh[7 * n1 + ky];
  for (int i = tid; i < 8 * n1; i += blockDim.x) sgh[i] = a.gh[i];

  // Phase A: modal face fluxes sigma_u = (1-alpha)(v_nb - v) - beta (a + a_nb),
  // sigma_v = (1-alpha) a - alpha a_nb + tau (v_nb - v)  (Sec. 2.2.1); alpha per face
  // (the alternating flux is oriented: 1 on E and N faces, 0 on W and S), 1/2 on walls
  const R beta = a.beta, tau = a.tau;
  for (int i = tid; i < ne * 4 * n1; i += blockDim.x) {
    const int el = i / (4 * n1);
    const int r = i - el * 4 * n1;
    const int f = r / n1, j = r - f * n1;
    const long e = e0 + el;
    const int ex = (int)(e % a.nx), ey = (int)(e / a.nx);
    // Neighbour across face f (periodic wrap).  On a wall face (its side is not periodic
    // and the element touches it) the exterior state is the mirror of the element's own
    // traces: read its own face with the sign -1 (Dirichlet) or +1 (Neumann).
    const int kf = (a.bcbits >> (2 * f)) & 3;
    long enb;
    int fnb;
    bool wall;
    if (f == 0) { wall = ex + 1 == a.nx; enb = (long)ey * a.nx + (wall ? 0 : ex + 1); fnb = 1; }
    else if (f == 1) { wall = ex == 0; enb = (long)ey * a.nx + (wall ? a.nx - 1 : ex - 1); fnb = 0; }
    else if (f == 2) { wall = ey + 1 == a.ny; enb = (long)(wall ? 0 : ey + 1) * a.nx + ex; fnb = 3; }
    else { wall = ey == 0; enb = (long)(wall ? a.ny - 1 : ey - 1) * a.nx + ex; fnb = 2; }
    wall = wall && kf != 0;
    const T* ts = a.tr_in + e * 8 * n1 + 2 * f * n1;
    const T* tn = wall ? ts : a.tr_in + enb * 8 * n1 + 2 * fnb * n1;
    const R as = ts[j], vs = ts[n1 + j];
    R an = tn[j], vn = tn[n1 + j];
    if (wall && kf == 1) {
      an = -an;
      vn = -vn;
    }
    const R alpha = wall ? R(0.5) : (R)a.alf[f];
    const R jv = vn - vs;
    sig[(el * 8 + 2 * f) * n1 + j] = (R(1) - alpha) * jv - beta * (as + an);
    sig[(el * 8 + 2 * f + 1) * n1 + j] = (R(1) - alpha) * as - alpha * an + tau * jv;
  }
  __syncthreads();

  // Phase B: modal right-hand side and the RK stage update
  const R c2 = a.c2;
#pragma unroll
  for (int l = 0; l < EPB; ++l) {
    if (l >= ne) break;
    const R* s = sig + l * 8 * n1;
    // the stage value the right-hand side is evaluated at
    R ub = (R)ru[l], vb = (R)rv[l];
    if constexpr (MIX) {
      ub = STAGE == 1 ? yu[l] : yu[l] + (R)ru[l];
      vb = STAGE == 1 ? yv[l] : yv[l] + (R)rv[l];
    }
    const R Lu = gEk * s[0 * n1 + ky] + gWk * s[2 * n1 + ky] + gNk * s[4 * n1 + kx] +
                 gSk * s[6 * n1 + kx];
    const R Lv = hEk * s[1 * n1 + ky] + hWk * s[3 * n1 + ky] + hNk * s[5 * n1 + kx] +
                 hSk * s[7 * n1 + kx];
    const R ku = vb + il * Lu;
    R kv = c2 * (Lv - lm * ub);
    const long g = (e0 + l) * nn + tid;
    if constexpr (FRC) {
      // + sum_k s_k(t) Psi^T M g_k: the modal coefficients of the interpolated g_k
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < a.nf) kv += a.fw[4 * (STAGE - 1) + k] * (R)a.frc[k * a.frc_stride + g];
    }
    R su, sv;     // the new stage value (its traces go to the next stage)
    rk_stage_store<T, STAGE>(a, g, ru[l], rv[l], xu[l], xv[l], yu[l], yv[l], ub, vb, ku, kv, su,
                             sv);
    snew[(l * 2) * nn + tid] = su;
    snew[(l * 2 + 1) * nn + tid] = sv;
  }
  __syncthreads();

  // Phase C: modal face traces of the new state for the next stage
  for (int i = tid; i < ne * 8 * n1; i += blockDim.x) {
    const int el = i / (8 * n1);
    const int r = i - el * 8 * n1;
    const int f2 = r / n1, j = r - f2 * n1;
    const R* F = snew + (el * 2 + (f2 & 1)) * nn;
    const R* gg = sgh + f2 * n1;
    a.tr_out[e0 * 8 * n1 + i] =
        (T)((f2 < 4) ? dot_row<R, N1C>(gg, F, j, n1) : dot_col<R, N1C>(gg, F, j, n1));
  }
}

template <typename T, int STAGE, int N1C, int EPB, bool FRC>
__global__ __launch_bounds__(1024) void k_stage(StageArgs<T> a) {
  stage_tile<T, STAGE, N1C, EPB, FRC>(a, blockIdx.x);
}

// Grouped, persistent form: the tiles of several problems of one class (same T, N+1,
// EPB) in one launch.  Problem i owns tiles [tile_start[i], tile_start[i+1]); block b
// takes tiles b, b + gridDim.x, ... in increasing order, so its problem index only
// moves forward.  Every tile of every problem is independent within a stage.
template <typename T, int STAGE, int N1C, int EPB>
__global__ __launch_bounds__(1024) void k_stage_group(const StageArgs<T>* __restrict__ args,
                                                      const long* __restrict__ tile_start,
                                                      int nprob) {
  const long total = tile_start[nprob];
  int pi = 0;
  for (long b = blockIdx.x; b < total; b += gridDim.x) {
    while (pi + 1 < nprob && b >= tile_start[pi + 1]) ++pi;
    // the source-term build: without a source (nf = 0) it adds nothing, so members stay
    // bitwise equal to their solo runs
    stage_tile<T, STAGE, N1C, EPB, true>(args[pi], b - tile_start[pi]);
    __syncthreads();   // the next tile reuses the LDS
  }
}

// ---------------------------------------------------------------------------------
// Energy 1/2 sum (Vbar^2 + c^2 Lambda Ubar^2) (Psi^T M Psi = I, Psi^T S Psi = Lambda),
// FP64, two passes with a fixed reduction tree (deterministic).
// ---------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_energy_partial(const T* __restrict__ Ub,
                                                        const T* __restrict__ Vb,
                                                        const double* __restrict__ lam, double c2,
                                                        int nn, long total,
                                                        double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int idx = (int)(i % nn);
    const double u = (double)Ub[i], v = (double)Vb[i];
    s += v * v + c2 * lam[idx] * u * u;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_fixed(const double* __restrict__ part, int n,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = 0.5 * red[0];
}

// count of non-finite entries (end-of-run check)
template <typename T>
__global__ void k_count_nonfinite(const T* __restrict__ a, long n, unsigned int* __restrict__ cnt) {
  unsigned int c = 0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    if (!isfinite((double)a[i])) ++c;
  if (c) atomicAdd(cnt, c);
}

// ---------------------------------------------------------------------------------
// host launch wrappers
// ---------------------------------------------------------------------------------
hipError_t launch_eig(const double* M, const double* S, int n, double* work, double* Psi,
                      double* lam, int* info, hipStream_t st) {
  hipLaunchKernelGGL(k_eig_pencil, dim3(1), dim3(1), 0, st, M, S, n, work, Psi, lam, info);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_to_modal(const double* U, T* Ub, const double* Px, const double* Py, int n1,
                           long nel, hipStream_t st) {
  if (nel == 0) return hipSuccess;
  size_t sh = 2 * n1 * n1 * sizeof(double);
  hipLaunchKernelGGL(k_to_modal<T>, dim3((unsigned)nel), dim3(256), sh, st, U, Ub, Px, Py, n1, nel);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_to_nodal(const T* Ub, double* U, const double* Psx, const double* Psy, int n1,
                           long nel, hipStream_t st) {
  if (nel == 0) return hipSuccess;
  size_t sh = 2 * n1 * n1 * sizeof(double);
  hipLaunchKernelGGL(k_to_nodal<T>, dim3((unsigned)nel), dim3(256), sh, st, Ub, U, Psx, Psy, n1, nel);
  return hipGetLastError();
}

template <typename S, typename T>
hipError_t launch_traces(const S* Ub, const S* Vb, const double* gh, T* tr, int n1, long nel,
                         hipStream_t st) {
  const long total = nel * 8 * n1;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL((k_traces<S, T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, Ub,
                     Vb, gh, tr, n1, nel);
  return hipGetLastError();
}

template <typename T, int STAGE, int N1C, int EPB>
static hipError_t launch_stage_t(const StageArgs<T>& a, hipStream_t st) {
  const int n1 = a.n1;
  const size_t sh = stage_lds_bytes(n1, EPB);
  const unsigned nblk = (unsigned)((a.nel + EPB - 1) / EPB);
  if (a.nf > 0)
    hipLaunchKernelGGL((k_stage<T, STAGE, N1C, EPB, true>), dim3(nblk), dim3(n1 * n1), sh, st, a);
  else
    hipLaunchKernelGGL((k_stage<T, STAGE, N1C, EPB, false>), dim3(nblk), dim3(n1 * n1), sh, st, a);
  return hipGetLastError();
}

// Elements per workgroup: 4 when they fit 64 KiB of LDS, else fewer (in FP32, 8 measured
// 1 % slower than 4 on the 256 x 256, N = 16 workload).
template <typename T, int STAGE, int N1C>
static hipError_t dispatch_epb(const StageArgs<T>& a, hipStream_t st) {
  auto bytes = [&](int epb) { return stage_lds_bytes(a.n1, epb); };
  if (a.n1 * a.n1 > 1024) return hipErrorInvalidValue;
  constexpr int E0 = 4;
  if (bytes(E0) <= 65536) return launch_stage_t<T, STAGE, N1C, E0>(a, st);
  if (bytes(2) <= 65536) return launch_stage_t<T, STAGE, N1C, 2>(a, st);
  if (bytes(1) <= 65536) return launch_stage_t<T, STAGE, N1C, 1>(a, st);
  return hipErrorInvalidValue;
}

template <typename T, int STAGE>
static hipError_t dispatch_n1(const StageArgs<T>& a, hipStream_t st) {
  switch (a.n1) {
    case 9: return dispatch_epb<T, STAGE, 9>(a, st);
    case 13: return dispatch_epb<T, STAGE, 13>(a, st);
    case 17: return dispatch_epb<T, STAGE, 17>(a, st);
    default: return dispatch_epb<T, STAGE, 0>(a, st);
  }
}

template <typename T>
hipError_t launch_stage(int stage, const StageArgs<T>& a, hipStream_t st) {
  if (a.nel == 0) return hipSuccess;
  switch (stage) {
    case 1: return dispatch_n1<T, 1>(a, st);
    case 2: return dispatch_n1<T, 2>(a, st);
    case 3: return dispatch_n1<T, 3>(a, st);
    default: return dispatch_n1<T, 4>(a, st);
  }
}

size_t stage_lds_bytes(int n1, int epb) {
  return (size_t)(8 * n1 + epb * 8 * n1 + epb * 2 * n1 * n1) * sizeof(double);
}

template <typename T, int STAGE, int N1C, int EPB>
static hipError_t launch_group_t(const StageArgs<T>* args, const long* tile_start, int nprob,
                                 int n1, unsigned grid, hipStream_t st) {
  const size_t sh = stage_lds_bytes(n1, EPB);
  hipLaunchKernelGGL((k_stage_group<T, STAGE, N1C, EPB>), dim3(grid), dim3(n1 * n1), sh, st, args,
                     tile_start, nprob);
  return hipGetLastError();
}

template <typename T, int STAGE, int N1C>
static hipError_t group_epb(int epb, const StageArgs<T>* args, const long* ts, int np, int n1,
                            unsigned grid, hipStream_t st) {
  switch (epb) {
    case 1: return launch_group_t<T, STAGE, N1C, 1>(args, ts, np, n1, grid, st);
    case 2: return launch_group_t<T, STAGE, N1C, 2>(args, ts, np, n1, grid, st);
    case 4: return launch_group_t<T, STAGE, N1C, 4>(args, ts, np, n1, grid, st);
    case 8: return launch_group_t<T, STAGE, N1C, 8>(args, ts, np, n1, grid, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int STAGE>
static hipError_t group_n1(int epb, const StageArgs<T>* args, const long* ts, int np, int n1,
                           unsigned grid, hipStream_t st) {
  switch (n1) {
    case 9: return group_epb<T, STAGE, 9>(epb, args, ts, np, n1, grid, st);
    case 13: return group_epb<T, STAGE, 13>(epb, args, ts, np, n1, grid, st);
    case 17: return group_epb<T, STAGE, 17>(epb, args, ts, np, n1, grid, st);
    default: return group_epb<T, STAGE, 0>(epb, args, ts, np, n1, grid, st);
  }
}

template <typename T>
hipError_t launch_stage_group(int stage, int n1, int epb, const StageArgs<T>* args,
                              const long* tile_start, int nprob, unsigned grid, hipStream_t st) {
  if (nprob <= 0 || grid == 0) return hipSuccess;
  if (n1 * n1 > 1024 || stage_lds_bytes(n1, epb) > 65536) return hipErrorInvalidValue;
  switch (stage) {
    case 1: return group_n1<T, 1>(epb, args, tile_start, nprob, n1, grid, st);
    case 2: return group_n1<T, 2>(epb, args, tile_start, nprob, n1, grid, st);
    case 3: return group_n1<T, 3>(epb, args, tile_start, nprob, n1, grid, st);
    default: return group_n1<T, 4>(epb, args, tile_start, nprob, n1, grid, st);
  }
}

template <typename T>
int stage_group_occupancy(int stage, int n1, int epb) {
  (void)stage;
  // blocks per CU allowed by LDS (64 KiB per block at most, 160 KiB per CU) and threads
  const size_t lds = stage_lds_bytes(n1, epb);
  int by_lds = (int)((160 * 1024) / (lds ? lds : 1));
  int by_thr = 2048 / (((n1 * n1 + 63) / 64) * 64);
  int b = by_lds < by_thr ? by_lds : by_thr;
  return b < 1 ? 1 : b;
}

template <typename T>
hipError_t launch_energy(const T* Ub, const T* Vb, const double* lam, double c2, int nn, long nel,
                         double* part, int npart, double* out, hipStream_t st) {
  const long total = nel * (long)nn;
  hipLaunchKernelGGL(k_energy_partial<T>, dim3(npart), dim3(256), 0, st, Ub, Vb, lam, c2, nn,
                     total, part);
  hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, st, part, npart, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_count_nonfinite(const T* a, long n, unsigned int* cnt, hipStream_t st) {
  if (n == 0) return hipSuccess;
  long nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_count_nonfinite<T>, dim3((unsigned)nb), dim3(256), 0, st, a, n, cnt);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------------
// Box elements in three dimensions (Sec. 2.2 with d = 3; Sec. 3.1 / 3.2 Kronecker forms).
//
// The same modal-state scheme: Psi = Psi_x (x) Psi_y (x) Psi_z, Lambda = lambda_x (+)
// lambda_y (+) lambda_z, and the face terms are rank one per face: on the east face
// Psi^T F_u = c^2 (Psi_x^T dR_x) (x) (modal face coefficients of sigma_u), the face
// coefficients indexed by the two tangential modes.  Traces [e][12][n1^2]: slot 2f
// (a) and 2f + 1 (v) of face f = E, W, N, S, T, B; the face arrays are indexed
// [kz][ky] (E, W), [kz][kx] (N, S) and [ky][kx] (T, B).
// Thread map: one workgroup of n1^3 threads handles EPB consecutive elements, thread t
// owns the modal index (kx, ky, kz) = (t mod n1, (t div n1) mod n1, t div n1^2).
// ---------------------------------------------------------------------------------
__host__ __device__ inline size_t stage3_lds_doubles(int n1, int epb) {
  return (size_t)12 * n1 + (size_t)epb * 12 * n1 * n1 + (size_t)epb * 2 * n1 * n1 * n1;
}

template <typename T, int STAGE, int N1C, int EPB>
__device__ __forceinline__ void stage_tile3(const StageArgs<T>& a, long tile) {
  constexpr bool MIX = sizeof(T) == 4;
  using R = double;
  const int n1 = N1C > 0 ? N1C : a.n1;
  const int n2 = n1 * n1, n3 = n2 * n1;
  const int tid = threadIdx.x;                   // blockDim.x == n3
  const int kx = tid % n1, ky = (tid / n1) % n1, kz = tid / n2;
  extern __shared__ unsigned char smem_raw[];
  R* sgh = reinterpret_cast<R*>(smem_raw);       // [12][n1] face tables
  R* sig = sgh + 12 * n1;                        // [EPB][12][n2] modal face fluxes
  R* snew = sig + EPB * 12 * n2;                 // [EPB][2][n3] new stage values
  const long e0 = tile * EPB;
  const int ne = (int)min((long)EPB, a.nel - e0);

  T ru[EPB], rv[EPB], xu[EPB], xv[EPB];
  R yu[EPB], yv[EPB];
#pragma unroll
  for (int l = 0; l < EPB; ++l) {
    ru[l] = rv[l] = xu[l] = xv[l] = T(0);
    yu[l] = yv[l] = R(0);
    if (l < ne) {
      const long g = (e0 + l) * n3 + tid;
      if constexpr (MIX) {
        yu[l] = ld_state(&a.y64_u[g]);
        yv[l] = ld_state(&a.y64_v[g]);
        if (STAGE > 1) {
          ru[l] = ld_state(&a.in_u[g]);
          rv[l] = ld_state(&a.in_v[g]);
        }
        if (STAGE == 4) {
          xu[l] = ld_state(&a.aux_u[g]);
          xv[l] = ld_state(&a.aux_v[g]);
        }
      } else {
        ru[l] = ld_state(&a.in_u[g]);
        rv[l] = ld_state(&a.in_v[g]);
        if (STAGE > 1) {
          xu[l] = ld_state(&a.aux_u[g]);
          xv[l] = ld_state(&a.aux_v[g]);
        }
      }
    }
  }
  const R il = a.invL[tid], lm = a.lam[tid];
  const R gEk = a.gh[0 * n1 + kx], hEk = a.gh[1 * n1 + kx];
  const R gWk = a.gh[2 * n1 + kx], hWk = a.gh[3 * n1 + kx];
  const R gNk = a.gh[4 * n1 + ky], hNk = a.gh[5 * n1 + ky];
  const R gSk = a.gh[6 * n1 + ky], hSk = a.gh[7 * n1 + ky];
  const R gTk = a.gh[8 * n1 + kz], hTk = a.gh[9 * n1 + kz];
  const R gBk = a.gh[10 * n1 + kz], hBk = a.gh[11 * n1 + kz];
  for (int i = tid; i < 12 * n1; i += blockDim.x) sgh[i] = a.gh[i];

  // Phase A: modal face fluxes of the six faces (Sec. 2.2.1), mirror states on walls
  const R beta = a.beta, tau = a.tau;
  const long nxy = (long)a.nx * a.ny;
  for (int i = tid; i < ne * 6 * n2; i += blockDim.x) {
    const int el = i / (6 * n2);
    const int r = i - el * 6 * n2;
    const int f = r / n2, j = r - f * n2;
    const long e = e0 + el;
    const int ez = (int)(e / nxy);
    const int rem = (int)(e - ez * nxy);
    const int ey = rem / a.nx, ex = rem - (rem / a.nx) * a.nx;
    const int kf = (a.bcbits >> (2 * f)) & 3;
    int nbx = ex, nby = ey, nbz = ez, fnb;
    bool wall;
    if (f == 0) { wall = ex + 1 == a.nx; nbx = wall ? 0 : ex + 1; fnb = 1; }
    else if (f == 1) { wall = ex == 0; nbx = wall ? a.nx - 1 : ex - 1; fnb = 0; }
    else if (f == 2) { wall = ey + 1 == a.ny; nby = wall ? 0 : ey + 1; fnb = 3; }
    else if (f == 3) { wall = ey == 0; nby = wall ? a.ny - 1 : ey - 1; fnb = 2; }
    else if (f == 4) { wall = ez + 1 == a.nz; nbz = wall ? 0 : ez + 1; fnb = 5; }
    else { wall = ez == 0; nbz = wall ? a.nz - 1 : ez - 1; fnb = 4; }
    wall = wall && kf != 0;
    const long enb = ((long)nbz * a.ny + nby) * a.nx + nbx;
    const T* ts = a.tr_in + e * 12 * n2 + 2 * f * n2;
    const T* tn = wall ? ts : a.tr_in + enb * 12 * n2 + 2 * fnb * n2;
    const R as = ts[j], vs = ts[n2 + j];
    R an = tn[j], vn = tn[n2 + j];
    if (wall && kf == 1) {
      an = -an;
      vn = -vn;
    }
    const R alpha = wall ? R(0.5) : (R)a.alf[f];
    const R jv = vn - vs;
    sig[(el * 12 + 2 * f) * n2 + j] = (R(1) - alpha) * jv - beta * (as + an);
    sig[(el * 12 + 2 * f + 1) * n2 + j] = (R(1) - alpha) * as - alpha * an + tau * jv;
  }
  __syncthreads();

  // Phase B: modal right-hand side and the RK stage update
  const R c2 = a.c2;
  const int jx = kz * n1 + ky, jy = kz * n1 + kx, jz = ky * n1 + kx;
#pragma unroll
  for (int l = 0; l < EPB; ++l) {
    if (l >= ne) break;
    const R* s = sig + l * 12 * n2;
    R ub = (R)ru[l], vb = (R)rv[l];
    if constexpr (MIX) {
      ub = STAGE == 1 ? yu[l] : yu[l] + (R)ru[l];
      vb = STAGE == 1 ? yv[l] : yv[l] + (R)rv[l];
    }
    const R Lu = gEk * s[0 * n2 + jx] + gWk * s[2 * n2 + jx] + gNk * s[4 * n2 + jy] +
                 gSk * s[6 * n2 + jy] + gTk * s[8 * n2 + jz] + gBk * s[10 * n2 + jz];
    const R Lv = hEk * s[1 * n2 + jx] + hWk * s[3 * n2 + jx] + hNk * s[5 * n2 + jy] +
                 hSk * s[7 * n2 + jy] + hTk * s[9 * n2 + jz] + hBk * s[11 * n2 + jz];
    const R ku = vb + il * Lu;
    const R kv = c2 * (Lv - lm * ub);
    const long g = (e0 + l) * n3 + tid;
    R su, sv;
    rk_stage_store<T, STAGE>(a, g, ru[l], rv[l], xu[l], xv[l], yu[l], yv[l], ub, vb, ku, kv, su,
                             sv);
    snew[(l * 2) * n3 + tid] = su;
    snew[(l * 2 + 1) * n3 + tid] = sv;
  }
  __syncthreads();

  // Phase C: modal face traces of the new state for the next stage
  for (int i = tid; i < ne * 12 * n2; i += blockDim.x) {
    const int el = i / (12 * n2);
    const int r = i - el * 12 * n2;
    const int f2 = r / n2, j = r - f2 * n2;
    const R* F = snew + (el * 2 + (f2 & 1)) * n3;
    const R* gg = sgh + f2 * n1;
    R acc = 0;
    if (f2 < 4) {                 // x faces: j = kz n1 + ky, contract kx
      for (int k = 0; k < n1; ++k) acc += gg[k] * F[j * n1 + k];
    } else if (f2 < 8) {          // y faces: j = kz n1 + kx, contract ky
      const int jz_ = j / n1, jx_ = j - jz_ * n1;
      for (int k = 0; k < n1; ++k) acc += gg[k] * F[(jz_ * n1 + k) * n1 + jx_];
    } else {                      // z faces: j = ky n1 + kx, contract kz
      for (int k = 0; k < n1; ++k) acc += gg[k] * F[k * n2 + j];
    }
    a.tr_out[e0 * 12 * n2 + i] = (T)acc;
  }
}

template <typename T, int STAGE, int N1C, int EPB>
__global__ __launch_bounds__(1024) void k_stage3(StageArgs<T> a) {
  stage_tile3<T, STAGE, N1C, EPB>(a, blockIdx.x);
}

// nodal -> modal on box elements: three 1D contractions through LDS (one workgroup per
// element, any block size)
template <typename T>
__global__ void k_to_modal3(const double* __restrict__ U, T* __restrict__ Ub,
                            const double* __restrict__ Px, const double* __restrict__ Py,
                            const double* __restrict__ Pz, int n1, long nel) {
  extern __shared__ double sh[];
  const int n2 = n1 * n1, n3 = n2 * n1;
  double* u = sh;
  double* t1 = sh + n3;
  const long e = blockIdx.x;
  if (e >= nel) return;
  for (int i = threadIdx.x; i < n3; i += blockDim.x) u[i] = U[e * n3 + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n3; i += blockDim.x) {      // (iz, iy, kx)
    const int zy = i / n1, kx = i - zy * n1;
    double s = 0.0;
    for (int ix = 0; ix < n1; ++ix) s += Px[kx * n1 + ix] * u[zy * n1 + ix];
    t1[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n3; i += blockDim.x) {      // (iz, ky, kx)
    const int iz = i / n2, ky = (i / n1) % n1, kx = i % n1;
    double s = 0.0;
    for (int iy = 0; iy < n1; ++iy) s += Py[ky * n1 + iy] * t1[(iz * n1 + iy) * n1 + kx];
    u[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n3; i += blockDim.x) {      // (kz, ky, kx)
    const int kz = i / n2, yx = i - kz * n2;
    double s = 0.0;
    for (int iz = 0; iz < n1; ++iz) s += Pz[kz * n1 + iz] * u[iz * n2 + yx];
    Ub[e * n3 + i] = (T)s;
  }
}

// modal -> nodal: U = (Psi_z (x) Psi_y (x) Psi_x) Ubar
template <typename T>
__global__ void k_to_nodal3(const T* __restrict__ Ub, double* __restrict__ U,
                            const double* __restrict__ Psx, const double* __restrict__ Psy,
                            const double* __restrict__ Psz, int n1, long nel) {
  extern __shared__ double sh[];
  const int n2 = n1 * n1, n3 = n2 * n1;
  double* u = sh;
  double* t1 = sh + n3;
  const long e = blockIdx.x;
  if (e >= nel) return;
  for (int i = threadIdx.x; i < n3; i += blockDim.x) u[i] = (double)Ub[e * n3 + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n3; i += blockDim.x) {      // (kz, ky, ix)
    const int zy = i / n1, ix = i - zy * n1;
    double s = 0.0;
    for (int kx = 0; kx < n1; ++kx) s += Psx[ix * n1 + kx] * u[zy * n1 + kx];
    t1[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n3; i += blockDim.x) {      // (kz, iy, ix)
    const int kz = i / n2, iy = (i / n1) % n1, ix = i % n1;
    double s = 0.0;
    for (int ky = 0; ky < n1; ++ky) s += Psy[iy * n1 + ky] * t1[(kz * n1 + ky) * n1 + ix];
    u[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n3; i += blockDim.x) {      // (iz, iy, ix)
    const int iz = i / n2, yx = i - iz * n2;
    double s = 0.0;
    for (int kz = 0; kz < n1; ++kz) s += Psz[iz * n1 + kz] * u[kz * n2 + yx];
    U[e * n3 + i] = s;
  }
}

// modal face traces of a 3D state (set_state; the stage kernels write their own)
template <typename S, typename T>
__global__ void k_traces3(const S* __restrict__ Ub, const S* __restrict__ Vb,
                          const double* __restrict__ gh, T* __restrict__ tr, int n1, long nel) {
  const int n2 = n1 * n1, n3 = n2 * n1;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nel * 12 * n2) return;
  const long e = i / (12 * n2);
  const int r = (int)(i - e * 12 * n2);
  const int f2 = r / n2, j = r - f2 * n2;
  const S* F = ((f2 & 1) ? Vb : Ub) + e * n3;
  const double* g = gh + f2 * n1;
  double acc = 0;
  if (f2 < 4) {
    for (int k = 0; k < n1; ++k) acc += g[k] * (double)F[j * n1 + k];
  } else if (f2 < 8) {
    const int jz = j / n1, jx = j - jz * n1;
    for (int k = 0; k < n1; ++k) acc += g[k] * (double)F[(jz * n1 + k) * n1 + jx];
  } else {
    for (int k = 0; k < n1; ++k) acc += g[k] * (double)F[k * n2 + j];
  }
  tr[i] = (T)acc;
}

template <typename T>
hipError_t launch_to_modal3(const double* U, T* Ub, const double* Px, const double* Py,
                            const double* Pz, int n1, long nel, hipStream_t st) {
  if (nel == 0) return hipSuccess;
  const size_t sh = 2 * (size_t)n1 * n1 * n1 * sizeof(double);
  hipLaunchKernelGGL(k_to_modal3<T>, dim3((unsigned)nel), dim3(256), sh, st, U, Ub, Px, Py, Pz,
                     n1, nel);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_to_nodal3(const T* Ub, double* U, const double* Psx, const double* Psy,
                            const double* Psz, int n1, long nel, hipStream_t st) {
  if (nel == 0) return hipSuccess;
  const size_t sh = 2 * (size_t)n1 * n1 * n1 * sizeof(double);
  hipLaunchKernelGGL(k_to_nodal3<T>, dim3((unsigned)nel), dim3(256), sh, st, Ub, U, Psx, Psy, Psz,
                     n1, nel);
  return hipGetLastError();
}

template <typename S, typename T>
hipError_t launch_traces3(const S* Ub, const S* Vb, const double* gh, T* tr, int n1, long nel,
                          hipStream_t st) {
  const long total = nel * 12 * n1 * n1;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL((k_traces3<S, T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     Ub, Vb, gh, tr, n1, nel);
  return hipGetLastError();
}

template <typename T, int STAGE, int N1C, int EPB>
static hipError_t launch_stage3_t(const StageArgs<T>& a, hipStream_t st) {
  const int n1 = a.n1;
  const size_t sh = stage3_lds_doubles(n1, EPB) * sizeof(double);
  const unsigned nblk = (unsigned)((a.nel + EPB - 1) / EPB);
  hipLaunchKernelGGL((k_stage3<T, STAGE, N1C, EPB>), dim3(nblk), dim3(n1 * n1 * n1), sh, st, a);
  return hipGetLastError();
}

// Elements per workgroup: 2 where the tile fits 64 KiB of LDS, else 1.
template <typename T, int STAGE, int N1C>
static hipError_t dispatch3_epb(const StageArgs<T>& a, hipStream_t st) {
  if (a.n1 * a.n1 * a.n1 > 1024) return hipErrorInvalidValue;
  if (stage3_lds_doubles(a.n1, 2) * sizeof(double) <= 65536)
    return launch_stage3_t<T, STAGE, N1C, 2>(a, st);
  return launch_stage3_t<T, STAGE, N1C, 1>(a, st);
}

template <typename T, int STAGE>
static hipError_t dispatch3_n1(const StageArgs<T>& a, hipStream_t st) {
  switch (a.n1) {
    case 9: return dispatch3_epb<T, STAGE, 9>(a, st);
    case 10: return dispatch3_epb<T, STAGE, 10>(a, st);
    default: return dispatch3_epb<T, STAGE, 0>(a, st);
  }
}

template <typename T>
hipError_t launch_stage3(int stage, const StageArgs<T>& a, hipStream_t st) {
  if (a.nel == 0) return hipSuccess;
  switch (stage) {
    case 1: return dispatch3_n1<T, 1>(a, st);
    case 2: return dispatch3_n1<T, 2>(a, st);
    case 3: return dispatch3_n1<T, 3>(a, st);
    default: return dispatch3_n1<T, 4>(a, st);
  }
}

#define GDW_INST(T)                                                                              \
  template hipError_t launch_to_modal<T>(const double*, T*, const double*, const double*, int,    \
                                         long, hipStream_t);                                     \
  template hipError_t launch_to_nodal<T>(const T*, double*, const double*, const double*, int,    \
                                         long, hipStream_t);                                     \
  template hipError_t launch_stage<T>(int, const StageArgs<T>&, hipStream_t);                    \
  template hipError_t launch_energy<T>(const T*, const T*, const double*, double, int, long,       \
                                       double*,                                                  \
                                       int, double*, hipStream_t);                               \
  template hipError_t launch_count_nonfinite<T>(const T*, long, unsigned int*, hipStream_t);       \
  template hipError_t launch_stage_group<T>(int, int, int, const StageArgs<T>*, const long*, int, \
                                            unsigned, hipStream_t);                              \
  template int stage_group_occupancy<T>(int, int, int);                                          \
  template hipError_t launch_to_modal3<T>(const double*, T*, const double*, const double*,        \
                                          const double*, int, long, hipStream_t);                 \
  template hipError_t launch_to_nodal3<T>(const T*, double*, const double*, const double*,        \
                                          const double*, int, long, hipStream_t);                 \
  template hipError_t launch_stage3<T>(int, const StageArgs<T>&, hipStream_t);

GDW_INST(double)
GDW_INST(float)
template hipError_t launch_traces<double, double>(const double*, const double*, const double*,
                                                  double*, int, long, hipStream_t);
template hipError_t launch_traces<double, float>(const double*, const double*, const double*,
                                                 float*, int, long, hipStream_t);
template hipError_t launch_traces3<double, double>(const double*, const double*, const double*,
                                                   double*, int, long, hipStream_t);
template hipError_t launch_traces3<double, float>(const double*, const double*, const double*,
                                                  float*, int, long, hipStream_t);

}  // namespace gdw
