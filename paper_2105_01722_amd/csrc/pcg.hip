// Variable-coefficient and mapped-element path (Sec. 7, Sec. 7.1).
//
// Elements are images of the reference square under an isoparametric GD map
// (X, Y)(r, s); c^2 is a GD function too.  With A = d(X,Y)/d(r,s), J = det A and
// K = c^2 J A^{-1} A^{-T}, the element matrices of DG1 / DG2 are
//   M_J = int phi phi J,  S_K = int grad_r phi^T K grad_r phi,  w = int phi J,
// integrated with (p+1)^2 Gauss points per cell, and the face terms use (p+1) Gauss
// points per face cell with c^2 (n . grad phi) dS = Nh^T K grad_r phi ds and
// dS = s_J ds.  The extra equation DG1_extra enters as S_hat = S_K + (kappa/|Omega|) w w^T.
//
// Every RK stage is one kernel, one workgroup per element:
//   face fluxes from the (a, v) traces at the face points of the element and its
//   neighbours -> lifts F_u, F_v -> r = -S_K U + F_v -> PCG for S_hat y = F_u and
//   M_J z = r (tensor-product preconditioner from element averages, warm start from
//   the previous stage) -> dU/dt = V + y, dV/dt = z -> RK stage update -> traces
//   of the new value for the next stage.
// The element operator of the running solve sits in LDS (upper half, stencil.h);
// on Cartesian meshes M_J = |Omega| M_ref (x) M_ref is inverted exactly by the
// preconditioner itself and is not stored.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <type_traits>
#include <vector>

#include "pcg.h"
#include "stencil.h"

namespace gdw {

// ---------------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------------
// Wave-wide sum through DPP lane moves (no LDS traffic); every lane returns the sum.
template <int CTRL, int ROW_MASK, bool BC>
__device__ inline double dpp_mov(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, BC);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, BC);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double wave_sum(double v) {
  v += dpp_mov<0xb1, 0xf, false>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov<0x4e, 0xf, false>(v);    // quad_perm [2,3,0,1]: quad sums
  v += dpp_mov<0x141, 0xf, false>(v);   // row_half_mirror: 8-lane sums
  v += dpp_mov<0x140, 0xf, false>(v);   // row_mirror: 16-lane row sums
  v += dpp_mov<0x142, 0xa, false>(v);   // row_bcast:15 into rows 1, 3
  v += dpp_mov<0x143, 0xc, false>(v);   // row_bcast:31 into rows 2, 3: lane 63 = total
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Deterministic workgroup sum of K values held by the threads t < nact (the other
// threads pass zeros and may be anywhere in the workgroup); fixed wave order.
// red: 16*K doubles.  Every thread returns the sums.  TRAIL = false leaves out the closing
// barrier: the caller then passes another barrier before red is written again.
template <int K, bool TRAIL = true>
__device__ inline void block_sum(double (&v)[K], double* red, int nact) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = (nact + 63) >> 6;
  if (w < nw) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double s = wave_sum(v[k]);
      if (lane == 0) red[k * 16 + w] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[k * 16 + i];
    v[k] = s;
  }
  if constexpr (TRAIL) __syncthreads();
}

// Deterministic workgroup sum of two values over all threads (fixed wave order).
__device__ inline void block_sum2(double& a, double& b, double* red) {
  double v[2] = {a, b};
  block_sum<2>(v, red, blockDim.x);
  a = v[0];
  b = v[1];
}

// Row i = (ix, iy) of a symmetric element operator stored as its upper half.
template <typename TA, typename TX, typename TACC>
__device__ inline TACC sym_row(const TA* A, const int* rowoff, const TX* x, int ix, int iy, int p,
                               int N, int n1) {
  const int xl = st_lo(ix, p), xh = st_hi(ix, p, N), yh = st_hi(iy, p, N);
  TACC acc = 0;
  const TA* r = A + rowoff[iy * n1 + ix];
  int k = 0;
  for (int jx = ix; jx <= xh; ++jx) acc += (TACC)r[k++] * (TACC)x[iy * n1 + jx];
  for (int jy = iy + 1; jy <= yh; ++jy)
    for (int jx = xl; jx <= xh; ++jx) acc += (TACC)r[k++] * (TACC)x[jy * n1 + jx];
  for (int jx = xl; jx < ix; ++jx)
    acc += (TACC)A[rowoff[iy * n1 + jx] + (ix - jx)] * (TACC)x[iy * n1 + jx];
  for (int jy = st_lo(iy, p); jy < iy; ++jy)
    for (int jx = xl; jx <= xh; ++jx)
      acc += (TACC)A[rowoff[jy * n1 + jx] + st_pos(jx, jy, ix, iy, p, N)] * (TACC)x[jy * n1 + jx];
  return acc;
}

// Z = Psi diag(dinv) Psi^T R on the (N+1)^2 grid (thread t owns index t); tmp is scratch.
template <typename T>
__device__ inline void pinv_apply(const T* R, T* tmp, T* Z, const T* Psi, T dinv, int n1, int nn) {
  const int t = threadIdx.x;
  const int a = t / n1, b = t - (t / n1) * n1;    // t = a*n1 + b
  if (t < nn) {                                   // tmp[ky][ix] = sum_iy Psi[iy][ky] R[iy][ix]
    T s = 0;
    for (int iy = 0; iy < n1; ++iy) s += Psi[iy * n1 + a] * R[iy * n1 + b];
    tmp[t] = s;
  }
  __syncthreads();
  if (t < nn) {                                   // Z[ky][kx] = dinv sum_ix tmp[ky][ix] Psi[ix][kx]
    T s = 0;
    for (int ix = 0; ix < n1; ++ix) s += tmp[a * n1 + ix] * Psi[ix * n1 + b];
    Z[t] = s * dinv;
  }
  __syncthreads();
  if (t < nn) {                                   // tmp[iy][kx] = sum_ky Psi[iy][ky] Z[ky][kx]
    T s = 0;
    for (int ky = 0; ky < n1; ++ky) s += Psi[a * n1 + ky] * Z[ky * n1 + b];
    tmp[t] = s;
  }
  __syncthreads();
  if (t < nn) {                                   // Z[iy][ix] = sum_kx tmp[iy][kx] Psi[ix][kx]
    T s = 0;
    for (int kx = 0; kx < n1; ++kx) s += tmp[a * n1 + kx] * Psi[b * n1 + kx];
    Z[t] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------
// Assembly of S_K, M_J (upper halves), w and the element averages.  One workgroup
// per element, cells in sequence; each stored entry is updated by one thread per
// cell, and the cells are separated by barriers.
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_assemble(PcgGeom g, const double* __restrict__ X,
                                                  const double* __restrict__ Y,
                                                  const double* __restrict__ C2, PcgElem el,
                                                  long nel) {
  const long e = blockIdx.x;
  if (e >= nel) return;
  const int t = threadIdx.x, N = g.N, p = g.p, n1 = g.n1, nn = g.nn, m = g.m, mm = m * m;
  __shared__ double qJ[64], qrr[64], qss[64], qrs[64];
  __shared__ double Bx[64], Dx[64], By[64], Dy[64];
  __shared__ double red[32];
  double* S = el.S + e * g.nst;
  double* M = el.M ? el.M + e * g.nst : nullptr;
  double* w = el.w + e * nn;
  for (int i = t; i < g.nst; i += blockDim.x) {
    S[i] = 0.0;
    if (M) M[i] = 0.0;
  }
  for (int i = t; i < nn; i += blockDim.x) w[i] = 0.0;
  const double* Xe = X + e * nn;
  const double* Ye = Y + e * nn;
  const double* Ce = C2 + e * nn;
  double iKrr = 0, iKss = 0, icJ = 0, iA = 0;
  __syncthreads();
  for (int kx = 0; kx < N; ++kx) {
    for (int ky = 0; ky < N; ++ky) {
      const int sx = g.cs[kx], sy = g.cs[ky];
      if (t < mm) {
        Bx[t] = g.cb[kx * mm + t];
        Dx[t] = g.cd[kx * mm + t];
        By[t] = g.cb[ky * mm + t];
        Dy[t] = g.cd[ky * mm + t];
      }
      __syncthreads();
      if (t < mm) {      // geometry at Gauss point (qa, qb) of the cell
        const int qa = t % m, qb = t / m;
        double xr = 0, xs = 0, yr = 0, ys = 0, cq = 0;
        for (int jy = 0; jy < m; ++jy)
          for (int jx = 0; jx < m; ++jx) {
            const int nd = (sy + jy) * n1 + sx + jx;
            const double br = Dx[qa * m + jx] * By[qb * m + jy];
            const double bs = Bx[qa * m + jx] * Dy[qb * m + jy];
            const double bv = Bx[qa * m + jx] * By[qb * m + jy];
            xr += br * Xe[nd];
            xs += bs * Xe[nd];
            yr += br * Ye[nd];
            ys += bs * Ye[nd];
            cq += bv * Ce[nd];
          }
        const double J = xr * ys - xs * yr;
        const double wq = g.gw[qa] * g.gw[qb] / ((double)N * N);
        const double krr = cq * (xs * xs + ys * ys) / J;
        const double kss = cq * (xr * xr + yr * yr) / J;
        const double krs = -cq * (xr * xs + yr * ys) / J;
        qJ[t] = wq * J;
        qrr[t] = wq * krr;
        qss[t] = wq * kss;
        qrs[t] = wq * krs;
        iKrr += wq * krr;
        iKss += wq * kss;
        icJ += wq * cq * J;
        iA += wq * J;
      }
      __syncthreads();
      // local pairs (a, b) of the cell's (p+1)^2 functions, upper half only
      for (int pr = t; pr < mm * mm; pr += blockDim.x) {
        const int a = pr / mm, b = pr - (pr / mm) * mm;
        const int ax = a % m, ay = a / m, bx = b % m, by = b / m;
        const int ix = sx + ax, iy = sy + ay, jx = sx + bx, jy = sy + by;
        const int i = iy * n1 + ix, j = jy * n1 + jx;
        if (i > j) continue;
        double ss = 0, ms = 0;
        for (int qb = 0; qb < m; ++qb)
          for (int qa = 0; qa < m; ++qa) {
            const int q = qb * m + qa;
            const double pa = Bx[qa * m + ax] * By[qb * m + ay];
            const double pb = Bx[qa * m + bx] * By[qb * m + by];
            const double ra = Dx[qa * m + ax] * By[qb * m + ay];
            const double rb = Dx[qa * m + bx] * By[qb * m + by];
            const double sa = Bx[qa * m + ax] * Dy[qb * m + ay];
            const double sb = Bx[qa * m + bx] * Dy[qb * m + by];
            ms += qJ[q] * pa * pb;
            ss += qrr[q] * ra * rb + qss[q] * sa * sb + qrs[q] * (ra * sb + sa * rb);
          }
        const int pos = g.rowoff[i] + st_pos(ix, iy, jx, jy, p, N);
        S[pos] += ss;
        if (M) M[pos] += ms;
      }
      if (t < mm) {
        const int ax = t % m, ay = t / m;
        double ws = 0;
        for (int qb = 0; qb < m; ++qb)
          for (int qa = 0; qa < m; ++qa)
            ws += qJ[qb * m + qa] * Bx[qa * m + ax] * By[qb * m + ay];
        w[(sy + ay) * n1 + sx + ax] += ws;
      }
      __syncthreads();
    }
  }
  block_sum2(iKrr, iKss, red);
  block_sum2(icJ, iA, red);
  if (t == 0) {
    double* sc = el.sc + e * 8;
    const double kappa = icJ / iA;
    sc[0] = kappa / iA;
    sc[1] = iKrr;
    sc[2] = iKss;
    sc[3] = kappa * iA;
    sc[4] = iA;
    sc[5] = icJ;
    sc[6] = 0.0;
    sc[7] = 0.0;
  }
}

// Geometry at the face points: (K Nh)_r, (K Nh)_s and c^2 s_J.  Faces E (r = 1), W (r = 0),
// N (s = 1), S (s = 0); point q = k*m + a is Gauss point a of face cell k.
__global__ void k_face_geom(PcgGeom g, const double* __restrict__ X, const double* __restrict__ Y,
                            const double* __restrict__ C2, PcgElem el, long nel) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nel * 4 * g.nq) return;
  const long e = id / (4 * g.nq);
  const int r = (int)(id - e * 4 * g.nq);
  const int f = r / g.nq, q = r - f * g.nq;
  const int k = q / g.m, a = q - k * g.m, m = g.m, n1 = g.n1, N = g.N;
  const int s0 = g.cs[k];
  const double* cb = g.cb + (k * m + a) * m;
  const double* cd = g.cd + (k * m + a) * m;
  const double* dn = (f == 0 || f == 2) ? g.dR : g.dL;
  const int node = (f == 0 || f == 2) ? N : 0;
  const double* Xe = X + e * g.nn;
  const double* Ye = Y + e * g.nn;
  const double* Ce = C2 + e * g.nn;
  double xn = 0, yn = 0, xt = 0, yt = 0, cq = 0;   // normal / tangential derivatives
  for (int j = 0; j < m; ++j) {
    const int l = s0 + j;   // node index along the face
    double gx = 0, gy = 0;
    for (int i = 0; i < n1; ++i) {
      const int nd = (f < 2) ? l * n1 + i : i * n1 + l;
      gx += dn[i] * Xe[nd];
      gy += dn[i] * Ye[nd];
    }
    const int fnd = (f < 2) ? l * n1 + node : node * n1 + l;
    xn += cb[j] * gx;
    yn += cb[j] * gy;
    xt += cd[j] * Xe[fnd];
    yt += cd[j] * Ye[fnd];
    cq += cb[j] * Ce[fnd];
  }
  double xr, xs, yr, ys, nr, ns;
  if (f < 2) {              // E / W: normal coordinate r, tangent s
    xr = xn; yr = yn; xs = xt; ys = yt;
    nr = f == 0 ? 1.0 : -1.0; ns = 0.0;
  } else {                  // N / S: normal coordinate s, tangent r
    xs = xn; ys = yn; xr = xt; yr = yt;
    nr = 0.0; ns = f == 2 ? 1.0 : -1.0;
  }
  const double J = xr * ys - xs * yr;
  const double krr = cq * (xs * xs + ys * ys) / J;
  const double kss = cq * (xr * xr + yr * yr) / J;
  const double krs = -cq * (xr * xs + yr * ys) / J;
  double* out = el.face + id * 3;
  out[0] = krr * nr + krs * ns;
  out[1] = krs * nr + kss * ns;
  out[2] = cq * sqrt(xt * xt + yt * yt);
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// Upper-half FP64 operators [nel][nst] -> FP32 block layout hi = fl32(a), lo = fl32(a - hi),
// both positions (i, j) and (j, i) of entry h (dst[2h], dst[2h+1]).
__global__ void k_split_hilo(const double* __restrict__ half, const int* __restrict__ dst, int nst,
                             int nnz, long nel, float* __restrict__ hi, float* __restrict__ lo) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nel * nst) return;
  const long e = id / nst;
  const int h = (int)(id - e * nst);
  const double v = half[id];
  const float vh = (float)v;
  const float vl = (float)(v - (double)vh);
  const int2 d2 = reinterpret_cast<const int2*>(dst)[h];
  hi[e * nnz + d2.x] = vh;
  hi[e * nnz + d2.y] = vh;
  lo[e * nnz + d2.x] = vl;
  lo[e * nnz + d2.y] = vl;
}

// ---------------------------------------------------------------------------------
// (a, v) traces at the face points of a nodal state held in LDS (U, V), written to
// tr[4][nq][2].  G: 4*n1 doubles of scratch.
// ---------------------------------------------------------------------------------
__device__ void face_traces(const PcgGeom& g, const double* fc, const double* U, const double* V,
                            double* G, double* tr) {
  const int t = threadIdx.x, n1 = g.n1, N = g.N, m = g.m, nq = g.nq;
  if (t < 4 * n1) {       // normal-derivative line of each face
    const int f = t / n1, l = t - (t / n1) * n1;
    const double* dn = (f == 0 || f == 2) ? g.dR : g.dL;
    double s = 0;
    if (f < 2)
      for (int i = 0; i < n1; ++i) s += dn[i] * U[l * n1 + i];
    else
      for (int i = 0; i < n1; ++i) s += dn[i] * U[i * n1 + l];
    G[t] = s;
  }
  __syncthreads();
  for (int id = t; id < 4 * nq; id += blockDim.x) {
    const int f = id / nq, q = id - (id / nq) * nq;
    const int k = q / m, a = q - (q / m) * m, s0 = g.cs[k];
    const double* cb = g.cb + (k * m + a) * m;
    const double* cd = g.cd + (k * m + a) * m;
    const int node = (f == 0 || f == 2) ? N : 0;
    double un = 0, ut = 0, vv = 0;
    for (int j = 0; j < m; ++j) {
      const int l = s0 + j;
      const int fnd = (f < 2) ? l * n1 + node : node * n1 + l;
      un += cb[j] * G[f * n1 + l];
      ut += cd[j] * U[fnd];
      vv += cb[j] * V[fnd];
    }
    const double* F = fc + id * 3;
    const double ur = f < 2 ? un : ut, us = f < 2 ? ut : un;
    tr[id * 2] = (F[0] * ur + F[1] * us) / F[2];
    tr[id * 2 + 1] = vv;
  }
}

__global__ __launch_bounds__(1024) void k_pcg_traces(PcgGeom g, PcgElem el,
                                                     const double* __restrict__ U,
                                                     const double* __restrict__ V,
                                                     double* __restrict__ tr, long nel) {
  extern __shared__ double shd[];
  const long e = blockIdx.x;
  const int nn = g.nn;
  double* u = shd;
  double* v = u + nn;
  double* G = v + nn;
  for (int i = threadIdx.x; i < nn; i += blockDim.x) {
    u[i] = U[e * nn + i];
    v[i] = V[e * nn + i];
  }
  __syncthreads();
  face_traces(g, el.face + e * 4 * g.nq * 3, u, v, G, tr + e * 4 * g.nq * 2);
}

// ---------------------------------------------------------------------------------
// Element operator in LDS.  FULL: every coupled entry of a row stored as the
// rectangle jy in [lo(iy), hi(iy)] x jx in [lo(ix), hi(ix)] (row start fo[r]); a row
// is split over Q threads (thread part q takes jy = lo(iy) + q, + Q, ...) and the Q
// partial sums are added in a fixed order.  HALF: the upper half as stored in HBM
// (stencil.h), one thread per row; used when the full rectangle does not fit.
// ---------------------------------------------------------------------------------
struct PcgShared {
  double* A;        // operator (FULL or HALF layout)
  double* part;     // [Q][nn] partial row sums (FULL)
  double *x, *r, *z, *d, *q, *tmp, *b;
  double* Psi;
  double* red;
  const int* fo;    // FULL row starts [nn+1]
  const int* ho;    // HALF row starts [nn+1]
  int Q;
  int full;
};

// (A x)_t for t < nn (other threads return 0).  Contains barriers; x must be complete.
__device__ inline double op_apply(const PcgGeom& g, const PcgShared& W, const double* x) {
  const int t = threadIdx.x, nn = g.nn, n1 = g.n1, p = g.p, N = g.N;
  if (W.full) {
    if (t < W.Q * nn) {
      const int r = t % nn, qp = t / nn;
      const int ix = r % n1, iy = r / n1;
      const int xl = st_lo(ix, p), w = st_w(ix, p, N), yl = st_lo(iy, p), yh = st_hi(iy, p, N);
      double acc = 0.0;
      for (int jy = yl + qp; jy <= yh; jy += W.Q) {
        const double* a = W.A + W.fo[r] + (jy - yl) * w;
        const double* xx = x + jy * n1 + xl;
        for (int k = 0; k < w; ++k) acc += a[k] * xx[k];
      }
      W.part[qp * nn + r] = acc;
    }
    __syncthreads();
    double y = 0.0;
    if (t < nn)
      for (int qp = 0; qp < W.Q; ++qp) y += W.part[qp * nn + t];
    return y;
  }
  return t < nn ? sym_row<double, double, double>(W.A, W.ho, x, t % n1, t / n1, p, N, n1) : 0.0;
}

// Copy one element operator from its HBM upper half into LDS.  In FULL mode entry h of
// the upper half, (i, j), goes to both (i, j) and (j, i) of the full rectangles; the
// two destinations come from the precomputed table dst[2h], dst[2h+1], so that the HBM
// reads are a plain coalesced sweep.
__device__ inline void op_load(const PcgGeom& g, const PcgShared& W, const double* __restrict__ half,
                               const int* __restrict__ dst) {
  const int t = threadIdx.x;
  if (!W.full) {
    for (int i = t; i < g.nst; i += blockDim.x) W.A[i] = half[i];
    return;
  }
  for (int h = t; h < g.nst; h += blockDim.x) {
    const double v = half[h];
    const int2 d2 = reinterpret_cast<const int2*>(dst)[h];
    W.A[d2.x] = v;
    W.A[d2.y] = v;
  }
}

// PCG on one element system; thread t owns index t.  Rank-1 term cw * w (w^T x) when
// cw != 0 (S_hat).  Two workgroup reductions per iteration: d.q, then
// (r.r, r.z, w.z) after the preconditioner (z is formed before the convergence test).
// Returns the iteration count (maxit + 1 if it did not converge).
// sc: this owner's nodal scale of the preconditioner (P^-1 r -> sc P^-1 (sc r); 1 for S_hat).
__device__ int pcg_solve(const PcgGeom& g, const PcgShared& W, double cw, double wt, double dinv,
                         double rtol, int maxit, double sc = 1.0) {
  const int t = threadIdx.x, nn = g.nn, n1 = g.n1;
  const bool own = t < nn;
  double s2[2] = {own ? wt * W.x[t] : 0.0, own ? W.b[t] * W.b[t] : 0.0};
  block_sum<2>(s2, W.red, nn);
  const double wx = s2[0], bb = s2[1];
  if (bb == 0.0) {
    if (own) W.x[t] = 0.0;
    __syncthreads();
    return 0;
  }
  {
    const double ax = op_apply(g, W, W.x) + cw * wt * wx;
    if (own) {
      W.r[t] = W.b[t] - ax;
      W.q[t] = W.r[t] * sc;
    }
  }
  __syncthreads();
  pinv_apply<double>(W.q, W.tmp, W.z, W.Psi, dinv, n1, nn);
  if (own) W.z[t] *= sc;
  double s3[3] = {own ? W.r[t] * W.r[t] : 0.0, own ? W.r[t] * W.z[t] : 0.0,
                  own ? wt * W.z[t] : 0.0};
  block_sum<3>(s3, W.red, nn);
  const double tol2 = rtol * rtol * bb;
  if (s3[0] <= tol2) return 0;
  double rz = s3[1], wd = s3[2];
  if (own) W.d[t] = W.z[t];
  __syncthreads();
  for (int it = 1; it <= maxit; ++it) {
    const double qv = op_apply(g, W, W.d) + cw * wt * wd;
    double s1[1] = {own ? W.d[t] * qv : 0.0};
    block_sum<1>(s1, W.red, nn);
    const double alpha = rz / s1[0];
    if (own) {
      W.x[t] += alpha * W.d[t];
      W.r[t] -= alpha * qv;
      W.q[t] = W.r[t] * sc;
    }
    __syncthreads();
    pinv_apply<double>(W.q, W.tmp, W.z, W.Psi, dinv, n1, nn);
    if (own) W.z[t] *= sc;
    double s3b[3] = {own ? W.r[t] * W.r[t] : 0.0, own ? W.r[t] * W.z[t] : 0.0,
                     own ? wt * W.z[t] : 0.0};
    block_sum<3>(s3b, W.red, nn);
    if (s3b[0] <= tol2) return it;
    const double bet = s3b[1] / rz;
    rz = s3b[1];
    wd = s3b[2] + bet * wd;
    if (own) W.d[t] = W.z[t] + bet * W.d[t];
    __syncthreads();
  }
  return maxit + 1;
}

// ---------------------------------------------------------------------------------
// The fused RK stage of the variable-coefficient path (FP64).
// ---------------------------------------------------------------------------------
// size of the full-rectangle operator, rows padded to odd lengths (as the host's fo)
static int full_nnz(const PcgGeom& g) {
  int tot = 0;
  for (int r = 0; r < g.nn; ++r) {
    const int len = st_w(r % g.n1, g.p, g.N) * st_w(r / g.n1, g.p, g.N);
    tot += len + (len % 2 == 0 ? 1 : 0);
  }
  return tot;
}

static int full_parts(const PcgGeom& g) {
  int q = 1024 / g.nn;
  if (q > 2 * g.p + 1) q = 2 * g.p + 1;
  return q < 1 ? 1 : q;
}

// doubles / ints of the LDS part common to both operator layouts (Psi excluded)
__host__ __device__ inline size_t common_doubles(const PcgGeom& g) {
  return (size_t)4 * g.nn + g.n1 + 2 * g.N * g.m * g.m + g.m + 2 * g.n1 + 4 * g.nq * 3 +
         4 * g.nq * 2 + 16 * g.n1 + 64;
}
__host__ __device__ inline size_t common_ints(const PcgGeom& g) { return (size_t)g.N + 2 * g.n1; }

static size_t stage_lds(const PcgGeom& g, int full) {
  const size_t nd = (size_t)(full ? full_nnz(g) + full_parts(g) * g.nn : g.nst)  // A, part
                    + 8 * g.nn + common_doubles(g);        // x r z d q tmp b Psi + common
  const size_t ni = 2 * (g.nn + 1) + common_ints(g);      // fo ho + common
  return nd * sizeof(double) + ni * sizeof(int);
}

size_t pcg_stage_lds_bytes(const PcgGeom& g, int mixed) {
  (void)mixed;
  const size_t f = stage_lds(g, 1);
  return f <= 160 * 1024 ? f : stage_lds(g, 0);
}

static int stage_full(const PcgGeom& g) { return stage_lds(g, 1) <= 160 * 1024 ? 1 : 0; }

// (a, v) traces at the face points of a nodal state in LDS (tables in LDS).
struct FaceTabs {
  const double *cb, *cd, *gw, *dL, *dR, *fc;
  const int *cs, *ck0, *ck1;
};

__device__ void face_traces_lds(const PcgGeom& g, const FaceTabs& T, const double* U,
                                const double* V, double* G, double* __restrict__ tr) {
  const int t = threadIdx.x, n1 = g.n1, N = g.N, m = g.m, nq = g.nq;
  if (t < 4 * n1) {
    const int f = t / n1, l = t - (t / n1) * n1;
    const double* dn = (f == 0 || f == 2) ? T.dR : T.dL;
    double s = 0;
    if (f < 2)
      for (int i = 0; i < n1; ++i) s += dn[i] * U[l * n1 + i];
    else
      for (int i = 0; i < n1; ++i) s += dn[i] * U[i * n1 + l];
    G[t] = s;
  }
  __syncthreads();
  for (int id = t; id < 4 * nq; id += blockDim.x) {
    const int f = id / nq, q = id - (id / nq) * nq;
    const int k = q / m, a = q - (q / m) * m, s0 = T.cs[k];
    const double* cb = T.cb + (k * m + a) * m;
    const double* cd = T.cd + (k * m + a) * m;
    const int node = (f == 0 || f == 2) ? N : 0;
    double un = 0, ut = 0, vv = 0;
    for (int j = 0; j < m; ++j) {
      const int l = s0 + j;
      const int fnd = (f < 2) ? l * n1 + node : node * n1 + l;
      un += cb[j] * G[f * n1 + l];
      ut += cd[j] * U[fnd];
      vv += cb[j] * V[fnd];
    }
    const double* F = T.fc + id * 3;
    const double ur = f < 2 ? un : ut, us = f < 2 ? ut : un;
    tr[id * 2] = (F[0] * ur + F[1] * us) / F[2];
    tr[id * 2 + 1] = vv;
  }
}

// ---------------------------------------------------------------------------------
// Parts of an RK stage that do not depend on the operator layout.
// ---------------------------------------------------------------------------------
struct StageCommon {
  double *U, *V, *Fu, *rv, *lamr, *lines, *red, *sig;
  double ms = 1.0;   // this owner's nodal scale of the M_J preconditioner
  bool gtab;                                 // cb, cd, face data read from global memory
  FaceTabs T;
  double ub, vb, yu, yv, xs0, xm0, wt;      // owner thread t < nn
  double cw, kbr, kbs, d00, area;
};


// Carve the common part from sp / ip (pointer arithmetic only).
__device__ __forceinline__ void stage_carve(const PcgGeom& g, double*& sp, int*& ip,
                                            StageCommon& C) {
  const int nn = g.nn, n1 = g.n1, N = g.N, m = g.m, nq = g.nq;
  C.U = sp;        sp += nn;
  C.V = sp;        sp += nn;
  C.Fu = sp;       sp += nn;
  C.rv = sp;       sp += nn;
  C.lamr = sp;     sp += n1;
  double* cb = sp; sp += N * m * m;
  double* cd = sp; sp += N * m * m;
  double* gw = sp; sp += m;
  double* dL = sp; sp += n1;
  double* dR = sp; sp += n1;
  double* fc = sp; sp += 4 * nq * 3;
  C.sig = sp;      sp += 4 * nq * 2;
  C.lines = sp;    sp += 16 * n1;
  C.red = sp;      sp += 64;
  int* cs = ip;    ip += N;
  int* ck0 = ip;   ip += n1;
  int* ck1 = ip;   ip += n1;
  C.T = FaceTabs{cb, cd, gw, dL, dR, fc, cs, ck0, ck1};
  C.gtab = false;
}

// Smaller common part: cb, cd and the face data stay in global memory (read through the
// caches) and sig lives in the caller's region `sigbuf` (4 nq * 2 doubles).
__device__ __forceinline__ void stage_carve_small(const PcgGeom& g, double*& sp, int*& ip,
                                                  double* sigbuf, StageCommon& C) {
  const int nn = g.nn, n1 = g.n1, N = g.N, m = g.m;
  C.U = sp;        sp += nn;
  C.V = sp;        sp += nn;
  C.Fu = sp;       sp += nn;
  C.rv = sp;       sp += nn;
  C.lamr = sp;     sp += n1;
  double* gw = sp; sp += m;
  double* dL = sp; sp += n1;
  double* dR = sp; sp += n1;
  C.lines = sp;    sp += 16 * n1;
  C.red = sp;      sp += 64;
  C.sig = sigbuf;
  int* cs = ip;    ip += N;
  int* ck0 = ip;   ip += n1;
  int* ck1 = ip;   ip += n1;
  C.T = FaceTabs{g.cb, g.cd, gw, dL, dR, nullptr, cs, ck0, ck1};
  C.gtab = true;
}

__host__ __device__ inline size_t common_small_doubles(const PcgGeom& g) {
  return (size_t)4 * g.nn + g.n1 + g.m + 2 * g.n1 + 16 * g.n1 + 64;
}

// Load the element-independent tables into the carved places (Psi with stride ps,
// padding rows / columns 0).  Visible to all threads after the next barrier.
__device__ __forceinline__ void stage_load_tables(const PcgGeom& g, double* Psi, int ps,
                                                  const StageCommon& C) {
  const int t = threadIdx.x, n1 = g.n1, N = g.N, m = g.m;
  double* cb = const_cast<double*>(C.T.cb);
  double* cd = const_cast<double*>(C.T.cd);
  double* gw = const_cast<double*>(C.T.gw);
  double* dL = const_cast<double*>(C.T.dL);
  double* dR = const_cast<double*>(C.T.dR);
  int* cs = const_cast<int*>(C.T.cs);
  int* ck0 = const_cast<int*>(C.T.ck0);
  int* ck1 = const_cast<int*>(C.T.ck1);
  for (int i = t; i < ps * ps; i += blockDim.x) {
    const int r = i / ps, k = i - (i / ps) * ps;
    Psi[i] = (r < n1 && k < n1) ? g.Psi[r * n1 + k] : 0.0;
  }
  if (!C.gtab)
    for (int i = t; i < N * m * m; i += blockDim.x) {
      cb[i] = g.cb[i];
      cd[i] = g.cd[i];
    }
  for (int i = t; i < n1; i += blockDim.x) {
    C.lamr[i] = g.lamr[i];
    dL[i] = g.dL[i];
    dR[i] = g.dR[i];
    ck0[i] = g.ck0[i];
    ck1[i] = g.ck1[i];
  }
  for (int i = t; i < m; i += blockDim.x) gw[i] = g.gw[i];
  for (int i = t; i < N; i += blockDim.x) cs[i] = g.cs[i];
}

// sum over aligned groups of 8 lanes (DPP); every lane of a group returns the sum
__device__ __forceinline__ double sum8(double v) {
  v += dpp_mov<0xb1, 0xf, false>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov<0x4e, 0xf, false>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov<0x141, 0xf, false>(v);   // row_half_mirror
  return v;
}

// Load the element's data and form the lifts: Fu = F_u, rv = F_v (the caller subtracts
// S_K U).  `after_first_barrier` runs once the element data are in LDS (operator load
// overlap).  Tables from stage_tables must be in place.  NODAL = false: only the lifts (the
// nodal state, warm starts and element scalars are not loaded).
template <int STAGE, bool NODAL = true, typename F>
__device__ __forceinline__ void stage_prologue(const PcgStageArgs& a, const long e,
                                               StageCommon& C, F&& after_first_barrier) {
  const PcgGeom& g = a.g;
  const int t = threadIdx.x, nn = g.nn, n1 = g.n1, N = g.N, m = g.m, nq = g.nq;
  const bool own = t < nn;
  const double* cb = C.T.cb;
  const double* cd = C.T.cd;
  const double* gw = C.T.gw;
  double* sig = C.sig;
  const int* cs = C.T.cs;
  const int* ck0 = C.T.ck0;
  const int* ck1 = C.T.ck1;
  const double* fcg = a.el.face + e * 4 * nq * 3;
  if (C.gtab) {
    C.T.fc = fcg;
  } else {
    double* fcl = const_cast<double*>(C.T.fc);
    for (int i = t; i < 4 * nq * 3; i += blockDim.x) fcl[i] = fcg[i];
  }
  const double* fc = C.T.fc;
  C.ub = C.vb = C.yu = C.yv = C.xs0 = C.xm0 = C.wt = 0.0;
  if (NODAL && own) {
    C.ub = a.in_u[e * nn + t];
    C.vb = a.in_v[e * nn + t];
    if (STAGE > 1) {
      C.yu = a.aux_u[e * nn + t];
      C.yv = a.aux_v[e * nn + t];
    }
    C.U[t] = C.ub;
    C.V[t] = C.vb;
    C.xs0 = a.xS[e * nn + t];
    C.xm0 = a.xM[e * nn + t];
    C.wt = a.el.w[e * nn + t];
    C.ms = a.el.msc ? a.el.msc[e * nn + t] : 1.0;
  }
  if constexpr (NODAL) {
    const double* sc = a.el.sc + e * 8;
    C.cw = sc[0];
    C.kbr = sc[1];
    C.kbs = sc[2];
    C.d00 = sc[3];
    C.area = sc[4];
  }
  const int ex = (int)(e % a.nx), ey = (int)(e / a.nx);
  __syncthreads();
  after_first_barrier();

  // ---- face fluxes sigma_u, sigma_v at the face points (Sec. 2.2.1) ----------------
  for (int id = t; id < 4 * nq; id += blockDim.x) {
    const int f = id / nq, q = id - (id / nq) * nq;
    // neighbour across face f (periodic wrap); a wall face (its side is not periodic and
    // the element touches it) reads its own trace instead, negated for Dirichlet: the
    // mirror exterior state
    int nbx = ex, nby = ey, fnb;
    bool wall;
    if (f == 0) { wall = ex + 1 == a.nx; nbx = wall ? 0 : ex + 1; fnb = 1; }
    else if (f == 1) { wall = ex == 0; nbx = wall ? a.nx - 1 : ex - 1; fnb = 0; }
    else if (f == 2) { wall = ey + 1 == a.ny; nby = wall ? 0 : ey + 1; fnb = 3; }
    else { wall = ey == 0; nby = wall ? a.ny - 1 : ey - 1; fnb = 2; }
    const int kf = (a.bcbits >> (2 * f)) & 3;
    wall = wall && kf != 0;
    const long enb = (long)nby * a.nx + nbx;
    const double* ts = a.tr_in + (e * 4 * nq + id) * 2;
    const double* tn = wall ? ts : a.tr_in + (enb * 4 * nq + fnb * nq + q) * 2;
    const double as = ts[0], vs = ts[1];
    double an = tn[0], vn = tn[1];
    if (wall && kf == 1) {
      an = -an;
      vn = -vn;
    }
    const double alpha = wall ? 0.5 : a.alf[f];
    const double jv = vn - vs;
    sig[id * 2] = (1.0 - alpha) * jv - a.beta * (as + an);
    sig[id * 2 + 1] = (1.0 - alpha) * as - alpha * an + a.tau * jv;
  }
  __syncthreads();
  // lifts: per face and node l along the face,
  //   cB[l] = sum_q wq sigma_u (K Nh)_normal B[q][l],  cD[l] = sum_q wq sigma_u (K Nh)_tangent D[q][l],
  //   cV[l] = sum_q wq c^2 s_J sigma_v B[q][l]
  // over the face cells k whose window holds l; 8 lanes per (face, node), lane kk takes
  // cells ck0[l] + kk, ck0[l] + kk + 8, ..., and the lanes' parts are added by DPP.  A node
  // lies in up to p + 1 + (p - 1) / 2 windows where the closure clamps them (11 at p = 7).
  for (int base = 0; base < 4 * n1 * 8; base += blockDim.x) {
    const int fl = (base + t) >> 3, kk = (base + t) & 7;
    double cB = 0, cD = 0, cV = 0;
    int f = 0, l = 0;
    if (fl < 4 * n1) {
      f = fl / n1;
      l = fl - f * n1;
      for (int k = ck0[l] + kk; k <= ck1[l]; k += 8) {
        const int j = l - cs[k];
#pragma unroll 2
        for (int qa = 0; qa < m; ++qa) {
          {
            const int id = f * nq + k * m + qa;
            const double wq = gw[qa] / N;
            const double* Fq = fc + id * 3;
            const double kn = f < 2 ? Fq[0] : Fq[1], kt = f < 2 ? Fq[1] : Fq[0];
            const double bj = cb[(k * m + qa) * m + j], dj = cd[(k * m + qa) * m + j];
            const double su = wq * sig[id * 2];
            cB += su * kn * bj;
            cD += su * kt * dj;
            cV += wq * Fq[2] * sig[id * 2 + 1] * bj;
          }
        }
      }
    }
    cB = sum8(cB);
    cD = sum8(cD);
    cV = sum8(cV);
    if (fl < 4 * n1 && kk == 0) {
      C.lines[(f * 4 + 0) * n1 + l] = cB;
      C.lines[(f * 4 + 1) * n1 + l] = cD;
      C.lines[(f * 4 + 2) * n1 + l] = cV;
    }
  }
  __syncthreads();
  const double* dL = C.T.dL;
  const double* dR = C.T.dR;
  if (own) {
    const int ix = t % n1, iy = t / n1;
    const double* LE = C.lines + 0 * 4 * n1;
    const double* LW = C.lines + 1 * 4 * n1;
    const double* LN = C.lines + 2 * 4 * n1;
    const double* LS = C.lines + 3 * 4 * n1;
    double fu = dR[ix] * LE[iy] + dL[ix] * LW[iy] + dR[iy] * LN[ix] + dL[iy] * LS[ix];
    double fv = 0;
    if (ix == N) { fu += LE[n1 + iy]; fv += LE[2 * n1 + iy]; }
    if (ix == 0) { fu += LW[n1 + iy]; fv += LW[2 * n1 + iy]; }
    if (iy == N) { fu += LN[n1 + ix]; fv += LN[2 * n1 + ix]; }
    if (iy == 0) { fu += LS[n1 + ix]; fv += LS[2 * n1 + ix]; }
    C.Fu[t] = fu;
    C.rv[t] = fv;
  }
}

// RK stage update from dU/dt = V + y, dV/dt = z, outputs, warm starts, traces of the new
// value and iteration counters.  Starts with a barrier-free register phase; y, z are the
// owner thread's solution entries.  SPLIT: y and z were stored by the solve kernels, which
// also keep the counters; only the update and the traces are done here.
template <int STAGE, bool SPLIT = false>
__device__ __forceinline__ void stage_epilogue(const PcgStageArgs& a, const long e,
                                               const StageCommon& C, double y, double z,
                                               int itS, int itM, int swS = 0, int swM = 0) {
  const PcgGeom& g = a.g;
  const int t = threadIdx.x, nn = g.nn;
  const bool own = t < nn;
  const double ku = C.vb + y, dt = a.dt;
  double kv = z;
  if (own) {
    const long gi = e * nn + t;
    if (a.nf > 0) {   // source term: M_J^-1 (M_J g_k) = g_k, added to dv/dt
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < a.nf) kv += a.f_w[4 * (STAGE - 1) + k] * a.frc[k * a.frc_stride + gi];
    }
    double nu, nv;
    if (STAGE == 1) {
      nu = C.ub + 0.5 * dt * ku;
      nv = C.vb + 0.5 * dt * kv;
    } else if (STAGE == 2) {
      nu = C.yu + 0.5 * dt * ku;
      nv = C.yv + 0.5 * dt * kv;
      a.acc_u[gi] = C.ub + 2.0 * nu - C.yu;
      a.acc_v[gi] = C.vb + 2.0 * nv - C.yv;
    } else if (STAGE == 3) {
      nu = C.yu + dt * ku;
      nv = C.yv + dt * kv;
    } else {
      nu = (C.yu + C.ub) * (1.0 / 3.0) + dt * (1.0 / 6.0) * ku;
      nv = (C.yv + C.vb) * (1.0 / 3.0) + dt * (1.0 / 6.0) * kv;
    }
    a.out_u[gi] = nu;
    a.out_v[gi] = nv;
    if constexpr (!SPLIT) {
      a.xS[gi] = y;
      a.xM[gi] = z;
    }
    C.U[t] = nu;
    C.V[t] = nv;
  }
  __syncthreads();
  face_traces_lds(g, C.T, C.U, C.V, C.lines, a.tr_out + e * 4 * g.nq * 2);
  if (!SPLIT && t == 0) {
    int* its = a.its + e * kItsPer;
    its[0] += itS > a.maxit ? a.maxit : itS;
    its[1] += itM > a.maxit ? a.maxit : itM;
    if (itS > its[2]) its[2] = itS;
    if (itM > its[3]) its[3] = itM;
    its[4] += swS;
    its[5] += swM;
    if (itS > a.maxit || itM > a.maxit) atomicMin(a.fail, (int)e);
  }
}

// ---------------------------------------------------------------------------------
// Stage with the row-rectangle operator layout (any N, p; FULL or HALF).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void pcg_stage_carve(const PcgStageArgs& a, PcgShared& W,
                                                StageCommon& C) {
  extern __shared__ double shd[];
  const PcgGeom& g = a.g;
  const int nn = g.nn;
  W.full = a.full;
  W.Q = a.full ? a.Q : 0;
  double* sp = shd;
  W.A = sp;            sp += a.full ? a.nnz_full : g.nst;
  W.part = sp;         sp += W.Q * nn;
  W.x = sp;            sp += nn;
  W.r = sp;            sp += nn;
  W.z = sp;            sp += nn;
  W.d = sp;            sp += nn;
  W.q = sp;            sp += nn;
  W.tmp = sp;          sp += nn;
  W.b = sp;            sp += nn;
  W.Psi = sp;          sp += nn;
  // ints after all doubles
  int* ip = reinterpret_cast<int*>(shd + (a.full ? a.nnz_full : g.nst) + W.Q * nn + 8 * nn +
                                   common_doubles(g));
  W.fo = ip;           ip += nn + 1;
  W.ho = ip;           ip += nn + 1;
  stage_carve(g, sp, ip, C);
  W.red = C.red;
}

__device__ __forceinline__ void pcg_stage_load_tables(const PcgStageArgs& a, const PcgShared& W,
                                                      const StageCommon& C) {
  const PcgGeom& g = a.g;
  int* fo = const_cast<int*>(W.fo);
  int* ho = const_cast<int*>(W.ho);
  for (int i = threadIdx.x; i <= g.nn; i += blockDim.x) {
    fo[i] = a.fo[i];
    ho[i] = g.rowoff[i];
  }
  stage_load_tables(g, W.Psi, g.n1, C);
}

template <int STAGE>
__device__ __forceinline__ void pcg_stage_elem(const PcgStageArgs& a, const long e,
                                               PcgShared& W, StageCommon& C) {
  const PcgGeom& g = a.g;
  const int t = threadIdx.x, nn = g.nn, n1 = g.n1;
  const bool own = t < nn;
  stage_prologue<STAGE>(a, e, C, [&]() { op_load(g, W, a.el.S + e * g.nst, a.dst); });
  // r = -S_K U + F_v   (op_apply starts with the operator / U complete: the barriers of
  // the prologue cover U and the operator load)
  {
    const double su = op_apply(g, W, C.U);
    if (own) C.rv[t] -= su;
  }
  // ---- S_hat y = F_u ------------------------------------------------------------------
  double dS = 1.0;
  if (own) {
    const int kx = t % n1, ky = t / n1;
    dS = t == 0 ? C.d00 : C.kbr * C.lamr[kx] + C.kbs * C.lamr[ky];
    if (a.el.dlog && t > 0) dS *= exp((double)a.el.dlog[e * nn + t]);
    W.x[t] = C.xs0;
    W.b[t] = C.Fu[t];
  }
  __syncthreads();
  int itS = pcg_solve(g, W, C.cw, C.wt, own ? 1.0 / dS : 0.0, a.rtol, a.maxit);
  if (itS > a.maxit && a.el.dlog) {
    // the corrected preconditioner failed: repeat with the plain one from the same start
    if (own) {
      const int kx = t % n1, ky = t / n1;
      dS = t == 0 ? C.d00 : C.kbr * C.lamr[kx] + C.kbs * C.lamr[ky];
      W.x[t] = C.xs0;
    }
    __syncthreads();
    itS = pcg_solve(g, W, C.cw, C.wt, own ? 1.0 / dS : 0.0, a.rtol, a.maxit);
  }
  const double y = own ? W.x[t] : 0.0;
  __syncthreads();
  // ---- M_J z = r --------------------------------------------------------------------
  int itM;
  if (a.mapped) {
    op_load(g, W, a.el.M + e * g.nst, a.dst);
    if (own) {
      W.x[t] = C.xm0;
      W.b[t] = C.rv[t];
    }
    __syncthreads();
    itM = pcg_solve(g, W, 0.0, 0.0, own ? 1.0 / C.area : 0.0, a.rtol, a.maxit, C.ms);
  } else {
    // Cartesian: M_J = |Omega| M_ref (x) M_ref = Psi_2^{-T} diag(|Omega|) Psi_2^{-1}, so the
    // preconditioner is the exact inverse (one PCG iteration).
    double bb1[1] = {own ? C.rv[t] * C.rv[t] : 0.0};
    block_sum<1>(bb1, W.red, nn);
    const double bb = bb1[0];
    pinv_apply<double>(C.rv, W.tmp, W.x, W.Psi, 1.0 / C.area, n1, nn);
    itM = bb > 0.0 ? 1 : 0;
  }
  const double z = own ? W.x[t] : 0.0;
  __syncthreads();
  stage_epilogue<STAGE>(a, e, C, y, z, itS, itM);
}

// ---------------------------------------------------------------------------------
// Stage with the column-block operator layout (N + 1 in {9, 13, 17}, FP64 operator in LDS).
//
// The operator is stored as blocks B(ix, jy) = { A[(ix, iy), (jx, jy)] : iy in band(jy),
// jx in band(ix) } (rows of length w(ix)).  A work unit (ix, jy, c) takes rows
// iy = lo(jy) + c*CH ... of its block: it reads the w(ix) values x[jy][band(ix)] once and
// forms CH partial row sums, which go to slot jy - lo(iy) of row (ix, iy); each row then
// adds its w(iy) partials in a fixed order.  Vectors of the solve are stored on an
// (N+2) x (N+2) padded grid (rows of even length), so the preconditioner's transforms run
// on 2 x 2 output blocks per thread without bounds tests.  The PCG recurrence is the
// single-reduction form of Chronopoulos and Gear: one workgroup reduction per iteration.
// ---------------------------------------------------------------------------------
// At most 768 threads (12 waves, 3 per SIMD), so that a lane may hold 170 VGPRs.
constexpr int kBlkMaxThreads = 768;

// Lanes per output of the preconditioner's transforms for nn outputs on at most maxt
// threads.
__host__ __device__ constexpr int blk_pinv_split(int nn, int maxt) {
  return 4 * nn <= maxt ? 4 : 2 * nn <= maxt ? 2 : 1;
}

// Block size of the register-operator kernels: 8 waves (2 per SIMD), so that a lane may
// hold 256 VGPRs.
constexpr int kRegMaxThreads = 512;

template <int N1C, typename TA = double, int MAXT = kBlkMaxThreads>
struct BlockSolve {
  TA* A;                                     // operator (block layout)
  double *P;                                 // row partials
  double *R, *U, *T, *Z, *DI, *Psi;
  const int *boff, *jc;
  int K, CH, WB, p, N;
};

template <int N1C, typename TA, int MT>
__device__ __forceinline__ double blk_apply(const BlockSolve<N1C, TA, MT>& W,
                                            const double* __restrict__ x) {
  constexpr int n1 = N1C, NP = N1C + 1, WM = N1C < 15 ? N1C : 15;
  const int t = threadIdx.x;
  if (t < n1 * W.K) {
    const int k = t / n1, ix = t - k * n1;
    const int jcv = W.jc[k], jy = jcv & 0xff, c = jcv >> 8;
    const int lox = st_lo(ix, W.p), wx = st_w(ix, W.p, W.N);
    const int loy = st_lo(jy, W.p), wy = st_w(jy, W.p, W.N);
    const int i0 = c * W.CH;
    const int ni = min(W.CH, wy - i0);
    double xs[WM];
#pragma unroll
    for (int q = 0; q < WM; ++q) xs[q] = q < wx ? x[jy * NP + lox + q] : 0.0;
    const TA* Ab = W.A + W.boff[jy * n1 + ix] + i0 * wx;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i < ni) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < WM; ++q)
          if (q < wx) acc += (double)Ab[i * wx + q] * xs[q];
        const int iy = loy + i0 + i;
        W.P[(iy * n1 + ix) * W.WB + (jy - st_lo(iy, W.p))] = acc;
      }
    }
  }
  __syncthreads();
  double y = 0.0;
  if (t < n1 * n1) {
    const int iy = t / n1;
    const int wiy = st_w(iy, W.p, W.N);
    const double* pr = W.P + t * W.WB;
    for (int q = 0; q < wiy; ++q) y += pr[q];
  }
  return y;
}

// out = Psi_2 diag(DI) Psi_2^T R on the padded grid; ends with a barrier.  Each of the
// four 1D transforms gives every output (a, b) to SP adjacent lanes (one quad), which
// split its sum over the contracted index and combine the parts with DPP lane moves, so
// that one batch of LDS loads per lane covers a phase.
template <int N1C, typename TA, int MT>
__device__ __forceinline__ void blk_pinv_lanes(const BlockSolve<N1C, TA, MT>& W,
                                               const double* __restrict__ R,
                                               double* __restrict__ out) {
  constexpr int n1 = N1C, NP = N1C + 1, nn = N1C * N1C;
  constexpr int SP = blk_pinv_split(nn, MT);
  constexpr int NT = (n1 + SP - 1) / SP;          // terms per lane
  const int t = threadIdx.x;
  const int o = t / SP, part = t - o * SP;
  const bool act = o < nn;
  const int a = act ? o / n1 : 0, b = act ? o - (o / n1) * n1 : 0;
  const double* Ps = W.Psi;
  auto combine = [&](double v) {
    if constexpr (SP >= 2) v += dpp_mov<0xb1, 0xf, false>(v);  // lanes ^1
    if constexpr (SP == 4) v += dpp_mov<0x4e, 0xf, false>(v);  // lanes ^2
    return v;
  };
  double s = 0.0;
  // T[a][b] = sum_i Psi[i][a] R[i][b]
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const int i = part + k * SP;
    if (act && i < n1) s += Ps[i * NP + a] * R[i * NP + b];
  }
  s = combine(s);
  if (act && part == 0) W.T[a * NP + b] = s;
  __syncthreads();
  // Z[a][b] = DI[a][b] sum_i T[a][i] Psi[i][b]
  s = 0.0;
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const int i = part + k * SP;
    if (act && i < n1) s += W.T[a * NP + i] * Ps[i * NP + b];
  }
  s = combine(s);
  if (act && part == 0) W.Z[a * NP + b] = s * W.DI[a * NP + b];
  __syncthreads();
  // T[a][b] = sum_k Psi[a][k] Z[k][b]
  s = 0.0;
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const int i = part + k * SP;
    if (act && i < n1) s += Ps[a * NP + i] * W.Z[i * NP + b];
  }
  s = combine(s);
  if (act && part == 0) W.T[a * NP + b] = s;
  __syncthreads();
  // out[a][b] = sum_k T[a][k] Psi[b][k]
  s = 0.0;
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const int i = part + k * SP;
    if (act && i < n1) s += W.T[a * NP + i] * Ps[b * NP + i];
  }
  s = combine(s);
  if (act && part == 0) out[a * NP + b] = s;
  __syncthreads();
}

typedef double pcg_d4 __attribute__((ext_vector_type(4)));

// The same four transforms on the FP64 matrix cores, for N + 1 <= 16: each is a 16 x 16 x 16
// product (zero padded) done by one wave as four v_mfma_f64_16x16x4 steps.  Lane l = 16 g + c
// holds A[c][4 s + g] and B[4 s + g][c] of step s and gets D[4 r + g][c] in register r.  So a
// product's D registers are the A operand of the next product read as a transpose
// (D[4 s + g][c] taken as A[c][4 s + g]), and the chain alternates
//   T1^T = R^T Psi,   T2 = T1 Psi,   Z = DI o T2,   T3^T = Z^T Psi^T,   out = T3 Psi^T
// with only R read from and only out written to LDS.  The other waves wait at the closing
// barrier.
template <int N1C, typename TA, int MT>
__device__ __forceinline__ void blk_pinv_mfma(const BlockSolve<N1C, TA, MT>& W,
                                              const double* __restrict__ R,
                                              double* __restrict__ out) {
  static_assert(N1C <= 16, "one 16 x 16 tile");
  constexpr int n1 = N1C, NP = N1C + 1;
  const int t = threadIdx.x;
  if (t < 64) {
    const int c = t & 15, g = t >> 4;
    const double* Ps = W.Psi;
    const bool cin = c < n1;
    double psk[4], pks[4];          // Psi[4s+g][c] and Psi[c][4s+g]
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + g;
      const bool in = cin && k < n1;
      psk[s] = in ? Ps[k * NP + c] : 0.0;
      pks[s] = in ? Ps[c * NP + k] : 0.0;
    }
    pcg_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + g;
      const double rv = (cin && k < n1) ? R[k * NP + c] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(rv, psk[s], acc, 0, 0, 0);
    }
    pcg_d4 acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[s], psk[s], acc2, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = 4 * r + g;
      acc2[r] *= (cin && a < n1) ? W.DI[a * NP + c] : 0.0;
    }
    pcg_d4 acc3 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(acc2[s], pks[s], acc3, 0, 0, 0);
    pcg_d4 acc4 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      acc4 = __builtin_amdgcn_mfma_f64_16x16x4f64(acc3[s], pks[s], acc4, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = 4 * r + g;
      if (cin && a < n1) out[a * NP + c] = acc4[r];
    }
  }
  __syncthreads();
}

// Preconditioner application: matrix cores where the grid fits one tile.
template <int N1C, typename TA, int MT>
__device__ __forceinline__ void blk_pinv(const BlockSolve<N1C, TA, MT>& W,
                                         const double* __restrict__ R, double* __restrict__ out) {
  if constexpr (N1C <= 16) blk_pinv_mfma(W, R, out);
  else blk_pinv_lanes(W, R, out);
}

// PCG (single-reduction recurrence) on (A_op + cw w w^T) x = b; owner thread t < nn holds
// x (in/out, warm start on entry), b and w.  Iteration count as pcg_solve.  zero_start:
// x = 0 on entry (the first product is skipped).  scaled (uniform over the block): the
// preconditioner is P^-1 r -> sc P^-1 (sc r) with sc this owner's nodal scale; the scaled
// vector is written back to W.U before the product reads it.
// EARLY: the stop test reads |r|^2 (one more workgroup reduction, in red[64..79], apart from
// the others' slots) as soon as r is updated, so a converged solve skips its last
// preconditioning and product; worth it where a product costs far more than a reduction
// (operators read from memory in every product).  The counts and iterates are those of the
// plain form.
template <int N1C, typename TA, int MT, typename App, bool EARLY = false>
__device__ __forceinline__ int blk_solve_g(const BlockSolve<N1C, TA, MT>& W, App&& apply, double* red,
                                           double& x, double bval, double cw, double wt,
                                           double rtol, int maxit, bool zero_start,
                                           bool scaled = false, double sc = 1.0) {
  constexpr int n1 = N1C, NP = N1C + 1, nn = N1C * N1C;
  const int t = threadIdx.x;
  const bool own = t < nn;
  const int pidx = own ? (t / n1) * NP + (t - (t / n1) * n1) : 0;
  double ax = 0.0;
  if (!zero_start) {
    if (own) W.U[pidx] = x;
    __syncthreads();
    ax = apply(W.U);
  }
  // The reductions leave out their closing barrier: every later write of red comes after
  // the barrier that publishes R, and each return passes one barrier.
  double s2[2] = {own ? wt * x : 0.0, own ? bval * bval : 0.0};
  block_sum<2, false>(s2, red, nn);
  const double bb = s2[1];
  if (bb == 0.0) {
    x = 0.0;
    __syncthreads();
    return 0;
  }
  double r = own ? bval - ax - cw * s2[0] * wt : 0.0;
  const double tol2 = rtol * rtol * bb;
  if constexpr (EARLY) {
    double e1[1] = {r * r};
    block_sum<1, false>(e1, red + 64, nn);
    if (e1[0] <= tol2) {
      __syncthreads();
      return 0;
    }
  }
  if (own) W.R[pidx] = scaled ? r * sc : r;
  __syncthreads();
  blk_pinv(W, W.R, W.U);
  double u = own ? W.U[pidx] : 0.0;
  if (scaled) {
    u *= sc;
    if (own) W.U[pidx] = u;
    __syncthreads();
  }
  double q = apply(W.U);
  double s4[4] = {r * u, q * u, wt * u, r * r};
  block_sum<4, false>(s4, red, nn);
  if (s4[3] <= tol2) {
    __syncthreads();
    return 0;
  }
  double gam = s4[0];
  double alpha = gam / (s4[1] + cw * s4[2] * s4[2]);
  double pv = u, sv = q + cw * s4[2] * wt;
  for (int it = 1; it <= maxit; ++it) {
    x += alpha * pv;
    r -= alpha * sv;
    if constexpr (EARLY) {
      double e1[1] = {r * r};
      block_sum<1, false>(e1, red + 64, nn);
      if (e1[0] <= tol2) {
        __syncthreads();
        return it;
      }
    }
    if (own) W.R[pidx] = scaled ? r * sc : r;
    __syncthreads();
    blk_pinv(W, W.R, W.U);
    u = own ? W.U[pidx] : 0.0;
    if (scaled) {
      u *= sc;
      if (own) W.U[pidx] = u;
      __syncthreads();
    }
    q = apply(W.U);
    double sr[4] = {r * u, q * u, wt * u, r * r};
    block_sum<4, false>(sr, red, nn);
    if (sr[3] <= tol2) {
      __syncthreads();
      return it;
    }
    const double gn = sr[0];
    const double dn = sr[1] + cw * sr[2] * sr[2];
    const double beta = gn / gam;
    alpha = gn / (dn - beta * gn / alpha);
    pv = u + beta * pv;
    sv = (q + cw * sr[2] * wt) + beta * sv;
    gam = gn;
  }
  __syncthreads();
  return maxit + 1;
}

template <int N1C, typename TA, int MT>
__device__ __forceinline__ int blk_solve(const BlockSolve<N1C, TA, MT>& W, double* red, double& x,
                                         double bval, double cw, double wt, double rtol, int maxit,
                                         bool zero_start = false, bool scaled = false,
                                         double sc = 1.0) {
  return blk_solve_g(W, [&W](const double* v) { return blk_apply(W, v); }, red, x, bval, cw, wt,
                     rtol, maxit, zero_start, scaled, sc);
}

// Copy one element operator from its HBM upper half into the block layout.
__device__ __forceinline__ void blk_load(const int nst, double* A, const double* __restrict__ half,
                                const int* __restrict__ dst) {
  // all loads of a lane first (8 per batch), then the LDS stores
  const int step = blockDim.x;
  for (int h0 = threadIdx.x; h0 < nst; h0 += 8 * step) {
    double v[8];
    int2 d2[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int h = h0 + k * step;
      if (h < nst) {
        v[k] = half[h];
        d2[k] = reinterpret_cast<const int2*>(dst)[h];
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int h = h0 + k * step;
      if (h < nst) {
        A[d2[k].x] = v[k];
        A[d2[k].y] = v[k];
      }
    }
  }
}

template <int N1C>
__host__ __device__ inline size_t blk_lds_doubles(const PcgGeom& g, int nnz_full, int WB) {
  constexpr int NP = N1C + 1;
  return (size_t)nnz_full + (size_t)g.nn * WB + 6 * NP * NP + common_doubles(g);
}

// ---------------------------------------------------------------------------------
// Mixed precision (FP32 operator for the inner iterations, FP64 residual refinement).
//
// The operator is split as A = A_hi + A_lo, A_hi = fl32(A), A_lo = fl32(A - A_hi) (their sum
// holds A to about 2^-48).  The inner PCG runs on A_hi, kept in LDS in FP32 (half the
// bytes of the FP64 operator, so that two elements fit a CU); the outer loop forms the
// true residual b - (A_hi + A_lo) x in FP64 with A_lo read from global memory and solves
// for the correction until the FP64 residual meets rtol.
// ---------------------------------------------------------------------------------
constexpr int kMaxSweeps = 8;
constexpr double kInnerTol = 1e-6;

// region sizes (in doubles) of the mixed layout
template <int N1C>
__host__ __device__ inline int mix_a_doubles(int nnz) { return (nnz + 1) / 2; }
template <int N1C>
__host__ __device__ inline int mix_p_doubles(const PcgGeom& g, int WB) {
  const int pf = g.nn * WB;                         // row partials
  const int sg = 4 * g.nq * 2;                      // face fluxes (prologue only)
  return pf > sg ? pf : sg;
}
template <int N1C>
__host__ __device__ inline size_t mix_lds_doubles(const PcgGeom& g, int nnz_full, int WB) {
  constexpr int NP = N1C + 1;
  return (size_t)mix_a_doubles<N1C>(nnz_full) + mix_p_doubles<N1C>(g, WB) + 6 * NP * NP +
         common_small_doubles(g);
}

// y_t = ((A_hi + A_lo) x)_t in FP64 for owner threads (row (ix, iy)); x padded, in LDS.
template <int N1C>
__device__ __forceinline__ double blk_apply64(const BlockSolve<N1C, float>& W,
                                              const float* __restrict__ lo,
                                              const double* __restrict__ x) {
  constexpr int n1 = N1C, NP = N1C + 1;
  const int t = threadIdx.x;
  double y = 0.0;
  if (t < n1 * n1) {
    const int iy = t / n1, ix = t - (t / n1) * n1;
    const int lox = st_lo(ix, W.p), wx = st_w(ix, W.p, W.N);
    const int loyi = st_lo(iy, W.p), hiyi = st_hi(iy, W.p, W.N);
    for (int jy = loyi; jy <= hiyi; ++jy) {
      const int off = W.boff[jy * n1 + ix] + (iy - st_lo(jy, W.p)) * wx;
      for (int q = 0; q < wx; ++q)
        y += ((double)W.A[off + q] + (double)lo[off + q]) * x[jy * NP + lox + q];
    }
  }
  return y;
}

// Refined solve of (A + cw w w^T) x = b: FP64 residuals, inner PCG on A_hi.  Returns the
// total inner iteration count (maxit + 1 on failure); *sweeps = residual evaluations - 1.
// The refinement contracts by about kappa(A) 2^-24 per sweep (entrywise rounding of an
// operator with strongly cancelling rows); where that stalls, the solve continues from the
// refined iterate as plain PCG with the FP64-accurate product (hi + lo) x.
template <int N1C>
__device__ __forceinline__ int blk_solve_mixed(const BlockSolve<N1C, float>& W,
                                               const float* __restrict__ lo, double* red,
                                               double& x, double bval, double cw, double wt,
                                               double rtol, int maxit, int* sweeps,
                                               bool scaled = false, double msc = 1.0) {
  constexpr int n1 = N1C, NP = N1C + 1, nn = N1C * N1C;
  const int t = threadIdx.x;
  const bool own = t < nn;
  const int pidx = own ? (t / n1) * NP + (t - (t / n1) * n1) : 0;
  double sb[1] = {own ? bval * bval : 0.0};
  block_sum<1>(sb, red, nn);
  const double bb = sb[0];
  *sweeps = 0;
  if (bb == 0.0) {
    x = 0.0;
    return 0;
  }
  const double tol2 = rtol * rtol * bb;
  int total = 0, sw = 0;
  for (; sw < kMaxSweeps; ++sw) {
    if (own) W.U[pidx] = x;
    __syncthreads();
    const double ax = blk_apply64(W, lo, W.U);
    double s1[1] = {own ? wt * x : 0.0};
    block_sum<1>(s1, red, nn);
    const double r = own ? bval - ax - cw * s1[0] * wt : 0.0;
    double s2[1] = {r * r};
    block_sum<1>(s2, red, nn);
    if (s2[0] <= tol2) {
      *sweeps = sw;
      return total;
    }
    const double sc = 1.0 / sqrt(s2[0]);
    // inner tolerance: what is left to reach rtol, but not below the FP32 operator's floor
    const double tin = fmax(kInnerTol, 0.5 * sqrt(tol2 / s2[0]));
    double c = 0.0;
    const int its = blk_solve<N1C, float>(W, red, c, r * sc, cw, wt, tin, maxit, true, scaled,
                                           msc);
    total += its > maxit ? maxit : its;
    if (its > maxit || total > maxit) break;
    x += c / sc;
  }
  *sweeps = sw + 1;
  // fallback: PCG with the accurate product from the current iterate
  const int its = blk_solve_g(W, [&W, lo](const double* v) { return blk_apply64(W, lo, v); }, red,
                              x, bval, cw, wt, rtol, maxit, false, scaled, msc);
  return its > maxit ? maxit + 1 : total + its;
}

template <int N1C, int MT = kBlkMaxThreads>
__device__ __forceinline__ void pcg2_stage_carve(const PcgStageArgs& a, BlockSolve<N1C, double, MT>& W,
                                                 StageCommon& C) {
  extern __shared__ double shd[];
  constexpr int NP = N1C + 1, nn = N1C * N1C;
  const PcgGeom& g = a.g;
  W.K = a.blk_K;
  W.CH = a.blk_CH;
  W.WB = a.blk_WB;
  W.p = g.p;
  W.N = g.N;
  double* sp = shd;
  W.A = sp;    sp += a.nnz_full;
  W.P = sp;    sp += nn * W.WB;
  W.R = sp;    sp += NP * NP;
  W.U = sp;    sp += NP * NP;
  W.T = sp;    sp += NP * NP;
  W.Z = sp;    sp += NP * NP;
  W.DI = sp;   sp += NP * NP;
  W.Psi = sp;  sp += NP * NP;
  int* ip = reinterpret_cast<int*>(shd + blk_lds_doubles<N1C>(g, a.nnz_full, W.WB));
  W.boff = ip;  ip += nn;
  W.jc = ip;    ip += W.K;
  stage_carve(g, sp, ip, C);
}

template <int STAGE, int N1C>
__device__ __forceinline__ void pcg2_stage_elem(const PcgStageArgs& a, const long e,
                                                BlockSolve<N1C>& W, StageCommon& C) {
  constexpr int n1 = N1C, NP = N1C + 1, nn = N1C * N1C;
  const PcgGeom& g = a.g;
  const int t = threadIdx.x;
  const bool own = t < nn;
  const int pidx = own ? (t / n1) * NP + (t - (t / n1) * n1) : 0;
  double* const Aop = W.A;
  const double* const Shalf = a.el.S + e * g.nst;
  const int* const bdst = a.blk_dst;
  const int nst = g.nst;
  stage_prologue<STAGE>(a, e, C, [Aop, Shalf, bdst, nst]() { blk_load(nst, Aop, Shalf, bdst); });
  // r = -S_K U + F_v   (operator, tables, U complete after the prologue's barriers)
  if (own) W.U[pidx] = C.U[t];
  __syncthreads();
  {
    const double su = blk_apply(W, W.U);
    if (own) C.rv[t] -= su;
  }
  // ---- S_hat y = F_u ------------------------------------------------------------------
  double dS = 1.0;
  if (own) {
    const int kx = t % n1, ky = t / n1;
    dS = t == 0 ? C.d00 : C.kbr * C.lamr[kx] + C.kbs * C.lamr[ky];
    if (a.el.dlog && t > 0) dS *= exp((double)a.el.dlog[e * nn + t]);
    W.DI[pidx] = 1.0 / dS;
  }
  double y = C.xs0;
  int itS = blk_solve(W, C.red, y, own ? C.Fu[t] : 0.0, C.cw, C.wt, a.rtol, a.maxit);
  if (itS > a.maxit && a.el.dlog) {
    if (own) {
      const int kx = t % n1, ky = t / n1;
      W.DI[pidx] = 1.0 / (t == 0 ? C.d00 : C.kbr * C.lamr[kx] + C.kbs * C.lamr[ky]);
    }
    y = C.xs0;
    itS = blk_solve(W, C.red, y, own ? C.Fu[t] : 0.0, C.cw, C.wt, a.rtol, a.maxit);
  }
  __syncthreads();
  // ---- M_J z = r --------------------------------------------------------------------
  int itM;
  double z;
  if (own) W.DI[pidx] = 1.0 / C.area;
  if (a.mapped) {
    blk_load(g.nst, W.A, a.el.M + e * g.nst, a.blk_dst);
    z = C.xm0;
    itM = blk_solve(W, C.red, z, own ? C.rv[t] : 0.0, 0.0, 0.0, a.rtol, a.maxit, false,
                    a.el.msc != nullptr, C.ms);
  } else {
    // Cartesian: the preconditioner is the exact inverse of M_J
    double bb1[1] = {own ? C.rv[t] * C.rv[t] : 0.0};
    if (own) W.R[pidx] = C.rv[t];
    block_sum<1>(bb1, C.red, nn);
    blk_pinv(W, W.R, W.U);
    z = own ? W.U[pidx] : 0.0;
    itM = bb1[0] > 0.0 ? 1 : 0;
  }
  __syncthreads();
  stage_epilogue<STAGE>(a, e, C, own ? y : 0.0, own ? z : 0.0, itS, itM);
}

// ---------------------------------------------------------------------------------
// Operator in registers (FP64, column-block work units).  The entries a work unit of the
// block product multiplies are the same in every iteration of a solve, so each unit keeps
// its CH x W entries in registers and an iteration reads only x and the row partials from
// LDS.  The entries come from a copy of the operator that set-up permutes into work-unit
// slot order (slot-major, so that every load of a wave is one contiguous run); the
// operator never passes through LDS, which holds only the vectors and row partials.
// Compiled for fixed (N + 1, p), which fixes W = min(2p + 1, N + 1) and the chunk height
// CH chosen by the same rule as the host tables.
// ---------------------------------------------------------------------------------
__host__ __device__ constexpr int blk_band_c(int k, int p, int N) {
  return (k + p < N ? k + p : N) - (k - p > 0 ? k - p : 0) + 1;
}
__host__ __device__ constexpr int blk_ch_c(int n1, int p, int maxt, int chmax = 8) {
  for (int ch = 1; ch <= chmax; ++ch) {
    int kk = 0;
    for (int jy = 0; jy < n1; ++jy) kk += (blk_band_c(jy, p, n1 - 1) + ch - 1) / ch;
    if (n1 * kk <= maxt) return ch;
  }
  return 0;
}

template <int N1C, int P>
struct RegOp {
  static constexpr int W = 2 * P + 1 < N1C ? 2 * P + 1 : N1C;
  static constexpr int CH = blk_ch_c(N1C, P, kRegMaxThreads);
  static_assert(CH > 0, "no chunk height fits the thread limit");
  double a[CH][W];
  int xoff;          // jy * NP + lo(ix): first x value of the unit
  int wx, ni;        // columns and rows of the unit (0 rows: no unit)
  int pd[CH];        // row-partial slot of each row
};

// Unit geometry of this thread and its CH x W entries, read from the element's slot-ordered
// operator `reg` ([slots][blk_threads], slot-major: the loads of a wave are contiguous).
template <int N1C, int P>
__device__ __forceinline__ void reg_gather(const PcgStageArgs& a,
                                           const BlockSolve<N1C, double, kRegMaxThreads>& W,
                                           RegOp<N1C, P>& R, const double* __restrict__ reg,
                                           int t = -1) {
  constexpr int n1 = N1C, NP = N1C + 1, WM = RegOp<N1C, P>::W, CH = RegOp<N1C, P>::CH;
  if (t < 0) t = threadIdx.x;
  const int T = a.blk_threads;
#pragma unroll
  for (int i = 0; i < CH; ++i)
#pragma unroll
    for (int q = 0; q < WM; ++q) R.a[i][q] = 0.0;
  R.xoff = 0;
  R.wx = 0;
  R.ni = 0;
  if (t < n1 * W.K) {
    const int k = t / n1, ix = t - k * n1;
    const int jcv = W.jc[k], jy = jcv & 0xff, c = jcv >> 8;
    const int lox = st_lo(ix, P), wx = st_w(ix, P, N1C - 1);
    const int loy = st_lo(jy, P), wy = st_w(jy, P, N1C - 1);
    const int i0 = c * CH;
    const int ni = min(CH, wy - i0);
    R.xoff = jy * NP + lox;
    R.wx = wx;
    R.ni = ni;
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int iy = loy + i0 + i;
      R.pd[i] = (iy * n1 + ix) * W.WB + (jy - st_lo(iy, P));
#pragma unroll
      for (int q = 0; q < WM; ++q)
        if (i < ni && q < wx) R.a[i][q] = reg[(size_t)(i * WM + q) * T + t];
    }
  }
}

// y_t = (A x)_t for owner threads, as blk_apply, with the entries from registers.
template <int N1C, int P>
__device__ __forceinline__ double reg_apply(const BlockSolve<N1C, double, kRegMaxThreads>& W,
                                            const RegOp<N1C, P>& R,
                                            const double* __restrict__ x) {
  constexpr int n1 = N1C, WM = RegOp<N1C, P>::W, CH = RegOp<N1C, P>::CH;
  const int t = threadIdx.x;
  if (R.ni > 0) {
    double xs[WM];
#pragma unroll
    for (int q = 0; q < WM; ++q) xs[q] = q < R.wx ? x[R.xoff + q] : 0.0;
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < WM; ++q) acc += R.a[i][q] * xs[q];
      if (i < R.ni) W.P[R.pd[i]] = acc;
    }
  }
  __syncthreads();
  double y = 0.0;
  if (t < n1 * n1) {
    // the row's partials (one per jy of its band, WB = WM slots a row), all loads first
    const int wiy = st_w(t / n1, P, N1C - 1);
    const double* pr = W.P + t * WM;
    double pv[WM];
#pragma unroll
    for (int q = 0; q < WM; ++q) pv[q] = q < wiy ? pr[q] : 0.0;
#pragma unroll
    for (int q = 0; q < WM; ++q) y += pv[q];
  }
  return y;
}

// ---------------------------------------------------------------------------------
// Streamed family (N + 1 = 17, p = 7): on 512 threads a work unit has CH = 9 rows of
// W = 15 entries, which do not fit its registers beside the CG state, so every product
// reads them from the slot-ordered copy in memory (a wave's loads of one slot are one
// contiguous run), one row of the unit at a time.  The unit geometry is that of reg_gather.
// ---------------------------------------------------------------------------------
constexpr int kMemMaxThreads = kRegMaxThreads;
constexpr int kMemMaxCh = 16;

template <int N1C, int P>
struct MemUnit {
  static constexpr int W = 2 * P + 1 < N1C ? 2 * P + 1 : N1C;
  static constexpr int CH = blk_ch_c(N1C, P, kMemMaxThreads, kMemMaxCh);
  static_assert(CH > 0, "no chunk height fits the thread limit");
  int xoff;          // jy * NP + lo(ix): first x value of the unit
  int wx, ni;        // columns and rows of the unit (0 rows: no unit)
  int ix, jy, iy0;   // column, block row and first row of the unit
};

// Tallest work unit of a register family (the streamed family's units are not held in
// registers).
static int pcg_unit_chmax(int n1, int p) { return n1 == 17 && p == 7 ? kMemMaxCh : 8; }

template <int N1C, int P>
__device__ __forceinline__ void mem_unit(const BlockSolve<N1C, double, kMemMaxThreads>& W,
                                         const int* __restrict__ unit, MemUnit<N1C, P>& G) {
  constexpr int n1 = N1C, NP = N1C + 1, CH = MemUnit<N1C, P>::CH;
  const int t = threadIdx.x;
  G.xoff = 0;
  G.wx = 0;
  G.ni = 0;
  G.ix = G.jy = G.iy0 = 0;
  if (t < n1 * W.K) {
    const int tu = unit ? unit[t] : t;            // this thread's unit
    const int k = tu / n1, ix = tu - k * n1;
    const int jcv = W.jc[k], jy = jcv & 0xff, c = jcv >> 8;
    const int lox = st_lo(ix, P);
    const int loy = st_lo(jy, P), wy = st_w(jy, P, N1C - 1);
    const int i0 = c * CH;
    G.xoff = jy * NP + lox;
    G.wx = st_w(ix, P, N1C - 1);
    G.ni = min(CH, wy - i0);
    G.ix = ix;
    G.jy = jy;
    G.iy0 = loy + i0;
  }
}

// y_t = (A x)_t for owner threads, as reg_apply, with the entries read from `reg` (the
// element's slot-ordered copy, kMemMaxThreads threads a slot), three rows of the unit at a
// time; a thread reads only its unit's slots.
template <int N1C, int P>
__device__ __forceinline__ double mem_apply(const BlockSolve<N1C, double, kMemMaxThreads>& W,
                                            const MemUnit<N1C, P>& G,
                                            const double* __restrict__ reg,
                                            const double* __restrict__ x) {
  constexpr int n1 = N1C, WM = MemUnit<N1C, P>::W;
  const int t = threadIdx.x;
  if (G.ni > 0) {
    double xs[WM];
#pragma unroll
    for (int q = 0; q < WM; ++q) xs[q] = x[G.xoff + q];
    const double* rp = reg + t;
    constexpr int rs = kMemMaxThreads;   // slot stride (the family's block size)
    // rows in groups of three: a group's loads are in flight together
#pragma unroll 1
    for (int i0 = 0; i0 < G.ni; i0 += 3) {
      double v[3][WM];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < WM; ++q)
          v[r][q] = (i0 + r < G.ni && q < G.wx) ? rp[(r * WM + q) * rs] : 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < WM; ++q) acc += v[r][q] * xs[q];
        const int iy = G.iy0 + i0 + r;
        if (i0 + r < G.ni) W.P[(iy * n1 + G.ix) * W.WB + (G.jy - st_lo(iy, P))] = acc;
      }
      rp += 3 * WM * rs;
    }
  }
  __syncthreads();
  double y = 0.0;
  if (t < n1 * n1) {
    const int wiy = st_w(t / n1, P, N1C - 1);
    const double* pr = W.P + t * WM;
    double pv[WM];
#pragma unroll
    for (int q = 0; q < WM; ++q) pv[q] = q < wiy ? pr[q] : 0.0;
#pragma unroll
    for (int q = 0; q < WM; ++q) y += pv[q];
  }
  return y;
}

template <int N1C>
__host__ __device__ inline size_t reg_lds_doubles(const PcgGeom& g, int WB) {
  constexpr int NP = N1C + 1;
  return (size_t)g.nn * WB + 6 * NP * NP + common_doubles(g);
}

template <int N1C>
__device__ __forceinline__ void pcg2r_stage_carve(const PcgStageArgs& a,
                                                  BlockSolve<N1C, double, kRegMaxThreads>& W,
                                                  StageCommon& C) {
  extern __shared__ double shd[];
  constexpr int NP = N1C + 1, nn = N1C * N1C;
  const PcgGeom& g = a.g;
  W.K = a.blk_K;
  W.CH = a.blk_CH;
  W.WB = a.blk_WB;
  W.p = g.p;
  W.N = g.N;
  double* sp = shd;
  W.A = nullptr;
  W.P = sp;    sp += nn * W.WB;
  W.R = sp;    sp += NP * NP;
  W.U = sp;    sp += NP * NP;
  W.T = sp;    sp += NP * NP;
  W.Z = sp;    sp += NP * NP;
  W.DI = sp;   sp += NP * NP;
  W.Psi = sp;  sp += NP * NP;
  int* ip = reinterpret_cast<int*>(shd + reg_lds_doubles<N1C>(g, W.WB));
  W.boff = ip;  ip += nn;
  W.jc = ip;    ip += W.K;
  stage_carve(g, sp, ip, C);
}

template <int STAGE, int N1C, int P>
__device__ __forceinline__ void pcg2r_stage_elem(const PcgStageArgs& a, const long e,
                                                 BlockSolve<N1C, double, kRegMaxThreads>& W,
                                                 StageCommon& C) {
  constexpr int n1 = N1C, NP = N1C + 1, nn = N1C * N1C;
  const PcgGeom& g = a.g;
  const int t = threadIdx.x;
  const bool own = t < nn;
  const int pidx = own ? (t / n1) * NP + (t - (t / n1) * n1) : 0;
  const size_t per = (size_t)RegOp<N1C, P>::CH * RegOp<N1C, P>::W * a.blk_threads;
  RegOp<N1C, P> R;
  stage_prologue<STAGE>(a, e, C, []() {});
  if (own) W.U[pidx] = C.U[t];
  reg_gather(a, W, R, a.el.Sreg + e * per);
  __syncthreads();
  auto applyS = [&W, &R](const double* v) { return reg_apply(W, R, v); };
  // r = -S_K U + F_v
  {
    const double su = applyS(W.U);
    if (own) C.rv[t] -= su;
  }
  // ---- S_hat y = F_u ------------------------------------------------------------------
  double dS = 1.0;
  if (own) {
    const int kx = t % n1, ky = t / n1;
    dS = t == 0 ? C.d00 : C.kbr * C.lamr[kx] + C.kbs * C.lamr[ky];
    if (a.el.dlog && t > 0) dS *= exp((double)a.el.dlog[e * nn + t]);
    W.DI[pidx] = 1.0 / dS;
  }
  double y = C.xs0;
  int itS = blk_solve_g(W, applyS, C.red, y, own ? C.Fu[t] : 0.0, C.cw, C.wt, a.rtol, a.maxit,
                        false);
  if (itS > a.maxit && a.el.dlog) {
    if (own) {
      const int kx = t % n1, ky = t / n1;
      W.DI[pidx] = 1.0 / (t == 0 ? C.d00 : C.kbr * C.lamr[kx] + C.kbs * C.lamr[ky]);
    }
    y = C.xs0;
    itS = blk_solve_g(W, applyS, C.red, y, own ? C.Fu[t] : 0.0, C.cw, C.wt, a.rtol, a.maxit,
                      false);
  }
  __syncthreads();
  // ---- M_J z = r --------------------------------------------------------------------
  int itM;
  double z;
  if (own) W.DI[pidx] = 1.0 / C.area;
  if (a.mapped) {
    reg_gather(a, W, R, a.el.Mreg + e * per);
    z = C.xm0;
    itM = blk_solve_g(W, applyS, C.red, z, own ? C.rv[t] : 0.0, 0.0, 0.0, a.rtol, a.maxit, false,
                      a.el.msc != nullptr, C.ms);
  } else {
    // Cartesian: the preconditioner is the exact inverse of M_J
    double bb1[1] = {own ? C.rv[t] * C.rv[t] : 0.0};
    if (own) W.R[pidx] = C.rv[t];
    block_sum<1>(bb1, C.red, nn);
    blk_pinv(W, W.R, W.U);
    z = own ? W.U[pidx] : 0.0;
    itM = bb1[0] > 0.0 ? 1 : 0;
  }
  __syncthreads();
  stage_epilogue<STAGE>(a, e, C, own ? y : 0.0, own ? z : 0.0, itS, itM);
}

template <int N1C>
__device__ __forceinline__ void pcg2m_stage_carve(const PcgStageArgs& a, BlockSolve<N1C, float>& W,
                                                  StageCommon& C) {
  extern __shared__ double shd[];
  constexpr int NP = N1C + 1, nn = N1C * N1C;
  const PcgGeom& g = a.g;
  W.K = a.blk_K;
  W.CH = a.blk_CH;
  W.WB = a.blk_WB;
  W.p = g.p;
  W.N = g.N;
  double* sp = shd;
  W.A = reinterpret_cast<float*>(sp);  sp += mix_a_doubles<N1C>(a.nnz_full);
  double* preg = sp;
  W.P = sp;    sp += mix_p_doubles<N1C>(g, W.WB);
  W.R = sp;    sp += NP * NP;
  W.U = sp;    sp += NP * NP;
  W.T = sp;    sp += NP * NP;
  W.Z = sp;    sp += NP * NP;
  W.DI = sp;   sp += NP * NP;
  W.Psi = sp;  sp += NP * NP;
  int* ip = reinterpret_cast<int*>(shd + mix_lds_doubles<N1C>(g, a.nnz_full, W.WB));
  W.boff = ip;  ip += nn;
  W.jc = ip;    ip += W.K;
  stage_carve_small(g, sp, ip, preg, C);
}

template <int N1C, typename TA, int MT>
__device__ __forceinline__ void blk_load_tables(const PcgStageArgs& a,
                                                const BlockSolve<N1C, TA, MT>& W,
                                                const StageCommon& C) {
  constexpr int NP = N1C + 1, nn = N1C * N1C;
  const int t = threadIdx.x;
  int* boff = const_cast<int*>(W.boff);
  int* jc = const_cast<int*>(W.jc);
  for (int i = t; i < nn; i += blockDim.x) boff[i] = a.blk_off[i];
  for (int i = t; i < W.K; i += blockDim.x) jc[i] = a.blk_jc[i];
  for (int i = t; i < 5 * NP * NP; i += blockDim.x) W.R[i] = 0.0;   // R U T Z DI (padding)
  stage_load_tables(a.g, W.Psi, NP, C);
}

// Copy an FP32 block-layout operator (nnz entries) from global memory into LDS.
__device__ __forceinline__ void blk_load32(int nnz, float* A, const float* __restrict__ src) {
  const int step = blockDim.x;
  for (int i0 = threadIdx.x; i0 < nnz; i0 += 8 * step) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = i0 + k * step;
      v[k] = i < nnz ? src[i] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = i0 + k * step;
      if (i < nnz) A[i] = v[k];
    }
  }
}

template <int STAGE, int N1C>
__device__ __forceinline__ void pcg2m_stage_elem(const PcgStageArgs& a, const long e,
                                                 BlockSolve<N1C, float>& W, StageCommon& C) {
  constexpr int n1 = N1C, NP = N1C + 1, nn = N1C * N1C;
  const int t = threadIdx.x;
  const bool own = t < nn;
  const int pidx = own ? (t / n1) * NP + (t - (t / n1) * n1) : 0;
  const int nnz = a.nnz_full;
  float* const Aop = W.A;
  const float* const Shi = a.el.Shi + e * nnz;
  const float* const Slo = a.el.Slo + e * nnz;
  stage_prologue<STAGE>(a, e, C, [Aop, Shi, nnz]() { blk_load32(nnz, Aop, Shi); });
  // r = -S_K U + F_v in FP64
  if (own) W.U[pidx] = C.U[t];
  __syncthreads();
  {
    const double su = blk_apply64(W, Slo, W.U);
    if (own) C.rv[t] -= su;
  }
  // ---- S_hat y = F_u ------------------------------------------------------------------
  double dS = 1.0;
  if (own) {
    const int kx = t % n1, ky = t / n1;
    dS = t == 0 ? C.d00 : C.kbr * C.lamr[kx] + C.kbs * C.lamr[ky];
    if (a.el.dlog && t > 0) dS *= exp((double)a.el.dlog[e * nn + t]);
    W.DI[pidx] = 1.0 / dS;
  }
  double y = C.xs0;
  int swS = 0, swM = 0;
  int itS = blk_solve_mixed(W, Slo, C.red, y, own ? C.Fu[t] : 0.0, C.cw, C.wt, a.rtol, a.maxit,
                            &swS);
  if (itS > a.maxit && a.el.dlog) {
    if (own) {
      const int kx = t % n1, ky = t / n1;
      W.DI[pidx] = 1.0 / (t == 0 ? C.d00 : C.kbr * C.lamr[kx] + C.kbs * C.lamr[ky]);
    }
    y = C.xs0;
    itS = blk_solve_mixed(W, Slo, C.red, y, own ? C.Fu[t] : 0.0, C.cw, C.wt, a.rtol, a.maxit,
                          &swS);
  }
  __syncthreads();
  // ---- M_J z = r --------------------------------------------------------------------
  int itM;
  double z;
  if (own) W.DI[pidx] = 1.0 / C.area;
  if (a.mapped) {
    blk_load32(nnz, W.A, a.el.Mhi + e * nnz);
    z = C.xm0;
    itM = blk_solve_mixed(W, a.el.Mlo + e * nnz, C.red, z, own ? C.rv[t] : 0.0, 0.0, 0.0, a.rtol,
                          a.maxit, &swM, a.el.msc != nullptr, C.ms);
  } else {
    // Cartesian: the preconditioner is the exact inverse of M_J (FP64 transforms)
    double bb1[1] = {own ? C.rv[t] * C.rv[t] : 0.0};
    if (own) W.R[pidx] = C.rv[t];
    block_sum<1>(bb1, C.red, nn);
    blk_pinv(W, W.R, W.U);
    z = own ? W.U[pidx] : 0.0;
    itM = bb1[0] > 0.0 ? 1 : 0;
  }
  __syncthreads();
  stage_epilogue<STAGE>(a, e, C, own ? y : 0.0, own ? z : 0.0, itS, itM, swS, swM);
}


// Grouped, persistent form over the elements of several problems (each with its own
// geometry and LDS layout, all fitting the launch's LDS size and block size).  Problem i
// owns elements [el_start[i], el_start[i+1]); block b takes b, b + gridDim.x, ...
// N1C > 0: every member uses the column-block layout with N + 1 = N1C; N1C = 0: every
// member uses the row layout.
template <int STAGE, int KEY>
__global__ __launch_bounds__((KEY & 64) ? kRegMaxThreads : KEY > 0 ? kBlkMaxThreads : 1024)
void k_pcg_stage_group(
    const PcgStageArgs* __restrict__ args, const long* __restrict__ el_start, int nprob) {
  constexpr int N1C = KEY & 31;            // N + 1 of the column-block families
  constexpr bool MIX = (KEY & 32) != 0;    // FP32 operator + FP64 refinement
  constexpr bool REG = (KEY & 64) != 0;    // FP64 operator in registers, degree KEY >> 7
  constexpr int PK = KEY >> 7;
  const long total = el_start[nprob];
  int pi = 0, cur = -1;
  for (long b = blockIdx.x; b < total; b += gridDim.x) {
    while (pi + 1 < nprob && b >= el_start[pi + 1]) ++pi;
    const PcgStageArgs& a = args[pi];
    StageCommon C;
    if constexpr (KEY == 0) {
      PcgShared W;
      pcg_stage_carve(a, W, C);
      if (pi != cur) {
        pcg_stage_load_tables(a, W, C);
        cur = pi;
      }
      pcg_stage_elem<STAGE>(a, b - el_start[pi], W, C);
    } else if constexpr (MIX) {
      BlockSolve<N1C, float> W;
      pcg2m_stage_carve<N1C>(a, W, C);
      if (pi != cur) {                     // a new problem: its tables
        blk_load_tables<N1C, float>(a, W, C);
        cur = pi;
      }
      pcg2m_stage_elem<STAGE, N1C>(a, b - el_start[pi], W, C);
    } else if constexpr (REG) {
      BlockSolve<N1C, double, kRegMaxThreads> W;
      pcg2r_stage_carve<N1C>(a, W, C);
      if (pi != cur) {
        blk_load_tables<N1C, double>(a, W, C);
        cur = pi;
      }
      pcg2r_stage_elem<STAGE, N1C, PK>(a, b - el_start[pi], W, C);
    } else {
      BlockSolve<N1C> W;
      pcg2_stage_carve<N1C>(a, W, C);
      if (pi != cur) {
        blk_load_tables<N1C, double>(a, W, C);
        cur = pi;
      }
      pcg2_stage_elem<STAGE, N1C>(a, b - el_start[pi], W, C);
    }
    __syncthreads();   // the next element reuses the LDS
  }
}

// ---------------------------------------------------------------------------------
// Split stage of the register-operator families (FP64).  The fused stage kernel pays, one
// element per CU at a time, the latency of the element's loads, face fluxes, lifts and
// traces inside its persistent loop.  Here those parts run as streaming kernels with many
// elements resident per CU, and the persistent kernels hold only the element solves:
//   k_pcg_lift<STAGE>     F_u, F_v from the traces (Sec. 2.2.1)              -> Fu, Fv
//   k_pcg_solve<0, ...>   r = F_v - S_K U (-> Fv) and S_hat y = F_u (-> xS); on Cartesian
//                         elements also M_J z = r by the exact inverse (-> xM)
//   k_pcg_solve<1, ...>   M_J z = r on mapped elements (-> xM)
//   k_pcg_update<STAGE>   the RK update from (y, z) and the traces of the new state
// The arithmetic of every part is that of the fused kernel, so both give the same state.
// ---------------------------------------------------------------------------------
__host__ __device__ inline size_t split_lds_doubles(const PcgGeom& g) {
  return common_doubles(g);
}
__host__ __device__ inline size_t split_lds_bytes(const PcgGeom& g) {
  return split_lds_doubles(g) * sizeof(double) + common_ints(g) * sizeof(int);
}

// Elements of a split launch: those of one problem (GRP = false: args[0].nel of them), or
// those of the n members of a group one after another (GRP: member k owns the elements
// start[k] .. start[k + 1] - 1, start[n] is the total).  The members of a group share N, p
// and the block layout, so one LDS layout serves all of them.  The single-problem kernels
// are separate instances, so that they carry no member bookkeeping.
template <bool GRP>
struct ElemRange {
  const long* start;
  int n;
  __device__ __forceinline__ long total(const PcgStageArgs* args) const {
    if constexpr (GRP) return start[n];
    return args[0].nel;
  }
  // member of element b, searched onward from member k (the elements of a workgroup come
  // in increasing order)
  __device__ __forceinline__ int member(long b, int k) const {
    if constexpr (GRP) {
      while (k + 1 < n && b >= start[k + 1]) ++k;
      return k;
    }
    return 0;
  }
  __device__ __forceinline__ long first(int k) const {
    if constexpr (GRP) return start[k];
    return 0;
  }
};

// LDS of the streaming kernels: the element-independent tables (loaded again when a
// workgroup moves on to another member) and the element's face data (the layout of
// stage_carve).
__device__ __forceinline__ void split_carve(const PcgGeom& g, StageCommon& C) {
  extern __shared__ double shd[];
  double* sp = shd;
  int* ip = reinterpret_cast<int*>(shd + split_lds_doubles(g));
  stage_carve(g, sp, ip, C);
}

template <int STAGE, bool GRP>
__global__ __launch_bounds__(512) void k_pcg_lift(const PcgStageArgs* __restrict__ args,
                                                  const long* __restrict__ el_start, int nprob) {
  const ElemRange<GRP> rg{el_start, nprob};
  const int t = threadIdx.x, nn = args[0].g.nn;
  StageCommon C;
  split_carve(args[0].g, C);
  if constexpr (!GRP) stage_load_tables(args[0].g, nullptr, 0, C);
  const long total = rg.total(args);
  int k = 0;
  [[maybe_unused]] int cur = -1;
  for (long b = blockIdx.x; b < total; b += gridDim.x) {
    k = rg.member(b, k);
    const PcgStageArgs& a = args[k];
    // (the previous element ended with a barrier; the prologue's first one publishes)
    if constexpr (GRP) {
      if (k != cur) {
        stage_load_tables(a.g, nullptr, 0, C);
        cur = k;
      }
    }
    const long e = b - rg.first(k);
    stage_prologue<STAGE, false>(a, e, C, []() {});
    if (t < nn) {
      a.Fu[e * nn + t] = C.Fu[t];
      a.Fv[e * nn + t] = C.rv[t];
    }
    __syncthreads();
  }
}

template <int STAGE, bool GRP>
__global__ __launch_bounds__(512) void k_pcg_update(const PcgStageArgs* __restrict__ args,
                                                    const long* __restrict__ el_start, int nprob) {
  const ElemRange<GRP> rg{el_start, nprob};
  const int t = threadIdx.x, nn = args[0].g.nn;
  StageCommon C;
  split_carve(args[0].g, C);
  double* fcl = const_cast<double*>(C.T.fc);
  if constexpr (!GRP) stage_load_tables(args[0].g, nullptr, 0, C);
  const long total = rg.total(args);
  int k = 0;
  [[maybe_unused]] int cur = -1;
  for (long b = blockIdx.x; b < total; b += gridDim.x) {
    k = rg.member(b, k);
    const PcgStageArgs& a = args[k];
    const PcgGeom& g = a.g;
    if constexpr (GRP) {
      if (k != cur) {
        stage_load_tables(g, nullptr, 0, C);
        cur = k;
      }
    }
    const long e = b - rg.first(k);
    double y = 0.0, z = 0.0;
    C.ub = C.vb = C.yu = C.yv = 0.0;
    if (t < nn) {
      const long gi = e * nn + t;
      C.ub = a.in_u[gi];
      C.vb = a.in_v[gi];
      if (STAGE > 1) {
        C.yu = a.aux_u[gi];
        C.yv = a.aux_v[gi];
      }
      y = a.xS[gi];
      z = a.xM[gi];
    }
    const double* fcg = a.el.face + e * 4 * g.nq * 3;
    for (int i = t; i < 4 * g.nq * 3; i += blockDim.x) fcl[i] = fcg[i];
    // (the epilogue's first barrier publishes the face data and the tables)
    stage_epilogue<STAGE, true>(a, e, C, y, z, 0, 0);
    __syncthreads();
  }
}

// doubles and ints of the solve kernels' LDS
template <int N1C>
__host__ __device__ constexpr size_t solve_lds_doubles(int WB) {
  return (size_t)N1C * N1C * WB + 6 * (N1C + 1) * (N1C + 1) + 64 + (N1C + 1);
}

__device__ __forceinline__ void split_count(const PcgStageArgs& a, long e, int slot, int it) {
  int* its = a.its + e * kItsPer;
  its[slot] += it > a.maxit ? a.maxit : it;
  if (it > its[slot + 2]) its[slot + 2] = it;
  if (it > a.maxit) atomicMin(a.fail, (int)e);
}

// MEM: the streamed family (operator entries read from memory in every product).
template <int OP, int N1C, int P, bool GRP, bool MEM = false>
__global__ __launch_bounds__(MEM ? kMemMaxThreads : kRegMaxThreads)
void k_pcg_solve(const PcgStageArgs* __restrict__ args, const long* __restrict__ el_start,
                 int nprob) {
  extern __shared__ double shd[];
  constexpr int n1 = N1C, NP = N1C + 1, nn = N1C * N1C;
  constexpr int MT = MEM ? kMemMaxThreads : kRegMaxThreads;
  using Unit = std::conditional_t<MEM, MemUnit<N1C, P>, RegOp<N1C, P>>;
  const ElemRange<GRP> rg{el_start, nprob};
  const PcgStageArgs& a0 = args[0];
  const int t = threadIdx.x;
  const bool own = t < nn;
  const int pidx = own ? (t / n1) * NP + (t - (t / n1) * n1) : 0;
  BlockSolve<N1C, double, MT> W;
  W.A = nullptr;
  W.K = a0.blk_K;
  W.CH = a0.blk_CH;
  W.WB = a0.blk_WB;
  W.p = a0.g.p;
  W.N = a0.g.N;
  double* sp = shd;
  W.P = sp;    sp += nn * W.WB;
  W.R = sp;    sp += NP * NP;
  W.U = sp;    sp += NP * NP;
  W.T = sp;    sp += NP * NP;
  W.Z = sp;    sp += NP * NP;
  W.DI = sp;   sp += NP * NP;
  W.Psi = sp;  sp += NP * NP;
  // the early stop test (its own slots) where a product costs more than a reduction: the
  // streamed operators, and the M_J solves (few iterations, so the saved product weighs more)
  constexpr bool EARLY = MEM || OP == 1;
  double* red = sp;  sp += EARLY ? 80 : 64;
  double* lamr = sp; sp += NP;
  int* jc = reinterpret_cast<int*>(sp);
  W.boff = nullptr;
  W.jc = jc;
  for (int i = t; i < W.K; i += blockDim.x) jc[i] = a0.blk_jc[i];
  for (int i = t; i < 5 * NP * NP; i += blockDim.x) W.R[i] = 0.0;   // R U T Z DI (padding)
  // the eigenbasis tables of member k (a group reloads them when a workgroup changes member)
  auto load_tables = [&](const PcgGeom& g) {
    for (int i = t; i < NP * NP; i += blockDim.x) {
      const int r = i / NP, q = i - (i / NP) * NP;
      W.Psi[i] = (r < n1 && q < n1) ? g.Psi[r * n1 + q] : 0.0;
    }
    for (int i = t; i < n1; i += blockDim.x) lamr[i] = g.lamr[i];
  };
  if constexpr (!GRP) load_tables(a0.g);
  __syncthreads();
  const int T = a0.blk_threads;
  const size_t per = (size_t)Unit::CH * Unit::W * T;
  Unit R;
  const double* opb = nullptr;   // MEM: the element's slot-ordered operator
  if constexpr (MEM) mem_unit(W, a0.blk_unit, R);
  auto apply = [&W, &R, &opb](const double* v) {
    if constexpr (MEM) return mem_apply(W, R, opb, v);
    else return reg_apply(W, R, v);
  };
  // the element's operator: into the registers, or where the products read it
  auto take = [&](const PcgStageArgs& a, const double* op) {
    if constexpr (MEM) opb = op;
    else reg_gather(a, W, R, op);
  };
  const long total = rg.total(args);
  int k = 0;
  [[maybe_unused]] int cur = -1;
  for (long b = blockIdx.x; b < total; b += gridDim.x) {
    k = rg.member(b, k);
    const PcgStageArgs& a = args[k];
    const PcgGeom& g = a.g;
    if constexpr (GRP) {
      if (k != cur) {   // (the previous element ended with a barrier)
        load_tables(g);
        cur = k;
        __syncthreads();
      }
    }
    const long e = b - rg.first(k);
    const long gi = e * nn + t;
    const double* scp = a.el.sc + e * 8;
    if constexpr (OP == 0) {
      double ub = 0.0, fu = 0.0, fv = 0.0, x0 = 0.0, wt = 0.0, dl = 0.0;
      if (own) {
        ub = a.in_u[gi];
        fu = a.Fu[gi];
        fv = a.Fv[gi];
        x0 = a.xS[gi];
        wt = a.el.w[gi];
        if (a.el.dlog) dl = (double)a.el.dlog[gi];
      }
      const double cw = scp[0], kbr = scp[1], kbs = scp[2], d00 = scp[3], area = scp[4];
      if (own) W.U[pidx] = ub;
      take(a, a.el.Sreg + e * per);
      __syncthreads();
      const double su = apply(W.U);
      const double rv = own ? fv - su : 0.0;      // r = -S_K U + F_v
      if (a.mapped) {
        if (own) a.Fv[gi] = rv;
      } else {
        // Cartesian: the preconditioner is the exact inverse of M_J
        double bb1[1] = {rv * rv};
        if (own) {
          W.DI[pidx] = 1.0 / area;
          W.R[pidx] = rv;
        }
        block_sum<1>(bb1, red, nn);
        blk_pinv(W, W.R, W.U);
        if (own) a.xM[gi] = W.U[pidx];
        if (t == 0) split_count(a, e, 1, bb1[0] > 0.0 ? 1 : 0);
      }
      // ---- S_hat y = F_u --------------------------------------------------------------
      if (own) {
        const int kx = t % n1, ky = t / n1;
        double dS = t == 0 ? d00 : kbr * lamr[kx] + kbs * lamr[ky];
        if (a.el.dlog && t > 0) dS *= exp(dl);
        W.DI[pidx] = 1.0 / dS;
      }
      double y = x0;
      using App = decltype(apply)&;
      int itS = blk_solve_g<N1C, double, MT, App, EARLY>(W, apply, red, y, own ? fu : 0.0, cw, wt,
                                                         a.rtol, a.maxit, false);
      if (itS > a.maxit && a.el.dlog) {
        if (own) {
          const int kx = t % n1, ky = t / n1;
          W.DI[pidx] = 1.0 / (t == 0 ? d00 : kbr * lamr[kx] + kbs * lamr[ky]);
        }
        y = x0;
        itS = blk_solve_g<N1C, double, MT, App, EARLY>(W, apply, red, y, own ? fu : 0.0, cw, wt,
                                                       a.rtol, a.maxit, false);
      }
      if (own) a.xS[gi] = y;
      if (t == 0) split_count(a, e, 0, itS);
    } else {
      // ---- M_J z = r (mapped elements) ------------------------------------------------
      double rv = 0.0, z = 0.0, ms = 1.0;
      if (own) {
        rv = a.Fv[gi];
        z = a.xM[gi];
        if (a.el.msc) ms = a.el.msc[gi];
        W.DI[pidx] = 1.0 / scp[4];
      }
      take(a, a.el.Mreg + e * per);
      const int itM = blk_solve_g<N1C, double, MT, decltype(apply)&, EARLY>(W, apply, red, z, own ? rv : 0.0, 0.0, 0.0, a.rtol, a.maxit,
                                  false, a.el.msc != nullptr, ms);
      if (own) a.xM[gi] = z;
      if (t == 0) split_count(a, e, 1, itM);
    }
    __syncthreads();   // the next element reuses the LDS
  }
}

// ---------------------------------------------------------------------------------
// Solve kernels with the CG vectors on one wave (N + 1 <= 16).  In the kernels above every
// owner thread holds one node, so each iteration needs four workgroup barriers (publish r,
// preconditioner, operator partials, reduction).  Here wave 0 holds the whole vectors of
// the solve in the operand layout of the preconditioner's matrix-core chain (lane
// l = 16 g + c owns the nodes (ix, iy) = (c, 4 s + g), s = 0..3), so the preconditioner
// reads and writes registers, the dot products are wave reductions (DPP, no LDS), and the
// only workgroup traffic of an iteration is the operator product: wave 0 publishes u in LDS,
// every work unit forms its partial row sums, wave 0 adds them.  Two barriers per
// iteration; the recurrence and its arithmetic are those of blk_solve_g.
// ---------------------------------------------------------------------------------
template <int N1C>
struct W0Lane {
  int g, c;
  __device__ __forceinline__ bool ok(int s) const { return c < N1C && 4 * s + g < N1C; }
  // node (c, 4 s + g): its index iy * (N + 1) + ix, and on the padded grid of the LDS vectors
  __device__ __forceinline__ int node(int s) const { return (4 * s + g) * N1C + c; }
  __device__ __forceinline__ int pad(int s) const { return (4 * s + g) * (N1C + 1) + c; }
};

template <int N1C>
__device__ __forceinline__ W0Lane<N1C> w0_lane() {
  W0Lane<N1C> L;
  const int t = threadIdx.x & 63;
  L.g = t >> 4;
  L.c = t & 15;
  return L;
}

// Partial row sums of the operator product of every work unit (no barrier).
template <int N1C, int P>
__device__ __forceinline__ void reg_units(const BlockSolve<N1C, double, kRegMaxThreads>& W,
                                          const RegOp<N1C, P>& R, const double* __restrict__ x) {
  constexpr int WM = RegOp<N1C, P>::W, CH = RegOp<N1C, P>::CH;
  if (R.ni > 0) {
    double xs[WM];
#pragma unroll
    for (int q = 0; q < WM; ++q) xs[q] = q < R.wx ? x[R.xoff + q] : 0.0;
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < WM; ++q) acc += R.a[i][q] * xs[q];
      if (i < R.ni) W.P[R.pd[i]] = acc;
    }
  }
}

// Wave 0: the rows of its nodes, each the sum of its partials in slot order.
template <int N1C, int P>
__device__ __forceinline__ void w0_rows(const BlockSolve<N1C, double, kRegMaxThreads>& W,
                                        const W0Lane<N1C>& L, double (&y)[4]) {
  constexpr int WM = RegOp<N1C, P>::W;
  double pv[4][WM];                      // all loads first
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int wiy = L.ok(s) ? st_w(4 * s + L.g, P, N1C - 1) : 0;
    const double* pr = W.P + L.node(s) * WM;
#pragma unroll
    for (int q = 0; q < WM; ++q) pv[s][q] = q < wiy ? pr[q] : 0.0;
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < WM; ++q) a += pv[s][q];
    y[s] = a;
  }
}

// Wave 0: out = Psi_2 diag(di) Psi_2^T r on registers (the chain of blk_pinv_mfma).
__device__ __forceinline__ void w0_pinv(const double (&psk)[4], const double (&pks)[4],
                                        const double (&di)[4], const double (&r)[4],
                                        double (&out)[4]) {
  pcg_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(r[s], psk[s], acc, 0, 0, 0);
  pcg_d4 acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 4; ++s)
    acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[s], psk[s], acc2, 0, 0, 0);
#pragma unroll
  for (int s = 0; s < 4; ++s) acc2[s] *= di[s];
  pcg_d4 acc3 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 4; ++s)
    acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(acc2[s], pks[s], acc3, 0, 0, 0);
  pcg_d4 acc4 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 4; ++s)
    acc4 = __builtin_amdgcn_mfma_f64_16x16x4f64(acc3[s], pks[s], acc4, 0, 0, 0);
#pragma unroll
  for (int s = 0; s < 4; ++s) out[s] = acc4[s];
}

struct W0Pre {
  double psk[4], pks[4];   // Psi[4 s + g][c], Psi[c][4 s + g] (0 outside)
  // FP32 chain: Psi[4 s + g][c], Psi[4 g + s][c], Psi[c][4 g + s] (0 outside)
  float psk1[4], psk2[4], pks2[4];
};

typedef float pcg_f4 __attribute__((ext_vector_type(4)));

// Node of the FP32 chain's output register s on lane (g, c): (c, 4 g + s).
template <int N1C>
__device__ __forceinline__ bool w0_ok2(const W0Lane<N1C>& L, int s) {
  return L.c < N1C && 4 * L.g + s < N1C;
}

// Wave 0: u = sc P^-1 (sc r) (sc = 1 when not scaled), written to W.U as well.  P32: the
// four transforms on the FP32 matrix cores (v_mfma_f32_16x16x4f32), whose output register r
// holds row 4 g + r (the FP64 instruction's holds 4 r + g): the products after the first
// take the K index 4 g + s, di comes in that layout (node (c, 4 g + s) in di[s]), and the
// result reaches the vector layout through U (LDS, same wave).  The recurrence, the
// operator products and the residuals stay FP64.
template <int N1C, bool P32 = false>
__device__ __forceinline__ void w0_precond(const BlockSolve<N1C, double, kRegMaxThreads>& W,
                                           const W0Lane<N1C>& L, const W0Pre& Pp,
                                           const double (&di)[4], const double (&sc)[4],
                                           bool scaled, const double (&r)[4], double (&u)[4]) {
  if constexpr (P32) {
    float rs[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) rs[s] = L.ok(s) ? (float)(scaled ? r[s] * sc[s] : r[s]) : 0.f;
    pcg_f4 a1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(rs[s], Pp.psk1[s], a1, 0, 0, 0);
    pcg_f4 a2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      a2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[s], Pp.psk2[s], a2, 0, 0, 0);
#pragma unroll
    for (int s = 0; s < 4; ++s) a2[s] *= (float)di[s];
    pcg_f4 a3 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      a3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[s], Pp.pks2[s], a3, 0, 0, 0);
    pcg_f4 a4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      a4 = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[s], Pp.pks2[s], a4, 0, 0, 0);
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (w0_ok2(L, s)) W.U[(4 * L.g + s) * (N1C + 1) + L.c] = (double)a4[s];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      u[s] = L.ok(s) ? W.U[L.pad(s)] : 0.0;
      if (scaled) {
        u[s] *= sc[s];
        if (L.ok(s)) W.U[L.pad(s)] = u[s];
      }
    }
  } else {
    double rs[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) rs[s] = L.ok(s) ? (scaled ? r[s] * sc[s] : r[s]) : 0.0;
    w0_pinv(Pp.psk, Pp.pks, di, rs, u);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (scaled) u[s] *= sc[s];
      if (L.ok(s)) W.U[L.pad(s)] = u[s];
    }
  }
}

__device__ __forceinline__ double w0_dot(const double (&a)[4], const double (&b)[4]) {
  double v = 0.0;
#pragma unroll
  for (int s = 0; s < 4; ++s) v += a[s] * b[s];
  return wave_sum(v);
}

// s_waitcnt immediate of gfx9-family targets that waits for vmcnt(0) only
// (vmcnt = bits 3:0 and 15:14, expcnt = bits 6:4, lgkmcnt = bits 11:8).
constexpr int kWaitVm0 = 0x0F70;

// Control word of the product rounds (LDS), written by wave 0 lane 0 before the first
// barrier of a round.
constexpr int kRoundProduct = 0, kRoundEnd = 1;

// Wave 0: one operator product.  U holds the input (written by wave 0 before the call); the
// work-unit waves form the partials between the two barriers; wave 0 then adds its rows.
template <int N1C, int P>
__device__ __forceinline__ void w0_product(const BlockSolve<N1C, double, kRegMaxThreads>& W,
                                           const W0Lane<N1C>& L, int* ctl, double (&y)[4]) {
  if (threadIdx.x == 0) *ctl = kRoundProduct;
  __syncthreads();
  __syncthreads();
  w0_rows<N1C, P>(W, L, y);
}

// Wave 0: end of an element for the work-unit waves (they then gather the next operator).
__device__ __forceinline__ void w0_end(int* ctl) {
  if (threadIdx.x == 0) *ctl = kRoundEnd;
  __syncthreads();
  __syncthreads();
}

// Work-unit waves: the product rounds of one element, until wave 0 ends it.
template <int N1C, int P>
__device__ __forceinline__ void unit_rounds(const BlockSolve<N1C, double, kRegMaxThreads>& W,
                                            const RegOp<N1C, P>& R, const int* ctl) {
  for (;;) {
    __syncthreads();
    const int cmd = __builtin_amdgcn_readfirstlane(*ctl);   // one value per wave: a scalar branch
    if (cmd == kRoundProduct) reg_units(W, R, W.U);
    __syncthreads();
    if (cmd == kRoundEnd) return;
  }
}

// Wave 0: PCG on (A + cw w w^T) x = b with the single-reduction recurrence of blk_solve_g;
// x, b, w, di, sc are wave 0's (entries outside the element 0), x is the warm start on entry
// and the solution on return; returns the iteration count (maxit + 1: no convergence).
template <int N1C, int P, bool P32 = false>
__device__ int w0_solve(const BlockSolve<N1C, double, kRegMaxThreads>& W, const W0Lane<N1C>& L,
                        const W0Pre& Pp, int* ctl, double (&x)[4], const double (&b)[4],
                        const double (&w)[4], const double (&di)[4], const double (&sc)[4],
                        bool scaled, double cw, double rtol, int maxit) {
  double r[4], u[4], q[4], pv[4], sv[4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
    if (L.ok(s)) W.U[L.pad(s)] = x[s];
  w0_product<N1C, P>(W, L, ctl, q);
  const double wx = w0_dot(w, x), bb = w0_dot(b, b);
  if (bb == 0.0) {
#pragma unroll
    for (int s = 0; s < 4; ++s) x[s] = 0.0;
    return 0;
  }
  const double tol2 = rtol * rtol * bb;
#pragma unroll
  for (int s = 0; s < 4; ++s) r[s] = L.ok(s) ? b[s] - q[s] - cw * wx * w[s] : 0.0;
  // The stop test reads |r|^2 as soon as r is updated (a wave reduction, no barrier), so a
  // converged solve skips the preconditioning and the product that the single-reduction
  // form would otherwise spend before the test; the counts and iterates are unchanged.
  if (w0_dot(r, r) <= tol2) return 0;
  w0_precond<N1C, P32>(W, L, Pp, di, sc, scaled, r, u);
  // The scalars are kept as 1/gamma and 1/alpha, so that an iteration needs the two
  // reciprocals 1/ru and 1/(dn - beta ru / alpha), which do not depend on each other,
  // instead of three divisions in sequence.
  double alpha = 0.0, igam = 0.0, ialpha = 0.0;
  for (int it = 0;; ++it) {
    w0_product<N1C, P>(W, L, ctl, q);
    const double ru = w0_dot(r, u), qu = w0_dot(q, u), wu = w0_dot(w, u);
    const double dn = qu + cw * wu * wu;
    const double iru = 1.0 / ru;
    if (it == 0) {
      ialpha = dn * iru;
      alpha = ru / dn;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        pv[s] = u[s];
        sv[s] = q[s] + cw * wu * w[s];
      }
    } else {
      const double beta = ru * igam;
      const double den = dn - beta * ru * ialpha;
      alpha = ru / den;
      ialpha = den * iru;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        pv[s] = u[s] + beta * pv[s];
        sv[s] = (q[s] + cw * wu * w[s]) + beta * sv[s];
      }
    }
    igam = iru;
    if (it == maxit) return maxit + 1;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      x[s] += alpha * pv[s];
      r[s] -= alpha * sv[s];
    }
    if (w0_dot(r, r) <= tol2) return it + 1;
    w0_precond<N1C, P32>(W, L, Pp, di, sc, scaled, r, u);
  }
}

// Wave 0 of the solve kernels: everything but the products.
template <int OP, int N1C, int P, bool P32 = false>
__device__ __forceinline__ void w0_element(const PcgStageArgs& a, long e,
                                           const BlockSolve<N1C, double, kRegMaxThreads>& W,
                                           const W0Lane<N1C>& L, const W0Pre& Pp, int* ctl) {
  constexpr int nn = N1C * N1C;
  const PcgGeom& g = a.g;
  const int t = threadIdx.x;
  const long e0 = e * nn;
  const double* scp = a.el.sc + e * 8;
  const double one[4] = {1.0, 1.0, 1.0, 1.0};
  if constexpr (OP == 0) {
    double ub[4] = {}, fu[4] = {}, fv[4] = {}, x0[4] = {}, wt[4] = {}, dl[4] = {};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (L.ok(s)) {
        const long gi = e0 + L.node(s);
        ub[s] = a.in_u[gi];
        fu[s] = a.Fu[gi];
        fv[s] = a.Fv[gi];
        x0[s] = a.xS[gi];
        wt[s] = a.el.w[gi];
        if (a.el.dlog) dl[s] = a.el.dscale[gi];
      }
    const double cw = scp[0], kbr = scp[1], kbs = scp[2], d00 = scp[3], area = scp[4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (L.ok(s)) W.U[L.pad(s)] = ub[s];
    double su[4], rv[4];
    w0_product<N1C, P>(W, L, ctl, su);
#pragma unroll
    for (int s = 0; s < 4; ++s) rv[s] = L.ok(s) ? fv[s] - su[s] : 0.0;   // r = -S_K U + F_v
    if (a.mapped) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (L.ok(s)) a.Fv[e0 + L.node(s)] = rv[s];
    } else {
      // Cartesian: the preconditioner is the exact inverse of M_J
      double dm[4], z[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) dm[s] = L.ok(s) ? 1.0 / area : 0.0;
      const double bb = w0_dot(rv, rv);
      w0_pinv(Pp.psk, Pp.pks, dm, rv, z);
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (L.ok(s)) a.xM[e0 + L.node(s)] = z[s];
      if (t == 0) split_count(a, e, 1, bb > 0.0 ? 1 : 0);
    }
    // ---- S_hat y = F_u ----------------------------------------------------------------
    // pass 1 with the plain preconditioner when the corrected one did not converge
    double y[4];
    int itS = 0;
    for (int pass = 0; pass < 2; ++pass) {
      double di[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        // node of di[s]: (c, 4 s + g), or (c, 4 g + s) for the FP32 chain
        const int iy = P32 ? 4 * L.g + s : 4 * s + L.g;
        const bool ok = P32 ? w0_ok2(L, s) : L.ok(s);
        double dS = 1.0;
        if (ok) {
          dS = (L.c == 0 && iy == 0) ? d00 : kbr * g.lamr[L.c] + kbs * g.lamr[iy];
          if (pass == 0 && a.el.dlog && !(L.c == 0 && iy == 0))
            dS *= P32 ? a.el.dscale[e0 + iy * N1C + L.c] : dl[s];
        }
        di[s] = ok ? 1.0 / dS : 0.0;
        y[s] = x0[s];
      }
      itS = w0_solve<N1C, P, P32>(W, L, Pp, ctl, y, fu, wt, di, one, false, cw, a.rtol, a.maxit);
      if (!(a.el.dlog && itS > a.maxit)) break;
    }
    w0_end(ctl);
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (L.ok(s)) a.xS[e0 + L.node(s)] = y[s];
    if (t == 0) split_count(a, e, 0, itS);
  } else {
    // ---- M_J z = r (mapped elements) --------------------------------------------------
    double rv[4] = {}, z[4] = {}, ms[4] = {1.0, 1.0, 1.0, 1.0}, di[4];
    const double zero[4] = {};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (L.ok(s)) {
        const long gi = e0 + L.node(s);
        rv[s] = a.Fv[gi];
        z[s] = a.xM[gi];
        if (a.el.msc) ms[s] = a.el.msc[gi];
      }
    const double area = scp[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) di[s] = (P32 ? w0_ok2(L, s) : L.ok(s)) ? 1.0 / area : 0.0;
    const int itM = w0_solve<N1C, P, P32>(W, L, Pp, ctl, z, rv, zero, di, ms, a.el.msc != nullptr, 0.0,
                                     a.rtol, a.maxit);
    w0_end(ctl);
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (L.ok(s)) a.xM[e0 + L.node(s)] = z[s];
    if (t == 0) split_count(a, e, 1, itM);
  }
}

// Solve kernels: wave 0 runs the recurrence (w0_element), waves 1.. hold the operator in
// registers (unit u = threadIdx.x - 64 of the slot-ordered copy) and form the products.  The
// two roles meet only at the barriers of the product rounds, so each keeps its own registers.
// P32: the preconditioner's transforms on the FP32 matrix cores (w0_precond).
template <int OP, int N1C, int P, bool GRP, bool P32 = false>
__global__ __launch_bounds__(kRegMaxThreads) void k_pcg_solve_w0(
    const PcgStageArgs* __restrict__ args, const long* __restrict__ el_start, int nprob) {
  static_assert(N1C <= 16, "one matrix-core tile");
  extern __shared__ double shd[];
  constexpr int n1 = N1C, NP = N1C + 1, nn = N1C * N1C;
  const ElemRange<GRP> rg{el_start, nprob};
  const PcgStageArgs& a0 = args[0];
  const int t = threadIdx.x;
  BlockSolve<N1C, double, kRegMaxThreads> W;
  W.A = nullptr;
  W.K = a0.blk_K;
  W.CH = a0.blk_CH;
  W.WB = a0.blk_WB;
  W.p = a0.g.p;
  W.N = a0.g.N;
  double* sp = shd;
  W.P = sp;  sp += nn * W.WB;
  W.U = sp;  sp += NP * NP;
  W.R = W.T = W.Z = W.DI = W.Psi = nullptr;
  int* ctl = reinterpret_cast<int*>(sp);
  int* jc = ctl + 1;
  W.boff = nullptr;
  W.jc = jc;
  for (int i = t; i < W.K; i += blockDim.x) jc[i] = a0.blk_jc[i];
  for (int i = t; i < NP * NP; i += blockDim.x) W.U[i] = 0.0;
  __syncthreads();
  const long total = rg.total(args);
  // The roles branch on the wave index held in a scalar register, so that each wave jumps
  // over the other role's code (and its barriers) instead of running it with no lanes on.
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  if (wave == 0) {
    const W0Lane<N1C> L = w0_lane<N1C>();
    W0Pre Pp;
    // the eigenbasis in the operand layout of the transforms (a group reloads it when the
    // workgroup changes member)
    auto load_pre = [&](const PcgGeom& g) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int q = 4 * s + L.g;
        const bool in = L.c < n1 && q < n1;
        Pp.psk[s] = in ? g.Psi[q * n1 + L.c] : 0.0;
        Pp.pks[s] = in ? g.Psi[L.c * n1 + q] : 0.0;
        if constexpr (P32) {
          const int q2 = 4 * L.g + s;
          const bool in2 = L.c < n1 && q2 < n1;
          Pp.psk1[s] = (float)Pp.psk[s];
          Pp.psk2[s] = in2 ? (float)g.Psi[q2 * n1 + L.c] : 0.f;
          Pp.pks2[s] = in2 ? (float)g.Psi[L.c * n1 + q2] : 0.f;
        }
      }
    };
    if constexpr (!GRP) load_pre(a0.g);
    int k = 0;
    [[maybe_unused]] int cur = -1;
    for (long b = blockIdx.x; b < total; b += gridDim.x) {
      k = rg.member(b, k);
      const PcgStageArgs& a = args[k];
      if constexpr (GRP) {
        if (k != cur) {
          load_pre(a.g);
          cur = k;
        }
      }
      w0_element<OP, N1C, P, P32>(a, b - rg.first(k), W, L, Pp, ctl);
    }
  } else {
    // two operator buffers: the next element's entries load while this element's rounds run
    const size_t per = (size_t)RegOp<N1C, P>::CH * RegOp<N1C, P>::W * a0.blk_threads;
    const int u = t - 64;
    const double* op0 = OP == 0 ? a0.el.Sreg : a0.el.Mreg;
    int k = 0;
    // slot-ordered operator of element b (b increases from call to call)
    auto opr = [&](long b) -> const double* {
      if constexpr (GRP) {
        k = rg.member(b, k);
        const PcgStageArgs& a = args[k];
        return (OP == 0 ? a.el.Sreg : a.el.Mreg) + (b - rg.first(k)) * per;
      }
      return op0 + b * per;
    };
    if constexpr (RegOp<N1C, P>::CH * RegOp<N1C, P>::W > 48) {
      // one buffer where two would not fit the registers
      RegOp<N1C, P> R;
      for (long b = blockIdx.x; b < total; b += gridDim.x) {
        reg_gather(a0, W, R, opr(b), u);
        unit_rounds<N1C, P>(W, R, ctl);
      }
      return;
    }
    // Each buffer is waited for (vmcnt(0), the units issue no other vector memory operation)
    // at the end of the rounds that overlap its loads, so that the rounds of an element
    // never wait on the loads of the next one.
    RegOp<N1C, P> R0, R1;
    long b = blockIdx.x;
    if (b < total) reg_gather(a0, W, R0, opr(b), u);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    while (b < total) {
      const long b1 = b + gridDim.x;
      if (b1 < total) reg_gather(a0, W, R1, opr(b1), u);
      unit_rounds<N1C, P>(W, R0, ctl);
      __builtin_amdgcn_s_waitcnt(kWaitVm0);
      if (b1 >= total) break;
      const long b2 = b1 + gridDim.x;
      if (b2 < total) reg_gather(a0, W, R0, opr(b2), u);
      unit_rounds<N1C, P>(W, R1, ctl);
      __builtin_amdgcn_s_waitcnt(kWaitVm0);
      b = b2;
    }
  }
}

// Energy sum_k 1/2 V^T M_J V + 1/2 U^T S_K U, one workgroup per element (partials), then a
// fixed-order sum.
__global__ __launch_bounds__(1024) void k_pcg_energy(PcgGeom g, PcgElem el,
                                                     const double* __restrict__ U,
                                                     const double* __restrict__ V, long nel,
                                                     double* __restrict__ part) {
  extern __shared__ double shd[];
  __shared__ double red[32];
  const long e = blockIdx.x;
  const int t = threadIdx.x, nn = g.nn, n1 = g.n1;
  double* u = shd;
  double* v = u + nn;
  for (int i = t; i < nn; i += blockDim.x) {
    u[i] = U[e * nn + i];
    v[i] = V[e * nn + i];
  }
  __syncthreads();
  double s = 0.0, unused = 0.0;
  if (t < nn) {
    const int ix = t % n1, iy = t / n1;
    const double su = sym_row<double, double, double>(el.S + e * g.nst, g.rowoff, u, ix, iy, g.p, g.N, n1);
    double mv;
    if (el.M) {
      mv = sym_row<double, double, double>(el.M + e * g.nst, g.rowoff, v, ix, iy, g.p, g.N, n1);
    } else {
      mv = 0.0;
      for (int jy = 0; jy < n1; ++jy)
        for (int jx = 0; jx < n1; ++jx) mv += g.Mref[iy * n1 + jy] * g.Mref[ix * n1 + jx] * v[jy * n1 + jx];
      mv *= el.sc[e * 8 + 4];
    }
    s = u[t] * su + v[t] * mv;
  }
  block_sum2(s, unused, red);
  if (t == 0) part[e] = s;
}

__global__ __launch_bounds__(256) void k_sum_part(const double* __restrict__ part, long n,
                                                  double* __restrict__ out) {
  __shared__ double red[32];
  double s = 0.0, unused = 0.0;
  for (long i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  block_sum2(s, unused, red);
  if (threadIdx.x == 0) out[0] = 0.5 * s;
}

// ---------------------------------------------------------------------------------
// Blocks of a persistent launch: every CU filled to the kernel's occupancy, at most one
// block per element.
static unsigned persistent_grid(const void* kernel, int threads, size_t lds, long nel) {
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
      ncu = 256;
  }
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, lds) != hipSuccess ||
      occ < 1)
    occ = 1;
  const long g = (long)ncu * occ;
  return (unsigned)(nel < g ? nel : g);
}

static int threads_for(int nn) {
  int b = ((nn + 63) / 64) * 64;
  return b < 256 ? 256 : b;
}

hipError_t launch_assemble(const PcgGeom& g, const double* X, const double* Y, const double* C2,
                           const PcgElem& el, long nel, hipStream_t st) {
  if (nel == 0) return hipSuccess;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)nel), dim3(256), 0, st, g, X, Y, C2, el, nel);
  return hipGetLastError();
}

hipError_t launch_face_geom(const PcgGeom& g, const double* X, const double* Y, const double* C2,
                            const PcgElem& el, long nel, hipStream_t st) {
  const long n = nel * 4 * g.nq;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_face_geom, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, X, Y, C2,
                     el, nel);
  return hipGetLastError();
}

// Nodal scale of the M_J preconditioner: s_i = sqrt(diag(P_M)_i / (M_J)_ii) with
// diag(P_M)_(iy,ix) = |Omega_k| Mref_(iy,iy) Mref_(ix,ix), so that s P_M^-1 s has the
// inverse diagonal scaling of M_J itself.
__global__ void k_mscale(PcgGeom g, PcgElem el, long nel) {
  const long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (id >= nel * g.nn) return;
  const long e = id / g.nn;
  const int i = (int)(id - e * g.nn), ix = i % g.n1, iy = i / g.n1;
  const double d = el.M[e * g.nst + g.rowoff[i] + st_pos(ix, iy, ix, iy, g.p, g.N)];
  const double pm = el.sc[e * 8 + 4] * g.Mref[iy * g.n1 + iy] * g.Mref[ix * g.n1 + ix];
  el.msc[id] = sqrt(pm / d);
}

__global__ void k_source_step(double* t_dev, double* w, double dt, SourceTerms f) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double t = t_dev[0];
  const double cs[4] = {0.0, 0.5, 0.5, 1.0};
  for (int s = 0; s < 4; ++s)
    for (int k = 0; k < 4; ++k)
      w[4 * s + k] = k < f.nf ? sin(f.omega[k] * (t + cs[s] * dt) + f.phase[k]) : 0.0;
  t_dev[0] = t + dt;
}

__global__ void k_set_clock(double* t_dev, double t) {
  if (blockIdx.x == 0 && threadIdx.x < 17) t_dev[threadIdx.x] = threadIdx.x == 0 ? t : 0.0;
}

hipError_t launch_set_clock(double* t_dev, double t, hipStream_t st) {
  hipLaunchKernelGGL(k_set_clock, dim3(1), dim3(64), 0, st, t_dev, t);
  return hipGetLastError();
}

hipError_t launch_source_step(double* t_dev, double* w, double dt, const SourceTerms& f,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_source_step, dim3(1), dim3(64), 0, st, t_dev, w, dt, f);
  return hipGetLastError();
}

hipError_t launch_mscale(const PcgGeom& g, const PcgElem& el, long nel, hipStream_t st) {
  const long n = nel * g.nn;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mscale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, el, nel);
  return hipGetLastError();
}

__global__ void k_reg_permute(const double* __restrict__ half, const int* __restrict__ gidx,
                              int nst, long per, long total, double* __restrict__ out) {
  for (long id = blockIdx.x * (long)blockDim.x + threadIdx.x; id < total;
       id += (long)gridDim.x * blockDim.x) {
    const long e = id / per, r = id - e * per;
    const int h = gidx[r];
    out[id] = h >= 0 ? half[e * nst + h] : 0.0;
  }
}

int pcg_reg_slots(int n1, int p) {
  if (!(pcg_family_key(n1, p, 1, 0) & 64)) return 0;
  return blk_ch_c(n1, p, kRegMaxThreads, pcg_unit_chmax(n1, p)) * std::min(2 * p + 1, n1);
}

hipError_t launch_reg_permute(const double* half, const int* gidx, int nst, int slots,
                              int threads, long nel, double* out, hipStream_t st) {
  const long per = (long)slots * threads, total = per * nel;
  if (total == 0) return hipSuccess;
  const long nb = std::min<long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_reg_permute, dim3((unsigned)nb), dim3(256), 0, st, half, gidx, nst, per,
                     total, out);
  return hipGetLastError();
}

hipError_t launch_split_hilo(const double* half, const int* dst, int nst, int nnz, long nel,
                             float* hi, float* lo, hipStream_t st) {
  const long n = nel * nst;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_hilo, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, half, dst,
                     nst, nnz, nel, hi, lo);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* a, float* b, long n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
  return hipGetLastError();
}

hipError_t launch_pcg_traces(const PcgGeom& g, const PcgElem& el, const double* U, const double* V,
                             double* tr, long nel, hipStream_t st) {
  if (nel == 0) return hipSuccess;
  const size_t sh = (2 * g.nn + 4 * g.n1) * sizeof(double);
  hipLaunchKernelGGL(k_pcg_traces, dim3((unsigned)nel), dim3(threads_for(g.nn)), sh, st, g, el, U,
                     V, tr, nel);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Column-block layout (host): tables, eligibility, LDS size.
// ---------------------------------------------------------------------------------
static size_t blk_lds_bytes(const PcgGeom& g, int nnz_full, int WB, int K, int mixed = 0) {
  size_t nd;
  if (pcg_family_key(g.n1, g.p, 1, mixed) & 64) {
    switch (g.n1) {
      case 9: nd = reg_lds_doubles<9>(g, WB); break;
      case 13: nd = reg_lds_doubles<13>(g, WB); break;
      case 17: nd = reg_lds_doubles<17>(g, WB); break;
      default: return (size_t)-1;
    }
    return nd * sizeof(double) + ((size_t)g.nn + K + common_ints(g)) * sizeof(int);
  }
  switch (g.n1) {
    case 9: nd = mixed ? mix_lds_doubles<9>(g, nnz_full, WB) : blk_lds_doubles<9>(g, nnz_full, WB); break;
    case 13: nd = mixed ? mix_lds_doubles<13>(g, nnz_full, WB) : blk_lds_doubles<13>(g, nnz_full, WB); break;
    case 17: nd = mixed ? mix_lds_doubles<17>(g, nnz_full, WB) : blk_lds_doubles<17>(g, nnz_full, WB); break;
    default: return (size_t)-1;
  }
  return nd * sizeof(double) + ((size_t)g.nn + K + common_ints(g)) * sizeof(int);
}

int pcg_block_tables(const PcgGeom& g, const std::vector<int>& rowoff, std::vector<int>& boff,
                     std::vector<int>& dst, std::vector<int>& jc, std::vector<int>& gidx,
                     std::vector<int>& unit, int* K, int* CH, int* WB, int* nnz, int* threads,
                     int mixed) {
  const int n1 = g.n1, N = g.N, p = g.p, nn = g.nn;
  if (n1 != 9 && n1 != 13 && n1 != 17) return 0;
  // the register-operator kernels run on fewer threads with taller chunks
  const bool reg = (pcg_family_key(n1, p, 1, mixed) & 64) != 0;
  const int maxt = reg ? kRegMaxThreads : kBlkMaxThreads;
  const int chmax = reg ? pcg_unit_chmax(n1, p) : 4;
  boff.assign(nn, 0);
  int off = 0, wb = 0;
  for (int jy = 0; jy < n1; ++jy)
    for (int ix = 0; ix < n1; ++ix) {
      boff[jy * n1 + ix] = off;
      off += st_w(ix, p, N) * st_w(jy, p, N);
    }
  for (int k = 0; k < n1; ++k) wb = std::max(wb, st_w(k, p, N));
  int ch = 1, kk = 0;
  for (ch = 1; ch <= chmax; ++ch) {
    kk = 0;
    for (int jy = 0; jy < n1; ++jy) kk += (st_w(jy, p, N) + ch - 1) / ch;
    if (n1 * kk <= maxt) break;
  }
  if (ch > chmax || kk > 255) return 0;
  if (reg && ch != blk_ch_c(n1, p, maxt, chmax)) return 0;   // the kernel's compiled CH
  jc.clear();
  for (int jy = 0; jy < n1; ++jy) {
    const int nc = (st_w(jy, p, N) + ch - 1) / ch;
    for (int c = 0; c < nc; ++c) jc.push_back(jy | (c << 8));
  }
  dst.assign((size_t)2 * g.nst, 0);
  for (int i = 0; i < nn; ++i) {
    const int ix = i % n1, iy = i / n1;
    for (int j = i; j < nn; ++j) {
      const int jx = j % n1, jy = j / n1;
      if (!st_in_upper(ix, iy, jx, jy, p, N)) continue;
      const int h = rowoff[i] + st_pos(ix, iy, jx, jy, p, N);
      // A[(ix,iy),(jx,jy)] in block (ix, jy), row iy, column jx; and its transpose
      dst[2 * h] = boff[jy * n1 + ix] + (iy - st_lo(jy, p)) * st_w(ix, p, N) + (jx - st_lo(ix, p));
      dst[2 * h + 1] = boff[iy * n1 + jx] + (jy - st_lo(iy, p)) * st_w(jx, p, N) + (ix - st_lo(jx, p));
    }
  }
  const int sp = blk_pinv_split(nn, maxt);      // lanes per output in blk_pinv
  const int thr = ((std::max(n1 * kk, sp * nn) + 63) / 64) * 64;
  if (thr > maxt) return 0;
  gidx.clear();
  unit.clear();
  if (reg) {
    // upper-half index of every (unit, row, column) slot: the inverse of dst
    std::vector<int> inv((size_t)off, -1);
    for (int h = 0; h < g.nst; ++h) {
      inv[dst[2 * h]] = h;
      inv[dst[2 * h + 1]] = h;
    }
    const int W = std::min(2 * p + 1, n1);
    // thread of each unit: the unit itself, or for the streamed family the units in order of
    // decreasing width and height, so that the threads that read a slot form a prefix and a
    // wave skips the cache lines of padding slots
    std::vector<int> pos(n1 * kk);
    for (int t = 0; t < n1 * kk; ++t) pos[t] = t;
    if (chmax == kMemMaxCh) {
      std::vector<int> ord(n1 * kk);
      for (int t = 0; t < n1 * kk; ++t) ord[t] = t;
      auto wxy = [&](int t) {
        const int k = t / n1, ix = t % n1, jy = jc[k] & 0xff, c = jc[k] >> 8;
        return std::make_pair(st_w(ix, p, N), std::min(ch, st_w(jy, p, N) - c * ch));
      };
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return wxy(a) > wxy(b); });
      unit = ord;
      for (int i = 0; i < n1 * kk; ++i) pos[ord[i]] = i;
    }
    gidx.assign((size_t)ch * W * thr, -1);
    for (int t = 0; t < n1 * kk; ++t) {
      const int k = t / n1, ix = t % n1;
      const int jy = jc[k] & 0xff, c = jc[k] >> 8;
      const int wx = st_w(ix, p, N), wy = st_w(jy, p, N);
      for (int i = 0; i < ch && c * ch + i < wy; ++i)
        for (int q = 0; q < wx; ++q) {
          const int h = inv[boff[jy * n1 + ix] + (c * ch + i) * wx + q];
          if (h < 0) return 0;                    // every block entry is an operator entry
          gidx[((size_t)i * W + q) * thr + pos[t]] = h;
        }
    }
  }
  const size_t lds = blk_lds_bytes(g, off, wb, kk, mixed);
  if (lds > 160 * 1024) return 0;
  *K = kk;
  *CH = ch;
  *WB = wb;
  *nnz = off;
  *threads = thr;
  return 1;
}

void pcg_stage_shape(const PcgGeom& g, int threads, int* full, int* Q, int* nnz_full, size_t* lds) {
  *full = stage_full(g);
  *nnz_full = full_nnz(g);
  int q = full_parts(g);
  if (*full) {
    const int qt = threads / g.nn;
    if (q > qt) q = qt;
    if (q < 1) q = 1;
  }
  *Q = q;
  *lds = stage_lds(g, *full);
}

int pcg_args_shape(PcgStageArgs& a, int threads, size_t* lds) {
  if (a.v2) {
    *lds = blk_lds_bytes(a.g, a.nnz_full, a.blk_WB, a.blk_K, a.mixed);
    return threads >= a.blk_threads;
  }
  pcg_stage_shape(a.g, threads, &a.full, &a.Q, &a.nnz_full, lds);
  return threads >= ((a.g.nn + 63) / 64) * 64;
}

// Kernel families of the grouped stage kernel: 0 (row layout), N + 1 (column blocks,
// FP64 operator in LDS), N + 1 + 32 (mixed), N + 1 + 64 + 128 p (FP64 operator in registers).
#define GDW_REG_KEY(n1, p) ((n1) | 64 | ((p) << 7))
#define GDW_PCG_KEYS(X)                                                                   \
  X(0) X(9) X(13) X(17) X(41) X(45) X(49)                                                 \
  X(GDW_REG_KEY(9, 3)) X(GDW_REG_KEY(9, 5)) X(GDW_REG_KEY(9, 7)) X(GDW_REG_KEY(13, 3))   \
  X(GDW_REG_KEY(13, 5)) X(GDW_REG_KEY(13, 7)) X(GDW_REG_KEY(17, 3)) X(GDW_REG_KEY(17, 5))

// The streamed family has the split stage only (no fused stage kernel).
#define GDW_MEM_KEY GDW_REG_KEY(17, 7)

static bool pcg_key_known(int key) {
#define GDW_K(k) if (key == (k)) return true;
  GDW_PCG_KEYS(GDW_K)
#undef GDW_K
  return key == GDW_MEM_KEY;
}

template <int STAGE, int N1C>
static hipError_t launch_group_k(const PcgStageArgs* args, const long* el_start, int nprob,
                                 unsigned grid, int threads, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k_pcg_stage_group<STAGE, N1C>), dim3(grid), dim3(threads), lds, st, args,
                     el_start, nprob);
  return hipGetLastError();
}

template <int STAGE>
static hipError_t launch_group_n1(int key, const PcgStageArgs* args, const long* el_start,
                                  int nprob, unsigned grid, int threads, size_t lds,
                                  hipStream_t st) {
  switch (key) {
#define GDW_K(k) \
    case k: return launch_group_k<STAGE, k>(args, el_start, nprob, grid, threads, lds, st);
    GDW_PCG_KEYS(GDW_K)
#undef GDW_K
    default: return hipErrorInvalidValue;
  }
}

template <int N1C>
static hipError_t group_attrs() {
  hipError_t e;
  const void* k[4] = {(const void*)k_pcg_stage_group<1, N1C>, (const void*)k_pcg_stage_group<2, N1C>,
                      (const void*)k_pcg_stage_group<3, N1C>, (const void*)k_pcg_stage_group<4, N1C>};
  for (int i = 0; i < 4; ++i)
    if ((e = hipFuncSetAttribute(k[i], hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024)) !=
        hipSuccess)
      return e;
  return hipSuccess;
}

hipError_t pcg_group_prepare() {
  hipError_t e = hipSuccess;
#define GDW_K(k) if (e == hipSuccess) e = group_attrs<k>();
  GDW_PCG_KEYS(GDW_K)
#undef GDW_K
  return e;
}

int pcg_group_max_threads(int key) {
  return (key & 64) ? kRegMaxThreads : key > 0 ? kBlkMaxThreads : 1024;
}

hipError_t launch_pcg_stage_group(int stage, int n1, const PcgStageArgs* args, const long* el_start,
                                  int nprob, unsigned grid, int threads, size_t lds, hipStream_t st) {
  if (nprob <= 0 || grid == 0) return hipSuccess;
  if (lds > 160 * 1024 || threads > pcg_group_max_threads(n1) || threads < 64)
    return hipErrorInvalidValue;
  switch (stage) {
    case 1: return launch_group_n1<1>(n1, args, el_start, nprob, grid, threads, lds, st);
    case 2: return launch_group_n1<2>(n1, args, el_start, nprob, grid, threads, lds, st);
    case 3: return launch_group_n1<3>(n1, args, el_start, nprob, grid, threads, lds, st);
    default: return launch_group_n1<4>(n1, args, el_start, nprob, grid, threads, lds, st);
  }
}

template <int STAGE>
static const void* group_kernel_n1(int key) {
  switch (key) {
#define GDW_K(k) \
    case k: return (const void*)k_pcg_stage_group<STAGE, k>;
    GDW_PCG_KEYS(GDW_K)
#undef GDW_K
    default: return nullptr;
  }
}

unsigned pcg_group_grid(int stage, int key, int threads, size_t lds, long nel) {
  const void* k = stage == 1 ? group_kernel_n1<1>(key) : stage == 2 ? group_kernel_n1<2>(key)
                : stage == 3 ? group_kernel_n1<3>(key) : group_kernel_n1<4>(key);
  return persistent_grid(k, threads, lds, nel);
}

int pcg_family_key(int n1, int p, int v2, int mixed) {
  if (!v2) return 0;
  if (mixed) return n1 + 32;
  const int rk = GDW_REG_KEY(n1, p);
  return pcg_key_known(rk) ? rk : n1;
}

int pcg_group_key(const PcgStageArgs& a) { return pcg_family_key(a.g.n1, a.g.p, a.v2, a.mixed); }

// ---- split stage (host) ---------------------------------------------------------------
bool pcg_split_key(int key) { return (key & 64) != 0 && pcg_key_known(key); }

bool pcg_pc32_supported(int n1, int p, int blk_threads) {
  return n1 <= 16 && pcg_split_key(pcg_family_key(n1, p, 1, 0)) &&
         64 + blk_threads <= kRegMaxThreads;
}

static int split_threads(const PcgGeom& g) {
  const int b = ((g.nn + 63) / 64) * 64;
  return b < 128 ? 128 : b;
}

// Elements of a split launch (device args, optional member table with its host copy, the
// member count and the element total).
struct SplitSet {
  const PcgStageArgs* args;
  const long* el_start;
  const long* h_start;
  int nprob;
  long total;
};

// Wave-0 solve launch (k_pcg_solve_w0), FP64 or FP32 preconditioner chain.
template <int N1C, int P, bool GRP, bool P32>
static hipError_t split_solve_w0(int op, const SplitSet& S, const PcgStageArgs& h,
                                 hipStream_t st) {
  const size_t lds = ((size_t)N1C * N1C * h.blk_WB + (N1C + 1) * (N1C + 1)) * sizeof(double) +
                     (size_t)(h.blk_K + 1) * sizeof(int);
  const int thr = 64 + h.blk_threads;
  const void* k = op == 0 ? (const void*)k_pcg_solve_w0<0, N1C, P, GRP, P32>
                          : (const void*)k_pcg_solve_w0<1, N1C, P, GRP, P32>;
  const unsigned grid = persistent_grid(k, thr, lds, S.total);
  if (op == 0)
    hipLaunchKernelGGL((k_pcg_solve_w0<0, N1C, P, GRP, P32>), dim3(grid), dim3(thr), lds, st,
                       S.args, S.el_start, S.nprob);
  else
    hipLaunchKernelGGL((k_pcg_solve_w0<1, N1C, P, GRP, P32>), dim3(grid), dim3(thr), lds, st,
                       S.args, S.el_start, S.nprob);
  return hipGetLastError();
}

template <int N1C, int P, bool GRP>
static hipError_t split_solve_t(int op, const SplitSet& S, const PcgStageArgs& h, int threads,
                                hipStream_t st) {
  if constexpr (N1C <= 16) {
    if (64 + h.blk_threads <= kRegMaxThreads) {
      // vectors on wave 0, work units on the waves after it
      if (h.pc32) return split_solve_w0<N1C, P, GRP, true>(op, S, h, st);
      return split_solve_w0<N1C, P, GRP, false>(op, S, h, st);
    }
  }
  if (h.pc32) return hipErrorInvalidValue;     // no FP32 chain in the per-node kernels
  // (+ 16 doubles: the M_J solve's early-test slots)
  const size_t lds = (solve_lds_doubles<N1C>(h.blk_WB) + (op == 1 ? 16 : 0)) * sizeof(double) +
                     (size_t)h.blk_K * sizeof(int);
  const void* k = op == 0 ? (const void*)k_pcg_solve<0, N1C, P, GRP>
                          : (const void*)k_pcg_solve<1, N1C, P, GRP>;
  const unsigned grid = persistent_grid(k, threads, lds, S.total);
  if (op == 0)
    hipLaunchKernelGGL((k_pcg_solve<0, N1C, P, GRP>), dim3(grid), dim3(threads), lds, st, S.args,
                       S.el_start, S.nprob);
  else
    hipLaunchKernelGGL((k_pcg_solve<1, N1C, P, GRP>), dim3(grid), dim3(threads), lds, st, S.args,
                       S.el_start, S.nprob);
  return hipGetLastError();
}

template <int N1C, int P>
static hipError_t split_solve(int op, const SplitSet& S, const PcgStageArgs& h, int threads,
                              hipStream_t st) {
  if constexpr (N1C <= 16) {
    if (S.el_start) return split_solve_t<N1C, P, true>(op, S, h, threads, st);
  } else {
    if (S.el_start) return hipErrorInvalidValue;   // launched per member (split_solves)
  }
  return split_solve_t<N1C, P, false>(op, S, h, threads, st);
}

// Solves of the streamed family: one problem per launch (groups launch per member).
template <int N1C, int P>
static hipError_t split_solve_mem(int op, const SplitSet& S, const PcgStageArgs& h, int threads,
                                  hipStream_t st) {
  if (S.el_start || h.pc32 || h.blk_threads != kMemMaxThreads || threads != kMemMaxThreads)
    return hipErrorInvalidValue;   // the kernel's compiled slot stride
  const size_t lds = (solve_lds_doubles<N1C>(h.blk_WB) + 16) * sizeof(double) +   // + early-test slots
                     (size_t)h.blk_K * sizeof(int);
  const void* k = op == 0 ? (const void*)k_pcg_solve<0, N1C, P, false, true>
                          : (const void*)k_pcg_solve<1, N1C, P, false, true>;
  const unsigned grid = persistent_grid(k, threads, lds, S.total);
  if (op == 0)
    hipLaunchKernelGGL((k_pcg_solve<0, N1C, P, false, true>), dim3(grid), dim3(threads), lds, st,
                       S.args, S.el_start, S.nprob);
  else
    hipLaunchKernelGGL((k_pcg_solve<1, N1C, P, false, true>), dim3(grid), dim3(threads), lds, st,
                       S.args, S.el_start, S.nprob);
  return hipGetLastError();
}

static hipError_t split_solve_key(int key, int op, const SplitSet& S, const PcgStageArgs& h,
                                  int threads, hipStream_t st) {
  switch (key) {
    case GDW_MEM_KEY: return split_solve_mem<17, 7>(op, S, h, threads, st);
    case GDW_REG_KEY(9, 3): return split_solve<9, 3>(op, S, h, threads, st);
    case GDW_REG_KEY(9, 5): return split_solve<9, 5>(op, S, h, threads, st);
    case GDW_REG_KEY(9, 7): return split_solve<9, 7>(op, S, h, threads, st);
    case GDW_REG_KEY(13, 3): return split_solve<13, 3>(op, S, h, threads, st);
    case GDW_REG_KEY(13, 5): return split_solve<13, 5>(op, S, h, threads, st);
    case GDW_REG_KEY(13, 7): return split_solve<13, 7>(op, S, h, threads, st);
    case GDW_REG_KEY(17, 3): return split_solve<17, 3>(op, S, h, threads, st);
    case GDW_REG_KEY(17, 5): return split_solve<17, 5>(op, S, h, threads, st);
    default: return hipErrorInvalidValue;
  }
}

template <int STAGE, bool GRP>
static hipError_t split_stream(int part, const SplitSet& S, const PcgStageArgs& h,
                               hipStream_t st) {
  const int threads = split_threads(h.g);
  const size_t lds = split_lds_bytes(h.g);
  const void* k = part == 0 ? (const void*)k_pcg_lift<STAGE, GRP>
                            : (const void*)k_pcg_update<STAGE, GRP>;
  const unsigned grid = persistent_grid(k, threads, lds, S.total);
  if (part == 0)
    hipLaunchKernelGGL((k_pcg_lift<STAGE, GRP>), dim3(grid), dim3(threads), lds, st, S.args,
                       S.el_start, S.nprob);
  else
    hipLaunchKernelGGL((k_pcg_update<STAGE, GRP>), dim3(grid), dim3(threads), lds, st, S.args,
                       S.el_start, S.nprob);
  return hipGetLastError();
}

template <int STAGE>
static hipError_t split_stream_g(int part, const SplitSet& S, const PcgStageArgs& h,
                                 hipStream_t st) {
  return S.el_start ? split_stream<STAGE, true>(part, S, h, st)
                    : split_stream<STAGE, false>(part, S, h, st);
}

static hipError_t split_stream_stage(int stage, int part, const SplitSet& S,
                                     const PcgStageArgs& h, hipStream_t st) {
  switch (stage) {
    case 1: return split_stream_g<1>(part, S, h, st);
    case 2: return split_stream_g<2>(part, S, h, st);
    case 3: return split_stream_g<3>(part, S, h, st);
    default: return split_stream_g<4>(part, S, h, st);
  }
}

// The solves of a set.  The per-node solve kernels (N + 1 = 17) sit at the register limit,
// where the member bookkeeping of a grouped walk costs spills (N + 1 = 17, p = 5: 66 VGPRs
// instead of 29); their groups launch one solve per member instead.
static hipError_t split_solves(int key, int op, const SplitSet& S, const PcgStageArgs& h,
                               int threads, hipStream_t st) {
  if (S.total == 0) return hipSuccess;
  if (S.el_start == nullptr || (key & 31) <= 16) return split_solve_key(key, op, S, h, threads, st);
  for (int k = 0; k < S.nprob; ++k) {
    const long n = S.h_start[k + 1] - S.h_start[k];
    if (n == 0) continue;
    const SplitSet one{S.args + k, nullptr, nullptr, 1, n};
    const hipError_t e = split_solve_key(key, op, one, h, threads, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static hipError_t split_stage(int stage, int key, const SplitSet& all, const SplitSet& mapped,
                              const PcgStageArgs& h, int threads, hipStream_t st) {
  if (all.total == 0) return hipSuccess;
  if (!pcg_split_key(key) || h.Fu == nullptr || h.Fv == nullptr || h.g.nn > 512 ||
      threads > kRegMaxThreads || threads < h.blk_threads)
    return hipErrorInvalidValue;
  hipError_t e;
  if ((e = split_stream_stage(stage, 0, all, h, st)) != hipSuccess) return e;
  if ((e = split_solves(key, 0, all, h, threads, st)) != hipSuccess) return e;
  if ((e = split_solves(key, 1, mapped, h, threads, st)) != hipSuccess) return e;
  return split_stream_stage(stage, 1, all, h, st);
}

hipError_t launch_pcg_split_stage(int stage, int key, const PcgStageArgs* a, const PcgStageArgs& h,
                                  int threads, size_t lds, hipStream_t st) {
  (void)lds;
  const SplitSet all{a, nullptr, nullptr, 1, h.nel};
  const SplitSet mapped{a, nullptr, nullptr, 1, h.mapped ? h.nel : 0};
  return split_stage(stage, key, all, mapped, h, threads, st);
}

hipError_t launch_pcg_split_group(int stage, int key, const PcgStageArgs* args,
                                  const long* el_start, const long* h_el_start, int nprob,
                                  const PcgStageArgs* args_m, const long* el_start_m,
                                  const long* h_el_start_m, int nprob_m, const PcgStageArgs& h,
                                  int threads, hipStream_t st) {
  if (nprob <= 0 || el_start == nullptr || h_el_start == nullptr ||
      (nprob_m > 0 && (args_m == nullptr || el_start_m == nullptr || h_el_start_m == nullptr)))
    return hipErrorInvalidValue;
  const SplitSet all{args, el_start, h_el_start, nprob, h_el_start[nprob]};
  const SplitSet mapped{args_m, el_start_m, h_el_start_m, nprob_m,
                        nprob_m > 0 ? h_el_start_m[nprob_m] : 0};
  return split_stage(stage, key, all, mapped, h, threads, st);
}

int pcg_single_shape(PcgStageArgs& a, int* threads, size_t* lds) {
  if (a.v2) {
    *threads = a.blk_threads;
    *lds = blk_lds_bytes(a.g, a.nnz_full, a.blk_WB, a.blk_K, a.mixed);
  } else {
    if (a.fo == nullptr || a.dst == nullptr) return 0;
    *threads = stage_full(a.g) ? 1024 : threads_for(a.g.nn);
    if (!pcg_args_shape(a, *threads, lds)) return 0;
  }
  return *lds <= 160 * 1024;
}

hipError_t launch_pcg_energy(const PcgGeom& g, const PcgElem& el, const double* U, const double* V,
                             long nel, double* part, int npart, double* out, hipStream_t st) {
  (void)npart;
  if (nel == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pcg_energy, dim3((unsigned)nel), dim3(threads_for(g.nn)),
                     2 * g.nn * sizeof(double), st, g, el, U, V, nel, part);
  hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(256), 0, st, part, nel, out);
  return hipGetLastError();
}

}  // namespace gdw
