// Zero-fill incomplete Cholesky (IC(0)) baseline for the element systems (Sec. 7.1).
//
// Sec. 7.1 solves the element matrices of DG1 / DG2 by PCG with an incomplete Cholesky
// preconditioner.  Here it is a baseline beside the tensor-product preconditioner of the
// time loop: the factor U (A ~ U^T U) keeps A's stencil (Sec. 3.1) and is stored in the
// same upper-half layout as the element operators (stencil.h).  For S_hat the factor is
// taken of S_hat's entries on S_K's stencil (the rank-one term w w^T is dense); the CG
// products use the whole S_hat.
//
// Kernels, one element per workgroup:
//   k_ic0_prepare  operator entries A (S_K or M_J) and the factor's input U = A (+ cw w w^T)
//   k_ic0_factor   right-looking IC(0) in place: for each pivot row k the updates of the
//                  (i, j) pairs of row k's stencil run in parallel, dropped off the stencil
//   k_ic0_pcg      one wave: CG vectors in LDS, products gathered row by row from the
//                  upper half, the two triangular solves level by level (host-computed
//                  level sets; each row's sum split across the lanes)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ic0.h"
#include "stencil.h"

namespace gdw {
namespace {

constexpr int kIc0MaxNodes = 17 * 17;

// column (jx, jy) of upper entry h of row (ix, iy) (inverse of st_pos)
__device__ inline void st_col(int ix, int iy, int h, int p, int N, int* jx, int* jy) {
  const int same = st_hi(ix, p, N) - ix + 1;
  if (h < same) {
    *jx = ix + h;
    *jy = iy;
    return;
  }
  h -= same;
  const int w = st_w(ix, p, N);
  *jy = iy + 1 + h / w;
  *jx = st_lo(ix, p) + h % w;
}

__global__ void k_ic0_prepare(PcgGeom g, PcgElem el, int op, long nel, double* A, double* U) {
  const long e = blockIdx.x;
  if (e >= nel) return;
  const int n1 = g.n1, N = g.N, p = g.p;
  const double* w = el.w + e * g.nn;
  const double cw = el.sc[e * 8 + 0];
  const double area = el.sc[e * 8 + 4];
  for (int i = 0; i < g.nn; ++i) {
    const int ix = i % n1, iy = i / n1;
    const int base = g.rowoff[i], cnt = g.rowoff[i + 1] - base;
    for (int h = threadIdx.x; h < cnt; h += blockDim.x) {
      int jx, jy;
      st_col(ix, iy, h, p, N, &jx, &jy);
      const long off = e * (long)g.nst + base + h;
      double a;
      if (op == 0)
        a = el.S[off];
      else if (el.M)
        a = el.M[off];
      else
        a = area * g.Mref[ix * n1 + jx] * g.Mref[iy * n1 + jy];
      A[off] = a;
      U[off] = op == 0 ? a + cw * w[i] * w[jy * n1 + jx] : a;
    }
  }
}

__global__ void k_ic0_factor(PcgGeom g, long nel, double* U, int* bad) {
  const long e = blockIdx.x;
  if (e >= nel) return;
  const int n1 = g.n1, N = g.N, p = g.p;
  double* Ue = U + e * (long)g.nst;
  for (int k = 0; k < g.nn; ++k) {
    const int kx = k % n1, ky = k / n1;
    const int base = g.rowoff[k], cnt = g.rowoff[k + 1] - base;
    const double d = Ue[base];
    if (!(d > 0.0)) {  // the same value in every lane: the whole group leaves
      if (threadIdx.x == 0) atomicMin(bad, (int)e);
      return;
    }
    const double piv = sqrt(d);
    __syncthreads();
    for (int h = threadIdx.x; h < cnt; h += blockDim.x)
      Ue[base + h] = h == 0 ? piv : Ue[base + h] / piv;
    __syncthreads();
    const int m = cnt - 1;
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
      const int a = 1 + t / m, b = 1 + t % m;
      if (b < a) continue;
      int ix, iy, jx, jy;
      st_col(kx, ky, a, p, N, &ix, &iy);
      st_col(kx, ky, b, p, N, &jx, &jy);
      if (!st_in_upper(ix, iy, jx, jy, p, N)) continue;  // fill: dropped
      Ue[g.rowoff[iy * n1 + ix] + st_pos(ix, iy, jx, jy, p, N)] -= Ue[base + a] * Ue[base + b];
    }
    __syncthreads();
  }
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// q = A d (+ cw w (w . d) for S_hat), one lane per row
__device__ void ic0_product(const PcgGeom& g, const double* Ae, const double* w, double cw,
                            const double* d, double* q) {
  const int n1 = g.n1, N = g.N, p = g.p;
  for (int i = threadIdx.x; i < g.nn; i += 64) {
    const int ix = i % n1, iy = i / n1;
    const int base = g.rowoff[i], cnt = g.rowoff[i + 1] - base;
    double s = 0.0;
    for (int h = 0; h < cnt; ++h) {
      int jx, jy;
      st_col(ix, iy, h, p, N, &jx, &jy);
      s += Ae[base + h] * d[jy * n1 + jx];
    }
    for (int ky = st_lo(iy, p); ky <= iy; ++ky)
      for (int kx = st_lo(ix, p); kx <= st_hi(ix, p, N); ++kx) {
        if (ky == iy && kx >= ix) break;
        s += Ae[g.rowoff[ky * n1 + kx] + st_pos(kx, ky, ix, iy, p, N)] * d[ky * n1 + kx];
      }
    q[i] = s;
  }
  if (w) {
    double part = 0.0;
    for (int i = threadIdx.x; i < g.nn; i += 64) part += w[i] * d[i];
    const double wd = cw * wave_sum(part);
    for (int i = threadIdx.x; i < g.nn; i += 64) q[i] += wd * w[i];
  }
  __syncthreads();
}

// z = (U^T U)^{-1} r: U^T y = r by the forward level sets, then U z = y by the backward ones
__device__ void ic0_apply(const PcgGeom& g, const double* Ue, const int* fw, const int* fws,
                          int nfw, const int* bw, const int* bws, int nbw, const double* r,
                          double* y, double* z) {
  const int n1 = g.n1, N = g.N, p = g.p;
  const int lane = threadIdx.x;
  for (int L = 0; L < nfw; ++L) {
    for (int s = fws[L]; s < fws[L + 1]; ++s) {
      const int i = fw[s];
      const int ix = i % n1, iy = i / n1;
      const int lo = st_lo(ix, p), wx = st_w(ix, p, N), ylo = st_lo(iy, p);
      const int nt = wx * (iy - ylo + 1);
      double part = 0.0;
      for (int t = lane; t < nt; t += 64) {
        const int kx = lo + t % wx, ky = ylo + t / wx;
        if (ky == iy && kx >= ix) continue;
        part += Ue[g.rowoff[ky * n1 + kx] + st_pos(kx, ky, ix, iy, p, N)] * y[ky * n1 + kx];
      }
      const double sum = wave_sum(part);
      if (lane == 0) y[i] = (r[i] - sum) / Ue[g.rowoff[i]];
    }
    __syncthreads();
  }
  for (int L = 0; L < nbw; ++L) {
    for (int s = bws[L]; s < bws[L + 1]; ++s) {
      const int i = bw[s];
      const int ix = i % n1, iy = i / n1;
      const int base = g.rowoff[i], cnt = g.rowoff[i + 1] - base;
      double part = 0.0;
      for (int h = 1 + lane; h < cnt; h += 64) {
        int jx, jy;
        st_col(ix, iy, h, p, N, &jx, &jy);
        part += Ue[base + h] * z[jy * n1 + jx];
      }
      const double sum = wave_sum(part);
      if (lane == 0) z[i] = (y[i] - sum) / Ue[base];
    }
    __syncthreads();
  }
}

__device__ inline double ic0_dot(const double* a, const double* b, int nn) {
  double part = 0.0;
  for (int i = threadIdx.x; i < nn; i += 64) part += a[i] * b[i];
  return wave_sum(part);
}

__global__ __launch_bounds__(64) void k_ic0_pcg(PcgGeom g, PcgElem el, int op, long nel,
                                                 const double* A, const double* U, const int* lv,
                                                 int nfw, int nbw, const double* b, double* x,
                                                 double rtol, int maxit, int* its, int* fail) {
  // six vectors of nn doubles in LDS, sized to the element so that more elements fit a CU
  extern __shared__ double ic0_lds[];
  const int nn = g.nn;
  double* sx = ic0_lds;
  double* sr = sx + nn;
  double* sz = sr + nn;
  double* sd = sz + nn;
  double* sq = sd + nn;
  double* sy = sq + nn;
  const long e = blockIdx.x;
  if (e >= nel) return;
  // level tables: forward rows [nn], forward starts [nfw + 1], backward rows, starts
  const int* fw = lv;
  const int* fws = lv + nn;
  const int* bw = fws + nfw + 1;
  const int* bws = bw + nn;
  const double* Ae = A + e * (long)g.nst;
  const double* Ue = U + e * (long)g.nst;
  const double* w = op == 0 ? el.w + e * nn : nullptr;
  const double cw = el.sc[e * 8 + 0];
  const double* be = b + e * nn;
  for (int i = threadIdx.x; i < nn; i += 64) {
    sx[i] = 0.0;
    sr[i] = be[i];
  }
  __syncthreads();
  const double nb = sqrt(ic0_dot(sr, sr, nn));
  int it = 0;
  bool conv = nb == 0.0;
  if (!conv) {
    ic0_apply(g, Ue, fw, fws, nfw, bw, bws, nbw, sr, sy, sz);
    for (int i = threadIdx.x; i < nn; i += 64) sd[i] = sz[i];
    __syncthreads();
    double rz = ic0_dot(sr, sz, nn);
    while (it < maxit) {
      ++it;
      ic0_product(g, Ae, w, cw, sd, sq);
      const double alpha = rz / ic0_dot(sd, sq, nn);
      for (int i = threadIdx.x; i < nn; i += 64) {
        sx[i] += alpha * sd[i];
        sr[i] -= alpha * sq[i];
      }
      __syncthreads();
      if (sqrt(ic0_dot(sr, sr, nn)) <= rtol * nb) {
        conv = true;
        break;
      }
      ic0_apply(g, Ue, fw, fws, nfw, bw, bws, nbw, sr, sy, sz);
      const double rzn = ic0_dot(sr, sz, nn);
      const double beta = rzn / rz;
      rz = rzn;
      for (int i = threadIdx.x; i < nn; i += 64) sd[i] = sz[i] + beta * sd[i];
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < nn; i += 64) x[e * nn + i] = sx[i];
  if (threadIdx.x == 0) {
    its[e] = it;
    if (!conv) atomicMin(fail, (int)e);
  }
}

}  // namespace

void ic0_levels(int N, int p, std::vector<int>& lv, int* nfw, int* nbw) {
  const int n1 = N + 1, nn = n1 * n1;
  std::vector<int> lf(nn, 0), lb(nn, 0);
  for (int i = 0; i < nn; ++i) {  // U^T y = r: row i needs the rows k < i of its stencil
    const int ix = i % n1, iy = i / n1;
    int m = -1;
    for (int ky = st_lo(iy, p); ky <= iy; ++ky)
      for (int kx = st_lo(ix, p); kx <= st_hi(ix, p, N); ++kx)
        if (ky < iy || kx < ix) m = std::max(m, lf[ky * n1 + kx]);
    lf[i] = m + 1;
  }
  for (int i = nn - 1; i >= 0; --i) {  // U z = y: row i needs the rows j > i of its stencil
    const int ix = i % n1, iy = i / n1;
    int m = -1;
    for (int jy = iy; jy <= st_hi(iy, p, N); ++jy)
      for (int jx = st_lo(ix, p); jx <= st_hi(ix, p, N); ++jx)
        if (jy > iy || jx > ix) m = std::max(m, lb[jy * n1 + jx]);
    lb[i] = m + 1;
  }
  auto sets = [&](const std::vector<int>& l, int* nl) {
    const int L = *std::max_element(l.begin(), l.end()) + 1;
    std::vector<int> rows, start(1, 0);
    for (int k = 0; k < L; ++k) {
      for (int i = 0; i < nn; ++i)
        if (l[i] == k) rows.push_back(i);
      start.push_back((int)rows.size());
    }
    lv.insert(lv.end(), rows.begin(), rows.end());
    lv.insert(lv.end(), start.begin(), start.end());
    *nl = L;
  };
  lv.clear();
  sets(lf, nfw);
  sets(lb, nbw);
}

hipError_t launch_ic0(const PcgGeom& g, const PcgElem& el, int op, long nel, double* A, double* U,
                      const int* lv, int nfw, int nbw, const double* b, double* x, double rtol,
                      int maxit, int* its, int* bad, int* fail, hipStream_t st) {
  if (g.nn > kIc0MaxNodes) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ic0_prepare, dim3((unsigned)nel), dim3(256), 0, st, g, el, op, nel, A, U);
  hipLaunchKernelGGL(k_ic0_factor, dim3((unsigned)nel), dim3(256), 0, st, g, nel, U, bad);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_ic0_pcg, dim3((unsigned)nel), dim3(64), 6 * (size_t)g.nn * sizeof(double), st,
                     g, el, op, nel, A, U, lv, nfw, nbw, b, x, rtol, maxit, its, fail);
  return hipGetLastError();
}

}  // namespace gdw
