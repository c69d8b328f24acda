// Learned correction of the tensor-product PCG preconditioner (not in the paper).
//
// A multilayer perceptron 64 -> H -> H -> K (ReLU) maps the standardised coefficient
// samples of an element ((c^2 - 1)/0.5 at the centres of an 8 x 8 subdivision of the
// reference square) to K = (N+1)^2 - 1 log-multipliers of the modal diagonal D of the
// S_hat preconditioner.  Weights are FP16 in the forward products (FP32 accumulation
// on the matrix cores, v_mfma_f32_16x16x16_f16); the backward products run on
// v_mfma_f32_16x16x4_f32 in FP32; Adam keeps FP32 master weights.
//
// Training data comes from the solver's own assembled operators: inputs = the
// coefficient samples, targets = log(d_k / D_k) with d = diag(Psi_2^T S_hat Psi_2).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cmath>

#include "mlp.h"
#include "stencil.h"

namespace gdw {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// C[m][n] (row-major, ldc) = sum_k A(m,k) B(k,n) (+ bias[n]), A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn].  One wave per 16 x 16 tile, 4 waves per workgroup.
// F16: A (FP32 in memory) and B (FP16 in memory) are fed to v_mfma_f32_16x16x16_f16;
// otherwise both are FP32 (v_mfma_f32_16x16x4_f32).  Out-of-range rows/cols/k read 0.
template <bool F16, typename TB>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A,
                                              long sam, long sak, const TB* __restrict__ B,
                                              long sbk, long sbn, const float* __restrict__ bias,
                                              float* __restrict__ C, long ldc, float* __restrict__ Crelu) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tiles_n = (N + 15) / 16;
  const int tile = blockIdx.x * 4 + wv;
  const int tm = tile / tiles_n, tn = tile - (tile / tiles_n) * tiles_n;
  if (tm * 16 >= M) return;                       // whole wave leaves together
  const int r = lane & 15, kb = lane >> 4;        // row (A) / column (B) index, k block
  const int m = tm * 16 + r, n = tn * 16 + r;
  float4_t acc = {0.f, 0.f, 0.f, 0.f};
  if constexpr (F16) {
    for (int k0 = 0; k0 < K; k0 += 16) {
      half4_t a, b;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int k = k0 + 4 * kb + h;
        a[h] = (_Float16)((m < M && k < K) ? A[m * sam + k * sak] : 0.f);
        b[h] = (_Float16)((n < N && k < K) ? (float)B[k * sbk + n * sbn] : 0.f);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, acc, 0, 0, 0);
    }
  } else {
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + kb;
      const float a = (m < M && k < K) ? A[m * sam + k * sak] : 0.f;
      const float b = (n < N && k < K) ? (float)B[k * sbk + n * sbn] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
  }
  // D layout: lane holds column (lane & 15) of rows 4*(lane >> 4) + v
  const int col = tn * 16 + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = tm * 16 + 4 * (lane >> 4) + v;
    if (row < M && col < N) {
      const float z = acc[v] + (bias ? bias[col] : 0.f);
      C[row * ldc + col] = z;
      if (Crelu) Crelu[row * ldc + col] = z > 0.f ? z : 0.f;
    }
  }
}

template <bool F16, typename TB>
static hipError_t gemm(int M, int N, int K, const float* A, long sam, long sak, const TB* B, long sbk,
                       long sbn, const float* bias, float* C, long ldc, float* Crelu, hipStream_t st) {
  const long tiles = (long)((M + 15) / 16) * ((N + 15) / 16);
  if (tiles == 0) return hipSuccess;
  hipLaunchKernelGGL((k_gemm<F16, TB>), dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st, M, N, K,
                     A, sam, sak, B, sbk, sbn, bias, C, ldc, Crelu);
  return hipGetLastError();
}

// dout = 2 (out - y) / (B K); per-block partial sums of (out - y)^2
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out, const float* __restrict__ y,
                                             long n, float scale, float* __restrict__ dout,
                                             double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float d = out[i] - y[i];
    dout[i] = scale * d;
    s += (double)d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss = sum(part) / n, added into acc[slot] (fixed order)
__global__ void k_loss_acc(const double* __restrict__ part, int np, double inv_n,
                           double* __restrict__ acc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < np; ++i) s += part[i];
  acc[0] += s * inv_n;
}

__global__ void k_relu_back(const float* __restrict__ dh, const float* __restrict__ z, long n,
                            float* __restrict__ dz) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dz[i] = z[i] > 0.f ? dh[i] : 0.f;
}

// db[j] = sum_i dz[i][j]  (thread per column, fixed order)
__global__ void k_colsum(const float* __restrict__ dz, int rows, int cols, float* __restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int i = 0; i < rows; ++i) s += dz[(long)i * cols + j];
  db[j] = s;
}

// Adam on the FP32 master parameters; refresh the FP16 copy of the weights
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long n, float lr, float b1, float b2, float eps,
                       float c1, float c2, _Float16* __restrict__ th16) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float t = th[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  th[i] = t;
  th16[i] = (_Float16)t;
}

__global__ void k_zero_f64(double* __restrict__ p, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void k_to_half(const float* __restrict__ a, long n, _Float16* __restrict__ b) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (_Float16)a[i];
}

// ---------------------------------------------------------------------------------
// Network passes
// ---------------------------------------------------------------------------------
static inline unsigned nb(long n) { return (unsigned)((n + 255) / 256); }

hipError_t mlp_forward(const MlpNet& net, const float* x, int B, MlpWork& w, hipStream_t st) {
  const int I = net.n_in, H = net.hidden, K = net.n_out;
  hipError_t e;
  if ((e = gemm<true, _Float16>(B, H, I, x, I, 1, net.w16 + net.oW1, 1, I, net.th + net.ob1, w.z1, H, w.h1, st)) != hipSuccess) return e;
  if ((e = gemm<true, _Float16>(B, H, H, w.h1, H, 1, net.w16 + net.oW2, 1, H, net.th + net.ob2, w.z2, H, w.h2, st)) != hipSuccess) return e;
  return gemm<true, _Float16>(B, K, H, w.h2, H, 1, net.w16 + net.oW3, 1, H, net.th + net.ob3, w.out, K, nullptr, st);
}

// gradient of mean((out - y)^2) into net.g; adds the batch loss to *loss_acc
hipError_t mlp_backward(const MlpNet& net, const float* x, const float* y, int B, MlpWork& w,
                        double* loss_acc, hipStream_t st) {
  const int I = net.n_in, H = net.hidden, K = net.n_out;
  hipError_t e;
  const long nout = (long)B * K;
  const int np = 64;
  hipLaunchKernelGGL(k_mse, dim3(np), dim3(256), 0, st, w.out, y, nout, 2.f / (float)nout, w.dout, w.part);
  hipLaunchKernelGGL(k_loss_acc, dim3(1), dim3(64), 0, st, w.part, np, 1.0 / (double)nout, loss_acc);
  // layer 3: dW3 = dout^T h2, db3 = colsum(dout), dh2 = dout W3
  if ((e = gemm<false, float>(K, H, B, w.dout, 1, K, w.h2, H, 1, nullptr, net.g + net.oW3, H, nullptr, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3(nb(K)), dim3(256), 0, st, w.dout, B, K, net.g + net.ob3);
  if ((e = gemm<false, _Float16>(B, H, K, w.dout, K, 1, net.w16 + net.oW3, H, 1, nullptr, w.dh, H, nullptr, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_relu_back, dim3(nb((long)B * H)), dim3(256), 0, st, w.dh, w.z2, (long)B * H, w.dz);
  // layer 2
  if ((e = gemm<false, float>(H, H, B, w.dz, 1, H, w.h1, H, 1, nullptr, net.g + net.oW2, H, nullptr, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3(nb(H)), dim3(256), 0, st, w.dz, B, H, net.g + net.ob2);
  if ((e = gemm<false, _Float16>(B, H, H, w.dz, H, 1, net.w16 + net.oW2, H, 1, nullptr, w.dh, H, nullptr, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_relu_back, dim3(nb((long)B * H)), dim3(256), 0, st, w.dh, w.z1, (long)B * H, w.dz);
  // layer 1
  if ((e = gemm<false, float>(H, I, B, w.dz, 1, H, x, I, 1, nullptr, net.g + net.oW1, I, nullptr, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3(nb(H)), dim3(256), 0, st, w.dz, B, H, net.g + net.ob1);
  return hipGetLastError();
}

hipError_t mlp_adam(MlpNet& net, float lr, hipStream_t st) {
  net.step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)net.step), c2 = 1.f - powf(b2, (float)net.step);
  hipLaunchKernelGGL(k_adam, dim3(nb(net.np)), dim3(256), 0, st, net.th, net.g, net.m, net.v, net.np,
                     lr, b1, b2, eps, c1, c2, net.w16);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_f64, dim3(nb(n)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t mlp_refresh_half(MlpNet& net, hipStream_t st) {
  hipLaunchKernelGGL(k_to_half, dim3(nb(net.np)), dim3(256), 0, st, net.th, net.np, net.w16);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Training data from the assembled element operators and inference into dlog
// ---------------------------------------------------------------------------------
// samples[e][64]: (c^2 - 1)/0.5 at the 8 x 8 centres (Bs[s][i]: basis at centre s);
// targets[e][nn-1]: log(d_k / D_k), d_k = psi_k^T S_hat psi_k (k >= 1).
__global__ __launch_bounds__(256) void k_precond_data(PcgGeom g, PcgElem el, const double* __restrict__ c2n,
                                                      const double* __restrict__ Bs,
                                                      float* __restrict__ samples,
                                                      float* __restrict__ targets, long nel) {
  const long e = blockIdx.x;
  if (e >= nel) return;
  const int t = threadIdx.x, n1 = g.n1, nn = g.nn, N = g.N, p = g.p;
  __shared__ double Psi[32 * 32];
  for (int i = t; i < nn; i += blockDim.x) Psi[i] = g.Psi[i];
  __syncthreads();
  if (t < 64 && samples) {
    const int sx = t % 8, sy = t / 8;
    double c = 0.0;
    for (int iy = 0; iy < n1; ++iy)
      for (int ix = 0; ix < n1; ++ix) c += Bs[sy * n1 + iy] * Bs[sx * n1 + ix] * c2n[e * nn + iy * n1 + ix];
    samples[e * 64 + t] = (float)((c - 1.0) / 0.5);
  }
  if (!targets) return;
  const double* S = el.S + e * g.nst;
  const double* sc = el.sc + e * 8;
  for (int k = t; k < nn; k += blockDim.x) {
    const int kx = k % n1, ky = k / n1;
    // psi_k(i) = Psi[iy][ky] Psi[ix][kx];  d = psi^T S psi + cw (w^T psi)^2
    double d = 0.0, wp = 0.0;
    int h = 0;
    for (int iy = 0; iy < n1; ++iy)
      for (int ix = 0; ix < n1; ++ix) {
        const double pi = Psi[iy * n1 + ky] * Psi[ix * n1 + kx];
        wp += el.w[e * nn + iy * n1 + ix] * pi;
        const int xh = st_hi(ix, p, N), xl = st_lo(ix, p), yh = st_hi(iy, p, N);
        double rs = S[h] * pi;                    // diagonal entry
        ++h;
        for (int jx = ix + 1; jx <= xh; ++jx) rs += 2.0 * S[h++] * Psi[iy * n1 + ky] * Psi[jx * n1 + kx];
        for (int jy = iy + 1; jy <= yh; ++jy) {
          const double py = Psi[jy * n1 + ky];
          for (int jx = xl; jx <= xh; ++jx) rs += 2.0 * S[h++] * py * Psi[jx * n1 + kx];
        }
        d += pi * rs;
      }
    d += sc[0] * wp * wp;
    if (k == 0) continue;
    const double D = sc[1] * g.lamr[kx] + sc[2] * g.lamr[ky];
    targets[e * (nn - 1) + k - 1] = (float)log(d / D);
  }
}

// dlog[e][0] = 0, dlog[e][k] = sanitised out[e][k-1]: non-finite -> 0 (plain), |o| <= 8;
// dscale = exp(dlog)
__global__ void k_set_dlog(const float* __restrict__ out, long nel, int nn, float* __restrict__ dlog,
                           double* __restrict__ dscale) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nel * nn) return;
  const long e = i / nn;
  const int k = (int)(i - e * nn);
  float o = k == 0 ? 0.f : out[e * (nn - 1) + k - 1];
  if (!isfinite(o)) o = 0.f;
  o = fminf(fmaxf(o, -8.f), 8.f);
  dlog[i] = o;
  dscale[i] = exp((double)o);
}

hipError_t launch_precond_data(const PcgGeom& g, const PcgElem& el, const double* c2n, const double* Bs,
                               float* samples, float* targets, long nel, hipStream_t st) {
  if (nel == 0) return hipSuccess;
  hipLaunchKernelGGL(k_precond_data, dim3((unsigned)nel), dim3(256), 0, st, g, el, c2n, Bs, samples,
                     targets, nel);
  return hipGetLastError();
}

hipError_t launch_set_dlog(const float* out, long nel, int nn, float* dlog, double* dscale,
                           hipStream_t st) {
  const long n = nel * nn;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_dlog, dim3(nb(n)), dim3(256), 0, st, out, nel, nn, dlog, dscale);
  return hipGetLastError();
}

}  // namespace gdw
