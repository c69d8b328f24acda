// Small MLP (learned preconditioner correction): parameters, workspaces, kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "pcg.h"

namespace gdw {

struct MlpNet {
  int n_in, hidden, n_out;
  long np;                          // number of parameters
  long oW1, ob1, oW2, ob2, oW3, ob3;  // offsets in the flat parameter vector
  float* th;                        // FP32 master parameters
  float* g;                         // gradient
  float* m;                         // Adam moments
  float* v;
  _Float16* w16;                    // FP16 copy used by the forward products
  long step;                        // Adam step count
};

struct MlpWork {
  int bmax;
  float *z1, *h1, *z2, *h2, *dh, *dz, *out, *dout;
  double* part;                     // [64] loss partial sums
  double* loss;                     // [epochs] accumulated losses
  int loss_len;
};

hipError_t mlp_forward(const MlpNet& net, const float* x, int B, MlpWork& w, hipStream_t st);
hipError_t mlp_backward(const MlpNet& net, const float* x, const float* y, int B, MlpWork& w,
                        double* loss_acc, hipStream_t st);
hipError_t mlp_adam(MlpNet& net, float lr, hipStream_t st);
hipError_t mlp_refresh_half(MlpNet& net, hipStream_t st);
hipError_t launch_precond_data(const PcgGeom& g, const PcgElem& el, const double* c2n, const double* Bs,
                               float* samples, float* targets, long nel, hipStream_t st);
hipError_t launch_set_dlog(const float* out, long nel, int nn, float* dlog, double* dscale,
                           hipStream_t st);
// p[0 .. n) = 0 (a kernel, so that it may be captured into a graph)
hipError_t launch_zero_f64(double* p, long n, hipStream_t st);

}  // namespace gdw
