// Context of one problem (the opaque gdw_ctx of the C ABI) and the stage-argument
// builders shared by the single-problem time loop and the batched one.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/gdw.h"
#include "fdm.h"
#include "gdw_internal.h"
#include "pcg.h"

#define GDW_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t _e = (call);                                                               \
    if (_e != hipSuccess) {                                                               \
      set_error(std::string(#call) + ": " + hipGetErrorString(_e));                       \
      return _e == hipErrorOutOfMemory ? GDW_ENOMEM : GDW_EHIP;                           \
    }                                                                                     \
  } while (0)

// "no failure" value of the PCG failure slot (hipMemset byte 0x7f); element ids are smaller
static constexpr int kFailNone = 0x7f7f7f7f;

struct gdw_ctx {
  gdw_desc d{};
  int n1 = 0;
  int dim = 2;                 // 2 or 3
  int nn = 0;                  // nodes per element, n1^dim
  long nel = 0;
  size_t elem_bytes = 0;       // sizeof(T) of the time-loop arithmetic
  double alf[6] = {0, 0, 0, 0, 0, 0};   // alpha of the E, W, N, S, T, B faces (Sec. 2.2.1)
  double beta = 0, tau = 0;
  // device buffers (time-loop type T)
  void* Y[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  void* tr[2] = {nullptr, nullptr};
  double* y64[2] = {nullptr, nullptr};   // FP32 arithmetic: the FP64 accumulation register y
  void* invL = nullptr;
  void* lam = nullptr;
  void* gh = nullptr;
  // device FP64 tables for the nodal <-> modal maps
  double* Psx = nullptr;
  double* Psy = nullptr;
  double* Px = nullptr;
  double* Py = nullptr;
  double* Psz = nullptr;       // 3D: the z direction's tables
  double* Pz = nullptr;
  double* epart = nullptr;     // energy partial sums + result
  unsigned int* nonfinite = nullptr;
  int npart = 1024;
  int trc = 0;                 // trace buffer holding the traces of y
  long long steps_taken = 0;
  int have_state = 0;
  // source term (FDM path): nf modal fields g_k [nf][nel][n1^2] in the time-loop type,
  // f = sum_k sin(f_omega[k] t + f_phase[k]) g_k; t = time since the last set_state
  int nf = 0;
  void* frc = nullptr;
  double f_omega[4] = {0, 0, 0, 0};
  double f_phase[4] = {0, 0, 0, 0};
  double t = 0.0;
  double* t_dev = nullptr;     // PCG path: device clock t, then the step's stage weights [16]
  int solver = GDW_SOLVE_FDM;  // resolved solver
  // ---- PCG path ----
  gdw::PcgGeom g{};
  gdw::PcgElem el{};
  void* own[24] = {};          // device tables of g (freed with the context)
  double* xS = nullptr;
  double* xM = nullptr;
  double* Fu = nullptr;     // split PCG stage: lifts F_u, F_v (then r) of every element
  double* Fv = nullptr;
  int* its = nullptr;
  int* fail = nullptr;
  double* coords = nullptr;    // Cartesian X, Y, constant c^2 when not given
  int have_coeff = 0;
  long long stages_since_state = 0;
  double rtol = 1e-12;
  int maxit = 200;
  const int* fo = nullptr;     // full stencil row starts (device)
  const int* dst = nullptr;    // full-rectangle destinations of the upper entries (device)
  double* c2n = nullptr;       // nodal c^2 as given to set_coeff (network inputs)
  const double* Bs = nullptr;  // [8][n1] basis values at the 8 sample centres
  // column-block operator layout (pcg.hip), used when blk_v2 = 1
  int blk_v2 = 0;
  const int* blk_off = nullptr;
  const int* blk_dst = nullptr;
  const int* blk_jc = nullptr;
  const int* blk_gidx = nullptr;
  const int* blk_unit = nullptr;
  int blk_K = 0, blk_CH = 0, blk_WB = 0, blk_nnz = 0, blk_threads = 0;
  // stage arguments of the PCG time loop in device memory (the grouped kernel, one problem)
  gdw::PcgStageArgs* d_pargs = nullptr;   // [4]
  long* d_pel = nullptr;                  // {0, nel}
  gdw::PcgStageArgs h_pargs[4] = {};
  double pargs_dt = -1.0;
  int pargs_ok = 0;                       // h_pargs / d_pargs match the context
  int pargs_used = 0;                     // kernels reading d_pargs have been queued
  int args_epoch = 0;                     // bumped whenever stage arguments change
  int p_threads = 0;
  size_t p_lds = 0;
  // IC(0) baseline workspace (first gdw_ic0_solve call): operator entries and factor
  // [nel][nst], level tables of the triangular solves, breakdown / maxit flags
  double* ic0_A = nullptr;
  double* ic0_U = nullptr;
  int* ic0_lv = nullptr;
  int* ic0_flags = nullptr;
  int ic0_nfw = 0, ic0_nbw = 0;
};


namespace gdw {

// Stage arguments of RK stage `stage` (1..4) of a constant-coefficient context (its
// y / Y / accumulator registers and trace buffers; see fdm.hip for the roles).
template <typename T>
StageArgs<T> fdm_stage_args(const gdw_ctx* c, int stage, double dt);

// Stage arguments of RK stage `stage` of a PCG context (full / Q / nnz_full left 0: the
// launchers set them).
PcgStageArgs pcg_stage_args(const gdw_ctx* c, int stage, double dt);
// The source terms of a context (for launch_source_step).
SourceTerms source_terms(const gdw_ctx* c);

}  // namespace gdw
