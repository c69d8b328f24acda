// Kernel launchers of the constant-coefficient (simultaneous diagonalisation) path.
#pragma once

#include <hip/hip_runtime.h>

namespace gdw {

// Arguments of one fused RK stage (see fdm.hip for the stage-by-stage roles).  T is the
// storage type of the stage registers and traces; the arithmetic is FP64 in both modes.
template <typename T>
struct StageArgs {
  const T* in_u;       // stage input, modal (FP32 storage: the stage increment)
  const T* in_v;
  const T* aux_u;      // y (stages 2, 3) or the accumulator (stage 4); unused in stage 1
  const T* aux_v;
  T* out_u;            // new stage value (may alias in_u for stages 2, 3)
  T* out_v;
  T* acc_u;            // stage 2 only: accumulator Yin + 2 Ynew - y (FP32: dY2 + 2 dY3)
  T* acc_v;
  double* y64_u;       // FP32 storage only: the FP64 register y, read by every stage and
  double* y64_v;       // written by stage 4 (in, aux and out then hold FP32 increments)
  const T* tr_in;      // modal traces of the stage input, [nel][8][n1]
  T* tr_out;           // modal traces of the new stage value
  const double* invL;  // [n1^d]: 1 / (sum of the directions' lambdas), entry 0 = 1
  const double* lam;   // [n1^d]: lambda_x + lambda_y (+ lambda_z)
  const double* gh;    // [2d][2][n1]: gE hE gW hW gN hN gS hS (gT hT gB hB)
  long nel;
  int nx, ny, n1;
  int nz;              // 3D only: elements in z (element e = (ez ny + ey) nx + ex)
  int bcbits;          // gdw_bc of side f (0 E, 1 W, 2 N, 3 S, 4 T, 5 B) in bits 2f, 2f+1
  double dt, c2, beta, tau;
  double alf[6];       // alpha of Sec. 2.2.1 on the E, W, N, S, T, B faces (1/2 on walls)
  // source term: nf terms (0..4), modal g_k at frc + k * frc_stride; the weights
  // fw[4 (stage - 1) + k] = sin(omega_k t_stage + phase_k) of the current step sit in
  // device memory (written by launch_source_step before the step's stages)
  const T* frc;
  long frc_stride;
  int nf;
  const double* fw;
};

hipError_t launch_eig(const double* M, const double* S, int n, double* work, double* Psi,
                      double* lam, int* info, hipStream_t st);
template <typename T>
hipError_t launch_to_modal(const double* U, T* Ub, const double* Px, const double* Py, int n1,
                           long nel, hipStream_t st);
template <typename T>
hipError_t launch_to_nodal(const T* Ub, double* U, const double* Psx, const double* Psy, int n1,
                           long nel, hipStream_t st);
// Traces (type T) of a modal state (type S).
template <typename S, typename T>
hipError_t launch_traces(const S* Ub, const S* Vb, const double* gh, T* tr, int n1, long nel,
                         hipStream_t st);
template <typename T>
hipError_t launch_stage(int stage, const StageArgs<T>& a, hipStream_t st);
// nn: nodes per element (n1^2 in 2D, n1^3 in 3D)
template <typename T>
hipError_t launch_energy(const T* Ub, const T* Vb, const double* lam, double c2, int nn, long nel,
                         double* part, int npart, double* out, hipStream_t st);

// ---- box elements in 3D (modal state [e][kz][ky][kx], traces [e][12][n1^2]) ----------
// nodal (FP64) <-> modal with P = Psi^{-1} = Psi^T M per direction
template <typename T>
hipError_t launch_to_modal3(const double* U, T* Ub, const double* Px, const double* Py,
                            const double* Pz, int n1, long nel, hipStream_t st);
template <typename T>
hipError_t launch_to_nodal3(const T* Ub, double* U, const double* Psx, const double* Psy,
                            const double* Psz, int n1, long nel, hipStream_t st);
template <typename S, typename T>
hipError_t launch_traces3(const S* Ub, const S* Vb, const double* gh, T* tr, int n1, long nel,
                          hipStream_t st);
// one fused RK stage on box elements; n1^3 <= 1024
template <typename T>
hipError_t launch_stage3(int stage, const StageArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_count_nonfinite(const T* a, long n, unsigned int* cnt, hipStream_t st);

// Grouped persistent stage launch over several problems of one class (T, n1, epb):
// args[i] are problem i's stage arguments (device memory), problem i owns tiles
// [tile_start[i], tile_start[i+1]) of epb elements; `grid` blocks stride over all tiles.
template <typename T>
hipError_t launch_stage_group(int stage, int n1, int epb, const StageArgs<T>* args,
                              const long* tile_start, int nprob, unsigned grid, hipStream_t st);
// LDS of one stage workgroup (FP64 arithmetic in both storage modes).
size_t stage_lds_bytes(int n1, int epb);
// Resident blocks per CU of the grouped stage kernel (LDS and thread limits).
template <typename T>
int stage_group_occupancy(int stage, int n1, int epb);

}  // namespace gdw
