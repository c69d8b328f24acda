// Kernel launchers of the constant-coefficient (simultaneous diagonalisation) path.
#pragma once

#include <hip/hip_runtime.h>

namespace gdw {

// Arguments of one fused RK stage (see fdm.hip for the stage-by-stage roles).
template <typename T>
struct StageArgs {
  const T* in_u;       // stage input, modal
  const T* in_v;
  const T* aux_u;      // y (stages 2, 3) or the accumulator (stage 4); unused in stage 1
  const T* aux_v;
  T* out_u;            // new stage value (may alias in_u for stages 2, 3)
  T* out_v;
  T* acc_u;            // stage 2 only: accumulator Yin + 2 Ynew - y
  T* acc_v;
  const T* tr_in;      // modal traces of the stage input, [nel][8][n1]
  T* tr_out;           // modal traces of the new stage value
  const T* invL;       // [n1*n1]: 1 / (lambda_x + lambda_y), entry (0,0) = 1
  const T* lam;        // [n1*n1]: lambda_x + lambda_y
  const T* gh;         // [8][n1]: gE hE gW hW gN hN gS hS
  long nel;
  int nx, ny, n1;
  int bcbits;          // gdw_bc of side f (0 E, 1 W, 2 N, 3 S) in bits 2f, 2f+1; 0: periodic
  T dt, c2, alpha, beta, tau;
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
template <typename T>
hipError_t launch_traces(const T* Ub, const T* Vb, const T* gh, T* tr, int n1, long nel,
                         hipStream_t st);
template <typename T>
hipError_t launch_stage(int stage, const StageArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_energy(const T* Ub, const T* Vb, const T* lam, double c2, int n1, long nel,
                         double* part, int npart, double* out, hipStream_t st);
template <typename T>
hipError_t launch_count_nonfinite(const T* a, long n, unsigned int* cnt, hipStream_t st);

// Grouped persistent stage launch over several problems of one class (T, n1, epb):
// args[i] are problem i's stage arguments (device memory), problem i owns tiles
// [tile_start[i], tile_start[i+1]) of epb elements; `grid` blocks stride over all tiles.
template <typename T>
hipError_t launch_stage_group(int stage, int n1, int epb, const StageArgs<T>* args,
                              const long* tile_start, int nprob, unsigned grid, hipStream_t st);
size_t stage_lds_bytes(int elem_bytes, int n1, int epb);
// Resident blocks per CU of the grouped stage kernel (LDS and thread limits).
template <typename T>
int stage_group_occupancy(int stage, int n1, int epb);

}  // namespace gdw
