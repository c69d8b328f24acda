// Variable-coefficient / mapped-element path: element assembly by quadrature and the
// fused RK stage with PCG element solves (Sec. 7.1).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace gdw {

// Per-element PCG counters: sum of S_hat iterations, sum of M_J iterations, largest of each,
// sum of refinement sweeps of each (mixed precision).
constexpr int kItsPer = 6;

// Tables shared by every element of a problem (device pointers).
struct PcgGeom {
  int N, p, n1, nn, m, nq, nst;
  const int* rowoff;    // [nn+1] start of each row's upper part (stencil.h)
  const int* cs;        // [N] first node of cell k's window
  const int* ck0;       // [n1] first cell whose window holds node i
  const int* ck1;       // [n1] last such cell
  const double* cb;     // [N][m][m] window function j at Gauss point a of cell k
  const double* cd;     // [N][m][m] its derivative d/dr (reference spacing 1/N)
  const double* gw;     // [m] Gauss weights on [0, 1]
  const double* dL;     // [n1] d/dr of the basis at r = 0
  const double* dR;     // [n1] d/dr of the basis at r = 1
  const double* Psi;    // [n1*n1] reference eigenbasis, Psi[i*n1 + k], Psi^T M_ref Psi = I
  const double* lamr;   // [n1] reference eigenvalues (lamr[0] = 0)
  const double* Mref;   // [n1*n1] 1D mass matrix on [0, 1] (Cartesian M_J = area Mref (x) Mref)
};

// Per-element data (device pointers).
struct PcgElem {
  double* S;            // [nel][nst] upper half of S_K
  double* M;            // [nel][nst] upper half of M_J (mapped meshes only)
  float* Shi;           // [nel][nnz_blk] mixed precision: fl32(S_K), column-block layout
  float* Slo;           // [nel][nnz_blk] fl32(S_K - Shi)
  float* Mhi;           // the same for M_J (mapped meshes)
  float* Mlo;
  double* w;            // [nel][nn] int phi_i J
  double* sc;           // [nel][8]: kappa/area, kbar_rr, kbar_ss, kappa*area, area, int c^2 J
  double* face;         // [nel][4][nq][3]: (K Nh)_r, (K Nh)_s, c^2 s_J at face points
  float* dlog;          // [nel][nn] log-scale of the S preconditioner diagonal (NULL: plain)
  double* dscale;       // [nel][nn] exp(dlog), set with dlog
  double* Sreg;         // register kernels: S_K in work-unit slot order,
  double* Mreg;         // [nel][slots][blk_threads] (0 in padding slots); M_J alike
  double* msc;          // [nel][nn] nodal scale of the M_J preconditioner (mapped meshes)
};

struct PcgStageArgs {
  PcgGeom g;
  PcgElem el;
  const double* in_u;   // stage input (nodal)
  const double* in_v;
  const double* aux_u;  // y (stages 2, 3) or the accumulator (stage 4)
  const double* aux_v;
  double* out_u;
  double* out_v;
  double* acc_u;        // stage 2 only
  double* acc_v;
  const double* tr_in;  // [nel][4][nq][2] (a, v) at face points of the stage input
  double* tr_out;
  double* xS;           // [nel][nn] warm start / solution of S_hat y = F_u
  double* xM;           // [nel][nn] warm start / solution of M_J z = r
  double* Fu;           // split stage: [nel][nn] F_u of the lift kernel
  double* Fv;           // split stage: [nel][nn] F_v, replaced by r = F_v - S_K U
  int* its;             // [nel][4]: sum S iterations, sum M iterations, max S, max M
  int* fail;            // smallest element id that hit maxit (0x7f7f7f7f if none)
  long nel;
  int nx, ny;
  int bcbits;           // gdw_bc of side f (0 E, 1 W, 2 N, 3 S) in bits 2f, 2f+1; 0: periodic
  int mapped;
  double dt, beta, tau, rtol, rtol_inner;
  double alf[4];        // alpha of Sec. 2.2.1 on the E, W, N, S faces (1/2 on wall faces)
  int maxit;
  int mixed;            // 1: FP32 operator for the inner PCG, FP64 residual refinement
  int pc32;             // 1: the preconditioner's transforms in FP32 inside the FP64 PCG
  const int* fo;        // [nn+1] row starts of the full stencil rectangles
  const int* dst;       // [nst][2] full-rectangle positions (i,j), (j,i) of upper entry h
  int full, Q, nnz_full;  // set by the launcher: LDS layout of the operator
  // column-block layout (N + 1 in {9, 13, 17}; see pcg.hip); v2 = 0 selects the row layout
  int v2;
  const int* blk_off;   // [nn] start of block (ix, jy) at index jy*(N+1) + ix
  const int* blk_dst;   // [nst][2] block-layout positions of upper entry h and its transpose
  const int* blk_jc;    // [blk_K] work units jy | (c << 8)
  const int* blk_gidx;  // register kernels: [CH * W][blk_threads] upper-half index of each
                        // unit entry (-1: padding)
  const int* blk_unit;  // streamed family: unit k * (N + 1) + ix of each thread (threads in
                        // order of the units' widths); nullptr: thread t is unit t
  int blk_K, blk_CH, blk_WB, blk_threads;
  // source term: nf nodal fields g_k at frc + k * frc_stride; dv/dt gains
  // sum_k f_w[4 (stage - 1) + k] g_k, the weights of the current step (written by
  // launch_source_step before the step's four stages)
  const double* frc;
  long frc_stride;
  int nf;
  const double* f_w;
};

struct SourceTerms {
  int nf;
  double omega[4], phase[4];
};

// One lane, before each RK4 step of the PCG path: the weights
// w[4 (s - 1) + k] = sin(omega_k (t + c_s dt) + phase_k) of the step's stages s = 1..4
// (c = 0, 1/2, 1/2, 1) from the device clock t = *t_dev, then t += dt.
hipError_t launch_source_step(double* t_dev, double* w, double dt, const SourceTerms& f,
                              hipStream_t st);
// Set the device clock to t and clear the 16 weights after it (one lane, stream-ordered).
hipError_t launch_set_clock(double* t_dev, double t, hipStream_t st);

// Column-block layout tables for one geometry; returns 0 when the layout does not apply
// (N + 1 not in {9, 13, 17}, or LDS or block size exceeded).  rowoff: upper-half row starts.
int pcg_block_tables(const PcgGeom& g, const std::vector<int>& rowoff, std::vector<int>& boff,
                     std::vector<int>& dst, std::vector<int>& jc, std::vector<int>& gidx,
                     std::vector<int>& unit, int* K, int* CH, int* WB, int* nnz, int* threads,
                     int mixed);
// FP32 hi / lo split of the upper-half operators into the column-block layout.
// Work-unit slots per thread (CH x W) of the register kernels, which load their entries from
// a slot-ordered copy of the operator; 0 for the other kernel families.
int pcg_reg_slots(int n1, int p);
// Nodal scale of the M_J preconditioner of every element into el.msc (needs el.M, el.sc).
hipError_t launch_mscale(const PcgGeom& g, const PcgElem& el, long nel, hipStream_t st);
// out[e][s][t] = half[e][gidx[s * threads + t]] (0 where gidx < 0), for every element.
hipError_t launch_reg_permute(const double* half, const int* gidx, int nst, int slots,
                              int threads, long nel, double* out, hipStream_t st);
hipError_t launch_split_hilo(const double* half, const int* dst, int nst, int nnz, long nel,
                             float* hi, float* lo, hipStream_t st);

hipError_t launch_assemble(const PcgGeom& g, const double* X, const double* Y, const double* C2,
                           const PcgElem& el, long nel, hipStream_t st);
hipError_t launch_face_geom(const PcgGeom& g, const double* X, const double* Y, const double* C2,
                            const PcgElem& el, long nel, hipStream_t st);
hipError_t launch_to_f32(const double* a, float* b, long n, hipStream_t st);
hipError_t launch_pcg_traces(const PcgGeom& g, const PcgElem& el, const double* U, const double* V,
                             double* tr, long nel, hipStream_t st);
// Kernel family of a problem for the grouped launch: N + 1 for the column-block layout,
// 0 for the row layout.
// Key of the grouped stage kernel for a problem: 0 (row layout), N + 1 (column blocks),
// N + 1 + 32 (mixed), or N + 1 + 64 + 128 p (FP64 operator held in registers).
int pcg_family_key(int n1, int p, int v2, int mixed);
int pcg_group_key(const PcgStageArgs& a);
// Block size and LDS of a problem launched alone (sets full / Q / nnz_full of the row
// layout); 0 if it does not fit a workgroup.
int pcg_single_shape(PcgStageArgs& a, int* threads, size_t* lds);
// Split stage of the register-operator families (key with bit 64, FP64), one problem:
// lifts (F_u, F_v), the S_hat solve (with r = F_v - S_K U and, on Cartesian elements, the
// exact M_J solve), the M_J solve (mapped elements) and the RK update with the new traces.
// a: device copy of the stage's arguments (Fu, Fv set); threads / lds from
// pcg_single_shape.
hipError_t launch_pcg_split_stage(int stage, int key, const PcgStageArgs* a, const PcgStageArgs& h,
                                  int threads, size_t lds, hipStream_t st);
// The same over a group of problems of one family (all members share N, p and the block
// layout; h is the host copy of a member's arguments): the lifts, the S_hat solves and the
// updates walk the nprob members of args (member k owns elements el_start[k] ..
// el_start[k + 1] - 1; h_el_start is the host copy of that table); the M_J solves walk the
// nprob_m members of args_m (the mapped ones, with their own tables; none if 0).
hipError_t launch_pcg_split_group(int stage, int key, const PcgStageArgs* args,
                                  const long* el_start, const long* h_el_start, int nprob,
                                  const PcgStageArgs* args_m, const long* el_start_m,
                                  const long* h_el_start_m, int nprob_m, const PcgStageArgs& h,
                                  int threads, hipStream_t st);
bool pcg_split_key(int key);
// Families that offer the preconditioner's transforms in FP32 (GDW_MIXED_PC32): the FP64
// register families on the wave-0 solve kernels (N + 1 <= 16, 64 + blk_threads <= 512).
bool pcg_pc32_supported(int n1, int p, int blk_threads);
// Persistent grid of the grouped kernel of family `key` for nel elements.
unsigned pcg_group_grid(int stage, int key, int threads, size_t lds, long nel);
size_t pcg_stage_lds_bytes(const PcgGeom& g, int mixed);
// LDS layout of the stage kernel for a block of `threads` threads: full-rectangle operator
// or not, row split Q, full operator size and LDS bytes.
void pcg_stage_shape(const PcgGeom& g, int threads, int* full, int* Q, int* nnz_full, size_t* lds);
// Layout of a problem's stage for a block of `threads` threads (row layout: sets full, Q,
// nnz_full); *lds = its LDS bytes.  Returns 0 if `threads` is too small for it.
int pcg_args_shape(PcgStageArgs& a, int threads, size_t* lds);
// Grouped persistent stage launch over several problems of one kernel family `key` (args
// in device memory, each shaped by pcg_args_shape for `threads`; lds >= every member's
// need).  A single problem is the group of one.
hipError_t launch_pcg_stage_group(int stage, int key, const PcgStageArgs* args, const long* el_start,
                                  int nprob, unsigned grid, int threads, size_t lds, hipStream_t st);
// Largest block size of the grouped stage kernel of family `key`.
int pcg_group_max_threads(int key);
// Allow the grouped stage kernels their full LDS (call before any graph capture).
hipError_t pcg_group_prepare();
hipError_t launch_pcg_energy(const PcgGeom& g, const PcgElem& el, const double* U, const double* V,
                             long nel, double* part, int npart, double* out, hipStream_t st);

}  // namespace gdw
