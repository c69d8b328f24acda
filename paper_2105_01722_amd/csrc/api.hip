// C ABI of libgdw (declared in include/gdw.h): context management, table set-up and
// the RK4 time loop of the constant-coefficient path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

#include "ctx.h"
#include "fdm.h"
#include "gdw_internal.h"
#include "ic0.h"
#include "mlp.h"
#include "pcg.h"
#include "stencil.h"

namespace gdw {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace gdw

using namespace gdw;

static void free_all(gdw_ctx* c) {
  auto F = [](void* p) { if (p) (void)hipFree(p); };
  for (auto& r : c->Y) for (auto& p : r) F(p);
  F(c->tr[0]); F(c->tr[1]); F(c->invL); F(c->lam); F(c->gh); F(c->frc); F(c->t_dev);
  F(c->y64[0]); F(c->y64[1]);
  F(c->Psx); F(c->Psy); F(c->Px); F(c->Py); F(c->Psz); F(c->Pz); F(c->epart); F(c->nonfinite);
  for (auto& p : c->own) F(p);
  F(c->el.S); F(c->el.M); F(c->el.Shi); F(c->el.Slo); F(c->el.Mhi); F(c->el.Mlo);
  F(c->el.Sreg); F(c->el.Mreg); F(c->el.msc);
  F(c->el.w); F(c->el.sc); F(c->el.face);
  F(c->el.dlog); F(c->el.dscale); F(c->xS); F(c->xM); F(c->Fu); F(c->Fv); F(c->its); F(c->fail); F(c->coords); F(c->c2n);
  F(c->d_pargs); F(c->d_pel);
  F(c->ic0_A); F(c->ic0_U); F(c->ic0_lv); F(c->ic0_flags);
}

// The stage arguments derived from the context (pointers of the element data) changed.
static void args_changed(gdw_ctx* c) {
  c->pargs_ok = 0;
  ++c->args_epoch;
}

extern "C" const char* gdw_version(void) { return "gdw 0.1 (gfx950)"; }

extern "C" const char* gdw_last_error(void) { return g_last_error.c_str(); }

static gdw_status validate(const gdw_desc* d) {
  if (!d) { set_error("desc is NULL"); return GDW_EINVAL; }
  if (d->p < 1 || d->p % 2 == 0) { set_error("p must be odd and >= 1"); return GDW_EINVAL; }
  if (d->p > 31) { set_error("p > 31 is not supported"); return GDW_EINVAL; }
  if (d->N < d->p) { set_error("N must be >= p"); return GDW_EINVAL; }
  if (d->N + 1 > 32) { set_error("N + 1 must be <= 32"); return GDW_EINVAL; }
  if (d->nx < 1 || d->ny < 1) { set_error("nx, ny must be >= 1"); return GDW_EINVAL; }
  if (!(d->Lx > 0) || !(d->Ly > 0) || !std::isfinite(d->Lx) || !std::isfinite(d->Ly)) {
    set_error("Lx, Ly must be finite and > 0"); return GDW_EINVAL;
  }
  if (!(d->c2 > 0) || !std::isfinite(d->c2)) { set_error("c2 must be finite and > 0"); return GDW_EINVAL; }
  if (d->flux != GDW_FLUX_CENTRAL && d->flux != GDW_FLUX_UPWIND && d->flux != GDW_FLUX_ALTERNATING) {
    set_error("unknown flux"); return GDW_EINVAL;
  }
  if (d->flux == GDW_FLUX_UPWIND && (!(d->xi > 0) || !std::isfinite(d->xi))) {
    set_error("xi must be finite and > 0 for the upwind flux"); return GDW_EINVAL;
  }
  if (d->precision != GDW_FP64 && d->precision != GDW_MIXED_FP32 && d->precision != GDW_MIXED_PC32) {
    set_error("unknown precision");
    return GDW_EINVAL;
  }
  if (d->solver != GDW_SOLVE_AUTO && d->solver != GDW_SOLVE_FDM && d->solver != GDW_SOLVE_PCG) {
    set_error("unknown solver"); return GDW_EINVAL;
  }
  const bool general = d->coeff_variable || d->mapped;
  if (d->solver == GDW_SOLVE_FDM && general) {
    set_error("the FDM solve needs a constant c^2 on Cartesian elements"); return GDW_EINVAL;
  }
  for (int k = 0; k < 4; ++k)
    if (d->bc[k] != GDW_BC_PERIODIC && d->bc[k] != GDW_BC_DIRICHLET && d->bc[k] != GDW_BC_NEUMANN) {
      set_error("unknown boundary kind"); return GDW_EINVAL;
    }
  if ((d->bc[0] == GDW_BC_PERIODIC) != (d->bc[1] == GDW_BC_PERIODIC) ||
      (d->bc[2] == GDW_BC_PERIODIC) != (d->bc[3] == GDW_BC_PERIODIC)) {
    set_error("a direction is periodic on both of its sides or on neither"); return GDW_EINVAL;
  }
  const bool pcg = d->solver == GDW_SOLVE_PCG || general;
  if (d->dim != 0 && d->dim != 2 && d->dim != 3) { set_error("dim must be 2 or 3"); return GDW_EINVAL; }
  if (d->dim == 3) {
    if (d->nz < 1) { set_error("nz must be >= 1"); return GDW_EINVAL; }
    if (!(d->Lz > 0) || !std::isfinite(d->Lz) || !std::isfinite(d->z0)) {
      set_error("Lz must be finite and > 0"); return GDW_EINVAL;
    }
    for (int k = 0; k < 2; ++k)
      if (d->bcz[k] != GDW_BC_PERIODIC && d->bcz[k] != GDW_BC_DIRICHLET && d->bcz[k] != GDW_BC_NEUMANN) {
        set_error("unknown boundary kind"); return GDW_EINVAL;
      }
    if ((d->bcz[0] == GDW_BC_PERIODIC) != (d->bcz[1] == GDW_BC_PERIODIC)) {
      set_error("a direction is periodic on both of its sides or on neither"); return GDW_EINVAL;
    }
    if (pcg) {
      set_error("3D runs on the constant-coefficient Cartesian path only"); return GDW_EUNSUPPORTED;
    }
    if ((d->N + 1) * (d->N + 1) * (d->N + 1) > 1024) {
      set_error("3D needs (N + 1)^3 <= 1024 (one thread per modal index of an element)");
      return GDW_EUNSUPPORTED;
    }
    if (double(d->nx) * d->ny * d->nz * (d->N + 1) * (d->N + 1) * (d->N + 1) > 4.0e9) {
      set_error("problem too large"); return GDW_EINVAL;
    }
  }
  if (pcg && d->p > 7) { set_error("the PCG path supports p <= 7"); return GDW_EUNSUPPORTED; }
  if (!pcg && d->precision == GDW_MIXED_PC32) {
    set_error("GDW_MIXED_PC32 applies to the PCG path only");
    return GDW_EUNSUPPORTED;
  }
  if (!std::isfinite(d->pcg_rtol)) { set_error("pcg_rtol must be finite"); return GDW_EINVAL; }
  const double nel = double(d->nx) * d->ny * (d->N + 1) * (d->N + 1);
  if (nel > 4.0e9) { set_error("problem too large"); return GDW_EINVAL; }
  return GDW_OK;
}

// Eigenbasis of one direction on the device (FP64) -> host copies of Psi and lambda.
static gdw_status eigen_dir(int N, int p, double H, std::vector<double>& Psi,
                            std::vector<double>& lam, std::vector<double>& M,
                            std::vector<double>& dL, std::vector<double>& dR) {
  const int n1 = N + 1;
  std::vector<double> Mh(n1 * n1), Sh(n1 * n1), dLh(n1), dRh(n1);
  gd1d_unit(N, p, Mh.data(), Sh.data(), dLh.data(), dRh.data());
  const double h = H / N;
  M.resize(n1 * n1);
  std::vector<double> S(n1 * n1);
  for (int i = 0; i < n1 * n1; ++i) { M[i] = h * Mh[i]; S[i] = Sh[i] / h; }
  dL.resize(n1); dR.resize(n1);
  for (int i = 0; i < n1; ++i) { dL[i] = dLh[i] / h; dR[i] = dRh[i] / h; }
  double *dM = nullptr, *dS = nullptr, *work = nullptr, *dPsi = nullptr, *dlam = nullptr;
  int* dinfo = nullptr;
  gdw_status st = GDW_OK;
  auto cleanup = [&]() {
    if (dM) (void)hipFree(dM); if (dS) (void)hipFree(dS); if (work) (void)hipFree(work);
    if (dPsi) (void)hipFree(dPsi); if (dlam) (void)hipFree(dlam); if (dinfo) (void)hipFree(dinfo);
  };
  hipError_t e = hipSuccess;
  do {
    if ((e = hipMalloc(&dM, n1 * n1 * sizeof(double))) != hipSuccess) break;
    if ((e = hipMalloc(&dS, n1 * n1 * sizeof(double))) != hipSuccess) break;
    if ((e = hipMalloc(&work, (3 * n1 * n1 + 5 * n1) * sizeof(double))) != hipSuccess) break;
    if ((e = hipMalloc(&dPsi, n1 * n1 * sizeof(double))) != hipSuccess) break;
    if ((e = hipMalloc(&dlam, n1 * sizeof(double))) != hipSuccess) break;
    if ((e = hipMalloc(&dinfo, (1 + n1) * sizeof(int))) != hipSuccess) break;
    if ((e = hipMemcpy(dM, M.data(), n1 * n1 * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) break;
    if ((e = hipMemcpy(dS, S.data(), n1 * n1 * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) break;
    if ((e = launch_eig(dM, dS, n1, work, dPsi, dlam, dinfo, nullptr)) != hipSuccess) break;
    if ((e = hipDeviceSynchronize()) != hipSuccess) break;
    Psi.resize(n1 * n1); lam.resize(n1);
    int info = 0;
    if ((e = hipMemcpy(Psi.data(), dPsi, n1 * n1 * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) break;
    if ((e = hipMemcpy(lam.data(), dlam, n1 * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) break;
    if ((e = hipMemcpy(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess) break;
    if (!info) { set_error("mass matrix is not positive definite"); st = GDW_EINVAL; }
  } while (0);
  cleanup();
  if (e != hipSuccess) {
    set_error(std::string("eigenbasis set-up: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? GDW_ENOMEM : GDW_EHIP;
  }
  return st;
}

template <typename T>
static gdw_status upload_as(void** dst, const std::vector<double>& src) {
  std::vector<T> tmp(src.begin(), src.end());
  GDW_HIP(hipMalloc(dst, tmp.size() * sizeof(T)));
  GDW_HIP(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
  return GDW_OK;
}

static gdw_status upload_tables(gdw_ctx* c, const std::vector<double>& gh,
                                const std::vector<double>& invL, const std::vector<double>& lam) {
  // FP64 in both storage modes (the stage arithmetic is FP64)
  gdw_status s;
  if ((s = upload_as<double>(&c->gh, gh)) != GDW_OK) return s;
  if ((s = upload_as<double>(&c->invL, invL)) != GDW_OK) return s;
  return upload_as<double>(&c->lam, lam);
}

static gdw_status create_fdm(const gdw_desc* d, gdw_ctx* c) {
  const int N = d->N, p = d->p, n1 = N + 1, nn = n1 * n1;

  std::vector<double> Psx, lx, Mx, dLx, dRx, Psy, ly, My, dLy, dRy;
  gdw_status s;
  if ((s = eigen_dir(N, p, d->Lx / d->nx, Psx, lx, Mx, dLx, dRx)) != GDW_OK) return s;
  if ((s = eigen_dir(N, p, d->Ly / d->ny, Psy, ly, My, dLy, dRy)) != GDW_OK) return s;

  // face tables: g = Psi^T dR (east/north), -Psi^T dL (west/south); h = rows N / 0 of Psi
  std::vector<double> gh(8 * n1), invL(nn), lam(nn), Px(nn), Py(nn);
  for (int k = 0; k < n1; ++k) {
    double gE = 0, gW = 0, gN = 0, gS = 0;
    for (int i = 0; i < n1; ++i) {
      gE += dRx[i] * Psx[i * n1 + k];
      gW -= dLx[i] * Psx[i * n1 + k];
      gN += dRy[i] * Psy[i * n1 + k];
      gS -= dLy[i] * Psy[i * n1 + k];
    }
    gh[0 * n1 + k] = gE; gh[1 * n1 + k] = Psx[N * n1 + k];
    gh[2 * n1 + k] = gW; gh[3 * n1 + k] = Psx[0 * n1 + k];
    gh[4 * n1 + k] = gN; gh[5 * n1 + k] = Psy[N * n1 + k];
    gh[6 * n1 + k] = gS; gh[7 * n1 + k] = Psy[0 * n1 + k];
  }
  // Lambda_hat = c^2 (lambda_x + lambda_y), (0,0) entry kappa = c^2 (DG1_extra); the
  // stage kernel uses c^2 / Lambda_hat.
  for (int ky = 0; ky < n1; ++ky)
    for (int kx = 0; kx < n1; ++kx) {
      const double l = lx[kx] + ly[ky];
      lam[ky * n1 + kx] = l;
      invL[ky * n1 + kx] = (kx == 0 && ky == 0) ? 1.0 : 1.0 / l;
    }
  // Psi^{-1} = Psi^T M per direction
  for (int k = 0; k < n1; ++k)
    for (int i = 0; i < n1; ++i) {
      double sx = 0, sy = 0;
      for (int j = 0; j < n1; ++j) {
        sx += Psx[j * n1 + k] * Mx[j * n1 + i];
        sy += Psy[j * n1 + k] * My[j * n1 + i];
      }
      Px[k * n1 + i] = sx;
      Py[k * n1 + i] = sy;
    }
  if ((s = upload_tables(c, gh, invL, lam)) != GDW_OK) return s;
  if ((s = upload_as<double>((void**)&c->Psx, Psx)) != GDW_OK) return s;
  if ((s = upload_as<double>((void**)&c->Psy, Psy)) != GDW_OK) return s;
  if ((s = upload_as<double>((void**)&c->Px, Px)) != GDW_OK) return s;
  if ((s = upload_as<double>((void**)&c->Py, Py)) != GDW_OK) return s;

  const size_t field = (size_t)c->nel * nn * c->elem_bytes;
  for (int r = 0; r < 3; ++r)
    for (auto& ptr : c->Y[r]) {
      if (r == 0 && c->elem_bytes == 4) continue;   // FP32 storage: y is y64
      GDW_HIP(hipMalloc(&ptr, field));
      GDW_HIP(hipMemset(ptr, 0, field));
    }
  if (c->elem_bytes == 4)
    for (auto& ptr : c->y64) {
      GDW_HIP(hipMalloc(&ptr, (size_t)c->nel * nn * sizeof(double)));
      GDW_HIP(hipMemset(ptr, 0, (size_t)c->nel * nn * sizeof(double)));
    }
  const size_t trb = (size_t)c->nel * 8 * n1 * c->elem_bytes;
  for (auto& t : c->tr) {
    GDW_HIP(hipMalloc(&t, trb));
    GDW_HIP(hipMemset(t, 0, trb));
  }
  GDW_HIP(hipMalloc(&c->epart, (c->npart + 1) * sizeof(double)));
  GDW_HIP(hipMalloc(&c->nonfinite, sizeof(unsigned int)));
  GDW_HIP(hipDeviceSynchronize());
  return GDW_OK;
}


// Box elements in 3D: the same tables per direction, face tables of the six faces
// [12][n1] (gE hE gW hW from x, gN hN gS hS from y, gT hT gB hB from z), Lambda over the
// three modal indices (Sec. 3.2 with d = 3).
static gdw_status create_fdm3(const gdw_desc* d, gdw_ctx* c) {
  const int N = d->N, p = d->p, n1 = N + 1, n2 = n1 * n1, n3 = n2 * n1;
  std::vector<double> Ps[3], lm[3], Mm[3], dL[3], dR[3];
  const double H[3] = {d->Lx / d->nx, d->Ly / d->ny, d->Lz / d->nz};
  gdw_status s;
  for (int k = 0; k < 3; ++k)
    if ((s = eigen_dir(N, p, H[k], Ps[k], lm[k], Mm[k], dL[k], dR[k])) != GDW_OK) return s;
  std::vector<double> gh(12 * n1), invL(n3), lam(n3), P[3];
  for (int dir = 0; dir < 3; ++dir) {
    for (int k = 0; k < n1; ++k) {
      double gR = 0, gL = 0;
      for (int i = 0; i < n1; ++i) {
        gR += dR[dir][i] * Ps[dir][i * n1 + k];
        gL -= dL[dir][i] * Ps[dir][i * n1 + k];
      }
      gh[(4 * dir + 0) * n1 + k] = gR; gh[(4 * dir + 1) * n1 + k] = Ps[dir][N * n1 + k];
      gh[(4 * dir + 2) * n1 + k] = gL; gh[(4 * dir + 3) * n1 + k] = Ps[dir][0 * n1 + k];
    }
    P[dir].resize(n2);
    for (int k = 0; k < n1; ++k)
      for (int i = 0; i < n1; ++i) {
        double sum = 0;
        for (int j = 0; j < n1; ++j) sum += Ps[dir][j * n1 + k] * Mm[dir][j * n1 + i];
        P[dir][k * n1 + i] = sum;
      }
  }
  for (int kz = 0; kz < n1; ++kz)
    for (int ky = 0; ky < n1; ++ky)
      for (int kx = 0; kx < n1; ++kx) {
        const int i = (kz * n1 + ky) * n1 + kx;
        const double l = lm[0][kx] + lm[1][ky] + lm[2][kz];
        lam[i] = l;
        invL[i] = i == 0 ? 1.0 : 1.0 / l;
      }
  if ((s = upload_tables(c, gh, invL, lam)) != GDW_OK) return s;
  if ((s = upload_as<double>((void**)&c->Psx, Ps[0])) != GDW_OK) return s;
  if ((s = upload_as<double>((void**)&c->Psy, Ps[1])) != GDW_OK) return s;
  if ((s = upload_as<double>((void**)&c->Psz, Ps[2])) != GDW_OK) return s;
  if ((s = upload_as<double>((void**)&c->Px, P[0])) != GDW_OK) return s;
  if ((s = upload_as<double>((void**)&c->Py, P[1])) != GDW_OK) return s;
  if ((s = upload_as<double>((void**)&c->Pz, P[2])) != GDW_OK) return s;
  const size_t field = (size_t)c->nel * n3 * c->elem_bytes;
  for (int r = 0; r < 3; ++r)
    for (auto& ptr : c->Y[r]) {
      if (r == 0 && c->elem_bytes == 4) continue;   // FP32 storage: y is y64
      GDW_HIP(hipMalloc(&ptr, field));
      GDW_HIP(hipMemset(ptr, 0, field));
    }
  if (c->elem_bytes == 4)
    for (auto& ptr : c->y64) {
      GDW_HIP(hipMalloc(&ptr, (size_t)c->nel * n3 * sizeof(double)));
      GDW_HIP(hipMemset(ptr, 0, (size_t)c->nel * n3 * sizeof(double)));
    }
  const size_t trb = (size_t)c->nel * 12 * n2 * c->elem_bytes;
  for (auto& t : c->tr) {
    GDW_HIP(hipMalloc(&t, trb));
    GDW_HIP(hipMemset(t, 0, trb));
  }
  GDW_HIP(hipMalloc(&c->epart, (c->npart + 1) * sizeof(double)));
  GDW_HIP(hipMalloc(&c->nonfinite, sizeof(unsigned int)));
  GDW_HIP(hipDeviceSynchronize());
  return GDW_OK;
}

// ---------------------------------------------------------------------------------
// PCG path set-up
// ---------------------------------------------------------------------------------
template <typename V>
static gdw_status own_upload(gdw_ctx* c, int slot, const std::vector<V>& v, const V** dst) {
  void* p = nullptr;
  GDW_HIP(hipMalloc(&p, v.size() * sizeof(V)));
  c->own[slot] = p;
  GDW_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice));
  *dst = (const V*)p;
  return GDW_OK;
}

static gdw_status create_pcg(const gdw_desc* d, gdw_ctx* c) {
  const int N = d->N, p = d->p, n1 = N + 1, nn = n1 * n1, m = p + 1;
  PcgGeom& g = c->g;
  g.N = N; g.p = p; g.n1 = n1; g.nn = nn; g.m = m; g.nq = N * m;
  std::vector<int> rowoff(nn + 1, 0), fo(nn + 1, 0), cs(N), ck0(n1, N), ck1(n1, -1);
  for (int i = 0; i < nn; ++i) {
    rowoff[i + 1] = rowoff[i] + st_count(i % n1, i / n1, p, N);
    // rows padded to an odd number of doubles: consecutive rows, read by consecutive
    // lanes, then start in different LDS bank pairs
    const int len = st_w(i % n1, p, N) * st_w(i / n1, p, N);
    fo[i + 1] = fo[i] + len + (len % 2 == 0 ? 1 : 0);
  }
  g.nst = rowoff[nn];
  for (int k = 0; k < N; ++k) {
    cs[k] = gd_window_start(k, N, p);
    for (int j = 0; j < m; ++j) {
      ck0[cs[k] + j] = std::min(ck0[cs[k] + j], k);
      ck1[cs[k] + j] = std::max(ck1[cs[k] + j], k);
    }
  }
  std::vector<double> xg(m), gw(m), cb((size_t)N * m * m), cd((size_t)N * m * m), val(n1), der(n1);
  gauss_legendre01(m, xg.data(), gw.data());
  for (int k = 0; k < N; ++k)
    for (int a = 0; a < m; ++a) {
      gd1d_eval_cell(N, p, k, k + xg[a], val.data(), der.data());
      for (int j = 0; j < m; ++j) {
        cb[(k * m + a) * m + j] = val[cs[k] + j];
        cd[(k * m + a) * m + j] = der[cs[k] + j] * N;
      }
    }
  // reference interval [0, 1]: element_1d with H = 1 gives M_ref, S_ref and d/dr vectors
  std::vector<double> Psi, lam, Mref, dL, dR;
  gdw_status s;
  if ((s = eigen_dir(N, p, 1.0, Psi, lam, Mref, dL, dR)) != GDW_OK) return s;
  if ((s = own_upload<int>(c, 0, rowoff, &g.rowoff)) != GDW_OK) return s;
  if ((s = own_upload<int>(c, 1, cs, &g.cs)) != GDW_OK) return s;
  if ((s = own_upload<int>(c, 2, ck0, &g.ck0)) != GDW_OK) return s;
  if ((s = own_upload<int>(c, 3, ck1, &g.ck1)) != GDW_OK) return s;
  if ((s = own_upload<double>(c, 4, cb, &g.cb)) != GDW_OK) return s;
  if ((s = own_upload<double>(c, 5, cd, &g.cd)) != GDW_OK) return s;
  if ((s = own_upload<double>(c, 6, gw, &g.gw)) != GDW_OK) return s;
  if ((s = own_upload<double>(c, 7, dL, &g.dL)) != GDW_OK) return s;
  if ((s = own_upload<double>(c, 8, dR, &g.dR)) != GDW_OK) return s;
  if ((s = own_upload<double>(c, 9, Psi, &g.Psi)) != GDW_OK) return s;
  if ((s = own_upload<double>(c, 10, lam, &g.lamr)) != GDW_OK) return s;
  if ((s = own_upload<double>(c, 11, Mref, &g.Mref)) != GDW_OK) return s;
  if ((s = own_upload<int>(c, 12, fo, &c->fo)) != GDW_OK) return s;
  {
    // basis values at the centres of an 8 x 8 subdivision (network inputs)
    std::vector<double> Bs((size_t)8 * n1), vv(n1), dd(n1);
    for (int sidx = 0; sidx < 8; ++sidx) {
      const double tt = (sidx + 0.5) / 8.0 * N;
      gd1d_eval_cell(N, p, std::min((int)tt, N - 1), tt, vv.data(), dd.data());
      for (int i = 0; i < n1; ++i) Bs[(size_t)sidx * n1 + i] = vv[i];
    }
    if ((s = own_upload<double>(c, 14, Bs, &c->Bs)) != GDW_OK) return s;
  }
  {
    // destinations of each stored upper entry (i, j) in the full rectangles: (i, j), (j, i)
    std::vector<int> dst((size_t)2 * g.nst);
    for (int i = 0; i < nn; ++i) {
      const int ix = i % n1, iy = i / n1;
      for (int j = i; j < nn; ++j) {
        const int jx = j % n1, jy = j / n1;
        if (!st_in_upper(ix, iy, jx, jy, p, N)) continue;
        const int h = rowoff[i] + st_pos(ix, iy, jx, jy, p, N);
        dst[2 * h] = fo[i] + (jy - st_lo(iy, p)) * st_w(ix, p, N) + (jx - st_lo(ix, p));
        dst[2 * h + 1] = fo[j] + (iy - st_lo(jy, p)) * st_w(jx, p, N) + (ix - st_lo(jx, p));
      }
    }
    if ((s = own_upload<int>(c, 13, dst, &c->dst)) != GDW_OK) return s;
  }
  {
    // column-block layout of the faster stage kernel, where it applies
    std::vector<int> boff, bdst, jc, gidx, unit;
    const int mixed = d->precision == GDW_MIXED_FP32;
    if (pcg_block_tables(g, rowoff, boff, bdst, jc, gidx, unit, &c->blk_K, &c->blk_CH,
                         &c->blk_WB, &c->blk_nnz, &c->blk_threads, mixed)) {
      if ((s = own_upload<int>(c, 15, boff, &c->blk_off)) != GDW_OK) return s;
      if ((s = own_upload<int>(c, 16, bdst, &c->blk_dst)) != GDW_OK) return s;
      if ((s = own_upload<int>(c, 17, jc, &c->blk_jc)) != GDW_OK) return s;
      if (!gidx.empty() && (s = own_upload<int>(c, 18, gidx, &c->blk_gidx)) != GDW_OK) return s;
      if (!unit.empty() && (s = own_upload<int>(c, 19, unit, &c->blk_unit)) != GDW_OK) return s;
      c->blk_v2 = 1;
    } else if (mixed) {
      set_error("mixed-precision PCG needs N + 1 in {9, 13, 17} and an FP32 element operator "
                "that fits a workgroup's LDS");
      return GDW_EUNSUPPORTED;
    }
  }
  // the split stage's solve kernels keep no operator in LDS; the fused stage kernel does
  if (d->precision == GDW_MIXED_PC32 &&
      !(c->blk_v2 && c->blk_gidx != nullptr && pcg_pc32_supported(g.n1, g.p, c->blk_threads))) {
    set_error("GDW_MIXED_PC32 needs N + 1 in {9, 13} with p in {5, 7}, or N + 1 = 13 with p = 3");
    return GDW_EUNSUPPORTED;
  }
  const bool split_stage = c->blk_v2 && c->blk_gidx != nullptr &&
                           d->precision != GDW_MIXED_FP32 &&
                           pcg_split_key(pcg_family_key(g.n1, g.p, 1, 0));
  if (!split_stage && pcg_stage_lds_bytes(g, 0) > 160 * 1024) {
    set_error("element operator does not fit the LDS of a workgroup (reduce N or p)");
    return GDW_EUNSUPPORTED;
  }
  const long nel = c->nel;
  const size_t nodal = (size_t)nel * nn * sizeof(double);
  GDW_HIP(hipMalloc(&c->el.S, (size_t)nel * g.nst * sizeof(double)));
  if (d->mapped) {
    GDW_HIP(hipMalloc(&c->el.M, (size_t)nel * g.nst * sizeof(double)));
    GDW_HIP(hipMalloc(&c->el.msc, (size_t)nel * nn * sizeof(double)));
  }
  GDW_HIP(hipMalloc(&c->el.w, nodal));
  GDW_HIP(hipMalloc(&c->el.sc, (size_t)nel * 8 * sizeof(double)));
  GDW_HIP(hipMalloc(&c->el.face, (size_t)nel * 4 * g.nq * 3 * sizeof(double)));
  for (auto& r : c->Y)
    for (auto& ptr : r) {
      GDW_HIP(hipMalloc(&ptr, nodal));
      GDW_HIP(hipMemset(ptr, 0, nodal));
    }
  const size_t trb = (size_t)nel * 4 * g.nq * 2 * sizeof(double);
  for (auto& t : c->tr) {
    GDW_HIP(hipMalloc(&t, trb));
    GDW_HIP(hipMemset(t, 0, trb));
  }
  GDW_HIP(hipMalloc(&c->xS, nodal));
  GDW_HIP(hipMalloc(&c->xM, nodal));
  GDW_HIP(hipMalloc(&c->its, (size_t)nel * kItsPer * sizeof(int)));
  if (d->precision == GDW_MIXED_FP32) {
    const size_t nb = (size_t)nel * c->blk_nnz * sizeof(float);
    GDW_HIP(hipMalloc(&c->el.Shi, nb));
    GDW_HIP(hipMalloc(&c->el.Slo, nb));
    if (d->mapped) {
      GDW_HIP(hipMalloc(&c->el.Mhi, nb));
      GDW_HIP(hipMalloc(&c->el.Mlo, nb));
    }
  }
  if (c->blk_v2 && c->blk_gidx) {
    // slot-ordered operator copies read by the register kernels
    const size_t nb = (size_t)nel * pcg_reg_slots(n1, p) * c->blk_threads * sizeof(double);
    GDW_HIP(hipMalloc(&c->el.Sreg, nb));
    if (d->mapped) GDW_HIP(hipMalloc(&c->el.Mreg, nb));
    if (pcg_split_key(pcg_family_key(n1, p, 1, 0))) {
      GDW_HIP(hipMalloc(&c->Fu, nodal));
      GDW_HIP(hipMalloc(&c->Fv, nodal));
    }
  }
  GDW_HIP(hipMalloc(&c->d_pargs, 4 * sizeof(PcgStageArgs)));
  GDW_HIP(hipMalloc(&c->d_pel, 2 * sizeof(long)));
  {
    const long pel[2] = {0, nel};
    GDW_HIP(hipMemcpy(c->d_pel, pel, sizeof(pel), hipMemcpyHostToDevice));
  }
  GDW_HIP(pcg_group_prepare());
  GDW_HIP(hipMalloc(&c->fail, sizeof(int)));
  GDW_HIP(hipMalloc(&c->epart, (size_t)(nel + 1) * sizeof(double)));
  GDW_HIP(hipMalloc(&c->nonfinite, sizeof(unsigned int)));
  // Cartesian node coordinates (from the global node index, so that both copies of a
  // face node are bitwise equal) and the constant c^2, used when set_coeff gets NULL
  std::vector<double> xyz((size_t)3 * nel * nn);
  for (int ey = 0; ey < d->ny; ++ey)
    for (int ex = 0; ex < d->nx; ++ex)
      for (int iy = 0; iy < n1; ++iy)
        for (int ix = 0; ix < n1; ++ix) {
          const size_t k = ((size_t)(ey * d->nx + ex) * n1 + iy) * n1 + ix;
          xyz[k] = d->x0 + (double)(ex * N + ix) * (d->Lx / ((double)d->nx * N));
          xyz[(size_t)nel * nn + k] = d->y0 + (double)(ey * N + iy) * (d->Ly / ((double)d->ny * N));
          xyz[(size_t)2 * nel * nn + k] = d->c2;
        }
  GDW_HIP(hipMalloc(&c->c2n, (size_t)nel * nn * sizeof(double)));
  GDW_HIP(hipMalloc(&c->coords, xyz.size() * sizeof(double)));
  GDW_HIP(hipMemcpy(c->coords, xyz.data(), xyz.size() * sizeof(double), hipMemcpyHostToDevice));
  c->rtol = d->pcg_rtol > 0 ? d->pcg_rtol : 1e-12;
  c->maxit = d->pcg_maxit > 0 ? d->pcg_maxit : 200;
  GDW_HIP(hipDeviceSynchronize());
  return GDW_OK;
}

static gdw_status create_impl(const gdw_desc* d, gdw_ctx* c) {
  c->d = *d;
  c->n1 = d->N + 1;
  c->dim = d->dim == 3 ? 3 : 2;
  c->nel = (long)d->nx * d->ny * (c->dim == 3 ? d->nz : 1);
  c->nn = c->n1 * c->n1 * (c->dim == 3 ? c->n1 : 1);
  c->elem_bytes = d->precision == GDW_MIXED_FP32 ? 4 : 8;
  // alternating flux: v* from the element on the low-coordinate side of a face, (grad u)*
  // from the one on the high side, i.e. alpha = 1 on an element's E and N faces and 0 on
  // its W and S faces (wall faces take 1/2 in the kernels)
  const bool alt = d->flux == GDW_FLUX_ALTERNATING;
  c->alf[0] = c->alf[2] = c->alf[4] = alt ? 1.0 : 0.5;
  c->alf[1] = c->alf[3] = c->alf[5] = alt ? 0.0 : 0.5;
  c->beta = d->flux == GDW_FLUX_UPWIND ? 0.5 * d->xi : 0.0;
  c->tau = d->flux == GDW_FLUX_UPWIND ? 0.5 / d->xi : 0.0;
  const bool pcg = d->solver == GDW_SOLVE_PCG || d->coeff_variable || d->mapped;
  c->solver = pcg ? GDW_SOLVE_PCG : GDW_SOLVE_FDM;
  if (c->dim == 3) return create_fdm3(d, c);
  return pcg ? create_pcg(d, c) : create_fdm(d, c);
}

extern "C" gdw_status gdw_create(const gdw_desc* desc, gdw_ctx** out) {
  if (!out) { set_error("out is NULL"); return GDW_EINVAL; }
  *out = nullptr;
  gdw_status s = validate(desc);
  if (s != GDW_OK) return s;
  gdw_ctx* c = new (std::nothrow) gdw_ctx();
  if (!c) { set_error("host allocation failed"); return GDW_ENOMEM; }
  s = create_impl(desc, c);
  if (s != GDW_OK) {
    free_all(c);
    delete c;
    return s;
  }
  *out = c;
  return GDW_OK;
}

extern "C" gdw_status gdw_set_coeff(gdw_ctx* c, const double* c2, const double* X, const double* Y,
                                    void* stream) {
  if (!c) { set_error("ctx is NULL"); return GDW_EINVAL; }
  if (c->solver != GDW_SOLVE_PCG) { set_error("gdw_set_coeff applies to the PCG path only"); return GDW_EINVAL; }
  if ((X == nullptr) != (Y == nullptr)) { set_error("give both X and Y or neither"); return GDW_EINVAL; }
  hipStream_t st = (hipStream_t)stream;
  const size_t nn = (size_t)c->g.nn;
  const double* Xd = X ? X : c->coords;
  const double* Yd = Y ? Y : c->coords + (size_t)c->nel * nn;
  const double* Cd = c2 ? c2 : c->coords + (size_t)2 * c->nel * nn;
  GDW_HIP(hipMemcpyAsync(c->c2n, Cd, (size_t)c->nel * nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  GDW_HIP(launch_assemble(c->g, Xd, Yd, Cd, c->el, c->nel, st));
  GDW_HIP(launch_face_geom(c->g, Xd, Yd, Cd, c->el, c->nel, st));
  if (c->el.msc) GDW_HIP(launch_mscale(c->g, c->el, c->nel, st));
  if (c->el.Sreg) {
    const int slots = pcg_reg_slots(c->g.n1, c->g.p);
    GDW_HIP(launch_reg_permute(c->el.S, c->blk_gidx, c->g.nst, slots, c->blk_threads, c->nel,
                               c->el.Sreg, st));
    if (c->el.Mreg)
      GDW_HIP(launch_reg_permute(c->el.M, c->blk_gidx, c->g.nst, slots, c->blk_threads, c->nel,
                                 c->el.Mreg, st));
  }
  if (c->el.Shi) {
    GDW_HIP(launch_split_hilo(c->el.S, c->blk_dst, c->g.nst, c->blk_nnz, c->nel, c->el.Shi,
                              c->el.Slo, st));
    if (c->el.M)
      GDW_HIP(launch_split_hilo(c->el.M, c->blk_dst, c->g.nst, c->blk_nnz, c->nel, c->el.Mhi,
                                c->el.Mlo, st));
  }
  c->have_coeff = 1;
  return GDW_OK;
}

template <typename T>
static hipError_t set_state_t(gdw_ctx* c, const double* U, const double* V, hipStream_t st) {
  hipError_t e;
  // FP64 storage: y = Y[0]; FP32 storage: y is the FP64 register y64 (traces in FP32)
  double* yu = sizeof(T) == 8 ? (double*)c->Y[0][0] : c->y64[0];
  double* yv = sizeof(T) == 8 ? (double*)c->Y[0][1] : c->y64[1];
  c->trc = 0;
  if (c->dim == 3) {
    if ((e = launch_to_modal3<double>(U, yu, c->Px, c->Py, c->Pz, c->n1, c->nel, st)) != hipSuccess) return e;
    if ((e = launch_to_modal3<double>(V, yv, c->Px, c->Py, c->Pz, c->n1, c->nel, st)) != hipSuccess) return e;
    return launch_traces3<double, T>(yu, yv, (const double*)c->gh, (T*)c->tr[0], c->n1, c->nel, st);
  }
  if ((e = launch_to_modal<double>(U, yu, c->Px, c->Py, c->n1, c->nel, st)) != hipSuccess) return e;
  if ((e = launch_to_modal<double>(V, yv, c->Px, c->Py, c->n1, c->nel, st)) != hipSuccess) return e;
  return launch_traces<double, T>(yu, yv, (const double*)c->gh, (T*)c->tr[0], c->n1, c->nel, st);
}

extern "C" gdw_status gdw_set_state(gdw_ctx* c, const double* U, const double* V, void* stream) {
  if (!c || !U || !V) { set_error("NULL argument"); return GDW_EINVAL; }
  hipStream_t st = (hipStream_t)stream;
  if (c->solver == GDW_SOLVE_PCG) {
    if (!c->have_coeff) { set_error("call gdw_set_coeff before gdw_set_state"); return GDW_EINVAL; }
    const size_t nodal = (size_t)c->nel * c->g.nn * sizeof(double);
    GDW_HIP(hipMemcpyAsync(c->Y[0][0], U, nodal, hipMemcpyDeviceToDevice, st));
    GDW_HIP(hipMemcpyAsync(c->Y[0][1], V, nodal, hipMemcpyDeviceToDevice, st));
    GDW_HIP(hipMemsetAsync(c->xS, 0, nodal, st));
    GDW_HIP(hipMemsetAsync(c->xM, 0, nodal, st));
    GDW_HIP(hipMemsetAsync(c->its, 0, (size_t)c->nel * kItsPer * sizeof(int), st));
    GDW_HIP(hipMemsetAsync(c->fail, 0x7f, sizeof(int), st));
    c->trc = 0;
    c->stages_since_state = 0;
    GDW_HIP(launch_pcg_traces(c->g, c->el, (const double*)c->Y[0][0], (const double*)c->Y[0][1],
                              (double*)c->tr[0], c->nel, st));
  } else {
    GDW_HIP(c->elem_bytes == 8 ? set_state_t<double>(c, U, V, st) : set_state_t<float>(c, U, V, st));
  }
  c->have_state = 1;
  c->t = 0.0;
  if (c->t_dev) GDW_HIP(launch_set_clock(c->t_dev, 0.0, st));
  return GDW_OK;
}

extern "C" gdw_status gdw_set_forcing(gdw_ctx* c, int nterms, const double* g_nodal,
                                      const double* omega, const double* phase, void* stream) {
  if (!c) { set_error("ctx is NULL"); return GDW_EINVAL; }
  if (nterms < 0 || nterms > 4) { set_error("nterms must be in 0..4"); return GDW_EINVAL; }
  if (c->dim == 3) { set_error("source terms are not offered in 3D"); return GDW_EUNSUPPORTED; }
  if (nterms > 0 && (!g_nodal || !omega || !phase)) { set_error("NULL argument"); return GDW_EINVAL; }
  for (int k = 0; k < nterms; ++k)
    if (!std::isfinite(omega[k]) || !std::isfinite(phase[k])) {
      set_error("omega and phase must be finite"); return GDW_EINVAL;
    }
  hipStream_t st = (hipStream_t)stream;
  const long per = c->nel * (long)c->n1 * c->n1;
  if (c->solver == GDW_SOLVE_PCG) {
    // nodal FP64 fields; the stage epilogue adds sum_k s_k g_k to dv/dt
    if (nterms > 0 && !c->frc) GDW_HIP(hipMalloc(&c->frc, (size_t)4 * per * sizeof(double)));
    if (nterms > 0 && !c->t_dev) {
      GDW_HIP(hipMalloc(&c->t_dev, 17 * sizeof(double)));   // clock, then 16 weights
      GDW_HIP(launch_set_clock(c->t_dev, c->t, st));
    }
    for (int k = 0; k < nterms; ++k) {
      GDW_HIP(hipMemcpyAsync((double*)c->frc + k * per, g_nodal + (size_t)k * per,
                             (size_t)per * sizeof(double), hipMemcpyDeviceToDevice, st));
      c->f_omega[k] = omega[k];
      c->f_phase[k] = phase[k];
    }
    GDW_HIP(hipStreamSynchronize(st));
    c->nf = nterms;
    c->pargs_ok = 0;   // the stage argument blocks carry the source
    ++c->args_epoch;
    return GDW_OK;
  }
  if (nterms > 0 && !c->frc)
    GDW_HIP(hipMalloc(&c->frc, (size_t)4 * per * c->elem_bytes));
  if (nterms > 0 && !c->t_dev) {
    GDW_HIP(hipMalloc(&c->t_dev, 17 * sizeof(double)));   // clock, then 16 weights
    GDW_HIP(launch_set_clock(c->t_dev, c->t, st));
  }
  for (int k = 0; k < nterms; ++k) {
    const double* g = g_nodal + (size_t)k * per;
    if (c->elem_bytes == 8)
      GDW_HIP(launch_to_modal<double>(g, (double*)c->frc + k * per, c->Px, c->Py, c->n1, c->nel, st));
    else
      GDW_HIP(launch_to_modal<float>(g, (float*)c->frc + k * per, c->Px, c->Py, c->n1, c->nel, st));
    c->f_omega[k] = omega[k];
    c->f_phase[k] = phase[k];
  }
  GDW_HIP(hipStreamSynchronize(st));
  c->nf = nterms;
  ++c->args_epoch;   // a batch rebuilds its captured step
  return GDW_OK;
}

namespace gdw {

// RK4 register roles per stage (both paths):
//   stage 1: in = y;          out = Y;  traces t0 -> t1
//   stage 2: in = Y, aux = y; out = Y, acc = A;  traces t1 -> t0
//   stage 3: in = Y, aux = y; out = Y;  traces t0 -> t1
//   stage 4: in = Y, aux = A; out = y;  traces t1 -> t0
template <typename P>
static void stage_roles(const gdw_ctx* c, int stage, P& a) {
  using T = typename std::remove_const<typename std::remove_pointer<decltype(a.in_u)>::type>::type;
  T* y_u = (T*)c->Y[0][0];
  T* y_v = (T*)c->Y[0][1];
  T* Y_u = (T*)c->Y[1][0];
  T* Y_v = (T*)c->Y[1][1];
  T* A_u = (T*)c->Y[2][0];
  T* A_v = (T*)c->Y[2][1];
  T* t0 = (T*)c->tr[c->trc];
  T* t1 = (T*)c->tr[c->trc ^ 1];
  a.aux_u = a.aux_v = nullptr;
  a.acc_u = a.acc_v = nullptr;
  switch (stage) {
    case 1:
      a.in_u = y_u; a.in_v = y_v; a.out_u = Y_u; a.out_v = Y_v;
      a.tr_in = t0; a.tr_out = t1;
      break;
    case 2:
      a.in_u = Y_u; a.in_v = Y_v; a.aux_u = y_u; a.aux_v = y_v;
      a.out_u = Y_u; a.out_v = Y_v; a.acc_u = A_u; a.acc_v = A_v;
      a.tr_in = t1; a.tr_out = t0;
      break;
    case 3:
      a.in_u = Y_u; a.in_v = Y_v; a.aux_u = y_u; a.aux_v = y_v;
      a.out_u = Y_u; a.out_v = Y_v;
      a.tr_in = t0; a.tr_out = t1;
      break;
    default:
      a.in_u = Y_u; a.in_v = Y_v; a.aux_u = A_u; a.aux_v = A_v;
      a.out_u = y_u; a.out_v = y_v;
      a.tr_in = t1; a.tr_out = t0;
      break;
  }
}

SourceTerms source_terms(const gdw_ctx* c) {
  SourceTerms f{};
  f.nf = c->nf;
  for (int k = 0; k < 4; ++k) {
    f.omega[k] = c->f_omega[k];
    f.phase[k] = c->f_phase[k];
  }
  return f;
}

template <typename T>
StageArgs<T> fdm_stage_args(const gdw_ctx* c, int stage, double dt) {
  StageArgs<T> a{};
  a.nel = c->nel;
  a.nx = c->d.nx;
  a.ny = c->d.ny;
  a.n1 = c->n1;
  a.dt = dt;
  a.c2 = c->d.c2;
  for (int k = 0; k < 6; ++k) a.alf[k] = c->alf[k];
  a.beta = c->beta;
  a.tau = c->tau;
  a.invL = (const double*)c->invL;
  a.lam = (const double*)c->lam;
  a.gh = (const double*)c->gh;
  a.nz = c->dim == 3 ? c->d.nz : 1;
  a.bcbits = 0;
  for (int k = 0; k < 4; ++k) a.bcbits |= (c->d.bc[k] & 3) << (2 * k);
  if (c->dim == 3)
    for (int k = 0; k < 2; ++k) a.bcbits |= (c->d.bcz[k] & 3) << (2 * (4 + k));
  a.nf = c->nf;
  a.frc = (const T*)c->frc;
  a.frc_stride = c->nel * (long)c->n1 * c->n1;
  a.fw = c->t_dev ? c->t_dev + 1 : nullptr;
  a.y64_u = c->y64[0];
  a.y64_v = c->y64[1];
  stage_roles(c, stage, a);
  return a;
}

template StageArgs<double> fdm_stage_args<double>(const gdw_ctx*, int, double);
template StageArgs<float> fdm_stage_args<float>(const gdw_ctx*, int, double);

PcgStageArgs pcg_stage_args(const gdw_ctx* c, int stage, double dt) {
  PcgStageArgs a{};
  a.g = c->g;
  a.el = c->el;
  a.xS = c->xS;
  a.xM = c->xM;
  a.Fu = c->Fu;
  a.Fv = c->Fv;
  a.its = c->its;
  a.fail = c->fail;
  a.nel = c->nel;
  a.nx = c->d.nx;
  a.ny = c->d.ny;
  a.bcbits = 0;
  for (int k = 0; k < 4; ++k) a.bcbits |= (c->d.bc[k] & 3) << (2 * k);
  a.nf = c->nf;
  a.frc = (const double*)c->frc;
  a.frc_stride = c->nel * (long)c->n1 * c->n1;
  a.f_w = c->t_dev ? c->t_dev + 1 : nullptr;
  a.mapped = c->d.mapped;
  a.dt = dt;
  for (int k = 0; k < 4; ++k) a.alf[k] = c->alf[k];
  a.beta = c->beta;
  a.tau = c->tau;
  a.rtol = c->rtol;
  a.rtol_inner = 1e-6;
  a.maxit = c->maxit;
  a.mixed = c->d.precision == GDW_MIXED_FP32 ? 1 : 0;
  a.pc32 = c->d.precision == GDW_MIXED_PC32 ? 1 : 0;
  a.fo = c->fo;
  a.dst = c->dst;
  if (c->blk_v2) {
    a.v2 = 1;
    a.blk_off = c->blk_off;
    a.blk_dst = c->blk_dst;
    a.blk_jc = c->blk_jc;
    a.blk_gidx = c->blk_gidx;
    a.blk_unit = c->blk_unit;
    a.blk_K = c->blk_K;
    a.blk_CH = c->blk_CH;
    a.blk_WB = c->blk_WB;
    a.blk_threads = c->blk_threads;
    a.nnz_full = c->blk_nnz;
  }
  stage_roles(c, stage, a);
  return a;
}

}  // namespace gdw

template <typename T>
static hipError_t run_t(gdw_ctx* c, double dt, int steps, hipStream_t st) {
  StageArgs<T> a[4];
  for (int k = 0; k < 4; ++k) a[k] = fdm_stage_args<T>(c, k + 1, dt);
  const SourceTerms src = source_terms(c);
  hipError_t e;
  for (int s = 0; s < steps; ++s) {
    if (c->nf > 0 && (e = launch_source_step(c->t_dev, c->t_dev + 1, dt, src, st)) != hipSuccess)
      return e;
    for (int k = 0; k < 4; ++k)
      if ((e = c->dim == 3 ? launch_stage3<T>(k + 1, a[k], st) : launch_stage<T>(k + 1, a[k], st)) !=
          hipSuccess)
        return e;
    c->t += dt;
  }
  return hipSuccess;
}

static hipError_t run_pcg(gdw_ctx* c, double dt, int steps, hipStream_t st) {
  hipError_t e;
  if (!c->pargs_ok || c->pargs_dt != dt) {
    // the argument blocks are read by kernels still queued on the stream: replace them
    // only after those have run
    if (c->pargs_used && (e = hipStreamSynchronize(st)) != hipSuccess) return e;
    for (int k = 0; k < 4; ++k) {
      c->h_pargs[k] = pcg_stage_args(c, k + 1, dt);
      if (!pcg_single_shape(c->h_pargs[k], &c->p_threads, &c->p_lds)) return hipErrorInvalidValue;
    }
    if ((e = hipMemcpyAsync(c->d_pargs, c->h_pargs, sizeof(c->h_pargs), hipMemcpyHostToDevice,
                            st)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    c->pargs_dt = dt;
    c->pargs_ok = 1;
  }
  c->pargs_used = 1;
  const int key = pcg_group_key(c->h_pargs[0]);
  const bool split = pcg_split_key(key) && c->Fu != nullptr;
  const SourceTerms src = source_terms(c);
  for (int s = 0; s < steps; ++s) {
    if (c->nf > 0 && (e = launch_source_step(c->t_dev, c->t_dev + 1, dt, src, st)) != hipSuccess)
      return e;
    for (int k = 0; k < 4; ++k) {
      if (split) {
        if ((e = launch_pcg_split_stage(k + 1, key, c->d_pargs + k, c->h_pargs[k], c->p_threads,
                                        c->p_lds, st)) != hipSuccess)
          return e;
        continue;
      }
      const unsigned grid = pcg_group_grid(k + 1, key, c->p_threads, c->p_lds, c->nel);
      if ((e = launch_pcg_stage_group(k + 1, key, c->d_pargs + k, c->d_pel, 1, grid, c->p_threads,
                                      c->p_lds, st)) != hipSuccess)
        return e;
    }
    c->t += dt;
  }
  c->stages_since_state += 4LL * steps;
  return hipSuccess;
}

extern "C" gdw_status gdw_run(gdw_ctx* c, double dt, int steps, void* stream) {
  if (!c) { set_error("ctx is NULL"); return GDW_EINVAL; }
  if (!(dt > 0) || !std::isfinite(dt)) { set_error("dt must be finite and > 0"); return GDW_EINVAL; }
  if (steps < 0) { set_error("steps must be >= 0"); return GDW_EINVAL; }
  if (!c->have_state) { set_error("no state: call gdw_set_state first"); return GDW_EINVAL; }
  hipStream_t st = (hipStream_t)stream;
  if (c->solver == GDW_SOLVE_PCG)
    GDW_HIP(run_pcg(c, dt, steps, st));
  else
    GDW_HIP(c->elem_bytes == 8 ? run_t<double>(c, dt, steps, st) : run_t<float>(c, dt, steps, st));
  c->steps_taken += steps;
  return GDW_OK;
}

extern "C" gdw_status gdw_get_state(gdw_ctx* c, double* U, double* V, void* stream) {
  if (!c || !U || !V) { set_error("NULL argument"); return GDW_EINVAL; }
  hipStream_t st = (hipStream_t)stream;
  if (c->solver == GDW_SOLVE_PCG) {
    const size_t nodal = (size_t)c->nel * c->g.nn * sizeof(double);
    GDW_HIP(hipMemcpyAsync(U, c->Y[0][0], nodal, hipMemcpyDeviceToDevice, st));
    GDW_HIP(hipMemcpyAsync(V, c->Y[0][1], nodal, hipMemcpyDeviceToDevice, st));
  } else if (c->dim == 3) {
    const double* yu = c->elem_bytes == 8 ? (const double*)c->Y[0][0] : c->y64[0];
    const double* yv = c->elem_bytes == 8 ? (const double*)c->Y[0][1] : c->y64[1];
    GDW_HIP(launch_to_nodal3<double>(yu, U, c->Psx, c->Psy, c->Psz, c->n1, c->nel, st));
    GDW_HIP(launch_to_nodal3<double>(yv, V, c->Psx, c->Psy, c->Psz, c->n1, c->nel, st));
  } else if (c->elem_bytes == 8) {
    GDW_HIP(launch_to_nodal<double>((const double*)c->Y[0][0], U, c->Psx, c->Psy, c->n1, c->nel, st));
    GDW_HIP(launch_to_nodal<double>((const double*)c->Y[0][1], V, c->Psx, c->Psy, c->n1, c->nel, st));
  } else {
    GDW_HIP(launch_to_nodal<double>(c->y64[0], U, c->Psx, c->Psy, c->n1, c->nel, st));
    GDW_HIP(launch_to_nodal<double>(c->y64[1], V, c->Psx, c->Psy, c->n1, c->nel, st));
  }
  return GDW_OK;
}

extern "C" gdw_status gdw_energy(gdw_ctx* c, double* E_host, void* stream) {
  if (!c || !E_host) { set_error("NULL argument"); return GDW_EINVAL; }
  hipStream_t st = (hipStream_t)stream;
  double* out;
  if (c->solver == GDW_SOLVE_PCG) {
    out = c->epart + c->nel;
    GDW_HIP(launch_pcg_energy(c->g, c->el, (const double*)c->Y[0][0], (const double*)c->Y[0][1],
                              c->nel, c->epart, (int)c->nel, out, st));
  } else {
    out = c->epart + c->npart;
    const bool f64 = c->elem_bytes == 8;
    GDW_HIP(launch_energy<double>(f64 ? (const double*)c->Y[0][0] : c->y64[0],
                                  f64 ? (const double*)c->Y[0][1] : c->y64[1],
                                  (const double*)c->lam, c->d.c2,
                                  c->nn, c->nel, c->epart, c->npart, out, st));
  }
  GDW_HIP(hipMemcpyAsync(E_host, out, sizeof(double), hipMemcpyDeviceToHost, st));
  GDW_HIP(hipStreamSynchronize(st));
  if (!std::isfinite(*E_host)) { set_error("energy is not finite"); return GDW_ENONFINITE; }
  return GDW_OK;
}

extern "C" gdw_status gdw_get_stats(gdw_ctx* c, gdw_stats* out, void* stream) {
  if (!c || !out) { set_error("NULL argument"); return GDW_EINVAL; }
  hipStream_t st = (hipStream_t)stream;
  std::memset(out, 0, sizeof(*out));
  out->steps_taken = c->steps_taken;
  out->dof_updates = c->steps_taken * c->nel * (long long)c->nn;
  out->n1 = c->n1;
  out->precision = c->d.precision;
  out->solver = c->solver;
  out->fail_elem = -1;
  const long n = c->nel * (long)c->nn;
  GDW_HIP(hipMemsetAsync(c->nonfinite, 0, sizeof(unsigned int), st));
  for (int f = 0; f < 2; ++f) {
    const double* y = (c->solver == GDW_SOLVE_PCG || c->elem_bytes == 8) ? (const double*)c->Y[0][f]
                                                                          : c->y64[f];
    GDW_HIP(launch_count_nonfinite<double>(y, n, c->nonfinite, st));
  }
  unsigned int cnt = 0;
  GDW_HIP(hipMemcpyAsync(&cnt, c->nonfinite, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
  int fail = kFailNone;
  std::vector<int> its;
  if (c->solver == GDW_SOLVE_PCG) {
    its.resize((size_t)c->nel * kItsPer);
    GDW_HIP(hipMemcpyAsync(its.data(), c->its, its.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    GDW_HIP(hipMemcpyAsync(&fail, c->fail, sizeof(int), hipMemcpyDeviceToHost, st));
  }
  GDW_HIP(hipStreamSynchronize(st));
  if (c->solver == GDW_SOLVE_PCG) {
    long long sS = 0, sM = 0, sw = 0;
    int mS = 0, mM = 0;
    for (long e = 0; e < c->nel; ++e) {
      const int* it = &its[(size_t)e * kItsPer];
      sS += it[0];
      sM += it[1];
      mS = std::max(mS, it[2]);
      mM = std::max(mM, it[3]);
      sw += it[4] + it[5];
    }
    const long long solves = c->stages_since_state * c->nel;
    out->solves = solves;
    out->mean_it_S = solves ? (double)sS / solves : 0.0;
    out->mean_it_M = solves ? (double)sM / solves : 0.0;
    out->max_it_S = mS;
    out->max_it_M = mM;
    out->mean_refine = solves ? (double)sw / (2.0 * solves) : 0.0;
    if (fail != kFailNone) {
      out->fail_elem = fail;
      set_error("a PCG element solve reached pcg_maxit");
      return GDW_ENOCONV;
    }
  }
  if (cnt) { set_error("state holds NaN or Inf"); return GDW_ENONFINITE; }
  return GDW_OK;
}

extern "C" void gdw_destroy(gdw_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  free_all(c);
  delete c;
}

// ---------------------------------------------------------------------------------
// Learned preconditioner correction
// ---------------------------------------------------------------------------------
struct gdw_mlp {
  MlpNet net{};
  MlpWork w{};
};

static void mlp_free(gdw_mlp* m) {
  auto F = [](void* p) { if (p) (void)hipFree(p); };
  F(m->net.th); F(m->net.g); F(m->net.m); F(m->net.v); F(m->net.w16);
  F(m->w.z1); F(m->w.h1); F(m->w.z2); F(m->w.h2); F(m->w.dh); F(m->w.dz); F(m->w.out);
  F(m->w.dout); F(m->w.part); F(m->w.loss);
}

static gdw_status mlp_alloc(gdw_mlp* m, int n_in, int hidden, int n_out, int bmax) {
  MlpNet& n = m->net;
  n.n_in = n_in; n.hidden = hidden; n.n_out = n_out;
  n.oW1 = 0;
  n.ob1 = n.oW1 + (long)hidden * n_in;
  n.oW2 = n.ob1 + hidden;
  n.ob2 = n.oW2 + (long)hidden * hidden;
  n.oW3 = n.ob2 + hidden;
  n.ob3 = n.oW3 + (long)n_out * hidden;
  n.np = n.ob3 + n_out;
  GDW_HIP(hipMalloc(&n.th, n.np * sizeof(float)));
  GDW_HIP(hipMalloc(&n.g, n.np * sizeof(float)));
  GDW_HIP(hipMalloc(&n.m, n.np * sizeof(float)));
  GDW_HIP(hipMalloc(&n.v, n.np * sizeof(float)));
  GDW_HIP(hipMalloc(&n.w16, n.np * sizeof(_Float16)));
  MlpWork& w = m->w;
  w.bmax = bmax;
  const size_t bh = (size_t)bmax * hidden * sizeof(float), bk = (size_t)bmax * n_out * sizeof(float);
  GDW_HIP(hipMalloc(&w.z1, bh)); GDW_HIP(hipMalloc(&w.h1, bh)); GDW_HIP(hipMalloc(&w.z2, bh));
  GDW_HIP(hipMalloc(&w.h2, bh)); GDW_HIP(hipMalloc(&w.dh, bh)); GDW_HIP(hipMalloc(&w.dz, bh));
  GDW_HIP(hipMalloc(&w.out, bk)); GDW_HIP(hipMalloc(&w.dout, bk));
  GDW_HIP(hipMalloc(&w.part, 64 * sizeof(double)));
  return GDW_OK;
}

static gdw_status mlp_upload(gdw_mlp* m, const std::vector<float>& th) {
  MlpNet& n = m->net;
  GDW_HIP(hipMemcpy(n.th, th.data(), n.np * sizeof(float), hipMemcpyHostToDevice));
  GDW_HIP(hipMemset(n.m, 0, n.np * sizeof(float)));
  GDW_HIP(hipMemset(n.v, 0, n.np * sizeof(float)));
  GDW_HIP(hipMemset(n.g, 0, n.np * sizeof(float)));
  n.step = 0;
  GDW_HIP(mlp_refresh_half(n, nullptr));
  GDW_HIP(hipDeviceSynchronize());
  return GDW_OK;
}

extern "C" gdw_status gdw_mlp_create(int n_in, int hidden, int n_out, unsigned long long seed,
                                     int max_batch, gdw_mlp** out) {
  if (!out) { set_error("out is NULL"); return GDW_EINVAL; }
  *out = nullptr;
  if (n_in < 1 || hidden < 1 || n_out < 1 || max_batch < 1 || hidden > 4096 || n_in > 4096 ||
      n_out > 4096 || max_batch > (1 << 20)) {
    set_error("invalid network sizes"); return GDW_EINVAL;
  }
  gdw_mlp* m = new (std::nothrow) gdw_mlp();
  if (!m) { set_error("host allocation failed"); return GDW_ENOMEM; }
  gdw_status s = mlp_alloc(m, n_in, hidden, n_out, max_batch);
  if (s == GDW_OK) {
    std::vector<float> th(m->net.np, 0.f);
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    auto normal = [&]() {
      const double u1 = std::max(U(rng), 1e-300), u2 = U(rng);
      return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    };
    auto fill = [&](long off, long cnt, int fan_in) {
      const double sd = std::sqrt(2.0 / fan_in);
      for (long i = 0; i < cnt; ++i) th[off + i] = (float)(sd * normal());
    };
    fill(m->net.oW1, (long)hidden * n_in, n_in);
    fill(m->net.oW2, (long)hidden * hidden, hidden);
    fill(m->net.oW3, (long)n_out * hidden, hidden);
    s = mlp_upload(m, th);
  }
  if (s != GDW_OK) {
    mlp_free(m);
    delete m;
    return s;
  }
  *out = m;
  return GDW_OK;
}

extern "C" gdw_status gdw_mlp_num_params(const gdw_mlp* m, long long* n) {
  if (!m || !n) { set_error("NULL argument"); return GDW_EINVAL; }
  *n = m->net.np;
  return GDW_OK;
}

extern "C" gdw_status gdw_mlp_get_params(gdw_mlp* m, float* host) {
  if (!m || !host) { set_error("NULL argument"); return GDW_EINVAL; }
  GDW_HIP(hipDeviceSynchronize());
  GDW_HIP(hipMemcpy(host, m->net.th, m->net.np * sizeof(float), hipMemcpyDeviceToHost));
  return GDW_OK;
}

extern "C" gdw_status gdw_mlp_set_params(gdw_mlp* m, const float* host) {
  if (!m || !host) { set_error("NULL argument"); return GDW_EINVAL; }
  GDW_HIP(hipDeviceSynchronize());
  std::vector<float> th(host, host + m->net.np);
  return mlp_upload(m, th);
}

static gdw_status mlp_forward_all(gdw_mlp* m, const float* x, long n, float* out, hipStream_t st) {
  const int B = m->w.bmax, I = m->net.n_in, K = m->net.n_out;
  for (long i0 = 0; i0 < n; i0 += B) {
    const int b = (int)std::min<long>(B, n - i0);
    GDW_HIP(mlp_forward(m->net, x + i0 * I, b, m->w, st));
    GDW_HIP(hipMemcpyAsync(out + i0 * K, m->w.out, (size_t)b * K * sizeof(float),
                           hipMemcpyDeviceToDevice, st));
  }
  return GDW_OK;
}

extern "C" gdw_status gdw_mlp_forward(gdw_mlp* m, const float* x, int n, float* out, void* stream) {
  if (!m || n < 0 || (n > 0 && (!x || !out))) { set_error("invalid argument"); return GDW_EINVAL; }
  return mlp_forward_all(m, x, n, out, (hipStream_t)stream);
}

extern "C" gdw_status gdw_mlp_grad(gdw_mlp* m, const float* x, const float* y, int n, float* grad,
                                   double* loss_host, void* stream) {
  if (!m || !x || !y || !grad || n < 1 || n > m->w.bmax) { set_error("invalid argument"); return GDW_EINVAL; }
  hipStream_t st = (hipStream_t)stream;
  double* acc = nullptr;
  GDW_HIP(hipMalloc(&acc, sizeof(double)));
  gdw_status s = GDW_OK;
  hipError_t e = hipMemsetAsync(acc, 0, sizeof(double), st);
  if (e == hipSuccess) e = mlp_forward(m->net, x, n, m->w, st);
  if (e == hipSuccess) e = mlp_backward(m->net, x, y, n, m->w, acc, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(grad, m->net.g, m->net.np * sizeof(float), hipMemcpyDeviceToDevice, st);
  double loss = 0.0;
  if (e == hipSuccess) e = hipMemcpyAsync(&loss, acc, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(acc);
  if (e != hipSuccess) { set_error(std::string("gdw_mlp_grad: ") + hipGetErrorString(e)); s = GDW_EHIP; }
  if (loss_host) *loss_host = loss;
  return s;
}

extern "C" gdw_status gdw_mlp_train(gdw_mlp* m, const float* x, const float* y, int n, int epochs,
                                    int batch, float lr, double* loss_host, void* stream) {
  if (!m || !x || !y || n < 1 || epochs < 0 || batch < 1 || batch > m->w.bmax || !(lr > 0)) {
    set_error("invalid argument"); return GDW_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  double* acc = nullptr;
  GDW_HIP(hipMalloc(&acc, std::max(epochs, 1) * sizeof(double)));
  hipError_t e = hipMemsetAsync(acc, 0, std::max(epochs, 1) * sizeof(double), st);
  const int I = m->net.n_in, K = m->net.n_out;
  const long nbatch = (n + batch - 1) / batch;
  for (int ep = 0; ep < epochs && e == hipSuccess; ++ep)
    for (long b = 0; b < nbatch && e == hipSuccess; ++b) {
      const long i0 = b * batch;
      const int bs = (int)std::min<long>(batch, n - i0);
      e = mlp_forward(m->net, x + i0 * I, bs, m->w, st);
      if (e == hipSuccess) e = mlp_backward(m->net, x + i0 * I, y + i0 * K, bs, m->w, acc + ep, st);
      if (e == hipSuccess) e = mlp_adam(m->net, lr, st);
    }
  std::vector<double> h(std::max(epochs, 1));
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), acc, h.size() * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(acc);
  if (e != hipSuccess) { set_error(std::string("gdw_mlp_train: ") + hipGetErrorString(e)); return GDW_EHIP; }
  if (loss_host)
    for (int ep = 0; ep < epochs; ++ep) loss_host[ep] = h[ep] / (double)nbatch;
  return GDW_OK;
}

// ---------------------------------------------------------------------------------
// Allocation-free network gradient.  The activations, the loss partial sums and the
// output gradient of one minibatch live in `scratch`, a file-scope device array of
// kScratchBytes on every device the library runs on (held until the process ends).
// Host code never passes `scratch` itself (its name is a host-side stand-in, not a
// device address): the device address comes from hipGetSymbolAddress, taken once per
// device with that device current, and is kept in g_scratch_ptr.
// ---------------------------------------------------------------------------------
static constexpr size_t kScratchBytes = (size_t)8 << 20;     // 8 MiB per device
static constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static gdw_status scratch_address(void** out) {
  int dev = -1;
  GDW_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) { set_error("device index out of range"); return GDW_EINVAL; }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    GDW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GDW_OK;
}

extern "C" gdw_status gdw_mlp_grad_noalloc(gdw_mlp* m, const float* x, const float* y, int n,
                                           float* grad, double* loss, void* stream) {
  if (!m || !x || !y || !grad || !loss || n < 1) { set_error("invalid argument"); return GDW_EINVAL; }
  const int H = m->net.hidden, K = m->net.n_out;
  const size_t part = 64 * sizeof(double);
  const size_t need = part + (size_t)n * (6 * (size_t)H + 2 * (size_t)K) * sizeof(float);
  if (need > kScratchBytes) {
    set_error("gdw_mlp_grad_noalloc: " + std::to_string(n) + " rows need " + std::to_string(need) +
              " bytes of scratch; the limit is " + std::to_string(kScratchBytes));
    return GDW_EINVAL;
  }
  void* base = nullptr;
  gdw_status s = scratch_address(&base);
  if (s != GDW_OK) return s;
  MlpWork w{};
  w.bmax = n;
  w.part = (double*)base;
  float* f = (float*)((unsigned char*)base + part);
  const size_t nh = (size_t)n * H, nk = (size_t)n * K;
  w.z1 = f; f += nh;
  w.h1 = f; f += nh;
  w.z2 = f; f += nh;
  w.h2 = f; f += nh;
  w.dh = f; f += nh;
  w.dz = f; f += nh;
  w.out = f; f += nk;
  w.dout = f;
  MlpNet net = m->net;      // same parameters; the gradient goes straight to `grad`
  net.g = grad;
  hipStream_t st = (hipStream_t)stream;
  GDW_HIP(launch_zero_f64(loss, 1, st));
  GDW_HIP(mlp_forward(net, x, n, w, st));
  GDW_HIP(mlp_backward(net, x, y, n, w, loss, st));
  return GDW_OK;
}

extern "C" void gdw_mlp_destroy(gdw_mlp* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  mlp_free(m);
  delete m;
}

extern "C" gdw_status gdw_precond_data(gdw_ctx* c, float* samples, float* targets, void* stream) {
  if (!c) { set_error("ctx is NULL"); return GDW_EINVAL; }
  if (c->solver != GDW_SOLVE_PCG || !c->have_coeff) {
    set_error("gdw_precond_data needs the PCG path after gdw_set_coeff"); return GDW_EINVAL;
  }
  GDW_HIP(launch_precond_data(c->g, c->el, c->c2n, c->Bs, samples, targets, c->nel, (hipStream_t)stream));
  return GDW_OK;
}

extern "C" gdw_status gdw_ic0_solve(gdw_ctx* c, int op, const double* b, double* x, double rtol,
                                    int maxit, int* its, void* stream) {
  if (!c || !b || !x || !its) { set_error("NULL argument"); return GDW_EINVAL; }
  if (c->solver != GDW_SOLVE_PCG || !c->have_coeff || c->dim != 2) {
    set_error("gdw_ic0_solve needs the 2D PCG path after gdw_set_coeff"); return GDW_EINVAL;
  }
  if (op != 0 && op != 1) { set_error("op must be 0 (S_hat) or 1 (M_J)"); return GDW_EINVAL; }
  if (!(rtol >= 0.0) || maxit < 1) { set_error("rtol >= 0 and maxit >= 1 required"); return GDW_EINVAL; }
  hipStream_t st = (hipStream_t)stream;
  const long nel = c->nel;
  if (!c->ic0_flags) {  // workspace of the first call, kept until gdw_destroy
    std::vector<int> lv;
    gdw::ic0_levels(c->g.N, c->g.p, lv, &c->ic0_nfw, &c->ic0_nbw);
    const size_t opb = (size_t)nel * c->g.nst * sizeof(double);
    hipError_t ea = hipMalloc(&c->ic0_A, opb);
    if (ea == hipSuccess) ea = hipMalloc(&c->ic0_U, opb);
    if (ea == hipSuccess) ea = hipMalloc(&c->ic0_lv, lv.size() * sizeof(int));
    if (ea == hipSuccess)
      ea = hipMemcpy(c->ic0_lv, lv.data(), lv.size() * sizeof(int), hipMemcpyHostToDevice);
    if (ea == hipSuccess) ea = hipMalloc(&c->ic0_flags, 2 * sizeof(int));
    if (ea != hipSuccess) {  // leave no half-made workspace behind
      for (void* q : {(void*)c->ic0_A, (void*)c->ic0_U, (void*)c->ic0_lv, (void*)c->ic0_flags})
        if (q) (void)hipFree(q);
      c->ic0_A = c->ic0_U = nullptr;
      c->ic0_lv = c->ic0_flags = nullptr;
      set_error(std::string("gdw_ic0_solve workspace: ") + hipGetErrorString(ea));
      return ea == hipErrorOutOfMemory ? GDW_ENOMEM : GDW_EHIP;
    }
  }
  int* flags = c->ic0_flags;
  hipError_t e = hipMemsetAsync(flags, 0x7f, 2 * sizeof(int), st);
  if (e == hipSuccess)
    e = gdw::launch_ic0(c->g, c->el, op, nel, c->ic0_A, c->ic0_U, c->ic0_lv, c->ic0_nfw,
                        c->ic0_nbw, b, x, rtol, maxit, its, flags, flags + 1, st);
  int hf[2] = {kFailNone, kFailNone};
  if (e == hipSuccess) e = hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_error(std::string("gdw_ic0_solve: ") + hipGetErrorString(e));
    return GDW_EHIP;
  }
  if (hf[0] != kFailNone) {
    set_error("IC(0) breakdown (non-positive pivot) in element " + std::to_string(hf[0]));
    return GDW_ENOCONV;
  }
  if (hf[1] != kFailNone) {
    set_error("IC(0)-PCG reached maxit in element " + std::to_string(hf[1]));
    return GDW_ENOCONV;
  }
  return GDW_OK;
}

static gdw_status ensure_dlog(gdw_ctx* c) {
  if (!c->el.dlog) {
    GDW_HIP(hipMalloc(&c->el.dlog, (size_t)c->nel * c->g.nn * sizeof(float)));
    GDW_HIP(hipMalloc(&c->el.dscale, (size_t)c->nel * c->g.nn * sizeof(double)));
    args_changed(c);
  }
  return GDW_OK;
}

extern "C" gdw_status gdw_set_precond_log(gdw_ctx* c, const float* log_scale, void* stream) {
  if (!c) { set_error("ctx is NULL"); return GDW_EINVAL; }
  if (c->solver != GDW_SOLVE_PCG) { set_error("PCG path only"); return GDW_EINVAL; }
  hipStream_t st = (hipStream_t)stream;
  if (!log_scale) {
    GDW_HIP(hipStreamSynchronize(st));
    if (c->el.dlog) (void)hipFree(c->el.dlog);
    if (c->el.dscale) (void)hipFree(c->el.dscale);
    c->el.dlog = nullptr;
    c->el.dscale = nullptr;
    args_changed(c);
    return GDW_OK;
  }
  gdw_status s = ensure_dlog(c);
  if (s != GDW_OK) return s;
  GDW_HIP(launch_set_dlog(log_scale, c->nel, c->g.nn, c->el.dlog, c->el.dscale, st));
  return GDW_OK;
}

extern "C" gdw_status gdw_set_precond_mlp(gdw_ctx* c, gdw_mlp* m, void* stream) {
  if (!c || !m) { set_error("NULL argument"); return GDW_EINVAL; }
  if (c->solver != GDW_SOLVE_PCG || !c->have_coeff) {
    set_error("gdw_set_precond_mlp needs the PCG path after gdw_set_coeff"); return GDW_EINVAL;
  }
  if (m->net.n_in != 64 || m->net.n_out != c->g.nn - 1) {
    set_error("network must map 64 samples to (N+1)^2 - 1 outputs"); return GDW_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  gdw_status s = ensure_dlog(c);
  if (s != GDW_OK) return s;
  float *smp = nullptr, *out = nullptr;
  GDW_HIP(hipMalloc(&smp, (size_t)c->nel * 64 * sizeof(float)));
  hipError_t e = hipMalloc(&out, (size_t)c->nel * (c->g.nn - 1) * sizeof(float));
  if (e == hipSuccess) e = launch_precond_data(c->g, c->el, c->c2n, c->Bs, smp, nullptr, c->nel, st);
  if (e == hipSuccess && mlp_forward_all(m, smp, c->nel, out, st) != GDW_OK) e = hipErrorUnknown;
  if (e == hipSuccess) e = launch_set_dlog(out, c->nel, c->g.nn, c->el.dlog, c->el.dscale, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(smp);
  if (out) (void)hipFree(out);
  if (e != hipSuccess) { set_error(std::string("gdw_set_precond_mlp: ") + hipGetErrorString(e)); return GDW_EHIP; }
  return GDW_OK;
}
