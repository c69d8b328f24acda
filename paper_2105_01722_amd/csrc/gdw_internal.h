// Internal declarations shared by the translation units of libgdw.
#pragma once

#include <cstddef>
#include <string>

#include "../../include/gdw.h"

namespace gdw {

// ---- host 1D GD construction (gd1d_host.cpp) ---------------------------------
void gauss_legendre01(int n, double* x, double* w);
int gd_window_start(int k, int N, int p);
// Unit-spacing mass, stiffness ((N+1)^2 row-major) and face derivative vectors.
void gd1d_unit(int N, int p, double* M, double* S, double* dL, double* dR);
// Values / t-derivatives of all N+1 basis functions at t inside cell k.
void gd1d_eval_cell(int N, int p, int k, double t, double* val, double* der);

// ---- error reporting (api.hip) ---------------------------------------------------
void set_error(const std::string& msg);

}  // namespace gdw
