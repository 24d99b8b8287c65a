// lsh_internal.hpp -- host-side pattern object shared by the library's sources.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lsh.h"
#include "lsh_fft.hpp"
#include "lsh_green.hpp"

struct lsh_pattern {
  // ---- Sec. 2.1: M, m, SNF M = U diag(e) V.  A two-dimensional pattern
  // (d = 2) is held as M = blockdiag(M2, 1): its frequencies all have k3 = 0,
  // so the three-dimensional operators act on it as their plane-strain forms.
  int d = 3;
  int64_t M[9];
  int64_t det;
  int64_t m;
  int64_t U[9], V[9];
  int64_t e[3];
  int64_t adjM[9];   // adj(M): M^{-1} = adj(M) / det
  FftPlan plan[3];   // radix plans per SNF axis (nst = -1 if unsupported)

  // ---- Sec. 2.2: generating function
  int kind = -1;
  double alpha[3] = {0, 0, 0};
  int nxi = 0;
  double Xi[3 * LSH_MAX_XI];
  int R = 16;
  int tail = 0;                  // Box spline: tail of the alias sums beyond R

  // ---- Def. (weak_pde): stiffness field
  int nphase = 0;
  std::vector<double> C_voigt;   // nphase * 36
  double C0_voigt[36];
  std::vector<uint8_t> phase;    // m, storage order
  int scheme = 0;                // lsh_scheme: 0 Lippmann-Schwinger, 1 variational

  // ---- device binding (one precision at a time)
  int bound_prec = -1;
  char* dev_persist = nullptr;
  size_t off_phase = 0, off_tw[3] = {0, 0, 0}, off_table = 0, off_dmat = 0, off_cmat = 0;
  bool has_table = false;

  // ---- kernel variants chosen by lsh_autotune, per precision (0: FP64, 1: FP32)
  int tuned[2] = {0, 0};
  int tune_choice[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};  // stress, axis 2, Green pass, schedule
};

// ---- helpers implemented in lsh_host.cpp
void lsh_set_error(const std::string& msg);
int lsh_fail(int status, const std::string& msg);
void lsh_green_params(const lsh_pattern* p, GreenParams* gp);
bool lsh_make_plan(int64_t N, FftPlan* pl);
void lsh_voigt_to_mandel(const double* Cv, double* Cm);
void lsh_voigt_to_tensor(const double* Cv, double* C4);
size_t lsh_align(size_t x);
