// lsh_host.cpp -- host half of the C ABI: patterns, Smith normal form, kernel
// and stiffness validation.
//
// Sec. 2.1: the pattern P(M) = M^{-1} Z^3 cap [-1/2,1/2)^3 of a regular integer
// matrix M has m = |det M| points; the generating set is G(M^T).  With the
// integer Smith normal form M = U diag(e1,e2,e3) V the point of grid index a is
// y = M^{-1} U a mod 1 and the frequency of grid index b is h = V^T b mod M^T,
// which turns the pattern DFT of eq. (Fouriermatrix) into a 3-D DFT over the
// grid Z_e1 x Z_e2 x Z_e3.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lsh_internal.hpp"

static thread_local std::string g_err;

void lsh_set_error(const std::string& msg) { g_err = msg; }
int lsh_fail(int status, const std::string& msg) {
  g_err = msg;
  return status;
}
extern "C" const char* lsh_last_error(void) { return g_err.c_str(); }

size_t lsh_align(size_t x) { return (x + 255) & ~(size_t)255; }

// ------------------------------------------------------------ integer algebra
static int64_t det3(const int64_t* A) {
  __int128 d = (__int128)A[0] * ((__int128)A[4] * A[8] - (__int128)A[5] * A[7]) -
               (__int128)A[1] * ((__int128)A[3] * A[8] - (__int128)A[5] * A[6]) +
               (__int128)A[2] * ((__int128)A[3] * A[7] - (__int128)A[4] * A[6]);
  return (int64_t)d;
}

static void adj3(const int64_t* A, int64_t* out) {
  // out = adj(A), A adj(A) = det(A) I
  out[0] = A[4] * A[8] - A[5] * A[7];
  out[1] = A[2] * A[7] - A[1] * A[8];
  out[2] = A[1] * A[5] - A[2] * A[4];
  out[3] = A[5] * A[6] - A[3] * A[8];
  out[4] = A[0] * A[8] - A[2] * A[6];
  out[5] = A[2] * A[3] - A[0] * A[5];
  out[6] = A[3] * A[7] - A[4] * A[6];
  out[7] = A[1] * A[6] - A[0] * A[7];
  out[8] = A[0] * A[4] - A[1] * A[3];
}

static int64_t egcd(int64_t a, int64_t b, int64_t* x, int64_t* y) {
  // x a + y b = g >= 0
  int64_t x0 = 1, y0 = 0, x1 = 0, y1 = 1;
  while (b != 0) {
    int64_t q = a / b, t;
    t = a - q * b; a = b; b = t;
    t = x0 - q * x1; x0 = x1; x1 = t;
    t = y0 - q * y1; y0 = y1; y1 = t;
  }
  if (a < 0) { a = -a; x0 = -x0; y0 = -y0; }
  *x = x0;
  *y = y0;
  return a;
}

// Smith normal form by Bezout row/column operations on a working copy A,
// keeping M = U A V throughout.  Returns false on a singular matrix.
static bool snf3(const int64_t* M, int64_t* U, int64_t* e, int64_t* V) {
  int64_t A[3][3];
  int64_t Um[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, Vm[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int i = 0; i < 9; ++i) A[i / 3][i % 3] = M[i];
  for (int t = 0; t < 3; ++t) {
    for (int guard = 0; guard < 10000; ++guard) {
      int bi = -1, bj = -1;
      for (int i = t; i < 3; ++i)
        for (int j = t; j < 3; ++j)
          if (A[i][j] != 0 && (bi < 0 || std::llabs(A[i][j]) < std::llabs(A[bi][bj]))) { bi = i; bj = j; }
      if (bi < 0) return false;
      if (bi != t) {  // swap rows of A, columns of U
        for (int k = 0; k < 3; ++k) { std::swap(A[t][k], A[bi][k]); std::swap(Um[k][t], Um[k][bi]); }
      }
      if (bj != t) {  // swap columns of A, rows of V
        for (int k = 0; k < 3; ++k) { std::swap(A[k][t], A[k][bj]); std::swap(Vm[t][k], Vm[bj][k]); }
      }
      for (int i = t + 1; i < 3; ++i) {
        if (A[i][t] == 0) continue;
        int64_t x, y;
        const int64_t a = A[t][t], b = A[i][t];
        const int64_t g = egcd(a, b, &x, &y);
        const int64_t ap = a / g, bp = b / g;
        for (int k = 0; k < 3; ++k) {  // rows: [t; i] <- [[x, y], [-bp, ap]] [t; i]
          const int64_t rt = A[t][k], ri = A[i][k];
          A[t][k] = x * rt + y * ri;
          A[i][k] = -bp * rt + ap * ri;
        }
        for (int k = 0; k < 3; ++k) {  // U <- U E^{-1}, E^{-1} = [[ap, -y], [bp, x]]
          const int64_t ct = Um[k][t], ci = Um[k][i];
          Um[k][t] = ap * ct + bp * ci;
          Um[k][i] = -y * ct + x * ci;
        }
      }
      for (int j = t + 1; j < 3; ++j) {
        if (A[t][j] == 0) continue;
        int64_t x, y;
        const int64_t a = A[t][t], b = A[t][j];
        const int64_t g = egcd(a, b, &x, &y);
        const int64_t ap = a / g, bp = b / g;
        for (int k = 0; k < 3; ++k) {  // cols: [t, j] <- [t, j] [[x, -bp], [y, ap]]
          const int64_t ct = A[k][t], cj = A[k][j];
          A[k][t] = x * ct + y * cj;
          A[k][j] = -bp * ct + ap * cj;
        }
        for (int k = 0; k < 3; ++k) {  // V <- F^{-1} V, F^{-1} = [[ap, bp], [-y, x]]
          const int64_t rt = Vm[t][k], rj = Vm[j][k];
          Vm[t][k] = ap * rt + bp * rj;
          Vm[j][k] = -y * rt + x * rj;
        }
      }
      bool clean = true;
      for (int i = t + 1; i < 3; ++i) clean = clean && A[i][t] == 0;
      if (!clean) continue;
      int bad = -1;
      for (int i = t + 1; i < 3; ++i)
        for (int j = t + 1; j < 3; ++j)
          if (A[i][j] % A[t][t] != 0) bad = i;
      if (bad >= 0) {  // row_t += row_bad; U: col_bad -= col_t
        for (int k = 0; k < 3; ++k) { A[t][k] += A[bad][k]; Um[k][bad] -= Um[k][t]; }
        continue;
      }
      break;
    }
    if (A[t][t] < 0) {
      for (int k = 0; k < 3; ++k) { A[t][k] = -A[t][k]; Um[k][t] = -Um[k][t]; }
    }
  }
  for (int i = 0; i < 3; ++i) {
    e[i] = A[i][i];
    for (int j = 0; j < 3; ++j) { U[3 * i + j] = Um[i][j]; V[3 * i + j] = Vm[i][j]; }
  }
  return e[0] > 0 && e[1] > 0 && e[2] > 0 && e[1] % e[0] == 0 && e[2] % e[1] == 0;
}

// ---------------------------------------------------------------- FFT plans
bool lsh_make_plan(int64_t N, FftPlan* pl) {
  pl->N = (int)N;
  pl->nst = 0;
  int64_t n = N;
  static const int rads[] = {8, 4, 2, 3, 5, 7, 11, 13};
  for (int r : rads) {
    while (n % r == 0 && pl->nst < LSH_MAX_STAGES) {
      pl->rad[pl->nst++] = r;
      n /= r;
    }
  }
  if (n != 1) {
    pl->nst = -1;
    return false;
  }
  return true;
}

// --------------------------------------------------------------- conversions
static const int kPair[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};

void lsh_voigt_to_mandel(const double* Cv, double* Cm) {
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J)
      Cm[6 * I + J] = Cv[6 * I + J] * (I < 3 ? 1.0 : M_SQRT2) * (J < 3 ? 1.0 : M_SQRT2);
}

void lsh_voigt_to_tensor(const double* Cv, double* C4) {
  int idx[3][3];
  for (int I = 0; I < 6; ++I) idx[kPair[I][0]][kPair[I][1]] = idx[kPair[I][1]][kPair[I][0]] = I;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) C4[((i * 3 + j) * 3 + k) * 3 + l] = Cv[6 * idx[i][j] + idx[k][l]];
}

static bool spd6(const double* Cm) {
  // Cholesky of a 6x6 symmetric matrix
  double L[36] = {0};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = Cm[6 * i + j];
      for (int k = 0; k < j; ++k) s -= L[6 * i + k] * L[6 * j + k];
      if (i == j) {
        if (!(s > 0.0)) return false;
        L[6 * i + i] = sqrt(s);
      } else {
        L[6 * i + j] = s / L[6 * j + j];
      }
    }
  return true;
}

static int check_stiffness(const double* Cv, const char* what) {
  double mx = 0.0;
  for (int i = 0; i < 36; ++i) {
    if (!std::isfinite(Cv[i])) return lsh_fail(LSH_EINVAL, std::string(what) + " has a non-finite entry");
    mx = std::max(mx, fabs(Cv[i]));
  }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < i; ++j)
      if (fabs(Cv[6 * i + j] - Cv[6 * j + i]) > 1e-12 * mx)
        return lsh_fail(LSH_ENOTELLIPTIC, std::string(what) + " is not symmetric (major symmetry)");
  double Cm[36];
  lsh_voigt_to_mandel(Cv, Cm);
  if (!spd6(Cm)) return lsh_fail(LSH_ENOTELLIPTIC, std::string(what) + " is not positive definite");
  return LSH_OK;
}

void lsh_green_params(const lsh_pattern* p, GreenParams* gp) {
  memset(gp, 0, sizeof(*gp));
  gp->kind = p->kind;
  gp->flat3 = p->d == 2 ? 1 : 0;
  gp->nxi = p->nxi;
  gp->tail = p->kind == LSH_BOXSPLINE ? p->tail : 0;
  gp->nslow = 0;
  for (int i = 0; i < 3 && gp->tail; ++i) {
    if (p->d == 2 && i == 2) continue;  // the embedding's third axis carries no aliases
    int cnt = 0, col = -1;
    for (int c = 0; c < p->nxi; ++c)
      if (p->Xi[3 * c + i] != 0.0) {
        ++cnt;
        col = c;
      }
    if (cnt == 1 && fabs(p->Xi[3 * col + i]) == 1.0) {
      gp->slow_axis[gp->nslow] = i;
      gp->slow_col[gp->nslow] = col;
      ++gp->nslow;
    }
  }
  gp->R = p->R;
  gp->m = p->m;
  for (int i = 0; i < 3; ++i) gp->e[i] = p->e[i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      gp->VT[3 * i + j] = p->V[3 * j + i];
      gp->MT[3 * i + j] = p->M[3 * j + i];
      // sign(det) adj(M^T) = sign(det) adj(M)^T
      gp->A[3 * i + j] = (p->det > 0 ? 1 : -1) * p->adjM[3 * j + i];
    }
  for (int i = 0; i < 3; ++i) gp->alpha[i] = p->alpha[i];
  gp->xi_int = 1;
  for (int i = 0; i < 3 * LSH_MAX_XI; ++i) {
    gp->Xi[i] = p->Xi[i];
    if (p->Xi[i] != floor(p->Xi[i])) gp->xi_int = 0;
  }
  lsh_voigt_to_tensor(p->C0_voigt, gp->C0);
  // isotropic C0 (to 1e-13 of its largest entry) with mu0 > 0, lam0 + 2 mu0 > 0
  const double* C = p->C0_voigt;
  const double lam = C[1], mu = C[21];
  double mx = 0.0;
  for (int i = 0; i < 36; ++i) mx = fmax(mx, fabs(C[i]));
  bool iso = mu > 0.0 && lam + 2.0 * mu > 0.0;
  for (int I = 0; I < 6 && iso; ++I)
    for (int J = 0; J < 6; ++J) {
      double want = 0.0;
      if (I < 3 && J < 3) want = lam + (I == J ? 2.0 * mu : 0.0);
      if (I >= 3 && I == J) want = mu;
      if (fabs(C[6 * I + J] - want) > 1e-13 * mx) iso = false;
    }
  gp->iso = iso ? 1 : 0;
  gp->mu0 = iso ? mu : 1.0;
  gp->riso = iso ? (lam + mu) / (mu * (lam + 2.0 * mu)) : 0.0;
}

// ------------------------------------------------------------------ the ABI
extern "C" int lsh_create_pattern(int d, const int64_t* Md, lsh_pattern** out) {
  if (!out || !Md) return lsh_fail(LSH_EINVAL, "null argument");
  *out = nullptr;
  if (d != 2 && d != 3) return lsh_fail(LSH_EINVAL, "d must be 2 or 3");
  // d = 2: M = blockdiag(M2, 1) (a single point along the third axis)
  int64_t M[9];
  if (d == 3) {
    memcpy(M, Md, sizeof(M));
  } else {
    const int64_t E[9] = {Md[0], Md[1], 0, Md[2], Md[3], 0, 0, 0, 1};
    memcpy(M, E, sizeof(M));
  }
  for (int i = 0; i < 9; ++i)
    if (std::llabs(M[i]) > (1 << 20)) return lsh_fail(LSH_EUNSUPPORTED, "entries of M beyond 2^20");
  const int64_t det = det3(M);
  if (det == 0) return lsh_fail(LSH_ESINGULAR, "det M == 0: the pattern needs a regular matrix");
  if (std::llabs(det) > ((int64_t)1 << 31)) return lsh_fail(LSH_EUNSUPPORTED, "|det M| beyond 2^31 points");
  lsh_pattern* p = new lsh_pattern();
  p->d = d;
  memcpy(p->M, M, sizeof(p->M));
  p->det = det;
  p->m = std::llabs(det);
  adj3(M, p->adjM);
  if (!snf3(M, p->U, p->e, p->V)) {
    delete p;
    return lsh_fail(LSH_ESINGULAR, "Smith normal form failed (singular matrix)");
  }
  // check M == U diag(e) V exactly
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      __int128 s = 0;
      for (int k = 0; k < 3; ++k) s += (__int128)p->U[3 * i + k] * p->e[k] * p->V[3 * k + j];
      if (s != M[3 * i + j]) {
        delete p;
        // only an int64 overflow inside the elimination can break the identity
        return lsh_fail(LSH_EUNSUPPORTED, "M's entries are too large for the exact integer Smith normal form");
      }
    }
  for (int i = 0; i < 3; ++i) lsh_make_plan(p->e[i], &p->plan[i]);
  memset(p->Xi, 0, sizeof(p->Xi));
  *out = p;
  return LSH_OK;
}

extern "C" void lsh_destroy(lsh_pattern* p) { delete p; }

extern "C" int lsh_pattern_info(const lsh_pattern* p, int64_t* m, int64_t e[3]) {
  if (!p) return lsh_fail(LSH_EINVAL, "null pattern");
  if (m) *m = p->m;
  if (e) for (int i = 0; i < 3; ++i) e[i] = p->e[i];
  return LSH_OK;
}

extern "C" int lsh_pattern_snf(const lsh_pattern* p, int64_t U[9], int64_t V[9]) {
  if (!p || !U || !V) return lsh_fail(LSH_EINVAL, "null argument");
  memcpy(U, p->U, sizeof(p->U));
  memcpy(V, p->V, sizeof(p->V));
  return LSH_OK;
}

extern "C" int lsh_pattern_points(const lsh_pattern* p, int64_t* y) {
  if (!p || !y) return lsh_fail(LSH_EINVAL, "null argument");
  // y_num = center_mod(sign(det) adj(M) U a, m)
  int64_t T[9];
  const int64_t s = p->det > 0 ? 1 : -1;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      int64_t v = 0;
      for (int k = 0; k < 3; ++k) v += p->adjM[3 * i + k] * p->U[3 * k + j];
      T[3 * i + j] = s * v;
    }
  const int64_t m = p->m, h = m / 2;
  int64_t idx = 0;
  for (int64_t a0 = 0; a0 < p->e[0]; ++a0)
    for (int64_t a1 = 0; a1 < p->e[1]; ++a1)
      for (int64_t a2 = 0; a2 < p->e[2]; ++a2, ++idx)
        for (int i = 0; i < 3; ++i) {
          __int128 v = (__int128)T[3 * i] * a0 + (__int128)T[3 * i + 1] * a1 + (__int128)T[3 * i + 2] * a2;
          int64_t r = (int64_t)((v + h) % m);
          if (r < 0) r += m;
          // d = 2: the third coordinate is 0 for every point and is not returned
          if (i < p->d) y[p->d * idx + i] = r - h;
        }
  return LSH_OK;
}

extern "C" int lsh_set_kernel(lsh_pattern* p, lsh_kernel kind, const double* params, int nparams) {
  if (!p) return lsh_fail(LSH_EINVAL, "null pattern");
  p->tuned[0] = p->tuned[1] = 0;
  if (nparams < 0 || (nparams > 0 && !params)) return lsh_fail(LSH_EINVAL, "bad parameter array");
  for (int i = 0; i < nparams; ++i)
    if (!std::isfinite(params[i])) return lsh_fail(LSH_EINVAL, "non-finite kernel parameter");
  switch (kind) {
    case LSH_DIRICHLET:
    case LSH_DIRICHLET_MODIFIED:
      if (nparams != 0) return lsh_fail(LSH_EINVAL, "Dirichlet kernels take no parameters");
      break;
    case LSH_DLVP:
      if (nparams != p->d) return lsh_fail(LSH_EINVAL, "dlVP needs alpha[d]");
      for (int i = 0; i < nparams; ++i)
        if (!(params[i] >= 0.0 && params[i] <= 1.0)) return lsh_fail(LSH_EINVAL, "dlVP alpha must lie in [0, 1]");
      for (int i = 0; i < 3; ++i) p->alpha[i] = i < nparams ? params[i] : 0.5;  // d = 2: the third factor is 1 at x3 = 0
      break;
    case LSH_BOXSPLINE: {
      const int d = p->d;
      if (nparams < 1) return lsh_fail(LSH_EINVAL, "Box spline needs {s, Xi[d s], R}");
      const int s = (int)params[0];
      // d = 2 appends the direction e3 (its factor vanishes at every alias z3 != 0)
      if (s < d || s + (3 - d) > LSH_MAX_XI || (double)s != params[0])
        return lsh_fail(LSH_EINVAL, "Box spline: s must be an integer in [d, 16 - (3 - d)]");
      if (nparams < 1 + d * s || nparams > 3 + d * s)
        return lsh_fail(LSH_EINVAL, "Box spline: expected {s, Xi[d s]} and optionally R and the tail flag");
      double XiXt[9] = {0};
      memset(p->Xi, 0, sizeof(p->Xi));
      for (int c = 0; c < s; ++c)
        for (int i = 0; i < d; ++i) p->Xi[3 * c + i] = params[1 + i * s + c];
      if (d == 2) p->Xi[3 * s + 2] = 1.0;
      const int sx = s + (3 - d);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int c = 0; c < sx; ++c) XiXt[3 * i + j] += p->Xi[3 * c + i] * p->Xi[3 * c + j];
      const double dd = XiXt[0] * (XiXt[4] * XiXt[8] - XiXt[5] * XiXt[7]) - XiXt[1] * (XiXt[3] * XiXt[8] - XiXt[5] * XiXt[6]) +
                        XiXt[2] * (XiXt[3] * XiXt[7] - XiXt[4] * XiXt[6]);
      if (!(dd > 1e-12)) return lsh_fail(LSH_EINVAL, "Box spline directions must span R^d (Sec. 2.2)");
      p->nxi = sx;
      p->R = 16;
      p->tail = 0;
      if (nparams == 3 + d * s) {
        const double t = params[2 + d * s];
        if (t != 0.0 && t != 1.0) return lsh_fail(LSH_EINVAL, "Box spline: the tail flag must be 0 or 1");
        p->tail = (int)t;
      }
      if (nparams >= 2 + d * s) {
        const double r = params[1 + d * s];
        if (!(r >= 0 && r <= 64) || (double)(int)r != r) return lsh_fail(LSH_EINVAL, "Box spline: R must be an integer in [0, 64]");
        p->R = (int)r;
      }
      break;
    }
    default:
      return lsh_fail(LSH_EINVAL, "unknown kernel kind");
  }
  p->kind = (int)kind;
  p->bound_prec = -1;  // device data must be rebuilt
  return LSH_OK;
}

extern "C" int lsh_set_scheme(lsh_pattern* p, lsh_scheme scheme) {
  if (!p) return lsh_fail(LSH_EINVAL, "null pattern");
  if (scheme != LSH_SCHEME_LS && scheme != LSH_SCHEME_VE && scheme != LSH_SCHEME_CG && scheme != LSH_SCHEME_LS_INC)
    return lsh_fail(LSH_EINVAL, "unknown scheme");
  if (p->scheme != (int)scheme) {
    p->scheme = (int)scheme;
    p->bound_prec = -1;  // the stress matrices on the device depend on the scheme
  }
  return LSH_OK;
}

// d = 2: 3x3 Voigt matrices (11, 22, 12), symmetric positive definite in Mandel form.
static int check_stiffness_plane(const double* Cv, const char* what) {
  double mx = 0.0;
  for (int i = 0; i < 9; ++i) {
    if (!std::isfinite(Cv[i])) return lsh_fail(LSH_EINVAL, std::string(what) + " has a non-finite entry");
    mx = std::max(mx, fabs(Cv[i]));
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < i; ++j)
      if (fabs(Cv[3 * i + j] - Cv[3 * j + i]) > 1e-12 * mx)
        return lsh_fail(LSH_ENOTELLIPTIC, std::string(what) + " is not symmetric (major symmetry)");
  const double w[3] = {1.0, 1.0, M_SQRT2};
  double A[9];
  for (int i = 0; i < 9; ++i) A[i] = Cv[i] * w[i / 3] * w[i % 3];
  // leading principal minors of the Mandel matrix
  const double d1 = A[0], d2 = A[0] * A[4] - A[1] * A[3];
  const double d3 = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                    A[2] * (A[3] * A[7] - A[4] * A[6]);
  if (!(d1 > 0.0 && d2 > 0.0 && d3 > 0.0))
    return lsh_fail(LSH_ENOTELLIPTIC, std::string(what) + " is not positive definite");
  return LSH_OK;
}

// d = 2 (plane strain): a 3x3 Voigt matrix becomes the 6x6 one whose in-plane
// block (Voigt rows and columns 11, 22, 12) it is and whose other entries are
// those of a template T shared by C0 and every phase, so that C - C0 vanishes
// outside the in-plane block and the 33 and anti-plane strains stay zero.  For
// an isotropic C0 the template is the three-dimensional isotropic tensor with
// C0's Lame constants (the solver then uses its isotropic Green operator);
// otherwise it has no couplings and diagonal (C11 + C22)/2, C66, C66.
static void plane_template(const double* C02, double* T) {
  for (int i = 0; i < 36; ++i) T[i] = 0.0;
  double mx = 0.0;
  for (int i = 0; i < 9; ++i) mx = std::max(mx, fabs(C02[i]));
  const double c11 = C02[0], c12 = C02[1], c16 = C02[2], c22 = C02[4], c26 = C02[5], c66 = C02[8];
  const double tol = 1e-13 * mx;
  const bool iso = fabs(c11 - c22) <= tol && fabs(c16) <= tol && fabs(c26) <= tol &&
                   fabs(c66 - 0.5 * (c11 - c12)) <= tol;
  if (iso) {
    const double lam = c12, mu = c66;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) T[6 * i + j] = lam + (i == j ? 2.0 * mu : 0.0);
    T[21] = T[28] = T[35] = mu;
  } else {
    T[14] = 0.5 * (c11 + c22);
    T[21] = T[28] = c66;
  }
}

static void embed_plane(const double* C2, const double* T, double* C6) {
  static const int map[3] = {0, 1, 5};
  for (int i = 0; i < 36; ++i) C6[i] = T[i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C6[6 * map[i] + map[j]] = C2[3 * i + j];
}

extern "C" int lsh_set_stiffness(lsh_pattern* p, int nphase, const double* C_voigt, const double* C0_voigt,
                                 const uint8_t* phase) {
  if (!p || !C_voigt || !C0_voigt || !phase) return lsh_fail(LSH_EINVAL, "null argument");
  if (nphase < 1 || nphase > 256) return lsh_fail(LSH_EINVAL, "nphase must be in [1, 256]");
  if (p->d == 2) {
    for (int q = 0; q < nphase; ++q) {
      int st = check_stiffness_plane(C_voigt + 9 * q, "phase stiffness");
      if (st) return st;
    }
    int st = check_stiffness_plane(C0_voigt, "reference stiffness C0");
    if (st) return st;
    for (int64_t i = 0; i < p->m; ++i)
      if (phase[i] >= nphase) return lsh_fail(LSH_EINVAL, "phase index out of range");
    double T[36];
    plane_template(C0_voigt, T);
    p->nphase = nphase;
    p->C_voigt.assign(36 * (size_t)nphase, 0.0);
    for (int q = 0; q < nphase; ++q) embed_plane(C_voigt + 9 * q, T, p->C_voigt.data() + 36 * q);
    embed_plane(C0_voigt, T, p->C0_voigt);
    p->phase.assign(phase, phase + p->m);
    p->bound_prec = -1;
    return LSH_OK;
  }
  for (int q = 0; q < nphase; ++q) {
    int st = check_stiffness(C_voigt + 36 * q, "phase stiffness");
    if (st) return st;
  }
  int st = check_stiffness(C0_voigt, "reference stiffness C0");
  if (st) return st;
  for (int64_t i = 0; i < p->m; ++i)
    if (phase[i] >= nphase) return lsh_fail(LSH_EINVAL, "phase index out of range");
  p->nphase = nphase;
  p->C_voigt.assign(C_voigt, C_voigt + 36 * nphase);
  memcpy(p->C0_voigt, C0_voigt, sizeof(p->C0_voigt));
  p->phase.assign(phase, phase + p->m);
  p->bound_prec = -1;
  return LSH_OK;
}
