// lsh_green.hpp -- the Green operator and the periodised Green operator on the GPU.
//
// Def. (projection), eq. (gamma): Gamma0_k tau = sym(k (x) K(k)^{-1} tau k),
// K_im(k) = sum_jl C0_ijlm k_j k_l (the acoustic tensor), Gamma0_0 = 0.
// Def. (gamma_tilde_fourier) with orthonormalised translates:
//   Gamma^p_h = sum_z w(x+z) Gamma0_{h+M^T z} / sum_z w(x+z),  w = g^2, x = M^{-T} h,
// where g is the generating function's weight (Sec. 2.2).  The solver applies
// the Hermitian part (Gamma^p_h + Gamma^p_{-h})/2, which keeps real strain
// fields real; it differs from Gamma^p only where the representative of -h is
// not -h (the -1/2 faces of the cube) for the Dirichlet kernel and for the
// truncated Box-spline sum.
//
// All of this runs in double precision.  Matrices are 6x6 symmetric in Mandel
// form, stored as the 21-entry upper triangle row by row.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define LSH_MAX_XI 16

struct GreenParams {
  int kind;          // lsh_kernel
  int nxi;           // Box spline: number of directions
  int R;             // Box spline: alias box [-R, R]^3
  int flat3;         // two-dimensional pattern: the third axis carries no aliases
  int tail;          // Box spline: add the aliases beyond R along the slow axes
  int xi_int;        // Box spline: every direction has integer entries
  int iso;           // C0 isotropic: Gamma0 = S(n)/mu0 - riso Q(n) (see below)
  double mu0, riso;
  int nslow;         // slow axes: one direction with a unit entry there, all others zero
  int slow_axis[3];
  int slow_col[3];
  int64_t m;         // |det M|
  int64_t e[3];      // SNF diagonal
  int64_t VT[9];     // h = V^T b
  int64_t A[9];      // sign(det M) adj(M^T): m x = A h
  int64_t MT[9];     // M^T
  double alpha[3];   // dlVP
  double Xi[3 * LSH_MAX_XI];  // Box directions, column s at Xi[3 s + i]
  double C0[81];     // C0_ijkl
};

// upper-triangle index of (I, J), I <= J, 6x6
__host__ __device__ constexpr int tri_idx(int I, int J) { return I * 6 - (I * (I - 1)) / 2 + (J - I); }

// Representative of v mod m in [-m/2, m/2) (the half-open cube rule).  The
// quotient is estimated in double and corrected, which is exact for
// |v| < 2^52 and avoids 64-bit integer division.
__device__ __forceinline__ int64_t center_mod(int64_t v, int64_t m) {
  const int64_t h = m / 2;
  const int64_t u = v + h;
  int64_t q = (int64_t)floor((double)u / (double)m);
  int64_t r = u - q * m;
  if (r < 0) r += m;
  if (r >= m) r -= m;
  return r - h;
}

// Reduce h into G(M^T): returns h_rep and x_num (x = x_num / m in [-1/2,1/2)^3).
__device__ __forceinline__ void reduce_freq(const GreenParams& gp, const int64_t h[3], int64_t hr[3],
                                            int64_t xn[3]) {
  int64_t z[3];
  for (int i = 0; i < 3; ++i) {
    const int64_t v = gp.A[3 * i] * h[0] + gp.A[3 * i + 1] * h[1] + gp.A[3 * i + 2] * h[2];
    xn[i] = center_mod(v, gp.m);
    // (v - xn) is an exact multiple of m: the double quotient rounds to it
    z[i] = (int64_t)rint((double)(v - xn[i]) / (double)gp.m);
  }
  for (int i = 0; i < 3; ++i) hr[i] = h[i] - (gp.MT[3 * i] * z[0] + gp.MT[3 * i + 1] * z[1] + gp.MT[3 * i + 2] * z[2]);
}

// Mandel index pairs (11,22,33,23,13,12)
__device__ __forceinline__ void mandel_pair(int I, int& a, int& b) {
  const int A_[6] = {0, 1, 2, 1, 0, 0};
  const int B_[6] = {0, 1, 2, 2, 2, 1};
  a = A_[I];
  b = B_[I];
}

// acc += w * Gamma0_k (21 entries).  k need not be normalised.
__device__ inline void add_gamma0(const GreenParams& gp, const double k[3], double w, double acc[21]) {
  double K[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int mm = 0; mm < 3; ++mm) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int l = 0; l < 3; ++l) s += gp.C0[((i * 3 + j) * 3 + l) * 3 + mm] * k[j] * k[l];
      K[i][mm] = s;
    }
  // N = K^{-1} (K symmetric positive definite for k != 0 and elliptic C0)
  const double c00 = K[1][1] * K[2][2] - K[1][2] * K[2][1];
  const double c01 = K[1][2] * K[2][0] - K[1][0] * K[2][2];
  const double c02 = K[1][0] * K[2][1] - K[1][1] * K[2][0];
  const double det = K[0][0] * c00 + K[0][1] * c01 + K[0][2] * c02;
  const double id = 1.0 / det;
  double N[3][3];
  N[0][0] = c00 * id;
  N[1][0] = c01 * id;
  N[2][0] = c02 * id;
  N[0][1] = (K[0][2] * K[2][1] - K[0][1] * K[2][2]) * id;
  N[1][1] = (K[0][0] * K[2][2] - K[0][2] * K[2][0]) * id;
  N[2][1] = (K[0][1] * K[2][0] - K[0][0] * K[2][1]) * id;
  N[0][2] = (K[0][1] * K[1][2] - K[0][2] * K[1][1]) * id;
  N[1][2] = (K[0][2] * K[1][0] - K[0][0] * K[1][2]) * id;
  N[2][2] = (K[0][0] * K[1][1] - K[0][1] * K[1][0]) * id;
  const double SQ2 = 1.41421356237309504880168872420969808;
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    int a, b;
    mandel_pair(I, a, b);
    const double cI = I < 3 ? 1.0 : SQ2;
#pragma unroll
    for (int J = I; J < 6; ++J) {
      const int t = tri_idx(I, J);
      int c, d;
      mandel_pair(J, c, d);
      const double cJ = J < 3 ? 1.0 : SQ2;
      const double G = 0.25 * (k[a] * N[b][c] * k[d] + k[b] * N[a][c] * k[d] + k[a] * N[b][d] * k[c] +
                               k[b] * N[a][d] * k[c]);
      acc[t] += w * cI * cJ * G;
    }
  }
}

__device__ __forceinline__ double trap_weight(double t, double a) {
  t = fabs(t);
  if (a <= 0.0) return t < 0.5 ? 1.0 : (t == 0.5 ? 0.5 : 0.0);
  double v = ((1.0 + a) * 0.5 - t) / a;
  return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
}

// g(x)^2 for the analytic kernels and the Box spline
__device__ inline double kernel_weight(const GreenParams& gp, const double x[3]) {
  if (gp.kind == 0) {  // Dirichlet
    return (x[0] >= -0.5 && x[0] < 0.5 && x[1] >= -0.5 && x[1] < 0.5 && x[2] >= -0.5 && x[2] < 0.5) ? 1.0 : 0.0;
  }
  if (gp.kind == 1 || gp.kind == 2) {
    double g = 1.0;
    for (int i = 0; i < 3; ++i) g *= trap_weight(x[i], gp.kind == 1 ? 0.0 : gp.alpha[i]);
    return g * g;
  }
  // Box spline: prod sinc(pi xi^T x), sinc t = sin t / t
  double g = 1.0;
  for (int s = 0; s < gp.nxi; ++s) {
    const double u = gp.Xi[3 * s] * x[0] + gp.Xi[3 * s + 1] * x[1] + gp.Xi[3 * s + 2] * x[2];
    if (u != 0.0) g *= sinpi(u) / (3.14159265358979323846264338327950288 * u);
  }
  return g * g;
}

// ------------------------------------------------------ isotropic C0 path ---
// For an isotropic reference stiffness (Lame lam0, mu0) the Green operator of
// eq. (gamma) is Gamma0_k = S(n)/mu0 - r Q(n), n = k/|k|, r = (lam0+mu0)/(mu0(lam0+2mu0)),
// with S(n): tau -> sym(n (x) tau n) and Q(n): tau -> (n.tau n) n (x) n.  Both
// are linear in the moments n n^T and n n n n, so the weighted alias sum of
// Def. (gamma_tilde_fourier) only needs the 6 second and 15 fourth moments of
// the alias directions; the 6x6 matrix follows from them.
struct IsoMoments {
  double a[6];   // sum w n_i n_j, Mandel pair order (00,11,22,12,02,01)
  double q[15];  // sum w n_i n_j n_k n_l, i<=j<=k<=l in lexicographic order
  double w;      // sum w
};

__device__ __forceinline__ int q4_index(int i, int j, int k, int l) {
  // sort (i,j,k,l) ascending, then rank among the 15 multisets of {0,1,2}
  int s[4] = {i, j, k, l};
  for (int x = 0; x < 3; ++x)
    for (int y = 0; y < 3 - x; ++y)
      if (s[y] > s[y + 1]) {
        const int t = s[y];
        s[y] = s[y + 1];
        s[y + 1] = t;
      }
  // counts of 0s, 1s (the rest are 2s) determine the multiset
  int c0 = 0, c1 = 0;
  for (int x = 0; x < 4; ++x) {
    c0 += s[x] == 0;
    c1 += s[x] == 1;
  }
  // enumerate multisets in lexicographic order: c0 from 4 down to 0, then c1 down
  int idx = 0;
  for (int a = 4; a > c0; --a) idx += 4 - a + 1;
  return idx + (4 - c0 - c1);
}

__device__ __forceinline__ void iso_add(IsoMoments& M, const double k[3], double w) {
  const double inv = rsqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  const double n0 = k[0] * inv, n1 = k[1] * inv, n2 = k[2] * inv;
  const double p00 = n0 * n0, p11 = n1 * n1, p22 = n2 * n2, p12 = n1 * n2, p02 = n0 * n2, p01 = n0 * n1;
  M.a[0] += w * p00;
  M.a[1] += w * p11;
  M.a[2] += w * p22;
  M.a[3] += w * p12;
  M.a[4] += w * p02;
  M.a[5] += w * p01;
  // 4th moments in the q4_index order: c0 = 4,3,2,1,0 blocks
  M.q[0] += w * p00 * p00;   // 0000
  M.q[1] += w * p00 * p01;   // 0001
  M.q[2] += w * p00 * p02;   // 0002
  M.q[3] += w * p00 * p11;   // 0011
  M.q[4] += w * p00 * p12;   // 0012
  M.q[5] += w * p00 * p22;   // 0022
  M.q[6] += w * p01 * p11;   // 0111
  M.q[7] += w * p01 * p12;   // 0112
  M.q[8] += w * p01 * p22;   // 0122
  M.q[9] += w * p02 * p22;   // 0222
  M.q[10] += w * p11 * p11;  // 1111
  M.q[11] += w * p11 * p12;  // 1112
  M.q[12] += w * p11 * p22;  // 1122
  M.q[13] += w * p12 * p22;  // 1222
  M.q[14] += w * p22 * p22;  // 2222
  M.w += w;
}

// 21-entry Mandel matrix from normalised moments
__device__ inline void iso_matrix(const IsoMoments& M, double mu0, double r, double G[21]) {
  const double SQ2 = 1.41421356237309504880168872420969808;
  const double iw = 1.0 / M.w;
  double A[3][3];
  A[0][0] = M.a[0] * iw;
  A[1][1] = M.a[1] * iw;
  A[2][2] = M.a[2] * iw;
  A[1][2] = A[2][1] = M.a[3] * iw;
  A[0][2] = A[2][0] = M.a[4] * iw;
  A[0][1] = A[1][0] = M.a[5] * iw;
  const double imu = 1.0 / mu0;
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    int a, b;
    mandel_pair(I, a, b);
    const double cI = I < 3 ? 1.0 : SQ2;
#pragma unroll
    for (int J = I; J < 6; ++J) {
      const int t = tri_idx(I, J);
      int c, d;
      mandel_pair(J, c, d);
      const double cJ = J < 3 ? 1.0 : SQ2;
      const double S = 0.25 * ((b == c) * A[a][d] + (b == d) * A[a][c] + (a == c) * A[b][d] + (a == d) * A[b][c]);
      const double Q = M.q[q4_index(a, b, c, d)] * iw;
      G[t] = cI * cJ * (imu * S - r * Q);
    }
  }
}

// Isotropic version of gamma_sym_at for the analytic kernels (Dirichlet,
// modified Dirichlet, dlVP): same alias sets and symmetrisation.  Gamma0 for
// an isotropic C0 is S(n)/mu0 - r Q(n), linear in the second and fourth
// moments of the direction n, so Gamma^p needs only the weighted moments of
// the alias directions (6 + 15 numbers, independent of C0).
//
// iso_moments: the normalised moments at bin b; false (moments zero) at h = 0.
// Each representative's weights are normalised up front (its weight sum
// factors over the axes), so one accumulator suffices.
__device__ inline bool iso_moments(const GreenParams& gp, int64_t b0, int64_t b1, int64_t b2, IsoMoments& M) {
  M = IsoMoments{};
  const int64_t b[3] = {b0, b1, b2};
  int64_t h[3];
  for (int i = 0; i < 3; ++i) h[i] = gp.VT[3 * i] * b[0] + gp.VT[3 * i + 1] * b[1] + gp.VT[3 * i + 2] * b[2];
  int64_t hr[3], xn[3];
  reduce_freq(gp, h, hr, xn);
  if (hr[0] == 0 && hr[1] == 0 && hr[2] == 0) return false;
  const double invm = 1.0 / (double)gp.m;
  const bool face = (2 * xn[0] == -gp.m) || (2 * xn[1] == -gp.m) || (2 * xn[2] == -gp.m);
  const int nrep = (face && gp.kind == 0) ? 2 : 1;
  for (int rep = 0; rep < nrep; ++rep) {
    int64_t hh[3] = {hr[0], hr[1], hr[2]}, xx[3] = {xn[0], xn[1], xn[2]};
    if (rep == 1) {
      const int64_t hm[3] = {-hr[0], -hr[1], -hr[2]};
      reduce_freq(gp, hm, hh, xx);
    }
    // per axis: the offsets z_i in {0, +-1} whose weight is non-zero (the
    // trapezoid of half-width (1+alpha)/2 reaches at most one neighbour)
    int nz[3], zs[3];
    double w0[3], w1[3];
    double W = 1.0;  // sum over aliases of prod_i g_i^2 = prod_i sum_z g_i(z)^2
    for (int i = 0; i < 3; ++i) {
      nz[i] = 1;
      zs[i] = 0;
      w1[i] = 0.0;
      if (gp.kind == 0) {
        w0[i] = 1.0;
        continue;
      }
      const double x0 = (double)xx[i] * invm;
      const double a = gp.kind == 1 ? 0.0 : gp.alpha[i];
      w0[i] = trap_weight(x0, a);
      const int sgn = x0 < 0.0 ? 1 : -1;
      const double g1 = trap_weight(x0 + sgn, a);
      if (g1 > 0.0) {
        zs[i] = sgn;
        w1[i] = g1;
        nz[i] = 2;
      }
      W *= w0[i] * w0[i] + w1[i] * w1[i];
    }
    const double f = 1.0 / (W * nrep);
    // one alias at a time (kept rolled: unrolled, the aliases' moments would
    // all be live at once)
    const int nal = nz[0] * nz[1] * nz[2];
#pragma unroll 1
    for (int c = 0; c < nal; ++c) {
      const int i0 = c / (nz[1] * nz[2]), i1 = (c / nz[2]) % nz[1], i2 = c % nz[2];
      const double g = (i0 ? w1[0] : w0[0]) * (i1 ? w1[1] : w0[1]) * (i2 ? w1[2] : w0[2]);
      const double w = g * g * f;
      if (w <= 0.0) continue;
      // k = h + M^T z in double: every term is an integer below 2^53, exact
      const double z0 = i0 ? (double)zs[0] : 0.0, z1 = i1 ? (double)zs[1] : 0.0, z2 = i2 ? (double)zs[2] : 0.0;
      double kd[3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
        kd[i] = (double)hh[i] + (double)gp.MT[3 * i] * z0 + (double)gp.MT[3 * i + 1] * z1 +
                (double)gp.MT[3 * i + 2] * z2;
      if (kd[0] == 0.0 && kd[1] == 0.0 && kd[2] == 0.0) continue;
      iso_add(M, kd, w);
    }
  }
  return true;
}

// The 21 Mandel entries of S/mu0 - r Q from normalised moments a (6: the
// pairs 00,11,22,12,02,01) and q (15, q4_index order); out(t, v).
template <typename Out>
__device__ inline void iso_emit(const double a[6], const double q[15], double mu0, double r, Out&& out) {
  const double SQ2 = 1.41421356237309504880168872420969808;
  const double imu = 1.0 / mu0;
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    int ia, ib;
    mandel_pair(I, ia, ib);
    const double cI = I < 3 ? 1.0 : SQ2;
#pragma unroll
    for (int J = I; J < 6; ++J) {
      int ic, id;
      mandel_pair(J, ic, id);
      const double cJ = J < 3 ? 1.0 : SQ2;
      auto Am = [&](int u, int v) {
        const int lo = u < v ? u : v, hi = u < v ? v : u;
        return lo == hi ? a[lo] : a[6 - lo - hi];
      };
      const double S = 0.25 * ((ib == ic) * Am(ia, id) + (ib == id) * Am(ia, ic) + (ia == ic) * Am(ib, id) +
                               (ia == id) * Am(ib, ic));
      out(tri_idx(I, J), cI * cJ * (imu * S - r * q[q4_index(ia, ib, ic, id)]));
    }
  }
}

template <typename Out>
__device__ inline void gamma_iso_emit(const GreenParams& gp, double mu0, double r, int64_t b0, int64_t b1, int64_t b2,
                                      Out&& out) {
  IsoMoments M;
  if (!iso_moments(gp, b0, b1, b2, M)) {
    for (int t = 0; t < 21; ++t) out(t, 0.0);
    return;
  }
  iso_emit(M.a, M.q, mu0, r, out);
}

__device__ inline void gamma_sym_iso(const GreenParams& gp, double mu0, double r, int64_t b0, int64_t b1, int64_t b2,
                                     double G[21]) {
  gamma_iso_emit(gp, mu0, r, b0, b1, b2, [&](int t, double v) { G[t] = v; });
}

// Box spline, the aliases beyond [-R, R] along a slow axis i: only the
// direction xi* varies along the line z_perp + t e_i, and the weight the line
// keeps outside |t| <= R is w_perp (1 - sum_{|n| <= R} sinc^2(pi (c + n))),
// c = xi*^T (x + z_perp), by the identity sum_n sinc^2(pi (c + n)) = 1.  There
// k = h + M^T z turns towards M^T e_i, so those aliases carry Gamma0 of M^T e_i
// (the term odd in 1/t cancels between the half-lines; what remains is
// O(R^-3) against O(R^-1) for plain truncation).
template <typename Add>
__device__ inline void box_tail(const GreenParams& gp, const double x0[3], int r, Add&& add, double* den) {
  const double PI = 3.14159265358979323846264338327950288;
  for (int a = 0; a < gp.nslow; ++a) {
    const int i = gp.slow_axis[a], sc = gp.slow_col[a];
    const int j0 = i == 0 ? 1 : 0, j1 = i == 2 ? 1 : 2;
    const int r0 = (gp.flat3 && j0 == 2) ? 0 : r, r1 = (gp.flat3 && j1 == 2) ? 0 : r;
    double tw = 0.0;
    for (int u = -r0; u <= r0; ++u)
      for (int v = -r1; v <= r1; ++v) {
        double y[3] = {x0[0], x0[1], x0[2]};
        y[j0] += u;
        y[j1] += v;
        double wp = 1.0;
        for (int s = 0; s < gp.nxi; ++s) {
          if (s == sc) continue;
          const double t = gp.Xi[3 * s] * y[0] + gp.Xi[3 * s + 1] * y[1] + gp.Xi[3 * s + 2] * y[2];
          if (t != 0.0) {
            const double g = sinpi(t) / (PI * t);
            wp *= g * g;
          }
        }
        if (wp <= 0.0) continue;
        const double c = gp.Xi[3 * sc] * y[0] + gp.Xi[3 * sc + 1] * y[1] + gp.Xi[3 * sc + 2] * y[2];
        const double sp = sinpi(c);
        double line;
        if (sp == 0.0) {  // c an integer: one term of the line carries the whole weight
          line = fabs(rint(c)) <= (double)r ? 1.0 : 0.0;
        } else {
          double q2 = 0.0;
          for (int m = -r; m <= r; ++m) {
            const double q = c + m;
            q2 += 1.0 / (q * q);
          }
          line = sp * sp * q2 / (PI * PI);
        }
        tw += wp * (1.0 - line);
      }
    if (tw != 0.0) {
      const double kd[3] = {(double)gp.MT[i], (double)gp.MT[3 + i], (double)gp.MT[6 + i]};
      add(kd, tw);
      *den += tw;
    }
  }
}

// Weighted alias sum for the representative h_rep (x_num its M^{-T} numerator):
// acc = sum_z w Gamma0, returns sum_z w.  With an isotropic C0 the sum runs
// over the alias directions' moments, and Gamma0's closed form is applied once
// at the end (Gamma0 is linear in them).  z over {-1,0,1}^3 (modified
// Dirichlet, dlVP), {0} (Dirichlet) or [-R,R]^3 (Box); z3 = 0 only for a
// two-dimensional pattern (its third weight factor vanishes at every z3 != 0).
// ISO: 1 moment form, 0 general form, -1 chosen by gp.iso at run time.
template <int ISO = -1>
__device__ inline double alias_sum(const GreenParams& gp, const int64_t hr[3], const int64_t xn[3], double acc[21]) {
  const bool iso = ISO >= 0 ? ISO == 1 : gp.iso != 0;
  for (int t = 0; t < 21; ++t) acc[t] = 0.0;
  const double invm = 1.0 / (double)gp.m;
  const double x0[3] = {(double)xn[0] * invm, (double)xn[1] * invm, (double)xn[2] * invm};
  int r = 0;
  if (gp.kind == 1 || gp.kind == 2) r = 1;
  if (gp.kind == 3) r = gp.R;
  const int r2 = gp.flat3 ? 0 : r;
  // Box spline with integer directions: xi^T z is an integer, so every alias
  // has the same sin^2(pi xi^T x) and only the denominators (pi xi^T x)^2 vary.
  // sq = prod_s sin^2(pi xi_s^T x0); 0 when some xi_s^T x0 is an integer,
  // where the direct form below decides which aliases keep weight.
  double sq = 0.0;
  if (gp.kind == 3 && gp.xi_int) {
    sq = 1.0;
    for (int s = 0; s < gp.nxi; ++s) {
      const double sp = sinpi(gp.Xi[3 * s] * x0[0] + gp.Xi[3 * s + 1] * x0[1] + gp.Xi[3 * s + 2] * x0[2]);
      sq *= sp * sp;
    }
  }
  double den = 0.0;
  IsoMoments M;
  if (iso) {
    for (int t = 0; t < 6; ++t) M.a[t] = 0.0;
    for (int t = 0; t < 15; ++t) M.q[t] = 0.0;
    M.w = 0.0;
  }
  auto add = [&](const double kd[3], double w) {
    if (iso)
      iso_add(M, kd, w);
    else
      add_gamma0(gp, kd, w, acc);
  };
  for (int z0 = -r; z0 <= r; ++z0)
    for (int z1 = -r; z1 <= r; ++z1)
      for (int z2 = -r2; z2 <= r2; ++z2) {
        const double x[3] = {x0[0] + z0, x0[1] + z1, x0[2] + z2};
        double w;
        if (sq > 0.0) {
          double pr = 1.0;
          for (int s = 0; s < gp.nxi; ++s) {
            const double u = 3.14159265358979323846264338327950288 *
                             (gp.Xi[3 * s] * x[0] + gp.Xi[3 * s + 1] * x[1] + gp.Xi[3 * s + 2] * x[2]);
            pr *= u * u;
          }
          w = sq / pr;
        } else {
          w = kernel_weight(gp, x);
        }
        if (w <= 0.0) continue;
        const int64_t kk[3] = {hr[0] + gp.MT[0] * z0 + gp.MT[1] * z1 + gp.MT[2] * z2,
                               hr[1] + gp.MT[3] * z0 + gp.MT[4] * z1 + gp.MT[5] * z2,
                               hr[2] + gp.MT[6] * z0 + gp.MT[7] * z1 + gp.MT[8] * z2};
        den += w;
        if (kk[0] == 0 && kk[1] == 0 && kk[2] == 0) continue;  // Gamma0_0 = 0
        const double kd[3] = {(double)kk[0], (double)kk[1], (double)kk[2]};
        add(kd, w);
      }
  if (gp.kind == 3 && gp.tail) box_tail(gp, x0, r, add, &den);
  if (iso) iso_emit(M.a, M.q, gp.mu0, gp.riso, [&](int t, double v) { acc[t] = v; });
  return den;
}

// Hermitian-symmetrised Gamma^p at SNF bin b (b1 may be any index mod e1).
// Returns the bracket sum of the weights at b (0 => translates degenerate).
template <int ISO = -1>
__device__ inline double gamma_sym_at(const GreenParams& gp, int64_t b0, int64_t b1, int64_t b2, double G[21]) {
  const int64_t b[3] = {b0, b1, b2};
  int64_t h[3];
  for (int i = 0; i < 3; ++i) h[i] = gp.VT[3 * i] * b[0] + gp.VT[3 * i + 1] * b[1] + gp.VT[3 * i + 2] * b[2];
  int64_t hr[3], xn[3];
  reduce_freq(gp, h, hr, xn);
  if (hr[0] == 0 && hr[1] == 0 && hr[2] == 0) {
    for (int t = 0; t < 21; ++t) G[t] = 0.0;
    return 1.0;
  }
  const bool face = (2 * xn[0] == -gp.m) || (2 * xn[1] == -gp.m) || (2 * xn[2] == -gp.m);
  const double den = alias_sum<ISO>(gp, hr, xn, G);
  for (int t = 0; t < 21; ++t) G[t] /= den;
  // the even kernels on the faces of the modified Dirichlet / dlVP family are
  // already symmetric (their alias set is mirrored); Dirichlet and the
  // truncated Box sum are not.
  if (face && (gp.kind == 0 || gp.kind == 3)) {
    const int64_t hm[3] = {-hr[0], -hr[1], -hr[2]};
    int64_t hr2[3], xn2[3];
    reduce_freq(gp, hm, hr2, xn2);
    double G2[21];
    const double den2 = alias_sum<ISO>(gp, hr2, xn2, G2);
    for (int t = 0; t < 21; ++t) G[t] = 0.5 * (G[t] + G2[t] / den2);
    return den < den2 ? den : den2;
  }
  return den;
}
