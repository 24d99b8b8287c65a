// lsh_twopass.hip -- the Basic Scheme iteration in two passes for gfx950.
//
// Thm. (pde_discretization), eq. (pde_coefficients), iterated as in Sec. 4 on
// the SNF grid (the pattern DFT of eq. (Fouriermatrix) as a 3-D DFT); the
// schedule and the state layout are described in lsh_twopass.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lsh_twopass.hpp"

namespace {

// ------------------------------------------------------------- stress pass ---
// One block: load L, coset r of axis 2 (i2 = r + P j, j < Q) and W consecutive
// i3.  LDS: axis-1 twiddles [N1], w_Q^k [Q], w_n2^{r q} [Q], the tile
// Z[k < N1][(pair, j, w)] (component pairs (0,1), (2,3), (4,5) share one complex
// axis-1 line), then (C_p - C0) of the first NDL phases.
//
// Tile order: the chip hands blocks to its eight XCDs in turn, so block b of
// a load runs on XCD b mod 8 (the grid's width is a multiple of 8 for every
// variant built).  Each XCD's share of the tiles is one range of the (r, i3)
// tiles with i3 fastest: the blocks one XCD runs side by side read and write
// neighbouring W-element runs of one coset, which share 128-byte lines in that
// XCD's L2 (a run is 32 or 64 bytes), as do the phase bytes they read.
template <typename T, int N1, int Q, int W, int NT, int NDL = 16>
__global__ void __launch_bounds__(NT) k_stress2(Geo g, const C2<T>* __restrict__ tw0, const C2<T>* __restrict__ tw1,
                                                const C2<T>* __restrict__ X, C2<T>* __restrict__ Y,
                                                const Inst* __restrict__ insts, const int* __restrict__ inst_of,
                                                const double* __restrict__ eps0, const int* __restrict__ stop_iter,
                                                const int* __restrict__ itp) {
  using T2 = C2<T>;
  constexpr int H = N1 / 2 + 1;
  constexpr int NC3 = 3 * Q * W;  // LDS columns (pair, j, w)
  constexpr int NU = H * 3 * W;   // load and store items (k, pair, w), all Q at once
  constexpr int UT = (NU + NT - 1) / NT;
  constexpr int NP = N1 * Q * W;  // points of the tile
  constexpr int PT = (NP + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* twl = reinterpret_cast<T2*>(smem_raw);
  T2* twq = twl + N1;
  T2* twr = twq + Q;
  T2* Z = twr + Q;
  T* Dl = reinterpret_cast<T*>(Z + N1 * NC3);
  const int L = blockIdx.y;
  if (*itp >= stop_iter[L]) return;
  const int P = g.n2 / Q;
  const int nw = g.n3 / W;
  int r, a30;
  {
    const int nb = gridDim.x, b = blockIdx.x;
    const int x = b & 7, base = nb >> 3, extra = nb & 7;
    const int t = x * base + (x < extra ? x : extra) + (b >> 3);
    r = t / nw;
    a30 = (t - r * nw) * W;
  }
  const Inst& in = insts[inst_of[L]];
  const uint8_t* __restrict__ phase = in.phase;
  const T* __restrict__ dmat = reinterpret_cast<const T*>(in.dmat);
  const int nphase = in.nphase;
  const long long n23 = (long long)g.n2 * g.n3;
  const long long PN3 = (long long)P * g.n3;
  const int tid = threadIdx.x;

  // the state at every q for item (k, pair, w), both components of the pair
  T2 xa[UT][Q], xb[UT][Q];
#pragma unroll
  for (int i = 0; i < UT; ++i) {
    const int u = tid + i * NT;
    const int w = u % W, p = (u / W) % 3, k = u / (3 * W);
    const bool ok = NU % NT == 0 || u < NU;
    const long long off = ((long long)k * Q * P + r) * g.n3 + a30 + w;
    const T2* pa = X + (long long)(L * 6 + 2 * p) * g.spec + off;
    const T2* pb = pa + g.spec;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      xa[i][q] = ok ? pa[q * PN3] : T2{0, 0};
      xb[i][q] = ok ? pb[q * PN3] : T2{0, 0};
    }
  }
  // phase indices of the tile's points (a1, j, w), used after the C2R
  int ph[PT];
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int idx = tid + i * NT;
    const int w = idx % W, j = (idx / W) % Q, a1 = idx / (Q * W);
    ph[i] = (NP % NT == 0 || idx < NP) ? phase[(long long)a1 * n23 + (long long)(r + P * j) * g.n3 + a30 + w] : 0;
  }
  stage_twiddles<T>(twl, tw0, N1);
  for (int i = tid; i < Q; i += NT) {
    twq[i] = tw1[i * P];
    twr[i] = tw1[i * r];
  }
  {
    const int nd = nphase < NDL ? nphase : NDL;
    for (int i = tid; i < 36 * nd; i += NT) Dl[i] = dmat[i];
  }
  __syncthreads();

  // conjugate twiddle, Q-point inverse DFT over q (to j), Hermitian extension
  // of the pair lines: Z_p[k] = X_{2p}[k] + i X_{2p+1}[k] on the full axis
#pragma unroll
  for (int i = 0; i < UT; ++i) {
    const int u = tid + i * NT;
    if (NU % NT == 0 || u < NU) {
      const int w = u % W, p = (u / W) % 3, k = u / (3 * W);
#pragma unroll
      for (int q = 1; q < Q; ++q) {
        T2 t = twr[q];
        t.y = -t.y;
        xa[i][q] = cmul(xa[i][q], t);
        xb[i][q] = cmul(xb[i][q], t);
      }
      reg_fft<T, +1, Q>(xa[i], twq);
      reg_fft<T, +1, Q>(xb[i], twq);
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const int col = (p * Q + j) * W + w;
        const T2 a = xa[i][j], b = xb[i][j];
        if (k == 0 || 2 * k == N1) {
          Z[k * NC3 + col] = T2{a.x, b.x};
        } else {
          Z[k * NC3 + col] = T2{a.x - b.y, a.y + b.x};
          Z[(N1 - k) * NC3 + col] = T2{a.x + b.y, b.x - a.y};
        }
      }
    }
  }
  __syncthreads();
  fft_static<T, +1, N1, NC3, true, NT>(Z, 1, NC3, twl);

  // tau = (C_p - C0):(E + eps0) at the tile's points
  {
    const double* e0 = eps0 + 6 * L;
    const T ep[6] = {(T)e0[0], (T)e0[1], (T)e0[2], (T)e0[3], (T)e0[4], (T)e0[5]};
    auto stress = [&](int idx, const T* D) {
      const int w = idx % W, j = (idx / W) % Q, a1 = idx / (Q * W);
      T2* z = Z + a1 * NC3 + j * W + w;
      const T2 z0 = z[0], z1 = z[Q * W], z2 = z[2 * Q * W];
      const T E[6] = {z0.x + ep[0], z0.y + ep[1], z1.x + ep[2], z1.y + ep[3], z2.x + ep[4], z2.y + ep[5]};
      T t[6];
      stress6<T>(D, E, t);
      z[0] = T2{t[0], t[1]};
      z[Q * W] = T2{t[2], t[3]};
      z[2 * Q * W] = T2{t[4], t[5]};
    };
    // separate loops so that the LDS reads stay LDS instructions
    if (nphase <= NDL) {
#pragma unroll
      for (int i = 0; i < PT; ++i) {
        const int idx = tid + i * NT;
        if (NP % NT == 0 || idx < NP) stress(idx, Dl + 36 * ph[i]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < PT; ++i) {
        const int idx = tid + i * NT;
        if (NP % NT == 0 || idx < NP) stress(idx, dmat + 36 * ph[i]);
      }
    }
  }
  __syncthreads();
  fft_static<T, -1, N1, NC3, true, NT>(Z, 1, NC3, twl);

  // unpack the pairs (half spectrum k < H), Q-point DFT over j (to q), twiddle
#pragma unroll
  for (int i = 0; i < UT; ++i) {
    const int u = tid + i * NT;
    if (NU % NT == 0 || u < NU) {
      const int w = u % W, p = (u / W) % 3, k = u / (3 * W);
      T2 ya[Q], yb[Q];
      const T hf = (T)0.5;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const int col = (p * Q + j) * W + w;
        const T2 zk = Z[k * NC3 + col];
        const T2 zn = Z[((N1 - k) % N1) * NC3 + col];
        ya[j] = T2{hf * (zk.x + zn.x), hf * (zk.y - zn.y)};
        yb[j] = T2{hf * (zk.y + zn.y), hf * (zn.x - zk.x)};
      }
      reg_fft<T, -1, Q>(ya, twq);
      reg_fft<T, -1, Q>(yb, twq);
      const long long off = ((long long)k * Q * P + r) * g.n3 + a30 + w;
      T2* qa = Y + (long long)(L * 6 + 2 * p) * g.spec + off;
      T2* qb = qa + g.spec;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const T2 t = twr[q];
        qa[q * PN3] = q ? cmul(ya[q], t) : ya[q];
        qb[q * PN3] = q ? cmul(yb[q], t) : yb[q];
      }
    }
  }
}

// -Gamma^p_h/m applied to the Mandel 6-vector v at the integer frequency h of
// the pattern diag(n, n, n) with the Dirichlet kernel and an isotropic C0
// (Lame lambda0, mu0):  Gamma0_k tau = sym(u (x) tau u)/mu0 - r (u . tau u)
// u (x) u, u = k/|k|, r = (lambda0 + mu0)/(mu0 (lambda0 + 2 mu0)), so that no
// table is read and no operator is held; on the -n/2 faces the Hermitian part
// averages it with the direction whose face coordinates are negated (the
// representative of -h).  h = 0 gives 0.
template <typename T>
__device__ __forceinline__ void iso_dirichlet_apply(C2<T> v[6], int h0, int h1, int h2, int n, T imu, T r, T scale) {
  using T2 = C2<T>;
  const T RS2 = (T)0.70710678118654752440, SQ2 = (T)1.41421356237309504880;
  if (h0 == 0 && h1 == 0 && h2 == 0) {
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = T2{0, 0};
    return;
  }
  // tau from Mandel: diagonal, then (12, 02, 01) with the 1/sqrt2 of the shear entries
  const T2 t00 = v[0], t11 = v[1], t22 = v[2];
  const T2 t12 = T2{v[3].x * RS2, v[3].y * RS2}, t02 = T2{v[4].x * RS2, v[4].y * RS2},
           t01 = T2{v[5].x * RS2, v[5].y * RS2};
  const bool f0 = 2 * h0 == -n, f1 = 2 * h1 == -n, f2 = 2 * h2 == -n;
  const int nd = (f0 || f1 || f2) ? 2 : 1;
  T2 R[6] = {T2{0, 0}, T2{0, 0}, T2{0, 0}, T2{0, 0}, T2{0, 0}, T2{0, 0}};  // 00 11 22 12 02 01
  for (int d = 0; d < nd; ++d) {
    const T k0 = (T)((d && f0) ? -h0 : h0), k1 = (T)((d && f1) ? -h1 : h1), k2 = (T)((d && f2) ? -h2 : h2);
    const T inv = (T)1 / sqrt(k0 * k0 + k1 * k1 + k2 * k2);
    const T u0 = k0 * inv, u1 = k1 * inv, u2 = k2 * inv;
    T2 w[3];
    w[0] = T2{t00.x * u0 + t01.x * u1 + t02.x * u2, t00.y * u0 + t01.y * u1 + t02.y * u2};
    w[1] = T2{t01.x * u0 + t11.x * u1 + t12.x * u2, t01.y * u0 + t11.y * u1 + t12.y * u2};
    w[2] = T2{t02.x * u0 + t12.x * u1 + t22.x * u2, t02.y * u0 + t12.y * u1 + t22.y * u2};
    const T2 sd = T2{u0 * w[0].x + u1 * w[1].x + u2 * w[2].x, u0 * w[0].y + u1 * w[1].y + u2 * w[2].y};
    const T u[3] = {u0, u1, u2};
    const int pa[6] = {0, 1, 2, 1, 0, 0}, pb[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
    for (int I = 0; I < 6; ++I) {
      const int a = pa[I], b = pb[I];
      const T hs = (T)0.5 * imu, ruu = r * u[a] * u[b];
      R[I].x += hs * (u[a] * w[b].x + u[b] * w[a].x) - ruu * sd.x;
      R[I].y += hs * (u[a] * w[b].y + u[b] * w[a].y) - ruu * sd.y;
    }
  }
  const T f = nd == 2 ? (T)0.5 * scale : scale;
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    const T c = I < 3 ? f : f * SQ2;
    v[I] = T2{R[I].x * c, R[I].y * c};
  }
}

// -------------------------------------------------------------- Green pass ---
// One block: position (k1, q) and a chunk of up to six loads of one instance,
// one load at a time.  LDS: axis-3 twiddles [N3], w_P^k [P], lines
// [(s, comp)][LS] along axis 3.  The Green operator -Gamma^p/m of the tile's
// bins (k1, q + Q s, k3) is formed once per chunk into registers (each thread
// keeps the NB2 bins it multiplies) from the table or the alias moments (GM =
// GREEN_TABLE, GREEN_MOMENTS), or applied in closed form per bin for the
// Dirichlet kernel on diag(n, n, n) (GM = GREEN_ISO, iso_dirichlet_apply).
// Per load: the tile's P n3 values of
// each component come in with the P-point DFT over r done in registers (the
// next load's values are fetched while this one is transformed), the axis-3
// transforms run in LDS, and the values go out through the inverse
// transforms, the inverse P-point DFT again in registers, with the Cauchy
// residual's partial sums (double).
// PF: fetch the next load's values while the current one is transformed (else
// each load's values are fetched when its turn comes, which frees the
// registers that hold them through the rest of the loop).  INC: the build for
// the increment scheme (upd = UPD_INC); the other build serves UPD_LS and
// UPD_VE, whose output stage then carries no increment store.
template <typename T, int P, int N3, int NT, int GM, bool PF = true, bool INC = false>
__global__ void __launch_bounds__(NT) k_green3(Geo g, const C2<T>* __restrict__ tw1, const C2<T>* __restrict__ tw2,
                                               const C2<T>* __restrict__ tau, const C2<T>* __restrict__ Pold,
                                               C2<T>* __restrict__ Pnew, const T* __restrict__ table,
                                               const Inst* __restrict__ insts, const int* __restrict__ inst_of,
                                               const int* __restrict__ chunks, const int* __restrict__ stop_iter,
                                               const int* __restrict__ itp, int npos, double* __restrict__ partial,
                                               int upd, C2<T>* __restrict__ dP) {
  using T2 = C2<T>;
  static_assert(GM == GREEN_TABLE || GM == GREEN_MOMENTS || GM == GREEN_ISO,
                "tabled Green operators or the Dirichlet closed form");
  constexpr int LS = N3 + 1;  // odd line stride: the same entry of neighbouring lines in other banks
  constexpr int NLN = 6 * P;  // lines (s, comp)
  constexpr int NI = 6 * N3;  // items (comp, i3) of the P-point stages
  constexpr int IT = (NI + NT - 1) / NT;
  constexpr int NB = P * N3;  // bins of the tile
  constexpr int NB2 = (NB + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* tw3 = reinterpret_cast<T2*>(smem_raw);
  T2* twP = tw3 + N3;
  T2* lines = twP + P;
  const int Q = g.n2 / P;
  const int pos = blockIdx.x;
  const int k1 = pos / Q, q = pos % Q;
  const int Lbeg = chunks[2 * blockIdx.y], Lend = chunks[2 * blockIdx.y + 1];
  const int it = *itp;
  {
    bool any = false;
    for (int L = Lbeg; L < Lend; ++L) any = any || it < stop_iter[L];
    if (!any) return;
  }
  const int tid = threadIdx.x;
  const double wk1 = (k1 == 0 || 2 * k1 == g.n1) ? 1.0 : 2.0;
  const long long row = (long long)(k1 * Q + q) * P * N3;  // the tile's first element in a component

  // tau of item i of load L: P values at stride n3
  T2 pf[IT][P];
  auto fetch = [&](int L) {
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int u = tid + i * NT;
      const int c = u / N3, i3 = u % N3;
      const bool ok = NI % NT == 0 || u < NI;
      const T2* src = tau + (long long)(L * 6 + (ok ? c : 0)) * g.spec + row + (ok ? i3 : 0);
#pragma unroll
      for (int rr = 0; rr < P; ++rr) pf[i][rr] = ok ? src[rr * N3] : T2{0, 0};
    }
  };
  auto next_active = [&](int L) {
    while (L < Lend && it >= stop_iter[L]) ++L;
    return L;
  };
  int L = next_active(Lbeg);
  if (PF) fetch(L);  // in flight while the Green operator is formed

  stage_twiddles<T>(tw3, tw2, N3);
  for (int i = tid; i < P; i += NT) twP[i] = tw1[i * Q];
  // -Gamma^p_h / m at this thread's bins (k1, k2 = q + Q s, k3), b = tid + k NT
  T Gr[GM == GREEN_ISO ? 1 : NB2][21];  // the closed form (GREEN_ISO) holds no operator
  const double mu0 = insts[inst_of[Lbeg]].mu0, riso = insts[inst_of[Lbeg]].riso;
  if constexpr (GM != GREEN_ISO) {
    const double scale = -1.0 / (double)g.m;
#pragma unroll
    for (int k = 0; k < NB2; ++k) {
      const int b = tid + k * NT;
      const int s = (b < NB ? b : 0) / N3, k3 = (b < NB ? b : 0) % N3;
      const long long pos2 = (long long)k1 * g.n2 + q + Q * s;
      if constexpr (GM == GREEN_TABLE) {
        const T* tb = table + pos2 * 21 * N3 + k3;
#pragma unroll
        for (int t = 0; t < 21; ++t) Gr[k][t] = (T)(scale * (double)tb[(long long)t * N3]);
      } else {
        moments_emit(table, pos2, N3, k3, mu0, riso, [&](int t, double v) { Gr[k][t] = (T)(scale * v); });
      }
    }
  }
  __syncthreads();

  while (L < Lend) {
    if (!PF) fetch(L);
    // P-point DFT over r on the way in (item (c, i3), consecutive items
    // consecutive i3), then the next active load's values are fetched
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int u = tid + i * NT;
      if (NI % NT == 0 || u < NI) {
        const int c = u / N3, i3 = u % N3;
        T2 v[P];
#pragma unroll
        for (int rr = 0; rr < P; ++rr) v[rr] = pf[i][rr];
        reg_fft<T, -1, P>(v, twP);
#pragma unroll
        for (int s = 0; s < P; ++s) lines[(s * 6 + c) * LS + i3] = v[s];
      }
    }
    const int Lnext = next_active(L + 1);
    if (PF && Lnext < Lend) fetch(Lnext);
    __syncthreads();
    fft_static<T, -1, N3, NLN, false, NT>(lines, LS, 1, tw3);

#pragma unroll
    for (int k = 0; k < NB2; ++k) {
      const int b = tid + k * NT;
      if (NB % NT == 0 || b < NB) {
        const int s = b / N3, k3 = b - s * N3;
        T2 v[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = lines[(s * 6 + c) * LS + k3];
        if constexpr (GM == GREEN_ISO) {
          // signed frequency of each index: [-n/2, n/2)
          const int f[3] = {k1, q + Q * s, k3};
          int h[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) h[i] = 2 * f[i] >= N3 ? f[i] - N3 : f[i];
          iso_dirichlet_apply<T>(v, h[0], h[1], h[2], N3, (T)(1.0 / mu0), (T)riso, (T)(-1.0 / (double)g.m));
#pragma unroll
          for (int I = 0; I < 6; ++I) lines[(s * 6 + I) * LS + k3] = v[I];
        } else {
#pragma unroll
          for (int I = 0; I < 6; ++I) {
            T2 y = T2{0, 0};
#pragma unroll
            for (int J = 0; J < 6; ++J) {
              const T gij = Gr[k][I <= J ? tri_idx(I, J) : tri_idx(J, I)];
              y.x += gij * v[J].x;
              y.y += gij * v[J].y;
            }
            lines[(s * 6 + I) * LS + k3] = y;
          }
        }
      }
    }
    __syncthreads();
    fft_static<T, +1, N3, NLN, false, NT>(lines, LS, 1, tw3);

    // inverse P-point DFT over s on the way out; the residual against the
    // previous iterate in this (k1, q, r, i3) domain
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int u = tid + i * NT;
      if (NI % NT == 0 || u < NI) {
        const int c = u / N3, i3 = u % N3;
        const long long g0 = (long long)(L * 6 + c) * g.spec + row + i3;
        T2 v[P];
#pragma unroll
        for (int s = 0; s < P; ++s) v[s] = lines[(s * 6 + c) * LS + i3];
        reg_fft<T, +1, P>(v, twP);
#pragma unroll
        for (int rr = 0; rr < P; ++rr) {
          double d2;
          T2 nv;
          if constexpr (INC) {
            nv = green_update<T>(v[rr], Pold[g0 + rr * N3], UPD_INC, it, dP, g0 + rr * N3, &d2);
          } else {
            // variational scheme: the pass computes the correction, added to the old state
            const T2 po = Pold[g0 + rr * N3];
            nv = upd == UPD_VE ? cadd(v[rr], po) : v[rr];
            const double dx = (double)nv.x - (double)po.x, dy = (double)nv.y - (double)po.y;
            d2 = dx * dx + dy * dy;
          }
          Pnew[g0 + rr * N3] = nv;
          acc[0] += d2;
          acc[1] += (double)nv.x * (double)nv.x + (double)nv.y * (double)nv.y;
        }
      }
    }
    double tot[2];
    block_sum<2>(acc, tot);  // ends with a barrier: the lines are free for the next load
    if (tid == 0) {
      partial[((long long)L * npos + pos) * 2] = wk1 * tot[0];
      partial[((long long)L * npos + pos) * 2 + 1] = wk1 * tot[1];
    }
    L = Lnext;
  }
}

// ------------------------------------------------------ state conversions ---
// One thread per (load, comp, k1, r, i3); Q <= QMAX values each.
constexpr int QMAX = 16;
template <typename T>
__global__ void __launch_bounds__(256) k_to_split(Geo g, int Q, const C2<T>* __restrict__ tw1,
                                                  const C2<T>* __restrict__ X, C2<T>* __restrict__ Xs, int nload) {
  using T2 = C2<T>;
  const int P = g.n2 / Q;
  const long long per = (long long)g.h1 * P * g.n3;
  const long long n = per * 6 * nload;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long long)gridDim.x * 256) {
    const long long lc = t / per;
    const long long rem = t % per;
    const int i3 = (int)(rem % g.n3);
    const int r = (int)((rem / g.n3) % P);
    const int k1 = (int)(rem / ((long long)g.n3 * P));
    const T2* src = X + lc * g.spec + (long long)k1 * g.n2 * g.n3 + i3;
    T2* dst = Xs + lc * g.spec + (long long)k1 * Q * P * g.n3 + (long long)r * g.n3 + i3;
    T2 x[QMAX];
    for (int j = 0; j < Q; ++j) x[j] = src[(long long)(r + P * j) * g.n3];
    const T inv = (T)(1.0 / Q);
    for (int q = 0; q < Q; ++q) {
      T2 acc = T2{0, 0};
      for (int j = 0; j < Q; ++j) acc = cadd(acc, cmul(x[j], tw1[((j * q) % Q) * P]));
      acc = cmul(acc, tw1[r * q]);
      dst[(long long)q * P * g.n3] = T2{acc.x * inv, acc.y * inv};
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_from_split(Geo g, int Q, const C2<T>* __restrict__ tw1,
                                                    const C2<T>* __restrict__ Xs0, const C2<T>* __restrict__ Xs1,
                                                    C2<T>* __restrict__ X, const int* __restrict__ stop_iter,
                                                    const int* __restrict__ itp, int nload) {
  using T2 = C2<T>;
  const int P = g.n2 / Q;
  const long long per = (long long)g.h1 * P * g.n3;
  const long long n = per * 6 * nload;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long long)gridDim.x * 256) {
    const long long lc = t / per;
    const int L = (int)(lc / 6);
    const int its = min(stop_iter[L], *itp);
    const T2* Xs = (its & 1) ? Xs1 : Xs0;
    const long long rem = t % per;
    const int i3 = (int)(rem % g.n3);
    const int r = (int)((rem / g.n3) % P);
    const int k1 = (int)(rem / ((long long)g.n3 * P));
    const T2* src = Xs + lc * g.spec + (long long)k1 * Q * P * g.n3 + (long long)r * g.n3 + i3;
    T2* dst = X + lc * g.spec + (long long)k1 * g.n2 * g.n3 + i3;
    T2 x[QMAX];
    for (int q = 0; q < Q; ++q) {
      T2 w = tw1[r * q];
      w.y = -w.y;
      x[q] = cmul(src[(long long)q * P * g.n3], w);
    }
    for (int j = 0; j < Q; ++j) {
      T2 acc = T2{0, 0};
      for (int q = 0; q < Q; ++q) {
        T2 w = tw1[((j * q) % Q) * P];
        w.y = -w.y;
        acc = cadd(acc, cmul(x[q], w));
      }
      dst[(long long)(r + P * j) * g.n3] = acc;
    }
  }
}

// ----------------------------------------------------------- candidates ---
template <int N1, int Q, int W>
constexpr int stress2_nt() {
  return N1 * Q * W >= 2048 ? 512 : 256;
}
// threads of a Green-pass block: one per (comp, i3) item, and at most two
// bins per thread in FP32 (one in FP64) for the operator kept in registers
template <typename T, int P, int N3>
constexpr int green3_nt() {
  const int per = sizeof(T) == 8 ? 1 : 2;
  const int a = 6 * N3, b = (P * N3 + per - 1) / per;
  int nt = ((a > b ? a : b) + 63) / 64 * 64;
  return nt > 1024 ? 1024 : nt;
}

// a variant for the SNF grid (N1, N2, N3) with N2 = Q P, stress tiles W wide,
// and the Green pass with or without the next load's prefetch
template <typename T, int N1, int N2, int N3, int Q, int W, bool PF = true>
void add_cand(const Geo& g, TwoPass<T>* out, int maxn, int* n) {
  constexpr int P = N2 / Q;
  static_assert(P * Q == N2, "Q divides the axis-2 length");
  static_assert(Q <= QMAX, "the state conversions hold Q values per thread");
  static_assert(N3 % W == 0, "W divides the axis-3 length");
  if (*n >= maxn || g.n1 != N1 || g.n2 != N2 || g.n3 != N3) return;
  TwoPass<T> c;
  constexpr int NTS = stress2_nt<N1, Q, W>();
  constexpr int NTG = green3_nt<T, P, N3>();
  c.s2 = k_stress2<T, N1, Q, W, NTS>;
  c.g3[GREEN_TABLE] = k_green3<T, P, N3, NTG, GREEN_TABLE, PF>;
  c.g3[GREEN_MOMENTS] = k_green3<T, P, N3, NTG, GREEN_MOMENTS, PF>;
  c.g3inc[GREEN_TABLE] = k_green3<T, P, N3, NTG, GREEN_TABLE, PF, true>;
  c.g3inc[GREEN_MOMENTS] = k_green3<T, P, N3, NTG, GREEN_MOMENTS, PF, true>;
  c.g3[GREEN_ISO] = k_green3<T, P, N3, NTG, GREEN_ISO, PF>;
  c.g3inc[GREEN_ISO] = k_green3<T, P, N3, NTG, GREEN_ISO, PF, true>;
  c.Q = Q;
  c.P = P;
  c.W = W;
  c.nts = NTS;
  c.ntg = NTG;
  c.ldss = sizeof(C2<T>) * ((size_t)N1 + 2 * Q + (size_t)N1 * 3 * Q * W) + sizeof(T) * 36 * 16;
  c.ldsg = sizeof(C2<T>) * ((size_t)N3 + P + (size_t)6 * P * (N3 + 1));
  out[(*n)++] = c;
}

template <typename T, int N, int Q, int W, bool PF = true>
void add_cubic(const Geo& g, TwoPass<T>* out, int maxn, int* n) {
  add_cand<T, N, N, N, Q, W, PF>(g, out, maxn, n);
}

template <typename T>
int candidates_t(const Geo& g, TwoPass<T>* out, int maxn) {
  int n = 0;
  // cubic SNF grids of the batched size classes; the first candidate of each
  // is the default
  if (g.n1 != g.n2 || g.n2 != g.n3) return 0;
  if constexpr (sizeof(T) == 4) {
    switch (g.n1) {
      case 32:
        add_cubic<T, 32, 4, 8>(g, out, maxn, &n);
        add_cubic<T, 32, 2, 16>(g, out, maxn, &n);
        add_cubic<T, 32, 4, 8, false>(g, out, maxn, &n);
        break;
      case 48:
        add_cubic<T, 48, 4, 8>(g, out, maxn, &n);
        add_cubic<T, 48, 3, 8>(g, out, maxn, &n);
        add_cubic<T, 48, 3, 8, false>(g, out, maxn, &n);
        break;
      case 64:
        add_cubic<T, 64, 4, 8>(g, out, maxn, &n);
        add_cubic<T, 64, 8, 4>(g, out, maxn, &n);
        add_cubic<T, 64, 4, 8, false>(g, out, maxn, &n);
        break;
      case 96:
        add_cubic<T, 96, 6, 8>(g, out, maxn, &n);
        add_cubic<T, 96, 6, 4>(g, out, maxn, &n);
        add_cubic<T, 96, 8, 4>(g, out, maxn, &n);
        // without the Green pass's prefetch (fewer registers live across the
        // load loop: at 96 points the prefetching build spills)
        add_cubic<T, 96, 6, 4, false>(g, out, maxn, &n);
        add_cubic<T, 96, 8, 4, false>(g, out, maxn, &n);
        break;
      default:
        break;
    }
  } else {
    // FP64: the Green operator of two bins per thread does not fit the
    // registers beyond the smallest grid
    if (g.n1 == 32) add_cubic<T, 32, 4, 8>(g, out, maxn, &n);
  }
  return n;
}

template <typename T>
void to_split_t(const Geo& g, int Q, const C2<T>* tw1, const C2<T>* X, C2<T>* Xs, int nload, hipStream_t st) {
  const long long n = (long long)g.h1 * (g.n2 / Q) * g.n3 * 6 * nload;
  const int nblk = (int)std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_to_split<T>, dim3(nblk), dim3(256), 0, st, g, Q, tw1, X, Xs, nload);
}

template <typename T>
void from_split_t(const Geo& g, int Q, const C2<T>* tw1, const C2<T>* Xs0, const C2<T>* Xs1, C2<T>* X,
                  const int* stop_iter, const int* itp, int nload, hipStream_t st) {
  const long long n = (long long)g.h1 * (g.n2 / Q) * g.n3 * 6 * nload;
  const int nblk = (int)std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_from_split<T>, dim3(nblk), dim3(256), 0, st, g, Q, tw1, Xs0, Xs1, X, stop_iter, itp, nload);
}

}  // namespace

int twopass_candidates(const Geo& g, TwoPass<float>* out, int maxn) { return candidates_t<float>(g, out, maxn); }
int twopass_candidates(const Geo& g, TwoPass<double>* out, int maxn) { return candidates_t<double>(g, out, maxn); }

void twopass_to_split(const Geo& g, int Q, const C2<float>* tw1, const C2<float>* X, C2<float>* Xs, int nload,
                      hipStream_t st) {
  to_split_t<float>(g, Q, tw1, X, Xs, nload, st);
}
void twopass_to_split(const Geo& g, int Q, const C2<double>* tw1, const C2<double>* X, C2<double>* Xs, int nload,
                      hipStream_t st) {
  to_split_t<double>(g, Q, tw1, X, Xs, nload, st);
}
void twopass_from_split(const Geo& g, int Q, const C2<float>* tw1, const C2<float>* Xs0, const C2<float>* Xs1,
                        C2<float>* X, const int* stop_iter, const int* itp, int nload, hipStream_t st) {
  from_split_t<float>(g, Q, tw1, Xs0, Xs1, X, stop_iter, itp, nload, st);
}
void twopass_from_split(const Geo& g, int Q, const C2<double>* tw1, const C2<double>* Xs0, const C2<double>* Xs1,
                        C2<double>* X, const int* stop_iter, const int* itp, int nload, hipStream_t st) {
  from_split_t<double>(g, Q, tw1, Xs0, Xs1, X, stop_iter, itp, nload, st);
}
