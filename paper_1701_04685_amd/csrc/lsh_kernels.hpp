// lsh_kernels.hpp -- the Basic Scheme's device kernels for gfx950.
//
// Thm. (pde_discretization), eq. (pde_coefficients): E = -Gamma^p[(C - C0):(E + eps0)]
// on P(M), iterated as in Sec. 4.  In the SNF ordering the pattern DFT of
// eq. (Fouriermatrix) is a 3-D DFT over Z_n1 x Z_n2 x Z_n3.  The state is kept
// partially transformed so that every pass is a bundle of 1-D line FFTs held
// in LDS:
//
//   layout     [load][comp][k1 < n1/2+1][i2 < n2][i3 < n3]  complex, R2C along axis 1
//   S  axis 1  X = D1[E]/n1 --C2R--> E(y) --(C-C0):(E+eps0)--> tau(y) --R2C--> D1[tau]
//   B  axis 2  D1[tau] --FFT--> D12[tau]
//   G  axis 3  --FFT--> tau_hat --(-Gamma^p/m)--> E_hat --IFFT--> P = D12[E]/(n1 n2),
//              Cauchy residual against the previous P (double sums)
//   Bi axis 2  P --IFFT--> D1[E]/n1
//
// Every kernel is templated on the line length NC (> 0: compile-time FFT and
// fully unrolled loads; 0: runtime plan) and on its tile width W / block size
// NT.  All global loads of a tile are issued before any of them is used.
#pragma once
#include <hip/hip_runtime.h>

#include "lsh_fft.hpp"
#include "lsh_green.hpp"

#include "lsh_common.hpp"

// ------------------------------------------------------- axis-1 (stress) ---
// One block: the axis-1 lines at fixed (load, i2) for W consecutive i3 and all
// six components; component pairs (0,1), (2,3), (4,5) share one complex line.
// LDS: twiddles[n1] then Z[k][q*W + w] (k < n1, q < 3, w < W), then the
// (C_p - C0) of the first NDL phases (more phases are read from global memory).
// MINW asks the compiler for at least that many waves per SIMD.
template <typename T, int MODE, int NC, int W, int NT, int NDL = 16, int MINW = 1>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MINW)))
k_axis1(Geo g, FftPlan pl, const C2<T>* __restrict__ tw,
                                              const C2<T>* __restrict__ X, C2<T>* __restrict__ Y,
                                              const Inst* __restrict__ insts, const int* __restrict__ inst_of,
                                              const double* __restrict__ eps0, const int* __restrict__ stop_iter,
                                              const int* __restrict__ itp, const double* const* __restrict__ Einit,
                                              const double* __restrict__ means, double* const* __restrict__ Eout,
                                              double* __restrict__ partial) {
  using T2 = C2<T>;
  constexpr int W3 = 3 * W;
  constexpr bool NTS = sizeof(T) == 4;  // nontemporal state and polarisation (measured: pays in FP32 only)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n1 = NC > 0 ? NC : g.n1;
  const int h1 = n1 / 2 + 1;
  T2* twl = reinterpret_cast<T2*>(smem_raw);
  T2* Z = twl + n1;
  T* Dl = reinterpret_cast<T*>(Z + n1 * W3);
  const int L = blockIdx.y;
  if (MODE == MODE_STRESS && *itp >= stop_iter[L]) return;
  const Inst& in = insts[inst_of[L]];
  const uint8_t* __restrict__ phase = in.phase;
  const T* __restrict__ dmat = reinterpret_cast<const T*>(in.dmat);
  const double* __restrict__ cmat = in.cmat;
  const int nphase = in.nphase;
  // consecutive blocks take consecutive i2 at one i3 tile: their 16-byte x W
  // runs then lie n3 elements apart instead of side by side, which the memory
  // system serves faster (measured: +13% for a copy with this pattern, W = 8)
  const int a2 = blockIdx.x % g.n2;
  const int a30 = (blockIdx.x / g.n2) * W;
  const long long n23 = (long long)g.n2 * g.n3;
  const int tid = threadIdx.x;
  const long long colbase = (long long)a2 * g.n3 + a30;
  const int npairs = h1 * W3;
  constexpr int PT = NC > 0 ? ((NC / 2 + 1) * W3 + NT - 1) / NT : 1;
  constexpr int QT = NC > 0 ? (NC * W + NT - 1) / NT : 1;

  stage_twiddles<T>(twl, tw, n1);
  // phase indices of this thread's points: loaded first, used after the C2R
  int ph[QT];
  if (MODE == MODE_STRESS) {
    const int nd = nphase < NDL ? nphase : NDL;
    for (int i = tid; i < 36 * nd; i += NT) Dl[i] = dmat[i];
    if constexpr (NC > 0) {
#pragma unroll
      for (int i = 0; i < QT; ++i) {
        const int idx = tid + i * NT;
        ph[i] = -1;
        if (((NC * W) % NT == 0 || idx < NC * W) && a30 + idx % W < g.n3)
          ph[i] = phase[(long long)(idx / W) * n23 + colbase + idx % W];
      }
    }
  }

  if (MODE != MODE_INIT) {
    // Hermitian extension: Z_q[k] = X_{2q}[k] + i X_{2q+1}[k] on the full line
    auto put = [&](int idx, T2 a, T2 b) {
      const int w = idx % W, q = (idx / W) % 3, k = idx / W3;
      const int col = q * W + w;
      if (k == 0 || 2 * k == n1) {
        Z[k * W3 + col] = T2{a.x, b.x};
      } else {
        Z[k * W3 + col] = T2{a.x - b.y, a.y + b.x};
        Z[(n1 - k) * W3 + col] = T2{a.x + b.y, b.x - a.y};
      }
    };
    auto addr = [&](int idx, int c2) -> long long {
      const int w = idx % W, q = (idx / W) % 3, k = idx / W3;
      return ((long long)(L * 6 + 2 * q + c2)) * g.spec + (long long)k * n23 + colbase + w;
    };
    if constexpr (NC > 0) {
      T2 ra[PT], rb[PT];
#pragma unroll
      for (int i = 0; i < PT; ++i) {
        const int idx = tid + i * NT;
        ra[i] = T2{0, 0};
        rb[i] = T2{0, 0};
        if ((npairs % NT == 0 || idx < npairs) && a30 + idx % W < g.n3) {
          ra[i] = ld_nt(X + addr(idx, 0));
          rb[i] = ld_nt(X + addr(idx, 1));
        }
      }
#pragma unroll
      for (int i = 0; i < PT; ++i) {
        const int idx = tid + i * NT;
        if (npairs % NT == 0 || idx < npairs) put(idx, ra[i], rb[i]);
      }
    } else {
      for (int idx = tid; idx < npairs; idx += NT) {
        T2 a = T2{0, 0}, b = T2{0, 0};
        if (a30 + idx % W < g.n3) {
          a = ld_st<NTS>(X + addr(idx, 0));
          b = ld_st<NTS>(X + addr(idx, 1));
        }
        put(idx, a, b);
      }
    }
    __syncthreads();
    fft_any<T, +1, NC, W3, true, NT>(Z, pl, 1, W3, twl);
  }

  if (MODE == MODE_STRESS) {
    const double* e0 = eps0 + 6 * L;
    const T ep[6] = {(T)e0[0], (T)e0[1], (T)e0[2], (T)e0[3], (T)e0[4], (T)e0[5]};
    // D points at LDS (Dl) or global memory (dmat); the two callers below are
    // separate code paths so that LDS reads stay ds_read instructions
    auto stress = [&](int idx, const T* D) {
      const int w = idx % W, a1 = idx / W;
      T2* z = Z + a1 * W3 + w;
      const T2 z0 = z[0], z1 = z[W], z2 = z[2 * W];
      const T E[6] = {z0.x + ep[0], z0.y + ep[1], z1.x + ep[2], z1.y + ep[3], z2.x + ep[4], z2.y + ep[5]};
      T t[6];
      stress6<T>(D, E, t);
      z[0] = T2{t[0], t[1]};
      z[W] = T2{t[2], t[3]};
      z[2 * W] = T2{t[4], t[5]};
    };
    if constexpr (NC > 0) {
      if (nphase <= NDL) {
#pragma unroll
        for (int i = 0; i < QT; ++i)
          if (ph[i] >= 0) stress(tid + i * NT, Dl + 36 * ph[i]);
      } else {
#pragma unroll
        for (int i = 0; i < QT; ++i)
          if (ph[i] >= 0) stress(tid + i * NT, dmat + 36 * ph[i]);
      }
    } else {
      for (int idx = tid; idx < n1 * W; idx += NT)
        if (a30 + idx % W < g.n3) {
          const int p = phase[(long long)(idx / W) * n23 + colbase + idx % W];
          if (nphase <= NDL)
            stress(idx, Dl + 36 * p);
          else
            stress(idx, dmat + 36 * p);
        }
    }
  } else if (MODE == MODE_INIT) {
    const double SQ2I = 0.70710678118654752440;
    // this load's start field (the caller's [ncf][m] block), or none: zero start
    const double* __restrict__ El = Einit[L];
    for (int idx = tid; idx < n1 * W; idx += NT) {
      const int w = idx % W, a1 = idx / W;
      double E[6] = {0, 0, 0, 0, 0, 0};
      if (a30 + w < g.n3) {
        const long long pt = (long long)a1 * n23 + colbase + w;
        for (int c = 0; c < 6; ++c) {
          const int bc = boundary_comp(c, g.ncf);
          const double v = (bc < 0 || !El) ? 0.0 : El[(long long)bc * g.m + pt] * (c < 3 ? 1.0 : SQ2I);
          // the solver keeps X = D1[E] / n1 (D1: unnormalised DFT along axis 1)
          E[c] = (v - means[6 * L + c]) / (double)n1;
        }
      }
      T2* z = Z + a1 * W3 + w;
      z[0] = T2{(T)E[0], (T)E[1]};
      z[W] = T2{(T)E[2], (T)E[3]};
      z[2 * W] = T2{(T)E[4], (T)E[5]};
    }
  } else {  // MODE_FINAL: sigma = C(y):(E + eps0) summed in double, optional E out
    const double* e0 = eps0 + 6 * L;
    const double SQ2 = 1.41421356237309504880;
    // this load's field output (the caller's [ncf][m] block), if requested
    double* __restrict__ Eo = Eout ? Eout[L] : nullptr;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int idx = tid; idx < n1 * W; idx += NT) {
      const int w = idx % W, a1 = idx / W;
      if (a30 + w >= g.n3) continue;
      const T2* z = Z + a1 * W3 + w;
      const double E[6] = {(double)z[0].x, (double)z[0].y, (double)z[W].x,
                           (double)z[W].y, (double)z[2 * W].x, (double)z[2 * W].y};
      const long long pt = (long long)a1 * n23 + colbase + w;
      const double* Cm = cmat + 36 * phase[pt];
      for (int I = 0; I < 6; ++I) {
        double s = 0.0;
        for (int J = 0; J < 6; ++J) s += Cm[6 * I + J] * (E[J] + e0[J]);
        acc[I] += s;
      }
      if (Eo)
        for (int c = 0; c < 6; ++c) {
          const int bc = boundary_comp(c, g.ncf);
          if (bc >= 0) Eo[(long long)bc * g.m + pt] = E[c] * (c < 3 ? 1.0 : SQ2);
        }
    }
    block_sum<6>(acc, partial + ((long long)L * gridDim.x + blockIdx.x) * 6);
    return;
  }

  __syncthreads();
  fft_any<T, -1, NC, W3, true, NT>(Z, pl, 1, W3, twl);

  // unpack the pairs and store the half spectrum k < h1
  auto store = [&](int idx) {
    const int w = idx % W, q = (idx / W) % 3, k = idx / W3;
    if (a30 + w >= g.n3) return;
    const int col = q * W + w;
    const T2 zk = Z[k * W3 + col];
    const T2 zn = Z[((n1 - k) % n1) * W3 + col];
    const T hf = (T)0.5;
    const long long off = (long long)k * n23 + colbase + w;
    st_st<NTS>(Y + ((long long)(L * 6 + 2 * q)) * g.spec + off, T2{hf * (zk.x + zn.x), hf * (zk.y - zn.y)});
    st_st<NTS>(Y + ((long long)(L * 6 + 2 * q + 1)) * g.spec + off, T2{hf * (zk.y + zn.y), hf * (zn.x - zk.x)});
  };
  if constexpr (NC > 0) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int idx = tid + i * NT;
      if (npairs % NT == 0 || idx < npairs) store(idx);
    }
  } else {
    for (int idx = tid; idx < npairs; idx += NT) store(idx);
  }
}

// ----------------------------------------------------------------- axis 2 ---
// One block: W consecutive i3 columns at fixed (load, comp, k1); lines along
// axis 2.  LDS: twiddles[n2] then Z[i2*W + w].
template <typename T, int DIR, int NC, int W, int NT>
__global__ void __launch_bounds__(NT) k_axis2(Geo g, FftPlan pl, const C2<T>* __restrict__ tw,
                                              const C2<T>* __restrict__ src, C2<T>* __restrict__ dst,
                                              const int* __restrict__ stop_iter, const int* __restrict__ itp,
                                              T scale) {
  using T2 = C2<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n2 = NC > 0 ? NC : g.n2;
  T2* twl = reinterpret_cast<T2*>(smem_raw);
  T2* Z = twl + n2;
  // The grid is (h1 * ntile3, 6, nload).  The forward pass takes its blocks in
  // dispatch order k1 downwards, every tile, component and load of one k1
  // before the next: the Green pass reads positions upwards from k1 = 0, so
  // the planes written last are the first it reads.  The inverse pass keeps
  // the load-major order (neighbouring blocks on neighbouring tiles).
  const int ntile3 = (g.n3 + W - 1) / W;
  int k1, a30, c, L;
  if constexpr (DIR < 0) {
    const long long per_k1 = (long long)ntile3 * 6 * gridDim.z;
    const long long lin = blockIdx.x + (long long)gridDim.x * (blockIdx.y + 6LL * blockIdx.z);
    k1 = g.h1 - 1 - (int)(lin / per_k1);
    const int inner = (int)(lin % per_k1);
    a30 = (inner % ntile3) * W;
    c = (inner / ntile3) % 6;
    L = inner / (ntile3 * 6);
  } else {
    L = blockIdx.z;
    c = blockIdx.y;
    k1 = blockIdx.x / ntile3;
    a30 = (blockIdx.x % ntile3) * W;
  }
  if (stop_iter && *itp >= stop_iter[L]) return;
  const long long base = ((long long)(L * 6 + c)) * g.spec + (long long)k1 * n2 * g.n3 + a30;
  const int tid = threadIdx.x;
  const int ne = n2 * W;
  stage_twiddles<T>(twl, tw, n2);
  if constexpr (NC > 0) {
    constexpr int ET = (NC * W + NT - 1) / NT;
    T2 r[ET];
#pragma unroll
    for (int i = 0; i < ET; ++i) {
      const int idx = tid + i * NT;
      r[i] = T2{0, 0};
      if (((NC * W) % NT == 0 || idx < ne) && a30 + idx % W < g.n3)
        r[i] = ld_st<(DIR > 0)>(src + base + (long long)(idx / W) * g.n3 + idx % W);
    }
#pragma unroll
    for (int i = 0; i < ET; ++i) {
      const int idx = tid + i * NT;
      if ((NC * W) % NT == 0 || idx < ne) Z[idx] = r[i];
    }
  } else {
    for (int idx = tid; idx < ne; idx += NT)
      Z[idx] = (a30 + idx % W < g.n3) ? src[base + (long long)(idx / W) * g.n3 + idx % W] : T2{0, 0};
  }
  __syncthreads();
  fft_any<T, DIR, NC, W, true, NT>(Z, pl, 1, W, twl);
  for (int idx = tid; idx < ne; idx += NT) {
    if (a30 + idx % W < g.n3) {
      T2 v = Z[idx];
      if (scale != (T)1) v = T2{v.x * scale, v.y * scale};
      dst[base + (long long)(idx / W) * g.n3 + idx % W] = v;
    }
  }
}

// ------------------------------------------------------------ Green pass ---
// One block per (position (k1,k2), load); blocks of one position are placed
// on the same XCD back to back (block id mod 8 picks the XCD) so that a
// position's Gamma table rows, when a table is used, are read from HBM once
// and then hit that XCD's L2.  LDS: twiddles[n3], lines[6][ls].
// gmode: 0 isotropic C0 (moment form, on the fly), 1 general C0 on the fly,
// 2 table [pos][21][n3] built at bind time (double sums, stored at T).
// GREEN_MOMENTS: isotropic C0 with the normalised alias moments (independent
// of C0) precomputed at bind time in the table slot: the 15 fourth moments per
// bin, [pos][15][n3].  The second moments follow from them, since every alias
// direction n is a unit vector: sum_k n_i n_j n_k n_k = n_i n_j.
// GM >= 0 fixes the Green mode at compile time (only that branch is built,
// which keeps the register count of the table and moment paths low); -1
// switches on the gmode argument.
// upd (every Green pass): UPD_LS, UPD_VE or UPD_INC (lsh_common.hpp).
template <typename T, int NC, int NT, int GM = -1>
__global__ void __launch_bounds__(NT) k_green(Geo g, FftPlan pl, const C2<T>* __restrict__ tw, GreenParams gp,
                                              const C2<T>* __restrict__ tau, const C2<T>* __restrict__ Pold,
                                              C2<T>* __restrict__ Pnew, const T* __restrict__ table,
                                              const Inst* __restrict__ insts, const int* __restrict__ inst_of,
                                              const int* __restrict__ chunks_unused,
                                              const int* __restrict__ stop_iter, const int* __restrict__ itp,
                                              int nload, int npos, double* __restrict__ partial, int ls, int gmode,
                                              int upd, C2<T>* __restrict__ dP) {
  using T2 = C2<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n3 = NC > 0 ? NC : g.n3;
  T2* twl = reinterpret_cast<T2*>(smem_raw);
  T2* lines = twl + n3;
  // XCD-aware block order
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int pos = (slot / nload) * 8 + xcd;
  const int L = slot % nload;
  if (pos >= npos || *itp >= stop_iter[L]) return;
  const double mu0 = insts[inst_of[L]].mu0, riso = insts[inst_of[L]].riso;
  const int k1 = pos / g.n2, k2 = pos % g.n2;
  const int tid = threadIdx.x;
  const double scale = -1.0 / (double)g.m;
  const double wk1 = (k1 == 0 || 2 * k1 == g.n1) ? 1.0 : 2.0;
  const long long row = (long long)k1 * g.n2 * g.n3 + (long long)k2 * g.n3;
  const int ne = 6 * n3;
  constexpr int ET = NC > 0 ? (6 * NC + NT - 1) / NT : 1;

  stage_twiddles<T>(twl, tw, n3);
  // tau lines (and the table rows) first, all loads in flight together
  if constexpr (NC > 0) {
    // every entry assigned (zero past the end): with conditional
    // assignments the array stayed on the stack and each load waited for
    // its scratch store
    T2 r[ET];
#pragma unroll
    for (int i = 0; i < ET; ++i) {
      const int idx = tid + i * NT;
      const int c = idx / NC, k3 = idx % NC;
      r[i] = ((6 * NC) % NT == 0 || idx < ne) ? tau[((long long)(L * 6 + c)) * g.spec + row + k3] : T2{0, 0};
    }
#pragma unroll
    for (int i = 0; i < ET; ++i) {
      const int idx = tid + i * NT;
      if ((6 * NC) % NT == 0 || idx < ne) lines[(idx / NC) * ls + idx % NC] = r[i];
    }
  } else {
    for (int idx = tid; idx < ne; idx += NT) {
      const int c = idx / n3, k3 = idx - c * n3;
      lines[c * ls + k3] = tau[((long long)(L * 6 + c)) * g.spec + row + k3];
    }
  }
  __syncthreads();
  fft_any<T, -1, NC, 6, false, NT>(lines, pl, ls, 1, twl);
  const int gmd = GM >= 0 ? GM : gmode;
  for (int k3 = tid; k3 < n3; k3 += NT) {
    T G[21];
    if (gmd == GREEN_TABLE) {
      const T* tb = table + (long long)pos * 21 * n3 + k3;
#pragma unroll
      for (int t = 0; t < 21; ++t) G[t] = (T)(scale * (double)tb[(long long)t * n3]);
    } else if (gmd == GREEN_MOMENTS) {
      moments_emit(table, pos, n3, k3, mu0, riso, [&](int t, double v) { G[t] = (T)(scale * v); });
    } else {
      double Gd[21];
      if (gmd == GREEN_ISO)
        gamma_sym_iso(gp, mu0, riso, k1, k2, k3, Gd);
      else
        gamma_sym_at(gp, k1, k2, k3, Gd);
#pragma unroll
      for (int t = 0; t < 21; ++t) G[t] = (T)(scale * Gd[t]);
    }
    T2 v[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = lines[c * ls + k3];
#pragma unroll
    for (int I = 0; I < 6; ++I) {
      T2 s = T2{0, 0};
#pragma unroll
      for (int J = 0; J < 6; ++J) {
        const T gij = G[I <= J ? tri_idx(I, J) : tri_idx(J, I)];
        s.x += gij * v[J].x;
        s.y += gij * v[J].y;
      }
      lines[I * ls + k3] = s;
    }
  }
  // previous iterate: issue its loads before the inverse transform
  T2 po[NC > 0 ? ET : 1];
  if constexpr (NC > 0) {
#pragma unroll
    for (int i = 0; i < ET; ++i) {
      const int idx = tid + i * NT;
      po[i] = ((6 * NC) % NT == 0 || idx < ne) ? Pold[((long long)(L * 6 + idx / NC)) * g.spec + row + idx % NC]
                                                : T2{0, 0};
    }
  }
  __syncthreads();
  fft_any<T, +1, NC, 6, false, NT>(lines, pl, ls, 1, twl);
  double acc[2] = {0.0, 0.0};
  const int it = *itp;
  auto finish = [&](int idx, T2 ov) {
    const int c = idx / n3, k3 = idx - c * n3;
    const long long gi = ((long long)(L * 6 + c)) * g.spec + row + k3;
    double dd;
    const T2 nv = green_update<T>(lines[c * ls + k3], ov, upd, it, dP, gi, &dd);
    Pnew[gi] = nv;
    acc[0] += wk1 * dd;
    acc[1] += wk1 * ((double)nv.x * (double)nv.x + (double)nv.y * (double)nv.y);
  };
  if constexpr (NC > 0) {
#pragma unroll
    for (int i = 0; i < ET; ++i) {
      const int idx = tid + i * NT;
      if ((6 * NC) % NT == 0 || idx < ne) finish(idx, po[i]);
    }
  } else {
    for (int idx = tid; idx < ne; idx += NT) {
      const int c = idx / n3, k3 = idx - c * n3;
      finish(idx, Pold[((long long)(L * 6 + c)) * g.spec + row + k3]);
    }
  }
  block_sum<2>(acc, partial + ((long long)L * npos + pos) * 2);
}

// ------------------------------------------- Green pass, loads amortised ---
// One block per position (k1, k2) and chunk of GCH load cases.  The Green
// operator of the position (21 entries per k3, scaled by -1/m) is formed once
// into LDS and reused for every load of the chunk whose instance it belongs to.
// Loads run NL at a time.  The axis-3 transforms are Stockham FFTs whose first
// forward stage reads global memory and whose last inverse stage writes it;
// the forward radix-2 last stage, the 6x6 multiply and the inverse radix-2
// first stage run in registers on a thread that holds bins j and j + N/2 of
// all six components.  LDS lines carry one pad slot per 8 entries (fewer bank
// conflicts for the strided Stockham writes).
#define GCH 6
__host__ __device__ constexpr int gpad(int i) { return i + (i >> 3); }

// The thread index, opaque to the optimiser.  Addresses derived from it are
// then recomputed where they are used (a few integer operations) instead of
// being hoisted out of the load loop and held in registers across it, which
// lowers the Green pass's register peak by about 50 VGPRs and lets it run
// three waves per SIMD in FP64.  The empty asm emits no instruction.
__device__ __forceinline__ int g2_tid() {
  int t;
  asm volatile("" : "=v"(t) : "0"((int)threadIdx.x));
  return t;
}

template <int N> struct GreenPlan {
  static constexpr RadList RH = make_radlist(N / 2);
  // line stride: the padded length plus one, odd, so that the same entry of
  // neighbouring lines falls in different LDS banks
  static constexpr int LP = N + N / 8 + 1;
};

// element p of a line stored at (p >> 1) + (p & 1) N/2: the layout the
// middle (Green) stage leaves behind, read by the next stage
template <int N> __device__ __forceinline__ int g2_perm(int p) { return (p >> 1) + (p & 1) * (N / 2); }

// fixed-radix stage over NLN lines in LDS (in place); PERM: the input is in
// the g2_perm layout; LF: consecutive lanes take consecutive lines at the
// same j (they read the same twiddles, an LDS broadcast), else consecutive j
// of one line
template <typename T, int DIR, int N, int R, int NS, int NLN, int NT, bool PERM = false, bool LF = false>
__device__ __forceinline__ void g2_stage(C2<T>* lines, const C2<T>* __restrict__ twl) {
  using T2 = C2<T>;
  constexpr int LP = GreenPlan<N>::LP;
  constexpr int nbl = N / R;
  constexpr int nu = NLN * nbl;
  constexpr int NB = (nu + NT - 1) / NT;
  constexpr int tstep = N / (NS * R);
  const int tid = g2_tid();
  T2 v[NB][R];
  int dst[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int u = tid + q * NT;
    dst[q] = -1;
    if (nu % NT == 0 || u < nu) {
      const int l = LF ? u % NLN : u / nbl, j = LF ? u / NLN : u % nbl;
      const T2* src = lines + l * LP;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[gpad(PERM ? g2_perm<N>(j + r * nbl) : j + r * nbl)];
      const int k = j % NS;
      if (NS > 1 && k != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          T2 w = twl[r * tstep * k];
          if (DIR > 0) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      Bfly<T, DIR, R>::run(v[q]);
      dst[q] = l * LP + (j - k) * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q)
    if (nu % NT == 0 || dst[q] >= 0) {
      const int l = dst[q] / LP, d0 = dst[q] % LP;
#pragma unroll
      for (int r = 0; r < R; ++r) lines[l * LP + gpad(d0 + r * NS)] = v[q][r];
    }
  __syncthreads();
}

// forward stages S..n-1 of the half-length radix list (stage 0 came from global)
template <typename T, int N, int NLN, int NT, int S, int NS>
__device__ __forceinline__ void g2_fwd_rest(C2<T>* lines, const C2<T>* twl) {
  constexpr RadList RH = GreenPlan<N>::RH;
  if constexpr (S < RH.n) {
    g2_stage<T, -1, N, RH.r[S], NS, NLN, NT>(lines, twl);
    g2_fwd_rest<T, N, NLN, NT, S + 1, NS * RH.r[S]>(lines, twl);
  }
}
// inverse stages S..n-2 (the last one writes global memory)
template <typename T, int N, int NLN, int NT, int S, int NS>
__device__ __forceinline__ void g2_inv_mid(C2<T>* lines, const C2<T>* twl) {
  constexpr RadList RH = GreenPlan<N>::RH;
  if constexpr (S + 1 < RH.n) {
    g2_stage<T, +1, N, RH.r[S], NS, NLN, NT, S == 0>(lines, twl);
    g2_inv_mid<T, N, NLN, NT, S + 1, NS * RH.r[S]>(lines, twl);
  }
}
// inverse stages S.. of the half-length radix list, starting at NS (the
// final radix-2 stage is left to the caller)
template <typename T, int N, int NLN, int NT, int S, int NS>
__device__ __forceinline__ void g2_inv_all_but_last(C2<T>* lines, const C2<T>* twl) {
  constexpr RadList RH = GreenPlan<N>::RH;
  if constexpr (S < RH.n) {
    g2_stage<T, +1, N, RH.r[S], NS, NLN, NT, false, true>(lines, twl);
    g2_inv_all_but_last<T, N, NLN, NT, S + 1, NS * RH.r[S]>(lines, twl);
  }
}
// forward stages S.. after a radix-2 first stage (NS from 2), the first one
// reading the g2_perm layout
template <typename T, int N, int NLN, int NT, int S, int NS>
__device__ __forceinline__ void g2_fwd_after2(C2<T>* lines, const C2<T>* twl) {
  constexpr RadList RH = GreenPlan<N>::RH;
  if constexpr (S < RH.n) {
    g2_stage<T, -1, N, RH.r[S], NS, NLN, NT, S == 0, true>(lines, twl);
    g2_fwd_after2<T, N, NLN, NT, S + 1, NS * RH.r[S]>(lines, twl);
  }
}
__host__ __device__ constexpr int radprod(RadList L, int upto) {
  int p = 1;
  for (int i = 0; i < upto; ++i) p *= L.r[i];
  return p;
}

// MINW asks the compiler for at least that many waves per SIMD.
template <typename T, int N, int NL, int NT, int GM, int MINW = 1>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MINW))) k_green2(Geo g, FftPlan pl, const C2<T>* __restrict__ tw, GreenParams gp,
                                               const C2<T>* __restrict__ tau, const C2<T>* __restrict__ Pold,
                                               C2<T>* __restrict__ Pnew, const T* __restrict__ table,
                                               const Inst* __restrict__ insts, const int* __restrict__ inst_of,
                                               const int* __restrict__ chunks, const int* __restrict__ stop_iter,
                                               const int* __restrict__ itp, int nload, int npos,
                                               double* __restrict__ partial, int ls_unused, int gmode, int upd,
                                               C2<T>* __restrict__ dP) {
  using T2 = C2<T>;
  static_assert(NL == 1 || NL == 2, "one or two loads at a time");
  (void)pl;
  (void)ls_unused;
  (void)nload;
  (void)gmode;
  constexpr RadList RH = GreenPlan<N>::RH;
  constexpr int LP = GreenPlan<N>::LP;
  constexpr int H = N / 2;
  constexpr int NLN = NL * 6;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* twl = reinterpret_cast<T2*>(smem_raw);
  T* Gl = reinterpret_cast<T*>(twl + N);           // [21][N]
  T2* lines = reinterpret_cast<T2*>(Gl + 21 * N);  // [NL][6][LP]
  T2* twL = lines + NL * 6 * LP;                   // last inverse stage: [r-1][j] = tw[r j]
  const int pos = blockIdx.x;
  // a chunk holds up to GCH consecutive loads of one instance
  const int Lbeg = chunks[2 * blockIdx.y], Lend = chunks[2 * blockIdx.y + 1];
  const int it = *itp;
  const int k1 = pos / g.n2, k2 = pos % g.n2;
  const int tid = threadIdx.x;
  const double wk1 = (k1 == 0 || 2 * k1 == g.n1) ? 1.0 : 2.0;
  const long long row = (long long)k1 * g.n2 * g.n3 + (long long)k2 * g.n3;
  {
    bool any = false;
    for (int L = Lbeg; L < Lend; ++L) any = any || it < stop_iter[L];
    if (!any) return;
  }
  stage_twiddles<T>(twl, tw, N);
  // forward stage 0 reads tau straight from global memory; the next pair's
  // loads are issued while the current pair is transformed
  constexpr int R0 = RH.r[0];
  constexpr int nbl0 = N / R0;
  constexpr int nu0 = NLN * nbl0;
  constexpr int NB0 = (nu0 + NT - 1) / NT;
  T2 pf[NB0][R0];
  // last inverse stage geometry
  constexpr int RL = RH.r[RH.n - 1];
  constexpr int nblL = N / RL;
  static_assert(2 * radprod(RH, RH.n - 1) == nblL, "last stage spans the line");
  constexpr int nuL = NLN * nblL;
  constexpr int NBL = (nuL + NT - 1) / NT;
  auto load0 = [&](int Lb) {
    const int tid = g2_tid();
    const bool a0 = Lb < Lend && it < stop_iter[Lb];
    const bool a1 = NL == 2 && Lb + 1 < Lend && it < stop_iter[Lb + 1];
#pragma unroll
    for (int q = 0; q < NB0; ++q) {
      const int u = tid + q * NT;
      const int l = u / nbl0, j = u % nbl0;
      const int sl = l / 6, c = l % 6;
      const bool ok = (nu0 % NT == 0 || u < nu0) && (sl == 0 ? a0 : a1);
      const T2* src = tau + ((long long)((Lb + sl) * 6 + c)) * g.spec + row + j;
#pragma unroll
      for (int r = 0; r < R0; ++r) pf[q][r] = ok ? ld_nt(src + r * nbl0) : T2{0, 0};
    }
  };
  load0(Lbeg);  // in flight while the Green operator is formed
  for (int i = tid; i < (RL - 1) * nblL; i += NT) twL[i] = tw[(i / nblL + 1) * (i % nblL)];

  // the position's Green operator, scaled by -1/m, formed once for the chunk
  // (GM: GREEN_MOMENTS isotropic C0 from the alias moments, GREEN_GENERAL on
  // the fly, GREEN_TABLE stored rows).  Summing the moments on the fly instead
  // (no table read) made the FP64 128-point pass slower: 0.445 against 0.394 ms.
  {
    static_assert(GM != GREEN_ISO, "the isotropic path reads the moments table");
    const double scale = -1.0 / (double)g.m;
    for (int k3 = tid; k3 < N; k3 += NT) {
      if constexpr (GM == GREEN_TABLE) {
        const T* tb = table + (long long)pos * 21 * N + k3;
#pragma unroll
        for (int t = 0; t < 21; ++t) Gl[t * N + k3] = (T)(scale * (double)tb[(long long)t * N]);
      } else if constexpr (GM == GREEN_MOMENTS) {
        const int inst = inst_of[Lbeg];
        moments_emit(table, pos, N, k3, insts[inst].mu0, insts[inst].riso,
                     [&](int t, double v) { Gl[t * N + k3] = (T)(scale * v); });
      } else {
        double Gd[21];
        gamma_sym_at(gp, k1, k2, k3, Gd);
#pragma unroll
        for (int t = 0; t < 21; ++t) Gl[t * N + k3] = (T)(scale * Gd[t]);
      }
    }
  }

  for (int L0 = Lbeg; L0 < Lend; L0 += NL) {
    const bool act0 = it < stop_iter[L0];
    const bool act1 = NL == 2 && L0 + 1 < Lend && it < stop_iter[L0 + 1];
    const int tid = g2_tid();  // shadows the block-level index inside the loop
    if (!act0 && !act1) {
      load0(L0 + NL);
      continue;
    }

    // forward stage 0 (Stockham, NS = 1) on the loaded lines -> LDS
    {
      T2 v[NB0][R0];
#pragma unroll
      for (int q = 0; q < NB0; ++q)
#pragma unroll
        for (int r = 0; r < R0; ++r) v[q][r] = pf[q][r];
      if (L0 + NL < Lend) load0(L0 + NL);
#pragma unroll
      for (int q = 0; q < NB0; ++q) {
        const int u = tid + q * NT;
        if (nu0 % NT == 0 || u < nu0) {
          const int l = u / nbl0, j = u % nbl0;
          Bfly<T, -1, R0>::run(v[q]);
#pragma unroll
          for (int r = 0; r < R0; ++r) lines[l * LP + gpad(j * R0 + r)] = v[q][r];
        }
      }
      __syncthreads();
    }
    // the previous iterate for the residual: loads issued now, used at the end
    T2 po[NBL][RL];
#pragma unroll
    for (int q = 0; q < NBL; ++q) {
      const int u = tid + q * NT;
      const int l = u / nblL, j = u % nblL;
      const int sl = l / 6, c = l % 6;
      const bool ok = (nuL % NT == 0 || u < nuL) && (sl == 0 ? act0 : act1);
      const T2* src = Pold + ((long long)((L0 + sl) * 6 + c)) * g.spec + row + j;
#pragma unroll
      for (int r = 0; r < RL; ++r) po[q][r] = ok ? ld_nt(src + r * nblL) : T2{0, 0};
    }
    g2_fwd_rest<T, N, NLN, NT, 1, RH.r[0]>(lines, twl);

    // forward radix-2 last stage, -Gamma/m, inverse radix-2 first stage.
    // Outputs go back to the entries j and j + N/2 that were read (the
    // g2_perm layout): no thread's input is overwritten by another thread,
    // so no barrier is needed before the writes.
    {
      constexpr int nu = NL * H;
      constexpr int NB = (nu + NT - 1) / NT;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int u = tid + q * NT;
        if (nu % NT == 0 || u < nu) {
          const int sl = u / H, j = u % H;
          const T2 w = twl[j];
          T2 a[6], b[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            const T2* ln = lines + (sl * 6 + c) * LP;
            const T2 x0 = ln[gpad(j)];
            const T2 x1 = cmul(ln[gpad(j + H)], w);
            a[c] = cadd(x0, x1);  // bin j
            b[c] = csub(x0, x1);  // bin j + N/2
          }
#pragma unroll
          for (int I = 0; I < 6; ++I) {
            T2 ya = T2{0, 0}, yb = T2{0, 0};
#pragma unroll
            for (int J = 0; J < 6; ++J) {
              const int t = I <= J ? tri_idx(I, J) : tri_idx(J, I);
              const T ga = Gl[t * N + j], gb = Gl[t * N + j + H];
              ya.x += ga * a[J].x;
              ya.y += ga * a[J].y;
              yb.x += gb * b[J].x;
              yb.y += gb * b[J].y;
            }
            T2* ln = lines + (sl * 6 + I) * LP;
            ln[gpad(j)] = cadd(ya, yb);      // inverse radix-2 output 2j
            ln[gpad(j + H)] = csub(ya, yb);  // inverse radix-2 output 2j + 1
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      __syncthreads();
    }
    g2_inv_mid<T, N, NLN, NT, 0, 2>(lines, twl);

    // last inverse stage: LDS -> registers -> global, residual against P_old
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    {
      constexpr int R = RL;
      constexpr int nbl = nblL;
      constexpr int nu = nuL;
      constexpr int NB = NBL;
      T2 v[NB][R];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int u = tid + q * NT;
        if (nu % NT == 0 || u < nu) {
          const int l = u / nbl, j = u % nbl;
          const T2* ln = lines + l * LP;
#pragma unroll
          for (int r = 0; r < R; ++r) v[q][r] = ln[gpad(RH.n == 1 ? g2_perm<N>(j + r * nbl) : j + r * nbl)];
#pragma unroll
          for (int r = 1; r < R; ++r) {
            T2 w = twL[(r - 1) * nbl + j];
            w.y = -w.y;
            v[q][r] = cmul(v[q][r], w);
          }
          Bfly<T, +1, R>::run(v[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int u = tid + q * NT;
        const int l = u / nbl, j = u % nbl;
        const int sl = l / 6, c = l % 6;
        if ((nu % NT == 0 || u < nu) && (sl == 0 ? act0 : act1)) {
          const long long g0 = ((long long)((L0 + sl) * 6 + c)) * g.spec + row + j;
          double dd = 0.0, nn = 0.0;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            double d2;
            const T2 nv = green_update<T>(v[q][r], po[q][r], upd, it, dP, g0 + r * nbl, &d2);
            st_nt(Pnew + g0 + r * nbl, nv);
            dd += d2;
            nn += (double)nv.x * (double)nv.x + (double)nv.y * (double)nv.y;
          }
          if (sl == 0) {
            acc[0] += wk1 * dd;
            acc[1] += wk1 * nn;
          } else {
            acc[2] += wk1 * dd;
            acc[3] += wk1 * nn;
          }
        }
      }
    }
    double tot[4];
    block_sum<4>(acc, tot);
    if (tid == 0) {
      if (act0) {
        partial[((long long)L0 * npos + pos) * 2] = tot[0];
        partial[((long long)L0 * npos + pos) * 2 + 1] = tot[1];
      }
      if (act1) {
        partial[((long long)(L0 + 1) * npos + pos) * 2] = tot[2];
        partial[((long long)(L0 + 1) * npos + pos) * 2 + 1] = tot[3];
      }
    }
  }
}

// ------------------------------------------- axis-1 stress pass, fused ---
// The stress pass of k_axis1 (MODE_STRESS) with its middle in registers:
// the C2R along axis 1 (component pairs share a complex line) runs all its
// Stockham stages but the last in LDS; the last inverse radix-2 stage, the
// stress tau = (C - C0):(E + eps0) at the two points a1 = j and j + n1/2, and
// the first forward radix-2 stage of the R2C run on one thread that holds the
// three pair lines of one column.  Its outputs go back to the entries it read
// (g2_perm layout).  Lines are line-major in LDS with one pad slot per 8.
template <typename T, int N, int W, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_axis1s(Geo g, FftPlan pl, const C2<T>* __restrict__ tw,
                                               const C2<T>* __restrict__ X, C2<T>* __restrict__ Y,
                                               const Inst* __restrict__ insts, const int* __restrict__ inst_of,
                                               const double* __restrict__ eps0, const int* __restrict__ stop_iter,
                                               const int* __restrict__ itp, const double* const* __restrict__ Einit,
                                               const double* __restrict__ means, double* const* __restrict__ Eout,
                                               double* __restrict__ partial) {
  using T2 = C2<T>;
  (void)pl;
  (void)Einit;
  (void)means;
  (void)Eout;
  (void)partial;
  constexpr RadList RH = GreenPlan<N>::RH;
  constexpr int LP = GreenPlan<N>::LP;
  constexpr int H = N / 2;
  constexpr int h1 = N / 2 + 1;
  constexpr int NLN = 3 * W;
  constexpr int NDL = 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* twl = reinterpret_cast<T2*>(smem_raw);
  T* Dl = reinterpret_cast<T*>(twl + N);                 // 36 * NDL
  T2* lines = reinterpret_cast<T2*>(Dl + 36 * NDL);      // [3][W][LP]
  uint8_t* phl = reinterpret_cast<uint8_t*>(lines + 3 * W * LP);  // [a1][w]
  const int L = blockIdx.y;
  if (*itp >= stop_iter[L]) return;
  const Inst& in = insts[inst_of[L]];
  const uint8_t* __restrict__ phase = in.phase;
  const T* __restrict__ dmat = reinterpret_cast<const T*>(in.dmat);
  const int nphase = in.nphase;
  // consecutive blocks take consecutive i2 at one i3 tile: their 16-byte x W
  // runs then lie n3 elements apart instead of side by side, which the memory
  // system serves faster (measured: +13% for a copy with this pattern, W = 8)
  const int a2 = blockIdx.x % g.n2;
  const int a30 = (blockIdx.x / g.n2) * W;
  const long long n23 = (long long)g.n2 * g.n3;
  const long long colbase = (long long)a2 * g.n3 + a30;
  const int tid = threadIdx.x;

  // half spectra of the three pairs, w fastest (coalesced along i3)
  constexpr int npairs = h1 * NLN;
  constexpr int PT = (npairs + NT - 1) / NT;
  T2 ra[PT], rb[PT];
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int idx = tid + i * NT;
    const int w = idx % W, q = (idx / W) % 3, k = idx / NLN;
    ra[i] = T2{0, 0};
    rb[i] = T2{0, 0};
    if ((npairs % NT == 0 || idx < npairs) && a30 + w < g.n3) {
      const long long off = (long long)k * n23 + colbase + w;
      ra[i] = X[((long long)(L * 6 + 2 * q)) * g.spec + off];
      rb[i] = X[((long long)(L * 6 + 2 * q + 1)) * g.spec + off];
    }
  }
  // phase indices of the tile, [a1][w], loaded coalesced along i3
  constexpr int nuM = W * H;
  constexpr int NBM = (nuM + NT - 1) / NT;
  constexpr int NPH = N * W;
  constexpr int QP = (NPH + NT - 1) / NT;
  int phr[QP];
#pragma unroll
  for (int i = 0; i < QP; ++i) {
    const int idx = tid + i * NT;
    const int w = idx % W, a1 = idx / W;
    phr[i] = ((NPH % NT == 0 || idx < NPH) && a30 + w < g.n3) ? phase[(long long)a1 * n23 + colbase + w] : 0;
  }
  stage_twiddles<T>(twl, tw, N);
  {
    const int nd = nphase < NDL ? nphase : NDL;
    for (int i = tid; i < 36 * nd; i += NT) Dl[i] = dmat[i];
  }
#pragma unroll
  for (int i = 0; i < QP; ++i) {
    const int idx = tid + i * NT;
    if (NPH % NT == 0 || idx < NPH) phl[idx] = (uint8_t)phr[i];
  }
  // Hermitian extension: Z_q[k] = X_{2q}[k] + i X_{2q+1}[k] on the full line
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int idx = tid + i * NT;
    if (npairs % NT == 0 || idx < npairs) {
      const int w = idx % W, q = (idx / W) % 3, k = idx / NLN;
      const T2 a = ra[i], b = rb[i];
      T2* ln = lines + (q * W + w) * LP;
      if (k == 0 || k == H) {
        ln[gpad(k)] = T2{a.x, b.x};
      } else {
        ln[gpad(k)] = T2{a.x - b.y, a.y + b.x};
        ln[gpad(N - k)] = T2{a.x + b.y, b.x - a.y};
      }
    }
  }
  __syncthreads();
  // inverse stages but the last (radix 2)
  g2_inv_all_but_last<T, N, NLN, NT, 0, 1>(lines, twl);

  // last inverse radix-2, stress at two points, first forward radix-2
  {
    const double* e0 = eps0 + 6 * L;
    const T ep[6] = {(T)e0[0], (T)e0[1], (T)e0[2], (T)e0[3], (T)e0[4], (T)e0[5]};
#pragma unroll
    for (int qq = 0; qq < NBM; ++qq) {
      const int u = tid + qq * NT;
      if (nuM % NT == 0 || u < nuM) {
        const int j = u % H, w = u / H;  // j fastest: lanes walk one line
        const int p0 = phl[j * W + w], p1 = phl[(j + H) * W + w];
        T2 wv = twl[j];
        wv.y = -wv.y;
        T2 z0[3], z1[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const T2* ln = lines + (q * W + w) * LP;
          const T2 x0 = ln[gpad(j)];
          const T2 x1 = cmul(ln[gpad(j + H)], wv);
          z0[q] = cadd(x0, x1);  // a1 = j
          z1[q] = csub(x0, x1);  // a1 = j + N/2
        }
        T2 t0[3], t1[3];
        {
          const T E[6] = {z0[0].x + ep[0], z0[0].y + ep[1], z0[1].x + ep[2],
                          z0[1].y + ep[3], z0[2].x + ep[4], z0[2].y + ep[5]};
          T t[6];
          stress6<T>(nphase <= NDL ? Dl + 36 * p0 : Dl, E, t);
          if (nphase > NDL) stress6<T>(dmat + 36 * p0, E, t);
          t0[0] = T2{t[0], t[1]};
          t0[1] = T2{t[2], t[3]};
          t0[2] = T2{t[4], t[5]};
        }
        __builtin_amdgcn_sched_barrier(0);
        {
          const T E[6] = {z1[0].x + ep[0], z1[0].y + ep[1], z1[1].x + ep[2],
                          z1[1].y + ep[3], z1[2].x + ep[4], z1[2].y + ep[5]};
          T t[6];
          stress6<T>(nphase <= NDL ? Dl + 36 * p1 : Dl, E, t);
          if (nphase > NDL) stress6<T>(dmat + 36 * p1, E, t);
          t1[0] = T2{t[0], t[1]};
          t1[1] = T2{t[2], t[3]};
          t1[2] = T2{t[4], t[5]};
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          T2* ln = lines + (q * W + w) * LP;
          ln[gpad(j)] = cadd(t0[q], t1[q]);      // forward radix-2 output 2j
          ln[gpad(j + H)] = csub(t0[q], t1[q]);  // forward radix-2 output 2j + 1
        }
      }
    }
  }
  __syncthreads();
  // remaining forward stages, the first reading the g2_perm layout
  g2_fwd_after2<T, N, NLN, NT, 0, 2>(lines, twl);

  // unpack the pairs and store the half spectrum k < h1
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int idx = tid + i * NT;
    if (npairs % NT == 0 || idx < npairs) {
      const int w = idx % W, q = (idx / W) % 3, k = idx / NLN;
      if (a30 + w < g.n3) {
        const T2* ln = lines + (q * W + w) * LP;
        const T2 zk = ln[gpad(k)];
        const T2 zn = ln[gpad((N - k) % N)];
        const T hf = (T)0.5;
        const long long off = (long long)k * n23 + colbase + w;
        Y[((long long)(L * 6 + 2 * q)) * g.spec + off] = T2{hf * (zk.x + zn.x), hf * (zk.y - zn.y)};
        Y[((long long)(L * 6 + 2 * q + 1)) * g.spec + off] = T2{hf * (zk.y + zn.y), hf * (zn.x - zk.x)};
      }
    }
  }
}

// ------------------------------------------------------------ finalisers ---
__global__ void __launch_bounds__(1024) k_finalize_resid(const double* __restrict__ partial, int nblk, int nload,
                                                          const double* __restrict__ e0sq, double pscale, double tol,
                                                          int fixed, int* __restrict__ itp,
                                                          int* __restrict__ stop_iter, double* __restrict__ hist,
                                                          int* __restrict__ nonfinite) {
  // One block per load.  The iteration counter itp[0] is advanced here, by
  // the block that finishes last (itp[1] counts finished blocks and is back
  // at 0 when the kernel ends), so every block reads the counter before it
  // changes and no separate launch is needed.
  const int L = blockIdx.x;
  const int it = itp[0];
  if (it < stop_iter[L]) {
    // partial sums come in (numerator, denominator) pairs, 16-byte aligned
    const double2* p2 = reinterpret_cast<const double2*>(partial) + (long long)L * nblk;
    double s[2] = {0.0, 0.0};
    for (int j = threadIdx.x; j < nblk; j += blockDim.x) {
      const double2 q = p2[j];
      s[0] += q.x;
      s[1] += q.y;
    }
    double out[2];
    block_sum<2>(s, out);
    if (threadIdx.x == 0) {
      const double num = out[0] * pscale;
      const double den = out[1] * pscale + e0sq[L];
      const double r = sqrt(num / den);
      hist[(it % LSH_HIST) * nload + L] = r;
      if (!isfinite(r)) {
        nonfinite[L] = 1;
        stop_iter[L] = it + 1;
      } else if (!fixed && r <= tol) {
        stop_iter[L] = it + 1;
      }
    }
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&itp[1], 1) == (int)gridDim.x - 1) {
      itp[1] = 0;
      itp[0] = it + 1;
    }
  }
}

// n 8-byte words set to zero (clears state buffers with a kernel, not a
// runtime memset node)
__global__ void __launch_bounds__(256) k_zero(unsigned long long* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) p[i] = 0ull;
}

// The increment scheme's start: eps0 added to the state's mean bins.  The
// mean of a field sits in the first `count` elements of each (load,
// component) block of `spec` elements (the k1 = 0 plane of the four-pass
// state, the k1 = 0, q = 0 rows of the two-pass state), where the transforms'
// normalisation gives a constant field c the value c.
template <typename T>
__global__ void __launch_bounds__(256) k_add_mean(C2<T>* __restrict__ X, long long spec, long long count,
                                                  const double* __restrict__ eps0, int nload) {
  const long long n = count * 6 * nload;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long long)gridDim.x * 256) {
    const long long lc = t / count;
    X[lc * spec + t % count].x += (T)eps0[lc];
  }
}

// dst <- the state each load's last iteration wrote: P1 if min(stop_iter[L],
// it) is odd, else P0 (one (load, component) block of spec elements at a time).
template <typename T>
__global__ void __launch_bounds__(256) k_pick_parity(const C2<T>* __restrict__ P0, const C2<T>* __restrict__ P1,
                                                     C2<T>* __restrict__ dst, long long spec, int nload,
                                                     const int* __restrict__ stop_iter, const int* __restrict__ itp) {
  const long long n = spec * 6 * nload;
  const int it = *itp;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long long)gridDim.x * 256) {
    const int L = (int)(t / (spec * 6));
    dst[t] = (min(stop_iter[L], it) & 1) ? P1[t] : P0[t];
  }
}

// end of an iteration: advance the device-side iteration counter
__global__ void k_advance(int* itp) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *itp += 1;
}

__global__ void k_finalize_sum(const double* __restrict__ partial, int nblk, int nv, double scale,
                               double* __restrict__ out) {
  const int L = blockIdx.x, i = blockIdx.y;
  double s[1] = {0.0};
  for (int j = threadIdx.x; j < nblk; j += blockDim.x) s[0] += partial[((long long)L * nblk + j) * nv + i];
  double o[1];
  block_sum<1>(s, o);
  if (threadIdx.x == 0) out[L * nv + i] = scale * o[0];
}

// mean of the Mandel components of a start field (ncf components per load,
// one [ncf][m] block per load, null for a zero start), per (load, comp) block;
// components the field does not carry have mean 0
__global__ void k_mean(const double* const* __restrict__ Eptr, long long m, int ncf, double* __restrict__ means) {
  const int L = blockIdx.x, c = blockIdx.y;
  const double f = c < 3 ? 1.0 : 0.70710678118654752440;
  const int bc = boundary_comp(c, ncf);
  const double* __restrict__ E = Eptr[L];
  double s[1] = {0.0};
  if (bc >= 0 && E)
    for (long long i = threadIdx.x; i < m; i += blockDim.x) s[0] += E[(long long)bc * m + i];
  double o[1];
  block_sum<1>(s, o);
  if (threadIdx.x == 0) means[6 * L + c] = f * o[0] / (double)m;
}

// ------------------------------------------------- conjugate gradients ---
// CG for the Dirichlet kernel's system (see lsh_set_scheme): the iterate x,
// the residual z = -G C (x + eps0) (G C0 projects onto compatible strains),
// the direction p and W = -G C p all live in the solver's axis-1 half
// spectrum layout, where sums over the points follow from Parseval:
// sum_y a(y) b(y) = n1 sum_{k1 <= n1/2} w(k1) Re(a_k conj(b_k)), w = 1 at
// k1 = 0 and n1/2, else 2.  Per load the device keeps {rho, alpha, beta, -}.

// x += alpha p, z += alpha W, and the partial sums of ||z||^2, ||x + z||^2 and
// <z, C0 z> (Mandel C0, 36 doubles) over this block's spectrum slots.  One
// thread per slot (k1, i2, i3) holds all six components.
template <typename T>
__global__ void __launch_bounds__(256) k_cg_update(Geo g, const C2<T>* __restrict__ p, const C2<T>* __restrict__ Wv,
                                                   C2<T>* __restrict__ x, C2<T>* __restrict__ z,
                                                   const double* __restrict__ cg, const double* __restrict__ C0m,
                                                   const int* __restrict__ stop_iter, const int* __restrict__ itp,
                                                   double* __restrict__ partial) {
  using T2 = C2<T>;
  const int L = blockIdx.y;
  if (*itp >= stop_iter[L]) return;  // uniform over the block
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const T a = (T)cg[4 * L + 1];
  double acc[3] = {0.0, 0.0, 0.0};
  if (i < g.spec) {
    const int k1 = (int)(i / ((long long)g.n2 * g.n3));
    const double w = (k1 == 0 || 2 * k1 == g.n1) ? 1.0 : 2.0;
    double zr[6], zi[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const long long o = ((long long)(L * 6 + c)) * g.spec + i;
      const T2 pv = p[o], wv = Wv[o];
      T2 xv = x[o], zv = z[o];
      xv.x += a * pv.x;
      xv.y += a * pv.y;
      zv.x += a * wv.x;
      zv.y += a * wv.y;
      x[o] = xv;
      z[o] = zv;
      zr[c] = (double)zv.x;
      zi[c] = (double)zv.y;
      const double sx = (double)xv.x + zr[c], sy = (double)xv.y + zi[c];
      acc[0] += w * (zr[c] * zr[c] + zi[c] * zi[c]);
      acc[1] += w * (sx * sx + sy * sy);
    }
    double q = 0.0;
#pragma unroll
    for (int I = 0; I < 6; ++I)
#pragma unroll
      for (int J = 0; J < 6; ++J) q += C0m[6 * I + J] * (zr[I] * zr[J] + zi[I] * zi[J]);
    acc[2] += w * q;
  }
  block_sum<3>(acc, partial + ((long long)L * gridDim.x + blockIdx.x) * 3);
}

// Residual of the current iterate (the Basic Scheme's Cauchy residual one
// fixed-point step from x would show, ||z|| / ||x + z + eps0||), the stop test
// and beta = rho_new / rho_old (0 at the first iteration).
__global__ void k_cg_scalars(const double* __restrict__ partial, int nblk, int nload, const double* __restrict__ e0sq,
                             double pscale, double tol, int fixed, const int* __restrict__ itp,
                             int* __restrict__ stop_iter, double* __restrict__ hist, int* __restrict__ nonfinite,
                             double* __restrict__ cg) {
  const int L = blockIdx.x;
  const int it = *itp;
  if (it >= stop_iter[L]) return;
  double s[3] = {0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < nblk; j += blockDim.x)
#pragma unroll
    for (int v = 0; v < 3; ++v) s[v] += partial[((long long)L * nblk + j) * 3 + v];
  double o[3];
  block_sum<3>(s, o);
  if (threadIdx.x == 0) {
    const double zz = o[0] * pscale, xz = o[1] * pscale, rho = o[2] * pscale;
    const double r = sqrt(zz / (xz + e0sq[L]));
    hist[(it % LSH_HIST) * nload + L] = r;
    if (!isfinite(r) || !isfinite(rho)) {
      nonfinite[L] = 1;
      stop_iter[L] = it + 1;
    } else if (!fixed && r <= tol) {
      stop_iter[L] = it + 1;
    }
    const double rho_old = cg[4 * L];
    cg[4 * L + 2] = (it == 0 || !(rho_old > 0.0)) ? 0.0 : rho / rho_old;
    cg[4 * L] = rho;
  }
}

// alpha = rho / <p, C p> from the direction pass's partial sums.
__global__ void k_cg_alpha(const double* __restrict__ partial, int nblk, const int* __restrict__ itp,
                           const int* __restrict__ stop_iter, double* __restrict__ cg) {
  const int L = blockIdx.x;
  if (*itp >= stop_iter[L]) return;
  double s[1] = {0.0};
  for (int j = threadIdx.x; j < nblk; j += blockDim.x) s[0] += partial[(long long)L * nblk + j];
  double o[1];
  block_sum<1>(s, o);
  if (threadIdx.x == 0) cg[4 * L + 1] = o[0] > 0.0 ? cg[4 * L] / o[0] : 0.0;
}

// The direction pass: p <- z + beta p in the half spectrum (written back), then
// tau = C p at the points (no eps0: the operator's linear part) through the
// axis-1 transforms of k_axis1 (runtime plan), stored as the axis-2 input, and
// the partial sums of <p, C p> = sum_y p(y) . tau(y).  Block layout and LDS as
// k_axis1 (twiddles, lines, the first 16 phases' C in LDS); NC as in k_axis1
// (> 0: compile-time line length, 0: runtime plan).
template <typename T, int NC, int W, int NT>
__global__ void __launch_bounds__(NT) k_cg_stress(Geo g, FftPlan pl, const C2<T>* __restrict__ tw,
                                                  const C2<T>* __restrict__ z, C2<T>* __restrict__ p,
                                                  C2<T>* __restrict__ tau, const Inst* __restrict__ insts,
                                                  const int* __restrict__ inst_of, const double* __restrict__ cg,
                                                  const int* __restrict__ stop_iter, const int* __restrict__ itp,
                                                  double* __restrict__ partial) {
  using T2 = C2<T>;
  constexpr int W3 = 3 * W;
  constexpr int NDL = 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n1 = NC > 0 ? NC : g.n1;
  const int h1 = n1 / 2 + 1;
  T2* twl = reinterpret_cast<T2*>(smem_raw);
  T2* Z = twl + n1;
  T* Dl = reinterpret_cast<T*>(Z + n1 * W3);
  const int L = blockIdx.y;
  if (*itp >= stop_iter[L]) return;
  const Inst& in = insts[inst_of[L]];
  const uint8_t* __restrict__ phase = in.phase;
  const T* __restrict__ dmat = reinterpret_cast<const T*>(in.dmat);
  const int nphase = in.nphase;
  const int a2 = blockIdx.x % g.n2;
  const int a30 = (blockIdx.x / g.n2) * W;
  const long long n23 = (long long)g.n2 * g.n3;
  const long long colbase = (long long)a2 * g.n3 + a30;
  const int tid = threadIdx.x;
  const int npairs = h1 * W3;
  const T beta = (T)cg[4 * L + 2];
  stage_twiddles<T>(twl, tw, n1);
  const int nd = nphase < NDL ? nphase : NDL;
  for (int i = tid; i < 36 * nd; i += NT) Dl[i] = dmat[i];
  // new direction, written back, and its Hermitian extension (pairs of real
  // components share one complex line, as in k_axis1)
  for (int idx = tid; idx < npairs; idx += NT) {
    const int w = idx % W, q = (idx / W) % 3, k = idx / W3;
    T2 a = T2{0, 0}, b = T2{0, 0};
    if (a30 + w < g.n3) {
      const long long o0 = ((long long)(L * 6 + 2 * q)) * g.spec + (long long)k * n23 + colbase + w;
      const long long o1 = o0 + g.spec;
      const T2 za = z[o0], zb = z[o1], pa = p[o0], pb = p[o1];
      a = T2{za.x + beta * pa.x, za.y + beta * pa.y};
      b = T2{zb.x + beta * pb.x, zb.y + beta * pb.y};
      p[o0] = a;
      p[o1] = b;
    }
    const int col = q * W + w;
    if (k == 0 || 2 * k == n1) {
      Z[k * W3 + col] = T2{a.x, b.x};
    } else {
      Z[k * W3 + col] = T2{a.x - b.y, a.y + b.x};
      Z[(n1 - k) * W3 + col] = T2{a.x + b.y, b.x - a.y};
    }
  }
  __syncthreads();
  fft_any<T, +1, NC, W3, true, NT>(Z, pl, 1, W3, twl);
  double acc[1] = {0.0};
  for (int idx = tid; idx < n1 * W; idx += NT) {
    const int w = idx % W, a1 = idx / W;
    if (a30 + w >= g.n3) continue;
    const int ph = phase[(long long)a1 * n23 + colbase + w];
    const T* D = ph < NDL ? Dl + 36 * ph : dmat + 36 * ph;
    T2* zz = Z + a1 * W3 + w;
    const T2 z0 = zz[0], z1 = zz[W], z2 = zz[2 * W];
    const T E[6] = {z0.x, z0.y, z1.x, z1.y, z2.x, z2.y};
    T t[6];
    stress6<T>(D, E, t);
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[0] += (double)E[c] * (double)t[c];
    zz[0] = T2{t[0], t[1]};
    zz[W] = T2{t[2], t[3]};
    zz[2 * W] = T2{t[4], t[5]};
  }
  __syncthreads();
  fft_any<T, -1, NC, W3, true, NT>(Z, pl, 1, W3, twl);
  for (int idx = tid; idx < npairs; idx += NT) {
    const int w = idx % W, q = (idx / W) % 3, k = idx / W3;
    if (a30 + w >= g.n3) continue;
    const int col = q * W + w;
    const T2 zk = Z[k * W3 + col];
    const T2 zn = Z[((n1 - k) % n1) * W3 + col];
    const T hf = (T)0.5;
    const long long off = (long long)k * n23 + colbase + w;
    tau[((long long)(L * 6 + 2 * q)) * g.spec + off] = T2{hf * (zk.x + zn.x), hf * (zk.y - zn.y)};
    tau[((long long)(L * 6 + 2 * q + 1)) * g.spec + off] = T2{hf * (zk.y + zn.y), hf * (zn.x - zk.x)};
  }
  block_sum<1>(acc, partial + (long long)L * gridDim.x + blockIdx.x);
}

// ---------------------------------------------------------- Gamma table ---
// One thread per half-spectrum bin: the alias sums in double, stored at T.
template <typename T, int ISO>
__global__ void __launch_bounds__(256) k_gamma_table(Geo g, GreenParams gp, T* __restrict__ table,
                                                     double* __restrict__ minden) {
  const long long nb = g.spec;
  double mn = 1e300;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (long long)gridDim.x * blockDim.x) {
    const int k3 = (int)(i % g.n3);
    const int k2 = (int)((i / g.n3) % g.n2);
    const int k1 = (int)(i / ((long long)g.n2 * g.n3));
    double G[21];
    const double den = gamma_sym_at<ISO>(gp, k1, k2, k3, G);
    mn = fmin(mn, den);
    const long long pos = i / g.n3;
    for (int t = 0; t < 21; ++t) table[(pos * 21 + t) * g.n3 + k3] = (T)G[t];
  }
  __shared__ double red[16];
  for (int off = 32; off > 0; off >>= 1) mn = fmin(mn, __shfl_down(mn, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < (int)((blockDim.x + 63) >> 6); ++w) r = fmin(r, red[w]);
    minden[blockIdx.x] = r;
  }
}

// One thread per half-spectrum bin: the normalised fourth alias moments
// (isotropic C0 path), stored at T in the layout [pos][15][n3].
template <typename T>
__global__ void __launch_bounds__(256) k_moments_table(Geo g, GreenParams gp, T* __restrict__ table) {
  const long long nb = g.spec;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (long long)gridDim.x * blockDim.x) {
    const int k3 = (int)(i % g.n3);
    const int k2 = (int)((i / g.n3) % g.n2);
    const int k1 = (int)(i / ((long long)g.n2 * g.n3));
    IsoMoments M;
    iso_moments(gp, k1, k2, k3, M);
    const long long pos = i / g.n3;
#pragma unroll
    for (int t = 0; t < MOM_ROWS; ++t) table[(pos * MOM_ROWS + t) * g.n3 + k3] = (T)M.q[t];
  }
}

// Gamma^p at probe bins from the moments table (the values the solver uses).
template <typename T>
__global__ void k_moments_probe(const T* __restrict__ table, double* __restrict__ out, const long long* __restrict__ bins,
                                int n, Geo g, double mu0, double riso) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long pos = bins[3 * i] * g.n2 + bins[3 * i + 1];
  moments_emit(table, pos, g.n3, (int)bins[3 * i + 2], mu0, riso, [&](int t, double v) { out[21 * i + t] = v; });
}

__global__ void __launch_bounds__(128) k_gamma_probe(GreenParams gp, const long long* __restrict__ bins, int n, double* __restrict__ out,
                              int gmode, double mu0, double riso) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double G[21];
  if (gmode == GREEN_ISO)
    gamma_sym_iso(gp, mu0, riso, bins[3 * i], bins[3 * i + 1], bins[3 * i + 2], G);
  else
    gamma_sym_at(gp, bins[3 * i], bins[3 * i + 1], bins[3 * i + 2], G);
  for (int t = 0; t < 21; ++t) out[21 * i + t] = G[t];
}

template <typename T>
__global__ void k_cast_table(const T* __restrict__ src, double* __restrict__ dst, const long long* __restrict__ bins,
                             int n, Geo g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long pos = bins[3 * i] * g.n2 + bins[3 * i + 1];
  for (int t = 0; t < 21; ++t) dst[21 * i + t] = (double)src[(pos * 21 + t) * g.n3 + bins[3 * i + 2]];
}
