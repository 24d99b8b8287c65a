// lsh_solver.hip -- the Basic Scheme on P(M) for gfx950.
//
// Thm. (pde_discretization), eq. (pde_coefficients):
//     E_y = -Gamma^p[(C - C0):(E + eps0)]_y ,  y in P(M),
// iterated as in Sec. 4.  In the SNF ordering the pattern DFT is a 3-D DFT
// over Z_n1 x Z_n2 x Z_n3 (n = SNF diagonal).  The iteration state is kept
// partially transformed so that every pass is a 1-D line transform:
//
//   spectrum layout  [load][comp][k1 < n1/2+1][i2 < n2][i3 < n3]  (complex)
//   with the real-to-complex transform along axis 1.
//
//   S  (axis 1) : E(k1,a2,a3) --C2R--> E(y) --(C-C0):(E+eps0)--> tau(y) --R2C--> tau(k1,a2,a3)
//   B  (axis 2) : tau(k1,a2,a3) --FFT--> tau(k1,k2,a3)
//   G  (axis 3) : --FFT--> tau_hat(b) --  -Gamma^p_b / m  --> E_hat(b) --IFFT--> E(k1,k2,a3)
//                 plus the Cauchy residual against the previous E(k1,k2,a3)
//   Bi (axis 2) : E(k1,k2,a3) --IFFT--> E(k1,a2,a3)
//
// Six strain components are Mandel form; the two halves of each component
// pair ride in one complex line for the axis-1 real transforms.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "lsh_internal.hpp"

#define LSH_MAXE 16
#define LSH_HIST 64  // device ring of residuals per load

namespace {

struct Geo {
  int n1, n2, n3, h1;
  long long m;
  long long spec;  // h1 * n2 * n3
};

template <typename T> using C2 = typename cpx<T>::t;

// ------------------------------------------------------------ reductions ---
template <int NV>
__device__ void block_sum(double v[NV], double* out) {
  __shared__ double red[16][NV];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += __shfl_down(v[i], off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wid][i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[w][i];
      out[i] = s;
    }
  }
  __syncthreads();
}

// ------------------------------------------------------- axis-1 (stress) ---
enum { MODE_STRESS = 0, MODE_FINAL = 1, MODE_INIT = 2 };

// One block: lines along axis 1 at fixed (load, a2) for W consecutive a3 and
// all six components (three complex lines per column).  LDS holds
// Z[k][q*W + w], k < n1, q < 3, w < W.
template <typename T, int MODE>
__global__ void __launch_bounds__(512) k_axis1(Geo g, FftPlan pl, const C2<T>* __restrict__ tw,
                                               const C2<T>* __restrict__ X, C2<T>* __restrict__ Y,
                                               const uint8_t* __restrict__ phase, const T* __restrict__ dmat,
                                               const double* __restrict__ cmat, const double* __restrict__ eps0,
                                               const int* __restrict__ stop_iter, int it,
                                               const double* __restrict__ Einit, const double* __restrict__ means,
                                               double* __restrict__ Eout, double* __restrict__ partial, int W) {
  using T2 = C2<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* Z = reinterpret_cast<T2*>(smem_raw);
  const int L = blockIdx.y;
  if (MODE == MODE_STRESS && it >= stop_iter[L]) return;
  const int ntile3 = (g.n3 + W - 1) / W;
  const int a2 = blockIdx.x / ntile3;
  const int a30 = (blockIdx.x % ntile3) * W;
  const int n1 = g.n1, h1 = g.h1, W3 = 3 * W;
  const long long n23 = (long long)g.n2 * g.n3;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const long long colbase = (long long)a2 * g.n3 + a30;

  if (MODE != MODE_INIT) {
    // Hermitian extension: Z_q[k] = X_{2q}[k] + i X_{2q+1}[k] on the full line
    for (int idx = tid; idx < h1 * W3; idx += nthr) {
      const int w = idx % W, q = (idx / W) % 3, k = idx / W3;
      T2 a = T2{0, 0}, b = T2{0, 0};
      if (a30 + w < g.n3) {
        const long long off = (long long)k * n23 + colbase + w;
        a = X[((long long)(L * 6 + 2 * q)) * g.spec + off];
        b = X[((long long)(L * 6 + 2 * q + 1)) * g.spec + off];
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
    fft_lines<T, +1, LSH_MAXE>(Z, pl, W3, 1, W3, true, tw);
  }

  if (MODE == MODE_STRESS) {
    const double* e0 = eps0 + 6 * L;
    const T ep[6] = {(T)e0[0], (T)e0[1], (T)e0[2], (T)e0[3], (T)e0[4], (T)e0[5]};
    for (int idx = tid; idx < n1 * W; idx += nthr) {
      const int w = idx % W, a1 = idx / W;
      if (a30 + w >= g.n3) continue;
      T2* z = Z + a1 * W3 + w;
      const T2 z0 = z[0], z1 = z[W], z2 = z[2 * W];
      const T E[6] = {z0.x + ep[0], z0.y + ep[1], z1.x + ep[2], z1.y + ep[3], z2.x + ep[4], z2.y + ep[5]};
      const int p = phase[(long long)a1 * n23 + colbase + w];
      const T* D = dmat + 36 * p;
      T t[6];
#pragma unroll
      for (int I = 0; I < 6; ++I) {
        T s = 0;
#pragma unroll
        for (int J = 0; J < 6; ++J) s += D[6 * I + J] * E[J];
        t[I] = s;
      }
      z[0] = T2{t[0], t[1]};
      z[W] = T2{t[2], t[3]};
      z[2 * W] = T2{t[4], t[5]};
    }
  } else if (MODE == MODE_INIT) {
    const double SQ2I = 0.70710678118654752440;
    for (int idx = tid; idx < n1 * W; idx += nthr) {
      const int w = idx % W, a1 = idx / W;
      double E[6] = {0, 0, 0, 0, 0, 0};
      if (a30 + w < g.n3) {
        const long long pt = (long long)a1 * n23 + colbase + w;
        for (int c = 0; c < 6; ++c) {
          const double v = Einit[((long long)(L * 6 + c)) * g.m + pt] * (c < 3 ? 1.0 : SQ2I);
          // the solver keeps E(k1,a2,a3) = D1[E] / n1 (D1: unnormalised DFT along axis 1)
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
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int idx = tid; idx < n1 * W; idx += nthr) {
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
      if (Eout)
        for (int c = 0; c < 6; ++c) Eout[((long long)(L * 6 + c)) * g.m + pt] = E[c] * (c < 3 ? 1.0 : SQ2);
    }
    block_sum<6>(acc, partial + ((long long)L * gridDim.x + blockIdx.x) * 6);
    return;
  }

  __syncthreads();
  fft_lines<T, -1, LSH_MAXE>(Z, pl, W3, 1, W3, true, tw);

  // unpack the pairs and store the half spectrum k < h1
  for (int idx = tid; idx < h1 * W3; idx += nthr) {
    const int w = idx % W, q = (idx / W) % 3, k = idx / W3;
    if (a30 + w >= g.n3) continue;
    const int col = q * W + w;
    const T2 zk = Z[k * W3 + col];
    const T2 zn = Z[((n1 - k) % n1) * W3 + col];
    const T hf = (T)0.5;
    const T2 xa = T2{hf * (zk.x + zn.x), hf * (zk.y - zn.y)};
    const T2 xb = T2{hf * (zk.y + zn.y), hf * (zn.x - zk.x)};
    const long long off = (long long)k * n23 + colbase + w;
    Y[((long long)(L * 6 + 2 * q)) * g.spec + off] = xa;
    Y[((long long)(L * 6 + 2 * q + 1)) * g.spec + off] = xb;
  }
}

// ----------------------------------------------------------------- axis 2 ---
// One block: W consecutive i3 columns at fixed (load, comp, k1); lines along
// axis 2, LDS element-major lds[i2*W + w].
template <typename T, int DIR>
__global__ void __launch_bounds__(512) k_axis2(Geo g, FftPlan pl, const C2<T>* __restrict__ tw,
                                               const C2<T>* __restrict__ src, C2<T>* __restrict__ dst,
                                               const int* __restrict__ stop_iter, int it, int W, T scale) {
  using T2 = C2<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* Z = reinterpret_cast<T2*>(smem_raw);
  const int L = blockIdx.z, c = blockIdx.y;
  if (stop_iter && it >= stop_iter[L]) return;
  const int ntile3 = (g.n3 + W - 1) / W;
  const int k1 = blockIdx.x / ntile3;
  const int a30 = (blockIdx.x % ntile3) * W;
  const long long base = ((long long)(L * 6 + c)) * g.spec + (long long)k1 * g.n2 * g.n3 + a30;
  const int n2 = g.n2, tid = threadIdx.x, nthr = blockDim.x;
  for (int idx = tid; idx < n2 * W; idx += nthr) {
    const int w = idx % W, e = idx / W;
    Z[idx] = (a30 + w < g.n3) ? src[base + (long long)e * g.n3 + w] : T2{0, 0};
  }
  __syncthreads();
  fft_lines<T, DIR, LSH_MAXE>(Z, pl, W, 1, W, true, tw);
  for (int idx = tid; idx < n2 * W; idx += nthr) {
    const int w = idx % W, e = idx / W;
    if (a30 + w < g.n3) {
      T2 v = Z[idx];
      if (scale != (T)1) v = T2{v.x * scale, v.y * scale};
      dst[base + (long long)e * g.n3 + w] = v;
    }
  }
}

// ------------------------------------------------------------ Green pass ---
// One block per (k1, k2): the six axis-3 lines of every load.  Gamma for the
// block's n3 bins is computed once (double, scaled by -1/m, cast to T) and
// reused for all loads when it fits in LDS.
template <typename T>
__global__ void __launch_bounds__(512) k_green(Geo g, FftPlan pl, const C2<T>* __restrict__ tw, GreenParams gp,
                                                const C2<T>* __restrict__ tau, const C2<T>* __restrict__ Pold,
                                                C2<T>* __restrict__ Pnew, const T* __restrict__ table,
                                                const int* __restrict__ stop_iter, int it, int nload,
                                                double* __restrict__ partial, int ls, int cacheG) {
  using T2 = C2<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* lines = reinterpret_cast<T2*>(smem_raw);
  T* Gs = reinterpret_cast<T*>(smem_raw + sizeof(T2) * 6 * ls);
  const int n3 = g.n3, tid = threadIdx.x, nthr = blockDim.x;
  const int k1 = blockIdx.x / g.n2, k2 = blockIdx.x % g.n2;
  const double scale = -1.0 / (double)g.m;
  const double wk1 = (k1 == 0 || 2 * k1 == g.n1) ? 1.0 : 2.0;
  const long long row = (long long)k1 * g.n2 * g.n3 + (long long)k2 * g.n3;
  bool any = false;
  for (int L = 0; L < nload; ++L) any = any || (it < stop_iter[L]);
  if (!any) return;
  if (cacheG) {
    for (int k3 = tid; k3 < n3; k3 += nthr) {
      double G[21];
      if (table) {
        const T* tb = table + (row + k3) * 21;
        for (int t = 0; t < 21; ++t) G[t] = (double)tb[t];
      } else {
        gamma_sym_at(gp, k1, k2, k3, G);
      }
      for (int t = 0; t < 21; ++t) Gs[k3 * 21 + t] = (T)(scale * G[t]);
    }
  }
  for (int L = 0; L < nload; ++L) {
    if (it >= stop_iter[L]) continue;
    __syncthreads();
    for (int idx = tid; idx < 6 * n3; idx += nthr) {
      const int c = idx / n3, k3 = idx - c * n3;
      lines[c * ls + k3] = tau[((long long)(L * 6 + c)) * g.spec + row + k3];
    }
    __syncthreads();
    fft_lines<T, -1, LSH_MAXE>(lines, pl, 6, ls, 1, false, tw);
    for (int k3 = tid; k3 < n3; k3 += nthr) {
      T G[21];
      if (cacheG) {
        for (int t = 0; t < 21; ++t) G[t] = Gs[k3 * 21 + t];
      } else {
        double Gd[21];
        if (table) {
          const T* tb = table + (row + k3) * 21;
          for (int t = 0; t < 21; ++t) Gd[t] = (double)tb[t];
        } else {
          gamma_sym_at(gp, k1, k2, k3, Gd);
        }
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
    __syncthreads();
    fft_lines<T, +1, LSH_MAXE>(lines, pl, 6, ls, 1, false, tw);
    double acc[2] = {0.0, 0.0};
    for (int idx = tid; idx < 6 * n3; idx += nthr) {
      const int c = idx / n3, k3 = idx - c * n3;
      const long long gi = ((long long)(L * 6 + c)) * g.spec + row + k3;
      const T2 nv = lines[c * ls + k3];
      const T2 ov = Pold[gi];
      Pnew[gi] = nv;
      const double dx = (double)nv.x - (double)ov.x, dy = (double)nv.y - (double)ov.y;
      acc[0] += wk1 * (dx * dx + dy * dy);
      acc[1] += wk1 * ((double)nv.x * (double)nv.x + (double)nv.y * (double)nv.y);
    }
    block_sum<2>(acc, partial + ((long long)L * gridDim.x + blockIdx.x) * 2);
  }
}

// ------------------------------------------------------------ finalisers ---
__global__ void k_finalize_resid(const double* __restrict__ partial, int nblk, int nload,
                                 const double* __restrict__ e0sq, double pscale, double tol, int fixed, int it,
                                 int* __restrict__ stop_iter, double* __restrict__ hist, int* __restrict__ nonfinite) {
  const int L = blockIdx.x;
  if (it >= stop_iter[L]) return;
  double s[2] = {0.0, 0.0};
  for (int j = threadIdx.x; j < nblk; j += blockDim.x) {
    s[0] += partial[((long long)L * nblk + j) * 2];
    s[1] += partial[((long long)L * nblk + j) * 2 + 1];
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

__global__ void k_finalize_sum(const double* __restrict__ partial, int nblk, int nv, double scale,
                               double* __restrict__ out) {
  // out[L*nv + i] = scale * sum_j partial[(L*nblk + j)*nv + i]; one block per (L, i)
  const int L = blockIdx.x, i = blockIdx.y;
  double s[1] = {0.0};
  for (int j = threadIdx.x; j < nblk; j += blockDim.x) s[0] += partial[((long long)L * nblk + j) * nv + i];
  double o[1];
  block_sum<1>(s, o);
  if (threadIdx.x == 0) out[L * nv + i] = scale * o[0];
}

// mean of the Mandel components of a start field, per (load, comp) block
__global__ void k_mean(const double* __restrict__ E, long long m, double* __restrict__ means) {
  const int L = blockIdx.x, c = blockIdx.y;
  const double f = c < 3 ? 1.0 : 0.70710678118654752440;
  double s[1] = {0.0};
  for (long long i = threadIdx.x; i < m; i += blockDim.x) s[0] += E[((long long)(L * 6 + c)) * m + i];
  double o[1];
  block_sum<1>(s, o);
  if (threadIdx.x == 0) means[6 * L + c] = f * o[0] / (double)m;
}

// ---------------------------------------------------------- Gamma table ---
// One thread per half-spectrum bin; double alias sums, stored at T.
template <typename T>
__global__ void k_gamma_table(Geo g, GreenParams gp, T* __restrict__ table, double* __restrict__ minden) {
  const long long nb = g.spec;
  double mn[1] = {1e300};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (long long)gridDim.x * blockDim.x) {
    const int k3 = (int)(i % g.n3);
    const int k2 = (int)((i / g.n3) % g.n2);
    const int k1 = (int)(i / ((long long)g.n2 * g.n3));
    double G[21];
    const double den = gamma_sym_at(gp, k1, k2, k3, G);
    mn[0] = fmin(mn[0], den);
    for (int t = 0; t < 21; ++t) table[i * 21 + t] = (T)G[t];
  }
  // block min via the sum helper on negated values is not a min; do it by hand
  __shared__ double red[16];
  double v = mn[0];
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < (int)((blockDim.x + 63) >> 6); ++w) r = fmin(r, red[w]);
    minden[blockIdx.x] = r;
  }
}

__global__ void k_gamma_probe(GreenParams gp, const long long* __restrict__ bins, int n,
                              const double* __restrict__ table, int use_table, Geo g, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double G[21];
  if (use_table) {
    const long long row = (bins[3 * i] * g.n2 + bins[3 * i + 1]) * g.n3 + bins[3 * i + 2];
    for (int t = 0; t < 21; ++t) G[t] = table[row * 21 + t];
  } else {
    gamma_sym_at(gp, bins[3 * i], bins[3 * i + 1], bins[3 * i + 2], G);
  }
  for (int t = 0; t < 21; ++t) out[21 * i + t] = G[t];
}

template <typename T>
__global__ void k_cast_table(const T* __restrict__ src, double* __restrict__ dst, const long long* __restrict__ bins,
                             int n, Geo g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long row = (bins[3 * i] * g.n2 + bins[3 * i + 1]) * g.n3 + bins[3 * i + 2];
  for (int t = 0; t < 21; ++t) dst[21 * i + t] = (double)src[row * 21 + t];
}

// ------------------------------------------------------------ host side ---
#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t err_ = (x);                                                                 \
    if (err_ != hipSuccess)                                                                \
      return lsh_fail(LSH_EDEVICE, std::string("HIP error: ") + hipGetErrorString(err_) + \
                                       " at " #x);                                        \
  } while (0)

Geo geo_of(const lsh_pattern* p) {
  Geo g;
  g.n1 = (int)p->e[0];
  g.n2 = (int)p->e[1];
  g.n3 = (int)p->e[2];
  g.h1 = g.n1 / 2 + 1;
  g.m = p->m;
  g.spec = (long long)g.h1 * g.n2 * g.n3;
  return g;
}

// Does an FFT of this plan over L lines fit nthr threads x LSH_MAXE registers?
bool plan_fits(const FftPlan& pl, int L, int nthr) {
  for (int s = 0; s < pl.nst; ++s) {
    const int R = pl.rad[s];
    const int maxb = std::max(1, LSH_MAXE / R);
    const long long nb = (long long)(pl.N / R) * L;
    if (nb > (long long)nthr * maxb) return false;
  }
  return true;
}

struct Launch {
  int W, nthr;
  size_t lds;
};

template <typename T>
bool choose_axis1(const Geo& g, const FftPlan& pl, Launch* out) {
  const int targets[] = {16, 8, 4, 2, 1};
  for (int W : targets) {
    if (W > 1 && W > g.n3) continue;
    for (int nthr : {256, 512}) {
      const size_t lds = sizeof(C2<T>) * (size_t)g.n1 * 3 * W;
      if (lds > 64 * 1024) continue;
      if (!plan_fits(pl, 3 * W, nthr)) continue;
      out->W = W;
      out->nthr = nthr;
      out->lds = lds;
      return true;
    }
  }
  return false;
}

template <typename T>
bool choose_axis2(const Geo& g, const FftPlan& pl, Launch* out) {
  const int targets[] = {32, 16, 8, 4, 2, 1};
  for (int W : targets) {
    if (W > 1 && W > g.n3) continue;
    if (sizeof(T) == 8 && W > 16) continue;
    for (int nthr : {256, 512}) {
      const size_t lds = sizeof(C2<T>) * (size_t)g.n2 * W;
      if (lds > 64 * 1024) continue;
      if (!plan_fits(pl, W, nthr)) continue;
      out->W = W;
      out->nthr = nthr;
      out->lds = lds;
      return true;
    }
  }
  return false;
}

template <typename T>
bool choose_green(const Geo& g, const FftPlan& pl, Launch* out, int* ls, int* cacheG) {
  *ls = g.n3 + ((g.n3 % 2 == 0) ? 1 : 0);
  for (int nthr = 64; nthr <= 512; nthr *= 2) {
    if (!plan_fits(pl, 6, nthr)) continue;
    if (nthr < std::min(512, g.n3)) continue;  // about one bin per thread
    size_t lds = sizeof(C2<T>) * 6 * (size_t)(*ls);
    const size_t gbytes = sizeof(T) * 21 * (size_t)g.n3;
    *cacheG = (lds + gbytes <= 64 * 1024) ? 1 : 0;
    if (*cacheG) lds += gbytes;
    if (lds > 64 * 1024) return false;
    out->W = 1;
    out->nthr = nthr;
    out->lds = lds;
    return true;
  }
  return false;
}

struct Plans {
  Launch a1, a2, gr;
  int ls, cacheG;
};

template <typename T>
int make_plans(const lsh_pattern* p, Plans* P) {
  const Geo g = geo_of(p);
  for (int i = 0; i < 3; ++i)
    if (p->plan[i].nst < 0)
      return lsh_fail(LSH_EUNSUPPORTED, "SNF factor e" + std::to_string(i + 1) + " = " + std::to_string(p->e[i]) +
                                            " has a prime factor above 13");
  if (!choose_axis1<T>(g, p->plan[0], &P->a1)) return lsh_fail(LSH_EUNSUPPORTED, "SNF factor e1 too large for one block");
  if (!choose_axis2<T>(g, p->plan[1], &P->a2)) return lsh_fail(LSH_EUNSUPPORTED, "SNF factor e2 too large for one block");
  if (!choose_green<T>(g, p->plan[2], &P->gr, &P->ls, &P->cacheG))
    return lsh_fail(LSH_EUNSUPPORTED, "SNF factor e3 too large for one block");
  return LSH_OK;
}

template <typename T>
void host_twiddles(int N, std::vector<C2<T>>* tw) {
  tw->resize(std::max(N, 1));
  for (int k = 0; k < N; ++k) {
    const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)k / (long double)N;
    (*tw)[k] = C2<T>{(T)cosl(a), (T)sinl(a)};
  }
}

size_t persistent_bytes_t(const lsh_pattern* p, size_t scal) {
  const Geo g = geo_of(p);
  size_t b = lsh_align((size_t)p->m);
  for (int i = 0; i < 3; ++i) b += lsh_align(2 * scal * (size_t)std::max<int64_t>(p->e[i], 1));
  b += lsh_align(scal * 36 * 256) + lsh_align(sizeof(double) * 36 * 256);
  b += lsh_align(sizeof(double) * 4096);  // per-block minima of the bracket sums
  if (p->kind == LSH_BOXSPLINE) b += lsh_align(scal * 21 * (size_t)g.spec);
  return b;
}

struct Profile {
  bool on = false;
  double ms[8] = {0};
  long long n[8] = {0};
};
Profile g_prof;

template <typename T>
int bind_t(lsh_pattern* p, void* dev, size_t bytes, hipStream_t st) {
  Plans P;
  int rc = make_plans<T>(p, &P);
  if (rc) return rc;
  const size_t need = persistent_bytes_t(p, sizeof(T));
  if (!dev || bytes < need) return lsh_fail(LSH_EWORKSPACE, "persistent buffer too small: need " + std::to_string(need));
  char* base = (char*)dev;
  size_t off = 0;
  p->off_phase = off;
  off += lsh_align((size_t)p->m);
  HIPCHK(hipMemcpyAsync(base + p->off_phase, p->phase.data(), (size_t)p->m, hipMemcpyHostToDevice, st));
  for (int i = 0; i < 3; ++i) {
    std::vector<C2<T>> tw;
    host_twiddles<T>((int)p->e[i], &tw);
    p->off_tw[i] = off;
    off += lsh_align(2 * sizeof(T) * (size_t)std::max<int64_t>(p->e[i], 1));
    HIPCHK(hipMemcpyAsync(base + p->off_tw[i], tw.data(), sizeof(C2<T>) * tw.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  // (C_p - C0) in T and C_p in double, Mandel
  std::vector<T> dm(36 * (size_t)p->nphase);
  std::vector<double> cm(36 * (size_t)p->nphase);
  double C0m[36];
  lsh_voigt_to_mandel(p->C0_voigt, C0m);
  for (int q = 0; q < p->nphase; ++q) {
    double Cm[36];
    lsh_voigt_to_mandel(p->C_voigt.data() + 36 * q, Cm);
    for (int i = 0; i < 36; ++i) {
      dm[36 * q + i] = (T)(Cm[i] - C0m[i]);
      cm[36 * q + i] = Cm[i];
    }
  }
  p->off_dmat = off;
  off += lsh_align(sizeof(T) * 36 * 256);
  p->off_cmat = off;
  off += lsh_align(sizeof(double) * 36 * 256);
  HIPCHK(hipMemcpyAsync(base + p->off_dmat, dm.data(), sizeof(T) * dm.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(base + p->off_cmat, cm.data(), sizeof(double) * cm.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  double* mins_dev = (double*)(base + off);
  off += lsh_align(sizeof(double) * 4096);
  p->has_table = false;
  if (p->kind == LSH_BOXSPLINE) {
    const Geo g = geo_of(p);
    p->off_table = off;
    off += lsh_align(sizeof(T) * 21 * (size_t)g.spec);
    GreenParams gp;
    lsh_green_params(p, &gp);
    const int nthr = 256;
    const int nblk = (int)std::min<long long>((g.spec + nthr - 1) / nthr, 4096);
    T* table = (T*)(base + p->off_table);
    hipLaunchKernelGGL(k_gamma_table<T>, dim3(nblk), dim3(nthr), 0, st, g, gp, table, mins_dev);
    HIPCHK(hipGetLastError());
    std::vector<double> mins(nblk);
    HIPCHK(hipMemcpyAsync(mins.data(), mins_dev, sizeof(double) * nblk, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double mn = 1e300;
    for (int i = 0; i < nblk; ++i) mn = std::min(mn, mins[i]);
    if (!(mn > 0.0))
      return lsh_fail(LSH_ENOINTERP, "a bracket sum of |c_k(f)|^2 vanishes: translates are not linearly independent");
    p->has_table = true;
  }
  p->dev_persist = base;
  p->bound_prec = sizeof(T) == 8 ? LSH_FP64 : LSH_FP32_MIXED;
  return LSH_OK;
}

struct WS {
  char* X;
  char* TAU;
  char* P[2];
  double* partial;
  double* eps0;
  double* e0sq;
  double* hist;
  double* sigma;
  double* means;
  int* stop_iter;
  int* nonfinite;
  size_t total;
};

template <typename T>
WS ws_layout(const lsh_pattern* p, int nload, const Plans& P, char* base) {
  const Geo g = geo_of(p);
  const size_t fb = lsh_align(sizeof(C2<T>) * 6 * (size_t)nload * g.spec);
  WS w;
  size_t off = 0;
  w.X = base + off; off += fb;
  w.TAU = base + off; off += fb;
  w.P[0] = base + off; off += fb;
  w.P[1] = base + off; off += fb;
  const long long nblkS = (long long)g.n2 * ((g.n3 + P.a1.W - 1) / P.a1.W);
  const long long nblkG = (long long)g.h1 * g.n2;
  const long long npart = std::max(nblkS * 6, nblkG * 2) * nload;
  w.partial = (double*)(base + off); off += lsh_align(sizeof(double) * npart);
  w.eps0 = (double*)(base + off); off += lsh_align(sizeof(double) * 6 * nload);
  w.e0sq = (double*)(base + off); off += lsh_align(sizeof(double) * nload);
  w.hist = (double*)(base + off); off += lsh_align(sizeof(double) * LSH_HIST * nload);
  w.sigma = (double*)(base + off); off += lsh_align(sizeof(double) * 6 * nload);
  w.means = (double*)(base + off); off += lsh_align(sizeof(double) * 6 * nload);
  w.stop_iter = (int*)(base + off); off += lsh_align(sizeof(int) * nload);
  w.nonfinite = (int*)(base + off); off += lsh_align(sizeof(int) * nload);
  w.total = off;
  return w;
}

// Per-kernel GPU time from event pairs recorded on the launch stream; read
// back only at the host's existing synchronisation points.
struct EvPool {
  struct Pend {
    int slot;
    hipEvent_t a, b;
  };
  std::vector<Pend> pending;
  std::vector<hipEvent_t> free_;
  hipEvent_t get() {
    if (free_.empty()) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      return e;
    }
    hipEvent_t e = free_.back();
    free_.pop_back();
    return e;
  }
  void flush() {  // call after the stream is synchronised
    for (auto& q : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
        g_prof.ms[q.slot] += ms;
        g_prof.n[q.slot] += 1;
      }
      free_.push_back(q.a);
      free_.push_back(q.b);
    }
    pending.clear();
  }
};
EvPool g_ev;

struct Timer {
  hipEvent_t a{}, b{};
  int slot;
  hipStream_t st;
  Timer(int s, hipStream_t stream) : slot(s), st(stream) {
    if (g_prof.on) {
      a = g_ev.get();
      b = g_ev.get();
      (void)hipEventRecord(a, st);
    }
  }
  ~Timer() {
    if (g_prof.on) {
      (void)hipEventRecord(b, st);
      g_ev.pending.push_back({slot, a, b});
    }
  }
};

template <typename T>
int solve_t(lsh_pattern* p, int nload, const double* eps0_voigt, double tol, int max_iter, void* dev_ws,
            size_t ws_bytes, hipStream_t st, const double* dev_E_init, double* dev_E_out, double* sigma_out,
            lsh_stats* stats, double* history) {
  using T2 = C2<T>;
  Plans P;
  int rc = make_plans<T>(p, &P);
  if (rc) return rc;
  const Geo g = geo_of(p);
  WS w = ws_layout<T>(p, nload, P, (char*)dev_ws);
  if (!dev_ws || ws_bytes < w.total) return lsh_fail(LSH_EWORKSPACE, "workspace too small: need " + std::to_string(w.total));
  GreenParams gp;
  lsh_green_params(p, &gp);
  char* base = p->dev_persist;
  const uint8_t* phase = (const uint8_t*)(base + p->off_phase);
  const T2* tw[3] = {(const T2*)(base + p->off_tw[0]), (const T2*)(base + p->off_tw[1]),
                     (const T2*)(base + p->off_tw[2])};
  const T* dmat = (const T*)(base + p->off_dmat);
  const double* cmat = (const double*)(base + p->off_cmat);
  const T* table = p->has_table ? (const T*)(base + p->off_table) : nullptr;

  // host-side setup: eps0 in Mandel, m |eps0|^2
  std::vector<double> e0(6 * nload), e0sq(nload);
  for (int L = 0; L < nload; ++L) {
    double s = 0.0;
    for (int c = 0; c < 6; ++c) {
      const double v = eps0_voigt[6 * L + c] * (c < 3 ? 1.0 : M_SQRT1_2);
      e0[6 * L + c] = v;
      s += v * v;
    }
    e0sq[L] = s * (double)p->m;
  }
  const bool fixed = tol < 0.0;
  std::vector<int> stop(nload, max_iter), nonfin(nload, 0);
  HIPCHK(hipMemcpyAsync(w.eps0, e0.data(), sizeof(double) * 6 * nload, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w.e0sq, e0sq.data(), sizeof(double) * nload, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w.stop_iter, stop.data(), sizeof(int) * nload, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w.nonfinite, nonfin.data(), sizeof(int) * nload, hipMemcpyHostToDevice, st));
  const size_t fb = sizeof(T2) * 6 * (size_t)nload * g.spec;

  const int nt3a = (g.n3 + P.a1.W - 1) / P.a1.W;
  const dim3 gridS(g.n2 * nt3a, nload);
  const int nt3b = (g.n3 + P.a2.W - 1) / P.a2.W;
  const dim3 gridB(g.h1 * nt3b, 6, nload);
  const dim3 gridG(g.h1 * g.n2);
  const int nblkS = g.n2 * nt3a;
  const int nblkG = g.h1 * g.n2;

  int cur = 0;  // P[cur] holds the previous E(k1,k2,a3)
  if (dev_E_init) {
    hipLaunchKernelGGL(k_mean, dim3(nload, 6), dim3(1024), 0, st, dev_E_init, (long long)g.m, w.means);
    hipLaunchKernelGGL((k_axis1<T, MODE_INIT>), gridS, dim3(P.a1.nthr), P.a1.lds, st, g, p->plan[0], tw[0],
                       (const T2*)nullptr, (T2*)w.X, phase, dmat, cmat, w.eps0, w.stop_iter, 0, dev_E_init, w.means,
                       (double*)nullptr, (double*)nullptr, P.a1.W);
    hipLaunchKernelGGL((k_axis2<T, -1>), gridB, dim3(P.a2.nthr), P.a2.lds, st, g, p->plan[1], tw[1],
                       (const T2*)w.X, (T2*)w.P[cur], (const int*)nullptr, 0, P.a2.W, (T)(1.0 / g.n2));
    HIPCHK(hipGetLastError());
  } else {
    HIPCHK(hipMemsetAsync(w.X, 0, fb, st));
    HIPCHK(hipMemsetAsync(w.P[cur], 0, fb, st));
  }

  // P(k1,k2,a3) = D12[E] / (n1 n2) (D12: unnormalised DFT over axes 1, 2), so by
  // Parseval sum_y |E|^2 = n1 n2 sum_{k1,k2,a3} w_k1 |P|^2 (w: half-spectrum weight)
  const double pscale = (double)g.n1 * (double)g.n2;
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<double> ring(LSH_HIST * nload);
  if (history)
    for (long long i = 0; i < (long long)nload * max_iter; ++i) history[i] = NAN;
  int it = 0;
  int done_iters = 0;
  const int check = fixed ? LSH_HIST : 8;
  for (it = 0; it < max_iter; ++it) {
    {
      Timer tm(0, st);
      hipLaunchKernelGGL((k_axis1<T, MODE_STRESS>), gridS, dim3(P.a1.nthr), P.a1.lds, st, g, p->plan[0], tw[0],
                         (const T2*)w.X, (T2*)w.TAU, phase, dmat, cmat, w.eps0, w.stop_iter, it,
                         (const double*)nullptr, (const double*)nullptr, (double*)nullptr, (double*)nullptr, P.a1.W);
    }
    {
      Timer tm(1, st);
      hipLaunchKernelGGL((k_axis2<T, -1>), gridB, dim3(P.a2.nthr), P.a2.lds, st, g, p->plan[1], tw[1],
                         (const T2*)w.TAU, (T2*)w.TAU, w.stop_iter, it, P.a2.W, (T)1);
    }
    {
      Timer tm(2, st);
      hipLaunchKernelGGL((k_green<T>), gridG, dim3(P.gr.nthr), P.gr.lds, st, g, p->plan[2], tw[2], gp,
                         (const T2*)w.TAU, (const T2*)w.P[cur], (T2*)w.P[1 - cur], table, w.stop_iter, it, nload,
                         w.partial, P.ls, P.cacheG);
    }
    {
      Timer tm(3, st);
      hipLaunchKernelGGL(k_finalize_resid, dim3(nload), dim3(256), 0, st, w.partial, nblkG, nload, w.e0sq, pscale, tol,
                         fixed ? 1 : 0, it, w.stop_iter, w.hist, w.nonfinite);
    }
    {
      Timer tm(4, st);
      hipLaunchKernelGGL((k_axis2<T, +1>), gridB, dim3(P.a2.nthr), P.a2.lds, st, g, p->plan[1], tw[1],
                         (const T2*)w.P[1 - cur], (T2*)w.X, w.stop_iter, it, P.a2.W, (T)1);
    }
    HIPCHK(hipGetLastError());
    cur = 1 - cur;
    done_iters = it + 1;
    if ((it + 1) % check == 0 || it + 1 == max_iter || (it + 1) % LSH_HIST == 0) {
      HIPCHK(hipMemcpyAsync(ring.data(), w.hist, sizeof(double) * LSH_HIST * nload, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(stop.data(), w.stop_iter, sizeof(int) * nload, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (g_prof.on) g_ev.flush();
      // copy the ring entries of iterations (it+1-k .. it] that are not yet copied
      const int first = std::max(0, it + 1 - LSH_HIST);
      if (history)
        for (int j = first; j <= it; ++j)
          for (int L = 0; L < nload; ++L)
            if (j < stop[L]) history[(long long)L * max_iter + j] = ring[(j % LSH_HIST) * nload + L];
      bool all = true;
      for (int L = 0; L < nload; ++L) all = all && stop[L] <= it + 1;
      if (all) break;
    }
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  HIPCHK(hipMemcpyAsync(ring.data(), w.hist, sizeof(double) * LSH_HIST * nload, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(stop.data(), w.stop_iter, sizeof(int) * nload, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(nonfin.data(), w.nonfinite, sizeof(int) * nload, hipMemcpyDeviceToHost, st));

  // final pass: sigma_bar at the last iterate, optional E out
  {
    Timer tm(5, st);
    hipLaunchKernelGGL((k_axis1<T, MODE_FINAL>), gridS, dim3(P.a1.nthr), P.a1.lds, st, g, p->plan[0], tw[0],
                       (const T2*)w.X, (T2*)nullptr, phase, dmat, cmat, w.eps0, w.stop_iter, 0,
                       (const double*)nullptr, (const double*)nullptr, dev_E_out, w.partial, P.a1.W);
    hipLaunchKernelGGL(k_finalize_sum, dim3(nload, 6), dim3(256), 0, st, w.partial, nblkS, 6, 1.0 / (double)g.m,
                       w.sigma);
  }
  HIPCHK(hipGetLastError());
  std::vector<double> sig(6 * nload);
  HIPCHK(hipMemcpyAsync(sig.data(), w.sigma, sizeof(double) * 6 * nload, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (g_prof.on) g_ev.flush();
  int status = LSH_OK;
  for (int L = 0; L < nload; ++L) {
    for (int c = 0; c < 6; ++c) sigma_out[6 * L + c] = sig[6 * L + c] * (c < 3 ? 1.0 : M_SQRT1_2);
    const int its = std::min(stop[L], done_iters);
    double last = NAN;
    if (its > 0) last = ring[((its - 1) % LSH_HIST) * nload + L];
    if (history)
      for (int j = std::max(0, its - LSH_HIST); j < its; ++j)
        history[(long long)L * max_iter + j] = ring[(j % LSH_HIST) * nload + L];
    const bool conv = !fixed && std::isfinite(last) && last <= tol;
    if (stats) {
      stats[L].iterations = its;
      stats[L].converged = conv ? 1 : 0;
      stats[L].residual = last;
      stats[L].seconds = secs;
    }
    if (nonfin[L]) status = LSH_ENONFINITE;
    else if (!fixed && !conv && status == LSH_OK) status = LSH_ENOTCONVERGED;
  }
  if (status == LSH_ENONFINITE) return lsh_fail(status, "non-finite residual (NaN/Inf) in the iteration");
  if (status == LSH_ENOTCONVERGED) return lsh_fail(status, "max_iter reached before the Cauchy residual met tol");
  return LSH_OK;
}

template <typename T>
int probe_t(const lsh_pattern* p, const int64_t* bins, int n, double* out, void* scratch, size_t sbytes, hipStream_t st) {
  const Geo g = geo_of(p);
  const size_t need = lsh_align(sizeof(long long) * 3 * n) + lsh_align(sizeof(double) * 21 * n);
  if (!scratch || sbytes < need) return lsh_fail(LSH_EWORKSPACE, "probe scratch too small: need " + std::to_string(need));
  for (int i = 0; i < n; ++i) {
    if (bins[3 * i] < 0 || bins[3 * i] >= g.h1 || bins[3 * i + 1] < 0 || bins[3 * i + 1] >= g.n2 ||
        bins[3 * i + 2] < 0 || bins[3 * i + 2] >= g.n3)
      return lsh_fail(LSH_EINVAL, "probe bin out of range");
  }
  long long* dbins = (long long*)scratch;
  double* dout = (double*)((char*)scratch + lsh_align(sizeof(long long) * 3 * n));
  HIPCHK(hipMemcpyAsync(dbins, bins, sizeof(long long) * 3 * n, hipMemcpyHostToDevice, st));
  GreenParams gp;
  lsh_green_params(p, &gp);
  if (p->has_table) {
    const T* table = (const T*)(p->dev_persist + p->off_table);
    hipLaunchKernelGGL((k_cast_table<T>), dim3((n + 127) / 128), dim3(128), 0, st, table, dout, dbins, n, g);
  } else {
    hipLaunchKernelGGL(k_gamma_probe, dim3((n + 127) / 128), dim3(128), 0, st, gp, dbins, n, (const double*)nullptr,
                       0, g, dout);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(out, dout, sizeof(double) * 21 * n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return LSH_OK;
}

}  // namespace

// ================================================================ the ABI ===
extern "C" int lsh_persistent_bytes(const lsh_pattern* p, lsh_precision prec, size_t* bytes) {
  if (!p || !bytes) return lsh_fail(LSH_EINVAL, "null argument");
  if (p->kind < 0) return lsh_fail(LSH_ESTATE, "lsh_set_kernel has not been called");
  if (prec != LSH_FP64 && prec != LSH_FP32_MIXED) return lsh_fail(LSH_EINVAL, "bad precision");
  *bytes = persistent_bytes_t(p, prec == LSH_FP64 ? 8 : 4);
  return LSH_OK;
}

extern "C" int lsh_bind(lsh_pattern* p, lsh_precision prec, void* dev, size_t bytes, void* stream) {
  if (!p) return lsh_fail(LSH_EINVAL, "null pattern");
  if (p->kind < 0) return lsh_fail(LSH_ESTATE, "lsh_set_kernel has not been called");
  if (p->nphase < 1) return lsh_fail(LSH_ESTATE, "lsh_set_stiffness has not been called");
  hipStream_t st = (hipStream_t)stream;
  if (prec == LSH_FP64) return bind_t<double>(p, dev, bytes, st);
  if (prec == LSH_FP32_MIXED) return bind_t<float>(p, dev, bytes, st);
  return lsh_fail(LSH_EINVAL, "bad precision");
}

extern "C" int lsh_gamma_probe(const lsh_pattern* p, lsh_precision prec, const int64_t* bins, int n, double* out,
                               void* scratch, size_t sbytes, void* stream) {
  if (!p || !bins || !out || n < 0) return lsh_fail(LSH_EINVAL, "bad argument");
  if (p->kind < 0) return lsh_fail(LSH_ESTATE, "lsh_set_kernel has not been called");
  if (p->bound_prec != (int)prec) return lsh_fail(LSH_ESTATE, "pattern not bound at this precision (lsh_bind)");
  if (n == 0) return LSH_OK;
  hipStream_t st = (hipStream_t)stream;
  return prec == LSH_FP64 ? probe_t<double>(p, bins, n, out, scratch, sbytes, st)
                          : probe_t<float>(p, bins, n, out, scratch, sbytes, st);
}

extern "C" int lsh_solve_bytes(const lsh_pattern* p, int nload, lsh_precision prec, size_t* bytes) {
  if (!p || !bytes) return lsh_fail(LSH_EINVAL, "null argument");
  if (nload < 1 || nload > 64) return lsh_fail(LSH_EINVAL, "nload must be in [1, 64]");
  if (prec == LSH_FP64) {
    Plans P;
    int rc = make_plans<double>(p, &P);
    if (rc) return rc;
    *bytes = ws_layout<double>(p, nload, P, nullptr).total;
  } else if (prec == LSH_FP32_MIXED) {
    Plans P;
    int rc = make_plans<float>(p, &P);
    if (rc) return rc;
    *bytes = ws_layout<float>(p, nload, P, nullptr).total;
  } else {
    return lsh_fail(LSH_EINVAL, "bad precision");
  }
  return LSH_OK;
}

extern "C" int lsh_solve(lsh_pattern* p, int nload, const double* eps0_voigt, double tol, int max_iter,
                         lsh_precision prec, void* dev_ws, size_t ws_bytes, void* stream, const double* dev_E_init,
                         double* dev_E_out, double* sigma_out, lsh_stats* stats, double* history) {
  if (!p || !eps0_voigt || !sigma_out) return lsh_fail(LSH_EINVAL, "null argument");
  if (nload < 1 || nload > 64) return lsh_fail(LSH_EINVAL, "nload must be in [1, 64]");
  if (max_iter < 1) return lsh_fail(LSH_EINVAL, "max_iter must be >= 1");
  if (!(tol == tol)) return lsh_fail(LSH_EINVAL, "tol is NaN");
  for (int i = 0; i < 6 * nload; ++i)
    if (!std::isfinite(eps0_voigt[i])) return lsh_fail(LSH_EINVAL, "non-finite macroscopic strain");
  if (p->kind < 0 || p->nphase < 1) return lsh_fail(LSH_ESTATE, "kernel or stiffness not set");
  if (p->bound_prec != (int)prec) return lsh_fail(LSH_ESTATE, "pattern not bound at this precision (lsh_bind)");
  hipStream_t st = (hipStream_t)stream;
  if (prec == LSH_FP64)
    return solve_t<double>(p, nload, eps0_voigt, tol, max_iter, dev_ws, ws_bytes, st, dev_E_init, dev_E_out,
                           sigma_out, stats, history);
  return solve_t<float>(p, nload, eps0_voigt, tol, max_iter, dev_ws, ws_bytes, st, dev_E_init, dev_E_out, sigma_out,
                        stats, history);
}

extern "C" int lsh_profile_enable(int on) {
  g_prof = Profile();
  g_prof.on = on != 0;
  return LSH_OK;
}

extern "C" int lsh_profile_read(double* ms, long long* counts, int n) {
  if (!ms || !counts || n < 0) return lsh_fail(LSH_EINVAL, "null argument");
  for (int i = 0; i < n && i < 8; ++i) {
    ms[i] = g_prof.ms[i];
    counts[i] = g_prof.n[i];
  }
  return LSH_OK;
}
