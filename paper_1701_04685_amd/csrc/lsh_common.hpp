// lsh_common.hpp -- device-side types and helpers shared by the solver's
// kernel sources: the SNF grid geometry, per-instance material data, block
// reductions, the stress mat-vec and the Green operator from alias moments.
// Everything here is a type, an inline function or a template, so the header
// may be included by more than one translation unit.
#pragma once
#include <hip/hip_runtime.h>

#include "lsh_fft.hpp"
#include "lsh_green.hpp"

#define LSH_HIST 64  // device ring of residuals per load

struct Geo {
  int n1, n2, n3, h1;
  long long m;
  long long spec;  // h1 * n2 * n3 complex values per component and load
  int ncf;         // components of the caller's real-space fields: 6, or 3 for d = 2
  int pad_;
};

// Where component c (internal order 11, 22, 33, 23, 13, 12) sits in a
// caller's field of ncf components: c itself for six, 11, 22, 12 -> 0, 1, 2
// for the three of a two-dimensional pattern, -1 for a component that such a
// field does not carry (it is zero there).
__host__ __device__ inline int boundary_comp(int c, int ncf) {
  return ncf == 6 ? c : (c < 2 ? c : (c == 5 ? 2 : -1));
}

template <typename T> using C2 = typename cpx<T>::t;

enum { MODE_STRESS = 0, MODE_FINAL = 1, MODE_INIT = 2 };

// One microstructure: its phase map and per-phase stiffness, and the isotropic
// reference constants used by the on-the-fly Green operator.  A solve holds
// one or many (batched) instances; load case L belongs to instance inst_of[L].
struct Inst {
  const uint8_t* phase;  // m phase indices, storage order
  const void* dmat;      // (C_p - C0) at the working precision, 36 per phase, Mandel
  const double* cmat;    // C_p in double, 36 per phase, Mandel
  int nphase;
  int pad_;
  double mu0;   // isotropic C0: shear modulus
  double riso;  // (lam0 + mu0) / (mu0 (lam0 + 2 mu0))
};

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

template <typename T>
__device__ __forceinline__ void stage_twiddles(C2<T>* dst, const C2<T>* __restrict__ src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// tau = D E for one point, D a 6x6 Mandel matrix (C_p - C0)
template <typename T>
__device__ __forceinline__ void stress6(const T* D, const T E[6], T t[6]) {
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    T s = 0;
#pragma unroll
    for (int J = 0; J < 6; ++J) s += D[6 * I + J] * E[J];
    t[I] = s;
  }
}

// Loads and stores of streamed fields (the state, the polarisation) with the
// nontemporal hint: the caches keep no line for them.  It pays where every
// line is read or written once per pass (the Green pass: 0.415 -> 0.361 ms at
// 128^3 FP64) and costs where the next pass would have found the lines in
// cache (the forward axis-2 pass's output) or where neighbouring blocks share
// partly used lines (the two-pass stress tiles' 32-byte runs); ld_st / st_st
// apply it when NT is set.
template <typename T2> struct natv2;
template <> struct natv2<float2> { typedef float __attribute__((ext_vector_type(2))) t; };
template <> struct natv2<double2> { typedef double __attribute__((ext_vector_type(2))) t; };
template <typename T2>
__device__ __forceinline__ T2 ld_nt(const T2* p) {
  using V = typename natv2<T2>::t;
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  return T2{v.x, v.y};
}
template <typename T2>
__device__ __forceinline__ void st_nt(T2* p, T2 v) {
  using V = typename natv2<T2>::t;
  V w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<V*>(p));
}

template <bool NT, typename T2>
__device__ __forceinline__ T2 ld_st(const T2* p) {
  if constexpr (NT) return ld_nt(p);
  else return *p;
}
template <bool NT, typename T2>
__device__ __forceinline__ void st_st(T2* p, T2 v) {
  if constexpr (NT) st_nt(p, v);
  else *p = v;
}

// How a Green pass turns its result v (its input transformed with
// -Gamma^p / m) into the new state, given the previous state ov:
//   UPD_LS   new = v (the input is the polarisation of the current iterate);
//   UPD_VE   new = ov + v (the variational scheme: v is the correction);
//   UPD_INC  iteration 0 as UPD_LS, with the increment v - ov written to dP;
//            later iterations take the polarisation's increment as input, so
//            new = ov + v and the increment is v itself.
// *d2 = |new - ov|^2 in double; for UPD_INC past iteration 0 it is |v|^2,
// taken from v rather than from the rounded difference of the states.
enum { UPD_LS = 0, UPD_VE = 1, UPD_INC = 2 };

template <typename T>
__device__ __forceinline__ C2<T> green_update(C2<T> v, C2<T> ov, int upd, int it, C2<T>* __restrict__ dP,
                                              long long gi, double* d2) {
  C2<T> nv;
  double dx, dy;
  if (upd == UPD_INC && it > 0) {
    nv = cadd(v, ov);
    dP[gi] = v;
    dx = (double)v.x;
    dy = (double)v.y;
  } else {
    nv = upd == UPD_VE ? cadd(v, ov) : v;
    if (upd == UPD_INC) dP[gi] = csub(v, ov);
    dx = (double)nv.x - (double)ov.x;
    dy = (double)nv.y - (double)ov.y;
  }
  *d2 = dx * dx + dy * dy;
  return nv;
}

// Green operator forms (see k_green in lsh_kernels.hpp).
enum { GREEN_ISO = 0, GREEN_GENERAL = 1, GREEN_TABLE = 2, GREEN_MOMENTS = 3 };

#define MOM_ROWS 15

// Gamma^p entry row t at bin (pos, k3) from a moments row set [pos][15][n3].
template <typename T, typename Out>
__device__ __forceinline__ void moments_emit(const T* __restrict__ table, long long pos, int n3, int k3, double mu0,
                                             double riso, Out&& out) {
  const T* tb = table + pos * MOM_ROWS * n3 + k3;
  double a[6], q[15];
#pragma unroll
  for (int t = 0; t < 15; ++t) q[t] = (double)tb[(long long)t * n3];
  // second moments, pairs (00,11,22,12,02,01): a_ij = sum_k q_ijkk, with q in
  // the order 0000 0001 0002 0011 0012 0022 0111 0112 0122 0222 1111 1112 1122
  // 1222 2222
  a[0] = q[0] + q[3] + q[5];
  a[1] = q[3] + q[10] + q[12];
  a[2] = q[5] + q[12] + q[14];
  a[3] = q[4] + q[11] + q[13];
  a[4] = q[2] + q[7] + q[9];
  a[5] = q[1] + q[6] + q[8];
  iso_emit(a, q, mu0, riso, out);
}
