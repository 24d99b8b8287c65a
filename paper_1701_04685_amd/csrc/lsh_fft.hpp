// lsh_fft.hpp -- line FFTs held in LDS, for the pattern DFT over the SNF grid.
//
// The pattern DFT of eq. (Fouriermatrix) (Sec. 2.1) is, in the SNF ordering, a
// 3-D DFT over Z_e1 x Z_e2 x Z_e3; the solver applies it one axis at a time to
// bundles of lines staged in LDS.  This file holds the building block: a
// self-sorting (Stockham) mixed-radix FFT over L lines of length N that sit in
// LDS at lds[l*ls + i*es].  Each stage reads every element into registers,
// synchronises, and writes the butterflies' outputs back in place, so one LDS
// buffer suffices.  Radices 2, 3, 4, 5, 7, 8 have hand-written butterflies;
// 11 and 13 use a direct DFT.  Twiddles come from a per-length table of
// exp(-2 pi i k / N), k < N, computed on the host in long double.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define LSH_MAX_STAGES 24

template <typename T> struct cpx;
template <> struct cpx<double> { using t = double2; };
template <> struct cpx<float> { using t = float2; };

template <typename T2> __device__ __forceinline__ T2 cadd(T2 a, T2 b) { return T2{a.x + b.x, a.y + b.y}; }
template <typename T2> __device__ __forceinline__ T2 csub(T2 a, T2 b) { return T2{a.x - b.x, a.y - b.y}; }
template <typename T2> __device__ __forceinline__ T2 cmul(T2 a, T2 b) {
  return T2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by -i (DIR = -1, forward) or +i (DIR = +1, inverse)
template <int DIR, typename T2> __device__ __forceinline__ T2 rot90(T2 a) {
  return DIR < 0 ? T2{a.y, -a.x} : T2{-a.y, a.x};
}

struct FftPlan {
  int N;                     // line length
  int nst;                   // number of stages
  int rad[LSH_MAX_STAGES];   // radix of each stage, product == N
};

// ------------------------------------------------------------ butterflies ---
template <typename T, int DIR, int R> struct Bfly;

template <typename T, int DIR> struct Bfly<T, DIR, 2> {
  using T2 = typename cpx<T>::t;
  __device__ static void run(T2* v) {
    T2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <typename T, int DIR> struct Bfly<T, DIR, 4> {
  using T2 = typename cpx<T>::t;
  __device__ static void run(T2* v) {
    T2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    T2 t2 = cadd(v[1], v[3]), t3 = rot90<DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <typename T, int DIR> struct Bfly<T, DIR, 8> {
  using T2 = typename cpx<T>::t;
  __device__ static void run(T2* v) {
    T2 e[4] = {v[0], v[2], v[4], v[6]};
    T2 o[4] = {v[1], v[3], v[5], v[7]};
    Bfly<T, DIR, 4>::run(e);
    Bfly<T, DIR, 4>::run(o);
    const T h = (T)0.70710678118654752440084436210484903928;
    // o[k] *= exp(DIR * 2 pi i k / 8)
    T2 o1 = DIR < 0 ? T2{h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)}
                    : T2{h * (o[1].x - o[1].y), h * (o[1].y + o[1].x)};
    T2 o2 = rot90<DIR>(o[2]);
    T2 o3 = DIR < 0 ? T2{h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)}
                    : T2{-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y)};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

template <typename T, int DIR> struct Bfly<T, DIR, 3> {
  using T2 = typename cpx<T>::t;
  __device__ static void run(T2* v) {
    const T c = (T)-0.5;
    const T s = (T)0.86602540378443864676372317075293618347;  // sin(2 pi / 3)
    T2 a = cadd(v[1], v[2]);
    T2 b = rot90<DIR>(csub(v[1], v[2]));  // DIR * i * (v1 - v2)
    T2 base = T2{v[0].x + c * a.x, v[0].y + c * a.y};
    v[0] = cadd(v[0], a);
    v[1] = T2{base.x + s * b.x, base.y + s * b.y};
    v[2] = T2{base.x - s * b.x, base.y - s * b.y};
  }
};

template <typename T, int DIR> struct Bfly<T, DIR, 5> {
  using T2 = typename cpx<T>::t;
  __device__ static void run(T2* v) {
    const T c1 = (T)0.30901699437494742410229341718281905886;   // cos(2 pi/5)
    const T c2 = (T)-0.80901699437494742410229341718281905886;  // cos(4 pi/5)
    const T s1 = (T)0.95105651629515357211643933337938214340;   // sin(2 pi/5)
    const T s2 = (T)0.58778525229247312916870595463907276860;   // sin(4 pi/5)
    T2 p1 = cadd(v[1], v[4]), m1 = csub(v[1], v[4]);
    T2 p2 = cadd(v[2], v[3]), m2 = csub(v[2], v[3]);
    T2 a1 = T2{v[0].x + c1 * p1.x + c2 * p2.x, v[0].y + c1 * p1.y + c2 * p2.y};
    T2 a2 = T2{v[0].x + c2 * p1.x + c1 * p2.x, v[0].y + c2 * p1.y + c1 * p2.y};
    T2 b1 = rot90<DIR>(T2{s1 * m1.x + s2 * m2.x, s1 * m1.y + s2 * m2.y});
    T2 b2 = rot90<DIR>(T2{s2 * m1.x - s1 * m2.x, s2 * m1.y - s1 * m2.y});
    v[0] = cadd(v[0], cadd(p1, p2));
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
  }
};

// Direct DFT for the remaining small primes: X_k = sum_r v_r W^{rk},
// W = exp(DIR 2 pi i / R).  Roots from sincospi in double.
template <typename T, int DIR, int R> struct BflyDirect {
  using T2 = typename cpx<T>::t;
  __device__ static void run(T2* v) {
    T2 out[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      T2 acc = v[0];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        double s, c;
        sincospi((double)DIR * 2.0 * (double)((r * k) % R) / (double)R, &s, &c);
        acc = cadd(acc, cmul(v[r], T2{(T)c, (T)s}));
      }
      out[k] = acc;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = out[k];
  }
};
template <typename T, int DIR> struct Bfly<T, DIR, 7> : BflyDirect<T, DIR, 7> {};
template <typename T, int DIR> struct Bfly<T, DIR, 11> : BflyDirect<T, DIR, 11> {};
template <typename T, int DIR> struct Bfly<T, DIR, 13> : BflyDirect<T, DIR, 13> {};

// ------------------------------------------------------------------ stage ---
// One Stockham stage of radix R over all L lines.  Butterfly b of a line reads
// x[j + r N/R] and writes y[(j/Ns) Ns R + j%Ns + r Ns], twiddled by
// exp(DIR 2 pi i r (j%Ns) / (Ns R)).  `line_fast` picks whether consecutive
// threads walk lines (element-major LDS layouts) or elements (line-major).
template <typename T, int DIR, int R, int MAXE>
__device__ __forceinline__ void fft_stage(typename cpx<T>::t* buf, int N, int L, int Ns, int ls, int es,
                                          bool line_fast, const typename cpx<T>::t* __restrict__ tw) {
  using T2 = typename cpx<T>::t;
  constexpr int MAXB = (MAXE / R) > 0 ? (MAXE / R) : 1;
  const int nthr = blockDim.x;
  const int tid = threadIdx.x;
  const int nbl = N / R;
  const int nb = nbl * L;
  const int tstep = N / (Ns * R);
  T2 v[MAXB][R];
  int dst[MAXB];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = tid + q * nthr;
    dst[q] = -1;
    if (b < nb) {
      int l, j;
      if (line_fast) {
        l = b % L;
        j = b / L;
      } else {
        l = b / nbl;
        j = b - l * nbl;
      }
      const T2* src = buf + l * ls;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[(j + r * nbl) * es];
      const int k = j % Ns;
      if (k != 0) {
        const int st = tstep * k;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          T2 w = tw[r * st];
          if (DIR > 0) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      Bfly<T, DIR, R>::run(v[q]);
      dst[q] = l * ls + ((j - k) * R + k) * es;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    if (dst[q] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[q] + r * Ns * es] = v[q][r];
    }
  }
  __syncthreads();
}

// Full FFT of L lines.  DIR = -1: forward, exp(-2 pi i ...); +1: inverse
// (unnormalised).  All threads of the block must call it.  SMOOTH: the plan's
// radices are 2, 3, 4, 5 and 8 only (the direct DFTs of 7, 11 and 13 are not
// built, which keeps the kernel's register count down).
template <typename T, int DIR, int MAXE, bool SMOOTH = false>
__device__ void fft_lines(typename cpx<T>::t* buf, const FftPlan& pl, int L, int ls, int es, bool line_fast,
                          const typename cpx<T>::t* __restrict__ tw) {
  int Ns = 1;
  for (int s = 0; s < pl.nst; ++s) {
    const int R = pl.rad[s];
    switch (R) {
      case 2: fft_stage<T, DIR, 2, MAXE>(buf, pl.N, L, Ns, ls, es, line_fast, tw); break;
      case 3: fft_stage<T, DIR, 3, MAXE>(buf, pl.N, L, Ns, ls, es, line_fast, tw); break;
      case 4: fft_stage<T, DIR, 4, MAXE>(buf, pl.N, L, Ns, ls, es, line_fast, tw); break;
      case 5: fft_stage<T, DIR, 5, MAXE>(buf, pl.N, L, Ns, ls, es, line_fast, tw); break;
      case 8: fft_stage<T, DIR, 8, MAXE>(buf, pl.N, L, Ns, ls, es, line_fast, tw); break;
      default:
        if constexpr (!SMOOTH) {
          if (R == 7) fft_stage<T, DIR, 7, MAXE>(buf, pl.N, L, Ns, ls, es, line_fast, tw);
          else if (R == 11) fft_stage<T, DIR, 11, MAXE>(buf, pl.N, L, Ns, ls, es, line_fast, tw);
          else if (R == 13) fft_stage<T, DIR, 13, MAXE>(buf, pl.N, L, Ns, ls, es, line_fast, tw);
        }
        break;
    }
    Ns *= R;
  }
}

// ------------------------------------------------- compile-time line FFT ---
// The same Stockham stages with the length, line count, layout and block size
// known at compile time: every index is a constant expression and each
// thread's butterflies are unrolled into registers.
struct RadList {
  int n;
  int r[LSH_MAX_STAGES];
};

__host__ __device__ constexpr RadList make_radlist(int N) {
  RadList L{0, {}};
  const int rads[8] = {8, 4, 2, 3, 5, 7, 11, 13};
  for (int i = 0; i < 8; ++i)
    while (N > 1 && N % rads[i] == 0 && L.n < LSH_MAX_STAGES) {
      L.r[L.n++] = rads[i];
      N /= rads[i];
    }
  return L;
}

template <typename T, int DIR, int N, int L, bool LF, int NT, int R, int NS>
__device__ __forceinline__ void fft_stage_static(typename cpx<T>::t* buf, int ls, int es,
                                                 const typename cpx<T>::t* __restrict__ tw) {
  using T2 = typename cpx<T>::t;
  constexpr int nbl = N / R;
  constexpr int nb = nbl * L;
  constexpr int NB = (nb + NT - 1) / NT;
  constexpr int tstep = N / (NS * R);
  const int tid = threadIdx.x;
  T2 v[NB][R];
  int dst[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int b = tid + q * NT;
    dst[q] = -1;
    if (nb % NT == 0 || b < nb) {
      const int l = LF ? (b % L) : (b / nbl);
      const int j = LF ? (b / L) : (b % nbl);
      const T2* src = buf + l * ls;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[(j + r * nbl) * es];
      const int k = j % NS;
      if (NS > 1 && k != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          T2 w = tw[r * tstep * k];
          if (DIR > 0) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      Bfly<T, DIR, R>::run(v[q]);
      dst[q] = l * ls + ((j - k) * R + k) * es;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q)
    if (nb % NT == 0 || dst[q] >= 0)
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[q] + r * NS * es] = v[q][r];
  __syncthreads();
}

template <typename T, int DIR, int N, int L, bool LF, int NT, int S = 0, int NS = 1>
__device__ __forceinline__ void fft_static(typename cpx<T>::t* buf, int ls, int es,
                                           const typename cpx<T>::t* __restrict__ tw) {
  constexpr RadList RL = make_radlist(N);
  if constexpr (S < RL.n) {
    constexpr int R = RL.r[S];
    fft_stage_static<T, DIR, N, L, LF, NT, R, NS>(buf, ls, es, tw);
    fft_static<T, DIR, N, L, LF, NT, S + 1, NS * R>(buf, ls, es, tw);
  }
}

// Dispatch: NC > 0 uses the compile-time path, NC == 0 the runtime plan,
// NC == -1 the runtime plan of a length whose radices are 2, 3, 4, 5, 8.
template <typename T, int DIR, int NC, int L, bool LF, int NT>
__device__ __forceinline__ void fft_any(typename cpx<T>::t* buf, const FftPlan& pl, int ls, int es,
                                        const typename cpx<T>::t* __restrict__ tw) {
  if constexpr (NC > 0) {
    fft_static<T, DIR, NC, L, LF, NT>(buf, ls, es, tw);
  } else {
    fft_lines<T, DIR, 16, NC < 0>(buf, pl, L, ls, es, LF, tw);
  }
}

// ------------------------------------------------- in-register line DFT ---
// The same Stockham stages on one thread's P values v[0..P) held in
// registers (P a compile-time length with radices from make_radlist): every
// index is a constant, so the data never leaves registers.  twP[k] =
// exp(-2 pi i k / P), k < P (forward; DIR = +1 conjugates, unnormalised).
template <typename T, int DIR, int P, int S = 0, int NS = 1>
__device__ __forceinline__ void reg_fft(typename cpx<T>::t (&v)[P], const typename cpx<T>::t* __restrict__ twP) {
  using T2 = typename cpx<T>::t;
  constexpr RadList RL = make_radlist(P);
  if constexpr (S < RL.n) {
    constexpr int R = RL.r[S];
    constexpr int nbl = P / R;
    constexpr int tstep = P / (NS * R);
    T2 y[P];
#pragma unroll
    for (int j = 0; j < nbl; ++j) {
      const int k = j % NS;
      T2 u[R];
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = v[j + r * nbl];
      if (NS > 1 && k != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          T2 w = twP[r * tstep * k];
          if (DIR > 0) w.y = -w.y;
          u[r] = cmul(u[r], w);
        }
      }
      Bfly<T, DIR, R>::run(u);
#pragma unroll
      for (int r = 0; r < R; ++r) y[(j - k) * R + k + r * NS] = u[r];
    }
#pragma unroll
    for (int i = 0; i < P; ++i) v[i] = y[i];
    reg_fft<T, DIR, P, S + 1, NS * R>(v, twP);
  }
}
