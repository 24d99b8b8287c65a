// lsh_twopass.hpp -- the Basic Scheme iteration in two passes: the interface
// between the solver (lsh_solver.hip) and the translation unit that holds the
// two passes' kernels (lsh_twopass.hip).
//
// The axis-2 DFT of length n2 = Q P is split in the four-step way.  With
// i2 = r + P j (r < P, j < Q) and k2 = q + Q s (q < Q, s < P),
//
//   F[q + Q s] = sum_r w_P^{r s} w_n2^{r q} sum_j f[r + P j] w_Q^{j q},
//
// w_N = exp(-2 pi i / N).  The inner Q-point DFTs (over j at fixed r) and the
// twiddle w_n2^{r q} join the axis-1 stress pass, whose tile then covers the
// coset r + P j of axis 2; the outer P-point DFTs (over r at fixed q) join the
// axis-3 Green pass, whose tile covers k2 = q + Q s.  The iteration state is
// kept between the two halves of axis 2:
//
//   layout [load][comp][k1 < n1/2+1][q < Q][r < P][i3 < n3]  (complex)
//
//   S2 (stress): X' --conj twiddle, Q-point IDFT over q--> (k1, i2, i3)
//        --C2R axis 1--> E(y) --(C - C0):(E + eps0)--> tau(y)
//        --R2C axis 1, Q-point DFT over j, twiddle--> TAU'
//   G3 (Green):  TAU' --P-point DFT over r--> (k1, k2, i3) --FFT axis 3-->
//        tau_hat --(-Gamma^p / m)--> --IFFT axis 3, P-point IDFT over s-->
//        X'_new, and the Cauchy residual against X'_old
//
// Both tiles read and write runs of W (stress) or P n3 (Green) consecutive
// elements.  Per voxel and load an iteration moves 30 s + 1 bytes (s the bytes
// of a real scalar) instead of the four-pass schedule's 54 s + 1.
#pragma once
#include "lsh_common.hpp"

template <typename T>
struct TwoPass {
  using S2 = void (*)(Geo, const C2<T>*, const C2<T>*, const C2<T>*, C2<T>*, const Inst*, const int*, const double*,
                      const int*, const int*);
  using G3 = void (*)(Geo, const C2<T>*, const C2<T>*, const C2<T>*, const C2<T>*, C2<T>*, const T*, const Inst*,
                      const int*, const int*, const int*, const int*, int, double*, int, C2<T>*);
  S2 s2 = nullptr;
  G3 g3[4] = {nullptr, nullptr, nullptr, nullptr};     // per Green mode (GREEN_TABLE, GREEN_MOMENTS built)
  G3 g3inc[4] = {nullptr, nullptr, nullptr, nullptr};  // the same for the increment scheme
  G3 green(int gmode, bool inc) const { return inc ? g3inc[gmode] : g3[gmode]; }
  int Q = 0, P = 0, W = 0;  // axis-2 split and the stress tile's width along i3
  int nts = 0, ntg = 0;     // threads per block of each pass
  size_t ldss = 0, ldsg = 0;
};

// The two-pass variants built for SNF grid g at precision T (at most maxn);
// returns how many.  None for grids outside the compiled set.
int twopass_candidates(const Geo& g, TwoPass<float>* out, int maxn);
int twopass_candidates(const Geo& g, TwoPass<double>* out, int maxn);

// State conversions between the four-pass layout X = D1[E]/n1 on
// (k1, i2, i3) and the split layout:
//   to_split:   Xs = (1/Q) w_n2^{r q} sum_j X[r + P j] w_Q^{j q}
//   from_split: X[r + P j] = sum_q w_n2^{-r q} Xs[q] w_Q^{-j q}, reading for
//               load L the buffer its last iteration wrote: Xs0 if
//               min(stop_iter[L], it) is even, else Xs1.
// tw1: the axis-2 twiddles exp(-2 pi i k / n2), k < n2.
void twopass_to_split(const Geo& g, int Q, const C2<float>* tw1, const C2<float>* X, C2<float>* Xs, int nload,
                      hipStream_t st);
void twopass_to_split(const Geo& g, int Q, const C2<double>* tw1, const C2<double>* X, C2<double>* Xs, int nload,
                      hipStream_t st);
void twopass_from_split(const Geo& g, int Q, const C2<float>* tw1, const C2<float>* Xs0, const C2<float>* Xs1,
                        C2<float>* X, const int* stop_iter, const int* itp, int nload, hipStream_t st);
void twopass_from_split(const Geo& g, int Q, const C2<double>* tw1, const C2<double>* Xs0, const C2<double>* Xs1,
                        C2<double>* X, const int* stop_iter, const int* itp, int nload, hipStream_t st);
