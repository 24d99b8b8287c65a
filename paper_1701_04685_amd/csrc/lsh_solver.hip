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
#include <mutex>
#include <string>
#include <vector>

#include "lsh_internal.hpp"

#include "lsh_kernels.hpp"
#include "lsh_twopass.hpp"

namespace {

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
  g.ncf = p->d == 2 ? 3 : 6;
  g.pad_ = 0;
  return g;
}

// Does a runtime-plan FFT over L lines fit nthr threads x 16 registers?
bool plan_fits(const FftPlan& pl, int L, int nthr) {
  for (int s = 0; s < pl.nst; ++s) {
    const int R = pl.rad[s];
    const int maxb = std::max(1, 16 / R);
    const long long nb = (long long)(pl.N / R) * L;
    if (nb > (long long)nthr * maxb) return false;
  }
  return true;
}

// A plan whose radices are all 2, 3, 4, 5 or 8: its runtime-plan kernels are
// built without the direct DFTs of the larger primes (NC = -1).
bool plan_smooth(const FftPlan& pl) {
  for (int s = 0; s < pl.nst; ++s) {
    const int r = pl.rad[s];
    if (r != 2 && r != 3 && r != 4 && r != 5 && r != 8) return false;
  }
  return true;
}

int lds_limit() {
  static int lim = -1;
  if (lim < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 64 * 1024;
    lim = v;
  }
  return lim;
}

// The kernel instantiations chosen for one pattern and precision.
template <typename T>
struct KernSet {
  using A1 = void (*)(Geo, FftPlan, const C2<T>*, const C2<T>*, C2<T>*, const Inst*, const int*, const double*,
                      const int*, const int*, const double* const*, const double*, double* const*, double*);
  using A2 = void (*)(Geo, FftPlan, const C2<T>*, const C2<T>*, C2<T>*, const int*, const int*, T);
  using GR = void (*)(Geo, FftPlan, const C2<T>*, GreenParams, const C2<T>*, const C2<T>*, C2<T>*, const T*,
                      const Inst*, const int*, const int*, const int*, const int*, int, int, double*, int, int, int,
                      C2<T>*);
  A1 a1[3] = {nullptr, nullptr, nullptr};  // MODE_STRESS, MODE_FINAL, MODE_INIT
  A2 a2[2] = {nullptr, nullptr};           // forward, inverse
  GR gr = nullptr;
  GR gr2[4] = {nullptr, nullptr, nullptr, nullptr};  // k_green2 per Green mode (ISO, GENERAL, TABLE, MOMENTS)
  int W1 = 0, NT1 = 0, W2 = 0, NT2 = 0, NTG = 0, lsG = 0;
  A1 a1s = nullptr;  // the stress-pass kernel in use (a candidate below)
  using ACG = void (*)(Geo, FftPlan, const C2<T>*, const C2<T>*, C2<T>*, C2<T>*, const Inst*, const int*,
                       const double*, const int*, const int*, double*);
  ACG a1cg = nullptr;  // conjugate gradients: direction and stress pass (runtime plans)
  int NT1s = 0, W1s = 0;
  size_t lds1s = 0;
  // autotuner candidates per pass; entry 0 is the default
  struct CStress { A1 fn; int nt; size_t lds; int W; };
  struct CAxis2 { A2 fwd, inv; int W, nt; size_t lds; };
  struct CGreen { GR fn[4]; int nt; size_t lds; int gch = GCH; };  // gch: loads per chunk
  std::vector<CStress> c1;
  std::vector<CAxis2> c2;
  std::vector<CGreen> cg;
  int green2 = 0;  // 1: k_green2 (grid: positions x load chunks), 0: k_green
  int gch = GCH;   // loads per Green-pass chunk (k_green2; fewer: more blocks, more table reads)
  size_t lds1 = 0, lds2 = 0, ldsG = 0;
  // two-pass schedule (lsh_twopass.hpp): its variants and the one in use (-1: four passes)
  std::vector<TwoPass<T>> tp;
  int tpi = -1;
};

constexpr int pick_w(int N, int bytes_per_col, int cap, int budget) {
  int w = cap;
  while (w > 1 && N * w * bytes_per_col > budget) w /= 2;
  return w;
}

// compile-time line lengths; every other length takes the runtime plan
#define LSH_SPECIAL_SIZES(X) X(16) X(32) X(48) X(64) X(96) X(125) X(128) X(256) X(512)

template <typename T, int NC, int W>
void put_axis1(KernSet<T>& K) {
  K.a1[0] = k_axis1<T, MODE_STRESS, NC, W, 256>;
  K.a1[1] = k_axis1<T, MODE_FINAL, NC, W, 256>;
  K.a1[2] = k_axis1<T, MODE_INIT, NC, W, 256>;
  K.a1cg = k_cg_stress<T, NC, W, 256>;
  K.W1 = W;
  K.NT1 = 256;
}

template <int N, int W>
constexpr int axis1s_nt() {
  int a = W * (N / 2), b = 3 * W * (N / 8);
  int nt = ((a > b ? a : b) + 63) / 64 * 64;
  return nt < 64 ? 64 : nt;
}

template <typename T, int NC>
bool axis1_special(const Geo& g, KernSet<T>& K) {
  constexpr int W = pick_w(NC, 3 * (int)sizeof(C2<T>), 16, 60 * 1024);
  if (g.n3 < W) return false;
  if constexpr (NC * 3 * W * sizeof(C2<T>) >= 32768) {
    K.a1[0] = k_axis1<T, MODE_STRESS, NC, W, 512>;
    K.a1[1] = k_axis1<T, MODE_FINAL, NC, W, 512>;
    K.a1[2] = k_axis1<T, MODE_INIT, NC, W, 512>;
    K.a1cg = k_cg_stress<T, NC, W, 512>;
    K.W1 = W;
    K.NT1 = 512;
  } else {
    put_axis1<T, NC, W>(K);
  }
  K.c1.clear();
  K.c1.push_back({K.a1[0], K.NT1, 0, W});  // k_axis1 (MODE_STRESS); LDS filled in by choose_axis1
  {
    // the same tile with the LDS phase table cut to two phases and the register
    // budget capped so that as many blocks run per CU as the LDS allows
    constexpr int NTo = NC * 3 * W * sizeof(C2<T>) >= 32768 ? 512 : 256;
    constexpr size_t lds_o = sizeof(C2<T>) * ((size_t)NC + (size_t)NC * 3 * W) + sizeof(T) * 36 * 2;
    constexpr int waves = (int)(163840 / lds_o) * NTo / 64;
    constexpr int MINW = (waves + 3) / 4 < 1 ? 1 : ((waves + 3) / 4 > 6 ? 6 : (waves + 3) / 4);
    // first in the list: the default when the pattern is not tuned
    if (lds_o <= (size_t)lds_limit())
      K.c1.insert(K.c1.begin(), {k_axis1<T, MODE_STRESS, NC, W, NTo, 2, MINW>, NTo, lds_o, W});
  }
  if constexpr (NC % 2 == 0 && axis1s_nt<NC, W>() <= 1024) {
    constexpr int NT = axis1s_nt<NC, W>();
    const size_t lds = sizeof(C2<T>) * (size_t)NC + sizeof(T) * 36 * 16 +
                       sizeof(C2<T>) * 3 * (size_t)W * GreenPlan<NC>::LP + (size_t)NC * W;
    if (lds <= (size_t)lds_limit()) K.c1.push_back({k_axis1s<T, NC, W, NT>, NT, lds, W});
  }
  if constexpr (W >= 4) {  // narrower tiles: more blocks per CU, shorter runs along i3
    constexpr int Wh = W / 2;
    const size_t lds = sizeof(C2<T>) * ((size_t)NC + (size_t)NC * 3 * Wh) + sizeof(T) * 36 * 16;
    K.c1.push_back({k_axis1<T, MODE_STRESS, NC, Wh, 256>, 256, lds, Wh});
  }
  if constexpr (W <= 16 && NC <= 256) {  // wider tiles: longer runs along i3, one block per CU
    constexpr int W2x = 2 * W;
    if (g.n3 >= W2x) {
      const size_t lds = sizeof(C2<T>) * ((size_t)NC + (size_t)NC * 3 * W2x) + sizeof(T) * 36 * 16;
      if (lds <= (size_t)lds_limit()) K.c1.push_back({k_axis1<T, MODE_STRESS, NC, W2x, 1024>, 1024, lds, W2x});
      if constexpr (NC % 2 == 0 && axis1s_nt<NC, W2x>() <= 1024) {
        constexpr int NT = axis1s_nt<NC, W2x>();
        const size_t lf = sizeof(C2<T>) * (size_t)NC + sizeof(T) * 36 * 16 +
                          sizeof(C2<T>) * 3 * (size_t)W2x * GreenPlan<NC>::LP + (size_t)NC * W2x;
        if (lf <= (size_t)lds_limit()) K.c1.push_back({k_axis1s<T, NC, W2x, NT>, NT, lf, W2x});
      }
    }
  }
  return true;
}

template <typename T>
bool choose_axis1(const Geo& g, const FftPlan& pl, KernSet<T>& K) {
  bool ok = false;
  K.c1.clear();
  switch (g.n1) {
#define X(N) \
  case N: ok = axis1_special<T, N>(g, K); break;
    LSH_SPECIAL_SIZES(X)
#undef X
    default: break;
  }
  if (!ok) {
    // runtime plan: widest tile (16, 4 or 1 columns) that fits
    const bool sm = plan_smooth(pl);
    if (g.n3 >= 16 && plan_fits(pl, 48, 256) && (size_t)g.n1 * 48 * sizeof(C2<T>) <= 60 * 1024) {
      if (sm) put_axis1<T, -1, 16>(K);
      else put_axis1<T, 0, 16>(K);
    } else if (g.n3 >= 4 && plan_fits(pl, 12, 256) && (size_t)g.n1 * 12 * sizeof(C2<T>) <= 60 * 1024) {
      if (sm) put_axis1<T, -1, 4>(K);
      else put_axis1<T, 0, 4>(K);
    } else if (plan_fits(pl, 3, 256)) {
      if (sm) put_axis1<T, -1, 1>(K);
      else put_axis1<T, 0, 1>(K);
    } else {
      return false;
    }
  }
  K.lds1 = sizeof(C2<T>) * ((size_t)g.n1 + (size_t)g.n1 * 3 * K.W1) + sizeof(T) * 36 * 16;
  if (K.c1.empty()) K.c1.push_back({K.a1[0], K.NT1, K.lds1, K.W1});
  for (auto& c : K.c1)
    if (c.fn == K.a1[0]) c.lds = K.lds1;
  return K.lds1 <= (size_t)lds_limit();
}

template <typename T, int NC, int W>
void put_axis2(KernSet<T>& K) {
  K.a2[0] = k_axis2<T, -1, NC, W, 256>;
  K.a2[1] = k_axis2<T, +1, NC, W, 256>;
  K.W2 = W;
  K.NT2 = 256;
}

template <typename T, int NC>
bool axis2_special(const Geo& g, KernSet<T>& K) {
  constexpr int W = pick_w(NC, (int)sizeof(C2<T>), sizeof(T) == 8 ? 16 : 32, 32 * 1024);
  if (g.n3 < W) return false;
  put_axis2<T, NC, W>(K);
  if constexpr (W >= 4) {
    constexpr int Wh = W / 2;
    K.c2.push_back({k_axis2<T, -1, NC, Wh, 256>, k_axis2<T, +1, NC, Wh, 256>, Wh, 256,
                    sizeof(C2<T>) * ((size_t)NC + (size_t)NC * Wh)});
  }
  if constexpr (W <= 32 && NC <= 256) {  // wider tiles: longer runs along i3, fewer blocks
    constexpr int W2x = 2 * W;
    const size_t lds = sizeof(C2<T>) * ((size_t)NC + (size_t)NC * W2x);
    if (g.n3 >= W2x && lds <= (size_t)lds_limit())
      K.c2.push_back({k_axis2<T, -1, NC, W2x, 512>, k_axis2<T, +1, NC, W2x, 512>, W2x, 512, lds});
  }
  return true;
}

template <typename T>
bool choose_axis2(const Geo& g, const FftPlan& pl, KernSet<T>& K) {
  bool ok = false;
  K.c2.clear();
  switch (g.n2) {
#define X(N) \
  case N: ok = axis2_special<T, N>(g, K); break;
    LSH_SPECIAL_SIZES(X)
#undef X
    default: break;
  }
  if (!ok) {
    const bool sm = plan_smooth(pl);
    if (g.n3 >= 16 && plan_fits(pl, 16, 256) && (size_t)g.n2 * 16 * sizeof(C2<T>) <= 60 * 1024) {
      if (sm) put_axis2<T, -1, 16>(K);
      else put_axis2<T, 0, 16>(K);
    } else if (g.n3 >= 4 && plan_fits(pl, 4, 256) && (size_t)g.n2 * 4 * sizeof(C2<T>) <= 60 * 1024) {
      if (sm) put_axis2<T, -1, 4>(K);
      else put_axis2<T, 0, 4>(K);
    } else if (plan_fits(pl, 1, 256)) {
      if (sm) put_axis2<T, -1, 1>(K);
      else put_axis2<T, 0, 1>(K);
    } else {
      return false;
    }
  }
  K.lds2 = sizeof(C2<T>) * ((size_t)g.n2 + (size_t)g.n2 * K.W2);
  K.c2.insert(K.c2.begin(), {K.a2[0], K.a2[1], K.W2, K.NT2, K.lds2});
  return K.lds2 <= (size_t)lds_limit();
}

template <int N, int NL>
constexpr int green2_nt() {
  // one thread per radix-8 butterfly over all lines of a pass
  int nt = (NL * 6 * (N / 8) + 63) / 64 * 64;
  return nt < 64 ? 64 : (nt > 512 ? 512 : nt);
}

template <typename T, int NC, int NL, int MINW = 1>
typename KernSet<T>::CGreen green2_cand() {
  constexpr int NT = green2_nt<NC, NL>();
  constexpr RadList RH = GreenPlan<NC>::RH;
  constexpr int RL = RH.r[RH.n - 1];
  typename KernSet<T>::CGreen c;
  c.fn[GREEN_ISO] = nullptr;  // the isotropic path reads the moments table
  // the on-the-fly general form needs more registers than a wave cap leaves
  // (capped at three waves it spills): always the uncapped build
  c.fn[GREEN_GENERAL] = k_green2<T, NC, NL, NT, GREEN_GENERAL, 1>;
  c.fn[GREEN_TABLE] = k_green2<T, NC, NL, NT, GREEN_TABLE, MINW>;
  c.fn[GREEN_MOMENTS] = k_green2<T, NC, NL, NT, GREEN_MOMENTS, MINW>;
  c.nt = NT;
  c.lds = sizeof(C2<T>) * (size_t)NC + sizeof(T) * 21 * (size_t)NC + sizeof(C2<T>) * (size_t)NL * 6 * GreenPlan<NC>::LP +
          sizeof(C2<T>) * (size_t)(RL - 1) * (NC / RL);
  return c;
}

template <typename T, int NC>
void green_special(const Geo& g, KernSet<T>& K) {
  K.cg.clear();
  if constexpr (NC % 2 == 0) {
    // FP64 at n3 = 128: two loads at a time capped at three waves per SIMD
    // (168 VGPRs, no spills; the uncapped build takes 170 and runs two).  At
    // the other lengths the cap either changes nothing or spills.
    if constexpr (sizeof(T) == 8 && NC == 128) K.cg.push_back(green2_cand<T, NC, 2, 3>());
    K.cg.push_back(green2_cand<T, NC, (NC <= 128 ? 2 : 1)>());
    if constexpr (NC <= 128) K.cg.push_back(green2_cand<T, NC, 1>());
    if constexpr (sizeof(T) == 8 && NC == 128) {
      // the same with chunks of three loads: twice the blocks, the moments read twice
      auto c3 = green2_cand<T, NC, 2, 3>();
      c3.gch = 3;
      K.cg.push_back(c3);
    }
    if constexpr (NC >= 256) {
      // long lines have few positions: chunks of two or three loads give more
      // blocks (a shorter last wave) for more reads of the position's operator
      auto c3 = green2_cand<T, NC, 1>();
      c3.gch = 3;
      K.cg.push_back(c3);
      auto c2 = green2_cand<T, NC, 1>();
      c2.gch = 2;
      K.cg.push_back(c2);
    }
    for (size_t i = K.cg.size(); i-- > 0;)
      if (K.cg[i].lds > (size_t)lds_limit()) K.cg.erase(K.cg.begin() + i);
    if (!K.cg.empty()) {
      for (int m = 0; m < 4; ++m) K.gr2[m] = K.cg[0].fn[m];
      K.gr = K.gr2[GREEN_MOMENTS];
      K.NTG = K.cg[0].nt;
      K.ldsG = K.cg[0].lds;
      K.green2 = 1;
      K.lsG = 0;
      return;
    }
  }
  constexpr int NT = NC <= 64 ? 64 : (NC <= 128 ? 128 : 256);
  K.gr = k_green<T, NC, NT>;
  if constexpr (NC % 2 == 1) {
    // odd lengths: one build per Green mode (the moment and table paths
    // then hold about 100 VGPRs instead of the on-the-fly paths' 220)
    K.gr2[GREEN_ISO] = k_green<T, NC, NT, GREEN_ISO>;
    K.gr2[GREEN_GENERAL] = k_green<T, NC, NT, GREEN_GENERAL>;
    K.gr2[GREEN_TABLE] = k_green<T, NC, NT, GREEN_TABLE>;
    K.gr2[GREEN_MOMENTS] = k_green<T, NC, NT, GREEN_MOMENTS>;
  }
  K.NTG = NT;
  (void)g;
}

// Runtime-plan Green pass of a smooth length: one build per Green mode (the
// branches of the other modes and the direct DFTs would otherwise set the
// register count).
template <typename T, int NT>
void put_green_rt(KernSet<T>& K) {
  K.gr2[GREEN_GENERAL] = k_green<T, -1, NT, GREEN_GENERAL>;
  K.gr2[GREEN_TABLE] = k_green<T, -1, NT, GREEN_TABLE>;
  K.gr2[GREEN_MOMENTS] = k_green<T, -1, NT, GREEN_MOMENTS>;
  K.gr = K.gr2[GREEN_MOMENTS];
}

template <typename T>
bool choose_green(const Geo& g, const FftPlan& pl, bool table, KernSet<T>& K) {
  bool ok = false;
  switch (g.n3) {
#define X(N) \
  case N: green_special<T, N>(g, K); ok = true; break;
    LSH_SPECIAL_SIZES(X)
#undef X
    default: break;
  }
  if (!ok) {
    int nt = 64;
    while (nt < 256 && (nt < g.n3 || !plan_fits(pl, 6, nt))) nt *= 2;
    // long lines (e.g. 1024, 2048) need more threads for their butterflies
    while (nt < 1024 && !plan_fits(pl, 6, nt)) nt *= 2;
    if (!plan_fits(pl, 6, nt)) return false;
    if (plan_smooth(pl)) {
      if (nt == 64) put_green_rt<T, 64>(K);
      else if (nt == 128) put_green_rt<T, 128>(K);
      else if (nt == 256) put_green_rt<T, 256>(K);
      else if (nt == 512) put_green_rt<T, 512>(K);
      else put_green_rt<T, 1024>(K);
    } else {
      if (nt == 64) K.gr = k_green<T, 0, 64>;
      else if (nt == 128) K.gr = k_green<T, 0, 128>;
      else if (nt == 256) K.gr = k_green<T, 0, 256>;
      else if (nt == 512) K.gr = k_green<T, 0, 512>;
      else K.gr = k_green<T, 0, 1024>;
    }
    K.NTG = nt;
  }
  (void)table;
  if (!K.green2) {
    K.lsG = g.n3 + ((g.n3 % 2 == 0) ? 1 : 0);
    K.ldsG = sizeof(C2<T>) * ((size_t)g.n3 + 6 * (size_t)K.lsG);
  }
  return K.ldsG <= (size_t)lds_limit();
}

// The frequency reduction on the GPU uses double-estimated quotients, exact
// while |sign(det) adj(M^T) V^T b| < 2^51 for every grid index b.
bool index_maps_in_range(const lsh_pattern* p) {
  GreenParams gp;
  lsh_green_params(p, &gp);
  long double hmax[3];
  for (int i = 0; i < 3; ++i) {
    hmax[i] = 0;
    for (int k = 0; k < 3; ++k) hmax[i] += fabsl((long double)gp.VT[3 * i + k]) * (long double)(p->e[k] - 1);
  }
  for (int i = 0; i < 3; ++i) {
    long double v = 0;
    for (int k = 0; k < 3; ++k) v += fabsl((long double)gp.A[3 * i + k]) * (hmax[k] + 1.0L);
    if (v + (long double)p->m >= 2251799813685248.0L) return false;
  }
  return true;
}

template <typename T>
int make_kernels(const lsh_pattern* p, bool table, KernSet<T>* K) {
  const Geo g = geo_of(p);
  if (!index_maps_in_range(p)) return lsh_fail(LSH_EUNSUPPORTED, "frequency index maps exceed 2^51");
  for (int i = 0; i < 3; ++i)
    if (p->plan[i].nst < 0)
      return lsh_fail(LSH_EUNSUPPORTED, "SNF factor e" + std::to_string(i + 1) + " = " + std::to_string(p->e[i]) +
                                            " has a prime factor above 13");
  if (!choose_axis1<T>(g, p->plan[0], *K)) return lsh_fail(LSH_EUNSUPPORTED, "SNF factor e1 too large for one block");
  if (!choose_axis2<T>(g, p->plan[1], *K)) return lsh_fail(LSH_EUNSUPPORTED, "SNF factor e2 too large for one block");
  if (!choose_green<T>(g, p->plan[2], table, *K)) return lsh_fail(LSH_EUNSUPPORTED, "SNF factor e3 too large for one block");
  K->tp.clear();
  if (p->scheme != LSH_SCHEME_CG) {
    TwoPass<T> c[8];
    const int n = twopass_candidates(g, c, 8);
    for (int i = 0; i < n; ++i)
      if (c[i].ldss <= (size_t)lds_limit() && c[i].ldsg <= (size_t)lds_limit()) K->tp.push_back(c[i]);
  }
  return LSH_OK;
}

// Allow dynamic LDS beyond the 64 KB default where a launch needs it.
template <typename F>
int allow_lds(F fn, size_t lds) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return lsh_fail(LSH_EUNSUPPORTED, std::string("LDS request refused: ") + hipGetErrorString(e));
  }
  return LSH_OK;
}

// Isotropic reference stiffness: Lame (lam0, mu0) if C0 has that form.
bool c0_isotropic(const lsh_pattern* p, double* lam0, double* mu0) {
  const double* C = p->C0_voigt;
  const double lam = C[1], mu = C[21];
  double mx = 0.0;
  for (int i = 0; i < 36; ++i) mx = std::max(mx, fabs(C[i]));
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) {
      double want = 0.0;
      if (I < 3 && J < 3) want = lam + (I == J ? 2.0 * mu : 0.0);
      if (I >= 3 && I == J) want = mu;
      if (fabs(C[6 * I + J] - want) > 1e-13 * mx) return false;
    }
  *lam0 = lam;
  *mu0 = mu;
  return true;
}

// Which form of the Green operator the solver uses for this pattern.
int green_mode(const lsh_pattern* p) {
  double l, m;
  if (p->kind == LSH_BOXSPLINE) return GREEN_TABLE;
  if (p->nphase >= 1 && c0_isotropic(p, &l, &m)) return GREEN_MOMENTS;
  if (p->kind == LSH_DIRICHLET) return GREEN_GENERAL;
  return GREEN_TABLE;
}

// The two-pass Green pass's operator form: with the Dirichlet kernel on
// M = diag(n, n, n) (SNF factors the identity, so the grid index is the
// frequency) and an isotropic C0 it applies Gamma0 in closed form and reads no
// table; otherwise the pattern's form.
int twopass_green_mode(const lsh_pattern* p, int gmode) {
  if (gmode != GREEN_MOMENTS || p->kind != LSH_DIRICHLET) return gmode;
  const int64_t* M = p->M;
  bool diag = M[0] > 0 && M[0] == M[4] && M[4] == M[8];
  for (int i = 0; i < 9; ++i) {
    if (i % 4 != 0 && M[i] != 0) diag = false;
    if (p->V[i] != (i % 4 == 0 ? 1 : 0)) diag = false;
  }
  return diag ? GREEN_ISO : gmode;
}

bool kind_has_table(const lsh_pattern* p) {
  // the table slot (21 rows per bin) holds Gamma^p rows (GREEN_TABLE) or the
  // 15 fourth alias moments (GREEN_MOMENTS); before the stiffness is known,
  // size for it
  if (p->nphase < 1) return true;
  const int gm = green_mode(p);
  return gm == GREEN_TABLE || gm == GREEN_MOMENTS;
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
  if (kind_has_table(p)) b += lsh_align(scal * 21 * (size_t)g.spec);
  return b;
}

struct Profile {
  bool on = false;
  unsigned mask = ~0u;  // slots timed while on
  double ms[8] = {0};
  long long n[8] = {0};
};
Profile g_prof;

template <typename T>
int bind_t(lsh_pattern* p, void* dev, size_t bytes, hipStream_t st) {
  KernSet<T> K;
  int rc = make_kernels<T>(p, kind_has_table(p), &K);
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
      // stress-pass matrix: C_p - C0 (Lippmann-Schwinger, either form), C_p
      // (variational, conjugate gradients)
      const bool ls = p->scheme == LSH_SCHEME_LS || p->scheme == LSH_SCHEME_LS_INC;
      dm[36 * q + i] = (T)(ls ? Cm[i] - C0m[i] : Cm[i]);
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
  if (kind_has_table(p)) {
    const Geo g = geo_of(p);
    p->off_table = off;
    off += lsh_align(sizeof(T) * 21 * (size_t)g.spec);
    GreenParams gp;
    lsh_green_params(p, &gp);
    const int nthr = 256;
    const int nblk = (int)std::min<long long>((g.spec + nthr - 1) / nthr, 4096);
    T* table = (T*)(base + p->off_table);
    if (green_mode(p) == GREEN_MOMENTS) {
      // the trapezoid weights of the analytic kernels never all vanish
      hipLaunchKernelGGL(k_moments_table<T>, dim3(nblk), dim3(nthr), 0, st, g, gp, table);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(st));
    } else {
      // isotropic C0: the alias sums run over direction moments
      if (gp.iso)
        hipLaunchKernelGGL((k_gamma_table<T, 1>), dim3(nblk), dim3(nthr), 0, st, g, gp, table, mins_dev);
      else
        hipLaunchKernelGGL((k_gamma_table<T, 0>), dim3(nblk), dim3(nthr), 0, st, g, gp, table, mins_dev);
      HIPCHK(hipGetLastError());
      std::vector<double> mins(nblk);
      HIPCHK(hipMemcpyAsync(mins.data(), mins_dev, sizeof(double) * nblk, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      double mn = 1e300;
      for (int i = 0; i < nblk; ++i) mn = std::min(mn, mins[i]);
      if (!(mn > 0.0))
        return lsh_fail(LSH_ENOINTERP, "a bracket sum of |c_k(f)|^2 vanishes: translates are not linearly independent");
    }
    p->has_table = true;
  }
  p->dev_persist = base;
  p->bound_prec = sizeof(T) == 8 ? LSH_FP64 : LSH_FP32_MIXED;
  return LSH_OK;
}

// One group of load cases that share the SNF grid, M, the generating function
// and the kernel instantiations: a single solve, or one size class of a batch.
struct GroupWS {
  char* X;
  char* TAU;
  char* P[2];
  char* EX[2];     // conjugate gradients: residual z and direction p
  double* cg;      // conjugate gradients: per load {rho, alpha, beta, -}
  double* C0m;     // conjugate gradients: C0 (Mandel)
  double* partial;
  double* eps0;
  double* eps0z;   // zeros: the stress pass's eps0 in the increment scheme
  double* e0sq;
  double* hist;
  double* sigma;
  double* means;
  const double** einit;  // per load: the caller's start field ([ncf][m] block) or null
  double** eout;         // per load: where the final field goes, or null
  int* stop_iter;
  int* nonfinite;
  int* itp;
  int* inst_of;
  int* chunks;  // per Green chunk: first load, end load (one instance, <= GCH loads)
  Inst* insts;
  size_t total;
};

template <typename T>
GroupWS group_layout(const Geo& g, int nload, int ninst, const KernSet<T>& K, char* base, bool cg = false) {
  const size_t fb = lsh_align(sizeof(C2<T>) * 6 * (size_t)nload * g.spec);
  GroupWS w;
  size_t off = 0;
  w.X = base + off; off += fb;
  w.TAU = base + off; off += fb;
  w.P[0] = base + off; off += fb;
  w.P[1] = base + off; off += fb;
  w.EX[0] = w.EX[1] = nullptr;
  w.cg = w.C0m = nullptr;
  if (cg) {
    w.EX[0] = base + off; off += fb;
    w.EX[1] = base + off; off += fb;
    w.cg = (double*)(base + off); off += lsh_align(sizeof(double) * 4 * nload);
    w.C0m = (double*)(base + off); off += lsh_align(sizeof(double) * 36);
  }
  const long long nblkS = (long long)g.n2 * ((g.n3 + K.W1 - 1) / K.W1);
  const long long nblkG = (long long)g.h1 * g.n2;
  const long long nblkU = (g.spec + 255) / 256;
  const long long npart = std::max(std::max(nblkS * 6, nblkG * 2), cg ? nblkU * 3 : 0LL) * nload;
  w.partial = (double*)(base + off); off += lsh_align(sizeof(double) * npart);
  w.eps0 = (double*)(base + off); off += lsh_align(sizeof(double) * 6 * nload);
  w.eps0z = (double*)(base + off); off += lsh_align(sizeof(double) * 6 * nload);
  w.e0sq = (double*)(base + off); off += lsh_align(sizeof(double) * nload);
  w.hist = (double*)(base + off); off += lsh_align(sizeof(double) * LSH_HIST * nload);
  w.sigma = (double*)(base + off); off += lsh_align(sizeof(double) * 6 * nload);
  w.means = (double*)(base + off); off += lsh_align(sizeof(double) * 6 * nload);
  w.einit = (const double**)(base + off); off += lsh_align(sizeof(double*) * nload);
  w.eout = (double**)(base + off); off += lsh_align(sizeof(double*) * nload);
  w.stop_iter = (int*)(base + off); off += lsh_align(sizeof(int) * nload);
  w.nonfinite = (int*)(base + off); off += lsh_align(sizeof(int) * nload);
  w.itp = (int*)(base + off); off += lsh_align(sizeof(int) * 2);
  w.inst_of = (int*)(base + off); off += lsh_align(sizeof(int) * nload);
  w.chunks = (int*)(base + off); off += lsh_align(sizeof(int) * 2 * nload);
  w.insts = (Inst*)(base + off); off += lsh_align(sizeof(Inst) * ninst);
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
  bool rec;
  Timer(int s, hipStream_t stream) : slot(s), st(stream), rec(g_prof.on && ((g_prof.mask >> s) & 1u)) {
    if (rec) {
      a = g_ev.get();
      b = g_ev.get();
      (void)hipEventRecord(a, st);
    }
  }
  ~Timer() {
    if (rec) {
      (void)hipEventRecord(b, st);
      g_ev.pending.push_back({slot, a, b});
    }
  }
};

// Host-side description of one instance (a bound pattern) in a group.
template <typename T>
Inst inst_of_pattern(const lsh_pattern* p) {
  Inst in;
  char* base = p->dev_persist;
  in.phase = (const uint8_t*)(base + p->off_phase);
  in.dmat = (const void*)(base + p->off_dmat);
  in.cmat = (const double*)(base + p->off_cmat);
  in.nphase = p->nphase;
  in.pad_ = 0;
  double lam0 = 0.0, mu0 = 1.0;
  c0_isotropic(p, &lam0, &mu0);
  in.mu0 = mu0;
  in.riso = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0));
  return in;
}

// The load cases of one group and where their results go.
struct GroupSpec {
  const lsh_pattern* rep;             // geometry, kernel, twiddles, table
  std::vector<const lsh_pattern*> inst;
  std::vector<int> inst_of;           // per load
  std::vector<double> eps0_voigt;     // 6 per load
  std::vector<double*> sigma_out;     // per load: 6 doubles
  std::vector<lsh_stats*> stats;      // per load (may be null)
  std::vector<double*> history;       // per load: max_iter doubles (may be null)
  std::vector<const double*> einit;   // per load: device start field [ncf][m] (may be null)
  std::vector<double*> eout;          // per load: device field output [ncf][m] (may be null)
};

template <typename T>
struct GroupRun {
  GroupSpec spec;
  KernSet<T> K;
  Geo g;
  GreenParams gp;
  int gmode;
  int gmode3;  // the two-pass Green pass's operator form (twopass_green_mode)
  GroupWS w;
  int nload;
  dim3 gridS, gridS1, gridB, gridG;  // gridS1: the stress pass (its own tile width)
  int npos, nblkS;
  std::vector<int> chunks;  // Green chunks: (first load, end load) pairs
  std::vector<int> stop;
  std::vector<double> ring;
};

// Select candidate ch[pass] for each pass (stress, axis 2, Green pass) and the
// schedule ch[3] (0: four passes; i > 0: two-pass variant i - 1, if it holds a
// kernel for this Green mode).
template <typename T>
void apply_choice(KernSet<T>& K, int gmode, const int ch[4]) {
  if (!K.c1.empty()) {
    const auto& c = K.c1[std::min<size_t>((size_t)ch[0], K.c1.size() - 1)];
    K.a1s = c.fn;
    K.NT1s = c.nt;
    K.lds1s = c.lds;
    K.W1s = c.W;
  }
  if (!K.c2.empty()) {
    const auto& c = K.c2[std::min<size_t>((size_t)ch[1], K.c2.size() - 1)];
    K.a2[0] = c.fwd;
    K.a2[1] = c.inv;
    K.W2 = c.W;
    K.NT2 = c.nt;
    K.lds2 = c.lds;
  }
  if (K.green2 && !K.cg.empty()) {
    const auto* cp = &K.cg[std::min<size_t>((size_t)ch[2], K.cg.size() - 1)];
    if (!cp->fn[gmode]) cp = &K.cg[0];  // a variant without this Green mode: the default
    const auto& c = *cp;
    for (int m = 0; m < 4; ++m) K.gr2[m] = c.fn[m];
    K.gch = c.gch;
    K.NTG = c.nt;
    K.ldsG = c.lds;
  }
  if (K.green2) K.gr = K.gr2[gmode];
  else if (K.gr2[gmode]) K.gr = K.gr2[gmode];
  K.tpi = -1;
  if (ch[3] > 0 && !K.tp.empty()) {
    const int i = std::min<int>(ch[3], (int)K.tp.size()) - 1;
    if (K.tp[i].g3[gmode]) K.tpi = i;
  }
}

inline int prec_index(const lsh_pattern* p) { return p->bound_prec == LSH_FP32_MIXED ? 1 : 0; }

// Green chunks: runs of at most K.gch consecutive loads of one instance, and
// the Green pass's grid.
template <typename T>
void make_chunks(GroupRun<T>& G) {
  G.chunks.clear();
  for (int L = 0; L < G.nload;) {
    int e = L + 1;
    while (e < G.nload && e - L < G.K.gch && G.spec.inst_of[e] == G.spec.inst_of[L]) ++e;
    G.chunks.push_back(L);
    G.chunks.push_back(e);
    L = e;
  }
  G.gridG = G.K.green2 ? dim3(G.npos, (unsigned)(G.chunks.size() / 2)) : dim3((G.npos + 7) / 8 * 8 * G.nload);
}

template <typename T>
int group_prepare(GroupRun<T>& G, char* base, size_t avail, size_t* used) {
  const lsh_pattern* p = G.spec.rep;
  int rc = make_kernels<T>(p, p->has_table, &G.K);
  if (rc) return rc;
  G.gmode = green_mode(p);
  G.gmode3 = twopass_green_mode(p, G.gmode);
  {
    const int pi = prec_index(p);
    const int zero[4] = {0, 0, 0, 0};
    apply_choice(G.K, G.gmode, p->tuned[pi] ? p->tune_choice[pi] : zero);
  }
  if (G.K.tpi >= 0) {
    rc = allow_lds(G.K.tp[G.K.tpi].s2, G.K.tp[G.K.tpi].ldss);
    const bool inc = G.spec.rep->scheme == LSH_SCHEME_LS_INC;
    if (!rc) rc = allow_lds(G.K.tp[G.K.tpi].green(G.gmode3, inc), G.K.tp[G.K.tpi].ldsg);
    if (rc) return rc;
  }
  rc = allow_lds(G.K.gr, G.K.ldsG);
  if (rc) return rc;
  rc = allow_lds(G.K.a1s, G.K.lds1s);
  if (rc) return rc;
  rc = allow_lds(G.K.a2[0], G.K.lds2);
  if (rc) return rc;
  rc = allow_lds(G.K.a2[1], G.K.lds2);
  if (rc) return rc;
  G.g = geo_of(p);
  lsh_green_params(p, &G.gp);
  G.nload = (int)G.spec.inst_of.size();
  G.w = group_layout<T>(G.g, G.nload, (int)G.spec.inst.size(), G.K, base, p->scheme == LSH_SCHEME_CG);
  if (!base || avail < G.w.total) return lsh_fail(LSH_EWORKSPACE, "workspace too small");
  *used = G.w.total;
  const int nt3a = (G.g.n3 + G.K.W1 - 1) / G.K.W1;
  G.gridS = dim3(G.g.n2 * nt3a, G.nload);
  G.gridS1 = dim3(G.g.n2 * ((G.g.n3 + G.K.W1s - 1) / G.K.W1s), G.nload);
  const int nt3b = (G.g.n3 + G.K.W2 - 1) / G.K.W2;
  G.gridB = dim3(G.g.h1 * nt3b, 6, G.nload);
  G.npos = G.g.h1 * G.g.n2;
  make_chunks(G);
  G.nblkS = G.g.n2 * nt3a;
  return LSH_OK;
}

// Clear `bytes` (a multiple of 8) of device memory on `st` with a fill kernel.
int zero_async(void* ptr, size_t bytes, hipStream_t st) {
  const long long n = (long long)(bytes / 8);
  const int nblk = (int)std::min<long long>((n + 255) / 256, 4096);
  if (n > 0) hipLaunchKernelGGL(k_zero, dim3(nblk), dim3(256), 0, st, (unsigned long long*)ptr, n);
  HIPCHK(hipGetLastError());
  return LSH_OK;
}

// Upload per-load constants and clear the state (zero start) or transform a start field.
template <typename T>
int group_init(GroupRun<T>& G, int max_iter, hipStream_t st) {
  using T2 = C2<T>;
  const int nload = G.nload;
  std::vector<double> e0(6 * nload), e0sq(nload);
  for (int L = 0; L < nload; ++L) {
    double s = 0.0;
    for (int c = 0; c < 6; ++c) {
      const double v = G.spec.eps0_voigt[6 * L + c] * (c < 3 ? 1.0 : M_SQRT1_2);
      e0[6 * L + c] = v;
      s += v * v;
    }
    e0sq[L] = s * (double)G.g.m;
  }
  std::vector<Inst> ins;
  for (auto* q : G.spec.inst) ins.push_back(inst_of_pattern<T>(q));
  G.stop.assign(nload, max_iter);
  std::vector<int> zeros(nload, 0);
  const int zero2[2] = {0, 0};  // iteration counter, finished-block count
  HIPCHK(hipMemcpyAsync(G.w.eps0, e0.data(), sizeof(double) * 6 * nload, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(G.w.e0sq, e0sq.data(), sizeof(double) * nload, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(G.w.stop_iter, G.stop.data(), sizeof(int) * nload, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(G.w.nonfinite, zeros.data(), sizeof(int) * nload, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(G.w.itp, zero2, sizeof(zero2), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(G.w.inst_of, G.spec.inst_of.data(), sizeof(int) * nload, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(G.w.chunks, G.chunks.data(), sizeof(int) * G.chunks.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(G.w.insts, ins.data(), sizeof(Inst) * ins.size(), hipMemcpyHostToDevice, st));
  const size_t fb = sizeof(T2) * 6 * (size_t)nload * G.g.spec;
  const lsh_pattern* p = G.spec.rep;
  char* base = p->dev_persist;
  const T2* tw0 = (const T2*)(base + p->off_tw[0]);
  const T2* tw1 = (const T2*)(base + p->off_tw[1]);
  bool any_init = false;
  for (const double* e : G.spec.einit) any_init = any_init || e != nullptr;
  if (any_init) {
    // loads without a start field start from zero (a null entry)
    HIPCHK(hipMemcpyAsync(G.w.einit, G.spec.einit.data(), sizeof(double*) * nload, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_mean, dim3(nload, 6), dim3(1024), 0, st, (const double* const*)G.w.einit, (long long)G.g.m,
                       G.g.ncf, G.w.means);
    hipLaunchKernelGGL(G.K.a1[MODE_INIT], G.gridS, dim3(G.K.NT1), G.K.lds1, st, G.g, p->plan[0], tw0,
                       (const T2*)nullptr, (T2*)G.w.X, (const Inst*)G.w.insts, (const int*)G.w.inst_of, G.w.eps0,
                       (const int*)G.w.stop_iter, (const int*)G.w.itp, (const double* const*)G.w.einit,
                       (const double*)G.w.means, (double* const*)nullptr, (double*)nullptr);
    if (G.K.tpi >= 0)  // the two-pass state: split along axis 2 (lsh_twopass.hpp)
      twopass_to_split(G.g, G.K.tp[G.K.tpi].Q, tw1, (const T2*)G.w.X, (T2*)G.w.P[0], nload, st);
    else
      hipLaunchKernelGGL(G.K.a2[0], G.gridB, dim3(G.K.NT2), G.K.lds2, st, G.g, p->plan[1], tw1, (const T2*)G.w.X,
                         (T2*)G.w.P[0], (const int*)nullptr, (const int*)nullptr, (T)(1.0 / G.g.n2));
    HIPCHK(hipGetLastError());
  } else {
    int rc = zero_async(G.w.X, fb, st);
    if (!rc) rc = zero_async(G.w.P[0], fb, st);
    if (rc) return rc;
  }
  if (p->scheme == LSH_SCHEME_LS_INC) {
    // the increment scheme's X at iteration 0: the start state (in the layout
    // its stress pass reads) with eps0 in the mean bins; its stress pass then
    // takes eps0 = 0 throughout
    int rc = zero_async(G.w.eps0z, sizeof(double) * 6 * nload, st);
    if (rc) return rc;
    long long count = (long long)G.g.n2 * G.g.n3;  // the k1 = 0 plane
    if (G.K.tpi >= 0) {
      HIPCHK(hipMemcpyAsync(G.w.X, G.w.P[0], fb, hipMemcpyDeviceToDevice, st));
      count = (long long)(G.g.n2 / G.K.tp[G.K.tpi].Q) * G.g.n3;  // its q = 0 rows
    }
    const long long n = count * 6 * nload;
    hipLaunchKernelGGL(k_add_mean<T>, dim3((unsigned)std::min<long long>((n + 255) / 256, 8192)), dim3(256), 0, st,
                       (T2*)G.w.X, (long long)G.g.spec, count, (const double*)G.w.eps0, nload);
    HIPCHK(hipGetLastError());
  }
  G.ring.assign(LSH_HIST * nload, NAN);
  return LSH_OK;
}

// The Green pass's update rule for the pattern's scheme (UPD_*, lsh_common.hpp).
inline int upd_of(const lsh_pattern* p) {
  return p->scheme == LSH_SCHEME_VE ? UPD_VE : (p->scheme == LSH_SCHEME_LS_INC ? UPD_INC : UPD_LS);
}

// Enqueue one Basic Scheme iteration of the group; `cur` picks which P buffer
// holds the previous iterate.  In the increment scheme (LSH_SCHEME_LS_INC) X
// holds the increment of the state (at iteration 0 the start state with eps0
// in its mean bins), the stress pass takes eps0 = 0, the Green pass writes the
// increment into X, and the inverse axis-2 pass transforms it in place.
// The passes of one iteration, launched one by one.
template <typename T>
void launch_stress(GroupRun<T>& G, hipStream_t st) {
  using T2 = C2<T>;
  const lsh_pattern* p = G.spec.rep;
  const T2* tw0 = (const T2*)(p->dev_persist + p->off_tw[0]);
  const double* e0 = p->scheme == LSH_SCHEME_LS_INC ? G.w.eps0z : G.w.eps0;
  hipLaunchKernelGGL(G.K.a1s, G.gridS1, dim3(G.K.NT1s), G.K.lds1s, st, G.g, p->plan[0], tw0, (const T2*)G.w.X,
                     (T2*)G.w.TAU,
                     (const Inst*)G.w.insts, (const int*)G.w.inst_of, e0, (const int*)G.w.stop_iter,
                     (const int*)G.w.itp, (const double* const*)nullptr, (const double*)nullptr,
                     (double* const*)nullptr, (double*)nullptr);
}

template <typename T>
void launch_axis2(GroupRun<T>& G, int dir, const C2<T>* src, C2<T>* dst, hipStream_t st) {
  using T2 = C2<T>;
  const lsh_pattern* p = G.spec.rep;
  const T2* tw1 = (const T2*)(p->dev_persist + p->off_tw[1]);
  hipLaunchKernelGGL(G.K.a2[dir], G.gridB, dim3(G.K.NT2), G.K.lds2, st, G.g, p->plan[1], tw1, src, dst,
                     (const int*)G.w.stop_iter, (const int*)G.w.itp, (T)1);
}

template <typename T>
void launch_green(GroupRun<T>& G, int cur, hipStream_t st) {
  using T2 = C2<T>;
  const lsh_pattern* p = G.spec.rep;
  const T2* tw2 = (const T2*)(p->dev_persist + p->off_tw[2]);
  const T* table = p->has_table ? (const T*)(p->dev_persist + p->off_table) : nullptr;
  hipLaunchKernelGGL(G.K.gr, G.gridG, dim3(G.K.NTG), G.K.ldsG, st, G.g, p->plan[2], tw2, G.gp, (const T2*)G.w.TAU,
                     (const T2*)G.w.P[cur], (T2*)G.w.P[1 - cur], table, (const Inst*)G.w.insts,
                     (const int*)G.w.inst_of, (const int*)G.w.chunks, (const int*)G.w.stop_iter,
                     (const int*)G.w.itp, G.nload, G.npos, G.w.partial, G.K.lsG, G.gmode, upd_of(G.spec.rep),
                     (T2*)G.w.X);
}

// The two passes of the two-pass schedule: P[cur] -> TAU -> P[1 - cur].
template <typename T>
void launch_twopass(GroupRun<T>& G, int cur, int which, hipStream_t st) {
  using T2 = C2<T>;
  const lsh_pattern* p = G.spec.rep;
  const TwoPass<T>& c = G.K.tp[G.K.tpi];
  const T2* tw0 = (const T2*)(p->dev_persist + p->off_tw[0]);
  const T2* tw1 = (const T2*)(p->dev_persist + p->off_tw[1]);
  const T2* tw2 = (const T2*)(p->dev_persist + p->off_tw[2]);
  const bool inc = p->scheme == LSH_SCHEME_LS_INC;  // the stress pass reads the increment in X
  if (which & 1)
    hipLaunchKernelGGL(c.s2, dim3(c.P * (G.g.n3 / c.W), G.nload), dim3(c.nts), c.ldss, st, G.g, tw0, tw1,
                       (const T2*)(inc ? G.w.X : G.w.P[cur]), (T2*)G.w.TAU, (const Inst*)G.w.insts,
                       (const int*)G.w.inst_of, (const double*)(inc ? G.w.eps0z : G.w.eps0),
                       (const int*)G.w.stop_iter, (const int*)G.w.itp);
  if (which & 2) {
    const T* table = p->has_table ? (const T*)(p->dev_persist + p->off_table) : nullptr;
    hipLaunchKernelGGL(c.green(G.gmode3, inc), dim3(G.g.h1 * c.Q, (unsigned)(G.chunks.size() / 2)), dim3(c.ntg),
                       c.ldsg, st,
                       G.g, tw1, tw2, (const T2*)G.w.TAU, (const T2*)G.w.P[cur], (T2*)G.w.P[1 - cur], table,
                       (const Inst*)G.w.insts, (const int*)G.w.inst_of, (const int*)G.w.chunks,
                       (const int*)G.w.stop_iter, (const int*)G.w.itp, G.g.h1 * c.Q, G.w.partial, upd_of(p),
                       (T2*)G.w.X);
  }
}

// One Basic Scheme iteration of a group: stress (axis 1), axis 2, Green pass
// (axis 3), residual, inverse axis 2; or the two passes of the two-pass
// schedule and the residual.
template <typename T>
int group_iterate(GroupRun<T>& G, int cur, double tol, bool fixed, hipStream_t st) {
  using T2 = C2<T>;
  if (G.K.tpi >= 0) {
    const int Q = G.K.tp[G.K.tpi].Q;
    {
      Timer tm(0, st);
      launch_twopass<T>(G, cur, 1, st);
    }
    {
      Timer tm(2, st);
      launch_twopass<T>(G, cur, 2, st);
    }
    {
      // Parseval in the split domain: sum_y |E|^2 = n1 Q sum w(k1) |X'|^2
      Timer tm(3, st);
      hipLaunchKernelGGL(k_finalize_resid, dim3(G.nload), dim3(1024), 0, st, (const double*)G.w.partial,
                         G.g.h1 * Q, G.nload, (const double*)G.w.e0sq, (double)G.g.n1 * (double)Q, tol,
                         fixed ? 1 : 0, G.w.itp, G.w.stop_iter, G.w.hist, G.w.nonfinite);
    }
    HIPCHK(hipGetLastError());
    return LSH_OK;
  }
  const double pscale = (double)G.g.n1 * (double)G.g.n2;
  {
    Timer tm(0, st);
    launch_stress<T>(G, st);
  }
  {
    Timer tm(1, st);
    launch_axis2<T>(G, 0, (const T2*)G.w.TAU, (T2*)G.w.TAU, st);
  }
  {
    Timer tm(2, st);
    launch_green<T>(G, cur, st);
  }
  {
    Timer tm(4, st);
    const bool inc = G.spec.rep->scheme == LSH_SCHEME_LS_INC;
    launch_axis2<T>(G, 1, (const T2*)(inc ? G.w.X : G.w.P[1 - cur]), (T2*)G.w.X, st);
  }
  {
    // residual, stop flags and the iteration counter's advance
    Timer tm(3, st);
    hipLaunchKernelGGL(k_finalize_resid, dim3(G.nload), dim3(1024), 0, st, (const double*)G.w.partial, G.npos,
                       G.nload, (const double*)G.w.e0sq, pscale, tol, fixed ? 1 : 0, G.w.itp, G.w.stop_iter,
                       G.w.hist, G.w.nonfinite);
  }
  HIPCHK(hipGetLastError());
  return LSH_OK;
}

// Autotuner: time each candidate of each pass on the group's own data (after
// a zero-start init) and keep the fastest; the caller re-initialises the state.
template <typename T>
int tune_group(GroupRun<T>& G, hipStream_t st, int choice[4], int ncand[4], float ms[4][LSH_TUNE_MAX]) {
  using T2 = C2<T>;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int ch[4] = {0, 0, 0, 0};
  // "pass" 3 is the schedule: a whole four-pass iteration with the variants
  // chosen before, against each two-pass variant's iteration
  int ntp = 0;
  for (const auto& c : G.K.tp) ntp += c.g3[G.gmode3] ? 1 : 0;
  const int nc[4] = {(int)G.K.c1.size(), (int)G.K.c2.size(), G.K.green2 ? (int)G.K.cg.size() : 1,
                     1 + (ntp == (int)G.K.tp.size() ? ntp : 0)};
  int rc = LSH_OK;
  for (int pass = 0; pass < 4 && rc == LSH_OK; ++pass) {
    ncand[pass] = nc[pass];
    float best = 1e30f;
    int bi = 0;
    for (int c = 0; c < nc[pass] && c < LSH_TUNE_MAX && rc == LSH_OK; ++c) {
      if (pass == 2 && G.K.green2 && !G.K.cg[c].fn[G.gmode]) {
        ms[pass][c] = 0.f;  // this variant has no kernel for the pattern's Green mode
        continue;
      }
      ch[pass] = c;
      apply_choice(G.K, G.gmode, ch);
      if (pass == 2) {  // the variant's chunk size
        make_chunks(G);
        HIPCHK(hipMemcpyAsync(G.w.chunks, G.chunks.data(), sizeof(int) * G.chunks.size(), hipMemcpyHostToDevice, st));
      }
      const int nt3b = (G.g.n3 + G.K.W2 - 1) / G.K.W2;
      G.gridB = dim3(G.g.h1 * nt3b, 6, G.nload);
      G.gridS1 = dim3(G.g.n2 * ((G.g.n3 + G.K.W1s - 1) / G.K.W1s), G.nload);
      if (pass == 0) rc = allow_lds(G.K.a1s, G.K.lds1s);
      if (pass == 1) {
        rc = allow_lds(G.K.a2[0], G.K.lds2);
        if (!rc) rc = allow_lds(G.K.a2[1], G.K.lds2);
      }
      if (pass == 2) rc = allow_lds(G.K.gr, G.K.ldsG);
      if (pass == 3 && G.K.tpi >= 0) {
        rc = allow_lds(G.K.tp[G.K.tpi].s2, G.K.tp[G.K.tpi].ldss);
        const bool inc = G.spec.rep->scheme == LSH_SCHEME_LS_INC;
        if (!rc) rc = allow_lds(G.K.tp[G.K.tpi].green(G.gmode3, inc), G.K.tp[G.K.tpi].ldsg);
      }
      if (rc) break;
      auto run = [&]() {
        if (pass == 0) launch_stress<T>(G, st);
        if (pass == 1) {
          launch_axis2<T>(G, 0, (const T2*)G.w.TAU, (T2*)G.w.TAU, st);
          launch_axis2<T>(G, 1, (const T2*)G.w.P[1], (T2*)G.w.X, st);
        }
        if (pass == 2) launch_green<T>(G, 0, st);
        if (pass == 3) {
          if (G.K.tpi >= 0) {
            launch_twopass<T>(G, 0, 3, st);
          } else {
            launch_stress<T>(G, st);
            launch_axis2<T>(G, 0, (const T2*)G.w.TAU, (T2*)G.w.TAU, st);
            launch_green<T>(G, 0, st);
            launch_axis2<T>(G, 1, (const T2*)G.w.P[1], (T2*)G.w.X, st);
          }
        }
      };
      run();
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < 3; ++r) run();
      (void)hipEventRecord(e1, st);
      if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = lsh_fail(LSH_EDEVICE, "autotuner launch failed");
        break;
      }
      float t = 0.f;
      (void)hipEventElapsedTime(&t, e0, e1);
      t /= 3.f;
      ms[pass][c] = t;
      if (t < best) {
        best = t;
        bi = c;
      }
    }
    ch[pass] = bi;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  apply_choice(G.K, G.gmode, ch);
  make_chunks(G);
  HIPCHK(hipMemcpyAsync(G.w.chunks, G.chunks.data(), sizeof(int) * G.chunks.size(), hipMemcpyHostToDevice, st));
  const int nt3b = (G.g.n3 + G.K.W2 - 1) / G.K.W2;
  G.gridB = dim3(G.g.h1 * nt3b, 6, G.nload);
  G.gridS1 = dim3(G.g.n2 * ((G.g.n3 + G.K.W1s - 1) / G.K.W1s), G.nload);
  for (int i = 0; i < 4; ++i) choice[i] = ch[i];
  return LSH_OK;
}

// Copy the residual ring and stop flags back; returns true when every load stopped.
template <typename T>
int group_poll(GroupRun<T>& G, int done, int max_iter, hipStream_t st, bool* all_done) {
  HIPCHK(hipMemcpyAsync(G.ring.data(), G.w.hist, sizeof(double) * LSH_HIST * G.nload, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(G.stop.data(), G.w.stop_iter, sizeof(int) * G.nload, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const int first = std::max(0, done - LSH_HIST);
  for (int L = 0; L < G.nload; ++L) {
    double* h = G.spec.history[L];
    if (!h) continue;
    for (int j = first; j < done && j < G.stop[L]; ++j) h[j] = G.ring[(j % LSH_HIST) * G.nload + L];
  }
  bool all = true;
  for (int L = 0; L < G.nload; ++L) all = all && G.stop[L] <= done;
  *all_done = all;
  (void)max_iter;
  return LSH_OK;
}

// Final pass: sigma_bar at the last iterate (and E out), stats; returns a status.
template <typename T>
int group_finish(GroupRun<T>& G, int done, double tol, bool fixed, double secs, hipStream_t st) {
  using T2 = C2<T>;
  const lsh_pattern* p = G.spec.rep;
  char* base = p->dev_persist;
  const T2* tw0 = (const T2*)(base + p->off_tw[0]);
  std::vector<int> nonfin(G.nload, 0);
  HIPCHK(hipMemcpyAsync(nonfin.data(), G.w.nonfinite, sizeof(int) * G.nload, hipMemcpyDeviceToHost, st));
  if (G.K.tpi >= 0) {  // back to the four-pass layout X, from the buffer each load's last iteration wrote
    twopass_from_split(G.g, G.K.tp[G.K.tpi].Q, (const T2*)(base + p->off_tw[1]), (const T2*)G.w.P[0],
                       (const T2*)G.w.P[1], (T2*)G.w.X, (const int*)G.w.stop_iter, (const int*)G.w.itp, G.nload, st);
  } else if (p->scheme == LSH_SCHEME_LS_INC) {
    // X holds the last increment; the state is the P buffer each load's last
    // iteration wrote, back through the inverse axis-2 transform (every load)
    const long long n = (long long)G.g.spec * 6 * G.nload;
    hipLaunchKernelGGL(k_pick_parity<T>, dim3((unsigned)std::min<long long>((n + 255) / 256, 8192)), dim3(256), 0,
                       st, (const T2*)G.w.P[0], (const T2*)G.w.P[1], (T2*)G.w.TAU, (long long)G.g.spec, G.nload,
                       (const int*)G.w.stop_iter, (const int*)G.w.itp);
    hipLaunchKernelGGL(G.K.a2[1], G.gridB, dim3(G.K.NT2), G.K.lds2, st, G.g, p->plan[1],
                       (const T2*)(base + p->off_tw[1]), (const T2*)G.w.TAU, (T2*)G.w.X, (const int*)nullptr,
                       (const int*)nullptr, (T)1);
  }
  bool any_out = false;
  for (double* e : G.spec.eout) any_out = any_out || e != nullptr;
  if (any_out)
    HIPCHK(hipMemcpyAsync(G.w.eout, G.spec.eout.data(), sizeof(double*) * G.nload, hipMemcpyHostToDevice, st));
  {
    Timer tm(5, st);
    hipLaunchKernelGGL(G.K.a1[MODE_FINAL], G.gridS, dim3(G.K.NT1), G.K.lds1, st, G.g, p->plan[0], tw0,
                       (const T2*)G.w.X, (T2*)nullptr, (const Inst*)G.w.insts, (const int*)G.w.inst_of, G.w.eps0,
                       (const int*)G.w.stop_iter, (const int*)G.w.itp, (const double* const*)nullptr,
                       (const double*)nullptr, any_out ? (double* const*)G.w.eout : (double* const*)nullptr,
                       G.w.partial);
    hipLaunchKernelGGL(k_finalize_sum, dim3(G.nload, 6), dim3(256), 0, st, (const double*)G.w.partial, G.nblkS, 6,
                       1.0 / (double)G.g.m, G.w.sigma);
  }
  HIPCHK(hipGetLastError());
  std::vector<double> sig(6 * G.nload);
  HIPCHK(hipMemcpyAsync(sig.data(), G.w.sigma, sizeof(double) * 6 * G.nload, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (g_prof.on) g_ev.flush();
  int status = LSH_OK;
  for (int L = 0; L < G.nload; ++L) {
    for (int c = 0; c < 6; ++c) {
      const int bc = boundary_comp(c, G.g.ncf);
      if (bc >= 0) G.spec.sigma_out[L][bc] = sig[6 * L + c] * (c < 3 ? 1.0 : M_SQRT1_2);
    }
    const int its = std::min(G.stop[L], done);
    double last = NAN;
    if (its > 0) last = G.ring[((its - 1) % LSH_HIST) * G.nload + L];
    if (G.spec.history[L])
      for (int j = std::max(0, its - LSH_HIST); j < its; ++j)
        G.spec.history[L][j] = G.ring[(j % LSH_HIST) * G.nload + L];
    const bool conv = !fixed && std::isfinite(last) && last <= tol;
    if (G.spec.stats[L]) {
      G.spec.stats[L]->iterations = its;
      G.spec.stats[L]->converged = conv ? 1 : 0;
      G.spec.stats[L]->residual = last;
      G.spec.stats[L]->seconds = secs;
    }
    if (nonfin[L]) status = LSH_ENONFINITE;
    else if (!fixed && !conv && status == LSH_OK) status = LSH_ENOTCONVERGED;
  }
  return status;
}

// Run groups to convergence.  Without per-kernel profiling the iterations are
// captured once into a HIP graph (two iterations, one per ping-pong parity,
// all groups as independent branches) and the graph is replayed; the
// iteration counter and the stop flags live on the device, so a replay after
// a load has converged only runs early-exit blocks for it.
template <typename T>
int run_groups(std::vector<GroupRun<T>>& groups, double tol, int max_iter, hipStream_t st, bool graphs = true) {
  const bool fixed = tol < 0.0;
  for (auto& G : groups) {
    for (auto* h : G.spec.history)
      if (h)
        for (int j = 0; j < max_iter; ++j) h[j] = NAN;
    int rc = group_init<T>(G, max_iter, st);
    if (rc) return rc;
  }
  const int check = fixed ? 32 : 8;
  const auto t0 = std::chrono::steady_clock::now();
  int done = 0;
  bool use_graph = graphs && !g_prof.on && st != nullptr;
  hipGraphExec_t gexec = nullptr;
  if (use_graph) {
    // Each group's two iterations form a branch of its own (forked from and
    // joined to `st` through events on side streams), so the groups of a batch
    // are independent in the graph and the GPU may run one group's kernels
    // beside another's instead of strictly after them.
    const size_t ng = groups.size();
    std::vector<hipStream_t> side(ng > 1 ? ng : 0, nullptr);
    std::vector<hipEvent_t> join(side.size(), nullptr);
    hipEvent_t fork = nullptr;
    auto release = [&]() {
      for (auto& x : side)
        if (x) (void)hipStreamDestroy(x);
      for (auto& x : join)
        if (x) (void)hipEventDestroy(x);
      if (fork) (void)hipEventDestroy(fork);
    };
    int rc = LSH_OK;
    if (ng > 1) {
      hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
      for (size_t i = 0; i < ng && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
      }
      if (e != hipSuccess) {
        release();
        return lsh_fail(LSH_EDEVICE, std::string("graph branches: ") + hipGetErrorString(e));
      }
    }
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
      release();
      return lsh_fail(LSH_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    if (ng > 1) {
      e = hipEventRecord(fork, st);
      for (size_t i = 0; i < ng && e == hipSuccess && rc == LSH_OK; ++i) {
        e = hipStreamWaitEvent(side[i], fork, 0);
        for (int par = 0; par < 2 && e == hipSuccess && rc == LSH_OK; ++par)
          rc = group_iterate<T>(groups[i], par, tol, fixed, side[i]);
        if (e == hipSuccess && rc == LSH_OK) e = hipEventRecord(join[i], side[i]);
        if (e == hipSuccess && rc == LSH_OK) e = hipStreamWaitEvent(st, join[i], 0);
      }
    } else {
      for (int par = 0; par < 2 && rc == LSH_OK; ++par) rc = group_iterate<T>(groups[0], par, tol, fixed, st);
    }
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    release();
    if (rc) return rc;
    if (e != hipSuccess || ec != hipSuccess)
      return lsh_fail(LSH_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : ec));
    e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return lsh_fail(LSH_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  while (done < max_iter) {
    const int step = std::min(check, max_iter - done);
    int k = 0;
    for (; k < step; ++k) {
      if (use_graph && (done + k) % 2 == 0 && k + 1 < step) {
        hipError_t e = hipGraphLaunch(gexec, st);
        if (e != hipSuccess) {
          (void)hipGraphExecDestroy(gexec);
          return lsh_fail(LSH_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
        }
        ++k;  // the graph holds two iterations
      } else {
        for (auto& G : groups) {
          int rc = group_iterate<T>(G, (done + k) % 2, tol, fixed, st);
          if (rc) return rc;
        }
      }
    }
    done += k;
    bool all = true;
    for (auto& G : groups) {
      bool a = false;
      int rc = group_poll<T>(G, done, max_iter, st, &a);
      if (rc) return rc;
      all = all && a;
    }
    if (g_prof.on) g_ev.flush();
    if (all) break;
  }
  if (gexec) (void)hipGraphExecDestroy(gexec);
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int status = LSH_OK;
  for (auto& G : groups) {
    int rc = group_finish<T>(G, done, tol, fixed, secs, st);
    if (rc == LSH_ENONFINITE || (rc && status == LSH_OK)) status = rc;
  }
  if (status == LSH_ENONFINITE) return lsh_fail(status, "non-finite residual (NaN/Inf) in the iteration");
  if (status == LSH_ENOTCONVERGED) return lsh_fail(status, "max_iter reached before the Cauchy residual met tol");
  return status;
}

// Conjugate gradients for the Dirichlet kernel's system (scheme LSH_SCHEME_CG):
// one application of the operator per iteration through the usual passes
// (direction and stress, axis 2, Green pass, axis 2 inverse), with the vector
// updates and reductions in k_cg_update / k_cg_scalars / k_cg_alpha.  Buffers:
// x = X, z = EX[0], p = EX[1], W = -G C p = P[0], Green output P[1].
template <typename T>
int cg_iterate(GroupRun<T>& G, double tol, bool fixed, hipStream_t st) {
  using T2 = C2<T>;
  const lsh_pattern* p = G.spec.rep;
  char* base = p->dev_persist;
  const T2* tw0 = (const T2*)(base + p->off_tw[0]);
  const long long nblkU = (G.g.spec + 255) / 256;
  {
    Timer tm(3, st);
    hipLaunchKernelGGL(k_cg_update<T>, dim3((unsigned)nblkU, G.nload), dim3(256), 0, st, G.g, (const T2*)G.w.EX[1],
                       (const T2*)G.w.P[0], (T2*)G.w.X, (T2*)G.w.EX[0], (const double*)G.w.cg,
                       (const double*)G.w.C0m, (const int*)G.w.stop_iter, (const int*)G.w.itp, G.w.partial);
    hipLaunchKernelGGL(k_cg_scalars, dim3(G.nload), dim3(256), 0, st, (const double*)G.w.partial, (int)nblkU,
                       G.nload, (const double*)G.w.e0sq, (double)G.g.n1, tol, fixed ? 1 : 0, (const int*)G.w.itp,
                       G.w.stop_iter, G.w.hist, G.w.nonfinite, G.w.cg);
  }
  {
    Timer tm(0, st);
    hipLaunchKernelGGL(G.K.a1cg, G.gridS, dim3(G.K.NT1), G.K.lds1, st, G.g, p->plan[0], tw0, (const T2*)G.w.EX[0],
                       (T2*)G.w.EX[1], (T2*)G.w.TAU, (const Inst*)G.w.insts, (const int*)G.w.inst_of,
                       (const double*)G.w.cg, (const int*)G.w.stop_iter, (const int*)G.w.itp, G.w.partial);
    hipLaunchKernelGGL(k_cg_alpha, dim3(G.nload), dim3(256), 0, st, (const double*)G.w.partial, (int)G.nblkS,
                       (const int*)G.w.itp, (const int*)G.w.stop_iter, G.w.cg);
  }
  {
    Timer tm(1, st);
    launch_axis2<T>(G, 0, (const T2*)G.w.TAU, (T2*)G.w.TAU, st);
  }
  {
    Timer tm(2, st);
    launch_green<T>(G, 0, st);  // TAU -> P[1] (P[0] is read as the unused previous iterate)
  }
  {
    Timer tm(4, st);
    launch_axis2<T>(G, 1, (const T2*)G.w.P[1], (T2*)G.w.P[0], st);
  }
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, G.w.itp);
  HIPCHK(hipGetLastError());
  return LSH_OK;
}

template <typename T>
int run_cg(GroupRun<T>& G, double tol, int max_iter, hipStream_t st) {
  using T2 = C2<T>;
  const bool fixed = tol < 0.0;
  for (auto* h : G.spec.history)
    if (h)
      for (int j = 0; j < max_iter; ++j) h[j] = NAN;
  int rc = group_init<T>(G, max_iter, st);  // x = X: zero or the start field
  if (rc) return rc;
  const lsh_pattern* p = G.spec.rep;
  const size_t fb = sizeof(T2) * 6 * (size_t)G.nload * G.g.spec;
  double c0m[36];
  lsh_voigt_to_mandel(p->C0_voigt, c0m);
  std::vector<double> cg0(4 * G.nload, 0.0);
  HIPCHK(hipMemcpyAsync(G.w.C0m, c0m, sizeof(c0m), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(G.w.cg, cg0.data(), sizeof(double) * cg0.size(), hipMemcpyHostToDevice, st));
  rc = zero_async(G.w.EX[1], fb, st);           // p = 0
  if (!rc) rc = zero_async(G.w.P[0], fb, st);  // W = 0: the first update leaves x, z as they are
  if (rc) return rc;
  // z = -G C (x + eps0): the usual passes on x with dmat = C and eps0
  {
    const T2* tw0 = (const T2*)(p->dev_persist + p->off_tw[0]);
    hipLaunchKernelGGL(G.K.a1[MODE_STRESS], G.gridS, dim3(G.K.NT1), G.K.lds1, st, G.g, p->plan[0], tw0,
                       (const T2*)G.w.X, (T2*)G.w.TAU, (const Inst*)G.w.insts, (const int*)G.w.inst_of, G.w.eps0,
                       (const int*)G.w.stop_iter, (const int*)G.w.itp, (const double* const*)nullptr,
                       (const double*)nullptr, (double* const*)nullptr, (double*)nullptr);
    launch_axis2<T>(G, 0, (const T2*)G.w.TAU, (T2*)G.w.TAU, st);
    launch_green<T>(G, 0, st);
    launch_axis2<T>(G, 1, (const T2*)G.w.P[1], (T2*)G.w.EX[0], st);
    HIPCHK(hipGetLastError());
  }
  const int check = fixed ? 32 : 8;
  const auto t0 = std::chrono::steady_clock::now();
  int done = 0;
  while (done < max_iter) {
    const int step = std::min(check, max_iter - done);
    for (int k = 0; k < step; ++k) {
      rc = cg_iterate<T>(G, tol, fixed, st);
      if (rc) return rc;
    }
    done += step;
    bool all = false;
    rc = group_poll<T>(G, done, max_iter, st, &all);
    if (rc) return rc;
    if (g_prof.on) g_ev.flush();
    if (all) break;
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int status = group_finish<T>(G, done, tol, fixed, secs, st);
  if (status == LSH_ENONFINITE) return lsh_fail(status, "non-finite residual (NaN/Inf) in the iteration");
  if (status == LSH_ENOTCONVERGED) return lsh_fail(status, "max_iter reached before the Cauchy residual met tol");
  return status;
}

// The caller's macroscopic strain of load L (6 Voigt entries, or 3 for d = 2)
// as the internal six-entry Voigt vector.
void push_eps0(const lsh_pattern* p, const double* eps0_voigt, int L, std::vector<double>* out) {
  const int nc = p->d == 2 ? 3 : 6;
  for (int c = 0; c < 6; ++c) {
    const int bc = boundary_comp(c, nc);
    out->push_back(bc < 0 ? 0.0 : eps0_voigt[nc * L + bc]);
  }
}

template <typename T>
int solve_t(lsh_pattern* p, int nload, const double* eps0_voigt, double tol, int max_iter, void* dev_ws,
            size_t ws_bytes, hipStream_t st, const double* dev_E_init, double* dev_E_out, double* sigma_out,
            lsh_stats* stats, double* history, bool graphs = true) {
  std::vector<GroupRun<T>> groups(1);
  GroupSpec& S = groups[0].spec;
  S.rep = p;
  S.inst = {p};
  for (int L = 0; L < nload; ++L) {
    S.inst_of.push_back(0);
    push_eps0(p, eps0_voigt, L, &S.eps0_voigt);
    S.sigma_out.push_back(sigma_out + (p->d == 2 ? 3 : 6) * L);
    S.stats.push_back(stats ? stats + L : nullptr);
    S.history.push_back(history ? history + (long long)L * max_iter : nullptr);
    const long long fl = (long long)L * (p->d == 2 ? 3 : 6) * p->m;  // one load's [ncf][m] block
    S.einit.push_back(dev_E_init ? dev_E_init + fl : nullptr);
    S.eout.push_back(dev_E_out ? dev_E_out + fl : nullptr);
  }
  size_t used = 0;
  int rc = group_prepare<T>(groups[0], (char*)dev_ws, dev_ws ? ws_bytes : 0, &used);
  if (rc) return rc;
  if (p->scheme == LSH_SCHEME_CG) {
    if (!groups[0].K.a1cg) return lsh_fail(LSH_EUNSUPPORTED, "conjugate gradients: no kernel for this SNF grid");
    return run_cg<T>(groups[0], tol, max_iter, st);
  }
  return run_groups<T>(groups, tol, max_iter, st, graphs);
}

// Batched solve: tasks grouped by SNF grid, M and generating function.
bool same_group(const lsh_pattern* a, const lsh_pattern* b) {
  if (a->d != b->d) return false;
  for (int i = 0; i < 9; ++i)
    if (a->M[i] != b->M[i]) return false;
  if (a->kind != b->kind || a->R != b->R || a->nxi != b->nxi || a->scheme != b->scheme || a->tail != b->tail)
    return false;
  for (int i = 0; i < 3; ++i)
    if (a->alpha[i] != b->alpha[i]) return false;
  for (int i = 0; i < 3 * LSH_MAX_XI; ++i)
    if (a->Xi[i] != b->Xi[i]) return false;
  const int ga = green_mode(a), gb = green_mode(b);
  if (ga != gb) return false;
  if (ga == GREEN_GENERAL || ga == GREEN_TABLE)  // these depend on C0 (ISO and moments do not)
    for (int i = 0; i < 36; ++i)
      if (a->C0_voigt[i] != b->C0_voigt[i]) return false;
  return true;
}

template <typename T>
int build_groups(const lsh_task* tasks, int ntask, int max_iter, std::vector<GroupRun<T>>* out) {
  std::vector<GroupRun<T>>& groups = *out;
  for (int t = 0; t < ntask; ++t) {
    const lsh_task& tk = tasks[t];
    if (!tk.p || !tk.eps0_voigt || !tk.sigma_out || tk.nload < 1) return lsh_fail(LSH_EINVAL, "bad task " + std::to_string(t));
    for (int i = 0; i < (tk.p->d == 2 ? 3 : 6) * tk.nload; ++i)
      if (!std::isfinite(tk.eps0_voigt[i])) return lsh_fail(LSH_EINVAL, "non-finite macroscopic strain");
    size_t gi = 0;
    for (; gi < groups.size(); ++gi)
      if (same_group(groups[gi].spec.rep, tk.p)) break;
    if (gi == groups.size()) {
      groups.emplace_back();
      groups.back().spec.rep = tk.p;
    }
    GroupSpec& S = groups[gi].spec;
    const int ii = (int)S.inst.size();
    S.inst.push_back(tk.p);
    for (int L = 0; L < tk.nload; ++L) {
      S.inst_of.push_back(ii);
      push_eps0(tk.p, tk.eps0_voigt, L, &S.eps0_voigt);
      S.sigma_out.push_back(tk.sigma_out + (tk.p->d == 2 ? 3 : 6) * L);
      S.stats.push_back(tk.stats ? tk.stats + L : nullptr);
      S.history.push_back(nullptr);
      const long long fl = (long long)L * (tk.p->d == 2 ? 3 : 6) * tk.p->m;
      S.einit.push_back(tk.dev_E_init ? tk.dev_E_init + fl : nullptr);
      S.eout.push_back(tk.dev_E_out ? tk.dev_E_out + fl : nullptr);
    }
  }
  (void)max_iter;
  return LSH_OK;
}

template <typename T>
int batch_bytes_t(const lsh_task* tasks, int ntask, size_t* bytes) {
  std::vector<GroupRun<T>> groups;
  int rc = build_groups<T>(tasks, ntask, 1, &groups);
  if (rc) return rc;
  size_t tot = 0;
  for (auto& G : groups) {
    KernSet<T> K;
    rc = make_kernels<T>(G.spec.rep, kind_has_table(G.spec.rep), &K);
    if (rc) return rc;
    tot += group_layout<T>(geo_of(G.spec.rep), (int)G.spec.inst_of.size(), (int)G.spec.inst.size(), K, nullptr).total;
  }
  *bytes = tot;
  return LSH_OK;
}

template <typename T>
int solve_batch_t(const lsh_task* tasks, int ntask, double tol, int max_iter, void* dev_ws, size_t ws_bytes,
                  hipStream_t st) {
  std::vector<GroupRun<T>> groups;
  int rc = build_groups<T>(tasks, ntask, max_iter, &groups);
  if (rc) return rc;
  char* base = (char*)dev_ws;
  size_t left = dev_ws ? ws_bytes : 0;
  for (auto& G : groups) {
    size_t used = 0;
    rc = group_prepare<T>(G, base, left, &used);
    if (rc) return rc;
    base += used;
    left -= used;
  }
  return run_groups<T>(groups, tol, max_iter, st);
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
  if (p->has_table && green_mode(p) == GREEN_MOMENTS) {
    const T* table = (const T*)(p->dev_persist + p->off_table);
    double lam0 = 0.0, mu0 = 1.0;
    c0_isotropic(p, &lam0, &mu0);
    hipLaunchKernelGGL((k_moments_probe<T>), dim3((n + 127) / 128), dim3(128), 0, st, table, dout, dbins, n, g, mu0,
                       (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)));
  } else if (p->has_table) {
    const T* table = (const T*)(p->dev_persist + p->off_table);
    hipLaunchKernelGGL((k_cast_table<T>), dim3((n + 127) / 128), dim3(128), 0, st, table, dout, dbins, n, g);
  } else {
    double lam0 = 0.0, mu0 = 1.0;
    c0_isotropic(p, &lam0, &mu0);
    hipLaunchKernelGGL(k_gamma_probe, dim3((n + 127) / 128), dim3(128), 0, st, gp, dbins, n, dout,
                       green_mode(p), mu0,
                       (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)));
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
    KernSet<double> K;
    int rc = make_kernels<double>(p, kind_has_table(p), &K);
    if (rc) return rc;
    *bytes = group_layout<double>(geo_of(p), nload, 1, K, nullptr, p->scheme == LSH_SCHEME_CG).total;
  } else if (prec == LSH_FP32_MIXED) {
    KernSet<float> K;
    int rc = make_kernels<float>(p, kind_has_table(p), &K);
    if (rc) return rc;
    *bytes = group_layout<float>(geo_of(p), nload, 1, K, nullptr, p->scheme == LSH_SCHEME_CG).total;
  } else {
    return lsh_fail(LSH_EINVAL, "bad precision");
  }
  return LSH_OK;
}

// Argument checks shared by lsh_solve and lsh_solve_noalloc.
static int check_solve_args(const lsh_pattern* p, int nload, const double* eps0_voigt, double tol, int max_iter,
                            lsh_precision prec, const double* sigma_out) {
  if (!p || !eps0_voigt || !sigma_out) return lsh_fail(LSH_EINVAL, "null argument");
  if (nload < 1 || nload > 64) return lsh_fail(LSH_EINVAL, "nload must be in [1, 64]");
  if (max_iter < 1) return lsh_fail(LSH_EINVAL, "max_iter must be >= 1");
  if (!(tol == tol)) return lsh_fail(LSH_EINVAL, "tol is NaN");
  for (int i = 0; i < (p->d == 2 ? 3 : 6) * nload; ++i)
    if (!std::isfinite(eps0_voigt[i])) return lsh_fail(LSH_EINVAL, "non-finite macroscopic strain");
  if (p->kind < 0 || p->nphase < 1) return lsh_fail(LSH_ESTATE, "kernel or stiffness not set");
  if (p->bound_prec != (int)prec) return lsh_fail(LSH_ESTATE, "pattern not bound at this precision (lsh_bind)");
  if (p->scheme == LSH_SCHEME_CG && (p->kind != LSH_DIRICHLET || p->m % 2 == 0))
    return lsh_fail(LSH_EUNSUPPORTED, "conjugate gradients need the Dirichlet kernel on a pattern of odd m");
  return LSH_OK;
}

extern "C" int lsh_solve(lsh_pattern* p, int nload, const double* eps0_voigt, double tol, int max_iter,
                         lsh_precision prec, void* dev_ws, size_t ws_bytes, void* stream, const double* dev_E_init,
                         double* dev_E_out, double* sigma_out, lsh_stats* stats, double* history) {
  const int rc = check_solve_args(p, nload, eps0_voigt, tol, max_iter, prec, sigma_out);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (prec == LSH_FP64)
    return solve_t<double>(p, nload, eps0_voigt, tol, max_iter, dev_ws, ws_bytes, st, dev_E_init, dev_E_out,
                           sigma_out, stats, history);
  return solve_t<float>(p, nload, eps0_voigt, tol, max_iter, dev_ws, ws_bytes, st, dev_E_init, dev_E_out, sigma_out,
                        stats, history);
}

template <typename T>
int autotune_t(lsh_pattern* p, int nload, void* dev_ws, size_t ws_bytes, hipStream_t st, lsh_tune_result* out) {
  std::vector<GroupRun<T>> groups(1);
  GroupRun<T>& G = groups[0];
  GroupSpec& S = G.spec;
  S.rep = p;
  S.inst = {p};
  std::vector<double> sig(6 * (size_t)nload);
  for (int L = 0; L < nload; ++L) {
    S.inst_of.push_back(0);
    for (int c = 0; c < 6; ++c) S.eps0_voigt.push_back(c == L % 6 ? 1.0 : 0.0);
    S.sigma_out.push_back(sig.data() + 6 * L);
    S.stats.push_back(nullptr);
    S.history.push_back(nullptr);
  }
  const int pi = prec_index(p);
  p->tuned[pi] = 0;  // time every candidate from the defaults
  size_t used = 0;
  int rc = group_prepare<T>(G, (char*)dev_ws, dev_ws ? ws_bytes : 0, &used);
  if (rc) return rc;
  rc = group_init<T>(G, 1, st);
  if (rc) return rc;
  int choice[4] = {0, 0, 0, 0}, ncand[4] = {1, 1, 1, 1};
  float ms[4][LSH_TUNE_MAX] = {{0}};
  rc = tune_group<T>(G, st, choice, ncand, ms);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(st));
  p->tuned[pi] = 1;
  for (int i = 0; i < 4; ++i) p->tune_choice[pi][i] = choice[i];
  if (out) {
    for (int i = 0; i < 4; ++i) {
      out->choice[i] = choice[i];
      out->ncand[i] = ncand[i];
      for (int c = 0; c < LSH_TUNE_MAX; ++c) out->ms[i][c] = c < ncand[i] ? ms[i][c] : 0.f;
    }
  }
  return LSH_OK;
}

extern "C" int lsh_autotune(lsh_pattern* p, int nload, lsh_precision prec, void* dev_ws, size_t ws_bytes,
                            void* stream, lsh_tune_result* out) {
  if (!p) return lsh_fail(LSH_EINVAL, "null pattern");
  if (nload < 1 || nload > 64) return lsh_fail(LSH_EINVAL, "nload must be in [1, 64]");
  if (p->kind < 0 || p->nphase < 1) return lsh_fail(LSH_ESTATE, "kernel or stiffness not set");
  if (p->bound_prec != (int)prec) return lsh_fail(LSH_ESTATE, "pattern not bound at this precision (lsh_bind)");
  hipStream_t st = (hipStream_t)stream;
  if (prec == LSH_FP64) return autotune_t<double>(p, nload, dev_ws, ws_bytes, st, out);
  return autotune_t<float>(p, nload, dev_ws, ws_bytes, st, out);
}

extern "C" int lsh_tune_set(lsh_pattern* p, lsh_precision prec, const int* choice) {
  if (!p || !choice) return lsh_fail(LSH_EINVAL, "null argument");
  if (prec != LSH_FP64 && prec != LSH_FP32_MIXED) return lsh_fail(LSH_EINVAL, "bad precision");
  for (int i = 0; i < 4; ++i)
    if (choice[i] < 0 || choice[i] >= LSH_TUNE_MAX) return lsh_fail(LSH_EINVAL, "variant index out of range");
  const int pi = prec == LSH_FP32_MIXED ? 1 : 0;
  for (int i = 0; i < 4; ++i) p->tune_choice[pi][i] = choice[i];
  p->tuned[pi] = 1;
  return LSH_OK;
}

extern "C" int lsh_tune_reset(lsh_pattern* p) {
  if (!p) return lsh_fail(LSH_EINVAL, "null pattern");
  p->tuned[0] = p->tuned[1] = 0;
  return LSH_OK;
}

extern "C" int lsh_profile_enable(int on) {
  g_prof = Profile();
  g_prof.on = on != 0;
  return LSH_OK;
}

extern "C" int lsh_profile_select(unsigned mask) {
  g_prof.mask = mask;
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

extern "C" int lsh_batch_bytes(const lsh_task* tasks, int ntask, lsh_precision prec, size_t* bytes) {
  if (!tasks || ntask < 1 || !bytes) return lsh_fail(LSH_EINVAL, "bad argument");
  for (int t = 0; t < ntask; ++t)
    if (!tasks[t].p || tasks[t].p->kind < 0) return lsh_fail(LSH_ESTATE, "task pattern without a kernel");
  if (prec == LSH_FP64) return batch_bytes_t<double>(tasks, ntask, bytes);
  if (prec == LSH_FP32_MIXED) return batch_bytes_t<float>(tasks, ntask, bytes);
  return lsh_fail(LSH_EINVAL, "bad precision");
}

extern "C" int lsh_solve_batch(const lsh_task* tasks, int ntask, double tol, int max_iter, lsh_precision prec,
                               void* dev_ws, size_t ws_bytes, void* stream) {
  if (!tasks || ntask < 1) return lsh_fail(LSH_EINVAL, "bad argument");
  if (max_iter < 1) return lsh_fail(LSH_EINVAL, "max_iter must be >= 1");
  if (!(tol == tol)) return lsh_fail(LSH_EINVAL, "tol is NaN");
  for (int t = 0; t < ntask; ++t) {
    const lsh_pattern* p = tasks[t].p;
    if (!p || p->kind < 0 || p->nphase < 1) return lsh_fail(LSH_ESTATE, "task pattern without kernel or stiffness");
    if (p->bound_prec != (int)prec) return lsh_fail(LSH_ESTATE, "task pattern not bound at this precision");
    if (p->scheme == LSH_SCHEME_CG) return lsh_fail(LSH_EUNSUPPORTED, "conjugate gradients run through lsh_solve only");
  }
  hipStream_t st = (hipStream_t)stream;
  if (prec == LSH_FP64) return solve_batch_t<double>(tasks, ntask, tol, max_iter, dev_ws, ws_bytes, st);
  if (prec == LSH_FP32_MIXED) return solve_batch_t<float>(tasks, ntask, tol, max_iter, dev_ws, ws_bytes, st);
  return lsh_fail(LSH_EINVAL, "bad precision");
}

// ------------------------------------------------ allocation-free solve ---
// The workspace of lsh_solve_noalloc: a fixed device array, one per GPU the
// library runs on, held until the process ends.  Host code never passes the
// array's name to a kernel or a copy (on the host it is only a stand-in
// symbol): it uses the device address hipGetSymbolAddress returns, looked up
// once per device with that device current.
static __device__ __align__(256) unsigned char scratch[LSH_NOALLOC_MAX_BYTES];

#define LSH_NOALLOC_MAX_DEVICES 64
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[LSH_NOALLOC_MAX_DEVICES];  // per device, null until looked up

static int scratch_address(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= LSH_NOALLOC_MAX_DEVICES) return lsh_fail(LSH_EUNSUPPORTED, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return lsh_fail(LSH_EDEVICE, std::string("scratch address lookup failed: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LSH_OK;
}

extern "C" int lsh_solve_noalloc(lsh_pattern* p, int nload, const double* eps0_voigt, double tol, int max_iter,
                                 lsh_precision prec, void* stream, const double* dev_E_init, double* dev_E_out,
                                 double* sigma_out, lsh_stats* stats, double* history) {
  int rc = check_solve_args(p, nload, eps0_voigt, tol, max_iter, prec, sigma_out);
  if (rc) return rc;
  size_t need = 0;
  rc = lsh_solve_bytes(p, nload, prec, &need);
  if (rc) return rc;
  if (need > (size_t)LSH_NOALLOC_MAX_BYTES)
    return lsh_fail(LSH_EWORKSPACE, "lsh_solve_noalloc: this solve needs " + std::to_string(need) +
                                        " bytes of workspace; the allocation-free entry point holds at most " +
                                        std::to_string((size_t)LSH_NOALLOC_MAX_BYTES) + " (use lsh_solve)");
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  // launches are issued one by one: no graph is instantiated (that would allocate)
  if (prec == LSH_FP64)
    return solve_t<double>(p, nload, eps0_voigt, tol, max_iter, ws, need, st, dev_E_init, dev_E_out, sigma_out, stats,
                           history, false);
  return solve_t<float>(p, nload, eps0_voigt, tol, max_iter, ws, need, st, dev_E_init, dev_E_out, sigma_out, stats,
                        history, false);
}
