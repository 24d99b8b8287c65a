// lsh_unet.hip -- U-Net warm start for the Basic Scheme: MFMA bf16 kernels and the
// host-side network (forward, backward, Adam) behind include/lsh_unet.h.
//
// Activations are channels-last bf16 ([z][y][x][channel], a buffer may hold
// several layers' channels side by side: a layer reads or writes the slice
// [off, off + C) of a row of `cs` channels).  3x3x3 convolutions use periodic
// padding (the unit cell is periodic).  A convolution is an implicit GEMM
//   out[p][n] = sum_{tap, k} in[p + d_tap][k] * w[tap][n][k]
// on v_mfma_f32_16x16x32_bf16 (A: 8 consecutive k of one row per lane, B: 8
// consecutive k of one column, D: 4 rows of one column).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "lsh.h"
#include "lsh_unet.h"

int lsh_fail(int status, const std::string& msg);
size_t lsh_align(size_t x);

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

__device__ __forceinline__ u16 f2bf(float f) {
  // round to nearest even
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ __forceinline__ bf16x8 ld8(const u16* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  bf16x8 r;
  memcpy(&r, &v, 16);
  return r;
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// -------------------------------------------------------------- conv GEMM ---
// Block: 4 waves; wave w takes 32 voxels (two 16-row tiles) x 32 output
// channels (two 16-column tiles).  flip = 1 uses -d_tap (backward data).
__global__ void __launch_bounds__(256) k_conv(const u16* __restrict__ in, int in_cs, int in_off, int K,
                                              const u16* __restrict__ wt, int N, const float* __restrict__ bias,
                                              int ks, int flip, u16* __restrict__ out_bf, float* __restrict__ out_f,
                                              int out_cs, int out_off, int relu, int D, int H, int W) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int V = D * H * W;
  const int m0 = blockIdx.x * 128 + wave * 32;
  const int n0 = blockIdx.y * 32;
  const int r = lane & 15, g = lane >> 4;
  int pz[2], py[2], px[2];
  bool ok[2];
  for (int mi = 0; mi < 2; ++mi) {
    const int p = m0 + 16 * mi + r;
    ok[mi] = p < V;
    const int pp = ok[mi] ? p : 0;
    px[mi] = pp % W;
    py[mi] = (pp / W) % H;
    pz[mi] = pp / (W * H);
  }
  f4 acc[2][2];
  for (int mi = 0; mi < 2; ++mi)
    for (int nj = 0; nj < 2; ++nj) acc[mi][nj] = f4{0, 0, 0, 0};
  const int ntap = ks * ks * ks;
  const int c = ks / 2;
  for (int t = 0; t < ntap; ++t) {
    int dz = t / (ks * ks) - c, dy = (t / ks) % ks - c, dx = t % ks - c;
    if (flip) {
      dz = -dz;
      dy = -dy;
      dx = -dx;
    }
    const u16* ain[2];
    for (int mi = 0; mi < 2; ++mi) {
      const int q = (wrap(pz[mi] + dz, D) * H + wrap(py[mi] + dy, H)) * W + wrap(px[mi] + dx, W);
      ain[mi] = in + (long long)q * in_cs + in_off + 8 * g;
    }
    const u16* wb = wt + ((long long)t * N + n0 + r) * K + 8 * g;
    for (int k0 = 0; k0 < K; k0 += 32) {
      bf16x8 a[2], b[2];
      for (int mi = 0; mi < 2; ++mi) a[mi] = ld8(ain[mi] + k0);
      for (int nj = 0; nj < 2; ++nj) b[nj] = ld8(wb + (long long)16 * nj * K + k0);
      for (int mi = 0; mi < 2; ++mi)
        for (int nj = 0; nj < 2; ++nj)
          acc[mi][nj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mi], b[nj], acc[mi][nj], 0, 0, 0);
    }
  }
  for (int mi = 0; mi < 2; ++mi)
    for (int nj = 0; nj < 2; ++nj) {
      const int ch = n0 + 16 * nj + r;
      const float bv = bias ? bias[ch] : 0.0f;
      for (int i = 0; i < 4; ++i) {
        const int p = m0 + 16 * mi + 4 * g + i;
        if (p >= V) continue;
        float v = acc[mi][nj][i] + bv;
        if (relu) v = fmaxf(v, 0.0f);
        if (out_f)
          out_f[(long long)p * out_cs + out_off + ch] = v;
        else
          out_bf[(long long)p * out_cs + out_off + ch] = f2bf(v);
      }
    }
}

// The same convolution with the input staged in LDS.  Block: an 8 x 2MT x 4
// (x, y, z) tile of output voxels and 16 NTL output channels; per chunk of 32
// input channels its 10 x (2MT + 2) x 6 halo (periodic; for 1x1 kernels the
// tile itself) comes into LDS once, and the 27 taps read their A fragments
// there instead of from the cache hierarchy (the global version re-reads every
// input row once per tap).
// Wave w takes the tile's voxels v = x + 8 y + 16 MT z in [16 MT w, 16 MT (w
// + 1)): MT row tiles of 16 (8 x 2 at one z) against the block's channels.
// Needs W % 8 == 0, H % (2 MT) == 0, D % 4 == 0.
// u16 per halo voxel: its 32 channels, unpadded (37.5 KB per block, so four
// blocks share a CU; padding to 40 spread the banks but, at 46.9 KB, allowed
// only three, and was slower: 2.71 against 2.58 ms per 128^3 prediction)
constexpr int HROW = 32;
template <int MT, int KS>
constexpr int halo_u16() {
  return (8 + KS - 1) * (2 * MT + KS - 1) * (4 + KS - 1) * HROW;
}

// Where an LDS-staged convolution reads its input.  Channel k of voxel p is
// in[p cs + off + k], except that
//   phase != null: the network's packed input (channel 0 the phase
//                  indicator 0/1, channels 1..31 zero), formed from the phase
//                  map as it is staged;
//   k < up_C:      the channel comes from the grid of half the side at p's
//                  parent, up[parent up_cs + k] (nearest upsampling, read in
//                  place instead of being copied out first).
struct ConvIn {
  const u16* in;
  int cs, off;
  const u16* up;
  int up_cs, up_C;
  const uint8_t* phase;
};
__host__ __device__ inline ConvIn plain_in(const u16* in, int cs, int off) {
  return ConvIn{in, cs, off, nullptr, 0, 0, nullptr};
}

// The tile's accumulation: acc[mi][nj][i] is output channel n0 + 16 nj + r of
// tile voxel 16 MT wave + 16 mi + 4 g + i (r = lane % 16, g = lane / 16).
template <int MT, int NTL, int KS>
__device__ __forceinline__ void conv_lds_tile(const ConvIn& src, int K,
                                              const u16* __restrict__ wt, int N, int flip, int D, int H, int W,
                                              int x0, int y0, int z0, int n0, u16* halo, f4 (&acc)[MT][NTL]) {
  constexpr int c = KS / 2;
  constexpr int TY = 2 * MT, HX = 8 + 2 * c, HY = TY + 2 * c, HZ = 4 + 2 * c, HV = HX * HY * HZ;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  // this lane's voxel in each of the wave's row tiles
  int vx[MT], vy[MT], vz[MT];
#pragma unroll
  for (int mi = 0; mi < MT; ++mi) {
    const int v = 16 * MT * wave + 16 * mi + r;
    vx[mi] = v & 7;
    vy[mi] = (v >> 3) % TY;
    vz[mi] = v / (8 * TY);
  }
#pragma unroll
  for (int mi = 0; mi < MT; ++mi)
#pragma unroll
    for (int nj = 0; nj < NTL; ++nj) acc[mi][nj] = f4{0, 0, 0, 0};
  constexpr int ntap = KS * KS * KS;
  for (int k0 = 0; k0 < K; k0 += 32) {
    // halo voxel h = hx + HX (hy + HY hz) <- input voxel (x0 - c + hx, y0 - c + hy, z0 - c + hz), periodic
    for (int sgm = tid; sgm < HV * 4; sgm += 256) {
      const int h = sgm >> 2, part = sgm & 3;
      const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
      const int zf = wrap(z0 - c + hz, D), yf = wrap(y0 - c + hy, H), xf = wrap(x0 - c + hx, W);
      const int q = (zf * H + yf) * W + xf;
      uint4 val;
      if (src.phase) {
        val = uint4{part == 0 && src.phase[q] ? 0x3F80u : 0u, 0u, 0u, 0u};  // bf16 1.0 in channel 0
      } else if (k0 < src.up_C) {
        const int qc = ((zf >> 1) * (H >> 1) + (yf >> 1)) * (W >> 1) + (xf >> 1);
        val = *reinterpret_cast<const uint4*>(src.up + (long long)qc * src.up_cs + k0 + 8 * part);
      } else {
        val = *reinterpret_cast<const uint4*>(src.in + (long long)q * src.cs + src.off + k0 + 8 * part);
      }
      *reinterpret_cast<uint4*>(halo + h * HROW + 8 * part) = val;
    }
    __syncthreads();
#pragma unroll 3
    for (int t = 0; t < ntap; ++t) {
      int dz = t / (KS * KS) - c, dy = (t / KS) % KS - c, dx = t % KS - c;
      if (flip) {
        dz = -dz;
        dy = -dy;
        dx = -dx;
      }
      bf16x8 a[MT], b[NTL];
#pragma unroll
      for (int mi = 0; mi < MT; ++mi) {
        const int h = (vx[mi] + c + dx) + HX * ((vy[mi] + c + dy) + HY * (vz[mi] + c + dz));
        a[mi] = ld8(halo + h * HROW + 8 * g);
      }
      const u16* wb = wt + ((long long)t * N + n0 + r) * K + k0 + 8 * g;
#pragma unroll
      for (int nj = 0; nj < NTL; ++nj) b[nj] = ld8(wb + (long long)16 * nj * K);
#pragma unroll
      for (int mi = 0; mi < MT; ++mi)
#pragma unroll
        for (int nj = 0; nj < NTL; ++nj)
          acc[mi][nj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mi], b[nj], acc[mi][nj], 0, 0, 0);
    }
    __syncthreads();  // the next chunk (or the caller's epilogue) overwrites the halo
  }
}

// grid point of tile voxel v = x + 8 y + 16 MT z of the tile at (x0, y0, z0)
template <int MT>
__device__ __forceinline__ long long tile_point(int v, int x0, int y0, int z0, int H, int W) {
  constexpr int TY = 2 * MT;
  return ((long long)(z0 + v / (8 * TY)) * H + y0 + (v >> 3) % TY) * W + x0 + (v & 7);
}

template <int MT, int NTL, int KS>
__global__ void __launch_bounds__(256) k_conv_lds(ConvIn src, int K,
                                                  const u16* __restrict__ wt, int N, const float* __restrict__ bias,
                                                  int flip, u16* __restrict__ out_bf,
                                                  float* __restrict__ out_f, int out_cs, int out_off, int relu, int D,
                                                  int H, int W) {
  constexpr int TY = 2 * MT;
  __shared__ __align__(16) u16 halo[halo_u16<MT, KS>()];
  const int tx = W / 8, ty = H / TY;
  const int x0 = 8 * (blockIdx.x % tx), y0 = TY * ((blockIdx.x / tx) % ty), z0 = 4 * (blockIdx.x / (tx * ty));
  const int n0 = blockIdx.y * 16 * NTL;
  f4 acc[MT][NTL];
  conv_lds_tile<MT, NTL, KS>(src, K, wt, N, flip, D, H, W, x0, y0, z0, n0, halo, acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int mi = 0; mi < MT; ++mi)
#pragma unroll
    for (int nj = 0; nj < NTL; ++nj) {
      const int ch = n0 + 16 * nj + r;
      const float bv = bias ? bias[ch] : 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // row 4 g + i of the row tile: the voxel the lane with r = 4 g + i holds
        const long long p = tile_point<MT>(16 * MT * wave + 16 * mi + 4 * g + i, x0, y0, z0, H, W);
        float val = acc[mi][nj][i] + bv;
        if (relu) val = fmaxf(val, 0.0f);
        if (out_f)
          out_f[p * out_cs + out_off + ch] = val;
        else
          out_bf[p * out_cs + out_off + ch] = f2bf(val);
      }
    }
}

// The head (1x1 convolution, 32 -> 64 channels, no activation) fused with the
// strain contraction of a prediction:
//   E[L][c][p] = (c < 3 ? 1 : sqrt2) sum_j eps0[L][j] y[p][6 j + c],
// y = the head's output channels 0..35 (unit load j, Mandel component c).  A
// block takes the conv tile of 8 x 8 x 4 voxels and output channels 0..47
// (three 16-column tiles cover the 36 used); its y rows (FP32, padded to 37
// words so that a wave reading one channel of 64 voxels hits distinct banks)
// go through LDS (the buffer that held the input tile), and each thread then
// forms one voxel's nload x 6 outputs, summed over j in ascending order in
// FP64.  y itself is not stored.
constexpr int YROW = 37;
static_assert(256 * YROW * 4 >= halo_u16<4, 1>() * 2, "the input tile fits the y buffer");
__global__ void __launch_bounds__(256) k_head_contract(const u16* __restrict__ in, int in_cs, int in_off,
                                                       const u16* __restrict__ wt, const float* __restrict__ bias,
                                                       const double* __restrict__ eps0, int nload,
                                                       double* __restrict__ E, int D, int H, int W) {
  constexpr int MT = 4, NTL = 3, TY = 2 * MT;
  __shared__ __align__(16) float ys[256 * YROW];
  const int tx = W / 8, ty = H / TY;
  const int x0 = 8 * (blockIdx.x % tx), y0 = TY * ((blockIdx.x / tx) % ty), z0 = 4 * (blockIdx.x / (tx * ty));
  f4 acc[MT][NTL];
  // the input tile's LDS is free again when the tile returns (it ends with a barrier)
  conv_lds_tile<MT, NTL, 1>(plain_in(in, in_cs, in_off), 32, wt, 64, 0, D, H, W, x0, y0, z0, 0,
                            reinterpret_cast<u16*>(ys), acc);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int mi = 0; mi < MT; ++mi)
#pragma unroll
    for (int nj = 0; nj < NTL; ++nj) {
      const int ch = 16 * nj + r;
      if (ch < 36) {
        const float bv = bias[ch];
#pragma unroll
        for (int i = 0; i < 4; ++i) ys[(16 * MT * wave + 16 * mi + 4 * g + i) * YROW + ch] = acc[mi][nj][i] + bv;
      }
    }
  __syncthreads();
  const long long V = (long long)D * H * W;
  const long long p = tile_point<MT>(tid, x0, y0, z0, H, W);
  const float* yv = ys + tid * YROW;
  for (int L = 0; L < nload; ++L)
    for (int c = 0; c < 6; ++c) {
      double s = 0.0;
      for (int j = 0; j < 6; ++j) s += eps0[6 * L + j] * (double)yv[6 * j + c];
      E[(long long)(6 * L + c) * V + p] = s * (c < 3 ? 1.0 : 1.41421356237309504880);
    }
}

// Whether a convolution on an n^3 grid with ks^3 taps runs LDS-staged (the
// grid tiles into its 8 x 8 x 4 voxel blocks).
bool lds_conv(int n, int ks) { return n % 8 == 0 && (ks == 3 || ks == 1); }

// Both convolutions behind one call: the LDS-staged one where lds_conv holds
// (64 output channels per block when N allows and the layer still has 2048
// blocks, so the halo is staged once for them, else 32), the global one
// elsewhere (the coarsest levels of small grids), which reads plain inputs only.
void launch_conv(const ConvIn& src, int K, const u16* wt, int N, const float* bias, int ks, int flip, u16* out_bf,
                 float* out_f, int out_cs, int out_off, int relu, int n, hipStream_t st) {
  const long long V = (long long)n * n * n;
  const bool lds = lds_conv(n, ks);
  const bool wide = N % 64 == 0 && (V / 256) * (N / 64) >= 2048;
  const dim3 grid((unsigned)(V / 256), wide ? N / 64 : N / 32);
  if (lds && wide && ks == 3)
    hipLaunchKernelGGL((k_conv_lds<4, 4, 3>), grid, dim3(256), 0, st, src, K, wt, N, bias, flip, out_bf, out_f, out_cs,
                       out_off, relu, n, n, n);
  else if (lds && wide)
    hipLaunchKernelGGL((k_conv_lds<4, 4, 1>), grid, dim3(256), 0, st, src, K, wt, N, bias, flip, out_bf, out_f, out_cs,
                       out_off, relu, n, n, n);
  else if (lds && ks == 3)
    hipLaunchKernelGGL((k_conv_lds<4, 2, 3>), grid, dim3(256), 0, st, src, K, wt, N, bias, flip, out_bf, out_f, out_cs,
                       out_off, relu, n, n, n);
  else if (lds)
    hipLaunchKernelGGL((k_conv_lds<4, 2, 1>), grid, dim3(256), 0, st, src, K, wt, N, bias, flip, out_bf, out_f, out_cs,
                       out_off, relu, n, n, n);
  else
    hipLaunchKernelGGL(k_conv, dim3((unsigned)((V + 127) / 128), N / 32), dim3(256), 0, st, src.in, src.cs, src.off, K,
                       wt, N, bias, ks, flip, out_bf, out_f, out_cs, out_off, relu, n, n, n);
}

// -------------------------------------------------------- weight gradient ---
// dW[t][co][ci] += sum_p dout[p][co] * in[p + d_t][ci]; block tile 32 co x 32 ci,
// a chunk of voxels per block (atomics across chunks).  Voxel tiles of 32 are
// staged in LDS transposed so each lane reads 8 consecutive voxels at once.
__global__ void __launch_bounds__(256) k_conv_wgrad(const u16* __restrict__ dout, int do_cs, int do_off, int Cout,
                                                    const u16* __restrict__ in, int in_cs, int in_off, int Cin, int ks,
                                                    float* __restrict__ dW, int D, int H, int W, int chunk) {
  __shared__ __align__(16) u16 As[32][40];  // [co][voxel], padded rows
  __shared__ __align__(16) u16 Bs[32][40];  // [ci][voxel]
  const int V = D * H * W;
  const int t = blockIdx.y;
  const int ntco = Cout / 32;
  const int co0 = (blockIdx.z % ntco) * 32, ci0 = (blockIdx.z / ntco) * 32;
  const int c = ks / 2;
  const int dz = t / (ks * ks) - c, dy = (t / ks) % ks - c, dx = t % ks - c;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int wm = (wave >> 1) * 16, wn = (wave & 1) * 16;
  f4 acc = f4{0, 0, 0, 0};
  const int p_begin = blockIdx.x * chunk;
  const int p_end = min(V, p_begin + chunk);
  // staging: thread -> (voxel v = tid / 8, 4 channels at 4 * (tid % 8))
  const int sv = threadIdx.x >> 3, sc = (threadIdx.x & 7) * 4;
  for (int p0 = p_begin; p0 < p_end; p0 += 32) {
    const int p = p0 + sv;
    uint2 va = make_uint2(0, 0), vb = make_uint2(0, 0);
    if (p < p_end) {
      va = *reinterpret_cast<const uint2*>(dout + (long long)p * do_cs + do_off + co0 + sc);
      const int x = p % W, y = (p / W) % H, z = p / (W * H);
      const int q = (wrap(z + dz, D) * H + wrap(y + dy, H)) * W + wrap(x + dx, W);
      vb = *reinterpret_cast<const uint2*>(in + (long long)q * in_cs + in_off + ci0 + sc);
    }
    __syncthreads();
    As[sc + 0][sv] = (u16)(va.x & 0xFFFF);
    As[sc + 1][sv] = (u16)(va.x >> 16);
    As[sc + 2][sv] = (u16)(va.y & 0xFFFF);
    As[sc + 3][sv] = (u16)(va.y >> 16);
    Bs[sc + 0][sv] = (u16)(vb.x & 0xFFFF);
    Bs[sc + 1][sv] = (u16)(vb.x >> 16);
    Bs[sc + 2][sv] = (u16)(vb.y & 0xFFFF);
    Bs[sc + 3][sv] = (u16)(vb.y >> 16);
    __syncthreads();
    const bf16x8 a = ld8(&As[wm + r][8 * g]);
    const bf16x8 b = ld8(&Bs[wn + r][8 * g]);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  for (int i = 0; i < 4; ++i) {
    const int co = co0 + wm + 4 * g + i, ci = ci0 + wn + r;
    atomicAdd(&dW[((long long)t * Cout + co) * Cin + ci], acc[i]);
  }
}

// dB[co] += sum_p dout[p][co]
__global__ void k_bias_grad(const u16* __restrict__ dout, int cs, int off, int C, int V, float* __restrict__ dB) {
  const int co = blockIdx.y * 64 + (threadIdx.x & 63);
  const int lanes = blockDim.x >> 6;
  float s = 0.0f;
  if (co < C)
    for (int p = blockIdx.x * lanes + (threadIdx.x >> 6); p < V; p += gridDim.x * lanes)
      s += bf2f(dout[(long long)p * cs + off + co]);
  if (co < C) atomicAdd(&dB[co], s);
}

// ------------------------------------------------------------- pointwise ---
__global__ void k_mask_relu(u16* __restrict__ g, int g_cs, int g_off, const u16* __restrict__ act, int a_cs,
                            int a_off, int C, long long V) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V * C) return;
  const long long p = i / C;
  const int ch = (int)(i % C);
  if (!(bf2f(act[p * a_cs + a_off + ch]) > 0.0f)) g[p * g_cs + g_off + ch] = 0;
}

// 2x2x2 average pooling (forward), output (D/2)^3.  One thread per 8 channels
// of an output voxel (16-byte loads and stores): C, the offsets and the row
// strides are multiples of 8 at every call.
__global__ void k_pool(const u16* __restrict__ in, int in_cs, int in_off, u16* __restrict__ out, int out_cs,
                       int out_off, int C, int D, int H, int W) {
  const int d = D / 2, h = H / 2, w = W / 2, C8 = C / 8;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)d * h * w * C8) return;
  const int ch = 8 * (int)(i % C8);
  const long long q = i / C8;
  const int x = (int)(q % w), y = (int)((q / w) % h), z = (int)(q / ((long long)w * h));
  float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 2; ++e) {
        const uint4 v = *reinterpret_cast<const uint4*>(
            in + (((long long)(2 * z + a) * H + 2 * y + b) * W + 2 * x + e) * in_cs + in_off + ch);
        const unsigned u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          s[2 * k] += bf2f((u16)(u[k] & 0xFFFFu));
          s[2 * k + 1] += bf2f((u16)(u[k] >> 16));
        }
      }
  unsigned o[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) o[k] = (unsigned)f2bf(0.125f * s[2 * k]) | ((unsigned)f2bf(0.125f * s[2 * k + 1]) << 16);
  *reinterpret_cast<uint4*>(out + q * out_cs + out_off + ch) = uint4{o[0], o[1], o[2], o[3]};
}

// pooling backward: dIn[child] += dOut[parent] / 8
__global__ void k_pool_bwd(const u16* __restrict__ dout, int do_cs, int do_off, u16* __restrict__ din, int di_cs,
                           int di_off, int C, int D, int H, int W) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)D * H * W * C) return;
  const int ch = (int)(i % C);
  const long long p = i / C;
  const int x = (int)(p % W), y = (int)((p / W) % H), z = (int)(p / ((long long)W * H));
  const long long q = ((long long)(z / 2) * (H / 2) + y / 2) * (W / 2) + x / 2;
  const float v = bf2f(din[p * di_cs + di_off + ch]) + 0.125f * bf2f(dout[q * do_cs + do_off + ch]);
  din[p * di_cs + di_off + ch] = f2bf(v);
}

// nearest upsampling x2 (forward): out (2D)^3 from in D^3; one thread per 8
// channels of an output voxel (16-byte copies; C, offsets and strides are
// multiples of 8 at every call)
__global__ void k_up(const u16* __restrict__ in, int in_cs, int in_off, u16* __restrict__ out, int out_cs, int out_off,
                     int C, int D, int H, int W) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int D2 = 2 * D, H2 = 2 * H, W2 = 2 * W, C8 = C / 8;
  if (i >= (long long)D2 * H2 * W2 * C8) return;
  const int ch = 8 * (int)(i % C8);
  const long long p = i / C8;
  const int x = (int)(p % W2), y = (int)((p / W2) % H2), z = (int)(p / ((long long)W2 * H2));
  const long long q = ((long long)(z / 2) * H + y / 2) * W + x / 2;
  *reinterpret_cast<uint4*>(out + p * out_cs + out_off + ch) =
      *reinterpret_cast<const uint4*>(in + q * in_cs + in_off + ch);
}

// upsampling backward: dIn[q] = sum of the 8 children of q
__global__ void k_up_bwd(const u16* __restrict__ dout, int do_cs, int do_off, u16* __restrict__ din, int di_cs,
                         int di_off, int C, int D, int H, int W) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)D * H * W * C) return;
  const int ch = (int)(i % C);
  const long long q = i / C;
  const int x = (int)(q % W), y = (int)((q / W) % H), z = (int)(q / ((long long)W * H));
  const int H2 = 2 * H, W2 = 2 * W;
  float s = 0.0f;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 2; ++e)
        s += bf2f(dout[(((long long)(2 * z + a) * H2 + 2 * y + b) * W2 + 2 * x + e) * do_cs + do_off + ch]);
  din[q * di_cs + di_off + ch] = f2bf(s);
}

// input: channel 0 = phase indicator, channels 1..31 = 0; one thread per 8
// channels of a voxel (16-byte stores)
__global__ void k_pack_input(const uint8_t* __restrict__ phase, long long V, u16* __restrict__ x) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V * 4) return;
  const long long p = i / 4;
  const unsigned c0 = (i % 4) == 0 ? (unsigned)f2bf(phase[p] ? 1.0f : 0.0f) : 0u;
  *reinterpret_cast<uint4*>(x + 8 * i) = uint4{c0, 0u, 0u, 0u};
}

// mean squared error over 36 channels: dy = 2 (y - T) / (V 36) (bf16, 64 channels), loss partial sums
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ T, long long V, u16* __restrict__ dy,
                      double* __restrict__ loss) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < V * 64) {
    const long long p = i / 64;
    const int ch = (int)(i % 64);
    float g = 0.0f;
    if (ch < 36) {
      const float d = y[i] - T[p * 36 + ch];
      s = (double)d * d;
      g = 2.0f * d / (float)(V * 36);
    }
    dy[i] = f2bf(g);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, s / (double)(V * 36));
}

// Adam on the flat float32 parameters; refreshes the bf16 copies in both
// layouts ([t][co][ci] forward, [t][ci][co] backward data).
struct LayerDesc {
  int cin, cout, ks;
  long long w_off, b_off;
};

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ gr, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1c, float b2c) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = gr[i];
  const float mi = 0.9f * m[i] + 0.1f * g;
  const float vi = 0.999f * v[i] + 0.001f * g * g;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / b1c) / (sqrtf(vi / b2c) + 1e-8f);
}

__global__ void k_cast_weights(const float* __restrict__ w, int ntap, int cout, int cin, u16* __restrict__ wf,
                               u16* __restrict__ wb) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = (long long)ntap * cout * cin;
  if (i >= n) return;
  const int ci = (int)(i % cin);
  const int co = (int)((i / cin) % cout);
  const int t = (int)(i / ((long long)cin * cout));
  const u16 h = f2bf(w[i]);
  wf[i] = h;
  wb[((long long)t * cin + ci) * cout + co] = h;
}

// T[p][6 j + c] = E6[j][c][p] (Voigt -> Mandel)
__global__ void k_pack_target(const double* __restrict__ E6, long long V, float* __restrict__ T) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V * 36) return;
  const long long p = i / 36;
  const int jc = (int)(i % 36);
  const int j = jc / 6, c = jc % 6;
  T[i] = (float)(E6[((long long)(j * 6 + c)) * V + p] * (c < 3 ? 1.0 : 0.70710678118654752440));
}

int blocks(long long n, int t) { return (int)((n + t - 1) / t); }

// clears n 4-byte words (a kernel rather than a memset node, so that a caller
// may capture the entry points that clear buffers into a HIP graph)
__global__ void k_zero_words(unsigned* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}
void zero_words(void* p, size_t bytes, hipStream_t st) {
  const long long n = (long long)(bytes / 4);
  if (n > 0)
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<long long>(blocks(n, 256), 4096)), dim3(256), 0, st,
                       (unsigned*)p, n);
}

}  // namespace

// ================================================================ network ===
struct lsh_unet {
  std::vector<LayerDesc> L;
  long long nparam = 0;
  // device parameter state
  float* w = nullptr;
  float* g = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  u16* wf = nullptr;
  u16* wb = nullptr;
  long long nw = 0;  // weights (without biases) for the bf16 copies
  int step = 0;
  float* head = nullptr;
};

namespace {

enum { E1A, E1B, E2A, E2B, E3A, E3B, D2A, D2B, D1A, D1B, HEAD, NLAYER };

struct Acts {
  // level 0 (n^3)
  u16 *x0, *e1a, *cat1, *d1a, *d1b;
  float *y;
  u16* dy;
  // level 1 ((n/2)^3)
  u16 *p1, *e2a, *cat2, *d2a, *d2b;
  // level 2 ((n/4)^3)
  u16 *p2, *e3a, *e3b;
  // gradients
  u16 *g_e1a, *g_cat1, *g_d1a, *g_d1b;
  u16 *g_p1, *g_e2a, *g_cat2, *g_d2a, *g_d2b;
  u16 *g_p2, *g_e3a, *g_e3b;
  double* loss;
  double* eps;  // up to 64 macroscopic strains for the prediction
  size_t total;
};

Acts act_layout(int n, bool training, char* base) {
  const long long V0 = (long long)n * n * n, V1 = V0 / 8, V2 = V0 / 64;
  Acts a;
  size_t off = 0;
  auto take = [&](long long elems, size_t es) {
    char* p = base + off;
    off += lsh_align((size_t)elems * es);
    return p;
  };
  a.x0 = (u16*)take(V0 * 32, 2);
  a.e1a = (u16*)take(V0 * 32, 2);
  a.cat1 = (u16*)take(V0 * 96, 2);
  a.d1a = (u16*)take(V0 * 32, 2);
  a.d1b = (u16*)take(V0 * 32, 2);
  a.p1 = (u16*)take(V1 * 32, 2);
  a.e2a = (u16*)take(V1 * 64, 2);
  a.cat2 = (u16*)take(V1 * 192, 2);
  a.d2a = (u16*)take(V1 * 64, 2);
  a.d2b = (u16*)take(V1 * 64, 2);
  a.p2 = (u16*)take(V2 * 64, 2);
  a.e3a = (u16*)take(V2 * 128, 2);
  a.e3b = (u16*)take(V2 * 128, 2);
  a.loss = (double*)take(1, 8);
  a.eps = (double*)take(64 * 6, 8);
  if (training) {
    a.y = (float*)take(V0 * 64, 4);  // a prediction forms the head and its contraction in one kernel
    a.dy = (u16*)take(V0 * 64, 2);
    a.g_e1a = (u16*)take(V0 * 32, 2);
    a.g_cat1 = (u16*)take(V0 * 96, 2);
    a.g_d1a = (u16*)take(V0 * 32, 2);
    a.g_d1b = (u16*)take(V0 * 32, 2);
    a.g_p1 = (u16*)take(V1 * 32, 2);
    a.g_e2a = (u16*)take(V1 * 64, 2);
    a.g_cat2 = (u16*)take(V1 * 192, 2);
    a.g_d2a = (u16*)take(V1 * 64, 2);
    a.g_d2b = (u16*)take(V1 * 64, 2);
    a.g_p2 = (u16*)take(V2 * 64, 2);
    a.g_e3a = (u16*)take(V2 * 128, 2);
    a.g_e3b = (u16*)take(V2 * 128, 2);
  }
  a.total = off;
  return a;
}

#define UCHK(x)                                                                                   \
  do {                                                                                            \
    hipError_t e_ = (x);                                                                          \
    if (e_ != hipSuccess) return lsh_fail(LSH_EDEVICE, std::string("HIP error: ") + hipGetErrorString(e_)); \
  } while (0)

// forward convolution of layer l
void conv_fwd(lsh_unet* net, int l, const ConvIn& src, u16* out_bf, float* out_f, int out_cs, int out_off, int relu,
              int n, hipStream_t st) {
  const LayerDesc& d = net->L[l];
  launch_conv(src, d.cin, (const u16*)(net->wf + d.w_off), d.cout, (const float*)(net->w + d.b_off), d.ks, 0, out_bf,
              out_f, out_cs, out_off, relu, n, st);
}

// backward of layer l given dPre (already masked): weight/bias grads and (if din) input grads
void conv_bwd(lsh_unet* net, int l, const u16* in, int in_cs, int in_off, const u16* dpre, int dp_cs, int dp_off,
              u16* din, int di_cs, int di_off, int n, hipStream_t st) {
  const LayerDesc& d = net->L[l];
  const long long V = (long long)n * n * n;
  const int ntap = d.ks * d.ks * d.ks;
  const int chunk = 2048;
  hipLaunchKernelGGL(k_conv_wgrad, dim3(blocks(V, chunk), ntap, (d.cout / 32) * (d.cin / 32)), dim3(256), 0, st, dpre,
                     dp_cs, dp_off, d.cout, in, in_cs, in_off, d.cin, d.ks, net->g + d.w_off, n, n, n, chunk);
  hipLaunchKernelGGL(k_bias_grad, dim3(std::min<long long>(blocks(V, 4), 512), blocks(d.cout, 64)), dim3(256), 0, st,
                     dpre, dp_cs, dp_off, d.cout, (int)V, net->g + d.b_off);
  if (din)
    launch_conv(plain_in(dpre, dp_cs, dp_off), d.cout, (const u16*)(net->wb + d.w_off), d.cin, (const float*)nullptr,
                d.ks, 1, din, (float*)nullptr, di_cs, di_off, 0, n, st);
}

void mask(u16* g, int g_cs, int g_off, const u16* act, int a_cs, int a_off, int C, int n, hipStream_t st) {
  const long long V = (long long)n * n * n;
  hipLaunchKernelGGL(k_mask_relu, dim3(blocks(V * C, 256)), dim3(256), 0, st, g, g_cs, g_off, act, a_cs, a_off, C, V);
}

// every layer up to the head's input (d1b).  in_place: the first layer forms
// its packed input from the phase map and the decoder's first convolutions
// read the upsampled channels from the coarser grid as they stage their
// halos, where those convolutions run LDS-staged (a prediction; training
// keeps the packed input and the concatenations, which its weight gradients
// read).
void trunk(lsh_unet* net, const Acts& a, const uint8_t* phase, int n, bool in_place, hipStream_t st) {
  const int n1 = n / 2, n2 = n / 4;
  const long long V0 = (long long)n * n * n;
  const bool f0 = in_place && lds_conv(n, 3), f1 = in_place && lds_conv(n1, 3);
  if (f0) {
    conv_fwd(net, E1A, ConvIn{nullptr, 0, 0, nullptr, 0, 0, phase}, a.e1a, nullptr, 32, 0, 1, n, st);
  } else {
    hipLaunchKernelGGL(k_pack_input, dim3(blocks(V0 * 4, 256)), dim3(256), 0, st, phase, V0, a.x0);
    conv_fwd(net, E1A, plain_in(a.x0, 32, 0), a.e1a, nullptr, 32, 0, 1, n, st);
  }
  conv_fwd(net, E1B, plain_in(a.e1a, 32, 0), a.cat1, nullptr, 96, 64, 1, n, st);
  hipLaunchKernelGGL(k_pool, dim3(blocks((long long)n1 * n1 * n1 * 4, 256)), dim3(256), 0, st, (const u16*)a.cat1, 96,
                     64, a.p1, 32, 0, 32, n, n, n);
  conv_fwd(net, E2A, plain_in(a.p1, 32, 0), a.e2a, nullptr, 64, 0, 1, n1, st);
  conv_fwd(net, E2B, plain_in(a.e2a, 64, 0), a.cat2, nullptr, 192, 128, 1, n1, st);
  hipLaunchKernelGGL(k_pool, dim3(blocks((long long)n2 * n2 * n2 * 8, 256)), dim3(256), 0, st, (const u16*)a.cat2,
                     192, 128, a.p2, 64, 0, 64, n1, n1, n1);
  conv_fwd(net, E3A, plain_in(a.p2, 64, 0), a.e3a, nullptr, 128, 0, 1, n2, st);
  conv_fwd(net, E3B, plain_in(a.e3a, 128, 0), a.e3b, nullptr, 128, 0, 1, n2, st);
  if (f1) {
    conv_fwd(net, D2A, ConvIn{a.cat2, 192, 0, a.e3b, 128, 128, nullptr}, a.d2a, nullptr, 64, 0, 1, n1, st);
  } else {
    hipLaunchKernelGGL(k_up, dim3(blocks((long long)n1 * n1 * n1 * 16, 256)), dim3(256), 0, st, (const u16*)a.e3b,
                       128, 0, a.cat2, 192, 0, 128, n2, n2, n2);
    conv_fwd(net, D2A, plain_in(a.cat2, 192, 0), a.d2a, nullptr, 64, 0, 1, n1, st);
  }
  conv_fwd(net, D2B, plain_in(a.d2a, 64, 0), a.d2b, nullptr, 64, 0, 1, n1, st);
  if (f0) {
    conv_fwd(net, D1A, ConvIn{a.cat1, 96, 0, a.d2b, 64, 64, nullptr}, a.d1a, nullptr, 32, 0, 1, n, st);
  } else {
    hipLaunchKernelGGL(k_up, dim3(blocks(V0 * 8, 256)), dim3(256), 0, st, (const u16*)a.d2b, 64, 0, a.cat1, 96, 0, 64,
                       n1, n1, n1);
    conv_fwd(net, D1A, plain_in(a.cat1, 96, 0), a.d1a, nullptr, 32, 0, 1, n, st);
  }
  conv_fwd(net, D1B, plain_in(a.d1a, 32, 0), a.d1b, nullptr, 32, 0, 1, n, st);
}

void forward(lsh_unet* net, const Acts& a, const uint8_t* phase, int n, hipStream_t st) {
  trunk(net, a, phase, n, false, st);
  conv_fwd(net, HEAD, plain_in(a.d1b, 32, 0), nullptr, a.y, 64, 0, 0, n, st);
  net->head = a.y;
}

void backward(lsh_unet* net, const Acts& a, int n, hipStream_t st) {
  const int n1 = n / 2, n2 = n / 4;
  const long long V0 = (long long)n * n * n, V1 = V0 / 8, V2 = V0 / 64;
  // head (no activation): dpre = dy
  conv_bwd(net, HEAD, a.d1b, 32, 0, a.dy, 64, 0, a.g_d1b, 32, 0, n, st);
  mask(a.g_d1b, 32, 0, a.d1b, 32, 0, 32, n, st);
  conv_bwd(net, D1B, a.d1a, 32, 0, a.g_d1b, 32, 0, a.g_d1a, 32, 0, n, st);
  mask(a.g_d1a, 32, 0, a.d1a, 32, 0, 32, n, st);
  conv_bwd(net, D1A, a.cat1, 96, 0, a.g_d1a, 32, 0, a.g_cat1, 96, 0, n, st);
  // upsampling 1 backward: g_cat1[0:64] -> g_d2b
  hipLaunchKernelGGL(k_up_bwd, dim3(blocks(V1 * 64, 256)), dim3(256), 0, st, (const u16*)a.g_cat1, 96, 0, a.g_d2b, 64,
                     0, 64, n1, n1, n1);
  mask(a.g_d2b, 64, 0, a.d2b, 64, 0, 64, n1, st);
  conv_bwd(net, D2B, a.d2a, 64, 0, a.g_d2b, 64, 0, a.g_d2a, 64, 0, n1, st);
  mask(a.g_d2a, 64, 0, a.d2a, 64, 0, 64, n1, st);
  conv_bwd(net, D2A, a.cat2, 192, 0, a.g_d2a, 64, 0, a.g_cat2, 192, 0, n1, st);
  hipLaunchKernelGGL(k_up_bwd, dim3(blocks(V2 * 128, 256)), dim3(256), 0, st, (const u16*)a.g_cat2, 192, 0, a.g_e3b,
                     128, 0, 128, n2, n2, n2);
  mask(a.g_e3b, 128, 0, a.e3b, 128, 0, 128, n2, st);
  conv_bwd(net, E3B, a.e3a, 128, 0, a.g_e3b, 128, 0, a.g_e3a, 128, 0, n2, st);
  mask(a.g_e3a, 128, 0, a.e3a, 128, 0, 128, n2, st);
  conv_bwd(net, E3A, a.p2, 64, 0, a.g_e3a, 128, 0, a.g_p2, 64, 0, n2, st);
  // pooling 2 backward adds into the e2b slice of g_cat2
  hipLaunchKernelGGL(k_pool_bwd, dim3(blocks(V1 * 64, 256)), dim3(256), 0, st, (const u16*)a.g_p2, 64, 0, a.g_cat2,
                     192, 128, 64, n1, n1, n1);
  mask(a.g_cat2, 192, 128, a.cat2, 192, 128, 64, n1, st);
  conv_bwd(net, E2B, a.e2a, 64, 0, a.g_cat2, 192, 128, a.g_e2a, 64, 0, n1, st);
  mask(a.g_e2a, 64, 0, a.e2a, 64, 0, 64, n1, st);
  conv_bwd(net, E2A, a.p1, 32, 0, a.g_e2a, 64, 0, a.g_p1, 32, 0, n1, st);
  hipLaunchKernelGGL(k_pool_bwd, dim3(blocks(V0 * 32, 256)), dim3(256), 0, st, (const u16*)a.g_p1, 32, 0, a.g_cat1, 96,
                     64, 32, n, n, n);
  mask(a.g_cat1, 96, 64, a.cat1, 96, 64, 32, n, st);
  conv_bwd(net, E1B, a.e1a, 32, 0, a.g_cat1, 96, 64, a.g_e1a, 32, 0, n, st);
  mask(a.g_e1a, 32, 0, a.e1a, 32, 0, 32, n, st);
  conv_bwd(net, E1A, a.x0, 32, 0, a.g_e1a, 32, 0, nullptr, 0, 0, n, st);
}

int refresh_bf16(lsh_unet* net, hipStream_t st) {
  for (const LayerDesc& d : net->L) {
    const long long nw = (long long)d.ks * d.ks * d.ks * d.cout * d.cin;
    hipLaunchKernelGGL(k_cast_weights, dim3(blocks(nw, 256)), dim3(256), 0, st, (const float*)(net->w + d.w_off),
                       d.ks * d.ks * d.ks, d.cout, d.cin, net->wf + d.w_off, net->wb + d.w_off);
  }
  UCHK(hipGetLastError());
  return LSH_OK;
}

}  // namespace

extern "C" int lsh_unet_create(int base, lsh_unet** out) {
  if (!out) return lsh_fail(LSH_EINVAL, "null argument");
  if (base != 32) return lsh_fail(LSH_EINVAL, "only base width 32 is built");
  lsh_unet* net = new lsh_unet();
  const int spec[NLAYER][3] = {{32, 32, 3}, {32, 32, 3},  {32, 64, 3},  {64, 64, 3}, {64, 128, 3}, {128, 128, 3},
                               {192, 64, 3}, {64, 64, 3}, {96, 32, 3}, {32, 32, 3}, {32, 64, 1}};
  long long off = 0;
  for (int l = 0; l < NLAYER; ++l) {
    LayerDesc d;
    d.cin = spec[l][0];
    d.cout = spec[l][1];
    d.ks = spec[l][2];
    d.w_off = off;
    off += (long long)d.ks * d.ks * d.ks * d.cin * d.cout;
    net->L.push_back(d);
  }
  net->nw = off;
  for (auto& d : net->L) {
    d.b_off = off;
    off += d.cout;
  }
  net->nparam = off;
  *out = net;
  return LSH_OK;
}

extern "C" void lsh_unet_destroy(lsh_unet* net) { delete net; }

extern "C" int lsh_unet_param_count(const lsh_unet* net, int64_t* count) {
  if (!net || !count) return lsh_fail(LSH_EINVAL, "null argument");
  *count = net->nparam;
  return LSH_OK;
}

extern "C" int lsh_unet_param_bytes(const lsh_unet* net, size_t* bytes) {
  if (!net || !bytes) return lsh_fail(LSH_EINVAL, "null argument");
  *bytes = 4 * lsh_align(sizeof(float) * net->nparam) + 2 * lsh_align(sizeof(u16) * net->nw);
  return LSH_OK;
}

extern "C" int lsh_unet_bind(lsh_unet* net, void* dev, size_t bytes, const float* params, void* stream) {
  if (!net || !dev || !params) return lsh_fail(LSH_EINVAL, "null argument");
  size_t need = 0;
  lsh_unet_param_bytes(net, &need);
  if (bytes < need) return lsh_fail(LSH_EWORKSPACE, "parameter buffer too small");
  hipStream_t st = (hipStream_t)stream;
  char* b = (char*)dev;
  const size_t fb = lsh_align(sizeof(float) * net->nparam);
  net->w = (float*)b;
  net->g = (float*)(b + fb);
  net->m = (float*)(b + 2 * fb);
  net->v = (float*)(b + 3 * fb);
  net->wf = (u16*)(b + 4 * fb);
  net->wb = (u16*)(b + 4 * fb + lsh_align(sizeof(u16) * net->nw));
  UCHK(hipMemcpyAsync(net->w, params, sizeof(float) * net->nparam, hipMemcpyHostToDevice, st));
  zero_words(net->g, 3 * fb, st);
  UCHK(hipGetLastError());
  net->step = 0;
  int rc = refresh_bf16(net, st);
  if (rc) return rc;
  UCHK(hipStreamSynchronize(st));
  return LSH_OK;
}

extern "C" int lsh_unet_get_params(const lsh_unet* net, float* params, void* stream) {
  if (!net || !params || !net->w) return lsh_fail(LSH_ESTATE, "network not bound");
  hipStream_t st = (hipStream_t)stream;
  UCHK(hipMemcpyAsync(params, net->w, sizeof(float) * net->nparam, hipMemcpyDeviceToHost, st));
  UCHK(hipStreamSynchronize(st));
  return LSH_OK;
}

extern "C" int lsh_unet_get_grads(const lsh_unet* net, float* grads, void* stream) {
  if (!net || !grads || !net->g) return lsh_fail(LSH_ESTATE, "network not bound");
  hipStream_t st = (hipStream_t)stream;
  UCHK(hipMemcpyAsync(grads, net->g, sizeof(float) * net->nparam, hipMemcpyDeviceToHost, st));
  UCHK(hipStreamSynchronize(st));
  return LSH_OK;
}

extern "C" int lsh_unet_zero_grad(lsh_unet* net, void* stream) {
  if (!net || !net->g) return lsh_fail(LSH_ESTATE, "network not bound");
  zero_words(net->g, sizeof(float) * net->nparam, (hipStream_t)stream);
  UCHK(hipGetLastError());
  return LSH_OK;
}

extern "C" int lsh_unet_act_bytes(const lsh_unet* net, int n, int training, size_t* bytes) {
  if (!net || !bytes) return lsh_fail(LSH_EINVAL, "null argument");
  if (n < 8 || n % 8 != 0) return lsh_fail(LSH_EINVAL, "grid side must be a positive multiple of 8");
  *bytes = act_layout(n, training != 0, nullptr).total;
  return LSH_OK;
}

extern "C" int lsh_unet_train_step(lsh_unet* net, const uint8_t* phase, const float* target, int n, float lr,
                                   void* dev_act, size_t act_bytes, void* stream, double* loss_out) {
  if (!net || !net->w || !phase || !target) return lsh_fail(LSH_EINVAL, "null argument or network not bound");
  if (n < 8 || n % 8 != 0) return lsh_fail(LSH_EINVAL, "grid side must be a positive multiple of 8");
  Acts a = act_layout(n, true, (char*)dev_act);
  if (!dev_act || act_bytes < a.total) return lsh_fail(LSH_EWORKSPACE, "activation workspace too small");
  hipStream_t st = (hipStream_t)stream;
  const long long V0 = (long long)n * n * n;
  forward(net, a, phase, n, st);
  zero_words(a.loss, sizeof(double), st);
  // gradient slices that are accumulated into (pool backward) start from the
  // conv backward-data results; the concat buffers are fully overwritten
  hipLaunchKernelGGL(k_mse, dim3(blocks(V0 * 64, 256)), dim3(256), 0, st, (const float*)a.y, target, V0, a.dy, a.loss);
  backward(net, a, n, st);
  UCHK(hipGetLastError());
  if (lr > 0.0f) {
    net->step += 1;
    const float b1c = 1.0f - powf(0.9f, (float)net->step);
    const float b2c = 1.0f - powf(0.999f, (float)net->step);
    hipLaunchKernelGGL(k_adam, dim3(blocks(net->nparam, 256)), dim3(256), 0, st, net->w, (const float*)net->g, net->m,
                       net->v, net->nparam, lr, b1c, b2c);
    int rc = refresh_bf16(net, st);
    if (rc) return rc;
    zero_words(net->g, sizeof(float) * net->nparam, st);
  }
  if (loss_out) {
    UCHK(hipMemcpyAsync(loss_out, a.loss, sizeof(double), hipMemcpyDeviceToHost, st));
    UCHK(hipStreamSynchronize(st));
  }
  return LSH_OK;
}

extern "C" int lsh_unet_predict(lsh_unet* net, const uint8_t* phase, int n, const double* eps0_voigt, int nload,
                                double* dev_E_out, void* dev_act, size_t act_bytes, void* stream) {
  if (!net || !net->w || !phase || !eps0_voigt || !dev_E_out || nload < 1 || nload > 64)
    return lsh_fail(LSH_EINVAL, "bad argument or network not bound");
  if (n < 8 || n % 8 != 0) return lsh_fail(LSH_EINVAL, "grid side must be a positive multiple of 8");
  Acts a = act_layout(n, false, (char*)dev_act);
  if (!dev_act || act_bytes < a.total) return lsh_fail(LSH_EWORKSPACE, "activation workspace too small");
  const LayerDesc& hd = net->L[HEAD];
  if (hd.cin != 32 || hd.cout != 64 || hd.ks != 1) return lsh_fail(LSH_ESTATE, "head layer is not 1x1, 32 -> 64");
  hipStream_t st = (hipStream_t)stream;
  const long long V0 = (long long)n * n * n;
  trunk(net, a, phase, n, true, st);
  UCHK(hipMemcpyAsync(a.eps, eps0_voigt, sizeof(double) * 6 * nload, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_head_contract, dim3((unsigned)(V0 / 256)), dim3(256), 0, st, (const u16*)a.d1b, 32, 0,
                     (const u16*)(net->wf + hd.w_off), (const float*)(net->w + hd.b_off), (const double*)a.eps, nload,
                     dev_E_out, n, n, n);
  net->head = nullptr;  // not formed by a prediction
  UCHK(hipGetLastError());
  UCHK(hipStreamSynchronize(st));
  return LSH_OK;
}

extern "C" int lsh_unet_head(const lsh_unet* net, int n, float* dst, void* stream) {
  if (!net || !dst || !net->head) return lsh_fail(LSH_ESTATE, "no forward pass yet");
  UCHK(hipMemcpyAsync(dst, net->head, sizeof(float) * 64 * (size_t)n * n * n, hipMemcpyDeviceToDevice,
                      (hipStream_t)stream));
  return LSH_OK;
}

extern "C" int lsh_unet_layers(const lsh_unet* net, int* nlayer, int* cin, int* cout, int* ks) {
  if (!net || !nlayer || !cin || !cout || !ks) return lsh_fail(LSH_EINVAL, "null argument");
  *nlayer = (int)net->L.size();
  for (size_t l = 0; l < net->L.size(); ++l) {
    cin[l] = net->L[l].cin;
    cout[l] = net->L[l].cout;
    ks[l] = net->L[l].ks;
  }
  return LSH_OK;
}

extern "C" int lsh_unet_pack_target(const double* E6, int n, float* T, void* stream) {
  if (!E6 || !T || n < 1) return lsh_fail(LSH_EINVAL, "bad argument");
  const long long V = (long long)n * n * n;
  hipLaunchKernelGGL(k_pack_target, dim3(blocks(V * 36, 256)), dim3(256), 0, (hipStream_t)stream, E6, V, T);
  UCHK(hipGetLastError());
  return LSH_OK;
}
