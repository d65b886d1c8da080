// Learned initialisation network on gfx950: BF16 MFMA convolutions (forward,
// backward-data, backward-weight) accumulating in FP32, the small layers
// around them, and the whole-network forward / backward / Adam sequence.
// Activations are NHWC bfloat16; parameters, their gradients and the
// optimiser state are FP32.
//
// A 3x3 convolution is an implicit GEMM: Y[p][co] = sum_k A[p][k] B[k][co],
// k = (ky * 3 + kx) * Cin + ci, A gathered from the input on the fly, B the
// packed weights [co][k] (k padded with zeros to a multiple of 32).  One wave
// computes 16 pixels x 16 NB output channels with v_mfma_f32_16x16x32_bf16:
//   A operand: lane l holds row (l & 15), k = 8 (l >> 4) .. + 7
//   B operand: lane l holds column (l & 15), k = 8 (l >> 4) .. + 7
//   result:    lane l holds column (l & 15), rows 4 (l >> 4) .. + 3
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>

#include "hg_device.hpp"
#include "hologen_nn.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

__host__ __device__ inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

__device__ __forceinline__ u16 f2bf(float f) {  // round to nearest, ties to even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 load8(const u16* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

// ---------------------------------------------------------------------------
// 3x3 convolution, zero padding 1.  X [P][Cin] (P = N H W pixels, NHWC),
// Wg [Cout][Kpad] bf16, Y [P][Cout].  Epilogue: + bias (nullable), ReLU
// (relu != 0), times (mask > 0) where mask (nullable) has Y's layout, then
// bf16.  grid.x = ceil(P / 64) (4 waves x 16 pixels), grid.y = Cout / (16 NB).
// ---------------------------------------------------------------------------
template <int NB, bool VEC>
__global__ __launch_bounds__(256) void k_conv3x3(const u16* __restrict__ X, const u16* __restrict__ Wg,
                                                 const float* __restrict__ bias, const u16* __restrict__ mask,
                                                 u16* __restrict__ Y, long P, int H, int W, int Cin, int Cout,
                                                 int Kpad, int relu) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long pbase = ((long)blockIdx.x * 4 + wave) * 16;
  if (pbase >= P) return;  // whole wave
  const int m = lane & 15, kb = lane >> 4;
  const long pa = pbase + m;
  const bool pvalid = pa < P;
  const long HW = (long)H * W;
  int y = 0, x = 0;
  const u16* xn = X;
  if (pvalid) {
    const long n = pa / HW;
    const int r = (int)(pa - n * HW);
    y = r / W;
    x = r - y * W;
    xn = X + (size_t)n * HW * Cin;
  }
  const int co0 = blockIdx.y * 16 * NB;
  const int K = 9 * Cin;
  f32x4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int kc = 0; kc < Kpad; kc += 32) {
    const int k = kc + kb * 8;
    bf16x8 a = zero8();
    if constexpr (VEC) {  // Cin % 8 == 0: the 8 k values are 8 channels of one tap
      if (pvalid && k < K) {
        const int tap = k / Cin, ci = k - tap * Cin;
        const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
        if (yy >= 0 && yy < H && xx >= 0 && xx < W) a = load8(xn + ((size_t)yy * W + xx) * Cin + ci);
      }
    } else {
      u16 tmp[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int kk = k + e;
        u16 v = 0;
        if (pvalid && kk < K) {
          const int tap = kk / Cin, ci = kk - tap * Cin;
          const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
          if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = xn[((size_t)yy * W + xx) * Cin + ci];
        }
        tmp[e] = v;
      }
      a = __builtin_bit_cast(bf16x8, tmp);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const bf16x8 b = load8(Wg + (size_t)(co0 + nb * 16 + m) * Kpad + k);
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int co = co0 + nb * 16 + m;
    const float bv = bias ? bias[co] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long p = pbase + 4 * kb + i;
      if (p < P) {
        const size_t o = (size_t)p * Cout + co;
        float v = acc[nb][i] + bv;
        if (relu) v = fmaxf(v, 0.f);
        if (mask && !(bf2f(mask[o]) > 0.f)) v = 0.f;
        Y[o] = f2bf(v);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The same convolution with the input tile staged in LDS (Cin % 8 == 0,
// W % 16 == 0).  A workgroup covers R rows x TW columns of one image for
// 16 NB output channels: it copies the (R + 2) x (TW + 2) x Cin halo tile
// into LDS with 16-byte loads (zeros outside the image), each wave runs GW
// 16-pixel groups against NB weight fragments per 32-wide k step (A
// fragments read from LDS, 16 bytes per lane), and the bf16 results go
// through an LDS staging tile so the stores (and the mask loads) are 16
// bytes per lane.  R TW = 64 GW.
// ---------------------------------------------------------------------------
// LDS elements per staged input pixel: Cin padded by 8 when Cin / 8 is even,
// so the pixel stride is an odd multiple of 16 bytes and the 16 pixel lanes
// of a 16-byte A-fragment read fall in distinct bank groups.
__host__ __device__ inline int tile_pixel_stride(int Cin) { return ((Cin / 8) & 1) ? Cin : Cin + 8; }

// Division by a runtime divisor d (the same for the whole launch) with one
// multiply-high: q = floor(i m / 2^32), m = ceil(2^32 / d), exact for
// i < 2^32 / d (d < 2^16 here, indices below 2^16); d = 1 is handled apart.
struct FastDiv {
  uint32_t d, m;
  __device__ __forceinline__ explicit FastDiv(uint32_t dd) : d(dd), m(dd > 1 ? 0xFFFFFFFFu / dd + 1u : 0u) {}
  __device__ __forceinline__ uint32_t div(uint32_t i) const { return d > 1 ? __umulhi(i, m) : i; }
};

// Global 16-byte load at a wave-uniform base plus a 32-bit byte offset (one
// scalar base register pair, no 64-bit address arithmetic per lane).
__device__ __forceinline__ bf16x8 load8_at(const u16* base, uint32_t byte_off) {
  typedef const __attribute__((address_space(1))) uint4* gp;
  return __builtin_bit_cast(bf16x8, *(gp)((const __attribute__((address_space(1))) char*)base + byte_off));
}

// A32: Cin % 32 == 0, so each 32-wide k step lies in one tap and its tap and
// first channel are the same for the whole wave (kept in scalar registers);
// otherwise (Cin = 16 or 48) each lane tracks its own (tap, channel).
template <int NB, int GW, bool A32>
__global__ __launch_bounds__(256) void k_conv3x3_tile(const u16* __restrict__ X, const u16* __restrict__ Wg,
                                                      const float* __restrict__ bias, const u16* __restrict__ mask,
                                                      u16* __restrict__ Y, int H, int W, int Cin, int Cout, int Kpad,
                                                      int relu, int TW, int R) {
  extern __shared__ __align__(16) u16 smem[];
  // grid: x = tile of the image (tiles_x per tile row), y = output-channel
  // block, z = image
  const int tiles_x = W / TW + (W % TW ? 1 : 0);
  const int ty = (int)blockIdx.x / tiles_x, tx = (int)blockIdx.x - ty * tiles_x;
  const int n = blockIdx.z;
  const int x0 = tx * TW, y0 = ty * R;
  const int TWp = TW + 2;
  const int PS = tile_pixel_stride(Cin);           // LDS elements per pixel
  u16* in = smem;                                  // [(R + 2)][(TW + 2)][PS]
  u16* outs = smem + (size_t)(R + 2) * TWp * PS;   // [R TW][16 NB]
  const int cpp = Cin / 8;                         // 16-byte chunks per pixel
  const u16* xn = X + (size_t)n * H * W * Cin;
  const int co0 = blockIdx.y * 16 * NB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kb = lane >> 4;
  float bv[NB];  // bias, fetched before the k loop
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) bv[nb] = bias ? bias[co0 + nb * 16 + m] : 0.f;
  {
    const FastDiv by_cpp((uint32_t)cpp), by_twp((uint32_t)TWp);
    const int nchunk = (R + 2) * TWp * cpp;
    for (int i = threadIdx.x; i < nchunk; i += 256) {
      const int pix = (int)by_cpp.div((uint32_t)i), c = i - pix * cpp;
      const int ly = (int)by_twp.div((uint32_t)pix), lx = pix - ly * TWp;
      const int gy = y0 + ly - 1, gx = x0 + lx - 1;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (gy >= 0 && gy < H && gx >= 0 && gx < W)
        v = *reinterpret_cast<const uint4*>(xn + ((size_t)gy * W + gx) * Cin + 8 * c);
      *reinterpret_cast<uint4*>(in + (size_t)pix * PS + 8 * c) = v;
    }
  }
  __syncthreads();
  const int gpr = TW / 16;
  const int K = 9 * Cin;
  f32x4 acc[GW][NB];
#pragma unroll
  for (int j = 0; j < GW; ++j)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[j][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  // LDS byte offset of lane m's pixel (tap (0, 0)) in group j, plus the
  // lane's channel offset 8 kb when the k steps are tap-aligned
  uint32_t abase[GW];
#pragma unroll
  for (int j = 0; j < GW; ++j) {
    const int g = wave * GW + j;
    const int r = g / gpr, xg = (g - r * gpr) * 16;
    abase[j] = (uint32_t)(((r * TWp + xg + m) * PS + (A32 ? 8 * kb : 0)) * 2);
  }
  auto lds8 = [&](uint32_t byte_off) { return *reinterpret_cast<const bf16x8*>(reinterpret_cast<const char*>(in) + byte_off); };
  // weight rows: byte offset of lane (m, kb)'s fragment of block nb at k = 0
  uint32_t woff[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) woff[nb] = (uint32_t)(((co0 + nb * 16 + m) * Kpad + 8 * kb) * 2);
  // k = kc + 8 kb as (tap, channel) of the next step to load: A32 tracks the
  // wave's (tap offset, first channel) of the step; otherwise each lane
  // tracks its own, with up to two wraps per step of 32 (Cin >= 16)
  int ci = A32 ? 0 : 8 * kb, kx = 0, toff = 0;
  auto wrap = [&]() {
    if (ci >= Cin) {
      ci -= Cin;
      const bool row_end = kx == 2;
      kx = row_end ? 0 : kx + 1;
      toff += row_end ? (TWp - 2) * PS : PS;
    }
  };
  if constexpr (!A32) {
    wrap();
    wrap();
  }
  // fragments of k step kl into (b, a), then advance the cursor.  Steps past
  // the last load the last step's weights again (a valid address) and zero A
  // fragments, so every step issues the same loads and the outstanding-load
  // count is the same on every path.
  auto load_step = [&](int kl, bf16x8 (&b)[NB], bf16x8 (&a)[GW]) {
    const u16* wk = Wg + (kl < Kpad ? kl : Kpad - 32);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) b[nb] = load8_at(wk, woff[nb]);
    const bool kv = A32 ? kl < Kpad : kl + 8 * kb < K;
    const uint32_t off = (uint32_t)((toff + ci) * 2);
#pragma unroll
    for (int j = 0; j < GW; ++j) a[j] = kv ? lds8(abase[j] + off) : zero8();
    ci += 32;
    wrap();
    if constexpr (!A32) wrap();
  };
  auto mma = [&](const bf16x8 (&b)[NB], const bf16x8 (&a)[GW]) {
#pragma unroll
    for (int j = 0; j < GW; ++j)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[j][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j], b[nb], acc[j][nb], 0, 0, 0);
  };
  // software pipeline over three register sets, unrolled three times so no
  // fragment is copied: step s uses set s mod 3 while the load for step s + 2
  // goes into the set step s - 1 used
  bf16x8 bs0[NB], bs1[NB], bs2[NB], as0[GW], as1[GW], as2[GW];
  const int nsteps = Kpad / 32, ntrip = nsteps / 3;
  load_step(0, bs0, as0);
  load_step(32, bs1, as1);
  int kc = 0;
  for (int tr = 0; tr < ntrip; ++tr, kc += 96) {
    load_step(kc + 64, bs2, as2);
    mma(bs0, as0);
    load_step(kc + 96, bs0, as0);
    mma(bs1, as1);
    load_step(kc + 128, bs1, as1);
    mma(bs2, as2);
  }
  // the last one or two steps (in sets 0 and 1)
  if (nsteps - 3 * ntrip >= 1) mma(bs0, as0);
  if (nsteps - 3 * ntrip >= 2) mma(bs1, as1);
  constexpr int CW = 16 * NB;  // staged channels per pixel
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
    for (int j = 0; j < GW; ++j) {
      const int g = wave * GW + j;
      const int r = g / gpr, xg = (g - r * gpr) * 16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = acc[j][nb][i] + bv[nb];
        if (relu) v = fmaxf(v, 0.f);
        outs[(r * TW + xg + 4 * kb + i) * CW + nb * 16 + m] = f2bf(v);
      }
    }
  }
  __syncthreads();
  constexpr int CPO = CW / 8;  // 16-byte chunks per staged pixel
  const FastDiv by_tw((uint32_t)TW);
  for (int i = threadIdx.x; i < R * TW * CPO; i += 256) {
    const int pl = i / CPO, c = i - pl * CPO;
    const int ly = (int)by_tw.div((uint32_t)pl), lx = pl - ly * TW;
    const int gy = y0 + ly, gx = x0 + lx;
    if (gy < H && gx < W) {
      uint4 v = *reinterpret_cast<const uint4*>(outs + pl * CW + 8 * c);
      const size_t o = (((size_t)n * H + gy) * W + gx) * Cout + co0 + 8 * c;
      if (mask) {
        const uint4 mk = *reinterpret_cast<const uint4*>(mask + o);
        uint32_t* vv = reinterpret_cast<uint32_t*>(&v);
        const uint32_t* mm = reinterpret_cast<const uint32_t*>(&mk);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t lo = bf2f((u16)(mm[q] & 0xFFFFu)) > 0.f ? 0x0000FFFFu : 0u;
          const uint32_t hi = bf2f((u16)(mm[q] >> 16)) > 0.f ? 0xFFFF0000u : 0u;
          vv[q] &= lo | hi;
        }
      }
      *reinterpret_cast<uint4*>(Y + o) = v;
    }
  }
}

// ---------------------------------------------------------------------------
// The convolution for Cin % 16 == 0 with input channels streamed in chunks
// of 32 (the last one 16 when Cin % 32 == 16): a workgroup covers a 4 x 64 pixel tile of one image for 16 NB
// output channels, wave w row w of the tile (four 16-pixel groups).  For
// each chunk, the 6 x 66 halo tile and the chunk's weights (9 taps x 16 NB
// channels x 32) go straight from global memory into LDS
// (global_load_lds_dwordx4, no registers held), 80 bytes per pixel or
// weight row (an odd multiple of 16 bytes: conflict-free fragment reads;
// the fifth 16 bytes are filler); then the nine taps run from LDS, A and B
// fragments read one tap ahead.  256 pixels share every weight row the
// workgroup stages, and the k loop issues no global loads, so two
// workgroups per CU overlap one's staging with the other's MFMAs.
// ---------------------------------------------------------------------------
#if defined(__HIP_DEVICE_COMPILE__)
#define NN_AS1(p) ((const __attribute__((address_space(1))) void*)(p))
#define NN_AS3(p) ((__attribute__((address_space(3))) void*)(p))
#else
#define NN_AS1(p) ((const void*)(p))
#define NN_AS3(p) ((void*)(p))
#endif
constexpr int kCcR = 4, kCcTW = 64, kCcC = 32;
constexpr int kCcTWp = kCcTW + 2;
constexpr int kCcSlot = 5;                                   // 16-byte slots per pixel or weight row
constexpr int kCcPix = (kCcR + 2) * kCcTWp;                  // halo pixels
constexpr int kCcInSlots = (kCcPix * kCcSlot + 255) / 256 * 256;  // whole wave instructions (4 waves)
template <int NB> constexpr int cc_w_slots() { return (9 * 16 * NB * kCcSlot + 255) / 256 * 256; }
template <int NB> constexpr int cc_lds_bytes() { return (kCcInSlots + cc_w_slots<NB>()) * 16; }

template <int NB>
__global__ __launch_bounds__(256, 2) void k_conv3x3_cc(const u16* __restrict__ X, const u16* __restrict__ Wg,
                                                       const float* __restrict__ bias, const u16* __restrict__ mask,
                                                       u16* __restrict__ Y, int H, int W, int Cin, int Cout, int Kpad,
                                                       int relu) {
  constexpr int WSL = cc_w_slots<NB>();
  static_assert(2 * cc_lds_bytes<NB>() <= 160 * 1024, "two workgroups per CU");
  static_assert(16 * NB * kCcR * kCcTW * 2 <= cc_lds_bytes<NB>(), "output staging fits");
  __shared__ __align__(16) char lds[cc_lds_bytes<NB>()];
  char* lin = lds;                      // [pixel][5 slots]
  char* lw = lds + kCcInSlots * 16;     // [tap][16 NB rows][5 slots]
  const int tiles_x = W / kCcTW + (W % kCcTW ? 1 : 0);
  const int ty = (int)blockIdx.x / tiles_x, tx = (int)blockIdx.x - ty * tiles_x;
  const int n = blockIdx.z;
  const int x0 = tx * kCcTW, y0 = ty * kCcR;
  const int co0 = blockIdx.y * 16 * NB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kb = lane >> 4;
  const u16* xn = X + (size_t)n * H * W * Cin;
  float bv[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) bv[nb] = bias ? bias[co0 + nb * 16 + m] : 0.f;
  // this lane's staging slots: wave instruction u fills slots
  // 64 (4 u + wave) .. + 63 (a wave-uniform LDS base), slot = lane + that base
  constexpr int NIN = kCcInSlots / 256, NWS = WSL / 256;
  // A chunk holds channels c0 .. c0 + 31, or c0 .. c0 + 15 when only 16 are
  // left (Cin % 32 == 16): then slots 2 and 3 of every pixel are filler and
  // the same slots of every weight row are zeroed, so they add nothing.
  int isrc[NIN];   // element offset of the slot's pixel in the image, or -1: outside (zero)
  int iq[NIN];     // the slot's 16-byte part (4: filler)
#pragma unroll
  for (int u = 0; u < NIN; ++u) {
    const int sl = 64 * (4 * u + wave) + lane;
    const int pix = sl / kCcSlot, q = sl - pix * kCcSlot;
    const int ly = pix / kCcTWp, lx = pix - ly * kCcTWp;
    const int gy = y0 + ly - 1, gx = x0 + lx - 1;
    const bool in_img = pix < kCcPix && gy >= 0 && gy < H && gx >= 0 && gx < W;
    isrc[u] = in_img ? (gy * W + gx) * Cin : -1;
    iq[u] = q;
  }
  int wsrc[NWS];   // element offset of the slot's weight row at k = tap Cin (spare slots: row 0)
  int wq[NWS];     // the slot's 16-byte part (4: filler; spare slots 4)
#pragma unroll
  for (int u = 0; u < NWS; ++u) {
    const int sl = 64 * (4 * u + wave) + lane;
    const int row = sl / kCcSlot, q = sl - row * kCcSlot;
    const int t = row / (16 * NB), co = row - t * 16 * NB;
    const bool real = row < 9 * 16 * NB;
    wsrc[u] = real ? (co0 + co) * Kpad + t * Cin : co0 * Kpad;
    wq[u] = real ? q : 4;
  }
  f32x4 acc[4][NB];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[j][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  // fragment byte offsets: A of group j at tap (0, 0), B of block nb at tap 0
  const uint32_t aoff = (uint32_t)(((wave * kCcTWp + m) * kCcSlot + kb) * 16);
  const uint32_t boff = (uint32_t)((m * kCcSlot + kb) * 16);
  auto frag = [](const char* p) { return *reinterpret_cast<const bf16x8*>(p); };
  auto ld = [&](int t, bf16x8 (&a)[4], bf16x8 (&b)[NB]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = frag(lin + aoff + (((t / 3) * kCcTWp + (t % 3) + 16 * j) * kCcSlot) * 16);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) b[nb] = frag(lw + boff + ((t * 16 * NB + nb * 16) * kCcSlot) * 16);
  };
  auto mma = [&](const bf16x8 (&a)[4], const bf16x8 (&b)[NB]) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[j][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j], b[nb], acc[j][nb], 0, 0, 0);
  };
  const int nchunk = (Cin + kCcC - 1) / kCcC;
  bf16x8 a0[4], b0[NB], a1[4], b1[NB];
  for (int c = 0; c < nchunk; ++c) {
    const int c0 = kCcC * c;
    const int qv = min(4, (Cin - c0) / 8);  // real 16-byte parts per pixel: 4, or 2 in a half chunk
    // stage chunk c (out-of-image pixels load the image's first element, then
    // are zeroed by the lane that staged them once its loads have landed;
    // filler slots load part 0 of their pixel or row)
#pragma unroll
    for (int u = 0; u < NIN; ++u)
      __builtin_amdgcn_global_load_lds(NN_AS1(xn + (isrc[u] >= 0 ? isrc[u] + c0 + 8 * (iq[u] < qv ? iq[u] : 0) : 0)),
                                       NN_AS3(lin + 1024 * (4 * u + wave)), 16, 0, 0);
#pragma unroll
    for (int u = 0; u < NWS; ++u)
      __builtin_amdgcn_global_load_lds(NN_AS1(Wg + wsrc[u] + c0 + 8 * (wq[u] < qv ? wq[u] : 0)),
                                       NN_AS3(lw + 1024 * (4 * u + wave)), 16, 0, 0);
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
    for (int u = 0; u < NIN; ++u)
      if (isrc[u] < 0) *reinterpret_cast<uint4*>(lin + 1024 * (4 * u + wave) + 16 * lane) = make_uint4(0, 0, 0, 0);
    if (qv < 4) {  // half chunk: zero the weight rows' parts 2 and 3
#pragma unroll
      for (int u = 0; u < NWS; ++u)
        if (wq[u] >= qv && wq[u] < 4)
          *reinterpret_cast<uint4*>(lw + 1024 * (4 * u + wave) + 16 * lane) = make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
    ld(0, a0, b0);
    ld(1, a1, b1); mma(a0, b0);
    ld(2, a0, b0); mma(a1, b1);
    ld(3, a1, b1); mma(a0, b0);
    ld(4, a0, b0); mma(a1, b1);
    ld(5, a1, b1); mma(a0, b0);
    ld(6, a0, b0); mma(a1, b1);
    ld(7, a1, b1); mma(a0, b0);
    ld(8, a0, b0); mma(a1, b1);
    mma(a0, b0);
    __syncthreads();  // the next chunk's staging overwrites these buffers
  }
  // epilogue: bias, ReLU, bf16, staged in LDS for 16-byte stores
  constexpr int CW = 16 * NB;
  u16* outs = reinterpret_cast<u16*>(lds);
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = acc[j][nb][i] + bv[nb];
        if (relu) v = fmaxf(v, 0.f);
        outs[(wave * kCcTW + 16 * j + 4 * kb + i) * CW + nb * 16 + m] = f2bf(v);
      }
  __syncthreads();
  constexpr int CPO = CW / 8;
  for (int i = threadIdx.x; i < kCcR * kCcTW * CPO; i += 256) {
    const int pl = i / CPO, c = i - pl * CPO;
    const int ly = pl / kCcTW, lx = pl - ly * kCcTW;
    const int gy = y0 + ly, gx = x0 + lx;
    if (gy < H && gx < W) {
      uint4 v = *reinterpret_cast<const uint4*>(outs + pl * CW + 8 * c);
      const size_t o = (((size_t)n * H + gy) * W + gx) * Cout + co0 + 8 * c;
      if (mask) {
        const uint4 mk = *reinterpret_cast<const uint4*>(mask + o);
        uint32_t* vv = reinterpret_cast<uint32_t*>(&v);
        const uint32_t* mm = reinterpret_cast<const uint32_t*>(&mk);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t lo = bf2f((u16)(mm[q] & 0xFFFFu)) > 0.f ? 0x0000FFFFu : 0u;
          const uint32_t hi = bf2f((u16)(mm[q] >> 16)) > 0.f ? 0xFFFF0000u : 0u;
          vv[q] &= lo | hi;
        }
      }
      *reinterpret_cast<uint4*>(Y + o) = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient: part[pb][co][k] = sum over pixel block pb of
// dY[p][co] A[p][k] (A = implicit im2col of X), i.e. dY^T A with pixels as
// the MFMA reduction dimension:
//   A operand (16 co x 32 px): lane l -> co (l & 15), pixels 8 (l >> 4) .. + 7
//   B operand (32 px x 16 k):  lane l -> k  (l & 15), pixels 8 (l >> 4) .. + 7
// grid.x = pixel blocks of pb_len pixels (a multiple of 32), grid.y = Cout/16,
// grid.z = ceil(Kpad / 64) (4 waves x 16 k).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_conv3x3_wgrad(const u16* __restrict__ X, const u16* __restrict__ dY,
                                                       float* __restrict__ part, float* __restrict__ bpart, long P,
                                                       int H, int W, int Cin, int Cout, int Kpad, long pb_len) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kb = lane >> 4;
  const int co = blockIdx.y * 16 + (lane & 15);
  const int kcol = (blockIdx.z * 4 + wave) * 16 + (lane & 15);
  const long HW = (long)H * W;
  const int K = 9 * Cin;
  const bool kvalid = kcol < K;
  int ci = 0, dyy = 0, dxx = 0;
  if (kvalid) {
    const int tap = kcol / Cin;
    ci = kcol - tap * Cin;
    dyy = tap / 3 - 1;
    dxx = tap % 3 - 1;
  }
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
  // the bias gradient (column sums of dY) rides along in one wave per pixel block
  const bool bias_wave = bpart && blockIdx.z == 0 && wave == 0;
  float bsum = 0.f;
  const long p_begin = (long)blockIdx.x * pb_len;
  const long p_end = std::min(p_begin + pb_len, P);
  for (long pc = p_begin; pc < p_end; pc += 32) {
    u16 av[8], bv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const long p = pc + kb * 8 + e;
      u16 ga = 0, gb = 0;
      if (p < p_end) {
        ga = dY[(size_t)p * Cout + co];
        if (kvalid) {
          const long n = p / HW;
          const int r = (int)(p - n * HW);
          const int yy = r / W + dyy, xx = r % W + dxx;
          if (yy >= 0 && yy < H && xx >= 0 && xx < W) gb = X[(((size_t)n * H + yy) * W + xx) * Cin + ci];
        }
      }
      av[e] = ga;
      bv[e] = gb;
    }
    if (bias_wave) {
#pragma unroll
      for (int e = 0; e < 8; ++e) bsum += bf2f(av[e]);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                  acc, 0, 0, 0);
  }
  if (kcol < Kpad) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int cor = blockIdx.y * 16 + 4 * kb + i;
      part[((size_t)blockIdx.x * Cout + cor) * Kpad + kcol] = acc[i];
    }
  }
  if (bias_wave) {  // lanes l, l ^ 16, l ^ 32, l ^ 48 hold the same channel
    bsum += __shfl_xor(bsum, 16);
    bsum += __shfl_xor(bsum, 32);
    if (lane < 16) bpart[(size_t)blockIdx.x * Cout + co] = bsum;
  }
}

// ---------------------------------------------------------------------------
// Weight gradient for Cin % 16 == 0 and Cout % 16 == 0 with the pixels on
// the MFMA's reduction axis and the operands transposed through LDS:
// part[pb][co][tap Cin + ci] = sum over pixel block pb of dY[p][co]
// X[p + tap offset][ci] (zero outside the image), i.e. D = dY^T X with
// M = 16 output channels, N = 16 input channels, K = 32 pixels.  A
// workgroup owns 16 NB output channels and one chunk of 32 input channels
// (16 in a last half chunk), and walks the 2 x 64 pixel tiles of its block:
// - the tile's dY goes to LDS as [co][pixel] (A fragments: 8 consecutive
//   pixels of one channel), its input halo as three copies [kx][ci][row][p]
//   shifted by the tap column kx, so that every B fragment (8 consecutive
//   pixels of one channel) is a 16-byte aligned read;
// - wave w takes the taps w, w + 4, w + 8 (< 9) for every output-channel
//   block: per 32-pixel step, NB A fragments and one B fragment per tap and
//   channel block, NB MFMAs per B;
// - wave 0 also sums dY over the pixels for the bias gradient.
// Channel strides are odd multiples of 16 bytes (conflict-free fragment
// reads).  The partials are reduced over pixel blocks, in order, by
// k_wgrad_reduce.
// ---------------------------------------------------------------------------
constexpr int kWgXP = 64;                 // pixels of a shifted halo row copy
constexpr int kWgCIS = 4 * kWgXP + 8;     // elements per input channel of a copy (4 halo rows)
constexpr int kWgDS = 2 * 64 + 8;         // elements per output channel of the dY tile

template <int NB>
__global__ __launch_bounds__(256, 2) void k_wgrad_cc(const u16* __restrict__ X, const u16* __restrict__ dY,
                                                     float* __restrict__ part, float* __restrict__ bpart, int H,
                                                     int W, int Cin, int Cout, int Kpad, int tpb, int ntiles) {
  __shared__ __align__(16) u16 xs[3 * 32 * kWgCIS];
  __shared__ __align__(16) u16 dys[16 * NB * kWgDS];
  const int tiles_x = (W + 63) / 64, tiles_img = tiles_x * ((H + 1) / 2);
  const int co0 = blockIdx.y * 16 * NB, c0 = blockIdx.z * 32;
  const int ncib = min(2, (Cin - c0) / 16);  // 16-channel blocks in this chunk
  const int qn = 2 * ncib;                   // 16-byte parts of a pixel's chunk
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kb = lane >> 4;
  f32x4 acc[3][2][NB];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[i][cb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) bsum[nb] = 0.f;
  const int t_end = min((int)blockIdx.x * tpb + tpb, ntiles);
  for (int tl = blockIdx.x * tpb; tl < t_end; ++tl) {
    const int n = tl / tiles_img, rem = tl - n * tiles_img;
    const int ty = rem / tiles_x, tx = rem - ty * tiles_x;
    const int y0 = 2 * ty, x0 = 64 * tx;
    __syncthreads();  // the previous tile's fragment reads are done
    // input halo: rows y0 - 1 .. y0 + 2, columns x0 - 1 .. x0 + 64
    for (int i = threadIdx.x; i < 4 * 66 * qn; i += 256) {
      const int q = i % qn, hp = i / qn;
      const int hy = hp / 66, hx = hp - hy * 66;
      const int gy = y0 - 1 + hy, gx = x0 - 1 + hx;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (gy >= 0 && gy < H && gx >= 0 && gx < W)
        v = *reinterpret_cast<const uint4*>(X + (((size_t)n * H + gy) * W + gx) * Cin + c0 + 8 * q);
      const u16* e = reinterpret_cast<const u16*>(&v);
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int p = hx - kx;
        if (p >= 0 && p < kWgXP) {
#pragma unroll
          for (int k = 0; k < 8; ++k) xs[(kx * 32 + 8 * q + k) * kWgCIS + hy * kWgXP + p] = e[k];
        }
      }
    }
    // dY of the tile's 2 x 64 pixels, transposed to [co][pixel]
    for (int i = threadIdx.x; i < 128 * 2 * NB; i += 256) {
      const int q = i % (2 * NB), pp = i / (2 * NB);
      const int r = pp >> 6, c = pp & 63;
      const int gy = y0 + r, gx = x0 + c;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (gy < H && gx < W)
        v = *reinterpret_cast<const uint4*>(dY + (((size_t)n * H + gy) * W + gx) * Cout + co0 + 8 * q);
      const u16* e = reinterpret_cast<const u16*>(&v);
#pragma unroll
      for (int k = 0; k < 8; ++k) dys[(8 * q + k) * kWgDS + pp] = e[k];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {  // 32-pixel steps: row ks / 2, columns 32 (ks % 2) ..
      const int r = ks >> 1, cc = (ks & 1) * 32;
      bf16x8 a[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        a[nb] = *reinterpret_cast<const bf16x8*>(dys + (nb * 16 + m) * kWgDS + r * 64 + cc + 8 * kb);
      if (wave == 0) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const u16* e = reinterpret_cast<const u16*>(&a[nb]);
#pragma unroll
          for (int k = 0; k < 8; ++k) bsum[nb] += bf2f(e[k]);
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int t = wave + 4 * i;
        if (t < 9) {  // wave-uniform
          const int ky = t / 3, kx = t - 3 * ky;
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) {
            if (cb < ncib) {  // uniform
              const bf16x8 b = *reinterpret_cast<const bf16x8*>(
                  xs + (kx * 32 + cb * 16 + m) * kWgCIS + (r + ky) * kWgXP + cc + 8 * kb);
#pragma unroll
              for (int nb = 0; nb < NB; ++nb)
                acc[i][cb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[nb], b, acc[i][cb][nb], 0, 0, 0);
            }
          }
        }
      }
    }
  }
  // partials: lane (m, kb) holds input channel m and output channels 4 kb .. + 3
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int t = wave + 4 * i;
    if (t >= 9) continue;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      if (cb >= ncib) continue;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int co = co0 + nb * 16 + 4 * kb + e;
          part[((size_t)blockIdx.x * Cout + co) * Kpad + t * Cin + c0 + cb * 16 + m] = acc[i][cb][nb][e];
        }
    }
  }
  if (bpart && blockIdx.z == 0 && wave == 0) {  // lanes m, m + 16, m + 32, m + 48 hold channel m's pixels
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float v = bsum[nb];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (lane < 16) bpart[(size_t)blockIdx.x * Cout + co0 + nb * 16 + m] = v;
    }
  }
}

// dw[co][k] (OHWI) = sum over the pixel blocks of part, in a fixed order.
// Sum of n values at p[0], p[stride], ... in a fixed order: eight
// interleaved running sums (b mod 8), so eight loads are in flight, added
// pairwise at the end.
__device__ __forceinline__ float sum_strided(const float* __restrict__ p, int n, size_t stride) {
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int b = 0;
  for (; b + 8 <= n; b += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += p[(size_t)(b + u) * stride];
  }
  for (int u = 0; b < n; ++b, ++u) a[u] += p[(size_t)b * stride];
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

__global__ void k_wgrad_reduce(const float* __restrict__ part, float* __restrict__ dw, int npb, int Cout, int Kpad,
                               int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Cout * K) return;
  const int co = i / K, k = i - co * K;
  dw[i] = sum_strided(part + (size_t)co * Kpad + k, npb, (size_t)Cout * Kpad);
}

// out[j] = sum_b part[b][j] in sum_strided's fixed order
__global__ void k_sum_parts(const float* __restrict__ part, float* __restrict__ out, int nparts, int ncol) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  out[j] = sum_strided(part + j, nparts, (size_t)ncol);
}

// ---------------------------------------------------------------------------
// Weight packing.  Forward: wg[co][k] = w[co][ky][kx][ci] (k = tap Cin + ci).
// Backward-data (the adjoint is a 3x3 convolution of dY with the spatially
// flipped, channel-transposed kernel): wg[ci][k'] = w[co][2-ky][2-kx][ci]
// with k' = tap Cout + co.
// ---------------------------------------------------------------------------
__global__ void k_pack_weights(const float* __restrict__ w, u16* __restrict__ wg, int Cout, int Cin, int Kpad,
                               int flip) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int rows = flip ? Cin : Cout, cols = flip ? 9 * Cout : 9 * Cin;
  if (i >= rows * Kpad) return;
  const int r = i / Kpad, k = i - r * Kpad;
  float v = 0.f;
  if (k < cols) {
    if (!flip) {
      v = w[(size_t)r * 9 * Cin + k];
    } else {
      const int tap = k / Cout, co = k - tap * Cout;
      const int ky = 2 - tap / 3, kx = 2 - tap % 3;
      v = w[(((size_t)co * 3 + ky) * 3 + kx) * Cin + r];
    }
  }
  wg[i] = f2bf(v);
}

// network input: per-image sum of T^2 (block partials, FP64) ...
__global__ __launch_bounds__(256) void k_sumsq_part(const float* __restrict__ t, double* __restrict__ part, long HW) {
  __shared__ double red[256];
  const long base = (long)blockIdx.y * HW;
  double s = 0.0;
  for (long p = (long)blockIdx.x * 256 + threadIdx.x; p < HW; p += (long)gridDim.x * 256) {
    const double v = t[base + p];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// ... then x = bf16(T sqrt(HW / sum T^2))
__global__ void k_input(const float* __restrict__ t, const double* __restrict__ part, int nparts, u16* __restrict__ x,
                        long HW) {
  const long base = (long)blockIdx.y * HW;
  double s = 0.0;
  for (int i = 0; i < nparts; ++i) s += part[(size_t)blockIdx.y * nparts + i];
  const float scale = s > 0.0 ? (float)sqrt((double)HW / s) : 0.f;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < HW; p += (long)gridDim.x * blockDim.x)
    x[base + p] = f2bf(t[base + p] * scale);
}

// ---- 16-byte (8-channel) versions of the element-wise layers below; used
// when the channel counts are multiples of 8.  They add in the same order as
// the scalar kernels.
__device__ __forceinline__ void unpack8(const uint4& q, float (&f)[8]) {
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    f[2 * i] = bf2f((u16)(w[i] & 0xFFFFu));
    f[2 * i + 1] = bf2f((u16)(w[i] >> 16));
  }
}
__device__ __forceinline__ uint4 pack8(const float (&f)[8]) {
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = (uint32_t)f2bf(f[2 * i]) | ((uint32_t)f2bf(f[2 * i + 1]) << 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}
__device__ __forceinline__ uint4 ld16(const u16* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ __forceinline__ void st16(u16* p, const uint4& v) { *reinterpret_cast<uint4*>(p) = v; }
__device__ __forceinline__ void apply_mask8(float (&f)[8], const u16* m) {
  float mk[8];
  unpack8(ld16(m), mk);
#pragma unroll
  for (int e = 0; e < 8; ++e)
    if (!(mk[e] > 0.f)) f[e] = 0.f;
}

__global__ void k_avgpool2_v8(const u16* __restrict__ x, u16* __restrict__ y, int N, int H, int W, int C) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
  if (i >= (long)N * Ho * Wo * C8) return;
  const int c8 = (int)(i % C8);
  long r = i / C8;
  const int xo = (int)(r % Wo);
  r /= Wo;
  const int yo = (int)(r % Ho);
  const long n = r / Ho;
  const size_t b = (((size_t)n * H + 2 * yo) * W + 2 * xo) * C + 8 * c8;
  const size_t rs = (size_t)W * C;
  float a[8], bb[8], c[8], d[8], o[8];
  unpack8(ld16(x + b), a);
  unpack8(ld16(x + b + C), bb);
  unpack8(ld16(x + b + rs), c);
  unpack8(ld16(x + b + rs + C), d);
#pragma unroll
  for (int e = 0; e < 8; ++e) o[e] = 0.25f * ((a[e] + bb[e]) + (c[e] + d[e]));
  st16(y + (size_t)i * 8, pack8(o));
}

__global__ void k_avgpool2_bwd_v8(const u16* __restrict__ dy, const u16* __restrict__ dskip,
                                  const u16* __restrict__ mask, u16* __restrict__ dx, int N, int H, int W, int C) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int C8 = C / 8;
  if (i >= (long)N * H * W * C8) return;
  const int c8 = (int)(i % C8);
  long r = i / C8;
  const int x = (int)(r % W);
  r /= W;
  const int yv = (int)(r % H);
  const long n = r / H;
  float g[8];
  unpack8(ld16(dy + (((size_t)n * (H / 2) + yv / 2) * (W / 2) + x / 2) * C + 8 * c8), g);
#pragma unroll
  for (int e = 0; e < 8; ++e) g[e] *= 0.25f;
  if (dskip) {
    float s2[8];
    unpack8(ld16(dskip + (size_t)i * 8), s2);
#pragma unroll
    for (int e = 0; e < 8; ++e) g[e] += s2[e];
  }
  if (mask) apply_mask8(g, mask + (size_t)i * 8);
  st16(dx + (size_t)i * 8, pack8(g));
}

__global__ void k_upcat_v8(const u16* __restrict__ lo, const u16* __restrict__ skip, u16* __restrict__ out, int N,
                           int H, int W, int C1, int C2) {
  const int C8 = (C1 + C2) / 8, L8 = C1 / 8;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)N * H * W * C8) return;
  const int c8 = (int)(i % C8);
  const long p = i / C8;
  uint4 v;
  if (c8 < L8) {
    const int x = (int)(p % W);
    const long r = p / W;
    const int yv = (int)(r % H);
    const long n = r / H;
    v = ld16(lo + (((size_t)n * (H / 2) + yv / 2) * (W / 2) + x / 2) * C1 + 8 * c8);
  } else {
    v = ld16(skip + (size_t)p * C2 + 8 * (c8 - L8));
  }
  st16(out + (size_t)i * 8, v);
}

__global__ void k_upcat_bwd_v8(const u16* __restrict__ dout, const u16* __restrict__ mask_lo, u16* __restrict__ dlo,
                               u16* __restrict__ dskip, int N, int H, int W, int C1, int C2) {
  const int C = C1 + C2, L8 = C1 / 8, S8 = C2 / 8;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nlo = (long)N * (H / 2) * (W / 2) * L8;
  const long nsk = (long)N * H * W * S8;
  if (i < nlo) {
    const int c8 = (int)(i % L8);
    long r = i / L8;
    const int xo = (int)(r % (W / 2));
    r /= (W / 2);
    const int yo = (int)(r % (H / 2));
    const long n = r / (H / 2);
    const size_t b = (((size_t)n * H + 2 * yo) * W + 2 * xo) * C + 8 * c8;
    const size_t rs = (size_t)W * C;
    float a[8], bb[8], c[8], d[8], o[8];
    unpack8(ld16(dout + b), a);
    unpack8(ld16(dout + b + C), bb);
    unpack8(ld16(dout + b + rs), c);
    unpack8(ld16(dout + b + rs + C), d);
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = (a[e] + bb[e]) + (c[e] + d[e]);
    if (mask_lo) apply_mask8(o, mask_lo + (size_t)i * 8);
    st16(dlo + (size_t)i * 8, pack8(o));
  } else if (i < nlo + nsk) {
    const long j = i - nlo;
    const int c8 = (int)(j % S8);
    const long p = j / S8;
    st16(dskip + (size_t)j * 8, ld16(dout + (size_t)p * C + C1 + 8 * c8));
  }
}

// 1x1 head with 16 input channels: one pixel per thread, two 16-byte loads
__global__ void k_head16(const u16* __restrict__ x, const float* __restrict__ w, const float* __restrict__ b,
                         float* __restrict__ out, long P) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float v[16];
  unpack8(ld16(x + (size_t)p * 16), *reinterpret_cast<float(*)[8]>(v));
  unpack8(ld16(x + (size_t)p * 16 + 8), *reinterpret_cast<float(*)[8]>(v + 8));
  float a0 = 0.f, a1 = 0.f;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    a0 += v[c] * bf2f(f2bf(w[c]));
    a1 += v[c] * bf2f(f2bf(w[16 + c]));
  }
  *reinterpret_cast<float2*>(out + 2 * p) = make_float2(a0 + b[0], a1 + b[1]);
}

// head backward-data with 16 channels, one pixel per thread
__global__ void k_head_bwd_data16(const float* __restrict__ dout, const float* __restrict__ w,
                                  const u16* __restrict__ x, u16* __restrict__ dx, long P) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const float2 d = *reinterpret_cast<const float2*>(dout + 2 * p);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float g[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = 8 * h + e;
      g[e] = d.x * bf2f(f2bf(w[c])) + d.y * bf2f(f2bf(w[16 + c]));
    }
    apply_mask8(g, x + (size_t)p * 16 + 8 * h);
    st16(dx + (size_t)p * 16 + 8 * h, pack8(g));
  }
}

// First layer (one input channel, 16 outputs): one pixel per thread, the nine
// taps summed in tap order in FP32, bias, ReLU, optional mask, two 16-byte
// stores.  Wg is the packed [16][32] operand (taps 0..8 used).
__global__ void k_conv_first16(const u16* __restrict__ X, const u16* __restrict__ Wg, const float* __restrict__ bias,
                               const u16* __restrict__ mask, u16* __restrict__ Y, long P, int H, int W, int Kpad,
                               int relu) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const long HW = (long)H * W;
  const long n = p / HW;
  const int r = (int)(p - n * HW);
  const int y = r / W, x = r - y * W;
  const u16* xn = X + (size_t)n * HW;
  float xv[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
    xv[t] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? bf2f(xn[(size_t)yy * W + xx]) : 0.f;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float o[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int co = 8 * h + e;
      float a = 0.f;
#pragma unroll
      for (int t = 0; t < 9; ++t) a += xv[t] * bf2f(Wg[co * Kpad + t]);
      a += bias ? bias[co] : 0.f;
      o[e] = relu ? fmaxf(a, 0.f) : a;
    }
    if (mask) apply_mask8(o, mask + (size_t)p * 16 + 8 * h);
    st16(Y + (size_t)p * 16 + 8 * h, pack8(o));
  }
}

// 2x2 average pool, NHWC bf16
__global__ void k_avgpool2(const u16* __restrict__ x, u16* __restrict__ y, int N, int H, int W, int C) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int Ho = H / 2, Wo = W / 2;
  if (i >= (long)N * Ho * Wo * C) return;
  const int c = (int)(i % C);
  long r = i / C;
  const int xo = (int)(r % Wo);
  r /= Wo;
  const int yo = (int)(r % Ho);
  const long n = r / Ho;
  const size_t b = (((size_t)n * H + 2 * yo) * W + 2 * xo) * C + c;
  const size_t rs = (size_t)W * C;
  const float s = (bf2f(x[b]) + bf2f(x[b + C])) + (bf2f(x[b + rs]) + bf2f(x[b + rs + C]));
  y[i] = f2bf(0.25f * s);
}

// dx = (0.25 dy[pooled pixel] + dskip) rounded to bf16, zeroed where
// mask <= 0 (dskip and mask nullable)
__global__ void k_avgpool2_bwd(const u16* __restrict__ dy, const u16* __restrict__ dskip, const u16* __restrict__ mask,
                               u16* __restrict__ dx, int N, int H, int W, int C) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)N * H * W * C) return;
  const int c = (int)(i % C);
  long r = i / C;
  const int x = (int)(r % W);
  r /= W;
  const int yv = (int)(r % H);
  const long n = r / H;
  float g = 0.25f * bf2f(dy[(((size_t)n * (H / 2) + yv / 2) * (W / 2) + x / 2) * C + c]);
  if (dskip) g += bf2f(dskip[i]);
  if (mask && !(bf2f(mask[i]) > 0.f)) g = 0.f;
  dx[i] = f2bf(g);
}

// out[..., :C1] = nearest 2x upsampling of lo (C1 channels), out[..., C1:] = skip (C2)
__global__ void k_upcat(const u16* __restrict__ lo, const u16* __restrict__ skip, u16* __restrict__ out, int N, int H,
                        int W, int C1, int C2) {
  const int C = C1 + C2;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)N * H * W * C) return;
  const int c = (int)(i % C);
  const long p = i / C;
  if (c < C1) {
    const int x = (int)(p % W);
    const long r = p / W;
    const int yv = (int)(r % H);
    const long n = r / H;
    out[i] = lo[(((size_t)n * (H / 2) + yv / 2) * (W / 2) + x / 2) * C1 + c];
  } else {
    out[i] = skip[(size_t)p * C2 + (c - C1)];
  }
}

// backward of k_upcat: dlo = bf16(sum of the 4 copies) zeroed where
// mask_lo <= 0 (nullable), dskip = the skip channels
__global__ void k_upcat_bwd(const u16* __restrict__ dout, const u16* __restrict__ mask_lo, u16* __restrict__ dlo,
                            u16* __restrict__ dskip, int N, int H, int W, int C1, int C2) {
  const int C = C1 + C2;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nlo = (long)N * (H / 2) * (W / 2) * C1;
  const long nsk = (long)N * H * W * C2;
  if (i < nlo) {
    const int c = (int)(i % C1);
    long r = i / C1;
    const int xo = (int)(r % (W / 2));
    r /= (W / 2);
    const int yo = (int)(r % (H / 2));
    const long n = r / (H / 2);
    const size_t b = (((size_t)n * H + 2 * yo) * W + 2 * xo) * C + c;
    const size_t rs = (size_t)W * C;
    float s = (bf2f(dout[b]) + bf2f(dout[b + C])) + (bf2f(dout[b + rs]) + bf2f(dout[b + rs + C]));
    if (mask_lo && !(bf2f(mask_lo[i]) > 0.f)) s = 0.f;
    dlo[i] = f2bf(s);
  } else if (i < nlo + nsk) {
    const long j = i - nlo;
    dskip[j] = dout[(size_t)(j / C2) * C + C1 + (j % C2)];
  }
}

// 1x1 head: out[p] = (sum_c x[p][c] w[0][c] + b[0], sum_c x[p][c] w[1][c] + b[1]),
// weights rounded to bf16, FP32 output (interleaved pairs, a complex64 layout)
__global__ void k_head(const u16* __restrict__ x, const float* __restrict__ w, const float* __restrict__ b,
                       float* __restrict__ out, long P, int C) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float a0 = 0.f, a1 = 0.f;
  for (int c = 0; c < C; ++c) {
    const float v = bf2f(x[(size_t)p * C + c]);
    a0 += v * bf2f(f2bf(w[c]));
    a1 += v * bf2f(f2bf(w[C + c]));
  }
  out[2 * p] = a0 + b[0];
  out[2 * p + 1] = a1 + b[1];
}

// Phase loss of image blockIdx.y against the label phasor y = lab/|lab|
// (lab = 0 counts as phase 0) weighted by amp.  Pass 1: block partials of
// S = sum amp z conj(y) (re, im) and of sum amp, z = out/|out|.
__global__ __launch_bounds__(256) void k_loss_part(const float* __restrict__ out, const float2* __restrict__ lab,
                                                   const float* __restrict__ amp, double* __restrict__ part,
                                                   long HW) {
  __shared__ double red[3][256];
  const long base = (long)blockIdx.y * HW;
  double sr = 0, si = 0, sw = 0;
  for (long p = (long)blockIdx.x * 256 + threadIdx.x; p < HW; p += (long)gridDim.x * 256) {
    const float a = out[2 * (base + p)], b = out[2 * (base + p) + 1];
    const float r = sqrtf(a * a + b * b) + 1e-12f;
    const float2 l = lab[base + p];
    const float lm = sqrtf(l.x * l.x + l.y * l.y);
    const float c = lm > 0.f ? l.x / lm : 1.f, s = lm > 0.f ? l.y / lm : 0.f;
    const float am = amp[base + p];
    sr += am * (a * c + b * s) / r;  // Re(z conj(y))
    si += am * (b * c - a * s) / r;  // Im(z conj(y))
    sw += am;
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = si;
  red[2][threadIdx.x] = sw;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 3 + q] = red[q][0];
}

// Pass 2: l_n = 1 - |S_n| / W_n and d(mean_n l_n)/d out.  With s = S/|S| the
// gradient of l_n is -Re(conj(s) amp conj(y) dz/d(a, b)) / W_n, where
// dz/da = 1/r - a (a + ib)/r^3 and dz/db = i/r - b (a + ib)/r^3.
__global__ __launch_bounds__(256) void k_loss_grad(const float* __restrict__ out, const float2* __restrict__ lab,
                                                   const float* __restrict__ amp, const double* __restrict__ part,
                                                   int nparts, float* __restrict__ dout, float* __restrict__ loss,
                                                   long HW, int batch) {
  const int n = blockIdx.y;
  double S_re = 0, S_im = 0, Wt = 0;
  for (int i = 0; i < nparts; ++i) {
    S_re += part[((size_t)n * nparts + i) * 3 + 0];
    S_im += part[((size_t)n * nparts + i) * 3 + 1];
    Wt += part[((size_t)n * nparts + i) * 3 + 2];
  }
  const double Sabs = sqrt(S_re * S_re + S_im * S_im);
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss) loss[n] = Wt > 0 ? (float)(1.0 - Sabs / Wt) : 0.f;
  const float hr = Sabs > 0 ? (float)(S_re / Sabs) : 1.f, hi = Sabs > 0 ? (float)(S_im / Sabs) : 0.f;
  const float scale = Wt > 0 ? (float)(1.0 / (Wt * batch)) : 0.f;
  const long base = (long)n * HW;
  for (long p = (long)blockIdx.x * 256 + threadIdx.x; p < HW; p += (long)gridDim.x * 256) {
    const float a = out[2 * (base + p)], b = out[2 * (base + p) + 1];
    const float r = sqrtf(a * a + b * b) + 1e-12f;
    const float2 l = lab[base + p];
    const float lm = sqrtf(l.x * l.x + l.y * l.y);
    const float c = lm > 0.f ? l.x / lm : 1.f, s = lm > 0.f ? l.y / lm : 0.f;
    const float am = amp[base + p];
    // coefficient of z: amp conj(s_hat) conj(y) = am (hr - i hi)(c - i s)
    const float cr = am * (hr * c - hi * s), cim = -am * (hr * s + hi * c);
    const float ir = 1.f / r, ir3 = ir * ir * ir;
    const float da_r = ir - a * a * ir3, da_i = -a * b * ir3;
    const float db_r = -b * a * ir3, db_i = ir - b * b * ir3;
    dout[2 * (base + p)] = -(cr * da_r - cim * da_i) * scale;
    dout[2 * (base + p) + 1] = -(cr * db_r - cim * db_i) * scale;
  }
}

// head backward-data: dx[p][c] = bf16(sum_o dout[p][o] bf16(w[o][c])), zeroed
// where x[p][c] <= 0 (x is the ReLU output feeding the head)
__global__ void k_head_bwd_data(const float* __restrict__ dout, const float* __restrict__ w,
                                const u16* __restrict__ x, u16* __restrict__ dx, long P, int C) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P * C) return;
  const long p = i / C;
  const int c = (int)(i - p * C);
  float g = dout[2 * p] * bf2f(f2bf(w[c])) + dout[2 * p + 1] * bf2f(f2bf(w[C + c]));
  if (!(bf2f(x[i]) > 0.f)) g = 0.f;
  dx[i] = f2bf(g);
}

// head parameter-gradient partials over pixel chunks: columns o C + c
// (weights), then 2 C + o (bias).  Thread t takes pixels p0 + t, p0 + t + 256,
// ... of its block's chunk and keeps the 2 C + 2 sums in registers; the block
// then adds the 256 thread sums of each column in thread order.
template <int C>
__global__ __launch_bounds__(256) void k_head_wgrad(const float* __restrict__ dout, const u16* __restrict__ x,
                                                    float* __restrict__ part, long P, long chunk) {
  constexpr int NC = 2 * C + 2;
  __shared__ float red[NC][257];
  const int t = threadIdx.x;
  const long p0 = (long)blockIdx.x * chunk;
  const long p1 = std::min(p0 + chunk, P);
  float s[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) s[j] = 0.f;
  for (long p = p0 + t; p < p1; p += 256) {
    const float2 d = *reinterpret_cast<const float2*>(dout + 2 * p);
    u16 xv[C];
#pragma unroll
    for (int q = 0; q < C / 8; ++q) *reinterpret_cast<uint4*>(xv + 8 * q) = reinterpret_cast<const uint4*>(x + (size_t)p * C)[q];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float xc = bf2f(xv[c]);
      s[c] += d.x * xc;
      s[C + c] += d.y * xc;
    }
    s[2 * C] += d.x;
    s[2 * C + 1] += d.y;
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) red[j][t] = s[j];
  __syncthreads();
  if (t < NC) {
    float a = 0.f;
    for (int i = 0; i < 256; ++i) a += red[t][i];
    part[(size_t)blockIdx.x * NC + t] = a;
  }
}

// generic channel count: one thread per column, serial over the chunk
__global__ void k_head_wgrad_any(const float* __restrict__ dout, const u16* __restrict__ x, float* __restrict__ part,
                                 long P, int C, long chunk) {
  const int j = threadIdx.x;
  const int ncol = 2 * C + 2;
  if (j >= ncol) return;
  const long p0 = (long)blockIdx.x * chunk;
  const long p1 = std::min(p0 + chunk, P);
  float s = 0.f;
  if (j < 2 * C) {
    const int o = j / C, c = j - o * C;
    for (long p = p0; p < p1; ++p) s += dout[2 * p + o] * bf2f(x[(size_t)p * C + c]);
  } else {
    const int o = j - 2 * C;
    for (long p = p0; p < p1; ++p) s += dout[2 * p + o];
  }
  part[(size_t)blockIdx.x * ncol + j] = s;
}

void head_wgrad_launch(const float* dout, const u16* x, float* part, long P, int C, int nparts, hipStream_t st) {
  const long chunk = (P + nparts - 1) / nparts;
  if (C == 16)
    hipLaunchKernelGGL(k_head_wgrad<16>, dim3(nparts), dim3(256), 0, st, dout, x, part, P, chunk);
  else
    hipLaunchKernelGGL(k_head_wgrad_any, dim3(nparts), dim3(256), 0, st, dout, x, part, P, C, chunk);
}

// Adam (Kingma and Ba): m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
// p -= lr (m / c1) / (sqrt(v / c2) + eps), c1 = 1 - b1^t, c2 = 1 - b2^t
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       long n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// e^{i psi0} of the quadratic replay-plane phase
// psi0 = 2 pi ((u - nx/2)^2 / nx + (v - ny/2)^2 / ny) at centred pixel i of an
// ny x nx plane, evaluated exactly through the integer residues of the squares.
__device__ __forceinline__ float2 quadratic_phasor(long pix, int ny, int nx) {
  const long u = pix % nx - nx / 2, v = pix / nx - ny / 2;
  const double frac = (double)((u * u) % nx) / nx + (double)((v * v) % ny) / ny;
  double sd, cd;
  sincospi(2.0 * frac, &sd, &cd);
  return make_float2((float)cd, (float)sd);
}

// replay-plane start field: field = T e^{i (arg y + [quad] psi0)}, y nullable
// (NULL or 0 counts as phase 0)
__global__ void k_replay_start(const float* __restrict__ t, const float2* __restrict__ y, float2* __restrict__ field,
                               int ny, int nx, int quad, long total) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const float tv = t[i];
  float2 e = make_float2(1.f, 0.f);
  if (y) {
    const float2 q = y[i];
    const float mg = sqrtf(q.x * q.x + q.y * q.y);
    if (mg > 0.f) e = make_float2(q.x / mg, q.y / mg);
  }
  if (quad) e = hg::cmul(e, quadratic_phasor(i % ((long)ny * nx), ny, nx));
  field[i] = make_float2(tv * e.x, tv * e.y);
}

// field *= e^{sign i psi0}
__global__ void k_apply_quadratic(float2* __restrict__ field, int ny, int nx, int sign, long total) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  float2 q = quadratic_phasor(i % ((long)ny * nx), ny, nx);
  if (sign < 0) q.y = -q.y;
  field[i] = hg::cmul(field[i], q);
}

__global__ void k_project_levels(const float2* __restrict__ g, uint8_t* __restrict__ levels, int L, long total) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  levels[i] = (uint8_t)hg::level_index(g[i], L);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
}  // namespace

namespace hg_internal {
void set_error(const char* msg);  // the buffer hg_last_error returns
}

namespace {

hg_status nn_fail(hg_status s, const char* msg) {
  hg_internal::set_error(msg);
  return s;
}
void clear_error() { hg_internal::set_error(""); }
hg_status nn_launch_status() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    char buf[256];
    snprintf(buf, sizeof(buf), "HIP launch failed: %s", hipGetErrorString(e));
    hg_internal::set_error(buf);
    return HG_ERR_HIP;
  }
  return HG_OK;
}
inline unsigned nblk(long n, int t) { return (unsigned)((n + t - 1) / t); }
inline int kpad_of(int K) { return (K + 31) / 32 * 32; }

// ---- element-wise launchers: 16-byte kernels when the channels allow ----
void pool_launch(const u16* x, u16* y, int N, int H, int W, int C, hipStream_t st) {
  if (C % 8 == 0) {
    const long cnt = (long)N * (H / 2) * (W / 2) * (C / 8);
    hipLaunchKernelGGL(k_avgpool2_v8, dim3(nblk(cnt, 256)), dim3(256), 0, st, x, y, N, H, W, C);
  } else {
    const long cnt = (long)N * (H / 2) * (W / 2) * C;
    hipLaunchKernelGGL(k_avgpool2, dim3(nblk(cnt, 256)), dim3(256), 0, st, x, y, N, H, W, C);
  }
}
void pool_bwd_launch(const u16* dy, const u16* dskip, const u16* mask, u16* dx, int N, int H, int W, int C,
                     hipStream_t st) {
  if (C % 8 == 0) {
    const long cnt = (long)N * H * W * (C / 8);
    hipLaunchKernelGGL(k_avgpool2_bwd_v8, dim3(nblk(cnt, 256)), dim3(256), 0, st, dy, dskip, mask, dx, N, H, W, C);
  } else {
    const long cnt = (long)N * H * W * C;
    hipLaunchKernelGGL(k_avgpool2_bwd, dim3(nblk(cnt, 256)), dim3(256), 0, st, dy, dskip, mask, dx, N, H, W, C);
  }
}
void upcat_launch(const u16* lo, const u16* skip, u16* out, int N, int H, int W, int C1, int C2, hipStream_t st) {
  if (C1 % 8 == 0 && C2 % 8 == 0) {
    const long cnt = (long)N * H * W * ((C1 + C2) / 8);
    hipLaunchKernelGGL(k_upcat_v8, dim3(nblk(cnt, 256)), dim3(256), 0, st, lo, skip, out, N, H, W, C1, C2);
  } else {
    const long cnt = (long)N * H * W * (C1 + C2);
    hipLaunchKernelGGL(k_upcat, dim3(nblk(cnt, 256)), dim3(256), 0, st, lo, skip, out, N, H, W, C1, C2);
  }
}
void upcat_bwd_launch(const u16* dout, const u16* mask_lo, u16* dlo, u16* dskip, int N, int H, int W, int C1, int C2,
                      hipStream_t st) {
  if (C1 % 8 == 0 && C2 % 8 == 0) {
    const long cnt = (long)N * (H / 2) * (W / 2) * (C1 / 8) + (long)N * H * W * (C2 / 8);
    hipLaunchKernelGGL(k_upcat_bwd_v8, dim3(nblk(cnt, 256)), dim3(256), 0, st, dout, mask_lo, dlo, dskip, N, H, W, C1,
                       C2);
  } else {
    const long cnt = (long)N * (H / 2) * (W / 2) * C1 + (long)N * H * W * C2;
    hipLaunchKernelGGL(k_upcat_bwd, dim3(nblk(cnt, 256)), dim3(256), 0, st, dout, mask_lo, dlo, dskip, N, H, W, C1,
                       C2);
  }
}
void head_launch(const u16* x, const float* w, const float* b, float* out, long P, int C, hipStream_t st) {
  if (C == 16)
    hipLaunchKernelGGL(k_head16, dim3(nblk(P, 256)), dim3(256), 0, st, x, w, b, out, P);
  else
    hipLaunchKernelGGL(k_head, dim3(nblk(P, 256)), dim3(256), 0, st, x, w, b, out, P, C);
}
void head_bwd_launch(const float* dout, const float* w, const u16* x, u16* dx, long P, int C, hipStream_t st) {
  if (C == 16)
    hipLaunchKernelGGL(k_head_bwd_data16, dim3(nblk(P, 256)), dim3(256), 0, st, dout, w, x, dx, P);
  else
    hipLaunchKernelGGL(k_head_bwd_data, dim3(nblk(P * C, 256)), dim3(256), 0, st, dout, w, x, dx, P, C);
}

// ---- layer launchers (arguments validated by the callers) ----
constexpr size_t kTileLdsMax = 64 * 1024;

// Smallest input channel count the channel-chunked kernel serves (below it
// the LDS-tiled kernel does): 32 by default; HG_CONV_CC_MIN overrides it
// for comparisons (a large value switches the chunked kernel off).
// Smallest input channel count the MFMA weight-gradient kernel serves (1:
// every Cin % 16 == 0 layer); HG_WGRAD_CC_MIN overrides it for comparisons.
int wgrad_cc_min_cin() {
  static const int v = [] {
    const char* e = getenv("HG_WGRAD_CC_MIN");
    return e ? atoi(e) : 1;
  }();
  return v;
}

int cc_min_cin() {
  static const int v = [] {
    const char* e = getenv("HG_CONV_CC_MIN");
    return e ? atoi(e) : 32;
  }();
  return v;
}

// Tile shape of k_conv3x3_tile for this layer, largest first; false if none fits.
bool tile_shape(int W, int Cin, int NB, int* R, int* TW, int* GW) {
  if (Cin % 8 || W % 16) return false;
  static const int cand[][3] = {{4, 64, 4}, {2, 64, 2}, {4, 32, 2}, {2, 32, 1}, {1, 64, 1}, {4, 16, 1}};
  for (const auto& c : cand) {
    if (c[1] > W && c[1] > 16) continue;
    const size_t lds = ((size_t)(c[0] + 2) * (c[1] + 2) * tile_pixel_stride(Cin) + (size_t)c[0] * c[1] * 16 * NB) * 2;
    if (lds > kTileLdsMax) continue;
    *R = c[0];
    *TW = c[1];
    *GW = c[2];
    return true;
  }
  return false;
}

template <int NB, bool A32>
void conv_tile_launch_a(int GW, dim3 grid, size_t lds, hipStream_t st, const u16* X, const u16* Wg, const float* bias,
                        const u16* mask, u16* Y, int H, int W, int Cin, int Cout, int Kp, int relu, int TW, int R) {
  if (GW == 4)
    hipLaunchKernelGGL((k_conv3x3_tile<NB, 4, A32>), grid, dim3(256), lds, st, X, Wg, bias, mask, Y, H, W, Cin, Cout,
                       Kp, relu, TW, R);
  else if (GW == 2)
    hipLaunchKernelGGL((k_conv3x3_tile<NB, 2, A32>), grid, dim3(256), lds, st, X, Wg, bias, mask, Y, H, W, Cin, Cout,
                       Kp, relu, TW, R);
  else
    hipLaunchKernelGGL((k_conv3x3_tile<NB, 1, A32>), grid, dim3(256), lds, st, X, Wg, bias, mask, Y, H, W, Cin, Cout,
                       Kp, relu, TW, R);
}
template <int NB>
void conv_tile_launch(int GW, dim3 grid, size_t lds, hipStream_t st, const u16* X, const u16* Wg, const float* bias,
                      const u16* mask, u16* Y, int H, int W, int Cin, int Cout, int Kp, int relu, int TW, int R) {
  if (Cin % 32 == 0)
    conv_tile_launch_a<NB, true>(GW, grid, lds, st, X, Wg, bias, mask, Y, H, W, Cin, Cout, Kp, relu, TW, R);
  else
    conv_tile_launch_a<NB, false>(GW, grid, lds, st, X, Wg, bias, mask, Y, H, W, Cin, Cout, Kp, relu, TW, R);
}

void conv_launch(const u16* X, const u16* Wg, const float* bias, const u16* mask, u16* Y, long P, int H, int W,
                 int Cin, int Cout, int relu, hipStream_t st) {
  const int nb16 = Cout / 16;
  const int NB = nb16 % 4 == 0 ? 4 : nb16 % 3 == 0 ? 3 : nb16 % 2 == 0 ? 2 : 1;
  int R, TW, GW;
  if (P / ((long)H * W) <= 65535 && Cin % 16 == 0 && Cin >= cc_min_cin() && W >= kCcTW &&
      (long)H * W * Cin < (1L << 31)) {
    // channel-chunked kernel, 4 x 64 pixel tiles (images on grid.z)
    const long N = P / ((long)H * W);
    const long tiles = (long)(H / kCcR + (H % kCcR ? 1 : 0)) * (W / kCcTW + (W % kCcTW ? 1 : 0));
    const dim3 grid((unsigned)tiles, nb16 / NB, (unsigned)N);
    const int Kp = kpad_of(9 * Cin);
#define HG_CC(NBV) \
  hipLaunchKernelGGL((k_conv3x3_cc<NBV>), grid, dim3(256), 0, st, X, Wg, bias, mask, Y, H, W, Cin, Cout, Kp, relu);
    switch (NB) {
      case 4: HG_CC(4) break;
      case 3: HG_CC(3) break;
      case 2: HG_CC(2) break;
      default: HG_CC(1) break;
    }
#undef HG_CC
    return;
  }
  if (P / ((long)H * W) <= 65535 && tile_shape(W, Cin, NB, &R, &TW, &GW)) {  // images on grid.z
    const long N = P / ((long)H * W);
    const long tiles = (long)(H / R + (H % R ? 1 : 0)) * (W / TW + (W % TW ? 1 : 0));
    const dim3 grid((unsigned)tiles, nb16 / NB, (unsigned)N);
    const size_t lds = ((size_t)(R + 2) * (TW + 2) * tile_pixel_stride(Cin) + (size_t)R * TW * 16 * NB) * 2;
    const int Kp = kpad_of(9 * Cin);
    switch (NB) {
      case 4: conv_tile_launch<4>(GW, grid, lds, st, X, Wg, bias, mask, Y, H, W, Cin, Cout, Kp, relu, TW, R); break;
      case 3: conv_tile_launch<3>(GW, grid, lds, st, X, Wg, bias, mask, Y, H, W, Cin, Cout, Kp, relu, TW, R); break;
      case 2: conv_tile_launch<2>(GW, grid, lds, st, X, Wg, bias, mask, Y, H, W, Cin, Cout, Kp, relu, TW, R); break;
      default: conv_tile_launch<1>(GW, grid, lds, st, X, Wg, bias, mask, Y, H, W, Cin, Cout, Kp, relu, TW, R); break;
    }
    return;
  }
  if (Cin == 1 && Cout == 16) {
    hipLaunchKernelGGL(k_conv_first16, dim3(nblk(P, 256)), dim3(256), 0, st, X, Wg, bias, mask, Y, P, H, W,
                       kpad_of(9), relu);
    return;
  }
  const dim3 grid(nblk(P, 64), nb16 / NB);
  const bool vec = (Cin % 8) == 0;
  const int Kp = kpad_of(9 * Cin);
#define HG_CONV(NBV)                                                                                               \
  if (vec)                                                                                                         \
    hipLaunchKernelGGL((k_conv3x3<NBV, true>), grid, dim3(256), 0, st, X, Wg, bias, mask, Y, P, H, W, Cin, Cout,   \
                       Kp, relu);                                                                                  \
  else                                                                                                             \
    hipLaunchKernelGGL((k_conv3x3<NBV, false>), grid, dim3(256), 0, st, X, Wg, bias, mask, Y, P, H, W, Cin, Cout, \
                       Kp, relu);
  switch (NB) {
    case 4: HG_CONV(4) break;
    case 3: HG_CONV(3) break;
    case 2: HG_CONV(2) break;
    default: HG_CONV(1) break;
  }
#undef HG_CONV
}

struct WgradPlan {
  long pb_len;
  int npb;
};
WgradPlan wgrad_plan(long P, int Cin, int Cout) {
  const int Kp = kpad_of(9 * Cin);
  const long tiles = (long)(Cout / 16) * ((Kp + 63) / 64);
  const long want = std::max(1L, 2048 / tiles);  // about 2048 workgroups in all
  long pb = (P + want - 1) / want;
  pb = std::max(256L, (pb + 31) / 32 * 32);
  return {pb, (int)((P + pb - 1) / pb)};
}
// The MFMA weight-gradient kernel (k_wgrad_cc): whether it serves a layer,
// its output-channel blocks, and a workgroup count of about 512 (two per CU
// resident) as blocks of consecutive 2 x 64 pixel tiles; more blocks make
// the partials' reduction cost more than they save.
constexpr long kWgTarget = 512;
bool wgrad_cc_ok(long P, int Cin, int Cout) {
  return Cin % 16 == 0 && Cout % 16 == 0 && Cin >= wgrad_cc_min_cin() && P * (long)std::max(Cin, Cout) < (1L << 31);
}
int wgrad_cc_nb(int Cout) {
  const int nb16 = Cout / 16;
  return nb16 % 4 == 0 ? 4 : nb16 % 2 == 0 ? 2 : 1;
}
long wgrad_cc_max_blocks(int Cin, int Cout) {
  const long gyz = (long)(Cout / 16 / wgrad_cc_nb(Cout)) * ((Cin + 31) / 32);
  return std::max(1L, kWgTarget / gyz);
}
size_t wgrad_ws_bytes(long P, int Cin, int Cout) {
  const WgradPlan w = wgrad_plan(P, Cin, Cout);
  long npb = w.npb;
  if (wgrad_cc_ok(P, Cin, Cout)) npb = std::max(npb, wgrad_cc_max_blocks(Cin, Cout));
  return al256((size_t)npb * Cout * kpad_of(9 * Cin) * sizeof(float)) + al256((size_t)npb * Cout * sizeof(float));
}
void wgrad_launch(const u16* X, const u16* dY, float* dw, float* db, long P, int H, int W, int Cin, int Cout,
                  char* ws, hipStream_t st) {
  const WgradPlan wp = wgrad_plan(P, Cin, Cout);
  const int Kp = kpad_of(9 * Cin);
  const bool cc = wgrad_cc_ok(P, Cin, Cout);
  // partial slots of the workspace (as sized by wgrad_ws_bytes)
  const long slots = cc ? std::max((long)wp.npb, wgrad_cc_max_blocks(Cin, Cout)) : wp.npb;
  float* part = reinterpret_cast<float*>(ws);
  float* bpart = db ? reinterpret_cast<float*>(ws + al256((size_t)slots * Cout * Kp * sizeof(float))) : nullptr;
  int npb = wp.npb;
  const long N = P / ((long)H * W);
  if (cc) {
    // MFMA over pixel tiles (k_wgrad_cc): blocks of consecutive 2 x 64
    // pixel tiles, at most wgrad_cc_max_blocks of them
    const int nb16 = Cout / 16, NB = wgrad_cc_nb(Cout);
    const long ntiles = N * ((H + 1) / 2) * ((W + 63) / 64);
    const long want = std::min(ntiles, wgrad_cc_max_blocks(Cin, Cout));
    const long tpb = (ntiles + want - 1) / want;
    npb = (int)((ntiles + tpb - 1) / tpb);
    const dim3 grid((unsigned)npb, nb16 / NB, (Cin + 31) / 32);
#define HG_WG(NBV)                                                                                                  \
  hipLaunchKernelGGL((k_wgrad_cc<NBV>), grid, dim3(256), 0, st, X, dY, part, bpart, H, W, Cin, Cout, Kp, (int)tpb, \
                     (int)ntiles);
    switch (NB) {
      case 4: HG_WG(4) break;
      case 2: HG_WG(2) break;
      default: HG_WG(1) break;
    }
#undef HG_WG
  } else {
    hipLaunchKernelGGL(k_conv3x3_wgrad, dim3(wp.npb, Cout / 16, (Kp + 63) / 64), dim3(256), 0, st, X, dY, part,
                       bpart, P, H, W, Cin, Cout, Kp, wp.pb_len);
  }
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblk((long)Cout * 9 * Cin, 256)), dim3(256), 0, st, part, dw, npb, Cout,
                     Kp, 9 * Cin);
  if (db) hipLaunchKernelGGL(k_sum_parts, dim3(nblk(Cout, 256)), dim3(256), 0, st, bpart, db, npb, Cout);
}

constexpr int kLossParts = 64;
constexpr int kHeadParts = 256;

// ---- the fixed network: encoder 16/32/64/128, decoder back to 16, head 2 ----
constexpr int kLevels = 4;
constexpr int kEnc[kLevels] = {16, 32, 64, 128};
enum { E0A, E0B, E1A, E1B, E2A, E2B, E3A, E3B, D2A, D2B, D1A, D1B, D0A, D0B, HEAD, NLAYER };

struct Layer {
  int cin, cout, level;
  size_t w, b;  // float offsets into the parameter vector
};

struct Net {
  Layer L[NLAYER];
  size_t nparams;
  Net() {
    int k = 0;
    int cin = 1;
    for (int l = 0; l < kLevels; ++l) {
      L[k++] = {cin, kEnc[l], l, 0, 0};
      L[k++] = {kEnc[l], kEnc[l], l, 0, 0};
      cin = kEnc[l];
    }
    for (int l = kLevels - 2; l >= 0; --l) {
      L[k++] = {cin + kEnc[l], kEnc[l], l, 0, 0};
      L[k++] = {kEnc[l], kEnc[l], l, 0, 0};
      cin = kEnc[l];
    }
    L[k++] = {cin, 2, 0, 0, 0};
    size_t off = 0;
    for (int i = 0; i < NLAYER; ++i) {
      L[i].w = off;
      off += (size_t)L[i].cout * (i == HEAD ? 1 : 9) * L[i].cin;
      L[i].b = off;
      off += L[i].cout;
    }
    nparams = off;
  }
};
const Net& net() {
  static const Net n;
  return n;
}
// decoder layer pair at level l: D{l}A, D{l}B
inline int dec_a(int l) { return D2A + 2 * (kLevels - 2 - l); }

// Workspace plan for a batch of B images of H x W (byte offsets).
struct Plan {
  long P[kLevels];  // pixels per level
  size_t wg_f[NLAYER], wg_b[NLAYER];
  size_t x;                       // input, bf16 [P0]
  size_t act[NLAYER];             // conv layer outputs
  size_t pool[kLevels - 1];       // pooled e{l}b outputs (input of e{l+1}a)
  size_t cat[kLevels - 1];        // decoder concatenations at level l
  size_t gbuf[3];                 // rotating gradient buffers
  size_t skipg[kLevels - 1];      // skip-connection gradients
  size_t dout;                    // fp32 [P0][2]
  size_t scratch;                 // wgrad partials / reductions
  size_t total;
};

Plan make_plan(int B, int H, int W) {
  const Net& n = net();
  Plan p{};
  for (int l = 0; l < kLevels; ++l) p.P[l] = (long)B * (H >> l) * (W >> l);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += al256(bytes);
    return o;
  };
  for (int i = 0; i < HEAD; ++i) {
    p.wg_f[i] = take((size_t)n.L[i].cout * kpad_of(9 * n.L[i].cin) * 2);
    p.wg_b[i] = i == E0A ? 0 : take((size_t)n.L[i].cin * kpad_of(9 * n.L[i].cout) * 2);
  }
  p.x = take((size_t)p.P[0] * 2);
  for (int i = 0; i < HEAD; ++i) p.act[i] = take((size_t)p.P[n.L[i].level] * n.L[i].cout * 2);
  for (int l = 0; l < kLevels - 1; ++l) p.pool[l] = take((size_t)p.P[l + 1] * kEnc[l] * 2);
  for (int l = 0; l < kLevels - 1; ++l) p.cat[l] = take((size_t)p.P[l] * (kEnc[l + 1] + kEnc[l]) * 2);
  size_t gb = 0;
  for (int l = 0; l < kLevels; ++l) {
    const int cmax = l < kLevels - 1 ? kEnc[l + 1] + kEnc[l] : kEnc[l];
    gb = std::max(gb, (size_t)p.P[l] * cmax * 2);
  }
  for (int j = 0; j < 3; ++j) p.gbuf[j] = take(gb);
  for (int l = 0; l < kLevels - 1; ++l) p.skipg[l] = take((size_t)p.P[l] * kEnc[l] * 2);
  p.dout = take((size_t)p.P[0] * 2 * sizeof(float));
  size_t sc = al256((size_t)B * 64 * sizeof(double));                    // input scaling
  sc = std::max(sc, al256((size_t)B * kLossParts * 3 * sizeof(double)));  // loss
  sc = std::max(sc, al256((size_t)kHeadParts * (2 * kEnc[0] + 2) * sizeof(float)));
  for (int i = 0; i < HEAD; ++i) sc = std::max(sc, wgrad_ws_bytes(p.P[n.L[i].level], n.L[i].cin, n.L[i].cout));
  p.scratch = take(sc);
  p.total = off;
  return p;
}

hg_status check_net_shape(int B, int H, int W) {
  if (B < 1 || H < 8 || W < 8 || (H % 8) || (W % 8))
    return nn_fail(HG_ERR_UNSUPPORTED_SIZE, "network needs batch >= 1 and height, width multiples of 8");
  if ((long)B * H * W * 48 > (1L << 31)) return nn_fail(HG_ERR_UNSUPPORTED_SIZE, "network batch too large");
  return HG_OK;
}
hg_status check_ws(const void* ws, size_t have, size_t need) {
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
    return nn_fail(HG_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  if (have < need) return nn_fail(HG_ERR_WORKSPACE, "workspace smaller than the query");
  return HG_OK;
}

}  // namespace

extern "C" {

/* ---------------- layer-level entry points ---------------- */

int hg_nn_kpad(int k) { return k < 1 ? 0 : kpad_of(k); }

hg_status hg_nn_pack_weights(const float* w, void* wg, int cout, int cin, int flip, void* stream) {
  clear_error();
  if (!w || !wg || cout < 1 || cin < 1)
    return nn_fail(HG_ERR_INVALID_ARG, "pack_weights: NULL buffer or channels < 1");
  const int Kp = flip ? kpad_of(9 * cout) : kpad_of(9 * cin);
  const long n = (long)(flip ? cin : cout) * Kp;
  hipLaunchKernelGGL(k_pack_weights, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, w, (u16*)wg, cout, cin,
                     Kp, flip);
  return nn_launch_status();
}

hg_status hg_nn_conv3x3(const void* x, const void* wg, const float* bias, const void* mask, void* y, int n, int h,
                        int w, int cin, int cout, int relu, void* stream) {
  clear_error();
  if (!x || !wg || !y) return nn_fail(HG_ERR_INVALID_ARG, "conv3x3: NULL buffer");
  if (n < 1 || h < 1 || w < 1 || cin < 1 || cout < 16 || (cout % 16))
    return nn_fail(HG_ERR_INVALID_ARG, "conv3x3: needs n, h, w, cin >= 1 and cout a multiple of 16");
  if ((long)n * h * w * std::max(cin, cout) > (1L << 31))
    return nn_fail(HG_ERR_UNSUPPORTED_SIZE, "conv3x3: tensor too large");
  conv_launch((const u16*)x, (const u16*)wg, bias, (const u16*)mask, (u16*)y, (long)n * h * w, h, w, cin, cout, relu,
              (hipStream_t)stream);
  return nn_launch_status();
}

size_t hg_nn_wgrad_workspace_size(int n, int h, int w, int cin, int cout) {
  if (n < 1 || h < 1 || w < 1 || cin < 1 || cout < 16 || (cout % 16) || cout > 256) return 0;
  return wgrad_ws_bytes((long)n * h * w, cin, cout);
}

hg_status hg_nn_conv3x3_wgrad(const void* x, const void* dy, float* dw, float* db, int n, int h, int w, int cin,
                              int cout, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!x || !dy || !dw) return nn_fail(HG_ERR_INVALID_ARG, "wgrad: NULL buffer");
  if (n < 1 || h < 1 || w < 1 || cin < 1 || cout < 16 || (cout % 16) || cout > 256)
    return nn_fail(HG_ERR_INVALID_ARG, "wgrad: needs cout a multiple of 16 up to 256");
  if ((long)n * h * w * std::max(cin, cout) > (1L << 31))
    return nn_fail(HG_ERR_UNSUPPORTED_SIZE, "wgrad: tensor too large");
  hg_status s = check_ws(ws, ws_bytes, hg_nn_wgrad_workspace_size(n, h, w, cin, cout));
  if (s != HG_OK) return s;
  wgrad_launch((const u16*)x, (const u16*)dy, dw, db, (long)n * h * w, h, w, cin, cout, (char*)ws,
               (hipStream_t)stream);
  return nn_launch_status();
}

hg_status hg_nn_avgpool2(const void* x, void* y, int n, int h, int w, int c, void* stream) {
  clear_error();
  if (!x || !y || n < 1 || h < 2 || w < 2 || ((h | w) & 1) || c < 1)
    return nn_fail(HG_ERR_INVALID_ARG, "avgpool2: NULL buffer or odd/small size");
  pool_launch((const u16*)x, (u16*)y, n, h, w, c, (hipStream_t)stream);
  return nn_launch_status();
}

hg_status hg_nn_avgpool2_backward(const void* dy, const void* dskip, const void* mask, void* dx, int n, int h, int w,
                                  int c, void* stream) {
  clear_error();
  if (!dy || !dx || n < 1 || h < 2 || w < 2 || ((h | w) & 1) || c < 1)
    return nn_fail(HG_ERR_INVALID_ARG, "avgpool2_backward: NULL buffer or odd/small size");
  pool_bwd_launch((const u16*)dy, (const u16*)dskip, (const u16*)mask, (u16*)dx, n, h, w, c, (hipStream_t)stream);
  return nn_launch_status();
}

hg_status hg_nn_upsample_concat(const void* lo, const void* skip, void* out, int n, int h, int w, int c1, int c2,
                                void* stream) {
  clear_error();
  if (!lo || !skip || !out || n < 1 || h < 2 || w < 2 || ((h | w) & 1) || c1 < 1 || c2 < 1)
    return nn_fail(HG_ERR_INVALID_ARG, "upsample_concat: NULL buffer or bad size");
  upcat_launch((const u16*)lo, (const u16*)skip, (u16*)out, n, h, w, c1, c2, (hipStream_t)stream);
  return nn_launch_status();
}

hg_status hg_nn_upsample_concat_backward(const void* dout, const void* mask_lo, void* dlo, void* dskip, int n, int h,
                                         int w, int c1, int c2, void* stream) {
  clear_error();
  if (!dout || !dlo || !dskip || n < 1 || h < 2 || w < 2 || ((h | w) & 1) || c1 < 1 || c2 < 1)
    return nn_fail(HG_ERR_INVALID_ARG, "upsample_concat_backward: NULL buffer or bad size");
  upcat_bwd_launch((const u16*)dout, (const u16*)mask_lo, (u16*)dlo, (u16*)dskip, n, h, w, c1, c2,
                   (hipStream_t)stream);
  return nn_launch_status();
}

hg_status hg_nn_head(const void* x, const float* w, const float* b, float* out, long pixels, int c, void* stream) {
  clear_error();
  if (!x || !w || !b || !out || pixels < 1 || c < 1) return nn_fail(HG_ERR_INVALID_ARG, "head: NULL buffer or size");
  head_launch((const u16*)x, w, b, out, pixels, c, (hipStream_t)stream);
  return nn_launch_status();
}

size_t hg_nn_loss_workspace_size(int batch) {
  return batch < 1 ? 0 : al256((size_t)batch * kLossParts * 3 * sizeof(double));
}

hg_status hg_nn_phase_loss(const float* out, const hg_complex* label, const float* amp, float* dout, float* loss,
                           int batch, long hw, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!out || !label || !amp || !dout || batch < 1 || hw < 1)
    return nn_fail(HG_ERR_INVALID_ARG, "phase_loss: NULL buffer or size");
  hg_status s = check_ws(ws, ws_bytes, hg_nn_loss_workspace_size(batch));
  if (s != HG_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const float2* lab = reinterpret_cast<const float2*>(label);
  hipLaunchKernelGGL(k_loss_part, dim3(kLossParts, batch), dim3(256), 0, st, out, lab, amp, (double*)ws, hw);
  hipLaunchKernelGGL(k_loss_grad, dim3(kLossParts, batch), dim3(256), 0, st, out, lab, amp, (const double*)ws,
                     kLossParts, dout, loss, hw, batch);
  return nn_launch_status();
}

size_t hg_nn_head_workspace_size(int c) {
  return c < 1 || 2 * c + 2 > 256 ? 0 : al256((size_t)kHeadParts * (2 * c + 2) * sizeof(float));
}

hg_status hg_nn_head_backward(const float* dout, const float* w, const void* x, void* dx, float* dwb, long pixels,
                              int c, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!dout || !w || !x || !dx || !dwb || pixels < 1 || c < 1 || 2 * c + 2 > 256)
    return nn_fail(HG_ERR_INVALID_ARG, "head_backward: NULL buffer or channels outside 1..127");
  hg_status s = check_ws(ws, ws_bytes, hg_nn_head_workspace_size(c));
  if (s != HG_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  float* part = (float*)ws;
  head_bwd_launch(dout, w, (const u16*)x, (u16*)dx, pixels, c, st);
  head_wgrad_launch(dout, (const u16*)x, part, pixels, c, kHeadParts, st);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, part, dwb, kHeadParts, 2 * c + 2);
  return nn_launch_status();
}

hg_status hg_nn_adam(float* params, const float* grads, float* m, float* v, long count, float lr, float beta1,
                     float beta2, float eps, int step, void* stream) {
  clear_error();
  if (!params || !grads || !m || !v || count < 1 || step < 1)
    return nn_fail(HG_ERR_INVALID_ARG, "adam: NULL buffer, count < 1 or step < 1");
  const float c1 = (float)(1.0 - pow((double)beta1, step)), c2 = (float)(1.0 - pow((double)beta2, step));
  hipLaunchKernelGGL(k_adam, dim3(nblk(count, 256)), dim3(256), 0, (hipStream_t)stream, params, grads, m, v, count,
                     lr, beta1, beta2, eps, c1, c2);
  return nn_launch_status();
}

/* ---------------- whole network ---------------- */

long hg_nn_param_count(void) { return (long)net().nparams; }

size_t hg_nn_workspace_size(int batch, int h, int w) {
  if (check_net_shape(batch, h, w) != HG_OK) return 0;
  return make_plan(batch, h, w).total;
}

hg_status hg_nn_forward(const float* params, const float* target, int batch, int h, int w, float* out, void* ws,
                        size_t ws_bytes, void* stream) {
  clear_error();
  if (!params || !target || !out) return nn_fail(HG_ERR_INVALID_ARG, "forward: NULL buffer");
  hg_status s = check_net_shape(batch, h, w);
  if (s != HG_OK) return s;
  const Plan p = make_plan(batch, h, w);
  s = check_ws(ws, ws_bytes, p.total);
  if (s != HG_OK) return s;
  const Net& n = net();
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  auto A = [&](size_t off) { return reinterpret_cast<u16*>(base + off); };
  for (int i = 0; i < HEAD; ++i) {
    const int Kp = kpad_of(9 * n.L[i].cin);
    const long cnt = (long)n.L[i].cout * Kp;
    hipLaunchKernelGGL(k_pack_weights, dim3(nblk(cnt, 256)), dim3(256), 0, st, params + n.L[i].w, A(p.wg_f[i]),
                       n.L[i].cout, n.L[i].cin, Kp, 0);
  }
  const long HW = (long)h * w;
  double* npart = reinterpret_cast<double*>(base + p.scratch);
  hipLaunchKernelGGL(k_sumsq_part, dim3(64, batch), dim3(256), 0, st, target, npart, HW);
  hipLaunchKernelGGL(k_input, dim3(64, batch), dim3(256), 0, st, target, (const double*)npart, 64, A(p.x), HW);
  auto conv = [&](int i, const u16* in) {
    const int l = n.L[i].level;
    conv_launch(in, A(p.wg_f[i]), params + n.L[i].b, nullptr, A(p.act[i]), p.P[l], h >> l, w >> l, n.L[i].cin,
                n.L[i].cout, 1, st);
  };
  const u16* cur = A(p.x);
  for (int l = 0; l < kLevels; ++l) {
    conv(2 * l, cur);
    conv(2 * l + 1, A(p.act[2 * l]));
    if (l < kLevels - 1) {
      pool_launch(A(p.act[2 * l + 1]), A(p.pool[l]), batch, h >> l, w >> l, kEnc[l], st);
      cur = A(p.pool[l]);
    } else {
      cur = A(p.act[2 * l + 1]);
    }
  }
  for (int l = kLevels - 2; l >= 0; --l) {
    const int ia = dec_a(l);
    const int c1 = kEnc[l + 1], c2 = kEnc[l];
    upcat_launch(cur, A(p.act[2 * l + 1]), A(p.cat[l]), batch, h >> l, w >> l, c1, c2, st);
    conv(ia, A(p.cat[l]));
    conv(ia + 1, A(p.act[ia]));
    cur = A(p.act[ia + 1]);
  }
  head_launch(cur, params + n.L[HEAD].w, params + n.L[HEAD].b, out, p.P[0], n.L[HEAD].cin, st);
  return nn_launch_status();
}

hg_status hg_nn_backward(const float* params, const float* out, const hg_complex* label, const float* amp, int batch,
                         int h, int w, float* grads, float* loss_out, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!params || !out || !label || !amp || !grads) return nn_fail(HG_ERR_INVALID_ARG, "backward: NULL buffer");
  hg_status s = check_net_shape(batch, h, w);
  if (s != HG_OK) return s;
  const Plan p = make_plan(batch, h, w);
  s = check_ws(ws, ws_bytes, p.total);
  if (s != HG_OK) return s;
  const Net& n = net();
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  auto A = [&](size_t off) { return reinterpret_cast<u16*>(base + off); };
  char* scratch = base + p.scratch;
  for (int i = E0B; i < HEAD; ++i) {
    const int Kp = kpad_of(9 * n.L[i].cout);
    const long cnt = (long)n.L[i].cin * Kp;
    hipLaunchKernelGGL(k_pack_weights, dim3(nblk(cnt, 256)), dim3(256), 0, st, params + n.L[i].w, A(p.wg_b[i]),
                       n.L[i].cout, n.L[i].cin, Kp, 1);
  }
  const long HW = (long)h * w;
  float* dout = reinterpret_cast<float*>(base + p.dout);
  const float2* lab = reinterpret_cast<const float2*>(label);
  hipLaunchKernelGGL(k_loss_part, dim3(kLossParts, batch), dim3(256), 0, st, out, lab, amp, (double*)scratch, HW);
  hipLaunchKernelGGL(k_loss_grad, dim3(kLossParts, batch), dim3(256), 0, st, out, lab, amp, (const double*)scratch,
                     kLossParts, dout, loss_out, HW, batch);
  int gi = 0;  // next rotating gradient buffer
  auto G = [&]() {
    u16* b = A(p.gbuf[gi]);
    gi = (gi + 1) % 3;
    return b;
  };
  // head: the masked gradient of d0b's output, and the head's own gradients
  // (its weights 2 c0 and bias 2 are adjacent in the parameter vector)
  const int c0 = n.L[HEAD].cin;
  u16* dh = G();
  {
    float* part = reinterpret_cast<float*>(scratch);
    head_bwd_launch(dout, params + n.L[HEAD].w, A(p.act[D0B]), dh, p.P[0], c0, st);
    head_wgrad_launch(dout, A(p.act[D0B]), part, p.P[0], c0, kHeadParts, st);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, part, grads + n.L[HEAD].w, kHeadParts, 2 * c0 + 2);
  }
  // one conv layer: dz (already masked) -> weight and bias gradients, and the
  // data gradient into dst, masked with `mask` (nullable); dst NULL skips it
  auto conv_bwd = [&](int i, const u16* in, const u16* dz, const u16* mask, u16* dst) {
    const int l = n.L[i].level;
    wgrad_launch(in, dz, grads + n.L[i].w, grads + n.L[i].b, p.P[l], h >> l, w >> l, n.L[i].cin, n.L[i].cout,
                 scratch, st);
    if (dst)
      conv_launch(dz, A(p.wg_b[i]), nullptr, mask, dst, p.P[l], h >> l, w >> l, n.L[i].cout, n.L[i].cin, 0, st);
  };
  // decoder, level 0 up to level kLevels - 2
  for (int l = 0; l < kLevels - 1; ++l) {
    const int ia = dec_a(l), ib = ia + 1;
    u16* dza = G();
    conv_bwd(ib, A(p.act[ia]), dh, A(p.act[ia]), dza);
    u16* dcat = G();
    conv_bwd(ia, A(p.cat[l]), dza, nullptr, dcat);
    const int c1 = kEnc[l + 1], c2 = kEnc[l];
    const u16* lower = l + 1 < kLevels - 1 ? A(p.act[dec_a(l + 1) + 1]) : A(p.act[E3B]);
    u16* dlo = G();
    upcat_bwd_launch(dcat, lower, dlo, A(p.skipg[l]), batch, h >> l, w >> l, c1, c2, st);
    dh = dlo;
  }
  // encoder, deepest level first; dh is the masked gradient of e{l}b's output
  // (at l < kLevels - 1 after adding the pooled path and the skip gradient)
  for (int l = kLevels - 1; l >= 0; --l) {
    if (l < kLevels - 1) {
      u16* d = G();
      pool_bwd_launch(dh, A(p.skipg[l]), A(p.act[2 * l + 1]), d, batch, h >> l, w >> l, kEnc[l], st);
      dh = d;
    }
    u16* dza = G();
    conv_bwd(2 * l + 1, A(p.act[2 * l]), dh, A(p.act[2 * l]), dza);
    const u16* ain = l == 0 ? A(p.x) : A(p.pool[l - 1]);
    u16* dpool = l == 0 ? nullptr : G();
    conv_bwd(2 * l, ain, dza, nullptr, dpool);
    dh = dpool;
  }
  return nn_launch_status();
}

/* ---------------- replay-plane phase -> SLM start levels ---------------- */

size_t hg_replay_phase_init_workspace_size(int batch, int ny, int nx) {
  if (batch < 1) return 0;
  const size_t prop = hg_workspace_size(HG_OP_PROPAGATE, ny, nx, 1);
  if (!prop) return 0;
  return al256((size_t)batch * ny * nx * sizeof(float2)) + prop;
}

hg_status hg_quadratic_phase_apply(hg_complex* field, int batch, int ny, int nx, int sign, void* stream) {
  clear_error();
  if (!field || batch < 1 || ny < 1 || nx < 1 || (sign != 1 && sign != -1))
    return nn_fail(HG_ERR_INVALID_ARG, "quadratic_phase_apply: NULL field, empty shape or sign not +-1");
  const long total = (long)batch * ny * nx;
  hipLaunchKernelGGL(k_apply_quadratic, dim3(nblk(total, 256)), dim3(256), 0, (hipStream_t)stream,
                     reinterpret_cast<float2*>(field), ny, nx, sign, total);
  return nn_launch_status();
}

hg_status hg_replay_phase_init(const hg_complex* phasor, const float* target, int batch, int ny, int nx,
                               int slm_levels, int add_quadratic, uint8_t* levels_out, void* ws, size_t ws_bytes,
                               void* stream) {
  clear_error();
  if (!target || !levels_out) return nn_fail(HG_ERR_INVALID_ARG, "replay_phase_init: NULL target or levels_out");
  if (slm_levels < 2 || slm_levels > 256)
    return nn_fail(HG_ERR_INVALID_ARG, "replay_phase_init: slm_levels must be in 2..256");
  const size_t need = hg_replay_phase_init_workspace_size(batch, ny, nx);
  if (!need) return nn_fail(HG_ERR_UNSUPPORTED_SIZE, "replay_phase_init: batch < 1 or unsupported grid");
  hg_status s = check_ws(ws, ws_bytes, need);
  if (s != HG_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const long px = (long)ny * nx, total = px * batch;
  float2* field = reinterpret_cast<float2*>(ws);
  const size_t fbytes = al256((size_t)total * sizeof(float2));
  char* pws = (char*)ws + fbytes;
  hipLaunchKernelGGL(k_replay_start, dim3(nblk(total, 256)), dim3(256), 0, st, target,
                     reinterpret_cast<const float2*>(phasor), field, ny, nx, add_quadratic ? 1 : 0, total);
  s = nn_launch_status();
  if (s != HG_OK) return s;
  for (int b = 0; b < batch; ++b) {
    hg_complex* f = reinterpret_cast<hg_complex*>(field + (size_t)b * px);
    s = hg_fresnel_propagate(f, f, ny, nx, 0.0, 0.0, 0.0, -1, pws, ws_bytes - fbytes, stream);
    if (s != HG_OK) return s;  // hg_last_error already holds the detail
  }
  hipLaunchKernelGGL(k_project_levels, dim3(nblk(total, 256)), dim3(256), 0, st, field, levels_out, slm_levels, total);
  return nn_launch_status();
}

}  // extern "C"
