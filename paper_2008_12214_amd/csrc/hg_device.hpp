// Device building blocks for the gfx950 hologram hot path: complex helpers,
// register-resident DFT butterflies, the LDS-staged Stockham FFT used by the
// row and column passes, Philox4x64-10 and the SLM phase projection.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {

// Global-memory pointer.  Pointers that reach a kernel inside a struct are
// generic; marking them global lets the compiler emit global_load/store
// instead of flat instructions, whose completion is tracked together with
// LDS traffic.
// (The host pass of HIP compilation only builds kernel stubs and sees plain
// pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T> using gptr = __attribute__((address_space(1))) T*;
#else
template <class T> using gptr = T*;
#endif
template <class T> __device__ __forceinline__ gptr<T> to_global(T* p) { return (gptr<T>)p; }
template <class T> __device__ __forceinline__ gptr<const T> to_global(const T* p) { return (gptr<const T>)p; }

// ---------------------------------------------------------------------------
// complex float helpers (interleaved float2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// a * (DIR * i): DIR = -1 is the forward transform kernel's -i.
template <int DIR> __device__ __forceinline__ float2 mul_i(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// ---------------------------------------------------------------------------
// DFT of length R on registers, natural order in and out.
// DIR = -1: exp(-2 pi i r q / R) (forward), DIR = +1: inverse (unscaled).
// Built by decimation in time: DFT_2R from two DFT_R and the factors W_2R^q.
// ---------------------------------------------------------------------------
template <int DIR> __device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_i<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

constexpr float kC8 = 0.70710678118654752440f;   // cos(pi/4)
constexpr float kC16 = 0.92387953251128675613f;  // cos(pi/8)
constexpr float kS16 = 0.38268343236508977173f;  // sin(pi/8)

// multiply by W_16^q = exp(DIR 2 pi i q / 16), q in [0, 8)
template <int DIR, int Q> __device__ __forceinline__ float2 w16(float2 a) {
  constexpr float s = (float)DIR;
  if constexpr (Q == 0) return a;
  else if constexpr (Q == 4) return mul_i<DIR>(a);
  else if constexpr (Q == 2) {  // (c8, s c8)
    return make_float2(kC8 * (a.x - s * a.y), kC8 * (a.y + s * a.x));
  } else if constexpr (Q == 6) {  // (-c8, s c8)
    return make_float2(-kC8 * (a.x + s * a.y), kC8 * (s * a.x - a.y));
  } else {
    constexpr float c = (Q == 1) ? kC16 : (Q == 3) ? kS16 : (Q == 5) ? -kS16 : -kC16;
    constexpr float sn = (Q == 1) ? kS16 : (Q == 3) ? kC16 : (Q == 5) ? kC16 : kS16;
    return cmul(a, make_float2(c, s * sn));
  }
}

template <int R, int DIR> struct Dft;

template <int DIR> struct Dft<1, DIR> {
  __device__ __forceinline__ static void run(float2 (&a)[1]) {}
};
template <int DIR> struct Dft<2, DIR> {
  __device__ __forceinline__ static void run(float2 (&a)[2]) {
    const float2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};
template <int DIR> struct Dft<4, DIR> {
  __device__ __forceinline__ static void run(float2 (&a)[4]) { dft4<DIR>(a[0], a[1], a[2], a[3]); }
};
template <int DIR> struct Dft<8, DIR> {
  __device__ __forceinline__ static void run(float2 (&a)[8]) {
    float2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    float2 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
    dft4<DIR>(e0, e1, e2, e3);
    dft4<DIR>(o0, o1, o2, o3);
    o1 = w16<DIR, 2>(o1);
    o2 = w16<DIR, 4>(o2);
    o3 = w16<DIR, 6>(o3);
    a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
    a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
    a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
    a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
  }
};
template <int DIR> struct Dft<16, DIR> {
  __device__ __forceinline__ static void run(float2 (&a)[16]) {
    float2 e[8], o[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) { e[q] = a[2 * q]; o[q] = a[2 * q + 1]; }
    Dft<8, DIR>::run(e);
    Dft<8, DIR>::run(o);
    o[1] = w16<DIR, 1>(o[1]); o[2] = w16<DIR, 2>(o[2]); o[3] = w16<DIR, 3>(o[3]);
    o[4] = w16<DIR, 4>(o[4]); o[5] = w16<DIR, 5>(o[5]); o[6] = w16<DIR, 6>(o[6]);
    o[7] = w16<DIR, 7>(o[7]);
#pragma unroll
    for (int q = 0; q < 8; ++q) { a[q] = cadd(e[q], o[q]); a[q + 8] = csub(e[q], o[q]); }
  }
};

// ---------------------------------------------------------------------------
// Stockham radix plan for a length-N transform held by T = N / E threads,
// E elements per thread.  Thread t holds x[t + T j], j < E, before and after.
// Radices are E (as often as it divides), then the remainder; a remainder of
// 2 is folded into the last E stage (E/2 * 4) to avoid a radix-2 pass.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }

template <int N, int E> struct Plan {
  static_assert((N & (N - 1)) == 0 && (E & (E - 1)) == 0 && N >= E && E >= 2, "powers of two");
  static constexpr int T = N / E;
  static constexpr int lgN = ilog2(N), lgE = ilog2(E);
  static constexpr int full = lgN / lgE, rem = lgN % lgE;
  static constexpr bool fold = (rem == 1 && full >= 1 && lgE >= 3);
  static constexpr int ns = full + (rem ? 1 : 0);
  __host__ __device__ static constexpr int lgradix(int s) {
    return fold ? (s < full - 1 ? lgE : (s == full - 1 ? lgE - 1 : 2))
                : (s < full ? lgE : rem);
  }
  __host__ __device__ static constexpr int radix(int s) { return 1 << lgradix(s); }
  __host__ __device__ static constexpr int stride(int s) { return s == 0 ? 1 : stride(s - 1) * radix(s - 1); }
};

// Per-stage twiddle table layout.  Stage s >= 1 (stride p, radix R) stores
// W_{pR}^{r k} for k < p, r = 1..R-1 at offset twoff(s) + k (R - 1) + r - 1,
// so one butterfly reads R - 1 consecutive entries.
template <int N, int E> struct TwLayout {
  using P = Plan<N, E>;
  __host__ __device__ static constexpr int size_of(int s) { return s == 0 ? 0 : P::stride(s) * (P::radix(s) - 1); }
  __host__ __device__ static constexpr int twoff(int s) { return s <= 1 ? 0 : twoff(s - 1) + size_of(s - 1); }
  __host__ __device__ static constexpr int total() { return twoff(P::ns - 1) + size_of(P::ns - 1); }
};

// Twiddle multiply: forward uses w, inverse conj(w); tables hold exp(-2 pi i m / n).
template <int DIR> __device__ __forceinline__ float2 twmul(float2 a, float2 w) {
  return DIR < 0 ? cmul(a, w) : cmulc(a, w);
}

// LDS element padding: one float2 of padding per 16 elements.  Stage
// strides in the plans used here are 1 (first radix-16 stage) or multiples
// of 16, so padded addresses stay affine in the butterfly index r and the
// compiler can use immediate offsets.
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 4); }

// One Stockham stage S and, recursively, the following ones.
//   Ex: LDS exchange policy with before_read(), before_write(), and
//       ld(e) / st(e, v) on padded element index e.
template <int N, int E, int DIR, int S, class Ex, class TWP>
__device__ __forceinline__ void fft_stage(float2 (&v)[E], int t, TWP tw, Ex& ex) {
  using P = Plan<N, E>;
  constexpr int R = P::radix(S), p = P::stride(S), T = P::T, M = E / R;
  constexpr bool last = (S == P::ns - 1);
  if constexpr (S > 0) {
    ex.before_read();
    if constexpr (T % 16 == 0) {
      const int rb = lds_pad(t);
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = ex.ld(rb + j * (T + T / 16));
    } else {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = ex.ld(lds_pad(t + T * j));
    }
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int i = t + T * m;
    const int k = i & (p - 1);
    float2 a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = v[m + r * M];
    if constexpr (p > 1) {
      constexpr int kTwOff = TwLayout<N, E>::twoff(S);
      const auto w = tw + kTwOff + k * (R - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) a[r] = twmul<DIR>(a[r], w[r - 1]);
    }
    Dft<R, DIR>::run(a);
#pragma unroll
    for (int r = 0; r < R; ++r) v[m + r * M] = a[r];
  }
  if constexpr (!last) {
    ex.before_write();
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int i = t + T * m;
      const int k = i & (p - 1);
      const int o = (i - k) * R + k;  // output index of r = 0
      if constexpr (p % 16 == 0) {
        const int wb = lds_pad(o);
#pragma unroll
        for (int r = 0; r < R; ++r) ex.st(wb + r * (p + p / 16), v[m + r * M]);
      } else if constexpr (p == 1 && R == 16) {
        const int wb = lds_pad(o);
#pragma unroll
        for (int r = 0; r < R; ++r) ex.st(wb + r, v[m + r * M]);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) ex.st(lds_pad(o + r * p), v[m + r * M]);
      }
    }
    fft_stage<N, E, DIR, S + 1>(v, t, tw, ex);
  }
}

// Hide a pointer's value from the optimiser.  Used so that table loads are
// issued where they are consumed instead of being hoisted (and kept live in
// registers) across whole transforms, which would cap occupancy.
template <class T> __device__ __forceinline__ T* launder(T* p) {
  asm volatile("" : "+v"(p));
  return p;
}
#if defined(__HIP_DEVICE_COMPILE__)
template <class T> __device__ __forceinline__ gptr<T> launder(gptr<T> p) {
  asm volatile("" : "+v"(p));
  return p;
}
#endif

// Unscaled length-N transform of the data held by this thread group, with
// twiddles from a table in global memory (read as global, not flat, loads:
// flat loads would also count against LDS completion waits).
template <int N, int E, int DIR, class Ex>
__device__ __forceinline__ void fft(float2 (&v)[E], int t, const float2* __restrict__ tw, Ex& ex) {
  fft_stage<N, E, DIR, 0>(v, t, launder(to_global(tw)), ex);
}

// LDS-resident twiddles (kept in the LDS address space so no table read
// becomes a flat or global access).
#if defined(__HIP_DEVICE_COMPILE__)
template <class T> using lptr = __attribute__((address_space(3))) T*;
#else
template <class T> using lptr = T*;
#endif
template <int N, int E, int DIR, class Ex>
__device__ __forceinline__ void fft_lds(float2 (&v)[E], int t, lptr<const float2> tw, Ex& ex) {
  fft_stage<N, E, DIR, 0>(v, t, tw, ex);
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 64x64->128 multiplies with the published multipliers and Weyl key bumps.
// ---------------------------------------------------------------------------
struct U64x4 { uint64_t a, b, c, d; };

__device__ __forceinline__ U64x4 philox4x64_10(U64x4 x, uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint64_t hi0 = __umul64hi(M0, x.a), lo0 = M0 * x.a;
    const uint64_t hi1 = __umul64hi(M1, x.c), lo1 = M1 * x.c;
    x = U64x4{hi1 ^ x.b ^ k0, lo1, hi0 ^ x.d ^ k1, lo0};
  }
  return x;
}

// Random words of a plane split into lines of length n: element i of line l
// takes word (i div n/4) of the block at counter (i mod n/4, l, 0, 0) under
// key (seed, (item << 32) | tag).  One block serves the four quarter-line
// elements i, i + n/4, i + n/2, i + 3n/4, which a thread of a length-n
// transform holding elements t + T j (E divisible by 4) owns together.
__device__ __forceinline__ U64x4 philox_line_block(uint64_t seed, uint32_t item, uint32_t tag, uint32_t i,
                                                   uint32_t line) {
  return philox4x64_10(U64x4{i, line, 0, 0}, seed, ((uint64_t)item << 32) | tag);
}
__device__ __forceinline__ uint64_t u64x4_word(const U64x4& o, int w) {
  return w == 0 ? o.a : w == 1 ? o.b : w == 2 ? o.c : o.d;
}

// exp(2 pi i u24 2^-24) for the top 24 bits of word.
__device__ __forceinline__ float2 philox_phasor(uint64_t word) {
  const float half_turns = (float)(uint32_t)(word >> 40) * 0x1p-23f;  // = 2 u24, exact
  float s, c;
  sincospif(half_turns, &s, &c);
  return make_float2(c, s);
}

// ---------------------------------------------------------------------------
// SLM projection.  L = 0: g/|g| (g = 0 -> 1).  L >= 2: nearest of the uniform
// levels 2 pi k / L, k = floor(arg(g) L / (2 pi) + 1/2) mod L.
// ---------------------------------------------------------------------------
// arg(g) in [-pi, pi] without a library call: octant reduction to
// z = min(|x|, |y|) / max(|x|, |y|) in [0, 1] and atan(z) = z P(z^2), P of
// degree 7 in z^2 fitted to atan on [0, 1] by iteratively reweighted least
// squares on Chebyshev nodes.  Maximum error 1e-7 rad in FP32 (about the
// resolution of FP32 near pi), so a level decision differs from the exact
// angle's only within 1e-7 rad of a boundary.  g = 0 gives 0.
__device__ __forceinline__ float fast_arg(float2 g) {
  const float ax = fabsf(g.x), ay = fabsf(g.y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float z = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
  const float z2 = z * z;
  float p = -4.054553044e-03f;
  p = fmaf(p, z2, 2.186295803e-02f);
  p = fmaf(p, z2, -5.591242735e-02f);
  p = fmaf(p, z2, 9.642214963e-02f);
  p = fmaf(p, z2, -1.390864230e-01f);
  p = fmaf(p, z2, 1.994657002e-01f);
  p = fmaf(p, z2, -3.332986144e-01f);
  p = fmaf(p, z2, 9.999993359e-01f);
  float a = p * z;
  if (ay > ax) a = 1.57079632679489662f - a;
  if (g.x < 0.0f) a = 3.14159265358979324f - a;
  return g.y < 0.0f ? -a : a;
}

__device__ __forceinline__ int level_index(float2 g, int L) {
  if (L == 2) return g.x < 0.0f ? 1 : 0;
  const float th = fast_arg(g);  // [-pi, pi]
  int k = (int)floorf(th * ((float)L * 0.15915494309189533577f) + 0.5f);
  k = k < 0 ? k + L : k;
  return k >= L ? k - L : k;
}

// The same decision for L = 4 or 8 without the arctangent: the nearest of
// the levels k 2 pi / L follows from the signs of g and, inside a quadrant,
// from comparing |y| with |x| (L = 4: boundary at pi/4) or with tan(pi/8) |x|
// and |x| with tan(pi/8) |y| (L = 8: boundaries at pi/8 and 3 pi/8).  The
// product's FP32 rounding moves a boundary by about 1e-7 rad.  g = 0 gives 0.
// Selects only (no branch on L): a projection loop over a thread's elements
// stays one basic block, so the compiler can overlap the elements' loads.
__device__ __forceinline__ int level_index_quad(float2 g, int L) {
  const float ax = fabsf(g.x), ay = fabsf(g.y);
  constexpr float kTan8 = 0.414213562373095049f;  // tan(pi/8)
  const bool l8 = L == 8;
  const float tq = l8 ? kTan8 : 1.0f;  // the first boundary: pi/8 or pi/4
  // level within the quadrant, 0 nearest the x axis: past the first
  // boundary, and (L = 8) past the second at 3 pi/8
  const bool a = ay > tq * ax, b = l8 && ax <= kTan8 * ay;
  const int q = a ? (b ? 2 : 1) : 0;
  const int up = g.x < 0.0f ? (L >> 1) - q : q;  // as if y >= 0
  return g.y < 0.0f ? (L - up) & (L - 1) : up;
}

__device__ __forceinline__ float2 level_phasor(int k, int L) {
  if (L == 2) return make_float2(k ? -1.0f : 1.0f, 0.0f);
  float s, c;
  sincospif((float)(2 * k) / (float)L, &s, &c);
  return make_float2(c, s);
}

// Amplitude SLM with L uniform transmissions k / (L - 1): the nearest to
// Re g is k = clamp(floor(Re g (L - 1) + 1/2), 0, L - 1).  s_lm1 carries the
// scale of g (1/sqrt(nx ny) for an unscaled transform) times L - 1.
__device__ __forceinline__ int amp_level(float gx, float s_lm1, int L) {
  const int k = (int)floorf(gx * s_lm1 + 0.5f);
  return min(max(k, 0), L - 1);
}
__device__ __forceinline__ float amp_value(int k, int L) { return (float)k / (float)(L - 1); }

__device__ __forceinline__ float2 unit_phase(float2 g) {
  const float m2 = g.x * g.x + g.y * g.y;
  if (!(m2 > 0.0f) || !(m2 < 3.0e38f)) return make_float2(1.0f, 0.0f);
  const float inv = rsqrtf(m2);
  return make_float2(g.x * inv, g.y * inv);
}

}  // namespace hg
