// Gerchberg-Saxton / weighted GS for small holograms (ny, nx <= 128) in one
// launch: one workgroup per problem keeps the whole complex field resident
// in LDS and runs set-up, every iteration and the final measurement itself.
// A problem this small moves only a few hundred kilobytes per iteration, so
// the multi-launch pipeline (two passes per iteration) is bound by launch
// latency; here an iteration costs a handful of workgroup barriers instead.
//
// The arithmetic is that of the multi-launch pipeline, step by step:
// target preparation (energy scaling, binary symmetrisation), the initial
// field (Philox phase, levels or field), the centring / Fresnel modulation,
// the row and column transforms with the same plans and twiddles, the
// replay constraint (and weight update), the projection onto the SLM
// levels, and the NMSE sums in FP64.  The transforms of the smaller sizes
// use 8 elements per thread (other radix plans than the pipeline's 16), and
// the NMSE partial sums are added in another order, so results agree with
// the pipeline's to rounding.
//
// Field layout in LDS: row y at padded row lds_pad(y), element x of a row at
// lds_pad(x), row pitch RP.  Every row and every column is then a transform
// line whose padded element e sits at a fixed stride (1 or RP), so both
// passes exchange in place in the one field array.
#include <hip/hip_runtime.h>

#include "hg_launch.hpp"

namespace hg {
namespace {

// One line of the LDS-resident field as the exchange buffer of its own
// transform: padded element e at base[e * STRIDE].  The line is overwritten
// in place, so each exchange has a barrier before the writes and before the
// reads (rows and columns span several waves of the workgroup).
template <int STRIDE> struct LineEx {
  lptr<float2> base;
  __device__ void before_read() { __syncthreads(); }
  __device__ void before_write() { __syncthreads(); }
  __device__ float2 ld(int e) const { return base[e * STRIDE]; }
  __device__ void st(int e, float2 v) { base[e * STRIDE] = v; }
};

// Elements per thread: 8 where the workgroup then has at most 512 threads
// (two waves per SIMD hide LDS and barrier latency on the one CU a problem
// runs on, with registers to spare), else 16.
template <int NY, int NX> constexpr int small_elements() { return NY * NX / 8 <= 512 ? 8 : 16; }

template <int NY, int NX> struct SmallShape {
  static constexpr int E = small_elements<NY, NX>();
  static constexpr int NT = NY * NX / E;           // threads: one per E elements
  static constexpr int TR = NX / E, TC = NY / E;   // threads per row / per column
  static constexpr int RP = NX + NX / 16 + 2;      // LDS pitch of a padded row
  static constexpr int VR = NY + NY / 16;          // padded rows
  static constexpr int TWX = TwLayout<NX, E>::total(), TWY = TwLayout<NY, E>::total();
  static constexpr size_t lds_bytes() {
    return (size_t)VR * RP * 8 + (size_t)(TWX + (NY == NX ? 0 : TWY)) * 8 + 256 * 8 + (kMaxWaves * 4 + 4) * 8;
  }
};

template <int NY, int NX, bool FRESNEL, bool WEIGHTED>
__global__ __launch_bounds__((NY * NX / small_elements<NY, NX>())) void k_small(Batch bt) {
  using S = SmallShape<NY, NX>;
  constexpr int E = S::E, NT = S::NT, TR = S::TR, TC = S::TC, RP = S::RP;
  static_assert(NT % 64 == 0 && NT <= 1024, "whole waves, one workgroup per problem");
  static_assert(S::lds_bytes() <= 160 * 1024, "field and tables fit in LDS");
  __shared__ float2 fld_s[S::VR * RP];
  __shared__ float2 twx_s[S::TWX];
  __shared__ float2 twy_s[NY == NX ? 1 : S::TWY];
  __shared__ float2 lvl_s[256];
  __shared__ double red[kMaxWaves][4];
  __shared__ double tot[4];
  const lptr<float2> fld = (lptr<float2>)fld_s;

  const int b = blockIdx.x;
  const Desc& d = bt.desc[b];
  const int L = uni(d.L), iters = uni(d.iters);
  const int amp = uni(d.mod);  // amplitude SLM
  const int user_w = uni(d.user_weights);
  gptr<const float> tg = to_global(uni_ptr(d.target));
  gptr<uint8_t> lev = to_global(uni_ptr(d.levels_out));
  double* nmse = uni_ptr(d.nmse_out);
  gptr<float2> fout = to_global(uni_ptr(d.field_out));
  gptr<float2> rout = to_global(uni_ptr(d.replay_out));
  gptr<float2> rdump = to_global(uni_ptr(d.r_out));  // one-iteration calls: replay before the constraint
  gptr<float2> gdump = to_global(uni_ptr(d.g_out));  // and the field before the projection
  const uint8_t* init_l = uni_ptr(d.init_levels);
  const float2* init_f = uni_ptr(d.init_field);
  const size_t off = (size_t)b * NY * NX;
  gptr<float> tp = to_global(bt.tprep + off);  // prepared target, [y][x]
  gptr<float> w = nullptr;                     // weights, [y][x]
  if constexpr (WEIGHTED) w = to_global(user_w ? uni_ptr(d.weights) : bt.wbuf + off);
  gptr<const float2> cx = to_global(static_cast<const float2*>(bt.chirp)) + (size_t)b * (NX + NY);

  // tables: staged twiddles (FP64-evaluated) and the level phasors
  for (int i = threadIdx.x; i < S::TWX; i += NT) twiddle_entry<NX, 1, E>(twx_s, i);
  if constexpr (NY != NX) {
    for (int i = threadIdx.x; i < S::TWY; i += NT) twiddle_entry<NY, 1, E>(twy_s, i);
  }
  if (L > 2 && !amp) {
    for (int i = threadIdx.x; i < L; i += NT) lvl_s[i] = level_phasor(i, L);
  }
  const lptr<const float2> twx = (lptr<const float2>)twx_s;
  const lptr<const float2> twy = NY == NX ? twx : (lptr<const float2>)twy_s;

  // column view: column cu, thread ct of its TC (lanes run along x);
  // row view: row ry, thread rt of its TR
  const int cu = threadIdx.x % NX, ct = threadIdx.x / NX;
  const int ry = threadIdx.x / TR, rt = threadIdx.x % TR;

  // ---- set-up: energy scaling, binary symmetrisation, weights -----------
  // (each thread prepares exactly the column elements it later constrains)
  float e = 0.0f;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const float tv = tg[(size_t)(ct + TC * j) * NX + cu];
    e += tv * tv;
  }
  block_sum4<NT>(e, 0.f, 0.f, 0.f, red, tot);
  const float scale = (float)sqrt((double)NX * (double)NY / tot[0]);
  float om = 0.f, ws0 = 0.f;
  const int um = (NX - cu) & (NX - 1);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int y = ct + TC * j;
    const int idx = y * NX + cu;
    float tv = tg[idx];
    if (L == 2 || amp) {  // binary phase or amplitude SLM: centro-symmetric replay
      const int ym = (NY - y) & (NY - 1);
      const float tm = tg[ym * NX + um];
      tv = sqrtf(0.5f * (tv * tv + tm * tm));
    }
    tv *= scale;
    if constexpr (WEIGHTED) {
      // a non-finite caller weight poisons its pixel's target, so the NMSE
      // turns NaN as for a non-finite target
      if (user_w && !__builtin_isfinite(w[idx])) tv = __builtin_nanf("");
    }
    tp[idx] = tv;
    if constexpr (WEIGHTED) {
      float wv = 1.0f;
      if (user_w) wv = w[idx];
      else w[idx] = 1.0f;
      if (tv > 0.f) { om += 1.f; ws0 += wv; }
    }
  }
  double omega = 1.0, wsum = 1.0;  // |Omega| and the weight sum of the previous iteration
  if constexpr (WEIGHTED) {
    block_sum4<NT>(om, ws0, 0.f, 0.f, red, tot);
    omega = tot[0];
    wsum = tot[1];
  }

  // ---- initial field and its forward row transform ----------------------
  float2 v[E];
  {
    const float2 cyv = FRESNEL ? static_cast<float2>(cx[NX + ry]) : make_float2(1.f, 0.f);
    if (init_f || init_l) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int idx = ry * NX + rt + TR * j;
        v[j] = init_f ? init_f[idx] : amp ? make_float2(amp_value(init_l[idx], L), 0.f) : level_phasor(init_l[idx], L);
      }
    } else {
      // Philox words over row lines; element j = g + (E/4) w
#pragma unroll
      for (int g = 0; g < E / 4; ++g) {
        const U64x4 o = philox_line_block(d.seed, d.item, 1u, (uint32_t)(rt + TR * g), (uint32_t)ry);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[g + (E / 4) * q] = philox_phasor(u64x4_word(o, q));
      }
    }
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = Mod<FRESNEL>(rt + TR * j, ry, cx, cyv).fwd(v[j]);
    LineEx<1> rex{fld + lds_pad(ry) * RP};
    fft_lds<NX, E, -1>(v, rt, twx, rex);
    __syncthreads();  // the transform's last reads of the row are done
#pragma unroll
    for (int j = 0; j < E; ++j) rex.base[lds_pad(rt + TR * j)] = v[j];
  }

  // ---- iterations k = 1..K, then k = K + 1 measures the final field ------
  const float2 cyv = FRESNEL ? static_cast<float2>(cx[NX + ry]) : make_float2(1.f, 0.f);
  LineEx<RP> cex{fld + lds_pad(cu)};
  LineEx<1> rex{fld + lds_pad(ry) * RP};
  for (int k = 1; k <= iters + 1; ++k) {
    const bool fin = (k == iters + 1);
    // column pass: forward transform, NMSE sums, constraint, inverse
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = cex.base[lds_pad(ct + TC * j) * RP];
    fft_lds<NY, E, -1>(v, ct, twy, cex);
    const float inv_m = WEIGHTED ? (float)((omega > 0.0 ? omega : 1.0) / wsum) : 1.0f;
    float s_ta = 0.f, s_aa = 0.f, s_tt = 0.f, s_w = 0.f;
    // amplitude SLM: the zero order (row NY/2 = element E/2 of ct = 0, column
    // NX/2) keeps R and stays out of the NMSE sums
    static_assert(TC * (E / 2) == NY / 2, "the zero order is element E/2 of column thread 0");
    const bool zo = amp && ct == 0 && cu == (NX >> 1);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int idx = (ct + TC * j) * NX + cu;
      const float2 Rr = v[j];  // unscaled replay, centred index (ct + TC j, cu)
      const float a2 = Rr.x * Rr.x + Rr.y * Rr.y;
      const float inv = a2 > 0.f ? __builtin_amdgcn_rsqf(a2) : 0.f;
      const float A = a2 * inv * bt.fwd_scale;  // |R| of the unitary transform
      const float Tv = tp[idx];
      const bool zj = j == E / 2 && zo;
      if (!zj) {
        s_ta += Tv * A;
        s_aa += A * A;
        s_tt += Tv * Tv;
      }
      if (fin) {
        if (rout) rout[idx] = cscale(Rr, bt.fwd_scale);
      } else {
        if (rdump) rdump[idx] = cscale(Rr, bt.fwd_scale);
        float tamp = Tv;
        if constexpr (WEIGHTED) {
          if (Tv > 0.f) {
            const float ratio = fmaxf(Tv, kWgsEps) * __builtin_amdgcn_rcpf(fmaxf(A, kWgsEps));
            const float wc = clamp_w(w[idx] * ratio * inv_m);
            const float wn = __builtin_amdgcn_exp2f(kWgsGamma * __builtin_amdgcn_logf(wc));
            w[idx] = wn;
            s_w += wn;
            tamp = wn * Tv;
          }
        }
        v[j] = a2 > 0.f ? cscale(Rr, tamp * inv) : make_float2(tamp, 0.f);
        if (zj) v[j] = cscale(Rr, bt.fwd_scale);
      }
    }
    block_sum4<NT>(s_ta, s_aa, s_tt, s_w, red, tot);
    if (threadIdx.x == 0) {
      const double e = nmse_from_sums(tot[0], tot[1], tot[2], bt.status);
      if (nmse) nmse[k - 1] = e;
    }
    if constexpr (WEIGHTED) wsum = tot[3];
    if (fin) break;
    fft_lds<NY, E, +1>(v, ct, twy, cex);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) cex.base[lds_pad(ct + TC * j) * RP] = v[j];
    __syncthreads();

    // row pass: inverse transform, projection, forward transform
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = rex.base[lds_pad(rt + TR * j)];
    fft_lds<NX, E, +1>(v, rt, twx, rex);
    const bool last = (k == iters);
    const float amp_s = bt.fwd_scale * (float)(L - 1);  // unitary scale times L - 1
    auto project = [&](auto kind, auto wr) {
      constexpr int KIND = decltype(kind)::value;  // 0 continuous, 2 binary, 3 other L
      constexpr bool WR = decltype(wr)::value;     // last iteration: write levels and field
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int x = rt + TR * j;
        const Mod<FRESNEL> md(x, ry, cx, cyv);
        const float2 g = md.inv(v[j]);
        float2 f;
        if constexpr (KIND == 0) {
          f = unit_phase(g);
        } else if constexpr (KIND == 5) {  // amplitude SLM: nearest transmission to Re g
          const int kl = amp_level(g.x, amp_s, L);
          f = make_float2(amp_value(kl, L), 0.f);
          if constexpr (WR) {
            if (lev) lev[ry * NX + x] = (uint8_t)kl;
          }
        } else {
          const int kl = level_index(g, KIND == 2 ? 2 : L);
          if constexpr (KIND == 2) f = level_phasor(kl, 2);
          else f = lvl_s[kl];
          if constexpr (WR) {
            if (lev) lev[ry * NX + x] = (uint8_t)kl;
          }
        }
        if constexpr (WR) {
          if (fout) fout[ry * NX + x] = f;
          if (gdump) gdump[ry * NX + x] = cscale(g, bt.fwd_scale);  // unitary backward
        }
        v[j] = md.fwd(f);
      }
    };
    auto by_kind = [&](auto wr) {
      if (amp) project(std::integral_constant<int, 5>{}, wr);
      else if (L == 2) project(std::integral_constant<int, 2>{}, wr);
      else if (L == 0) project(std::integral_constant<int, 0>{}, wr);
      else project(std::integral_constant<int, 3>{}, wr);
    };
    if (last) by_kind(std::true_type{});
    else by_kind(std::false_type{});
    fft_lds<NX, E, -1>(v, rt, twx, rex);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) rex.base[lds_pad(rt + TR * j)] = v[j];
  }
}

template <int NY, int NX>
void launch_small_t(const Batch& bt, int B, bool fresnel, bool weighted, hipStream_t st) {
  const dim3 grid(B), block(SmallShape<NY, NX>::NT);
  if (fresnel) {
    if (weighted) hipLaunchKernelGGL((k_small<NY, NX, true, true>), grid, block, 0, st, bt);
    else hipLaunchKernelGGL((k_small<NY, NX, true, false>), grid, block, 0, st, bt);
  } else {
    if (weighted) hipLaunchKernelGGL((k_small<NY, NX, false, true>), grid, block, 0, st, bt);
    else hipLaunchKernelGGL((k_small<NY, NX, false, false>), grid, block, 0, st, bt);
  }
}

}  // namespace

void launch_small(const Batch& bt, int B, bool fresnel, bool weighted, hipStream_t st) {
  if (bt.ny == 64 && bt.nx == 64) launch_small_t<64, 64>(bt, B, fresnel, weighted, st);
  else if (bt.ny == 64 && bt.nx == 128) launch_small_t<64, 128>(bt, B, fresnel, weighted, st);
  else if (bt.ny == 128 && bt.nx == 64) launch_small_t<128, 64>(bt, B, fresnel, weighted, st);
  else if (bt.ny == 128 && bt.nx == 128) launch_small_t<128, 128>(bt, B, fresnel, weighted, st);
}

}  // namespace hg
