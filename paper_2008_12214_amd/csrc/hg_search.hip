// Holographic search on the GPU (Holographic Search Algorithms section):
// direct search (greedy single-pixel trials) and simulated annealing (the
// same trials with a temperature-based chance of accepting a worse
// hologram).  One workgroup per hologram keeps the whole replay field in
// registers; a trial changes one SLM pixel, so every replay pixel changes by
// the same complex amount times that pixel's DFT kernel, and the error
// change is one reduction over the plane.  Trials are sequential within a
// hologram; holograms of a batch run in parallel.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include "hologen.h"
#include "hg_kernels.hpp"

namespace hg_internal {
void set_error(const char* msg);
}

namespace hg {
namespace {

constexpr uint32_t kTagSearch = 0x5A;  // Philox tag of the annealing draws

// Threads of a hologram of npx pixels: 16 replay pixels each, 64 to 1024.
constexpr int search_threads(int npx) { return npx / 16 < 64 ? 64 : (npx / 16 > 1024 ? 1024 : npx / 16); }

template <int NY, int NX> struct SearchShape {
  static constexpr int NPX = NY * NX;
  static constexpr int NT = search_threads(NPX);
  static constexpr int P = NPX / NT;  // replay pixels per thread
  static constexpr int NW = NT / 64;
  static_assert(NPX % NT == 0 && P >= 1, "whole pixels per thread");
};

struct SearchArgs {
  const float* target;         // [B][ny][nx] raw amplitude
  const uint8_t* init_levels;  // [B][ny][nx]
  uint8_t* levels_out;         // [B][ny][nx]
  double* err_out;             // [B][max_sweeps + 1]
  int* sweeps_out;             // [B] nullable
  float2* zbuf;                // [B][ny][nx] workspace: the row transform of the start field
  int L, algo, max_sweeps;
  double t0, alpha;
  uint64_t seed;
};

// Sum of one value over the workgroup in a fixed order, the same in every
// thread: FP32 inside each wave, FP64 over the waves.  slots alternates
// between two halves so that consecutive calls need one barrier each.
template <int NW>
__device__ __forceinline__ double group_sum(float v, double (*slots)[kMaxWaves], int& parity) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) slots[parity][threadIdx.x >> 6] = (double)v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += slots[parity][w];
  parity ^= 1;
  return s;
}

template <int NY, int NX>
__global__ __launch_bounds__(search_threads(NY * NX)) void k_search(SearchArgs a) {
  using S = SearchShape<NY, NX>;
  constexpr int NT = S::NT, P = S::P, NPX = S::NPX;
  __shared__ float2 twx[NX], twy[NY], lvl[256];
  __shared__ uint8_t lev[NPX];
  __shared__ double slots[2][kMaxWaves];
  const int b = blockIdx.x, L = a.L;
  const size_t off = (size_t)b * NPX;
  gptr<const float> tg = to_global(a.target + off);

  // tables: the DFT kernel e^{-2 pi i m / n} (FP64-evaluated) and the levels
  for (int m = threadIdx.x; m < NX; m += NT) {
    double s, c;
    sincospi(-2.0 * (double)m / (double)NX, &s, &c);
    twx[m] = make_float2((float)c, (float)s);
  }
  for (int m = threadIdx.x; m < NY; m += NT) {
    double s, c;
    sincospi(-2.0 * (double)m / (double)NY, &s, &c);
    twy[m] = make_float2((float)c, (float)s);
  }
  for (int k = threadIdx.x; k < L; k += NT) lvl[k] = level_phasor(k, L);
  for (int p = threadIdx.x; p < NPX; p += NT) lev[p] = a.init_levels[off + p];
  int parity = 0;

  // prepared target of this thread's replay pixels idx = tid + NT j, centred
  // (v, u): scaled to sum T^2 = NX NY, binary targets symmetrised
  float tv[P];
  int fq[P];  // the pixel's frequency indices: (v - NY/2) mod NY << 16 | (u - NX/2) mod NX
  float e = 0.f;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int idx = threadIdx.x + NT * j, v = idx / NX, u = idx % NX;
    float t = tg[idx];
    if (L == 2) {
      const float tm = tg[((NY - v) & (NY - 1)) * NX + ((NX - u) & (NX - 1))];
      t = sqrtf(0.5f * (t * t + tm * tm));
    }
    tv[j] = t;
    e += t * t;
    fq[j] = (((v - NY / 2) & (NY - 1)) << 16) | ((u - NX / 2) & (NX - 1));
  }
  const double energy = group_sum<S::NW>(e, slots, parity);
  const float tscale = (float)sqrt((double)NPX / energy);
#pragma unroll
  for (int j = 0; j < P; ++j) tv[j] *= tscale;

  // start replay: Z(y, u) = sum_x f(y, x) W_NX^{uc x} into the workspace,
  // then R(v, u) = sum_y Z(y, u) W_NY^{vc y} / sqrt(NX NY)
  gptr<float2> z = to_global(a.zbuf + off);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int idx = threadIdx.x + NT * j, y = idx / NX, u = idx % NX;
    const int ucu = (u - NX / 2) & (NX - 1);
    float2 acc = make_float2(0.f, 0.f);
    for (int x = 0; x < NX; ++x) {
      const float2 t = cmul(lvl[lev[y * NX + x]], twx[(ucu * x) & (NX - 1)]);
      acc = cadd(acc, t);
    }
    z[idx] = acc;
  }
  __threadfence_block();
  __syncthreads();
  const float sc = 1.0f / sqrtf((float)NPX);
  float2 r[P];
  float am[P];
  float e0 = 0.f;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int idx = threadIdx.x + NT * j, u = idx % NX;
    float2 acc = make_float2(0.f, 0.f);
    const int vcj = fq[j] >> 16;
    for (int y = 0; y < NY; ++y) acc = cadd(acc, cmul(z[y * NX + u], twy[(vcj * y) & (NY - 1)]));
    r[j] = cscale(acc, sc);
    am[j] = sqrtf(r[j].x * r[j].x + r[j].y * r[j].y);
    const float d = am[j] - tv[j];
    e0 += d * d;
  }
  double err = group_sum<S::NW>(e0, slots, parity);
  double* eo = a.err_out + (size_t)b * (a.max_sweeps + 1);
  if (threadIdx.x == 0) eo[0] = err;

  // Moving pixel (y, x) from level k to kn changes replay pixel j by
  // dh W(j; y, x) with dh = (phasor kn - phasor k) / sqrt(NX NY) and W the
  // centred DFT kernel; the trial sums the error change, an accepted trial
  // repeats the same arithmetic to update the replay (nothing is held
  // between the two, which keeps registers for the resident replay).
  auto moved = [&](int j, int y, int x, float2 dh) {
    const float2 kern = cmul(twx[((fq[j] & 0xffff) * x) & (NX - 1)], twy[((fq[j] >> 16) * y) & (NY - 1)]);
    return cadd(r[j], cmul(dh, kern));
  };
  auto trial = [&](int y, int x, int k, int kn) -> double {
    const float2 dh = cscale(csub(lvl[kn], lvl[k]), sc);
    float d = 0.f;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const float2 rn = moved(j, y, x, dh);
      const float an = sqrtf(rn.x * rn.x + rn.y * rn.y);
      d += (an - am[j]) * (an + am[j] - 2.f * tv[j]);
    }
    return group_sum<S::NW>(d, slots, parity);
  };
  auto accept = [&](int y, int x, int k, int kn) {
    const float2 dh = cscale(csub(lvl[kn], lvl[k]), sc);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      r[j] = moved(j, y, x, dh);
      am[j] = sqrtf(r[j].x * r[j].x + r[j].y * r[j].y);
    }
  };

  int sweeps = a.max_sweeps;
  for (int s = 1; s <= a.max_sweeps; ++s) {
    const double tau = a.t0 * pow(a.alpha, (double)(s - 1));
    bool changed = false;
    for (int p = 0; p < NPX; ++p) {
      const int y = p / NX, x = p % NX;
      int k = lev[p];  // this sweep has not written pixel p yet: no barrier needed
      if (a.algo == HG_SEARCH_DS) {
        for (int kn = 0; kn < L; ++kn) {
          if (kn == k) continue;
          const double de = trial(y, x, k, kn);
          if (de < -1e-12) {  // strict decrease, as the greedy rule
            accept(y, x, k, kn);
            err += de;
            k = kn;
            changed = true;
          }
        }
      } else {
        const U64x4 o = philox4x64_10(U64x4{(uint64_t)p, (uint64_t)s, 0, 0}, a.seed,
                                      ((uint64_t)b << 32) | kTagSearch);
        const int kn = (int)((k + 1 + (int)(((o.a >> 40) * (uint64_t)(L - 1)) >> 24)) % L);
        const double de = trial(y, x, k, kn);
        const double u = (double)(o.b >> 40) * 0x1p-24;
        if (de < 0.0 || (tau > 0.0 && u < exp(-de / tau))) {
          accept(y, x, k, kn);
          err += de;
          k = kn;
          changed = true;
        }
      }
      if (threadIdx.x == 0) lev[p] = (uint8_t)k;
    }
    // the error of the sweep's result, summed afresh (no drift of the
    // per-trial changes)
    float ee = 0.f;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const float d = am[j] - tv[j];
      ee += d * d;
    }
    err = group_sum<S::NW>(ee, slots, parity);
    if (threadIdx.x == 0) eo[s] = err;
    if (a.algo == HG_SEARCH_DS && !changed) {
      sweeps = s;
      for (int q = s + 1; q <= a.max_sweeps; ++q)
        if (threadIdx.x == 0) eo[q] = err;
      break;
    }
  }
  __syncthreads();  // the last level writes
  for (int p = threadIdx.x; p < NPX; p += NT) a.levels_out[off + p] = lev[p];
  if (a.sweeps_out && threadIdx.x == 0) a.sweeps_out[b] = sweeps;
}

bool search_size_ok(int n) { return n == 8 || n == 16 || n == 32 || n == 64; }

template <int NY>
hipError_t launch_search_x(int nx, int B, const SearchArgs& a, hipStream_t st) {
  switch (nx) {
#define HG_SEARCH_CASE(NXV)                                                                         \
  case NXV:                                                                                         \
    hipLaunchKernelGGL((k_search<NY, NXV>), dim3(B), dim3(SearchShape<NY, NXV>::NT), 0, st, a);     \
    break;
    HG_SEARCH_CASE(8)
    HG_SEARCH_CASE(16)
    HG_SEARCH_CASE(32)
    HG_SEARCH_CASE(64)
#undef HG_SEARCH_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_search(int ny, int nx, int B, const SearchArgs& a, hipStream_t st) {
  switch (ny) {
    case 8: return launch_search_x<8>(nx, B, a, st);
    case 16: return launch_search_x<16>(nx, B, a, st);
    case 32: return launch_search_x<32>(nx, B, a, st);
    case 64: return launch_search_x<64>(nx, B, a, st);
    default: return hipErrorInvalidValue;
  }
}

hg_status search_fail(hg_status st, const char* msg) {
  hg_internal::set_error(msg);
  return st;
}

}  // namespace
}  // namespace hg

extern "C" {

size_t hg_search_workspace_size(int ny, int nx, int batch) {
  if (!hg::search_size_ok(ny) || !hg::search_size_ok(nx) || batch < 1) return 0;
  return (size_t)batch * ny * nx * sizeof(float2);
}

hg_status hg_search(const float* targets, int batch, int ny, int nx, int slm_levels, int algorithm, int max_sweeps,
                    double t0, double alpha, uint64_t seed, const uint8_t* init_levels, uint8_t* levels_out,
                    double* error_out, int* sweeps_out, void* workspace, size_t workspace_bytes, void* stream) {
  using namespace hg;
  hg_internal::set_error("");
  if (!search_size_ok(ny) || !search_size_ok(nx))
    return search_fail(HG_ERR_UNSUPPORTED_SIZE, "holographic search: ny and nx must be 8, 16, 32 or 64");
  if (batch < 1) return search_fail(HG_ERR_INVALID_ARG, "holographic search: batch must be >= 1");
  if (!targets || !init_levels || !levels_out || !error_out)
    return search_fail(HG_ERR_INVALID_ARG, "holographic search: targets, init_levels, levels_out and error_out are required");
  if (slm_levels < 2 || slm_levels > 256)
    return search_fail(HG_ERR_INVALID_ARG, "holographic search: slm_levels must be 2..256 (phase levels)");
  if (algorithm != HG_SEARCH_DS && algorithm != HG_SEARCH_SA)
    return search_fail(HG_ERR_INVALID_ARG, "holographic search: algorithm must be HG_SEARCH_DS or HG_SEARCH_SA");
  if (max_sweeps < 1) return search_fail(HG_ERR_INVALID_ARG, "holographic search: max_sweeps must be >= 1");
  if (algorithm == HG_SEARCH_SA && !(t0 >= 0.0 && std::isfinite(t0) && alpha > 0.0 && std::isfinite(alpha)))
    return search_fail(HG_ERR_INVALID_ARG, "simulated annealing: t0 >= 0 and alpha > 0, both finite");
  const size_t need = hg_search_workspace_size(ny, nx, batch);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) || workspace_bytes < need)
    return search_fail(HG_ERR_WORKSPACE, "holographic search: workspace NULL, misaligned or too small");
  SearchArgs a{};
  a.target = targets;
  a.init_levels = init_levels;
  a.levels_out = levels_out;
  a.err_out = error_out;
  a.sweeps_out = sweeps_out;
  a.zbuf = static_cast<float2*>(workspace);
  a.L = slm_levels;
  a.algo = algorithm;
  a.max_sweeps = max_sweeps;
  a.t0 = t0;
  a.alpha = alpha;
  a.seed = seed;
  const hipError_t e = launch_search(ny, nx, batch, a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    char msg[256];
    snprintf(msg, sizeof(msg), "holographic search launch failed: %s", hipGetErrorString(e));
    return search_fail(HG_ERR_HIP, msg);
  }
  return HG_OK;
}

}  // extern "C"
