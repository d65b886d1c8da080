// C ABI of the hologram hot path (declared in include/hologen.h): argument
// validation on the host, workspace carving, launch configuration (default
// table or autotuned), and the launch sequences of the GS / weighted GS /
// OSPR / propagation pipelines on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "hologen.h"
#include "hg_launch.hpp"

// Scratch of hg_wgs_static: one copy of this array per GPU.  Host code uses
// it only through the per-device address that hipGetSymbolAddress returns
// (static_scratch below), never by its name.
static __device__ __align__(256) unsigned char scratch[HG_STATIC_SCRATCH_BYTES];

namespace {

using namespace hg;

thread_local char g_err[512] = "";

hg_status fail(hg_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

// ---------------------------------------------------------------------------
// optional per-launch timing with hipEvents
// ---------------------------------------------------------------------------
enum TimeCat { TC_COL = 0, TC_ROW = 1, TC_SETUP = 2 };
struct Timing {
  bool on = false;
  std::vector<hipEvent_t> pool;  // reusable events
  size_t used = 0;
  std::vector<std::pair<int, size_t>> marks;  // (category, index of the start event)
} g_timing;

hipEvent_t timing_event() {
  if (g_timing.used == g_timing.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_timing.pool.push_back(e);
  }
  return g_timing.pool[g_timing.used++];
}

// RAII bracket around one launch
struct TimeScope {
  int cat;
  hipStream_t st;
  size_t start = (size_t)-1;
  TimeScope(int c, hipStream_t s) : cat(c), st(s) {
    if (!g_timing.on) return;
    hipEvent_t e = timing_event();
    if (!e) return;
    start = g_timing.used - 1;
    (void)hipEventRecord(e, st);
  }
  ~TimeScope() {
    if (start == (size_t)-1) return;
    hipEvent_t e = timing_event();
    if (!e) return;
    (void)hipEventRecord(e, st);
    g_timing.marks.push_back({cat, start});
  }
};

bool pow2_in_range(int n) { return n >= 64 && n <= 4096 && (n & (n - 1)) == 0; }

template <class F> bool with_size(int n, F&& f) {
  switch (n) {
    case 64: f(std::integral_constant<int, 64>{}); return true;
    case 128: f(std::integral_constant<int, 128>{}); return true;
    case 256: f(std::integral_constant<int, 256>{}); return true;
    case 512: f(std::integral_constant<int, 512>{}); return true;
    case 1024: f(std::integral_constant<int, 1024>{}); return true;
    case 2048: f(std::integral_constant<int, 2048>{}); return true;
    case 4096: f(std::integral_constant<int, 4096>{}); return true;
    default: return false;
  }
}

// ---------------------------------------------------------------------------
// launch configuration: column-tile width C (by column length ny) and rows
// per row-pass workgroup RPB (by row length nx); defaults, overridden by
// hg_autotune / hg_set_launch_config for the same (ny, nx, batch class)
// ---------------------------------------------------------------------------
struct Cfg { int C, RPB; };

int min_col_tile(int ny) {
  for (int c : {1, 2, 4, 8, 16})
    if (col_ok(ny, c)) return c;
  return 16;
}

Cfg default_cfg(int ny, int nx, int B) {
  Cfg c{};
  switch (ny) {
    case 64: c.C = 16; break;
    case 128: c.C = 16; break;
    case 256: c.C = 8; break;
    case 512: c.C = 8; break;
    case 1024: c.C = 4; break;
    case 2048: c.C = 4; break;
    default: c.C = 2; break;
  }
  const int T = nx / kE;
  c.RPB = default_rpb(nx);  // 2048-wide rows: staged 4-row groups
  (void)B;
  return c;
}

int batch_class(int B) { return B >= 8 ? 1 : 0; }

std::mutex g_cfg_mu;
std::map<std::tuple<int, int, int>, Cfg> g_tuned;

Cfg get_cfg(int ny, int nx, int B) {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  auto it = g_tuned.find(std::make_tuple(ny, nx, batch_class(B)));
  return it != g_tuned.end() ? it->second : default_cfg(ny, nx, B);
}
bool has_tuned_cfg(int ny, int nx, int B) {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  return g_tuned.count(std::make_tuple(ny, nx, batch_class(B))) != 0;
}

// ---------------------------------------------------------------------------
// workspace layout of one size class (B problems of ny x nx)
// ---------------------------------------------------------------------------
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
  size_t status, desc, field, tprep, wbuf, accum, twx, twy, twy8, chirp, part, invm, total;
  int max_nblk, slots;
};

Layout make_layout(int op, int ny, int nx, int B, int kmax) {
  Layout L{};
  const size_t px = (size_t)ny * nx * B;
  L.max_nblk = nx / min_col_tile(ny);
  L.slots = (op == HG_OP_OSPR ? kmax : kmax + 1) + 1;  // + energy slot
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  L.status = take(sizeof(int));  // the call's numeric status word (first size class of a call)
  L.desc = take(sizeof(Desc) * B);
  L.field = take(px * sizeof(float2));
  L.tprep = take(px * sizeof(float));
  L.wbuf = take(op == HG_OP_WGS ? px * sizeof(float) : 0);
  L.accum = take(op == HG_OP_OSPR ? px * sizeof(float) : 0);
  L.twx = take(nx * sizeof(float2));
  L.twy = take(ny * sizeof(float2));
  L.twy8 = take(op == HG_OP_OSPR ? ny * sizeof(float2) : 0);  // column twiddles of the 8-element plan
  L.chirp = take((size_t)B * (nx + ny) * sizeof(float2));
  L.part = take((size_t)B * L.slots * L.max_nblk * 4 * sizeof(double));
  L.invm = take((size_t)B * sizeof(float));
  L.total = o;
  return L;
}

Layout make_prop_layout(int ny, int nx) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  L.twx = take(nx * sizeof(float2));
  L.twy = take(ny * sizeof(float2));
  L.chirp = take((size_t)(nx + ny) * sizeof(float2));
  L.total = o;
  return L;
}

template <class T> T* at(void* ws, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + off); }

double chirp_rate(double lambda, double pitch, double z) {
  if (!(z > 0.0) || !std::isfinite(z)) return 0.0;
  return pitch * pitch / (lambda * z);
}
bool is_fresnel(double lambda, double pitch, double z) { return chirp_rate(lambda, pitch, z) != 0.0; }

// ---------------------------------------------------------------------------
// small upload kernels: descriptors by value (no host->device copies, so the
// whole sequence stays on the stream and is graph-capturable)
// ---------------------------------------------------------------------------
struct DescPack { Desc d[8]; int count; };
__global__ void k_set_desc(Desc* dst, DescPack pk, int* clear_status) {
  const int i = threadIdx.x;
  if (i < pk.count) dst[i] = pk.d[i];
  if (clear_status && i == 0) *clear_status = 0;
}

__global__ void k_fill(float* p, size_t n, float v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hg_status check_launch() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HG_ERR_HIP, "HIP launch failed: %s", hipGetErrorString(e));
  return HG_OK;
}

// Descriptor upload; the first launch also clears the call's status word
// when clear_status is given (the first size class of a call).
void upload_descs(Desc* dst, const std::vector<Desc>& ds, hipStream_t st, int* clear_status = nullptr) {
  for (size_t i = 0; i < ds.size(); i += 8) {
    DescPack pk{};
    pk.count = (int)std::min<size_t>(8, ds.size() - i);
    for (int j = 0; j < pk.count; ++j) pk.d[j] = ds[i + j];
    hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(64), 0, st, dst + i, pk, i == 0 ? clear_status : nullptr);
  }
}

void launch_twiddles(float2* tw, int n, hipStream_t st) {
  with_size(n, [&](auto nc) { launch_twiddles_t<decltype(nc)::value>(tw, st); });
}
void launch_twiddles8(float2* tw, int n, hipStream_t st) {
  with_size(n, [&](auto nc) { launch_twiddles8_t<decltype(nc)::value>(tw, st); });
}

void launch_chirps(float2* chirp, int ny, int nx, const std::vector<double>& rates, hipStream_t st) {
  for (size_t i = 0; i < rates.size(); i += 32) {
    ChirpArgs ca{};
    ca.count = (int)std::min<size_t>(32, rates.size() - i);
    for (int j = 0; j < ca.count; ++j) ca.a[j] = rates[i + j];
    hipLaunchKernelGGL(k_chirps, dim3((nx + ny + 255) / 256, ca.count), dim3(256), 0, st, chirp, ny, nx, ca,
                       (int)i);
  }
}

// ---------------------------------------------------------------------------
// pass launchers
// ---------------------------------------------------------------------------
void launch_row(const Batch& bt, int RPB, int B, bool fresnel, int lk, int mode, int arg, const float2* pin,
                float2* pout, hipStream_t st) {
  TimeScope ts(TC_ROW, st);
  with_size(bt.nx, [&](auto nc) {
    launch_row_t<decltype(nc)::value>(RPB, fresnel, lk, bt, B, mode, arg, pin, pout, st);
  });
}

void launch_col(const Batch& bt, int C, int B, int mode, int arg, int adaptive, const float2* pin, float2* pout,
                hipStream_t st) {
  TimeScope ts(TC_COL, st);
  with_size(bt.ny, [&](auto nc) {
    launch_col_t<decltype(nc)::value>(C, bt, B, mode, arg, adaptive, pin, pout, st);
  });
}

void launch_col_prep(const Batch& bt, int C, int B, int mode, int arg, hipStream_t st) {
  TimeScope ts(TC_SETUP, st);
  with_size(bt.ny, [&](auto nc) { launch_col_prep_t<decltype(nc)::value>(C, bt, B, mode, arg, st); });
}

void launch_setup(const Batch& bt, int C, int B, int weighted, hipStream_t st) {
  TimeScope ts(TC_SETUP, st);
  with_size(bt.ny, [&](auto nc) { launch_setup_t<decltype(nc)::value>(C, bt, B, weighted, st); });
}

Batch make_batch(void* ws, const Layout& L, int ny, int nx, int C) {
  Batch bt{};
  bt.desc = at<Desc>(ws, L.desc);
  bt.field = at<float2>(ws, L.field);
  bt.tprep = at<float>(ws, L.tprep);
  bt.wbuf = at<float>(ws, L.wbuf);
  bt.accum = at<float>(ws, L.accum);
  bt.tw_x = at<float2>(ws, L.twx);
  bt.tw_y = ny != nx ? at<float2>(ws, L.twy) : bt.tw_x;
  bt.chirp = at<float2>(ws, L.chirp);
  bt.part = at<double>(ws, L.part);
  bt.invm = at<float>(ws, L.invm);
  bt.ny = ny;
  bt.nx = nx;
  bt.nblk = nx / C;
  bt.slots = L.slots;
  bt.fwd_scale = (float)(1.0 / std::sqrt((double)nx * (double)ny));
  return bt;
}

// Whole GS / WGS pipeline for one size class.
// status: the call's status word; cleared here when `first` (the call's first size class).
// f16: the class's field plane holds 16-bit elements (the default launch
// configuration, whose kernels exist for them, and their power-of-two scales).
hg_status run_gs_class(int ny, int nx, const std::vector<Desc>& ds, const std::vector<double>& rates, bool weighted,
                       void* ws, const Layout& L, hipStream_t st, int* status, bool first, bool f16 = false,
                       int class_b = 0) {
  const int B = (int)ds.size();
  int kmax = 0;
  bool all_bin = true;
  for (const Desc& d : ds) {
    kmax = std::max(kmax, d.iters);
    all_bin &= (d.L == 2 && !d.mod);
  }
  // 16-bit planes: the tile kernel's shape (256 threads: C = 4096 / ny) and
  // the default row grouping, the instantiations that exist for them
  const Cfg cfg = f16 ? Cfg{4096 / ny, default_rpb(nx)} : get_cfg(ny, nx, std::max(B, class_b));
  if (!col_ok(ny, cfg.C) || !rpb_ok(nx, cfg.RPB))  // a pass with no compiled kernel would launch nothing
    return fail(HG_ERR_INVALID_ARG, "no kernel for %d-column tiles / %d rows per group at %dx%d", cfg.C, cfg.RPB, ny, nx);
  Batch bt = make_batch(ws, L, ny, nx, cfg.C);
  bt.class_b = class_b;
  if (f16) {
    bt.f16 = 1;
    const int ex = ilog2(nx) / 2, ey = ilog2(ny) / 2;  // 2^-floor(log2(n) / 2)
    bt.s16_row = std::ldexp(1.0f, -ex);
    bt.inv16_row = std::ldexp(1.0f, ex);
    bt.s16_col = std::ldexp(1.0f, -ey);
    bt.inv16_col = std::ldexp(1.0f, ey);
  }
  // Liu-Taghizadeh or a region of interest: not in the single-launch
  // small-problem kernel; in the classic kernels' window instantiation
  bool any_lt = false, any_roi = false;
  for (const Desc& d : ds) {
    any_lt |= (d.lt != 0) || (d.roi != nullptr);
    any_roi |= d.roi != nullptr;
  }
  for (const Desc& d : ds) bt.dump |= (d.r_out != nullptr) ? 1 : 0;
  bt.any_lt = any_lt ? 1 : 0;  // the classic GS column kernels' window instantiation
  bt.any_roi = any_roi ? 1 : 0;  // the GS tile kernels' region instantiation
  bt.status = status;
  upload_descs(const_cast<Desc*>(bt.desc), ds, st, first ? status : nullptr);
  bool fresnel = false;
  for (double r : rates) fresnel |= (r != 0.0);
  if (small_ok(ny, nx) && small_enabled() && !any_lt) {
    // whole call in one launch, one workgroup per problem
    if (fresnel) launch_chirps(const_cast<float2*>(bt.chirp), ny, nx, rates, st);
    TimeScope ts(TC_COL, st);
    launch_small(bt, B, fresnel, weighted, st);
    return check_launch();
  }
  launch_twiddles(const_cast<float2*>(bt.tw_x), nx, st);
  if (ny != nx) launch_twiddles(const_cast<float2*>(bt.tw_y), ny, st);
  if (fresnel) launch_chirps(const_cast<float2*>(bt.chirp), ny, nx, rates, st);
  launch_setup(bt, cfg.C, B, weighted ? 1 : 0, st);
  bool all_quad = true;
  for (const Desc& d : ds) all_quad &= ((d.L == 4 || d.L == 8) && !d.mod);
  const int lk = all_bin ? LK_BIN : all_quad ? LK_QUAD : LK_ANY;
  // weighted GS: each row pass also sets 1 / m for the column pass after it
  bt.row_invm = weighted ? 1 : 0;
  launch_row(bt, cfg.RPB, B, fresnel, lk, ROW_INIT, 0, nullptr, nullptr, st);
  const int cmode = weighted ? COL_WGS : COL_GS;
  for (int k = 1; k <= kmax; ++k) {
    launch_col(bt, cfg.C, B, cmode, k, 0, nullptr, nullptr, st);
    launch_row(bt, cfg.RPB, B, fresnel, lk, ROW_ITER, k, nullptr, nullptr, st);
  }
  if (weighted) {
    TimeScope ts(TC_SETUP, st);
    hipLaunchKernelGGL(k_weights_out, dim3((unsigned)(((size_t)ny * nx + 255) / 256), B), dim3(256), 0, st, bt);
  }
  // final measurement pass of every distinct iteration count in the class
  std::vector<int> ks;
  for (const Desc& d : ds) ks.push_back(d.iters);
  std::sort(ks.begin(), ks.end());
  ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
  for (int k : ks) launch_col(bt, cfg.C, B, COL_FINAL, k + 1, 0, nullptr, nullptr, st);
  hipLaunchKernelGGL(k_finish, dim3(B, finish_grid_y(kmax + 1)), dim3(64 * kFinishPerBlock), 0, st, bt, B, 0);
  return check_launch();
}

// Plane bytes per chunk of a batched call (hg_set_batch_chunk): 128 MiB
// unless the environment sets HG_BATCH_CHUNK_MB; 0 runs each size class whole.
constexpr long long kDefaultChunkBytes = 128ll << 20;
static std::atomic<long long> g_chunk_bytes{[] {
  const char* e = std::getenv("HG_BATCH_CHUNK_MB");
  if (!e || !*e) return kDefaultChunkBytes;
  const long long mb = std::atoll(e);
  return mb > 0 ? (mb << 20) : 0ll;
}()};

// Problems per chunk of a size class of B problems of `per` plane bytes each
// under the chunk size (hg_set_batch_chunk), balanced over the chunks.
int chunk_problems(int B, size_t per, bool chunkable) {
  const size_t chunk = (size_t)g_chunk_bytes.load(std::memory_order_relaxed);
  if (chunk == 0 || !chunkable) return B;
  const int cap = (int)std::max<size_t>(1, std::min<size_t>((size_t)B, chunk / per));
  const int n = (B + cap - 1) / cap;
  return (B + n - 1) / n;
}

// Whole OSPR / adaptive OSPR pipeline for one size class: B problems with
// the same number of subframes, one batched launch per pass (class_b: problems of
// the whole class when this is one of its chunks).
hg_status run_ospr_class(int ny, int nx, const std::vector<Desc>& ds, int subframes, int adaptive, void* ws,
                         const Layout& L, hipStream_t st, int* status, bool first, int class_b = 0) {
  const int B = (int)ds.size();
  const int SB = std::max(B, class_b);  // kernel and tile choices follow the whole class
  Cfg cfg = get_cfg(ny, nx, SB);
  // fewer than 8 problems of 512 rows: 4-column tiles (the default unless a
  // configuration was tuned or set), which run with 8 elements per thread in
  // the column passes: twice the workgroups of the default tiles and half
  // the per-thread work
  if (ny == 512 && batch_class(SB) == 0 && !has_tuned_cfg(ny, nx, SB)) {
    cfg.C = 4;
    if (nx == 512) cfg.RPB = 4;  // 512-wide rows: 8 elements per thread there too, one wave per row
  }
  const bool e8 = ny == 512 && batch_class(SB) == 0 && cfg.C == 4 && column_kernel() == CK_TILE;
  if (!col_ok(ny, cfg.C) || !rpb_ok(nx, cfg.RPB))  // a pass with no compiled kernel would launch nothing
    return fail(HG_ERR_INVALID_ARG, "no kernel for %d-column tiles / %d rows per group at %dx%d", cfg.C, cfg.RPB, ny, nx);
  Batch bt = make_batch(ws, L, ny, nx, cfg.C);
  bt.status = status;
  upload_descs(const_cast<Desc*>(bt.desc), ds, st, first ? status : nullptr);
  launch_twiddles(const_cast<float2*>(bt.tw_x), nx, st);
  if (ny != nx) launch_twiddles(const_cast<float2*>(bt.tw_y), ny, st);
  if (e8) {
    bt.tw_y8 = at<float2>(ws, L.twy8);
    launch_twiddles8(const_cast<float2*>(bt.tw_y8), ny, st);
  }
  launch_setup(bt, cfg.C, B, 0, st);
  launch_col(bt, cfg.C, B, COL_OSPR_FIRST, 1, adaptive, nullptr, nullptr, st);
  for (int n = 1; n <= subframes; ++n) {
    launch_row(bt, cfg.RPB, B, false, LK_BIN, ROW_OSPR, n, nullptr, nullptr, st);
    launch_col(bt, cfg.C, B, n == subframes ? COL_OSPR_FINAL : COL_OSPR, n + 1, adaptive, nullptr, nullptr, st);
  }
  hipLaunchKernelGGL(k_finish, dim3(B, finish_grid_y(subframes)), dim3(64 * kFinishPerBlock), 0, st, bt, B, 1);
  return check_launch();
}

hg_status check_ws(void* ws, size_t bytes, size_t need) {
  if (!ws) return fail(HG_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(HG_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (bytes < need) return fail(HG_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", bytes, need);
  return HG_OK;
}

hg_status check_size(int ny, int nx) {
  if (!pow2_in_range(ny) || !pow2_in_range(nx))
    return fail(HG_ERR_UNSUPPORTED_SIZE, "ny=%d nx=%d: each must be a power of two in [64, 4096]", ny, nx);
  return HG_OK;
}

// slm_levels: the level count, with HG_SLM_AMPLITUDE or-ed in for an
// amplitude-modulating SLM.
int levels_of(int slm_levels) { return slm_levels & ~(HG_SLM_AMPLITUDE | HG_FIELD_FP16); }
int modulation_of(int slm_levels) { return (slm_levels & HG_SLM_AMPLITUDE) ? 1 : 0; }
int field16_of(int slm_levels) { return (slm_levels & HG_FIELD_FP16) ? 1 : 0; }

hg_status check_common(const float* target, int ny, int nx, int iters, int slm_levels) {
  hg_status s = check_size(ny, nx);
  if (s != HG_OK) return s;
  if (!target) return fail(HG_ERR_INVALID_ARG, "target is NULL");
  if (iters < 1) return fail(HG_ERR_INVALID_ARG, "iters=%d must be >= 1", iters);
  const int L = levels_of(slm_levels);
  if (!(L == 0 || (L >= 2 && L <= 256))) return fail(HG_ERR_INVALID_ARG, "slm_levels=%d: 0 or 2..256", L);
  if (modulation_of(slm_levels) && L < 2)
    return fail(HG_ERR_INVALID_ARG, "an amplitude SLM needs 2..256 levels (slm_levels=%d)", L);
  if (field16_of(slm_levels) && !f16_ok(ny))
    return fail(HG_ERR_UNSUPPORTED_SIZE, "16-bit field storage needs ny in {256, 512, 1024} (ny=%d)", ny);
  return HG_OK;
}

bool optics_ok(double lambda, double pitch, double z) {
  return !is_fresnel(lambda, pitch, z) ||
         (lambda > 0.0 && pitch > 0.0 && std::isfinite(lambda) && std::isfinite(pitch));
}

hg_status check_lt(bool weighted, int lt, int r0, int dr) {
  if (!lt) return HG_OK;
  if (weighted) return fail(HG_ERR_INVALID_ARG, "Liu-Taghizadeh is a GS variant (not weighted)");
  if (r0 < 0 || dr < 0) return fail(HG_ERR_INVALID_ARG, "lt_r0=%d and lt_dr=%d must be >= 0", r0, dr);
  return HG_OK;
}

// Host-side checks of a GS / WGS / LT call's arguments (no HIP call).
hg_status check_gs_args(bool weighted, const float* target, int ny, int nx, int iters, int L,
                        const uint8_t* init_levels, const uint8_t* levels_out, double lambda, double pitch, double z,
                        int lt, int lt_r0, int lt_dr) {
  hg_status s = check_common(target, ny, nx, iters, L);
  if (s != HG_OK) return s;
  s = check_lt(weighted, lt, lt_r0, lt_dr);
  if (s != HG_OK) return s;
  if (lt && modulation_of(L)) return fail(HG_ERR_INVALID_ARG, "Liu-Taghizadeh runs on phase SLMs only");
  L = levels_of(L);
  if (L >= 2 && !levels_out) return fail(HG_ERR_INVALID_ARG, "levels_out is required when slm_levels >= 2");
  if (init_levels && L < 2) return fail(HG_ERR_INVALID_ARG, "init_levels needs slm_levels >= 2");
  if (!optics_ok(lambda, pitch, z)) return fail(HG_ERR_INVALID_ARG, "Fresnel needs wavelength_m > 0 and pitch_m > 0");
  return HG_OK;
}

hg_status gs_common(bool weighted, const float* target, int ny, int nx, int iters, int L, uint64_t seed,
                    const uint8_t* init_levels, const hg_complex* init_field, double lambda, double pitch,
                    double z, uint8_t* levels_out, hg_complex* field_out, hg_complex* replay_out,
                    double* nmse_out, float* weights, void* ws, size_t ws_bytes, void* stream, int lt = 0,
                    int lt_r0 = 0, int lt_dr = 0, hg_complex* r_out = nullptr, hg_complex* g_out = nullptr) {
  g_err[0] = 0;
  hg_status s = check_gs_args(weighted, target, ny, nx, iters, L, init_levels, levels_out, lambda, pitch, z, lt,
                              lt_r0, lt_dr);
  if (s != HG_OK) return s;
  const int op = weighted ? HG_OP_WGS : HG_OP_GS;
  const Layout Lo = make_layout(op, ny, nx, 1, iters);
  s = check_ws(ws, ws_bytes, Lo.total);
  if (s != HG_OK) return s;
  Desc d{};
  d.target = target;
  d.levels_out = levels_out;
  d.nmse_out = nmse_out;
  d.field_out = reinterpret_cast<float2*>(field_out);
  d.replay_out = reinterpret_cast<float2*>(replay_out);
  d.weights = weights;
  d.user_weights = weights ? 1 : 0;
  d.init_levels = init_levels;
  d.init_field = reinterpret_cast<const float2*>(init_field);
  d.seed = seed;
  d.item = 0;
  d.L = levels_of(L);
  d.mod = modulation_of(L);
  d.iters = iters;
  d.lt = lt ? 1 : 0;
  d.lt_r0 = lt_r0;
  d.lt_dr = lt_dr;
  d.r_out = reinterpret_cast<float2*>(r_out);
  d.g_out = reinterpret_cast<float2*>(g_out);
  std::vector<Desc> ds{d};
  std::vector<double> rates{chirp_rate(lambda, pitch, z)};
  return run_gs_class(ny, nx, ds, rates, weighted, ws, Lo, static_cast<hipStream_t>(stream), at<int>(ws, Lo.status),
                      true, field16_of(L) != 0);
}

// Size classes of a batched call in order of first appearance: problems of
// one grid size and one field storage (complex64 or 16-bit) share launches.
struct ClassKey {
  int ny, nx, f16;
  bool operator<(const ClassKey& o) const { return std::tie(ny, nx, f16) < std::tie(o.ny, o.nx, o.f16); }
};
struct ClassPlan {
  std::vector<ClassKey> order;
  std::map<ClassKey, std::vector<int>> members;
};
int storage16_of(const hg_problem& p) { return (p.slm_levels & HG_FIELD_FP16) ? 1 : 0; }
int storage16_of(const hg_ospr_problem&) { return 0; }
template <class P>
ClassPlan plan_classes(const P* probs, int count) {
  ClassPlan cp;
  for (int i = 0; i < count; ++i) {
    const ClassKey key{probs[i].ny, probs[i].nx, storage16_of(probs[i])};
    if (!cp.members.count(key)) cp.order.push_back(key);
    cp.members[key].push_back(i);
  }
  return cp;
}

// Device address of `scratch` on the current device, looked up once per
// device and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hg_status static_scratch(void** out) {
  int dev = -1;
  const hipError_t ge = hipGetDevice(&dev);
  if (ge != hipSuccess) return fail(HG_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(ge));
  if (dev < 0 || dev >= kMaxDevices) return fail(HG_ERR_HIP, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(HG_ERR_HIP, "hipGetSymbolAddress of the static scratch failed on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HG_OK;
}

}  // namespace

// Single-launch path for small problems: on unless HG_SMALL_KERNEL=off or
// switched by hg_set_small_fused.
static std::atomic<int> g_small_fused{[] {
  const char* e = std::getenv("HG_SMALL_KERNEL");
  return (e && std::string(e) == "off") ? 0 : 1;
}()};

// Column-pass kernel kind (ColumnKernel): one tile per workgroup unless
// HG_COLUMN_KERNEL=persistent or =classic, or switched by hg_set_column_kernel.
static std::atomic<int> g_column_kernel{[] {
  const char* e = std::getenv("HG_COLUMN_KERNEL");
  if (e && std::string(e) == "persistent") return (int)hg::CK_PERSISTENT;
  if (e && std::string(e) == "classic") return (int)hg::CK_CLASSIC;
  return (int)hg::CK_TILE;
}()};

namespace hg {

bool small_enabled() { return g_small_fused.load(std::memory_order_relaxed) != 0; }
int column_kernel() { return g_column_kernel.load(std::memory_order_relaxed); }
}  // namespace hg

// Error text shared with the network translation unit (same thread-local
// buffer that hg_last_error returns).
namespace hg_internal {
void set_error(const char* msg) { snprintf(g_err, sizeof(g_err), "%s", msg); }
}  // namespace hg_internal

extern "C" {

const char* hg_status_string(hg_status s) {
  switch (s) {
    case HG_OK: return "ok";
    case HG_ERR_INVALID_ARG: return "invalid argument";
    case HG_ERR_UNSUPPORTED_SIZE: return "unsupported size";
    case HG_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case HG_ERR_HIP: return "HIP runtime error";
    case HG_ERR_NUMERIC: return "non-finite values in the NMSE sums";
  }
  return "unknown status";
}

const char* hg_last_error(void) { return g_err; }

hg_status hg_numeric_status(const void* workspace, void* stream) {
  g_err[0] = 0;
  if (!workspace) return fail(HG_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(HG_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
    return fail(HG_ERR_HIP, "hipStreamSynchronize failed");
  int flag = 0;
  if (hipMemcpy(&flag, workspace, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(HG_ERR_HIP, "hipMemcpy of the status word failed");
  if (flag) return fail(HG_ERR_NUMERIC, "a finisher saw non-finite NMSE sums (NaN or Inf in the target or weights)");
  return HG_OK;
}

void hg_timing_enable(int on) { g_timing.on = on != 0; }

hg_status hg_timing_read(hg_kernel_times* out) {
  g_err[0] = 0;
  if (!out) return fail(HG_ERR_INVALID_ARG, "out is NULL");
  *out = hg_kernel_times{};
  for (auto& m : g_timing.marks) {
    float ms = 0.f;
    if (hipEventSynchronize(g_timing.pool[m.second + 1]) != hipSuccess ||
        hipEventElapsedTime(&ms, g_timing.pool[m.second], g_timing.pool[m.second + 1]) != hipSuccess)
      return fail(HG_ERR_HIP, "hipEvent timing failed");
    if (m.first == TC_COL) { out->col_ms += ms; out->col_launches++; }
    else if (m.first == TC_ROW) { out->row_ms += ms; out->row_launches++; }
    else { out->setup_ms += ms; out->setup_launches++; }
  }
  g_timing.marks.clear();
  g_timing.used = 0;
  return HG_OK;
}

hg_status hg_set_column_kernel(int kind) {
  g_err[0] = 0;
  if (kind < CK_TILE || kind > CK_CLASSIC) return fail(HG_ERR_INVALID_ARG, "kind must be 0, 1 or 2");
  g_column_kernel.store(kind, std::memory_order_relaxed);
  return HG_OK;
}

hg_status hg_set_batch_chunk(size_t field_bytes) {
  g_err[0] = 0;
  if (field_bytes > ((size_t)1 << 40)) return fail(HG_ERR_INVALID_ARG, "chunk of %zu bytes beyond 1 TiB", field_bytes);
  g_chunk_bytes.store((long long)field_bytes, std::memory_order_relaxed);
  return HG_OK;
}

size_t hg_get_batch_chunk(void) { return (size_t)g_chunk_bytes.load(std::memory_order_relaxed); }

hg_status hg_set_small_fused(int enable) {
  g_err[0] = 0;
  if (enable != 0 && enable != 1) return fail(HG_ERR_INVALID_ARG, "enable must be 0 or 1");
  g_small_fused.store(enable, std::memory_order_relaxed);
  return HG_OK;
}

size_t hg_workspace_size(int op, int ny, int nx, int iters) {
  if (!pow2_in_range(ny) || !pow2_in_range(nx)) return 0;
  if (op == HG_OP_PROPAGATE) return make_prop_layout(ny, nx).total;
  if (op != HG_OP_GS && op != HG_OP_WGS && op != HG_OP_OSPR) return 0;
  if (iters < 1) return 0;
  return make_layout(op, ny, nx, 1, iters).total;
}

hg_status hg_gs(const float* target, int ny, int nx, int iters, int slm_levels, uint64_t seed,
                const uint8_t* init_levels, const hg_complex* init_field, double wavelength_m, double pitch_m,
                double z_m, uint8_t* levels_out, hg_complex* slm_field_out, hg_complex* replay_out,
                double* nmse_out, void* workspace, size_t workspace_bytes, void* stream) {
  return gs_common(false, target, ny, nx, iters, slm_levels, seed, init_levels, init_field, wavelength_m, pitch_m,
                   z_m, levels_out, slm_field_out, replay_out, nmse_out, nullptr, workspace, workspace_bytes, stream);
}

hg_status hg_wgs(const float* target, int ny, int nx, int iters, int slm_levels, uint64_t seed,
                 const uint8_t* init_levels, const hg_complex* init_field, double wavelength_m, double pitch_m,
                 double z_m, uint8_t* levels_out, hg_complex* slm_field_out, hg_complex* replay_out,
                 double* nmse_out, float* weights_inout, void* workspace, size_t workspace_bytes, void* stream) {
  return gs_common(true, target, ny, nx, iters, slm_levels, seed, init_levels, init_field, wavelength_m, pitch_m,
                   z_m, levels_out, slm_field_out, replay_out, nmse_out, weights_inout, workspace, workspace_bytes,
                   stream);
}

hg_status hg_wgs_static(const float* target, int ny, int nx, int iters, int slm_levels, uint64_t seed,
                        const uint8_t* init_levels, const hg_complex* init_field, double wavelength_m,
                        double pitch_m, double z_m, uint8_t* levels_out, hg_complex* slm_field_out,
                        hg_complex* replay_out, double* nmse_out, float* weights_inout, void* stream) {
  g_err[0] = 0;
  hg_status s = check_gs_args(true, target, ny, nx, iters, slm_levels, init_levels, levels_out, wavelength_m, pitch_m,
                              z_m, 0, 0, 0);
  if (s != HG_OK) return s;
  const size_t need = make_layout(HG_OP_WGS, ny, nx, 1, iters).total;
  if (need > HG_STATIC_SCRATCH_BYTES)
    return fail(HG_ERR_WORKSPACE, "hg_wgs_static: %d x %d with %d iterations needs %zu bytes of scratch, "
                "beyond the static scratch of %zu bytes (use hg_wgs with a workspace)", ny, nx, iters, need,
                (size_t)HG_STATIC_SCRATCH_BYTES);
  void* ws = nullptr;
  s = static_scratch(&ws);
  if (s != HG_OK) return s;
  return gs_common(true, target, ny, nx, iters, slm_levels, seed, init_levels, init_field, wavelength_m, pitch_m,
                   z_m, levels_out, slm_field_out, replay_out, nmse_out, weights_inout, ws, HG_STATIC_SCRATCH_BYTES,
                   stream);
}

hg_status hg_gs_step(const float* target, int ny, int nx, int slm_levels, int weighted, const uint8_t* levels_in,
                     const hg_complex* field_in, double wavelength_m, double pitch_m, double z_m, int lt_radius,
                     float* weights_inout, hg_complex* r_out, hg_complex* g_out, uint8_t* levels_out,
                     hg_complex* field_out, double* nmse_out, void* workspace, size_t workspace_bytes,
                     void* stream) {
  g_err[0] = 0;
  if ((levels_in == nullptr) == (field_in == nullptr))
    return fail(HG_ERR_INVALID_ARG, "exactly one of levels_in and field_in gives the start state");
  if (weighted && !weights_inout) return fail(HG_ERR_INVALID_ARG, "weighted step needs weights_inout (w_{k-1})");
  if (weighted && lt_radius >= 0) return fail(HG_ERR_INVALID_ARG, "Liu-Taghizadeh is a GS variant (not weighted)");
  const bool lt = lt_radius >= 0;
  return gs_common(weighted != 0, target, ny, nx, 1, slm_levels, 0, levels_in, field_in, wavelength_m, pitch_m, z_m,
                   levels_out, field_out, nullptr, nmse_out, weighted ? weights_inout : nullptr, workspace,
                   workspace_bytes, stream, lt ? 1 : 0, lt ? lt_radius : 0, 0, r_out, g_out);
}

hg_status hg_lt(const float* target, int ny, int nx, int iters, int slm_levels, uint64_t seed,
                const uint8_t* init_levels, const hg_complex* init_field, double wavelength_m, double pitch_m,
                double z_m, int lt_r0, int lt_dr, uint8_t* levels_out, hg_complex* slm_field_out,
                hg_complex* replay_out, double* nmse_out, void* workspace, size_t workspace_bytes, void* stream) {
  return gs_common(false, target, ny, nx, iters, slm_levels, seed, init_levels, init_field, wavelength_m, pitch_m,
                   z_m, levels_out, slm_field_out, replay_out, nmse_out, nullptr, workspace, workspace_bytes, stream,
                   1, lt_r0, lt_dr);
}

hg_status hg_ospr(const float* target, int ny, int nx, int subframes, int adaptive, uint64_t seed,
                  uint8_t* levels_out, double* nmse_out, float* accum_out, void* workspace, size_t workspace_bytes,
                  void* stream) {
  g_err[0] = 0;
  hg_status s = check_common(target, ny, nx, subframes, 2);
  if (s != HG_OK) return s;
  if (!levels_out) return fail(HG_ERR_INVALID_ARG, "levels_out is required");
  const Layout Lo = make_layout(HG_OP_OSPR, ny, nx, 1, subframes);
  s = check_ws(workspace, workspace_bytes, Lo.total);
  if (s != HG_OK) return s;
  Desc d{};
  d.target = target;
  d.levels_out = levels_out;
  d.nmse_out = nmse_out;
  d.accum_out = accum_out;
  d.seed = seed;
  d.L = 2;
  d.iters = subframes;
  return run_ospr_class(ny, nx, {d}, subframes, adaptive, workspace, Lo, static_cast<hipStream_t>(stream),
                        at<int>(workspace, Lo.status), true);
}

size_t hg_ospr_batched_workspace_size(const hg_ospr_problem* probs, int count, int subframes) {
  if (!probs || count < 1 || subframes < 1) return 0;
  for (int i = 0; i < count; ++i)
    if (!pow2_in_range(probs[i].ny) || !pow2_in_range(probs[i].nx)) return 0;
  const ClassPlan cp = plan_classes(probs, count);
  size_t total = 0;
  for (auto& key : cp.order)
    total += make_layout(HG_OP_OSPR, key.ny, key.nx, (int)cp.members.at(key).size(), subframes).total;
  return total;
}

hg_status hg_ospr_batched(const hg_ospr_problem* probs, int count, int subframes, int adaptive, void* workspace,
                          size_t workspace_bytes, void* stream) {
  g_err[0] = 0;
  if (!probs || count < 1) return fail(HG_ERR_INVALID_ARG, "problems is NULL or count < 1");
  for (int i = 0; i < count; ++i) {
    hg_status s = check_common(probs[i].target, probs[i].ny, probs[i].nx, subframes, 2);
    if (s != HG_OK) {
      std::string msg = g_err;
      return fail(s, "problem %d: %s", i, msg.c_str());
    }
    if (!probs[i].levels_out) return fail(HG_ERR_INVALID_ARG, "problem %d: levels_out is required", i);
  }
  const size_t need = hg_ospr_batched_workspace_size(probs, count, subframes);
  hg_status s = check_ws(workspace, workspace_bytes, need);
  if (s != HG_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const ClassPlan cp = plan_classes(probs, count);
  size_t off = 0;
  for (auto& key : cp.order) {
    const std::vector<int>& idx = cp.members.at(key);
    std::vector<Desc> ds;
    for (int i : idx) {
      Desc d{};
      d.target = probs[i].target;
      d.levels_out = probs[i].levels_out;
      d.nmse_out = probs[i].nmse_out;
      d.accum_out = probs[i].accum_out;
      d.seed = probs[i].seed;
      d.item = (uint32_t)i;
      d.L = 2;
      d.iters = subframes;
      ds.push_back(d);
    }
    const Layout Lo = make_layout(HG_OP_OSPR, key.ny, key.nx, (int)idx.size(), subframes);
    // chunks of at most the chunk size of field planes, as in hg_gs_batched
    // (16 problems of 1024^2 by default: their field and accumulator planes,
    // 192 MiB, measured faster than chunks of 8)
    const int B = (int)ds.size();
    const int cb = chunk_problems(B, (size_t)key.ny * key.nx * 8, true);
    for (int c0 = 0; c0 < B; c0 += cb) {
      const int nc = std::min(cb, B - c0);
      const std::vector<Desc> dc(ds.begin() + c0, ds.begin() + c0 + nc);
      const Layout Lc = nc == B ? Lo : make_layout(HG_OP_OSPR, key.ny, key.nx, nc, subframes);
      if (Lc.total > Lo.total) return fail(HG_ERR_INVALID_ARG, "chunk layout exceeds its class's workspace");
      s = run_ospr_class(key.ny, key.nx, dc, subframes, adaptive, static_cast<char*>(workspace) + off, Lc, st,
                         at<int>(workspace, 0), off == 0 && c0 == 0, B);
      if (s != HG_OK) return s;
    }
    off += Lo.total;
  }
  return HG_OK;
}

hg_status hg_fresnel_propagate(const hg_complex* in, hg_complex* out, int ny, int nx, double wavelength_m,
                               double pitch_m, double z_m, int direction, void* workspace, size_t workspace_bytes,
                               void* stream) {
  g_err[0] = 0;
  hg_status s = check_size(ny, nx);
  if (s != HG_OK) return s;
  if (!in || !out) return fail(HG_ERR_INVALID_ARG, "in and out must be non-NULL");
  if (direction != 1 && direction != -1) return fail(HG_ERR_INVALID_ARG, "direction must be +1 or -1");
  if (!optics_ok(wavelength_m, pitch_m, z_m))
    return fail(HG_ERR_INVALID_ARG, "Fresnel needs wavelength_m > 0 and pitch_m > 0");
  const bool fres = is_fresnel(wavelength_m, pitch_m, z_m);
  const Layout Lo = make_prop_layout(ny, nx);
  s = check_ws(workspace, workspace_bytes, Lo.total);
  if (s != HG_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Cfg cfg = get_cfg(ny, nx, 1);
  Batch bt{};
  bt.tw_x = at<float2>(workspace, Lo.twx);
  bt.tw_y = ny != nx ? at<float2>(workspace, Lo.twy) : bt.tw_x;
  bt.chirp = at<float2>(workspace, Lo.chirp);
  bt.ny = ny;
  bt.nx = nx;
  launch_twiddles(const_cast<float2*>(bt.tw_x), nx, st);
  if (ny != nx) launch_twiddles(const_cast<float2*>(bt.tw_y), ny, st);
  if (fres) launch_chirps(const_cast<float2*>(bt.chirp), ny, nx, {chirp_rate(wavelength_m, pitch_m, z_m)}, st);
  const float2* fin = reinterpret_cast<const float2*>(in);
  float2* fout = reinterpret_cast<float2*>(out);
  if (direction > 0) {
    launch_row(bt, cfg.RPB, 1, fres, LK_ANY, ROW_PROP_FWD, 0, fin, fout, st);
    launch_col(bt, cfg.C, 1, COL_PROP_FWD, 0, 0, fout, fout, st);
  } else {
    launch_col(bt, cfg.C, 1, COL_PROP_BWD, 0, 0, fin, fout, st);
    launch_row(bt, cfg.RPB, 1, fres, LK_ANY, ROW_PROP_BWD, 0, fout, fout, st);
  }
  return check_launch();
}

hg_status hg_random_phase(uint64_t seed, uint32_t item, uint32_t tag, int axis, int ny, int nx, hg_complex* out,
                          void* stream) {
  g_err[0] = 0;
  hg_status s = check_size(ny, nx);
  if (s != HG_OK) return s;
  if (!out) return fail(HG_ERR_INVALID_ARG, "out is NULL");
  if (axis != 0 && axis != 1) return fail(HG_ERR_INVALID_ARG, "axis must be 0 (column lines) or 1 (row lines)");
  const int nthreads = ny * nx / 4;
  hipLaunchKernelGGL(k_random_phase, dim3((nthreads + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<float2*>(out), seed, item, tag, ny, nx, axis);
  return check_launch();
}

size_t hg_gs_batched_workspace_size(const hg_problem* probs, int count) {
  if (!probs || count < 1) return 0;
  for (int i = 0; i < count; ++i)
    if (!pow2_in_range(probs[i].ny) || !pow2_in_range(probs[i].nx) || probs[i].iters < 1) return 0;
  const ClassPlan cp = plan_classes(probs, count);
  size_t total = 0;
  for (auto& key : cp.order) {
    int kmax = 0;
    for (int i : cp.members.at(key)) kmax = std::max(kmax, probs[i].iters);
    // the weighted layout is the larger one; one query serves both modes
    total += make_layout(HG_OP_WGS, key.ny, key.nx, (int)cp.members.at(key).size(), kmax).total;
  }
  return total;
}

hg_status hg_gs_batched(const hg_problem* probs, int count, int weighted, void* workspace, size_t workspace_bytes,
                        void* stream) {
  g_err[0] = 0;
  if (!probs || count < 1) return fail(HG_ERR_INVALID_ARG, "problems is NULL or count < 1");
  for (int i = 0; i < count; ++i) {
    const hg_problem& p = probs[i];
    hg_status s = check_common(p.target, p.ny, p.nx, p.iters, p.slm_levels);
    if (s != HG_OK) {
      std::string msg = g_err;
      return fail(s, "problem %d: %s", i, msg.c_str());
    }
    if (levels_of(p.slm_levels) >= 2 && !p.levels_out)
      return fail(HG_ERR_INVALID_ARG, "problem %d: levels_out required", i);
    if (!optics_ok(p.wavelength_m, p.pitch_m, p.z_m))
      return fail(HG_ERR_INVALID_ARG, "problem %d: Fresnel needs wavelength_m > 0 and pitch_m > 0", i);
    if (p.init_levels && levels_of(p.slm_levels) < 2)
      return fail(HG_ERR_INVALID_ARG, "problem %d: init_levels needs slm_levels >= 2", i);
    if (p.lt && modulation_of(p.slm_levels))
      return fail(HG_ERR_INVALID_ARG, "problem %d: Liu-Taghizadeh runs on phase SLMs only", i);
    s = check_lt(weighted != 0, p.lt, p.lt_r0, p.lt_dr);
    if (s != HG_OK) {
      std::string msg = g_err;
      return fail(s, "problem %d: %s", i, msg.c_str());
    }
    if (p.roi && (weighted || p.lt))
      return fail(HG_ERR_INVALID_ARG, "problem %d: a region of interest runs with plain GS (not weighted, not LT)", i);
  }
  const size_t need = hg_gs_batched_workspace_size(probs, count);
  hg_status s = check_ws(workspace, workspace_bytes, need);
  if (s != HG_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const ClassPlan cp = plan_classes(probs, count);
  size_t off = 0;
  for (auto& key : cp.order) {
    const std::vector<int>& idx = cp.members.at(key);
    std::vector<Desc> ds;
    std::vector<double> rates;
    int kmax = 0;
    for (int i : idx) {
      const hg_problem& p = probs[i];
      Desc d{};
      d.target = p.target;
      d.levels_out = p.levels_out;
      d.nmse_out = p.nmse_out;
      d.init_levels = p.init_levels;
      d.replay_out = reinterpret_cast<float2*>(p.replay_out);
      d.seed = p.seed;
      d.item = (uint32_t)i;
      d.L = levels_of(p.slm_levels);
      d.mod = modulation_of(p.slm_levels);
      d.iters = p.iters;
      d.lt = p.lt ? 1 : 0;
      d.lt_r0 = p.lt_r0;
      d.lt_dr = p.lt_dr;
      d.weights = weighted ? p.weights : nullptr;
      d.user_weights = (weighted && p.weights) ? 1 : 0;
      d.roi = p.roi;
      ds.push_back(d);
      rates.push_back(chirp_rate(p.wavelength_m, p.pitch_m, p.z_m));
      kmax = std::max(kmax, p.iters);
    }
    const Layout Lo = make_layout(HG_OP_WGS, key.ny, key.nx, (int)idx.size(), kmax);
    // Chunks of the class whose field planes fit the last-level cache (256 MB
    // Infinity Cache): the plane a pass writes is then mostly read back by
    // the next pass from the cache, not from HBM.  Each chunk runs its whole
    // pipeline in the class's workspace region before the next (stream
    // order); every problem keeps its own Philox item, and kernel and tile
    // choices follow the whole class, so results do not depend on the
    // chunking.  Single-launch small problems run whole.
    const int B = (int)ds.size();
    const int cb = chunk_problems(B, (size_t)key.ny * key.nx * (key.f16 ? 4 : 8),
                                  !(small_ok(key.ny, key.nx) && small_enabled()));
    for (int c0 = 0; c0 < B; c0 += cb) {
      const int nc = std::min(cb, B - c0);
      const std::vector<Desc> dc(ds.begin() + c0, ds.begin() + c0 + nc);
      const std::vector<double> rc(rates.begin() + c0, rates.begin() + c0 + nc);
      int kc = 0;
      for (const Desc& d : dc) kc = std::max(kc, d.iters);
      const Layout Lc = nc == B ? Lo : make_layout(HG_OP_WGS, key.ny, key.nx, nc, kc);
      if (Lc.total > Lo.total) return fail(HG_ERR_INVALID_ARG, "chunk layout exceeds its class's workspace");
      s = run_gs_class(key.ny, key.nx, dc, rc, weighted != 0, static_cast<char*>(workspace) + off, Lc, st,
                       at<int>(workspace, 0), off == 0 && c0 == 0, key.f16 != 0, B);
      if (s != HG_OK) return s;
    }
    off += Lo.total;
  }
  return HG_OK;
}

size_t hg_autotune_workspace_size(int ny, int nx, int batch) {
  if (!pow2_in_range(ny) || !pow2_in_range(nx) || batch < 1) return 0;
  const size_t px = (size_t)ny * nx * batch;
  return make_layout(HG_OP_WGS, ny, nx, batch, 4).total + align256(px * sizeof(float)) + align256(px);
}

hg_status hg_autotune(int ny, int nx, int batch, int* col_tile, int* rows_per_group, void* workspace,
                      size_t workspace_bytes, void* stream) {
  g_err[0] = 0;
  hg_status s = check_size(ny, nx);
  if (s != HG_OK) return s;
  if (batch < 1) return fail(HG_ERR_INVALID_ARG, "batch must be >= 1");
  s = check_ws(workspace, workspace_bytes, hg_autotune_workspace_size(ny, nx, batch));
  if (s != HG_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout Lo = make_layout(HG_OP_WGS, ny, nx, batch, 4);
  const size_t px = (size_t)ny * nx * batch;
  float* target = at<float>(workspace, Lo.total);
  uint8_t* levels = at<uint8_t>(workspace, Lo.total + align256(px * sizeof(float)));
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((px + 255) / 256)), dim3(256), 0, st, target, px, 1.0f);
  std::vector<Desc> ds(batch);
  for (int b = 0; b < batch; ++b) {
    ds[b] = Desc{};
    ds[b].target = target + (size_t)b * ny * nx;
    ds[b].levels_out = levels + (size_t)b * ny * nx;
    ds[b].seed = 1;
    ds[b].item = (uint32_t)b;
    ds[b].L = 2;
    ds[b].iters = 1 << 20;  // never the last iteration: no level writes
  }
  const bool was_on = g_timing.on;
  g_timing.on = false;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(HG_ERR_HIP, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(HG_ERR_HIP, "hipEventCreate failed");
  }
  auto time_ms = [&](auto&& body) {
    body();  // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < 3; ++r) body();
    (void)hipEventRecord(e1, st);
    float ms = 0.f;
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms;
  };
  const Cfg def = default_cfg(ny, nx, batch);
  Cfg best = def;
  float best_col = 1e30f, best_row = 1e30f;
  for (int C : {2, 4, 8, 16}) {
    if (!col_ok(ny, C) || C > nx) continue;
    Batch bt = make_batch(workspace, Lo, ny, nx, C);
    upload_descs(const_cast<Desc*>(bt.desc), ds, st);
    launch_twiddles(const_cast<float2*>(bt.tw_x), nx, st);
    if (ny != nx) launch_twiddles(const_cast<float2*>(bt.tw_y), ny, st);
    launch_setup(bt, C, batch, 1, st);
    launch_row(bt, def.RPB, batch, false, LK_BIN, ROW_INIT, 0, nullptr, nullptr, st);
    launch_col_prep(bt, C, batch, COL_WGS, 1, st);
    const float ms = time_ms([&] { launch_col(bt, C, batch, COL_WGS, 1, 0, nullptr, nullptr, st); });
    if (ms < best_col) { best_col = ms; best.C = C; }
  }
  for (int R : {1, 2, 4, 8, 16, 32, 64}) {
    if (!rpb_ok(nx, R) || R > ny) continue;
    Batch bt = make_batch(workspace, Lo, ny, nx, best.C);
    const float ms = time_ms([&] { launch_row(bt, R, batch, false, LK_BIN, ROW_ITER, 1, nullptr, nullptr, st); });
    if (ms < best_row) { best_row = ms; best.RPB = R; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g_timing.on = was_on;
  s = check_launch();
  if (s != HG_OK) return s;
  {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    g_tuned[std::make_tuple(ny, nx, batch_class(batch))] = best;
  }
  if (col_tile) *col_tile = best.C;
  if (rows_per_group) *rows_per_group = best.RPB;
  return HG_OK;
}

hg_status hg_set_launch_config(int ny, int nx, int batch, int col_tile, int rows_per_group) {
  g_err[0] = 0;
  hg_status s = check_size(ny, nx);
  if (s != HG_OK) return s;
  if (batch < 1) return fail(HG_ERR_INVALID_ARG, "batch must be >= 1");
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  const auto key = std::make_tuple(ny, nx, batch_class(batch));
  if (col_tile == 0 && rows_per_group == 0) {
    g_tuned.erase(key);
    return HG_OK;
  }
  if (!col_ok(ny, col_tile) || col_tile > nx)
    return fail(HG_ERR_INVALID_ARG, "column tile %d not compiled for ny=%d", col_tile, ny);
  if (!rpb_ok(nx, rows_per_group) || rows_per_group > ny)
    return fail(HG_ERR_INVALID_ARG, "rows per group %d not compiled for nx=%d", rows_per_group, nx);
  g_tuned[key] = Cfg{col_tile, rows_per_group};
  return HG_OK;
}

hg_status hg_get_launch_config(int ny, int nx, int batch, int* col_tile, int* rows_per_group) {
  g_err[0] = 0;
  hg_status s = check_size(ny, nx);
  if (s != HG_OK) return s;
  const Cfg c = get_cfg(ny, nx, std::max(batch, 1));
  if (col_tile) *col_tile = c.C;
  if (rows_per_group) *rows_per_group = c.RPB;
  return HG_OK;
}

}  // extern "C"
