// Kernels of the hologram hot path for gfx950.
//
// One iteration of GS / weighted GS is two passes over the complex64 SLM
// field held in one HBM buffer in natural [y][x] order:
//   column pass: forward column FFT -> replay constraint (+ NMSE partials,
//                weights) -> inverse column FFT, one workgroup per tile of C
//                columns, the whole column resident in registers + LDS;
//   row pass:    inverse row FFT -> SLM projection -> forward row FFT, one
//                group of NX/E threads per row.
// Both passes read and write every pixel exactly once (16 B/px each).  The
// replay plane is centred by modulating the SLM plane with (-1)^(x+y) (the
// DFT shift theorem), folded into the Fresnel chirp for Fresnel holograms,
// so target, weights and replay share the field's natural layout.
#pragma once
#include "hg_device.hpp"

namespace hg {

constexpr int kMaxWaves = 16;
constexpr int kE = 16;  // elements per thread in every transform
// Prepared-target value of a replay pixel outside a problem's region of
// interest (prepared targets are otherwise >= 0 or NaN).
constexpr float kRoiFree = -1.0f;

// Per-problem descriptor (device memory).  Replay-plane arrays are centred.
struct Desc {
  const float* target;        // raw target amplitude [ny][nx]
  uint8_t* levels_out;        // final levels (GS) or [subframes][ny][nx] (OSPR)
  double* nmse_out;           // iters+1 (GS) or subframes (OSPR)
  float2* field_out;          // final SLM field (nullable)
  float2* replay_out;         // final centred replay (nullable)
  float* weights;             // WGS weights: user buffer or workspace
  const uint8_t* init_levels; // nullable
  const float2* init_field;   // nullable
  union {
    float* accum_out;         // OSPR: accumulator out (nullable)
    const uint8_t* roi;       // GS: region of interest [ny][nx] (nonzero = controlled replay pixel; nullable),
                              // read only in batches with any_roi set (a 128-byte descriptor)
  };
  uint64_t seed;
  uint32_t item;              // Philox item
  int L;                      // SLM levels (0 = continuous)
  int mod;                    // 1: amplitude SLM (transmissions k / (L - 1)); 0: phase SLM
  int iters;                  // GS iterations / OSPR subframes
  int user_weights;           // weights came from the caller
  int lt;                     // Liu-Taghizadeh: constrain only the growing centred square
  int lt_r0, lt_dr;           //   of radius lt_r0 + (k-1) lt_dr at iteration k
  float2* r_out;              // one-iteration calls: replay of the start field, before the constraint (nullable)
  float2* g_out;              // one-iteration calls: SLM-plane field before the projection (nullable)
};
static_assert(sizeof(Desc) == 128, "descriptors at a power-of-two stride: two scalar-cache lines each");

// Launch-uniform view of one size class of problems (passed by value).
struct Batch {
  const Desc* desc;
  float2* field;        // [B][ny][nx]
  float* tprep;         // [B][ny][nx] prepared target
  float* wbuf;          // [B][ny][nx] workspace weights (if not user-owned)
  float* accum;         // [B][ny][nx] OSPR accumulator
  const float2* tw_x;   // staged twiddle table for length nx
  const float2* tw_y;   // staged twiddle table for length ny
  const float2* chirp;  // [B][nx + ny]: cx[x] (-1)^x, then cy[y] (-1)^y
  double* part;         // [B][slots][nblk][4] partial sums
  float* invm;          // [B] weighted GS: 1 / m_{k-1} of the current column pass
  int ny, nx;
  int nblk;             // column tiles per problem (= nx / C)
  int slots;            // partial slots per problem
  float fwd_scale;      // 1/sqrt(nx ny)
  int any_lt;           // some problem of the batch has a Liu-Taghizadeh region or a region of interest
  int* status;          // the call's numeric status word: nonzero once a finisher saw non-finite sums
  int dump;             // some problem asks for r_out: the first column pass runs its dumping instantiation
  int f16;              // the field plane holds two binary16 values per element (4 bytes), not complex64
  int row_invm;         // weighted GS: the row pass after column pass k (or the initial one, k = 0) sets
                        // invm of every problem for column pass k + 1 from the weight sums of slot k
  float s16_row, inv16_row;  // 16-bit planes: the row pass stores x s16_row, the column pass loads x inv16_row
  float s16_col, inv16_col;  // the column pass stores x s16_col, the row pass loads x inv16_col
  const float2* tw_y8;  // OSPR columns of 512 with 8 elements per thread: staged twiddles of that plan (else null)
  int any_roi;          // a GS batch in which some problem has a region of interest (Desc::roi is read;
                        // the GS tile kernels run COL_GSR)
  int class_b;          // problems of the whole size class when a call runs it in chunks (kernel choices
                        // follow the class, not the chunk); 0: the launch's own count
};

// 16-bit field storage: one element as two IEEE binary16 values (real in the
// low half), each rounded to nearest even from the value times a power-of-
// two scale (which changes no mantissa); loads undo the scale exactly.
__device__ __forceinline__ uint32_t pack_h2(float2 v, float s) {
  const _Float16 a = (_Float16)(v.x * s), b = (_Float16)(v.y * s);
  return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}
__device__ __forceinline__ float2 unpack_h2(uint32_t w, float inv_s) {
  const _Float16 a = __builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
  const _Float16 b = __builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
  return make_float2((float)a * inv_s, (float)b * inv_s);
}

__device__ __forceinline__ double* part_ptr(const Batch& bt, int b, int slot, int blk) {
  return bt.part + (((size_t)b * bt.slots + slot) * bt.nblk + blk) * 4;
}

// Workspace planes (field, prepared target, weights, OSPR accumulator) are
// stored in 4 x 4 tiles, tile rows in order: element (y, x) of a plane with
// nx columns sits at tix(y, x, nx).  A tile of the field is one 128-byte
// line, so a row pass over 4-row groups and a column pass over 4- or
// 8-column tiles both read and write whole lines.  Caller-owned arrays
// (targets, levels, fields, replays, weights) keep natural [y][x] order.
// (32-bit: a plane has at most 4096^2 elements.)
__host__ __device__ __forceinline__ uint32_t tix(int y, int x, int nx) {
  return (((uint32_t)y >> 2) * ((uint32_t)nx >> 2) + ((uint32_t)x >> 2)) * 16u + (uint32_t)((y & 3) * 4 + (x & 3));
}

// Liu-Taghizadeh: half-width of the target square of iteration k: centred
// replay index (v, u) is inside when max(|v - ny/2|, |u - nx/2|) is at most
// this.  Problems without the region get ny + nx, which no index exceeds.
__device__ __forceinline__ int lt_radius(const Desc& d, int k, int ny, int nx) {
  if (!d.lt) return ny + nx;
  const long long r = (long long)d.lt_r0 + (long long)(k - 1) * d.lt_dr;
  return (int)max(-1LL, min(r, (long long)(ny + nx)));
}

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2).
// Give each XCD a contiguous run of column tiles so neighbouring tiles, which
// share 128-byte lines when a tile is narrower than 16 columns, meet in the
// same L2.
__device__ __forceinline__ int xcd_tile(int bx, int nb) {
  return (nb & 7) ? bx : (bx & 7) * (nb >> 3) + (bx >> 3);
}

// ---------------------------------------------------------------------------
// LDS exchange policies (padded element index e, see lds_pad)
// ---------------------------------------------------------------------------
// Ordering point for LDS traffic of a single wave: a wave's LDS operations
// execute in program order, so only the compiler must be kept from moving
// them across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row transforms: private LDS region per row.  A row held by one wave
// (T <= 64 threads) exchanges through one buffer with wave-level ordering
// only; a row spread over several waves uses ping-pong buffers and one
// workgroup barrier per exchange.
// Values that are the same for the whole workgroup (descriptor fields read
// at a uniform address) moved into scalar registers, so that branches on
// them stay scalar branches.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
template <class T> __device__ __forceinline__ T* uni_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// Row exchange buffers.  A row inside one wave needs only wave-level LDS
// ordering.  A row spread over several waves uses two buffers (PP: one
// barrier per exchange) or, where LDS is short, one buffer with a barrier
// before the writes and another before the reads.
template <bool WAVE, bool PP = true> struct RowEx {
  float2* b[2];
  int w, rd;
  __device__ void before_read() {
    if constexpr (WAVE) {
      wave_lds_sync();
    } else {
      __syncthreads();
      if constexpr (PP) {
        rd = w;
        w ^= 1;
      }
    }
  }
  __device__ void before_write() {
    if constexpr (WAVE) wave_lds_sync();
    else if constexpr (!PP) __syncthreads();
  }
  __device__ float2 ld(int e) const { return (WAVE || !PP) ? b[0][e] : b[rd][e]; }
  __device__ void st(int e, float2 v) {
    if constexpr (WAVE || !PP) b[0][e] = v;
    else b[w][e] = v;
  }
};

// Column tile: C interleaved columns, element (e, c) at e * C + c.  With two
// tile buffers (PP) each exchange needs one barrier; with one, a barrier
// before the reads and another before the writes.
template <int C, bool PP> struct ColEx {
  float2* s;  // tile base + c
  int w = 0, rd = 0;
  int stride;                     // elements between the two buffers
  __device__ void before_read() {
    __syncthreads();
    if constexpr (PP) { rd = w; w ^= 1; }
  }
  __device__ void before_write() {
    if constexpr (!PP) __syncthreads();
  }
  __device__ float2 ld(int e) const { return PP ? s[rd * stride + e * C] : s[e * C]; }
  __device__ void st(int e, float2 v) {
    if constexpr (PP) s[w * stride + e * C] = v;
    else s[e * C] = v;
  }
};

// Two column tiles fit in LDS (with room for the reductions) when small enough.
// (Measured: a second buffer costs more occupancy than the barrier it saves,
// so it is off for every compiled tile.)
__host__ __device__ constexpr bool col_pingpong(int NY, int C) { return false && 2 * (NY + NY / 16) * C * 8 <= 150 * 1024; }

// ---------------------------------------------------------------------------
// deterministic block reductions into FP64
// ---------------------------------------------------------------------------
// One DPP move of a double (two 32-bit halves); lanes the control does not
// write, or whose source is out of range, read +0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xf, true);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over the wave's 64 lanes in a fixed order, returned to every lane:
// within quads (quad_perm 1,0,3,2 and 2,3,0,1), within rows of 16 (half-row
// and row mirrors), then rows 0+1 and 2+3 (row_bcast:15 into rows 1 and 3)
// and the two halves (row_bcast:31 into rows 2 and 3); lane 63 then holds
// the total.  Cross-lane moves by DPP, no LDS traffic.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);        // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);        // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);       // row_half_mirror
  v += dpp_f64<0x140>(v);       // row_mirror
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15, rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31, rows 2 and 3
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sums of four per-thread float values over the block, in a fixed order;
// results in tot[0..3] (valid for every thread on return).
template <int NT>
__device__ __forceinline__ void block_sum4(float a0, float a1, float a2, float a3, double (&red)[kMaxWaves][4],
                                           double (&tot)[4]) {
  constexpr int NW = (NT + 63) / 64;
  const double d0 = wave_sum((double)a0), d1 = wave_sum((double)a1);
  const double d2 = wave_sum((double)a2), d3 = wave_sum((double)a3);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { red[wv][0] = d0; red[wv][1] = d1; red[wv][2] = d2; red[wv][3] = d3; }
  __syncthreads();
  if (threadIdx.x < 4) {
    double acc = 0.0;
    for (int w = 0; w < NW; ++w) acc += red[w][threadIdx.x];
    tot[threadIdx.x] = acc;
  }
  __syncthreads();
}

// Sum field `f` of slot `slot` over all nblk tiles of problem b, in a fixed
// order (every block computes the identical value).
__device__ __forceinline__ double slot_total(const Batch& bt, int b, int slot, int f, double* bcast) {
  __syncthreads();
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int i = threadIdx.x; i < bt.nblk; i += 64) s += part_ptr(bt, b, slot, i)[f];
    s = wave_sum(s);
    if (threadIdx.x == 0) *bcast = s;
  }
  __syncthreads();
  return *bcast;
}

// Weighted GS: 1 / m of problem b, m the mean weight on the support, from the
// weight sums in slot k (the support size in the set-up slot), computed by
// one wave in slot_total's fixed order.
__device__ __forceinline__ void wgs_invm_wave(const Batch& bt, int b, int k) {
  const int lane = threadIdx.x & 63;
  double om = 0.0, ws = 0.0;
  for (int i = lane; i < bt.nblk; i += 64) {
    om += part_ptr(bt, b, bt.slots - 1, i)[1];
    ws += part_ptr(bt, b, k, i)[3];
  }
  om = wave_sum(om);
  ws = wave_sum(ws);
  if (lane == 0) bt.invm[b] = (float)((om > 0.0 ? om : 1.0) / ws);
}

// ---------------------------------------------------------------------------
// table kernels (FP64 arithmetic, stored as complex64)
// ---------------------------------------------------------------------------
// Staged twiddles of a length-N transform: stage s, butterfly class k,
// r = 1..R-1 -> exp(-2 pi i r k / (p R)).  Stages are walked at compile time.
template <int N, int S, int E = kE>
__device__ __forceinline__ void twiddle_entry(float2* tw, int m) {
  using P = Plan<N, E>;
  if constexpr (S < P::ns) {
    constexpr int R = P::radix(S), p = P::stride(S);
    constexpr int off = TwLayout<N, E>::twoff(S), sz = TwLayout<N, E>::size_of(S);
    if (m >= off && m < off + sz) {
      const int k = (m - off) / (R - 1), r = (m - off) % (R - 1) + 1;
      double sn, cs;
      sincospi(2.0 * (double)(r * k) / (double)(p * R), &sn, &cs);
      tw[m] = make_float2((float)cs, (float)-sn);
      return;
    }
    twiddle_entry<N, S + 1, E>(tw, m);
  }
}

template <int N, int E = kE>
__global__ void k_twiddles(float2* tw) {
  constexpr int total = TwLayout<N, E>::total();
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= total) return;
  twiddle_entry<N, 1, E>(tw, m);
}

// cx[x] = exp(i pi p^2 (x - nx/2)^2 / (lambda z)) (-1)^x, then cy likewise.
// a = p^2 / (lambda z) (0 for Fourier); phase in half-turns = a d^2, reduced
// exactly mod 2 before the FP64 sincospi.
struct ChirpArgs { double a[32]; int count; };
static __global__ void k_chirps(float2* chirp, int ny, int nx, ChirpArgs ca, int first) {
  const int b = blockIdx.y;
  if (b >= ca.count) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx + ny) return;
  const bool isx = i < nx;
  const int q = isx ? i : i - nx;
  const int n = isx ? nx : ny;
  const double d = (double)(q - n / 2);
  double ht = fmod(ca.a[b] * d * d, 2.0);
  if (q & 1) ht += 1.0;
  double s, c;
  sincospi(ht, &s, &c);
  chirp[(size_t)(first + b) * (nx + ny) + i] = make_float2((float)c, (float)s);
}

// The phase field of stream (seed, item, tag): axis 1 = row lines, 0 = column lines.
static __global__ void k_random_phase(float2* out, uint64_t seed, uint32_t item, uint32_t tag, int ny, int nx, int axis) {
  const int n = axis ? nx : ny, nl = axis ? ny : nx, q = n / 4;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= q * nl) return;
  const int i = id % q, l = id / q;
  const U64x4 o = philox_line_block(seed, item, tag, (uint32_t)i, (uint32_t)l);
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int e = i + w * q;
    const size_t idx = axis ? (size_t)l * nx + e : (size_t)e * nx + l;
    out[idx] = philox_phasor(u64x4_word(o, w));
  }
}

// ---------------------------------------------------------------------------
// set-up: target energy, prepared target, weights.  These share the column
// pass's tiling so their partials line up with its slots.
// ---------------------------------------------------------------------------
template <int NY, int C>
__global__ __launch_bounds__(C * (NY / kE)) void k_energy(Batch bt) {
  constexpr int T = NY / kE, NT = C * T;
  __shared__ double red[kMaxWaves][4];
  __shared__ double tot[4];
  const int b = blockIdx.y, blk = xcd_tile(blockIdx.x, gridDim.x);
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int u = blk * C + c;
  gptr<const float> tg = to_global(uni_ptr(bt.desc[b].target));
  const uint8_t* roi = bt.any_roi ? uni_ptr(bt.desc[b].roi) : nullptr;
  // loads first (straight-line), then the sum
  float v[kE];
#pragma unroll
  for (int j = 0; j < kE; ++j) v[j] = tg[(size_t)(t + T * j) * bt.nx + u];
  if (roi) {  // the target outside the region is ignored
    gptr<const uint8_t> rg = to_global(roi);
    uint32_t m[kE];
#pragma unroll
    for (int j = 0; j < kE; ++j) m[j] = rg[(size_t)(t + T * j) * bt.nx + u];
#pragma unroll
    for (int j = 0; j < kE; ++j) v[j] = m[j] ? v[j] : 0.f;
  }
  float e = 0.0f;
#pragma unroll
  for (int j = 0; j < kE; ++j) e += v[j] * v[j];
  block_sum4<NT>(e, 0.f, 0.f, 0.f, red, tot);
  if (threadIdx.x == 0) part_ptr(bt, b, bt.slots - 1, blk)[0] = tot[0];
}

template <int NY, int C>
__global__ __launch_bounds__(C * (NY / kE)) void k_prepare(Batch bt, int weighted) {
  constexpr int T = NY / kE, NT = C * T;
  __shared__ double red[kMaxWaves][4];
  __shared__ double tot[4];
  __shared__ double bc;
  const int b = blockIdx.y, blk = xcd_tile(blockIdx.x, gridDim.x);
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int u = blk * C + c;
  const Desc& d = bt.desc[b];
  const double e = slot_total(bt, b, bt.slots - 1, 0, &bc);
  const float scale = (float)sqrt((double)bt.nx * (double)bt.ny / e);
  const size_t off = (size_t)b * bt.ny * bt.nx;
  float* w = bt.wbuf + off;  // caller's weights are copied in here
  float om = 0.f, ws = 0.f;
  int rlo = NY, rhi = -1;  // this thread's first and last support row
  __shared__ int srow[2];  // the tile's (LDS atomics)
  if (threadIdx.x == 0) { srow[0] = NY; srow[1] = -1; }
  const int um = (bt.nx - u) & (bt.nx - 1);
  // the problem's choices: binary phase or amplitude SLM (centro-symmetric
  // replay: symmetrised target), region of interest, caller weights
  const bool sym = uni(d.L) == 2 || uni(d.mod);
  const uint8_t* roi = bt.any_roi ? uni_ptr(d.roi) : nullptr;
  const bool uw = weighted && uni(d.user_weights);
  gptr<const float> tg = to_global(uni_ptr(d.target));
  // Every load first, in straight-line code, so that all of them are in
  // flight together (with the element branches inside the loop below, each
  // element's load was waited for alone).
  float tv[kE], tm[kE], wv[kE];
  uint32_t cv[kE], cmv[kE];  // mask bytes of the pixel and of its mirror image
#pragma unroll
  for (int j = 0; j < kE; ++j) {
    tv[j] = tg[(size_t)(t + T * j) * bt.nx + u];
    tm[j] = 0.f;
    cv[j] = cmv[j] = 1u;
    wv[j] = 1.0f;
  }
  if (sym) {
#pragma unroll
    for (int j = 0; j < kE; ++j) tm[j] = tg[(size_t)((bt.ny - (t + T * j)) & (bt.ny - 1)) * bt.nx + um];
  }
  if (roi) {
    gptr<const uint8_t> rg = to_global(roi);
#pragma unroll
    for (int j = 0; j < kE; ++j) {
      cv[j] = rg[(size_t)(t + T * j) * bt.nx + u];
      cmv[j] = rg[(size_t)((bt.ny - (t + T * j)) & (bt.ny - 1)) * bt.nx + um];
    }
  }
  if (uw) {
    gptr<const float> wg = to_global(uni_ptr(d.weights));
#pragma unroll
    for (int j = 0; j < kE; ++j) wv[j] = wg[(size_t)(t + T * j) * bt.nx + u];
  }
#pragma unroll
  for (int j = 0; j < kE; ++j) {
    const int v = t + T * j;
    // region of interest: the target outside it is ignored, and a pixel
    // outside the controlled region (the region, with its mirror image for a
    // centro-symmetric replay) is marked by a negative prepared target: the
    // GS column passes leave it free and out of the NMSE
    float a = tv[j];
    bool ctl = true;
    if (roi) {
      ctl = cv[j] != 0u;
      a = ctl ? a : 0.f;
    }
    if (sym) {
      float m = tm[j];
      if (roi) {
        const bool cm = cmv[j] != 0u;
        m = cm ? m : 0.f;
        ctl = ctl || cm;
      }
      a = sqrtf(0.5f * (a * a + m * m));
    }
    a *= scale;
    if (!ctl) a = kRoiFree;
    const uint32_t ti = tix(v, u, bt.nx);
    // a non-finite caller weight poisons its pixel's target, so the NMSE
    // turns NaN as for a non-finite target
    if (!__builtin_isfinite(wv[j])) a = __builtin_nanf("");
    bt.tprep[off + ti] = a;
    // support: every pixel whose target is not exactly zero (a NaN or
    // negative value counts, so the column passes read it and the NMSE
    // turns non-finite as it does in every kernel)
    const bool sup = !(a == 0.f);
    if (weighted) {
      w[ti] = wv[j];
      if (sup) ws += wv[j];
    }
    if (sup) { om += 1.f; rlo = min(rlo, v); rhi = max(rhi, v); }
  }
  // slot slots-1 field 1: |Omega| of the tile, fields 2 and 3: its first and
  // last support row (the column passes read no target or weights outside
  // them); weighted: slot 0 field 3, the sum of w_0 over Omega
  __syncthreads();  // srow initialised
  atomicMin(&srow[0], rlo);
  atomicMax(&srow[1], rhi);
  block_sum4<NT>(om, ws, 0.f, 0.f, red, tot);
  __syncthreads();  // every thread's rows are in
  if (threadIdx.x == 0) {
    double* pp = part_ptr(bt, b, bt.slots - 1, blk);
    pp[1] = tot[0];
    pp[2] = (double)srow[0];
    pp[3] = (double)srow[1];
    if (weighted) part_ptr(bt, b, 0, blk)[3] = tot[1];
  }
}

// ---------------------------------------------------------------------------
// row pass
// ---------------------------------------------------------------------------
enum RowMode { ROW_INIT = 0, ROW_ITER = 1, ROW_OSPR = 2, ROW_PROP_FWD = 3, ROW_PROP_BWD = 4 };
// LK_BIN: every problem of the launch is binary phase (L = 2); LK_QUAD: every
// problem is 4- or 8-level phase (quadrant decision, no arctangent).  A
// launch-wide kind keeps the other projections' code, and its registers,
// out of the kernel.
enum LevelKind { LK_ANY = 0, LK_BIN = 1, LK_QUAD = 2 };

// Modulation m[y][x] applied before the forward row FFT and conjugated after
// the inverse one: (-1)^(x+y) for Fourier, chirp * (-1)^(x+y) for Fresnel
// (the sign is folded into the chirp tables).  Built once per element.
template <bool FRESNEL> struct Mod {
  float2 m;  // Fresnel: the chirp product; Fourier: (+-1, 0)
  __device__ __forceinline__ Mod(int x, int y, gptr<const float2> cx, float2 cyv) {
    if constexpr (FRESNEL) m = cmul(cx[x], cyv);
    else m = make_float2(((x + y) & 1) ? -1.0f : 1.0f, 0.0f);
  }
  __device__ __forceinline__ float2 fwd(float2 v) const {
    if constexpr (FRESNEL) return cmul(v, m);
    else return make_float2(v.x * m.x, v.y * m.x);
  }
  __device__ __forceinline__ float2 inv(float2 v) const {
    if constexpr (FRESNEL) return cmulc(v, m);
    else return make_float2(v.x * m.x, v.y * m.x);
  }
};

// Row groups of 4 rows (one row of 4 x 4 field tiles, NX / 4 tiles of 128
// contiguous bytes) move between HBM and the rows' LDS buffers with
// 16-byte accesses by the whole workgroup: chunk c holds elements
// x = 4 (c >> 3) + 2 (c & 1) + {0, 1} of row (c & 7) >> 1.  Staged rows are
// unpadded (element x at x), so each chunk is one aligned 16-byte LDS access
// and a row's chunks are contiguous.
template <int NX, int NT, int LW>
__device__ __forceinline__ void quad_to_lds(gptr<const float2> q, float2* lds) {
  constexpr int NCH = NX * 4 * 8 / 16;
  static_assert(LW % 2 == 0, "16-byte aligned rows");
#pragma unroll
  for (int m = 0; m < NCH / NT; ++m) {
    const int c = threadIdx.x + NT * m;
    const float4 val = reinterpret_cast<gptr<const float4>>(q)[c];
    const int rr = (c & 7) >> 1, x = 4 * (c >> 3) + 2 * (c & 1);
    *reinterpret_cast<float4*>(lds + rr * LW + x) = val;
  }
}
template <int NX, int NT, int LW>
__device__ __forceinline__ void lds_to_quad(const float2* lds, gptr<float2> q) {
  constexpr int NCH = NX * 4 * 8 / 16;
#pragma unroll
  for (int m = 0; m < NCH / NT; ++m) {
    const int c = threadIdx.x + NT * m;
    const int rr = (c & 7) >> 1, x = 4 * (c >> 3) + 2 * (c & 1);
    reinterpret_cast<gptr<float4>>(q)[c] = *reinterpret_cast<const float4*>(lds + rr * LW + x);
  }
}

// 16-bit planes: a 4 x 4 tile is 64 contiguous bytes, so chunk c (16 bytes)
// of a 4-row group holds the elements x = 4 (c >> 2) .. 4 (c >> 2) + 3 of
// row c & 3.  Staged rows stay float2 in LDS.
template <int NX, int NT, int LW>
__device__ __forceinline__ void quad16_to_lds(gptr<const uint32_t> q, float2* lds, float inv_s) {
  constexpr int NCH = NX;  // 4 rows x NX elements x 4 bytes / 16
  static_assert(LW % 2 == 0, "16-byte aligned rows");
#pragma unroll
  for (int m = 0; m < NCH / NT; ++m) {
    const int c = threadIdx.x + NT * m;
    const uint4 w = reinterpret_cast<gptr<const uint4>>(q)[c];
    const int rr = c & 3, x = 4 * (c >> 2);
    const float2 e0 = unpack_h2(w.x, inv_s), e1 = unpack_h2(w.y, inv_s);
    const float2 e2 = unpack_h2(w.z, inv_s), e3 = unpack_h2(w.w, inv_s);
    *reinterpret_cast<float4*>(lds + rr * LW + x) = make_float4(e0.x, e0.y, e1.x, e1.y);
    *reinterpret_cast<float4*>(lds + rr * LW + x + 2) = make_float4(e2.x, e2.y, e3.x, e3.y);
  }
}
template <int NX, int NT, int LW>
__device__ __forceinline__ void lds_to_quad16(const float2* lds, gptr<uint32_t> q, float s) {
  constexpr int NCH = NX;
#pragma unroll
  for (int m = 0; m < NCH / NT; ++m) {
    const int c = threadIdx.x + NT * m;
    const int rr = c & 3, x = 4 * (c >> 2);
    const float4 a = *reinterpret_cast<const float4*>(lds + rr * LW + x);
    const float4 b = *reinterpret_cast<const float4*>(lds + rr * LW + x + 2);
    uint4 w;
    w.x = pack_h2(make_float2(a.x, a.y), s);
    w.y = pack_h2(make_float2(a.z, a.w), s);
    w.z = pack_h2(make_float2(b.x, b.y), s);
    w.w = pack_h2(make_float2(b.z, b.w), s);
    reinterpret_cast<gptr<uint4>>(q)[c] = w;
  }
}

// MODE  ROW_INIT: build f0 (Philox, levels or field), forward FFT.
//       ROW_ITER: inverse FFT, project, forward FFT (iteration k = arg).
//       ROW_OSPR: as ROW_ITER with L = 2, writing subframe arg's levels.
//       ROW_PROP_FWD / _BWD: scaled propagation between pin and pout.
// Waves per SIMD asked of the compiler for the staged 4-row groups: within
// 128 registers per lane, two 512-thread workgroups of 2048-wide rows (or
// four 256-thread ones of 1024-wide rows) share a CU.  (Fresnel rows with a
// general level set spill a little under this cap, and still run faster than
// with one workgroup fewer per CU.)
template <int NX, int RPB> constexpr int row_min_waves() { return ((NX == 2048 || NX == 1024) && RPB == 4) ? 4 : 1; }

// F16: the field plane holds 16-bit elements (Batch::f16); ROW_INIT and
// ROW_ITER only.
// EE: elements per thread (16; 8 for the small-batch OSPR rows of 512, whose
// twiddles are then that plan's table).
template <int NX, int RPB, bool FRESNEL, int MODE, int LK, bool F16 = false, int EE = kE>
__global__ __launch_bounds__(RPB * (NX / EE), (row_min_waves<NX, RPB>())) void k_row(Batch bt, int arg,
                                                                                     const float2* pin, float2* pout) {
  static_assert(!F16 || MODE == ROW_INIT || MODE == ROW_ITER, "16-bit planes in GS / weighted GS only");
  constexpr int E = EE;
  using P = Plan<NX, E>;
  constexpr int T = P::T;
  constexpr bool XCH = P::ns > 1;
  constexpr bool WAVE = T <= 64;  // each row inside one wave
  static_assert(T % 4 == 0, "a thread's elements share one column of the 4 x 4 tiles");
  // one 4-row group per workgroup: stage the group's tiles through the rows'
  // LDS buffers for whole-line 16-byte accesses (rows of several waves then
  // exchange through one buffer each)
  constexpr bool STAGE = XCH && RPB == 4;
  // row buffer pitch; staged rows are offset by 4 elements (32 bytes) so
  // that the four rows of a group, which the staging's 16-byte accesses
  // interleave, start 8 banks apart and eight lanes fill the 32 banks once
  constexpr int LW = NX + NX / 16 + (STAGE ? 4 : 0);
  constexpr bool PP = !WAVE && !STAGE;
  constexpr int NBUF = PP ? 2 : 1;
  __shared__ __align__(16) float2 lds[XCH ? RPB * NBUF * LW : 1];
  // phasors of the problem's levels (general L, projection only)
  constexpr bool TAB = (MODE == ROW_ITER && (LK == LK_ANY || LK == LK_QUAD));
  __shared__ float2 lvl[TAB ? 256 : 1];
  const int b = blockIdx.y;
  // weighted GS: the next column pass's 1 / m of every problem, by the first
  // wave of the first workgroups dispatched (they have the whole launch to
  // finish it; the weight sums were complete before this launch began)
  if constexpr (MODE == ROW_INIT || MODE == ROW_ITER) {
    if (bt.row_invm && b == 0 && threadIdx.x < 64) {
      for (int p = blockIdx.x; p < (int)gridDim.y; p += (int)gridDim.x)
        wgs_invm_wave(bt, p, MODE == ROW_INIT ? 0 : arg);
    }
  }
  const int r = threadIdx.x / T, t = threadIdx.x % T;
  const int y = blockIdx.x * RPB + r;
  const size_t off = (size_t)b * bt.ny * NX;
  // this row's elements in the tiled field: x at row[(x >> 2) * 16 + (x & 3)]
  gptr<float2> row = to_global(bt.field + off + (size_t)(y >> 2) * (NX >> 2) * 16 + (y & 3) * 4);
  gptr<float2> quad = to_global(bt.field + off + (size_t)(y >> 2) * (NX >> 2) * 16);  // the group's tiles
  // the same element offsets in a 16-bit plane (4 bytes per element)
  gptr<uint32_t> row16 = to_global(reinterpret_cast<uint32_t*>(bt.field) + off + (size_t)(y >> 2) * (NX >> 2) * 16 +
                                   (y & 3) * 4);
  gptr<uint32_t> quad16 = to_global(reinterpret_cast<uint32_t*>(bt.field) + off + (size_t)(y >> 2) * (NX >> 2) * 16);
  gptr<const float2> cx = to_global(static_cast<const float2*>(bt.chirp)) + (size_t)b * (NX + bt.ny);
  const float2 cyv = FRESNEL ? static_cast<float2>(cx[NX + y]) : make_float2(1.f, 0.f);
  RowEx<WAVE, PP> ex;
  ex.b[0] = lds + (XCH ? r * NBUF * LW : 0);
  ex.b[1] = ex.b[0] + (XCH && !WAVE ? LW : 0);
  ex.w = 0;
  ex.rd = 0;
  float2 v[E];

  if constexpr (MODE == ROW_PROP_FWD || MODE == ROW_PROP_BWD) {
    gptr<const float2> src = to_global(pin + off + (size_t)y * NX);
    gptr<float2> dst = to_global(pout + off + (size_t)y * NX);
    const float s = rsqrtf((float)NX);
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = src[t + T * j];
    if constexpr (MODE == ROW_PROP_FWD) {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = cscale(Mod<FRESNEL>(t + T * j, y, cx, cyv).fwd(v[j]), s);
      fft<NX, E, -1>(v, t, bt.tw_x, ex);
    } else {
      fft<NX, E, +1>(v, t, bt.tw_x, ex);
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = cscale(Mod<FRESNEL>(t + T * j, y, cx, cyv).inv(v[j]), s);
    }
#pragma unroll
    for (int j = 0; j < E; ++j) dst[t + T * j] = v[j];
  } else {
    const Desc& d = bt.desc[b];
    if constexpr (MODE == ROW_INIT) {
      if (d.init_field || d.init_levels) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const size_t idx = (size_t)y * NX + t + T * j;
          v[j] = d.init_field ? d.init_field[idx]
                 : d.mod ? make_float2(amp_value(d.init_levels[idx], d.L), 0.f)
                         : level_phasor(d.init_levels[idx], d.L);
        }
      } else {
        // initial phase: Philox words over row lines; element j = g + (E/4) w
#pragma unroll
        for (int g = 0; g < E / 4; ++g) {
          const U64x4 o = philox_line_block(d.seed, d.item, 1u, (uint32_t)(t + T * g), (uint32_t)y);
#pragma unroll
          for (int w = 0; w < 4; ++w) v[g + (E / 4) * w] = philox_phasor(u64x4_word(o, w));
        }
      }
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = Mod<FRESNEL>(t + T * j, y, cx, cyv).fwd(v[j]);
    } else {
      const int iters = uni(d.iters);
      if (MODE == ROW_ITER && arg > iters) return;  // uniform per block
      const int L = (MODE == ROW_OSPR || LK == LK_BIN) ? 2 : uni(d.L);
      const bool amp = (MODE == ROW_ITER && LK == LK_ANY) && uni(d.mod);  // amplitude SLM
      const float amp_s = bt.fwd_scale * (float)(L - 1);  // unitary scale times L - 1
      const bool last = (MODE == ROW_OSPR) || (arg == iters);
      gptr<uint8_t> lev = to_global(uni_ptr(d.levels_out));
      gptr<float2> fout = to_global(uni_ptr(d.field_out));
      gptr<float2> gdump = to_global(uni_ptr(d.g_out));
      if (MODE == ROW_OSPR) lev += (size_t)(arg - 1) * bt.ny * NX;
      if constexpr (TAB) {
        if (L > 2 && !amp) {  // uniform per block
          for (int i = threadIdx.x; i < L; i += RPB * T) lvl[i] = level_phasor(i, L);
          __syncthreads();
        }
      }
      if constexpr (STAGE) {
        if constexpr (F16) quad16_to_lds<NX, RPB * T, LW>(quad16, lds, bt.inv16_col);
        else quad_to_lds<NX, RPB * T, LW>(quad, lds);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = ex.b[0][t + T * j];  // unpadded staging order
      } else if constexpr (F16) {
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = unpack_h2(row16[((t + T * j) >> 2) * 16 + (t & 3)], bt.inv16_col);
      } else {
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = row[((t + T * j) >> 2) * 16 + (t & 3)];
      }
      fft<NX, E, +1>(v, t, bt.tw_x, ex);
      // projection onto the SLM set, one code path per kind of level set
      // (uniform per block: 0 continuous, 2 binary, 4 four or eight levels,
      // 3 any other L) and per iteration kind (only the last writes levels
      // and the field)
      auto project = [&](auto kind, auto wr) {
        constexpr int KIND = decltype(kind)::value;
        constexpr bool WR = decltype(wr)::value;
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const int x = t + T * j;
          const Mod<FRESNEL> md(x, y, cx, cyv);
          const float2 g = md.inv(v[j]);
          float2 f;
          if constexpr (KIND == 0) {
            f = unit_phase(g);
          } else if constexpr (KIND == 5) {  // amplitude SLM: nearest transmission to Re g
            const int k = amp_level(g.x, amp_s, L);
            f = make_float2(amp_value(k, L), 0.f);
            if constexpr (WR) {
              if (lev) lev[(size_t)y * NX + x] = (uint8_t)k;
            }
          } else {
            const int k = KIND == 4 ? level_index_quad(g, L) : level_index(g, KIND == 2 ? 2 : L);
            if constexpr (KIND == 2) f = level_phasor(k, 2);
            else f = lvl[k];
            if constexpr (WR) {
              if (lev) lev[(size_t)y * NX + x] = (uint8_t)k;
            }
          }
          if constexpr (WR && MODE == ROW_ITER) {
            if (fout) fout[(size_t)y * NX + x] = f;
            if (gdump) gdump[(size_t)y * NX + x] = cscale(g, bt.fwd_scale);  // unitary backward
          }
          v[j] = md.fwd(f);
        }
      };
      auto by_kind = [&](auto wr) {
        if constexpr (LK == LK_QUAD) {
          project(std::integral_constant<int, 4>{}, wr);  // every problem 4 or 8 levels
        } else if constexpr (TAB) {
          if (amp) project(std::integral_constant<int, 5>{}, wr);
          else if (L == 2) project(std::integral_constant<int, 2>{}, wr);
          else if (L == 0) project(std::integral_constant<int, 0>{}, wr);
          else if (L == 4 || L == 8) project(std::integral_constant<int, 4>{}, wr);
          else project(std::integral_constant<int, 3>{}, wr);
        } else {
          project(std::integral_constant<int, 2>{}, wr);  // every problem binary
        }
      };
      if (last) by_kind(std::true_type{});
      else by_kind(std::false_type{});
    }
    fft<NX, E, -1>(v, t, bt.tw_x, ex);
    if constexpr (STAGE) {
      // the transform's reads of the row buffers are done (this wave's, or
      // the whole block's when a row spans several waves)
      if constexpr (WAVE) wave_lds_sync();
      else __syncthreads();
#pragma unroll
      for (int j = 0; j < E; ++j) ex.b[0][t + T * j] = v[j];  // unpadded staging order
      __syncthreads();
      if constexpr (F16) lds_to_quad16<NX, RPB * T, LW>(lds, quad16, bt.s16_row);
      else lds_to_quad<NX, RPB * T, LW>(lds, quad);
    } else if constexpr (F16) {
#pragma unroll
      for (int j = 0; j < E; ++j) row16[((t + T * j) >> 2) * 16 + (t & 3)] = pack_h2(v[j], bt.s16_row);
    } else {
#pragma unroll
      for (int j = 0; j < E; ++j) row[((t + T * j) >> 2) * 16 + (t & 3)] = v[j];
    }
  }
}

// ---------------------------------------------------------------------------
// column pass
// ---------------------------------------------------------------------------
enum ColMode {
  COL_GS = 0,          // iteration k = arg: partials for nmse[k-1], R' = T R/|R|
  COL_WGS = 1,         // as COL_GS with the weight update
  COL_GSR = 2,         // as COL_GS, in the tile kernels of a size class that holds a region of interest:
                       // pixels outside a region keep R and stay out of the NMSE sums
  COL_OSPR_FIRST = 3,  // T e^{i phi_1} -> inverse FFT
  COL_OSPR = 4,        // subframe arg >= 2: finish subframe arg-1, start arg
  COL_OSPR_FINAL = 5,  // finish the last subframe
  COL_FINAL = 8,       // GS/WGS pass K + 1: NMSE partials of the final field, replay out
  COL_PROP_FWD = 6,
  COL_PROP_BWD = 7
};

// weighted GS: amplitude floor (unit-rms units), leak exponent, clamp
constexpr float kWgsEps = 0.1f, kWgsGamma = 0.7f, kWMin = 1e-6f, kWMax = 1e6f;

// Weight clamp to [kWMin, kWMax] that keeps a NaN (fminf/fmaxf would replace
// it by a bound and so hide a non-finite caller weight from the finisher).
__device__ __forceinline__ float clamp_w(float x) {
  return x < kWMin ? kWMin : (x > kWMax ? kWMax : x);
}

// LT: the GS pass also applies Liu-Taghizadeh regions and regions of
// interest, and the final pass leaves pixels outside a region of interest out
// of its sums (separate instantiations, so that plain GS does not carry the
// tests' registers and its final pass sums exactly as the iterations do).
// DUMP: GS / WGS pass that also writes each problem's replay before the
// constraint to its r_out (one-iteration calls only; a separate instantiation).
template <int NY, int C, int MODE, bool LT = false, bool DUMP = false>
__global__ __launch_bounds__(C * (NY / kE)) void k_col(Batch bt, int arg, int adaptive, const float2* pin,
                                                       float2* pout) {
  constexpr int E = kE;
  using P = Plan<NY, E>;
  constexpr int T = P::T, NT = C * T;
  constexpr bool PP = col_pingpong(NY, C);
  constexpr int TILE = (NY + NY / 16) * C;
  __shared__ float2 lds[(PP ? 2 : 1) * TILE];
  __shared__ double red[kMaxWaves][4];
  __shared__ double tot[4];
  __shared__ double bc;
  const int b = blockIdx.y, blk = xcd_tile(blockIdx.x, gridDim.x);
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int u = blk * C + c;
  const int NX = bt.nx;
  const size_t off = (size_t)b * NY * NX;
  gptr<float2> fld = to_global(bt.field + off);
  ColEx<C, PP> ex;
  ex.s = lds + c;
  ex.stride = TILE;
  float2 v[E];

  if constexpr (MODE == COL_PROP_FWD || MODE == COL_PROP_BWD) {
    gptr<const float2> src = to_global(pin + off);
    gptr<float2> dst = to_global(pout + off);
    const float s = rsqrtf((float)NY);
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = src[(size_t)(t + T * j) * NX + u];
    if constexpr (MODE == COL_PROP_FWD) fft<NY, E, -1>(v, t, bt.tw_y, ex);
    else fft<NY, E, +1>(v, t, bt.tw_y, ex);
#pragma unroll
    for (int j = 0; j < E; ++j) dst[(size_t)(t + T * j) * NX + u] = cscale(v[j], s);
  } else if constexpr (MODE == COL_GS || MODE == COL_WGS || MODE == COL_FINAL) {
    const Desc& d = bt.desc[b];
    gptr<const float> tp = to_global(bt.tprep + off);
    // column pass k of a problem with K iterations: k <= K iterates (GS/WGS
    // launches), k = K + 1 only measures the final field (FINAL launch); a
    // problem whose K does not match the launch is idle in it.
    const int k = arg;
    if constexpr (MODE == COL_FINAL) {
      if (k != d.iters + 1) return;  // uniform per block
    } else {
      if (k > d.iters) return;
    }
    float inv_m = 1.0f;
    gptr<float> w = nullptr;
    if constexpr (MODE == COL_WGS) {
      const double om = slot_total(bt, b, bt.slots - 1, 1, &bc);
      const double wsum = slot_total(bt, b, k - 1, 3, &bc);
      inv_m = (float)((om > 0.0 ? om : 1.0) / wsum);
      w = to_global(bt.wbuf + off);
    }
    const int ltr = LT ? uni(lt_radius(d, k, NY, NX)) : 0;
    // amplitude SLM: the zero order (row NY/2 = element E/2 of t = 0, column
    // nx/2) keeps R and stays out of the NMSE sums
    static_assert(T * (E / 2) == NY / 2, "the zero order is element E/2 of thread row 0");
    const bool zo = d.mod && t == 0 && u == (NX >> 1);
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = fld[tix(t + T * j, u, NX)];
    fft<NY, E, -1>(v, t, bt.tw_y, ex);
    float s_ta = 0.f, s_aa = 0.f, s_tt = 0.f, s_w = 0.f;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const size_t idx = (size_t)(t + T * j) * NX + u;  // caller arrays
      const uint32_t ti = tix(t + T * j, u, NX);            // workspace planes
      const float2 Rr = v[j];  // unscaled replay, centred index (t + T j, u)
      const float a2 = Rr.x * Rr.x + Rr.y * Rr.y;
      const float inv = a2 > 0.f ? __builtin_amdgcn_rsqf(a2) : 0.f;
      const float A = a2 * inv * bt.fwd_scale;  // |R| of the unitary transform
      const float Tv = tp[ti];
      const bool zj = j == E / 2 && zo;
      // free pixels keep R and stay out of the NMSE: the zero order, and a
      // pixel outside the region of interest (a negative prepared target;
      // size classes holding a problem with a region run the LT
      // instantiations, so the others keep this pass's plain arithmetic)
      const bool fr = zj || (LT && (MODE == COL_FINAL || MODE == COL_GS) && Tv < 0.f);
      if (!fr) {
        s_ta += Tv * A;
        s_aa += A * A;
        s_tt += Tv * Tv;
      }
      if constexpr (MODE == COL_FINAL) {
        if (d.replay_out) to_global(d.replay_out)[idx] = cscale(Rr, bt.fwd_scale);
      } else {
        if constexpr (DUMP) {
          if (d.r_out) to_global(d.r_out)[idx] = cscale(Rr, bt.fwd_scale);
        }
        float amp = Tv;
        if constexpr (MODE == COL_WGS) {
          if (Tv > 0.f) {
            const float ratio = fmaxf(Tv, kWgsEps) * __builtin_amdgcn_rcpf(fmaxf(A, kWgsEps));
            const float wc = clamp_w(w[ti] * ratio * inv_m);
            const float wn = __builtin_amdgcn_exp2f(kWgsGamma * __builtin_amdgcn_logf(wc));
            w[ti] = wn;
            s_w += wn;
            amp = wn * Tv;
          }
        }
        v[j] = a2 > 0.f ? cscale(Rr, amp * inv) : make_float2(amp, 0.f);
        if constexpr (MODE == COL_GS && LT) {  // Liu-Taghizadeh: amplitude free outside the square
          const bool out = max(abs(t + T * j - (NY >> 1)), abs(u - (NX >> 1))) > ltr;
          v[j] = out ? cscale(Rr, bt.fwd_scale) : v[j];
        }
        if (fr) v[j] = cscale(Rr, bt.fwd_scale);
      }
    }
    block_sum4<NT>(s_ta, s_aa, s_tt, s_w, red, tot);
    if (threadIdx.x == 0) {
      double* pp = part_ptr(bt, b, k - 1, blk);
      pp[0] = tot[0]; pp[1] = tot[1]; pp[2] = tot[2];
      if (MODE == COL_WGS) part_ptr(bt, b, k, blk)[3] = tot[3];
    }
    if constexpr (MODE != COL_FINAL) {
      fft<NY, E, +1>(v, t, bt.tw_y, ex);
#pragma unroll
      for (int j = 0; j < E; ++j) fld[tix(t + T * j, u, NX)] = v[j];
    }
  } else {
    // OSPR.  Subframe n's column work: finish subframe n-1 (forward FFT,
    // accumulate, NMSE partials, feedback), then start subframe n (random
    // replay phase, inverse FFT).
    const Desc& d = bt.desc[b];
    gptr<const float> tp = to_global(bt.tprep + off);
    const int n = arg;
    gptr<float> acc = to_global(bt.accum + off);
    if constexpr (MODE != COL_OSPR_FIRST) {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = fld[tix(t + T * j, u, NX)];
      fft<NY, E, -1>(v, t, bt.tw_y, ex);
    }
    const float inv_prev = 1.0f / (float)(n - 1);
    float s_ta = 0.f, s_aa = 0.f, s_tt = 0.f;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const size_t idx = (size_t)(t + T * j) * NX + u;  // caller arrays
      const uint32_t ti = tix(t + T * j, u, NX);            // workspace planes
      const float Tv = tp[ti];
      float Tn = Tv;
      if constexpr (MODE != COL_OSPR_FIRST) {
        const float2 R = cscale(v[j], bt.fwd_scale);
        const float a = (n == 2 ? 0.f : acc[ti]) + (R.x * R.x + R.y * R.y);  // A_{n-1}
        if constexpr (MODE == COL_OSPR_FINAL) {
          if (d.accum_out) to_global(d.accum_out)[idx] = a;
        } else {
          acc[ti] = a;
        }
        const float avg = a * inv_prev;
        s_ta += Tv * __builtin_amdgcn_sqrtf(avg);
        s_aa += avg;
        s_tt += Tv * Tv;
        if (adaptive) Tn = __builtin_amdgcn_sqrtf(fmaxf(0.f, (float)n * Tv * Tv - a));
      }
      v[j] = make_float2(Tn, 0.f);  // amplitude of subframe n's replay target
    }
    if constexpr (MODE != COL_OSPR_FIRST) {
      block_sum4<NT>(s_ta, s_aa, s_tt, 0.f, red, tot);
      if (threadIdx.x == 0) {
        double* pp = part_ptr(bt, b, n - 2, blk);
        pp[0] = tot[0]; pp[1] = tot[1]; pp[2] = tot[2];
      }
    }
    if constexpr (MODE != COL_OSPR_FINAL) {
      // replay phase of subframe n: Philox words over column lines
#pragma unroll
      for (int g = 0; g < E / 4; ++g) {
        const U64x4 o = philox_line_block(d.seed, d.item, 0x100u + (uint32_t)n, (uint32_t)(t + T * g), (uint32_t)u);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int j = g + (E / 4) * w;
          v[j] = cscale(philox_phasor(u64x4_word(o, w)), v[j].x);
        }
      }
      fft<NY, E, +1>(v, t, bt.tw_y, ex);
#pragma unroll
      for (int j = 0; j < E; ++j) fld[tix(t + T * j, u, NX)] = v[j];
    }
  }
}

// ---------------------------------------------------------------------------
// column pass with wave-local transforms (NY <= 1024: the NY/16 threads of a
// column fit in one wave).  Phases:
//   A  coalesced tile load, thread (c, r) reads rows r + T i of column c,
//      into a column-major LDS tile;
//   B  each wave transforms its column(s) in LDS with wave-level ordering
//      only (no workgroup barrier inside the transform);
//   C  element-wise constraint back in the coalesced mapping, so target and
//      weight traffic is coalesced too; NMSE partials;
//   D  inverse transforms, wave-local again;
//   E  coalesced store.
// Four workgroup barriers in all.
// ---------------------------------------------------------------------------
template <int NY, int C>
__host__ __device__ constexpr int colw_stride() {
  // padded column length, chosen so that C columns x (64/C) rows of a wave
  // in the coalesced mapping hit distinct bank pairs
  return NY + NY / 16 + (((64 / C) - (NY + NY / 16)) % 32 + 32) % 32;
}

// LDS exchange inside one column region, ordered within the wave.
struct WaveColEx {
  float2* s;
  __device__ void before_read() { wave_lds_sync(); }
  __device__ void before_write() { wave_lds_sync(); }
  __device__ float2 ld(int e) const { return s[e]; }
  __device__ void st(int e, float2 v) { s[e] = v; }
};

// LT, DUMP as for k_col; F16: the field plane holds 16-bit elements (the final
// measurement pass of such calls)
template <int NY, int C, int MODE, bool LT = false, bool DUMP = false, bool F16 = false>
__global__ __launch_bounds__(C * (NY / kE)) void k_colw(Batch bt, int arg, int adaptive, const float2* pin,
                                                        float2* pout) {
  static_assert(!F16 || MODE == COL_FINAL, "16-bit planes: the tile kernel runs the iterations");
  constexpr int E = kE, T = NY / E, NT = C * T;
  static_assert(T <= 64 && 64 % T == 0, "a column must fit in one wave");
  constexpr int RS = colw_stride<NY, C>();
  __shared__ float2 tile[C * RS];
  __shared__ double red[kMaxWaves][4];
  __shared__ double tot[4];
  __shared__ double bc;
  const int b = blockIdx.y, blk = xcd_tile(blockIdx.x, gridDim.x);
  const int cc = threadIdx.x % C, r0 = threadIdx.x / C;  // coalesced mapping
  const int cw = threadIdx.x / T, tw = threadIdx.x % T;  // wave mapping
  const int u = blk * C + cc;
  const int NX = bt.nx;
  const size_t off = (size_t)b * NY * NX;
  gptr<float2> fld = to_global(bt.field + off);
  float2* mine = tile + cc * RS;  // column cc, coalesced mapping
  WaveColEx ex{tile + cw * RS};   // column cw, wave mapping
  const Desc& d = bt.desc[b];
  gptr<const float> tp = to_global(bt.tprep + off);
  constexpr bool GSK = (MODE == COL_GS || MODE == COL_WGS || MODE == COL_FINAL);
  const int k = arg;  // GS: column pass of iteration k; OSPR: subframe n = arg
  if constexpr (MODE == COL_FINAL) {
    if (k != d.iters + 1) return;  // uniform per block
  } else if constexpr (MODE == COL_GS || MODE == COL_WGS) {
    if (k > d.iters) return;
  }
  float inv_m = 1.0f;
  gptr<float> w = nullptr;
  if constexpr (MODE == COL_WGS) {
    const double om = slot_total(bt, b, bt.slots - 1, 1, &bc);
    const double wsum = slot_total(bt, b, k - 1, 3, &bc);
    inv_m = (float)((om > 0.0 ? om : 1.0) / wsum);
    w = to_global(bt.wbuf + off);
  }
  const int ltr = LT ? uni(lt_radius(d, k, NY, NX)) : 0;
  float2 v[E];

  // A + B: forward column transform of the field
  if constexpr (MODE != COL_OSPR_FIRST) {
#pragma unroll
    for (int i = 0; i < E; ++i) {
      if constexpr (F16) {
        v[i] = unpack_h2(to_global(reinterpret_cast<const uint32_t*>(bt.field) + off)[tix(r0 + T * i, u, NX)],
                         bt.inv16_row);
      } else {
        v[i] = fld[tix(r0 + T * i, u, NX)];
      }
    }
#pragma unroll
    for (int i = 0; i < E; ++i) mine[lds_pad(r0 + T * i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = ex.s[lds_pad(tw + T * j)];
    fft<NY, E, -1>(v, tw, bt.tw_y, ex);
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < E; ++j) ex.s[lds_pad(tw + T * j)] = v[j];
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);  // keep phase C's loads out of the transform
  }

  // C: element-wise, coalesced mapping (rows r0 + T i of column u).  The
  // table pointers are re-derived here so their loads are not hoisted above
  // the transform, where they would hold registers through it.
  tp = launder(tp);
  if constexpr (MODE == COL_WGS) w = launder(w);
  float s_ta = 0.f, s_aa = 0.f, s_tt = 0.f, s_w = 0.f;
  if constexpr (GSK) {
    // amplitude SLM: the zero order (row NY/2 = element E/2 of r0 = 0, column
    // nx/2) keeps R and stays out of the NMSE sums
    static_assert(T * (E / 2) == NY / 2, "the zero order is element E/2 of thread row 0");
    const bool zo = d.mod && r0 == 0 && u == (NX >> 1);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int row = r0 + T * i;
      const size_t idx = (size_t)row * NX + u;  // caller arrays
      const uint32_t ti = tix(row, u, NX);        // workspace planes
      const float2 Rr = mine[lds_pad(row)];  // unscaled replay at centred index (row, u)
      const float a2 = Rr.x * Rr.x + Rr.y * Rr.y;
      const float inv = a2 > 0.f ? __builtin_amdgcn_rsqf(a2) : 0.f;
      const float A = a2 * inv * bt.fwd_scale;  // |R| of the unitary transform
      const float Tv = tp[ti];
      const bool zj = i == E / 2 && zo;
      // free pixels keep R and stay out of the NMSE: the zero order, and a
      // pixel outside the region of interest (a negative prepared target;
      // size classes holding a problem with a region run the LT
      // instantiations, so the others keep this pass's plain arithmetic)
      const bool fr = zj || (LT && (MODE == COL_FINAL || MODE == COL_GS) && Tv < 0.f);
      if (!fr) {
        s_ta += Tv * A;
        s_aa += A * A;
        s_tt += Tv * Tv;
      }
      if constexpr (MODE == COL_FINAL) {
        if (d.replay_out) to_global(d.replay_out)[idx] = cscale(Rr, bt.fwd_scale);
      } else {
        if constexpr (DUMP) {
          if (d.r_out) to_global(d.r_out)[idx] = cscale(Rr, bt.fwd_scale);
        }
        float amp = Tv;
        if constexpr (MODE == COL_WGS) {
          if (Tv > 0.f) {
            const float ratio = fmaxf(Tv, kWgsEps) * __builtin_amdgcn_rcpf(fmaxf(A, kWgsEps));
            const float wc = clamp_w(w[ti] * ratio * inv_m);
            const float wn = __builtin_amdgcn_exp2f(kWgsGamma * __builtin_amdgcn_logf(wc));
            w[ti] = wn;
            s_w += wn;
            amp = wn * Tv;
          }
        }
        mine[lds_pad(row)] = a2 > 0.f ? cscale(Rr, amp * inv) : make_float2(amp, 0.f);
        if constexpr (MODE == COL_GS && LT) {  // Liu-Taghizadeh: amplitude free outside the square
          const bool out = max(abs(row - (NY >> 1)), abs(u - (NX >> 1))) > ltr;
          if (out) mine[lds_pad(row)] = cscale(Rr, bt.fwd_scale);
        }
        if (fr) mine[lds_pad(row)] = cscale(Rr, bt.fwd_scale);
      }
    }
    block_sum4<NT>(s_ta, s_aa, s_tt, s_w, red, tot);  // ends with a barrier
    if (threadIdx.x == 0) {
      double* pp = part_ptr(bt, b, k - 1, blk);
      pp[0] = tot[0]; pp[1] = tot[1]; pp[2] = tot[2];
      if (MODE == COL_WGS) part_ptr(bt, b, k, blk)[3] = tot[3];
    }
  } else {
    // OSPR: finish subframe n-1 (accumulate, NMSE partials, feedback), start
    // subframe n (random replay phase).  Element i = g + 4 w' of this thread
    // shares a Philox block with its quarter-column siblings.
    const int n = arg;
    gptr<float> acc = to_global(bt.accum + off);
    const float inv_prev = 1.0f / (float)(n - 1);
    float amp[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int row = r0 + T * i;
      const size_t idx = (size_t)row * NX + u;  // caller arrays
      const uint32_t ti = tix(row, u, NX);        // workspace planes
      const float Tv = tp[ti];
      float Tn = Tv;
      if constexpr (MODE != COL_OSPR_FIRST) {
        const float2 R = cscale(mine[lds_pad(row)], bt.fwd_scale);
        const float a = (n == 2 ? 0.f : acc[ti]) + (R.x * R.x + R.y * R.y);  // A_{n-1}
        if constexpr (MODE == COL_OSPR_FINAL) {
          if (d.accum_out) to_global(d.accum_out)[idx] = a;
        } else {
          acc[ti] = a;
        }
        const float avg = a * inv_prev;
        s_ta += Tv * __builtin_amdgcn_sqrtf(avg);
        s_aa += avg;
        s_tt += Tv * Tv;
        if (adaptive) Tn = __builtin_amdgcn_sqrtf(fmaxf(0.f, (float)n * Tv * Tv - a));
      }
      amp[i] = Tn;
    }
    if constexpr (MODE != COL_OSPR_FINAL) {
#pragma unroll
      for (int g = 0; g < E / 4; ++g) {
        const U64x4 o = philox_line_block(d.seed, d.item, 0x100u + (uint32_t)n, (uint32_t)(r0 + T * g), (uint32_t)u);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = g + (E / 4) * q;
          mine[lds_pad(r0 + T * i)] = cscale(philox_phasor(u64x4_word(o, q)), amp[i]);
        }
      }
    }
    if constexpr (MODE != COL_OSPR_FIRST) {
      block_sum4<NT>(s_ta, s_aa, s_tt, 0.f, red, tot);  // ends with a barrier
      if (threadIdx.x == 0) {
        double* pp = part_ptr(bt, b, n - 2, blk);
        pp[0] = tot[0]; pp[1] = tot[1]; pp[2] = tot[2];
      }
    } else {
      __syncthreads();
    }
  }
  if constexpr (MODE == COL_FINAL || MODE == COL_OSPR_FINAL) return;
  __builtin_amdgcn_sched_barrier(0);

  // D + E: inverse column transform, coalesced store
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = ex.s[lds_pad(tw + T * j)];
  fft<NY, E, +1>(v, tw, bt.tw_y, ex);
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < E; ++j) ex.s[lds_pad(tw + T * j)] = v[j];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < E; ++i) fld[tix(r0 + T * i, u, NX)] = mine[lds_pad(r0 + T * i)];
}

// ---------------------------------------------------------------------------
// Persistent, software-pipelined column pass for GS / weighted GS.
//
// A resident grid of workgroups walks the column tiles of the whole batch.
// While a workgroup transforms tile i, the field, target and weight columns
// of its tile i + 1 stream into a second LDS stage with direct-to-LDS loads
// (global_load_lds_dwordx4: 16 bytes per lane, no registers held), so HBM
// traffic never waits for the transforms.  Everything the transforms touch
// lives in LDS (stages, twiddles) and the only global accesses during the
// compute phase are stores, so nothing waits on the in-flight prefetch until
// the tile's end.  The two stages are distinct arrays and the loop is
// unrolled by two, so every LDS access names its stage statically.
//
// Tile order: column tiles that share 128-byte lines (of the tiled target
// and weights, when C = 4) are handed, in the same step, to workgroups on
// the same XCD (workgroups are dispatched round-robin over the 8 XCDs), so
// each line is fetched into one L2 once.
// ---------------------------------------------------------------------------
// Workgroup barrier that orders LDS traffic only: waits for this wave's LDS
// operations, then s_barrier.  The fenced __syncthreads() would also wait for
// the in-flight direct-to-LDS prefetch (counted by vmcnt), which is exactly
// what the pipelined pass must not do.  The memory clobber keeps the compiler
// from moving memory operations across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// ColEx<C, false> with LDS-only barriers.
template <int C> struct ColExL {
  float2* s;
  __device__ void before_read() { lds_barrier(); }
  __device__ void before_write() { lds_barrier(); }
  __device__ float2 ld(int e) const { return s[e * C]; }
  __device__ void st(int e, float2 v) { s[e * C] = v; }
};

// block_sum4 with LDS-only barriers.
template <int NT>
__device__ __forceinline__ void block_sum4_l(float a0, float a1, float a2, float a3, double (&red)[kMaxWaves][4],
                                             double (&tot)[4]) {
  constexpr int NW = (NT + 63) / 64;
  const double d0 = wave_sum((double)a0), d1 = wave_sum((double)a1);
  const double d2 = wave_sum((double)a2), d3 = wave_sum((double)a3);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  lds_barrier();
  if (lane == 0) { red[wv][0] = d0; red[wv][1] = d1; red[wv][2] = d2; red[wv][3] = d3; }
  lds_barrier();
  if (threadIdx.x < 4) {
    double acc = 0.0;
    for (int w = 0; w < NW; ++w) acc += red[w][threadIdx.x];
    tot[threadIdx.x] = acc;
  }
  lds_barrier();
}

// Make a uniform value available (loaded) at this point: later memory
// operations are not hoisted above it and the value is not re-loaded later.
__device__ __forceinline__ int pin_uniform(int x) {
  x = __builtin_amdgcn_readfirstlane(x);
  asm volatile("" : "+s"(x)::"memory");
  return x;
}
__device__ __forceinline__ const float* pin_uniform_ptr(const float* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  asm volatile("" : "+s"(lo), "+s"(hi)::"memory");
  return reinterpret_cast<const float*>(((uint64_t)hi << 32) | lo);
}

// Element at a 32-bit byte offset from a wave-uniform base: lets the
// compiler address with a scalar base plus one 32-bit VGPR offset.
template <class T> __device__ __forceinline__ gptr<T> at_bytes(gptr<T> p, uint32_t b) {
  return (gptr<T>)((__attribute__((address_space(1))) char*)p + b);
}

// Elements per thread of the tile transforms of k_colp / k_colq (the 16 of
// every other pass).
constexpr int kColpE = 16;

template <int NY, int C, int E = kColpE>
struct ColpShape {
  static constexpr int T = NY / E, NT = C * T;
  static constexpr int FE = (NY + NY / 16) * C;  // float2: padded exchange tile (unpadded fill first)
  static constexpr int TWN = TwLayout<NY, E>::total();
  // column tiles sharing a 128-byte line: a 4 x 4 tile of the field is a
  // whole line, one of the 4-byte target / weights half a line
  static constexpr int G = C >= 8 ? 1 : 8 / C;
};

template <int NY, int C, int E = kColpE>
__host__ __device__ constexpr int colp_lds_bytes() {
  using S = ColpShape<NY, C, E>;
  return 2 * S::FE * 8 + S::TWN * 8 + (kMaxWaves * 4 + 5) * 8;
}
// Compiled tile shapes (C columns of NY rows) of the pipelined pass.
__host__ __device__ constexpr bool colp_ok(int NY, int C) {
  return (NY == 1024 && (C == 4 || C == 8)) || (NY == 512 && (C == 8 || C == 16)) || (NY == 256 && C == 16);
}

#if defined(__HIP_DEVICE_COMPILE__)
#define HG_AS1(p) ((const __attribute__((address_space(1))) void*)(p))
#define HG_AS3(p) ((__attribute__((address_space(3))) void*)(p))
#else
#define HG_AS1(p) ((const void*)(p))
#define HG_AS3(p) ((void*)(p))
#endif

// Stage layout of a tile: the tiled field's own order, row quads of C / 4
// consecutive 4 x 4 tiles, so element (row, c) is at colp_sidx<C>(row, c).
template <int C> __device__ __forceinline__ int colp_sidx(int row, int c) {
  return ((row >> 2) * (C / 4) + (c >> 2)) * 16 + (row & 3) * 4 + (c & 3);
}

// Issue the direct-to-LDS loads of tile vt's field columns: per row quad,
// C / 4 tiles of 128 contiguous bytes (2 C chunks of 16 bytes).  Each wave
// instruction fills 64 consecutive chunks (1 KB of LDS from a wave-uniform
// base).
// F16: a 16-bit plane, whose 4 x 4 tile is 64 bytes (C chunks per row quad),
// lands in the stage as 4-byte elements in the same order.
template <int NY, int C, int E, bool F16 = false>
__device__ __forceinline__ void colp_prefetch(const Batch& bt, int vt, int tpp, float2* F) {
  using S = ColpShape<NY, C, E>;
  constexpr int EB = F16 ? 4 : 8;              // bytes per element
  constexpr int NW = S::NT / 64, CPQ = C * EB / 4;  // 16-byte chunks per row quad (4 rows x C columns)
  constexpr int EPC = 16 / EB;                 // elements per chunk
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b = vt / tpp, blk = vt - b * tpp;
  const int NX = bt.nx;
  const char* src = reinterpret_cast<const char*>(bt.field) +
                    ((size_t)b * NY * NX + (size_t)blk * C * 4) * EB;  // tile (0, blk C / 4)
  const size_t qstride = (size_t)(NX >> 2) * 16 * EB;                   // bytes per tile row
  char* dst = reinterpret_cast<char*>(F);
#pragma unroll
  for (int q = 0; q < NY * CPQ / 4 / S::NT; ++q) {
    const int base = (q * NW + wave) * 64;
    const int ch = base + lane;
    const int quad = ch / CPQ, part = ch - quad * CPQ;
    __builtin_amdgcn_global_load_lds(HG_AS1(src + quad * qstride + 16 * part), HG_AS3(dst + 16 * base), 16, 0, 0);
  }
  (void)EPC;
}

// Register-held per-tile inputs: activity, 1/m, the weight plane, target
// and weight columns.
template <int E> struct ColpIn {
  int active;
  int lt_r;     // Liu-Taghizadeh: radius of this iteration's target square (-1: whole plane)
  float inv_m;
  float* wout;  // the problem's weight plane (wave-uniform)
  int y0, y1;   // the tile's first and last support row (y1 < y0: none)
  int zo;       // amplitude SLM and the tile holds column nx/2: the zero order is here
  float tv[E], wv[E];
};

// Byte offset of element (t, u) of a 4-byte plane in the 4 x 4 tiled layout;
// rows t + T j of a tile column lie j T nx elements further on (T a multiple
// of 4), so one 32-bit offset per element addresses every plane from a
// wave-uniform base.
__device__ __forceinline__ uint32_t colp_b0(int t, int u, int nx) { return 4u * tix(t, u, nx); }

// Load tile vt's inputs.  Issued at the end of the previous tile, after its
// stores, so these loads and that tile's prefetch complete under one wait.
template <int NY, int C, int MODE, int E>
__device__ __forceinline__ void colp_load_in(const Batch& bt, int k, int vt, int tpp, ColpIn<E>& in) {
  constexpr int T = NY / E;
  static_assert(T % 4 == 0, "row step of whole 4-row groups");
  const int b = vt / tpp, blk = vt - b * tpp;
  const Desc& d = bt.desc[b];
  in.active = d.iters >= k;
  if (!in.active) return;
  in.lt_r = -1;
  if constexpr (MODE == COL_GS || MODE == COL_GSR) {
    if (d.lt) in.lt_r = (int)min((long long)d.lt_r0 + (long long)(k - 1) * d.lt_dr, (long long)(NY + bt.nx));
  }
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int u = blk * C + c;
  const int NX = bt.nx;
  in.zo = d.mod && blk == (NX >> 1) / C;
  const size_t off = (size_t)b * NY * NX;
  gptr<const float> tp = to_global(uni_ptr(bt.tprep + off));
  const uint32_t b0 = colp_b0(t, u, NX), bstep = 4u * (uint32_t)(T * NX);
  // The target is zero outside its support Omega, whose rows in this tile the
  // set-up pass recorded: a tile that misses Omega reads no target or
  // weights, one that meets it reads those of its support rows [y0, y1]
  // (other lanes read row y0's element, an L2 hit, and take 0)
  const double* ps = part_ptr(bt, b, bt.slots - 1, blk);
  const bool meets = ps[1] > 0.0;
  const int y0 = meets ? (int)ps[2] : 0, y1 = meets ? (int)ps[3] : -1;
  in.y0 = y0;
  in.y1 = y1;
  const uint32_t by0 = colp_b0(y0, u, NX);
  if (meets) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const bool sup = t + T * j >= y0 && t + T * j <= y1;
      const float x = *at_bytes(tp, sup ? b0 + bstep * j : by0);
      in.tv[j] = sup ? x : 0.f;
    }
  } else {
#pragma unroll
    for (int j = 0; j < E; ++j) in.tv[j] = 0.f;
  }
  if constexpr (MODE == COL_WGS) {
    in.inv_m = bt.invm[b];
    in.wout = uni_ptr(bt.wbuf + off);
    gptr<const float> w = to_global(in.wout);
    if (meets) {  // weights matter only where the target is nonzero
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const bool sup = t + T * j >= y0 && t + T * j <= y1;
        in.wv[j] = *at_bytes(w, sup ? b0 + bstep * j : by0);
      }
    }
  }
}

// One tile: transform the field in stage Fc with the register-held inputs
// while tile vtn's field streams into Fn; then load tile vtn's inputs and
// wait for everything (each wave for its own loads) before the barrier.
// LATE: this tile's target and weights are loaded here, after the forward
// transform, instead of ahead (in.active set by the caller).
template <int NY, int C, int MODE, int E, int PAR, class TWP, bool LATE = false, bool DUMP = false, bool F16 = false>
__device__ __forceinline__ void colp_tile(const Batch& bt, int k, int vt, int vtn, int total, int tpp,
                                          float2* __restrict__ Fc, float2* __restrict__ Fn, TWP tw,
                                          double (&red)[kMaxWaves][4], double (&tot)[4], ColpIn<E>& in) {
  using S = ColpShape<NY, C, E>;
  constexpr int T = S::T, NT = S::NT;
  constexpr bool WGS = MODE == COL_WGS;
  static_assert(2 * (NT / 64) <= kMaxWaves, "two tiles' per-wave partial slots");
  static_assert(Plan<NY, E>::ns > 1, "the inverse transform's exchange orders the slot writes before the reads");
  if (vtn < total) colp_prefetch<NY, C, E, F16>(bt, vtn, tpp, Fn);
  if (in.active) {
    const int b = vt / tpp, blk = vt - b * tpp;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int u = blk * C + c;
    const int NX = bt.nx;
    const size_t off = (size_t)b * NY * NX;
    float2 v[E];
    if constexpr (F16) {
      const uint32_t* F4 = reinterpret_cast<const uint32_t*>(Fc);
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = unpack_h2(F4[colp_sidx<C>(t + T * j, c)], bt.inv16_row);
    } else {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = Fc[colp_sidx<C>(t + T * j, c)];
    }
    ColExL<C> ex{Fc + c};
    fft_stage<NY, E, -1, 0>(v, t, tw, ex);
    if constexpr (LATE) colp_load_in<NY, C, MODE, E>(bt, k, vt, tpp, in);
    const uint32_t b0 = colp_b0(t, u, NX), bstep = 4u * (uint32_t)(T * NX);
    float s_ta = 0.f, s_aa = 0.f, s_tt = 0.f, s_w = 0.f;
    float s_off = 0.f;  // unscaled |R|^2 of the elements in row blocks off the support
    gptr<float> w = nullptr;
    if constexpr (WGS) w = to_global(in.wout);
    // This wave's lanes hold rows tw0 .. tw0 + 64/C - 1 (+ T j).  A block of
    // rows outside the tile's support rows has T = 0 throughout, so R' = 0
    // there (weights unused) and only |R|^2 enters the NMSE sums: a
    // wave-uniform branch skips the constraint (not for Liu-Taghizadeh, whose
    // free region keeps R, nor for the dumping pass).
    static_assert(64 % C == 0, "whole columns of lanes per wave");
    const int tw0 = uni((int)(threadIdx.x >> 6) * (64 / C));
    const bool all_rows = DUMP || in.lt_r >= 0;
    // amplitude SLM: the zero order (row NY/2 = t + T E/2 with t = 0, column
    // nx/2) keeps R and stays out of the NMSE sums
    static_assert(T * (E / 2) == NY / 2, "the zero order is element E/2 of thread row 0");
    const bool zo = in.zo && t == 0 && u == (NX >> 1);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int row = t + T * j;
      const float2 Rr = v[j];  // unscaled replay, centred index (row, u)
      const bool zj = j == E / 2 && zo;
      if (!all_rows && !(j == E / 2 && in.zo) && (tw0 + T * j > in.y1 || tw0 + 64 / C - 1 + T * j < in.y0)) {
        s_off = fmaf(Rr.x, Rr.x, fmaf(Rr.y, Rr.y, s_off));
        v[j] = make_float2(0.f, 0.f);
        continue;
      }
      const float a2 = Rr.x * Rr.x + Rr.y * Rr.y;
      const float inv = a2 > 0.f ? __builtin_amdgcn_rsqf(a2) : 0.f;
      const float A = a2 * inv * bt.fwd_scale;
      const float Tv = in.tv[j];
      // COL_GSR: a pixel outside the region of interest (negative prepared
      // target) keeps R and stays out of the NMSE sums, as does the
      // amplitude SLM's zero order.  Tz is the target with such pixels at 0
      // (a NaN target stays NaN).
      const bool rf = MODE == COL_GSR && Tv < 0.f;
      const float Tz = rf ? 0.f : Tv;
      if (!zj) {
        s_ta += Tz * A;
        s_aa += rf ? 0.f : A * A;
        s_tt += Tz * Tz;
      }
      if constexpr (DUMP) {  // one-iteration calls: the replay before the constraint
        const Desc& dd = bt.desc[b];
        if (dd.r_out) to_global(dd.r_out)[(size_t)row * NX + u] = cscale(Rr, bt.fwd_scale);
      }
      float amp = Tz;
      if constexpr (WGS) {
        if (Tv > 0.f) {
          const float ratio = fmaxf(Tv, kWgsEps) * __builtin_amdgcn_rcpf(fmaxf(A, kWgsEps));
          const float wc = clamp_w(in.wv[j] * ratio * in.inv_m);
          const float wn = __builtin_amdgcn_exp2f(kWgsGamma * __builtin_amdgcn_logf(wc));
          *at_bytes(w, b0 + bstep * j) = wn;
          s_w += wn;
          amp = wn * Tv;
        }
      }
      // R' = amp R/|R|, or R itself on a free pixel (unitary scale); R = 0
      // gives (amp, 0), which is 0 on a free pixel
      const float sc = rf ? bt.fwd_scale : amp * inv;
      v[j] = a2 > 0.f ? cscale(Rr, sc) : make_float2(amp, 0.f);
      if constexpr (MODE == COL_GS || MODE == COL_GSR) {  // Liu-Taghizadeh: amplitude free outside the square
        if (in.lt_r >= 0 && max(abs(t + T * j - (NY >> 1)), abs(u - (NX >> 1))) > in.lt_r)
          v[j] = cscale(Rr, bt.fwd_scale);
      }
      if (zj) v[j] = cscale(Rr, bt.fwd_scale);
    }
    s_aa = fmaf(s_off, bt.fwd_scale * bt.fwd_scale, s_aa);
    // the tile's partial sums: one FP64 sum per wave into this tile's LDS
    // slots now, added over the waves after the inverse transform, whose
    // barriers order the slot writes before those reads (alternate tiles use
    // alternate slots)
    {
      constexpr int NW = NT / 64;
      const double d0 = wave_sum((double)s_ta), d1 = wave_sum((double)s_aa);
      const double d2 = wave_sum((double)s_tt), d3 = wave_sum((double)s_w);
      double* slot = red[PAR * NW + (threadIdx.x >> 6)];
      if ((threadIdx.x & 63) == 0) { slot[0] = d0; slot[1] = d1; slot[2] = d2; slot[3] = d3; }
    }
    fft_stage<NY, E, +1, 0>(v, t, tw, ex);
    if (threadIdx.x < 4) {
      constexpr int NW = NT / 64;
      double acc = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) acc += red[PAR * NW + w][threadIdx.x];
      if (threadIdx.x < 3) part_ptr(bt, b, k - 1, blk)[threadIdx.x] = acc;
      else if (WGS) part_ptr(bt, b, k, blk)[3] = acc;
    }
    if constexpr (F16) {
      gptr<uint32_t> fld = to_global(uni_ptr(reinterpret_cast<uint32_t*>(bt.field) + off));
#pragma unroll
      for (int j = 0; j < E; ++j) *at_bytes(fld, b0 + bstep * j) = pack_h2(v[j], bt.s16_col);
    } else {
      gptr<float2> fld = to_global(uni_ptr(bt.field + off));
#pragma unroll
      for (int j = 0; j < E; ++j) *at_bytes(fld, 2u * (b0 + bstep * j)) = v[j];
    }
  }
  if (vtn < total) colp_load_in<NY, C, MODE, E>(bt, k, vtn, tpp, in);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

template <int NY, int C, int MODE, int E = kColpE>
__global__ __launch_bounds__(C * (NY / E))
void k_colp(Batch bt, int k, int nprob) {
  using S = ColpShape<NY, C, E>;
  static_assert(S::NT <= 1024 && S::NT % 64 == 0 && C >= 4, "pipelined column tile shape");
  static_assert(colp_lds_bytes<NY, C, E>() <= 160 * 1024, "the two stages must fit in LDS");
  __shared__ float2 FA[S::FE], FB[S::FE];
  __shared__ float2 TW[S::TWN];
  __shared__ double red[kMaxWaves][4];
  __shared__ double tot[4];
  // twiddles of this plan, FP64-evaluated into LDS
  for (int i = threadIdx.x; i < S::TWN; i += S::NT) twiddle_entry<NY, 1, E>(TW, i);
  const int tpp = bt.nx / C, total = tpp * nprob;
  const int NBK = gridDim.x;  // a multiple of 8 G
  const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
  const int slot = ((j / S::G) * 8 + xcd) * S::G + (j % S::G);
  int vt = slot;
  ColpIn<E> in;
  if (vt < total) {
    colp_prefetch<NY, C, E>(bt, vt, tpp, FA);
    colp_load_in<NY, C, MODE, E>(bt, k, vt, tpp, in);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const lptr<const float2> tw = (lptr<const float2>)TW;
  while (vt < total) {
    colp_tile<NY, C, MODE, E, 0>(bt, k, vt, vt + NBK, total, tpp, FA, FB, tw, red, tot, in);
    vt += NBK;
    if (vt >= total) break;
    colp_tile<NY, C, MODE, E, 1>(bt, k, vt, vt + NBK, total, tpp, FB, FA, tw, red, tot, in);
    vt += NBK;
  }
}

// One column tile per workgroup (the row pass's scheme): the pipelined
// pass's tile work without persistence, one LDS stage (35 KB) and twiddles
// from the global table, so that three (weighted: 136 registers) or four
// (plain GS) workgroups share a CU and hide each other's loads.  Capping the
// weighted kernel at 128 registers to fit four spills, and measured 9%
// slower.
template <int NY, int C, int MODE, int E = kColpE, bool DUMP = false, bool F16 = false>
__global__ __launch_bounds__(C * (NY / E))
void k_colq(Batch bt, int k, int nprob) {
  using S = ColpShape<NY, C, E>;
  static_assert(S::NT == 256, "4-wave workgroups, several per CU");
  __shared__ float2 FA[S::FE];
  __shared__ double red[kMaxWaves][4];
  __shared__ double tot[4];
  const int tpp = bt.nx / C, total = tpp * nprob;
  const int vt = xcd_tile(blockIdx.x, gridDim.x);
  if (vt >= total) return;  // uniform per block
  colp_prefetch<NY, C, E, F16>(bt, vt, tpp, FA);
  ColpIn<E> in;
  colp_load_in<NY, C, MODE, E>(bt, k, vt, tpp, in);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  colp_tile<NY, C, MODE, E, 0, decltype(launder(to_global(bt.tw_y))), false, DUMP, F16>(
      bt, k, vt, total, total, tpp, FA, FA, launder(to_global(bt.tw_y)), red, tot, in);
}


// OSPR column pass, one 4-column tile per workgroup (k_colq's scheme): for
// subframe n, finish subframe n-1 (forward transform, accumulate A, NMSE
// partials, feedback) and start subframe n (random replay phase, inverse
// transform).  The arithmetic is the classic OSPR column pass's.
template <int NY, int C, int MODE, int E = kColpE>
__global__ __launch_bounds__(C * (NY / E))
void k_colq_ospr(Batch bt, int n, int adaptive, int nprob) {
  using S = ColpShape<NY, C, E>;
  static_assert(S::NT == 256, "4-wave workgroups, several per CU");
  static_assert(Plan<NY, E>::ns > 1, "the inverse transform's exchange orders the slot writes before the reads");
  constexpr int T = S::T, NW = S::NT / 64;
  constexpr bool FIRST = MODE == COL_OSPR_FIRST, FINAL = MODE == COL_OSPR_FINAL;
  __shared__ float2 FA[S::FE];
  __shared__ double red[kMaxWaves][4];
  const int tpp = bt.nx / C, total = tpp * nprob;
  const int vt = xcd_tile(blockIdx.x, gridDim.x);
  if (vt >= total) return;  // uniform per block
  const int b = vt / tpp, blk = vt - b * tpp;
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int u = blk * C + c;
  const int NX = bt.nx;
  const size_t off = (size_t)b * NY * NX;
  const Desc& d = bt.desc[b];
  if constexpr (!FIRST) colp_prefetch<NY, C, E>(bt, vt, tpp, FA);
  // uniform bases: per element one 32-bit offset serves every plane (rows
  // t + T j of a 4x4-tiled plane lie j T NX elements apart)
  static_assert(T % 4 == 0, "row step of whole 4-row groups");
  gptr<const float> tp = to_global(uni_ptr(bt.tprep + off));
  gptr<float> acc = to_global(uni_ptr(bt.accum + off));
  const uint32_t b0 = 4u * tix(t, u, NX), bstep = 4u * (uint32_t)(T * NX);  // float byte offsets
  // the target is zero off its support, whose rows in this tile the set-up
  // pass recorded: read it on those rows only (other lanes read row y0's
  // element, an L2 hit, and take 0; a tile off the support reads none)
  const double* ps = part_ptr(bt, b, bt.slots - 1, blk);
  const bool meets = ps[1] > 0.0;
  const int y0 = meets ? (int)ps[2] : 0, y1 = meets ? (int)ps[3] : -1;
  const uint32_t by0 = 4u * tix(y0, u, NX);
  float tv[E], av[E];
  auto load_target = [&]() {
    if (meets) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const bool sup = t + T * j >= y0 && t + T * j <= y1;
        const float x = *at_bytes(tp, sup ? b0 + bstep * j : by0);
        tv[j] = sup ? x : 0.f;
      }
    } else {
#pragma unroll
      for (int j = 0; j < E; ++j) tv[j] = 0.f;
    }
  };
  // 8 elements per thread (small batches): target and A_{n-2} are loaded
  // with the field, their latency hidden by its; with 16, after the forward
  // transform, so fewer registers are live across it.  A_{n-2} is zero for
  // n = 2, where the plane holds no accumulation yet (loaded anyway and
  // discarded by a select: no branch per element).
  constexpr bool EARLY = E <= 8;
  if constexpr (FIRST || EARLY) load_target();
  if constexpr (!FIRST && EARLY) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const float x = *at_bytes(acc, b0 + bstep * j);
      av[j] = n == 2 ? 0.f : x;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const auto tw = launder(to_global(bt.tw_y));
  ColExL<C> ex{FA + c};
  float2 v[E];
  if constexpr (!FIRST) {
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = FA[colp_sidx<C>(t + T * j, c)];
    fft_stage<NY, E, -1, 0>(v, t, tw, ex);
    if constexpr (!EARLY) {
      load_target();
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const float x = *at_bytes(acc, b0 + bstep * j);
        av[j] = n == 2 ? 0.f : x;
      }
    }
    const float inv_prev = 1.0f / (float)(n - 1);
    float s_ta = 0.f, s_aa = 0.f, s_tt = 0.f;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const float2 R = cscale(v[j], bt.fwd_scale);
      const float a = av[j] + (R.x * R.x + R.y * R.y);  // A_{n-1}
      if constexpr (FINAL) {
        if (d.accum_out) to_global(d.accum_out)[(size_t)(t + T * j) * NX + u] = a;
      } else {
        *at_bytes(acc, b0 + bstep * j) = a;
      }
      const float Tv = tv[j];
      const float avg = a * inv_prev;
      s_ta += Tv * __builtin_amdgcn_sqrtf(avg);
      s_aa += avg;
      s_tt += Tv * Tv;
      // feedback as a select: a branch here makes the compiler copy tv[] per element
      const float tn = __builtin_amdgcn_sqrtf(fmaxf(0.f, (float)n * Tv * Tv - a));
      tv[j] = adaptive ? tn : Tv;
    }
    const double d0 = wave_sum((double)s_ta), d1 = wave_sum((double)s_aa), d2 = wave_sum((double)s_tt);
    if ((threadIdx.x & 63) == 0) {
      double* slot = red[threadIdx.x >> 6];
      slot[0] = d0; slot[1] = d1; slot[2] = d2;
    }
  }
  if constexpr (!FINAL) {
    // replay phase of subframe n: Philox words over column lines, element
    // j = g + (E/4) q of this thread in block g's word q
#pragma unroll
    for (int g = 0; g < E / 4; ++g) {
      const U64x4 o = philox_line_block(d.seed, d.item, 0x100u + (uint32_t)n, (uint32_t)(t + T * g), (uint32_t)u);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = g + (E / 4) * q;
        v[j] = cscale(philox_phasor(u64x4_word(o, q)), tv[j]);
      }
    }
    fft_stage<NY, E, +1, 0>(v, t, tw, ex);
    gptr<float2> fld = to_global(uni_ptr(bt.field + off));
#pragma unroll
    for (int j = 0; j < E; ++j) *at_bytes(fld, 2u * (b0 + bstep * j)) = v[j];
  } else {
    __syncthreads();  // the per-wave sums are in
  }
  if constexpr (!FIRST) {
    if (threadIdx.x < 3) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += red[w][threadIdx.x];
      part_ptr(bt, b, n - 2, blk)[threadIdx.x] = s;
    }
  }
}

// Copy the final weights of problems that passed their own weight array back
// to it (natural order from the tiled workspace plane).
static __global__ void k_weights_out(Batch bt) {
  const Desc& d = bt.desc[blockIdx.y];
  if (!d.user_weights) return;
  const long px = (long)bt.ny * bt.nx;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= px) return;
  const int y = (int)(i / bt.nx), x = (int)(i % bt.nx);
  d.weights[i] = bt.wbuf[(size_t)blockIdx.y * px + tix(y, x, bt.nx)];
}

// 1 / m_{k-1} of every problem for the pipelined weighted-GS column pass k:
// the same fixed-order sums as slot_total.
static __global__ __launch_bounds__(64) void k_wgs_invm(Batch bt, int k) { wgs_invm_wave(bt, blockIdx.x, k - 1); }

// NMSE = 1 - sta^2 / (stt saa) from the FP64 sums; a replay or target of
// zero energy gives 1.  Non-finite sums give NaN and raise the call's
// status word (read by hg_numeric_status).
__device__ __forceinline__ double nmse_from_sums(double sta, double saa, double stt, int* status) {
  if (!(__builtin_isfinite(sta) && __builtin_isfinite(saa) && __builtin_isfinite(stt))) {
    if (status) *status = 1;
    return __builtin_nan("");
  }
  return (saa > 0.0 && stt > 0.0) ? 1.0 - sta * sta / (stt * saa) : 1.0;
}

// nmse[k] = 1 - sta^2 / (stt saa) from the block partials of slot k; a GS
// problem has iters + 1 values, an OSPR problem `iters` (= subframes).  One
// wave per value: lane l sums tiles l, l + 64, ... and the wave adds the
// lanes (slot_total's fixed order), so a value costs nblk / 64 loads per lane
// instead of a chain of nblk loads in one thread.  Wave w of block (b, y)
// takes values k = 4 y + w, then k + 4 gridDim.y, ... of problem b.
constexpr int kFinishPerBlock = 4;
static __global__ void k_finish(Batch bt, int count, int ospr) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x & 63;
  if (b >= count) return;
  const Desc& d = bt.desc[b];
  if (!d.nmse_out) return;
  const int nk = d.iters + (ospr ? 0 : 1);
  for (int k = blockIdx.y * kFinishPerBlock + (int)(threadIdx.x >> 6); k < nk;
       k += (int)gridDim.y * kFinishPerBlock) {  // uniform per wave
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int i = lane; i < bt.nblk; i += 64) {
      const double* pp = part_ptr(bt, b, k, i);
      s0 += pp[0]; s1 += pp[1]; s2 += pp[2];
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) d.nmse_out[k] = nmse_from_sums(s0, s1, s2, bt.status);
  }
}
// Blocks along y for nk values (at most the grid limit; the waves loop).
inline unsigned finish_grid_y(int nk) {
  const int y = (nk + kFinishPerBlock - 1) / kFinishPerBlock;
  return (unsigned)(y < 65535 ? y : 65535);
}

}  // namespace hg
