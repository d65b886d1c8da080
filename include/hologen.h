/*
 * hologen.h -- C ABI of the MI355X (gfx950) hologram-generation hot path.
 *
 * The operations are those of the HoloGen paper (Christopher, Kadis, Gordon,
 * Wilkinson, arXiv 2008.12214): iterative Fourier transform algorithms
 * (Gerchberg-Saxton and weighted GS, "Iterative Fourier Transform
 * Algorithms" section), one-step phase retrieval and adaptive OSPR
 * ("Time-Averaged Algorithms" section), Fourier and Fresnel propagation
 * (Background section, Eqs. fouriertrans2d5c/d and the quadratic phase term
 * of Fresnel holograms), and projection onto binary or multi-level phase
 * SLMs (Algorithms section; Example section, Listing 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every buffer argument is a DEVICE pointer owned by the caller.  The
 *    library never frees caller memory, never allocates device memory and
 *    never synchronises the stream: work is enqueued on `stream` (a
 *    hipStream_t; NULL = the default stream) and the call returns.  Results
 *    are valid once the stream has reached that point.
 *  - Arrays are row-major [y][x] with Nx columns.  Complex data is
 *    interleaved complex64 (hg_complex).  Grid sizes ny and nx are
 *    independent powers of two in [64, 4096].
 *  - Transforms are unitary (1/sqrt(Nx Ny)).  Replay-plane arrays (target,
 *    weights, replay field, OSPR accumulator) are CENTRED: zero frequency
 *    at (ny/2, nx/2).  SLM-plane arrays (levels, SLM field) are in natural
 *    pixel order.
 *  - slm_levels: 0 = continuous phase (g/|g|); L in [2, 256] = uniform phase
 *    levels 2 pi k / L, k stored as uint8 (L = 2 is binary {0, pi}).  The
 *    level of a field value g is k = floor(arg(g) L / (2 pi) + 1/2) mod L.
 *  - The target amplitude is scaled internally so that sum T^2 = Nx Ny
 *    (automatic image scaling, "Floating Points" section); for L = 2 it is
 *    first symmetrised, T(u) <- sqrt((T(u)^2 + T(-u)^2)/2), because the
 *    replay of a real +-1 hologram is centro-symmetric.
 *  - NMSE is the scale-optimal normalised error of the replay amplitude A:
 *    1 - (sum T A)^2 / (sum T^2 sum A^2), sums in FP64 ("Error Metrics"
 *    section, Eq. mse, at the best uniform scale).
 *  - Random phases come from Philox4x64-10 (Salmon et al., SC'11) with key
 *    (seed, (item << 32) | tag).  The plane is split into lines of length n
 *    (axis 1: rows, n = nx; axis 0: columns, n = ny); element i of line l
 *    takes output word (i div n/4) of the block at counter
 *    (i mod n/4, l, 0, 0), and its phase is 2 pi (word >> 40) 2^-24.
 *    Tag 1 = initial SLM phase (axis 1); tag 0x100 + n = OSPR subframe n's
 *    replay phase (axis 0).
 *  - Workspace: `workspace` must hold at least the size returned by the
 *    matching *_workspace_size query, 256-byte aligned.  Its contents need
 *    no initialisation and are clobbered.  Calls that share a workspace
 *    must be ordered on one stream.
 *  - Errors: argument checks run on the host before any HIP call; on error
 *    nothing is enqueued and hg_last_error() holds a thread-local message.
 *    A HIP launch failure returns HG_ERR_HIP.  Non-finite values (a NaN or
 *    Inf in a target or in caller weights) cannot be reported by the call,
 *    which returns before the kernels run: the NMSE finisher writes NaN to
 *    nmse_out and raises a status word in the workspace, which
 *    hg_numeric_status() reads after the call (HG_ERR_NUMERIC).  A
 *    non-finite caller weight makes the set-up pass mark its pixel's
 *    prepared target NaN, so it is reported the same way.
 */
#ifndef HOLOGEN_H
#define HOLOGEN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hg_complex { float x, y; } hg_complex;

typedef enum hg_status {
  HG_OK = 0,
  HG_ERR_INVALID_ARG = 1,      /* null/inconsistent pointer, bad level count, iters < 1, ... */
  HG_ERR_UNSUPPORTED_SIZE = 2, /* ny or nx not a power of two in [64, 4096]                 */
  HG_ERR_WORKSPACE = 3,        /* workspace null, misaligned or smaller than the query      */
  HG_ERR_HIP = 4,              /* a HIP runtime call or kernel launch failed                */
  HG_ERR_NUMERIC = 5           /* the NMSE sums of a finished call were non-finite          */
} hg_status;

enum hg_op { HG_OP_GS = 1, HG_OP_WGS = 2, HG_OP_OSPR = 3, HG_OP_PROPAGATE = 4 };

/* Bytes of workspace needed by one call of `op` on an ny x nx grid with
 * `iters` iterations (GS/WGS) or subframes (OSPR); ignored for
 * HG_OP_PROPAGATE.  Returns 0 for unsupported arguments. */
size_t hg_workspace_size(int op, int ny, int nx, int iters);

/* SLM modulation (Background section: binary and multi-level phase or
 * amplitude schemes).  slm_levels = L alone selects a phase SLM: 0 is
 * continuous phase, 2..256 the uniform phases 2 pi k / L (L = 2 is binary
 * {0, pi}).  slm_levels = L | HG_SLM_AMPLITUDE (2 <= L <= 256) selects an
 * amplitude SLM with the uniform transmissions k / (L - 1) in [0, 1]
 * (binary {0, 1}); the projection takes the nearest transmission to Re g, g
 * at the unit-rms scale of the prepared target.  A non-negative
 * transmission always sends its mean into the zero-order (DC) pixel of the
 * replay, centred index (ny/2, nx/2), which no amplitude hologram controls:
 * for an amplitude SLM that pixel keeps R' = R and is left out of every
 * NMSE, and the target is symmetrised for every L as for binary phase (a
 * real field's replay is centro-symmetric).  Amplitude SLMs run in hg_gs,
 * hg_wgs, hg_gs_step, hg_wgs_static and hg_gs_batched (not Liu-Taghizadeh
 * or OSPR).  Levels out are the indices k.                                 */
#define HG_SLM_AMPLITUDE 0x10000

/* 16-bit field storage ("Floating Points" section: 16-, 32- and 64-bit
 * builds).  slm_levels | HG_FIELD_FP16 keeps the complex field between the
 * row and column passes as two IEEE binary16 values (4 bytes per element
 * instead of 8) in the workspace; every transform, constraint and projection
 * still computes in FP32.  The stored values are the unnormalised row
 * transform of the modulated SLM field and the unnormalised column inverse
 * transform of the constrained replay, each times 2^-floor(log2(n)/2) (n
 * the transform length: magnitudes near 1, no mantissa changed), rounded to
 * nearest even; a value beyond the binary16 range becomes infinite and the
 * NMSE NaN (HG_ERR_NUMERIC).  Accepted by hg_gs, hg_wgs, hg_lt, hg_gs_step
 * and hg_gs_batched for ny in {256, 512, 1024} (any supported nx); those
 * calls use the default launch configuration.  hg_workspace_size's answer
 * covers both storages.                                                     */
#define HG_FIELD_FP16 0x20000

/* Gerchberg-Saxton ("Iterative Fourier Transform Algorithms" section).
 *   target        [ny][nx] float, centred replay-plane amplitude, >= 0, not all 0
 *   iters         >= 1 iterations of: forward transform, replay constraint
 *                 R' = T R/|R| (R = 0 -> T), inverse transform, SLM projection
 *   slm_levels    0 or 2..256 (phase), or L | HG_SLM_AMPLITUDE (see above)
 *   seed          Philox seed of the initial phase (used when both init
 *                 pointers are NULL); the initial field is unquantised
 *   init_levels   nullable [ny][nx] uint8 start levels (< slm_levels, L >= 2)
 *   init_field    nullable [ny][nx] complex start field; wins over init_levels
 *   wavelength_m, pitch_m, z_m
 *                 Fresnel hologram when z_m > 0 and finite: chirp
 *                 exp(i pi p^2 ((x-nx/2)^2 + (y-ny/2)^2) / (lambda z)) applied
 *                 before the forward transform and conjugated after the
 *                 inverse; otherwise Fourier (both others ignored)
 *   levels_out    [ny][nx] uint8 final levels; required when slm_levels >= 2,
 *                 ignored (may be NULL) when slm_levels == 0
 *   slm_field_out nullable [ny][nx] complex final SLM field f_K
 *   replay_out    nullable [ny][nx] complex centred replay of f_K
 *   nmse_out      nullable iters+1 doubles: nmse[k] is the NMSE of the
 *                 replay of f_k (nmse[0] = initial field)                    */
hg_status hg_gs(const float* target, int ny, int nx, int iters, int slm_levels, uint64_t seed,
                const uint8_t* init_levels, const hg_complex* init_field,
                double wavelength_m, double pitch_m, double z_m,
                uint8_t* levels_out, hg_complex* slm_field_out, hg_complex* replay_out,
                double* nmse_out, void* workspace, size_t workspace_bytes, void* stream);

/* Weighted GS (named in the "Iterative Fourier Transform Algorithms"
 * section; the update rule is this library's reading, a leaky log-domain
 * integrator of the amplitude error):
 *   w_k = clamp(w_{k-1} max(T, 0.1) / max(|R|, 0.1) / m_{k-1}, 1e-6, 1e6)^0.7
 *   on T > 0 (w unchanged elsewhere), m_{k-1} = mean of w_{k-1} over T > 0,
 *   R' = w_k T R / |R|, with T and |R| at unit rms.
 * Arguments as hg_gs, plus
 *   weights_inout nullable [ny][nx] float centred weights: read as w_0 and
 *                 overwritten with w_K; NULL starts from w_0 = 1.            */
hg_status hg_wgs(const float* target, int ny, int nx, int iters, int slm_levels, uint64_t seed,
                 const uint8_t* init_levels, const hg_complex* init_field,
                 double wavelength_m, double pitch_m, double z_m,
                 uint8_t* levels_out, hg_complex* slm_field_out, hg_complex* replay_out,
                 double* nmse_out, float* weights_inout,
                 void* workspace, size_t workspace_bytes, void* stream);

/* One iteration from a caller-supplied state, with the intermediate fields
 * exposed for lock-step comparison ("Iterative Fourier Transform
 * Algorithms" section: GS, weighted GS or Liu-Taghizadeh).  From the SLM
 * field f_{k-1} (levels_in for slm_levels >= 2, or field_in; exactly one of
 * the two) and, when weighted, the weights w_{k-1} in weights_inout (the
 * lagged mean m_{k-1} is their mean over T > 0, as in hg_wgs), it computes
 * R_k = forward(f_{k-1}), the replay constraint, g = backward(R'_k) and
 * f_k = P_L(g), with the kernels of hg_gs / hg_wgs / hg_lt (the column pass
 * in the instantiation that also stores R_k).
 *   lt_radius     >= 0: Liu-Taghizadeh square of this radius (GS only);
 *                 < 0: none
 *   weights_inout [ny][nx] float, required when weighted: w_{k-1} in, w_k out
 *   r_out         nullable [ny][nx] complex: R_k, centred, before the constraint
 *   g_out         nullable [ny][nx] complex: g, SLM plane, before projection
 *   levels_out    [ny][nx] uint8 levels of f_k (required for slm_levels >= 2)
 *   field_out     nullable [ny][nx] complex f_k
 *   nmse_out      nullable 2 doubles: NMSE of R_k and of the replay of f_k
 * Other arguments, workspace (hg_workspace_size(op, ny, nx, 1)) and errors
 * as hg_gs / hg_wgs.                                                         */
hg_status hg_gs_step(const float* target, int ny, int nx, int slm_levels, int weighted,
                     const uint8_t* levels_in, const hg_complex* field_in,
                     double wavelength_m, double pitch_m, double z_m, int lt_radius,
                     float* weights_inout, hg_complex* r_out, hg_complex* g_out,
                     uint8_t* levels_out, hg_complex* field_out, double* nmse_out,
                     void* workspace, size_t workspace_bytes, void* stream);

/* Liu-Taghizadeh ("Iterative Fourier Transform Algorithms" section: part of
 * the replay field is targeted first and the part grows every iteration;
 * the region's shape and growth are this library's reading).  GS in which
 * iteration k = 1..iters constrains the amplitude only inside the centred
 * square |v - ny/2| <= r_k, |u - nx/2| <= r_k, r_k = lt_r0 + (k-1) lt_dr
 * pixels, and leaves it free outside (R' = R there).  NMSE is taken over the
 * whole plane.  Once r_k reaches max(ny, nx)/2 the iteration is plain GS.
 * Arguments as hg_gs, plus lt_r0 >= 0 and lt_dr >= 0.                       */
hg_status hg_lt(const float* target, int ny, int nx, int iters, int slm_levels, uint64_t seed,
                const uint8_t* init_levels, const hg_complex* init_field,
                double wavelength_m, double pitch_m, double z_m, int lt_r0, int lt_dr,
                uint8_t* levels_out, hg_complex* slm_field_out, hg_complex* replay_out,
                double* nmse_out, void* workspace, size_t workspace_bytes, void* stream);

/* OSPR / adaptive OSPR with binary-phase subframes ("Time-Averaged
 * Algorithms" section).  Subframe n = 1..subframes: random replay phase
 * phi_n (Philox tag 0x100 + n), h_n = binary projection of
 * IDFT(T_n e^{i phi_n}), A_n = A_{n-1} + |DFT(h_n)|^2,
 * nmse[n-1] = NMSE(T, sqrt(A_n / n)).  adaptive != 0 feeds back the missing
 * intensity, T_{n+1}^2 = max(0, (n+1) T^2 - A_n); adaptive == 0 keeps T.
 *   levels_out    [subframes][ny][nx] uint8 in {0, 1}, required
 *   nmse_out      nullable `subframes` doubles
 *   accum_out     nullable [ny][nx] float, A_N (centred)                     */
hg_status hg_ospr(const float* target, int ny, int nx, int subframes, int adaptive, uint64_t seed,
                  uint8_t* levels_out, double* nmse_out, float* accum_out,
                  void* workspace, size_t workspace_bytes, void* stream);

/* Unitary Fourier / Fresnel propagation of a complex field (Background
 * section).  direction = +1: SLM plane -> centred replay plane,
 * out = centre(DFT(in * Q)); direction = -1: centred replay -> SLM plane,
 * out = IDFT(uncentre(in)) * conj(Q).  Q is the chirp of hg_gs (Q = 1 when
 * z_m <= 0 or not finite).  in and out may alias.                            */
hg_status hg_fresnel_propagate(const hg_complex* in, hg_complex* out, int ny, int nx,
                               double wavelength_m, double pitch_m, double z_m, int direction,
                               void* workspace, size_t workspace_bytes, void* stream);

/* The random phase field the library draws: out[y][x] = exp(2 pi i u24)
 * with u24 the top 24 bits of the Philox word of element (y, x) of stream
 * (seed, item, tag) split into lines along `axis`, as described above.
 * (tag 1, axis 1, item 0) is hg_gs's initial SLM phase; (0x100 + n, axis 0)
 * is OSPR subframe n's replay phase.  No workspace.                         */
hg_status hg_random_phase(uint64_t seed, uint32_t item, uint32_t tag, int axis, int ny, int nx, hg_complex* out,
                          void* stream);

/* Batch processing (program summary: batch processing of many images):
 * many independent GS problems of possibly different sizes in one call.
 * Problems are grouped by (ny, nx); each group runs as one batched launch
 * per pass.  Per-problem fields mirror hg_gs (Philox item = index in the
 * array, so problem b draws key (seed, (b << 32) | 1) unless init_levels
 * is given).                                                                 */
typedef struct hg_problem {
  int ny, nx, slm_levels, iters;
  uint64_t seed;
  double wavelength_m, pitch_m, z_m;
  const float* target;
  uint8_t* levels_out;          /* required when slm_levels >= 2 */
  double* nmse_out;             /* nullable, iters+1 */
  const uint8_t* init_levels;   /* nullable start levels (slm_levels >= 2) */
  hg_complex* replay_out;       /* nullable centred replay of the final field */
  int lt;                       /* nonzero: Liu-Taghizadeh as hg_lt (GS only) */
  int lt_r0, lt_dr;             /* its region radius and growth, pixels >= 0 */
  int reserved_;                /* 0 */
  float* weights;               /* weighted calls: nullable [ny][nx] centred weights, read as w_0 and
                                   overwritten with w_K (as hg_wgs); NULL starts from 1. Ignored
                                   (may be set) when the call is not weighted */
  const uint8_t* roi;           /* nullable region of interest, see below (plain GS only) */
} hg_problem;

/* Region of interest (Background section: many applications care about part
 * of the replay field only, and restricting the error metric to that part
 * gives the algorithm more freedom; Algorithms section: amplitude freedom
 * where the replay is not controlled).  roi is a centred [ny][nx] uint8 mask,
 * nonzero = controlled replay pixel.  The target outside the mask is
 * ignored (it is zeroed before the preparation, so the energy scaling counts
 * the mask only).  The controlled region is the mask, united with its mirror
 * image T(-u) for binary phase and amplitude SLMs, whose replay is
 * centro-symmetric.  Inside the region the constraint is GS's,
 * R' = T R/|R|; outside R' = R; every NMSE (nmse_out) counts the region
 * only.  A problem with a region runs plain GS on a phase or amplitude SLM:
 * with weighted != 0 or lt != 0 the call fails with HG_ERR_INVALID_ARG.  A
 * target with no energy inside the mask gives NaN NMSEs (HG_ERR_NUMERIC).
 * Problems with a region run the multi-launch pipeline at every size.        */

/* Many OSPR / adaptive OSPR problems in one call ("Time-Averaged
 * Algorithms" section; the paper's batch processing of independent
 * holograms).  Every problem runs the same number of subframes and the same
 * adaptive flag; the problems are grouped by (ny, nx) as in hg_gs_batched,
 * one launch per pass for each size.  Problem i draws its subframe phases
 * with Philox item i and its own seed, so its results equal an hg_ospr call
 * with that seed only up to that item (problem 0 equals it bit for bit).
 * Per problem as hg_ospr: levels_out [subframes][ny][nx] required,
 * nmse_out (subframes doubles) and accum_out ([ny][nx], centred) nullable;
 * all device pointers owned by the caller.  `problems` is a HOST array of
 * `count` entries, read during the call only.  workspace: at least
 * hg_ospr_batched_workspace_size(problems, count, subframes) bytes of device
 * memory (HG_ERR_WORKSPACE otherwise).  Invalid sizes, count < 1,
 * subframes < 1 or a missing target or levels_out give
 * HG_ERR_INVALID_ARG / HG_ERR_UNSUPPORTED_SIZE before anything is enqueued. */
typedef struct hg_ospr_problem {
  int ny, nx;
  uint64_t seed;
  const float* target;
  uint8_t* levels_out;
  double* nmse_out;
  float* accum_out;
} hg_ospr_problem;

size_t hg_ospr_batched_workspace_size(const hg_ospr_problem* problems, int count, int subframes);
hg_status hg_ospr_batched(const hg_ospr_problem* problems, int count, int subframes, int adaptive,
                          void* workspace, size_t workspace_bytes, void* stream);

size_t hg_gs_batched_workspace_size(const hg_problem* problems, int count);
hg_status hg_gs_batched(const hg_problem* problems, int count, int weighted,
                        void* workspace, size_t workspace_bytes, void* stream);

/* Launch configuration and autotuning (the paper's FFT benchmarking, "Fast
 * Fourier Transforms" section, shows throughput is set by the transform;
 * the tile schedule that runs it fastest depends on grid size and batch).
 * Each (ny, nx, batch class) -- batch < 8 or >= 8 -- has a column-tile
 * width (columns per column-pass workgroup) and a row-pass group size (rows
 * per workgroup), from a built-in table unless tuned or set.
 * hg_autotune times every compiled candidate on the device (weighted-GS
 * column pass, binary row pass, on a synthetic flat target in `workspace`),
 * keeps the fastest for later calls in this process and returns it.  It
 * synchronises `stream`.  hg_set_launch_config installs a configuration
 * (0, 0 restores the built-in table); an uncompiled one is rejected.
 * Configurations change speed only: results are identical up to the order
 * of floating-point partial sums in the NMSE reduction.                     */
size_t hg_autotune_workspace_size(int ny, int nx, int batch);
hg_status hg_autotune(int ny, int nx, int batch, int* col_tile, int* rows_per_group, void* workspace,
                      size_t workspace_bytes, void* stream);
hg_status hg_set_launch_config(int ny, int nx, int batch, int col_tile, int rows_per_group);
hg_status hg_get_launch_config(int ny, int nx, int batch, int* col_tile, int* rows_per_group);

/* Small problems (ny and nx each 64 or 128) run a whole hg_gs / hg_wgs call,
 * or a size class of hg_gs_batched, in one launch: one workgroup per
 * problem with the field resident in LDS.  enable = 0 selects the
 * multi-launch pipeline for them instead, 1 (the default, unless the
 * environment sets HG_SMALL_KERNEL=off) the single launch.  Process-wide;
 * results are identical up to the order of the NMSE partial sums. */
hg_status hg_set_small_fused(int enable);

/* Batched GS and weighted GS (hg_gs_batched) run each size class in chunks
 * of problems whose field planes together take at most field_bytes (at
 * least one problem per chunk, the class split into chunks of equal size as
 * far as the count allows), one chunk after another on the call's
 * stream, each through all its iterations.  A chunk that fits the GPU's
 * last-level cache (256 MB Infinity Cache on MI355X) keeps the field a pass
 * writes there for the next pass, instead of a round trip through HBM.
 * 0 runs each class whole.  Default 128 MiB, unless the environment sets
 * HG_BATCH_CHUNK_MB.  Batched OSPR (hg_ospr_batched) chunks the same way
 * (by its field planes).
 * Process-wide; results are identical for every chunk
 * size (each problem keeps its own random stream and its own sums, and the
 * kernel and tile choices follow the whole size class); the workspace size
 * does not change.  Single-launch small problems (each side 64 or 128) are
 * not chunked.  HG_ERR_INVALID_ARG beyond 1 TiB.
 * hg_get_batch_chunk returns the current value. */
hg_status hg_set_batch_chunk(size_t field_bytes);
size_t hg_get_batch_chunk(void);

/* Kernel of the GS / weighted GS column passes, process-wide:
 *   0  one column tile per workgroup (the default, unless the environment
 *      sets HG_COLUMN_KERNEL=persistent or =classic);
 *   1  a persistent, software-pipelined pass for batches of at least 2048
 *      column tiles (each workgroup streams its next tile into LDS while it
 *      transforms the current one);
 *   2  the classic one-tile kernels only.
 * Sizes or batches a kind does not cover use the next kind that does.
 * Results agree to rounding (identical arithmetic; the compiler may contract
 * it differently in each kernel). */
hg_status hg_set_column_kernel(int kind);

/* Kernel timing (instrumentation for benchmarks).  While enabled, every
 * launch of a column pass, row pass or set-up kernel made by this process
 * is bracketed by a pair of hipEvents on the stream it is launched on.
 * hg_timing_read waits for the recorded events, returns the summed device
 * time (ms) and launch count per category since the last read, and resets
 * them.  Enabling adds host work per launch; leave it off otherwise.        */
typedef struct hg_kernel_times {
  double col_ms, row_ms, setup_ms;
  long long col_launches, row_launches, setup_launches;
} hg_kernel_times;
void hg_timing_enable(int on);
hg_status hg_timing_read(hg_kernel_times* out);

/* Numeric status of the last GS / WGS / LT / OSPR call (single or batched)
 * that used `workspace`: synchronises `stream` (the call's stream), then
 * returns HG_ERR_NUMERIC if that call's NMSE finisher saw non-finite sums
 * (its nmse_out holds NaN there), else HG_OK.  The word lives in the first
 * bytes of the workspace; each call clears it on the stream before its
 * kernels run, so the answer belongs to the latest call enqueued with that
 * workspace.  NULL or misaligned workspace: HG_ERR_INVALID_ARG.            */
hg_status hg_numeric_status(const void* workspace, void* stream);

/* Holographic search ("Holographic Search Algorithms" section): direct
 * search (DS) and simulated annealing (SA) on phase SLMs, one hologram per
 * workgroup, `batch` holograms of one size per call.
 *   targets      [batch][ny][nx] float raw replay amplitudes, prepared as
 *                for hg_gs (scaled to sum T^2 = nx ny; binary symmetrised)
 *   ny, nx       8, 16, 32 or 64 (the replay field lives in registers)
 *   slm_levels   2..256 phase levels 2 pi k / L
 *   algorithm    HG_SEARCH_DS: raster sweeps trying every other level at
 *                each pixel, keeping a change when the error
 *                E = sum (|R| - T)^2 (unit-rms scale) falls by more than
 *                1e-12, until a sweep keeps none (or max_sweeps);
 *                HG_SEARCH_SA: one proposal per pixel per sweep, level
 *                (k + 1 + floor(u0 (L - 1))) mod L, kept when E falls or
 *                when u1 < exp(-dE / tau), tau = t0 alpha^(s - 1) in the
 *                units of E, for max_sweeps sweeps; u0, u1 = the top 24
 *                bits of words 0 and 1 of the Philox4x64-10 block at
 *                counter (y nx + x, s, 0, 0), key (seed, (b << 32) | 0x5A)
 *                for hologram b
 *   init_levels  [batch][ny][nx] uint8 start levels (< slm_levels), required
 *   levels_out   [batch][ny][nx] uint8 final levels
 *   error_out    [batch][max_sweeps + 1] doubles: E before the first sweep
 *                and after each (DS: repeated after the last sweep run)
 *   sweeps_out   nullable [batch] ints: sweeps run (DS: including the sweep
 *                that kept no change)
 *   workspace    hg_search_workspace_size(ny, nx, batch) bytes (256-aligned)
 * Errors as hg_gs (sizes outside the list: HG_ERR_UNSUPPORTED_SIZE).       */
enum hg_search_algorithm { HG_SEARCH_DS = 0, HG_SEARCH_SA = 1 };
size_t hg_search_workspace_size(int ny, int nx, int batch);
hg_status hg_search(const float* targets, int batch, int ny, int nx, int slm_levels, int algorithm, int max_sweeps,
                    double t0, double alpha, uint64_t seed, const uint8_t* init_levels, uint8_t* levels_out,
                    double* error_out, int* sweeps_out, void* workspace, size_t workspace_bytes, void* stream);

/* Weighted GS with no workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc).  Arguments, results and errors as hg_wgs; the
 * scratch that hg_wgs takes as `workspace` is instead a file-scope device
 * array of HG_STATIC_SCRATCH_BYTES (32 MiB) in the library, one copy per GPU
 * the library runs on, held until the process ends.  Its device address is
 * looked up once per device (hipGetSymbolAddress) on the first call made
 * with that device current; the current device must be the stream's.
 *  - Sizes: a call whose hg_workspace_size(HG_OP_WGS, ny, nx, iters)
 *    exceeds HG_STATIC_SCRATCH_BYTES is rejected with HG_ERR_WORKSPACE
 *    before any HIP call (a 1024 x 1024 grid fits up to about 1700
 *    iterations, 2048 x 2048 does not fit).
 *  - The call allocates nothing: no hipMalloc, hipFree or allocating
 *    library routine.
 *  - Every call on one GPU shares that GPU's array, which keeps the last
 *    call's contents (each call initialises what it reads).  Calls that
 *    overlap on one GPU (different streams, or host threads without
 *    ordering) race on it and give undefined results.
 *  - The numeric status word sits in the shared array too; a non-finite
 *    input is reported by NaN in nmse_out.                                 */
#define HG_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
hg_status hg_wgs_static(const float* target, int ny, int nx, int iters, int slm_levels, uint64_t seed,
                        const uint8_t* init_levels, const hg_complex* init_field,
                        double wavelength_m, double pitch_m, double z_m,
                        uint8_t* levels_out, hg_complex* slm_field_out, hg_complex* replay_out,
                        double* nmse_out, float* weights_inout, void* stream);

/* Static text for a status code, and the thread-local detail of the last
 * error raised on this thread ("" if none). */
const char* hg_status_string(hg_status status);
const char* hg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HOLOGEN_H */
