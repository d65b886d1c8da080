// Launch layer: the kernel configurations compiled for each transform length
// and the launchers that pick one at run time.  Each length lives in its own
// translation unit (hg_n<N>.hip) so the kernels build in parallel.
#pragma once
#include <algorithm>
#include <cstdlib>
#include <string>

#include "hg_kernels.hpp"

namespace hg {

// Column-tile widths C compiled for a column length N (threads per tile
// C * N / 16 between 64 and 1024).
__host__ __device__ constexpr bool col_ok(int N, int C) {
  switch (N) {
    case 64: return C == 16;
    case 128: return C == 8 || C == 16;
    case 256: return C == 4 || C == 8 || C == 16;
    case 512: return C == 4 || C == 8 || C == 16;
    case 1024: return C == 4 || C == 8 || C == 16;
    case 2048: return C == 2 || C == 4 || C == 8;
    case 4096: return C == 2 || C == 4;
    default: return false;
  }
}
// Rows per row-pass workgroup compiled for a row length N (128 or 256
// threads; and one 4-row group of two-wave rows, 512 threads, at N = 2048).
__host__ __device__ constexpr bool rpb_ok(int N, int RPB) {
  const int T = N / kE;
  return (RPB * T == 128 || RPB * T == 256) || (T >= 256 && RPB == 1) || (T == 128 && RPB == 4);
}

// Default rows per row-pass workgroup for a row length N: one 4-row group of
// 1024- or 2048-wide rows, 256 threads for shorter rows, one row beyond.
__host__ __device__ constexpr int default_rpb(int N) {
  return N / kE >= 256 ? 1 : (N / kE == 128 ? 4 : 256 / (N / kE));
}

// 16-bit field planes (Batch::f16) run their column passes in the tile
// kernel, whose 256-thread tiles exist for these column lengths (with the
// default tile width), and their row passes with default_rpb rows.
__host__ __device__ constexpr bool f16_ok(int ny) { return ny == 256 || ny == 512 || ny == 1024; }

// Kernel of the GS / weighted GS column passes (hg_set_column_kernel):
//   CK_TILE        one column tile per workgroup (k_colq) where its
//                  256-thread tile is compiled, else as CK_PERSISTENT;
//   CK_PERSISTENT  the persistent pipelined pass (k_colp) for batches of at
//                  least 2048 column tiles, else the classic kernels;
//   CK_CLASSIC     the classic kernels (k_col / k_colw) only.
enum ColumnKernel { CK_TILE = 0, CK_PERSISTENT = 1, CK_CLASSIC = 2 };
int column_kernel();

// Small problems (each side 64 or 128) run whole in one workgroup with the
// field resident in LDS (hg_small.hip) unless switched off (hg_set_small_fused).
inline bool small_ok(int ny, int nx) { return (ny == 64 || ny == 128) && (nx == 64 || nx == 128); }
bool small_enabled();
void launch_small(const Batch& bt, int B, bool fresnel, bool weighted, hipStream_t st);

template <int N> void launch_col_t(int C, const Batch& bt, int B, int mode, int arg, int adaptive,
                                   const float2* pin, float2* pout, hipStream_t st);
template <int N> void launch_setup_t(int C, const Batch& bt, int B, int weighted, hipStream_t st);
// Work a column pass needs launched before it (the weighted-GS mean of the
// pipelined pass); kept out of the pass's own timing.
template <int N> void launch_col_prep_t(int C, const Batch& bt, int B, int mode, int arg, hipStream_t st);
template <int N> void launch_row_t(int RPB, bool fresnel, int lk, const Batch& bt, int B, int mode, int arg,
                                   const float2* pin, float2* pout, hipStream_t st);
template <int N> void launch_twiddles_t(float2* tw, hipStream_t st);
template <int N> void launch_twiddles8_t(float2* tw, hipStream_t st);  // the 8-element plan (512 only)
template <int N> constexpr int twiddle_count() { return TwLayout<N, kE>::total(); }

}  // namespace hg
