// Work decomposition shared by the host launch code and the device kernels.
#pragma once

// Threads per workgroup of the column passes and of the row passes.
#ifndef PSR_COL_THREADS
#define PSR_COL_THREADS 256
#endif
#ifndef PSR_ROW_THREADS
#define PSR_ROW_THREADS 512
#endif
#ifndef PSR_J0_THREADS
#define PSR_J0_THREADS 256
#endif
// The j0 passes below 256: smaller workgroups, more of them per CU.
#ifndef PSR_J0_THREADS_SMALL
#define PSR_J0_THREADS_SMALL 128
#endif
// Smallest grid size whose plane passes split each plane into two parts.
#ifndef PSR_PLANE_SPLIT_MIN
#define PSR_PLANE_SPLIT_MIN 256
#endif

namespace psr {

// Work split of a length-L line FFT: plan_TPL(L) threads per line, each
// holding plan_E(L) elements in registers.
__host__ __device__ constexpr int plan_E(int L) { return L < 16 ? L : 16; }
__host__ __device__ constexpr int plan_TPL(int L) { return L / plan_E(L); }
__host__ __device__ constexpr int imin(int a, int b) { return a < b ? a : b; }

// Column passes (FFT along j1 / j0, length res): tile_cols(res) lines per
// workgroup of cols_block(res) threads.
__host__ __device__ constexpr int tile_cols(int res) { return imin(res, PSR_COL_THREADS / plan_TPL(res)); }
__host__ __device__ constexpr int cols_block(int res) { return tile_cols(res) * plan_TPL(res); }

// The fused j0 passes (three transforms per line) may use their own tile.
__host__ __device__ constexpr int tile_j0(int res) {
  return imin(res, (res < 256 ? PSR_J0_THREADS_SMALL : PSR_J0_THREADS) / plan_TPL(res));
}
__host__ __device__ constexpr int j0_block(int res) { return tile_j0(res) * plan_TPL(res); }

// Row passes (splat + r2c and c2r + gather along j2; half-length complex
// lines of res/2): tile_rows(res) consecutive j1 lines of one j0 per
// workgroup of rows_block(res) threads. Points are binned by these tiles,
// two bins per tile (floor column b1 inside the tile, or on its last column,
// which also reaches the next tile): bin = b0 * 2 row_tiles(res) +
// 2 (b1 / tile_rows(res)) + (b1 is the tile's last column).
__host__ __device__ constexpr int tile_rows(int res) {
  // where a plane pass splits a plane of res <= 128 in two, bins must not be coarser than a part
  return imin(imin(res, PSR_ROW_THREADS / plan_TPL(res / 2)),
              (res >= PSR_PLANE_SPLIT_MIN && res <= 128) ? res / 2 : res);
}
__host__ __device__ constexpr int rows_block(int res) { return tile_rows(res) * plan_TPL(res / 2); }
// Workgroup size of the row passes. Up to 32 a row tile is the whole plane
// and its transforms take one thread per row (res threads); the workgroup
// is widened to 256 threads for the loops over the plane's points and
// samples, the threads beyond the rows transforming scratch rows.
__host__ __device__ constexpr int rows_wg(int res) { return res <= 32 ? 256 : rows_block(res); }
// LDS rows of a row-pass workgroup: the tile's rows plus the scratch rows
__host__ __device__ constexpr int rows_lds(int res) {
  return rows_wg(res) / plan_TPL(res / 2) > tile_rows(res) ? rows_wg(res) / plan_TPL(res / 2) : tile_rows(res);
}
__host__ __device__ constexpr int row_tiles(int res) { return res / tile_rows(res); }
__host__ __device__ constexpr int num_bins(int res) { return 2 * res * row_tiles(res); }

}  // namespace psr
