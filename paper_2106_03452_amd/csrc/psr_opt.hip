// gfx950 kernels of the optimisation-based reconstruction loop around the
// solver (Peng et al., "Shape As Points", main Sec. 3.2): points sampled on
// the Marching Cubes mesh (the p_mesh of Eq. 5) with their backward, the
// bidirectional Chamfer loss of Eq. 5 with its gradient, and the connected
// components of the mesh for the resampling from the largest component.
//
// Sampling: FP64 face areas, an FP64 inclusive scan (block sums, their scan,
// block-local scans), then per sample a binary search of u0 * total and the
// barycentric weights (1 - sqrt(u1), sqrt(u1) (1 - u2), sqrt(u1) u2).
// Chamfer: exact nearest neighbours over spatially sorted tiles whose boxes
// let whole tiles be skipped (the brute-force result: equal distances go to
// the lower index); FP64 sums for the loss.
// Components: label propagation over the triangles (atomic minimum) with
// pointer jumping until no label changes, FP64 areas per label, and the
// label with the greatest area (ties: the lowest label).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "psr_opt.h"

namespace psr {
namespace opt {

constexpr int kScanPer = 4;                 // areas per thread of a scan block
constexpr int kScanBlock = 256 * kScanPer;  // areas per scan block

__global__ __launch_bounds__(256) void k_face_area(const float* __restrict__ v, const int32_t* __restrict__ f,
                                                   int64_t nf, const float* __restrict__ w, double* __restrict__ a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nf) return;
  const int64_t i0 = f[3 * i], i1 = f[3 * i + 1], i2 = f[3 * i + 2];
  const double ax = (double)v[3 * i1] - v[3 * i0], ay = (double)v[3 * i1 + 1] - v[3 * i0 + 1],
               az = (double)v[3 * i1 + 2] - v[3 * i0 + 2];
  const double bx = (double)v[3 * i2] - v[3 * i0], by = (double)v[3 * i2 + 1] - v[3 * i0 + 1],
               bz = (double)v[3 * i2 + 2] - v[3 * i0 + 2];
  const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
  double ar = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
  if (w) ar *= (double)w[i];
  a[i] = ar;
}

__device__ __forceinline__ double block_excl_scan(double v, double* sh, double& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    const double x = t >= d ? sh[t - d] : 0.0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  total = sh[255];
  const double excl = sh[t] - v;
  __syncthreads();
  return excl;
}

// block b: the sum of its kScanBlock areas
__global__ __launch_bounds__(256) void k_scan_sums(const double* __restrict__ a, int64_t n, double* __restrict__ bs) {
  __shared__ double sh[256];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  double s = 0.0;
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < n) s += a[base + k];
  double tot;
  block_excl_scan(s, sh, tot);
  if (threadIdx.x == 0) bs[blockIdx.x] = tot;
}

// exclusive scan of the block sums in place (one workgroup); the grand total after them
__global__ __launch_bounds__(256) void k_scan_tops(double* __restrict__ bs, int nb) {
  __shared__ double sh[256];
  double carry = 0.0;
  for (int c = 0; c < nb; c += 256) {
    const int i = c + threadIdx.x;
    const double v = i < nb ? bs[i] : 0.0;
    double tot;
    const double ex = block_excl_scan(v, sh, tot);
    if (i < nb) bs[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) bs[nb] = carry;
}

// inclusive running sums of the areas
__global__ __launch_bounds__(256) void k_scan_local(double* __restrict__ a, int64_t n, const double* __restrict__ bs) {
  __shared__ double sh[256];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  double v[kScanPer], s = 0.0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < n ? a[base + k] : 0.0;
    s += v[k];
  }
  double tot;
  double run = bs[blockIdx.x] + block_excl_scan(s, sh, tot);
  for (int k = 0; k < kScanPer; ++k) {
    run += v[k];
    if (base + k < n) a[base + k] = run;
  }
}

__global__ __launch_bounds__(256) void k_sample(const float* __restrict__ v, const float* __restrict__ vn,
                                                const int32_t* __restrict__ f, int64_t nf,
                                                const double* __restrict__ csum, const float* __restrict__ u,
                                                int64_t m, float* __restrict__ pts, float* __restrict__ nrm,
                                                int32_t* __restrict__ face, float* __restrict__ bary) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const double t = (double)u[3 * i] * csum[nf - 1];
  // first face whose running sum exceeds t
  int64_t lo = 0, hi = nf - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (csum[mid] > t) hi = mid;
    else lo = mid + 1;
  }
  const float s = sqrtf(u[3 * i + 1]), u2 = u[3 * i + 2];
  const float b0 = 1.0f - s, b1 = s * (1.0f - u2), b2 = s * u2;
  const int64_t i0 = f[3 * lo], i1 = f[3 * lo + 1], i2 = f[3 * lo + 2];
#pragma unroll
  for (int d = 0; d < 3; ++d) pts[3 * i + d] = b0 * v[3 * i0 + d] + b1 * v[3 * i1 + d] + b2 * v[3 * i2 + d];
  if (nrm) {
    float n[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) n[d] = b0 * vn[3 * i0 + d] + b1 * vn[3 * i1 + d] + b2 * vn[3 * i2 + d];
    const float il = rsqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) nrm[3 * i + d] = n[d] * il;
  }
  face[i] = (int32_t)lo;
  bary[3 * i] = b0;
  bary[3 * i + 1] = b1;
  bary[3 * i + 2] = b2;
}

__global__ __launch_bounds__(256) void k_fill0(float* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) x[i] = 0.0f;
}

__global__ __launch_bounds__(256) void k_sample_bwd(const int32_t* __restrict__ f, const int32_t* __restrict__ face,
                                                    const float* __restrict__ bary, const float* __restrict__ dp,
                                                    int64_t m, float* __restrict__ dv) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const int64_t fi = face[i];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int64_t vi = f[3 * fi + k];
    const float b = bary[3 * i + k];
#pragma unroll
    for (int d = 0; d < 3; ++d) atomicAdd(&dv[3 * vi + d], b * dp[3 * i + d]);
  }
}

// ---------------------------------------------------------------------------
// Nearest neighbours for the Chamfer loss: an exact search that skips whole
// tiles of the reference cloud. Both clouds are counting-sorted into
// Morton-ordered cells of a grid over [0,1)^3 (16^3 to 64^3 cells by cloud
// size; points outside fall into the border cells), cut into tiles of
// kNnTile sorted points, and each tile gets its bounding box. A query group
// (kNnTile sorted queries) visits the reference tiles nearest its own box
// first and stops where every remaining box is farther than each query's
// best so far; a tile is skipped when no query's point-to-box bound reaches
// its best. The bounds use the same FP32
// operations as the distances (monotone rounding), so a skipped point is
// strictly farther than a distance already found: the result is the
// brute-force one, the squared FP32 distance minimised with equal distances
// going to the lower reference index.
// ---------------------------------------------------------------------------

// squared length, evaluated the same way for distances and for bounds
__device__ __forceinline__ float nn_d2(float ax, float ay, float az) {
  return __fmaf_rn(az, az, __fmaf_rn(ay, ay, ax * ax));
}

__device__ __forceinline__ int nn_cell_coord(float v, int cb) {
  const int top = (1 << cb) - 1;
  const float c = v * (float)(1 << cb);
  if (!(c >= 0.0f)) return 0;  // also NaN
  return c >= (float)top ? top : (int)c;
}

__device__ __forceinline__ uint32_t nn_spread(uint32_t v) {  // up to 8 bits -> every third bit
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Morton index of the point's cell in the 2^cb per axis grid
__device__ __forceinline__ int nn_key(float x, float y, float z, int cb) {
  return (int)(nn_spread(nn_cell_coord(x, cb)) | (nn_spread(nn_cell_coord(y, cb)) << 1) |
               (nn_spread(nn_cell_coord(z, cb)) << 2));
}

__global__ __launch_bounds__(256) void k_nn_zero(int* __restrict__ cnt, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) cnt[i] = 0;
}

// cell counts of both clouds (x: points [0, nx), y: the next ny)
__global__ __launch_bounds__(256) void k_nn_count(const float* __restrict__ x, int64_t nx,
                                                  const float* __restrict__ y, int64_t ny, int* __restrict__ cnt,
                                                  int cb) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nx + ny) return;
  const bool isy = i >= nx;
  const float* p = isy ? y + 3 * (i - nx) : x + 3 * i;
  atomicAdd(&cnt[(isy ? 1 << (3 * cb) : 0) + nn_key(p[0], p[1], p[2], cb)], 1);
}

// exclusive scan of one cloud's nc cell counts in place (workgroup = cloud;
// each thread owns nc / 1024 consecutive counts)
__global__ __launch_bounds__(1024) void k_nn_scan(int* __restrict__ cnt, int nc) {
  __shared__ int wsum[16];
  int4* c = reinterpret_cast<int4*>(cnt + (int64_t)blockIdx.x * nc);
  const int per4 = nc / 4096;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  int s = 0;
  for (int k = 0; k < per4; ++k) {
    const int4 a = c[t * per4 + k];
    s += a.x + a.y + a.z + a.w;
  }
  int inc = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(inc, d, 64);
    if (lane >= d) inc += u;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  int run = inc - s;
  for (int v = 0; v < wid; ++v) run += wsum[v];
  for (int k = 0; k < per4; ++k) {
    const int4 a = c[t * per4 + k];
    int4 o;
    o.x = run;
    o.y = o.x + a.x;
    o.z = o.y + a.y;
    o.w = o.z + a.z;
    run = o.w + a.w;
    c[t * per4 + k] = o;
  }
}

// points into cell order: (x, y, z, original index bits); the offsets end as
// the cells' ends
__global__ __launch_bounds__(256) void k_nn_scatter(const float* __restrict__ x, int64_t nx,
                                                    const float* __restrict__ y, int64_t ny, int* __restrict__ cnt,
                                                    float4* __restrict__ sx, float4* __restrict__ sy, int cb) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nx + ny) return;
  const bool isy = i >= nx;
  const int64_t k = isy ? i - nx : i;
  const float* p = (isy ? y : x) + 3 * k;
  const float a = p[0], b = p[1], c = p[2];
  const int pos = atomicAdd(&cnt[(isy ? 1 << (3 * cb) : 0) + nn_key(a, b, c, cb)], 1);
  (isy ? sy : sx)[pos] = make_float4(a, b, c, __int_as_float((int)k));
}

// bounding box of each tile (one wavefront per tile; NaN coordinates ignored)
__global__ __launch_bounds__(64) void k_nn_box(const float4* __restrict__ sx, int64_t nx,
                                               const float4* __restrict__ sy, int64_t ny, int64_t tx,
                                               float4* __restrict__ bx, float4* __restrict__ by) {
  const int64_t tb = blockIdx.x;
  const bool isy = tb >= tx;
  const int64_t t = isy ? tb - tx : tb, n = isy ? ny : nx;
  const int64_t i = t * kNnTile + threadIdx.x;
  const float inf = __int_as_float(0x7f800000);
  float lo[3] = {inf, inf, inf}, hi[3] = {-inf, -inf, -inf};
  if (i < n) {
    const float4 p = (isy ? sy : sx)[i];
    lo[0] = hi[0] = p.x;
    lo[1] = hi[1] = p.y;
    lo[2] = hi[2] = p.z;
    if (p.x != p.x) lo[0] = inf, hi[0] = -inf;
    if (p.y != p.y) lo[1] = inf, hi[1] = -inf;
    if (p.z != p.z) lo[2] = inf, hi[2] = -inf;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], d, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], d, 64));
    }
  }
  if (threadIdx.x == 0) {
    float4* b = (isy ? by : bx) + 2 * t;
    b[0] = make_float4(lo[0], lo[1], lo[2], 0.0f);
    b[1] = make_float4(hi[0], hi[1], hi[2], 0.0f);
  }
}

// float <-> int keys whose integer order is the float order (NaN excluded)
__device__ __forceinline__ int nn_ord(float f) {
  const int i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float nn_unord(int k) { return __int_as_float(k >= 0 ? k : k ^ 0x7fffffff); }

constexpr int kNnSmallBits = 4;                           // 16^3 cells
constexpr int kNnSmallCells = 1 << (3 * kNnSmallBits);
constexpr int kNnSmallTiles = 512;                        // clouds of up to 32768 points

// Small clouds (up to kNnSmallTiles tiles): the whole counting sort of one
// cloud in one workgroup (counts, scan and ranks in LDS), the tile boxes from
// LDS minima / maxima during the scatter; writes the sorted points, the
// cells' ends and the boxes, as the separate kernels do for larger clouds.
__global__ __launch_bounds__(1024) void k_nn_sort_small(const float* __restrict__ x, int64_t nx,
                                                        const float* __restrict__ y, int64_t ny,
                                                        int* __restrict__ cnt, float4* __restrict__ sx,
                                                        float4* __restrict__ sy, float4* __restrict__ bx,
                                                        float4* __restrict__ by) {
  __shared__ int hist[kNnSmallCells];
  __shared__ int bmin[3][kNnSmallTiles], bmax[3][kNnSmallTiles];
  __shared__ int wsum[16];
  const bool isy = blockIdx.x == 1;
  const float* p = isy ? y : x;
  const int n = (int)(isy ? ny : nx);
  float4* srt = isy ? sy : sx;
  float4* box = isy ? by : bx;
  int* ends = cnt + (isy ? kNnSmallCells : 0);
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int nt = (n + kNnTile - 1) / kNnTile;
  for (int k = t; k < kNnSmallCells; k += 1024) hist[k] = 0;
  for (int k = t; k < kNnSmallTiles; k += 1024) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      bmin[a][k] = 0x7fffffff;
      bmax[a][k] = (int)0x80000000;
    }
  }
  __syncthreads();
#pragma unroll 4
  for (int i = t; i < n; i += 1024) atomicAdd(&hist[nn_key(p[3 * i], p[3 * i + 1], p[3 * i + 2], kNnSmallBits)], 1);
  __syncthreads();
  {
    constexpr int PER = kNnSmallCells / 1024;
    int v[PER], s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      v[k] = hist[t * PER + k];
      s += v[k];
    }
    int inc = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int u = __shfl_up(inc, d, 64);
      if (lane >= d) inc += u;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int run = inc - s;
    for (int u = 0; u < wid; ++u) run += wsum[u];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      hist[t * PER + k] = run;
      run += v[k];
    }
  }
  __syncthreads();
#pragma unroll 4
  for (int i = t; i < n; i += 1024) {
    const float a = p[3 * i], b = p[3 * i + 1], c = p[3 * i + 2];
    const int pos = atomicAdd(&hist[nn_key(a, b, c, kNnSmallBits)], 1);
    srt[pos] = make_float4(a, b, c, __int_as_float(i));
    const int tl = pos / kNnTile;
    const float v[3] = {a, b, c};
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      if (v[e] == v[e]) {
        atomicMin(&bmin[e][tl], nn_ord(v[e]));
        atomicMax(&bmax[e][tl], nn_ord(v[e]));
      }
    }
  }
  __syncthreads();
  for (int k = t; k < kNnSmallCells; k += 1024) ends[k] = hist[k];
  const float inf = __int_as_float(0x7f800000);
  for (int k = t; k < nt; k += 1024) {
    float lo[3], hi[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      lo[e] = bmin[e][k] == 0x7fffffff ? inf : nn_unord(bmin[e][k]);
      hi[e] = bmax[e][k] == (int)0x80000000 ? -inf : nn_unord(bmax[e][k]);
    }
    box[2 * k] = make_float4(lo[0], lo[1], lo[2], 0.0f);
    box[2 * k + 1] = make_float4(hi[0], hi[1], hi[2], 0.0f);
  }
}

// squared distance bound from point q to box [lo, hi]
__device__ __forceinline__ float nn_box_d2(float qx, float qy, float qz, const float4& lo, const float4& hi) {
  return nn_d2(fmaxf(fmaxf(lo.x - qx, qx - hi.x), 0.0f), fmaxf(fmaxf(lo.y - qy, qy - hi.y), 0.0f),
               fmaxf(fmaxf(lo.z - qz, qz - hi.z), 0.0f));
}

// squared distance bound between boxes [al, ah] and [bl, bh]
__device__ __forceinline__ float nn_boxbox_d2(const float3& al, const float3& ah, const float4& bl, const float4& bh) {
  return nn_d2(fmaxf(fmaxf(bl.x - ah.x, al.x - bh.x), 0.0f), fmaxf(fmaxf(bl.y - ah.y, al.y - bh.y), 0.0f),
               fmaxf(fmaxf(bl.z - ah.z, al.z - bh.z), 0.0f));
}

// orders this wavefront's LDS writes before its own later reads (and the
// reverse) without a workgroup barrier: the wavefronts of a query group take
// different numbers of tiles
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct NnSide {
  const float4* q;   // sorted queries
  int64_t nq;
  const float4* r;   // sorted references
  const float4* box; // reference tile boxes (lo, hi)
  const int* rend;   // reference cell ends
  int64_t nr;
  int32_t* nn;
  float* dist;
};

constexpr int kNnWaves = 8;                  // wavefronts per query group
constexpr int kNnBlock = 64 * kNnWaves;       // threads of a query workgroup
constexpr int kNnCand = 512;  // tiles tested per pass: the capacity of the candidate list

// One group of kNnTile sorted queries per workgroup, kNnWaves wavefronts
// holding the same queries; groups [0, gx) search y from x, the rest x from y.
// 1. Each wavefront scans one of the kNnWaves tiles around the reference cell of
//    the group's first query; the largest best distance of the group then
//    bounds every neighbour.
// 2. The tiles whose box lies within that bound of the group's box are listed
//    in LDS with their boxes and sorted by the box-to-box bound (bitonic).
// 3. The wavefronts take the sorted tiles in turn (the next one's points
//    prefetched) and stop at the first whose box bound exceeds every lane's
//    best; a tile is passed over when no lane's point-to-box bound reaches
//    that lane's best. A lane's best is the lowest distance any wavefront has
//    reached for it (published in LDS after every tile).
// 4. The kNnWaves results per query are merged (lower distance, then lower
//    index).
__global__ __launch_bounds__(kNnBlock) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_nn_query(
    const NnSide A, const NnSide Bs, int64_t gx, int cb) {
  __shared__ float4 stg[kNnWaves][kNnTile];
  __shared__ float shb[kNnWaves][kNnTile];
  __shared__ int sidx[kNnWaves][kNnTile];
  __shared__ float4 cbox[kNnCand][2];  // lo (w: box bound), hi (w: tile - c0)
  __shared__ unsigned long long ckey[kNnCand];  // (box bound, slot in cbox)
  __shared__ int ncand;
  const bool second = blockIdx.x >= gx;
  const NnSide S = second ? Bs : A;
  const int64_t g = second ? blockIdx.x - gx : blockIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float inf = __int_as_float(0x7f800000), nan = __int_as_float(0x7fc00000);
  const int64_t gi = g * kNnTile + lane;
  const bool active = gi < S.nq;
  const float4 q = active ? S.q[gi] : make_float4(nan, nan, nan, 0.0f);
  // the group's box (NaN coordinates ignored)
  float3 ql = make_float3(inf, inf, inf), qh = make_float3(-inf, -inf, -inf);
  if (q.x == q.x) ql.x = qh.x = q.x;
  if (q.y == q.y) ql.y = qh.y = q.y;
  if (q.z == q.z) ql.z = qh.z = q.z;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    ql.x = fminf(ql.x, __shfl_xor(ql.x, d, 64));
    ql.y = fminf(ql.y, __shfl_xor(ql.y, d, 64));
    ql.z = fminf(ql.z, __shfl_xor(ql.z, d, 64));
    qh.x = fmaxf(qh.x, __shfl_xor(qh.x, d, 64));
    qh.y = fmaxf(qh.y, __shfl_xor(qh.y, d, 64));
    qh.z = fmaxf(qh.z, __shfl_xor(qh.z, d, 64));
  }
  const int64_t ntr = (S.nr + kNnTile - 1) / kNnTile;
  const int key = __builtin_amdgcn_readfirstlane(nn_key(q.x, q.y, q.z, cb));
  int64_t t0 = S.rend[key] / kNnTile;
  t0 = t0 > ntr - 1 ? ntr - 1 : t0;
  int64_t s0 = t0 - kNnWaves / 2 + 1 > ntr - kNnWaves ? ntr - kNnWaves : t0 - kNnWaves / 2 + 1;
  s0 = s0 < 0 ? 0 : s0;
  const int64_t s1 = s0 + kNnWaves - 1;  // the start tiles [s0, s1] (fewer when ntr < kNnWaves)
  float best = inf;
  int bi = 0x7fffffff;
  auto publish = [&]() { __hip_atomic_store(&shb[w][lane], best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); };
  // the lowest distance reached for this query by any wavefront so far
  auto reached = [&]() {
    float u = best;
#pragma unroll
    for (int v = 0; v < kNnWaves; ++v)
      u = fminf(u, __hip_atomic_load(&shb[v][lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
    return u;
  };
  auto group_bound = [&](float u) {
    float b = active ? u : 0.0f;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) b = fmaxf(b, __shfl_xor(b, d, 64));
    return b;
  };
  // this lane's point of tile t; a short last tile is padded with points at
  // infinity and the largest index, which never win
  auto tile_point = [&](int64_t t) {
    const int64_t i = t * kNnTile + lane;
    return i < S.nr ? S.r[i] : make_float4(inf, inf, inf, __int_as_float(0x7fffffff));
  };
  auto scan_tile = [&](const float4& p) {
    wave_sync();
    stg[w][lane] = p;
    wave_sync();
    // sixteen LDS reads in flight per batch
#pragma unroll 1
    for (int k0 = 0; k0 < kNnTile; k0 += 16) {
      float4 e[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) e[u] = stg[w][k0 + u];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const float d = nn_d2(e[u].x - q.x, e[u].y - q.y, e[u].z - q.z);
        const int j = __float_as_int(e[u].w);
        const bool better = (d < best) | ((d == best) & (j < bi));
        best = better ? d : best;
        bi = better ? j : bi;
      }
    }
    publish();
  };
  scan_tile(tile_point(s0 + w < ntr ? s0 + w : ntr - 1));
  __syncthreads();
  float bound = group_bound(reached());
  for (int64_t c0 = 0; c0 < ntr; c0 += kNnCand) {
    if (threadIdx.x == 0) ncand = 0;
    __syncthreads();
    const int64_t c1 = c0 + kNnCand < ntr ? c0 + kNnCand : ntr;
    for (int64_t t = c0 + threadIdx.x; t < c1; t += kNnBlock) {
      if (t >= s0 && t <= s1) continue;
      const float4 lo = S.box[2 * t], hi = S.box[2 * t + 1];
      const float lb = nn_boxbox_d2(ql, qh, lo, hi);
      if (lb <= bound) {
        const int k = atomicAdd(&ncand, 1);
        cbox[k][0] = make_float4(lo.x, lo.y, lo.z, lb);
        cbox[k][1] = make_float4(hi.x, hi.y, hi.z, __int_as_float((int)(t - c0)));
        ckey[k] = ((unsigned long long)__float_as_uint(lb) << 32) | (uint32_t)k;
      }
    }
    __syncthreads();
    const int nc = ncand;
    int np2 = 1;
    while (np2 < nc) np2 <<= 1;
    for (int i = nc + threadIdx.x; i < np2; i += kNnBlock) ckey[i] = ~0ull;
    __syncthreads();
    // ascending bitonic sort of the keys: the nearest boxes first
    for (int k = 2; k <= np2; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < np2; i += kNnBlock) {
          const int l = i ^ j;
          if (l > i) {
            const unsigned long long a = ckey[i], b = ckey[l];
            if ((a > b) == ((i & k) == 0)) {
              ckey[i] = b;
              ckey[l] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    auto slot = [&](int i) { return (int)(ckey[i] & 0xffffffffu); };
    float4 pf = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (w < nc) pf = tile_point(c0 + __float_as_int(cbox[slot(w)][1].w));
    for (int i = w; i < nc; i += kNnWaves) {
      const int k = slot(i);
      const float4 lo = cbox[k][0], hi = cbox[k][1];
      const float4 cur = pf;
      if (i + kNnWaves < nc) pf = tile_point(c0 + __float_as_int(cbox[slot(i + kNnWaves)][1].w));
      const float ub = reached();
      if (lo.w > group_bound(ub)) break;  // every later box is farther
      const bool need = active && nn_box_d2(q.x, q.y, q.z, lo, hi) <= ub;
      if (__any(need)) scan_tile(cur);
    }
    __syncthreads();
    bound = group_bound(reached());
  }
  sidx[w][lane] = bi;
  publish();
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int v = 1; v < kNnWaves; ++v) {
      const float d = shb[v][lane];
      const int j = sidx[v][lane];
      const bool better = (d < best) | ((d == best) & (j < bi));
      best = better ? d : best;
      bi = better ? j : bi;
    }
    if (active) {
      const int qi = __float_as_int(q.w);
      S.nn[qi] = bi == 0x7fffffff ? -1 : bi;
      S.dist[qi] = best;
    }
  }
}

// loss = mean(d_x) + mean(d_y), FP64 sums in a fixed order by point index
// (one workgroup: strided per-thread sums, then a fixed tree), so the loss
// does not depend on the order the search sorted the points in
__global__ __launch_bounds__(1024) void k_chamfer_loss(const float* __restrict__ dx, int64_t nx,
                                                       const float* __restrict__ dy, int64_t ny,
                                                       double* __restrict__ loss) {
  __shared__ double sh[16];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0;
#pragma unroll 8
  for (int64_t i = t; i < nx; i += 1024) a += dx[i];
#pragma unroll 8
  for (int64_t i = t; i < ny; i += 1024) b += dy[i];
  double v = a / (double)nx + b / (double)ny;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  if (t == 0) {
    double tot = 0.0;
    for (int w = 0; w < 16; ++w) tot += sh[w];
    *loss = tot;
  }
}

__global__ __launch_bounds__(256) void k_chamfer_bwd_x(const float* __restrict__ x, int64_t nx,
                                                       const float* __restrict__ y, const int32_t* __restrict__ nnx,
                                                       float* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nx) return;
  const int64_t j = nnx[i];
  const float s = 2.0f / (float)nx;
  if (j < 0) {  // no neighbour: the query holds NaN
#pragma unroll
    for (int d = 0; d < 3; ++d) g[3 * i + d] = __int_as_float(0x7fc00000);
    return;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) g[3 * i + d] = s * (x[3 * i + d] - y[3 * j + d]);
}

__global__ __launch_bounds__(256) void k_chamfer_bwd_y(const float* __restrict__ x, const float* __restrict__ y,
                                                       int64_t ny, const int32_t* __restrict__ nny,
                                                       float* __restrict__ g) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= ny) return;
  const int64_t i = nny[j];
  if (i < 0) return;  // no neighbour: the target point holds NaN
  const float s = 2.0f / (float)ny;
#pragma unroll
  for (int d = 0; d < 3; ++d) atomicAdd(&g[3 * i + d], s * (x[3 * i + d] - y[3 * j + d]));
}

__global__ void k_set_int(int32_t* __restrict__ p, int32_t v) { *p = v; }

__global__ __launch_bounds__(256) void k_lab_init(int32_t* __restrict__ lab, int64_t nv) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < nv) lab[i] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_lab_faces(const int32_t* __restrict__ f, int64_t nf, int32_t* __restrict__ lab,
                                                   int32_t* __restrict__ changed) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nf) return;
  const int32_t a = f[3 * i], b = f[3 * i + 1], c = f[3 * i + 2];
  const int32_t la = lab[a], lb = lab[b], lc = lab[c];
  const int32_t m = la < lb ? (la < lc ? la : lc) : (lb < lc ? lb : lc);
  bool ch = false;
  if (la > m) ch |= atomicMin(&lab[a], m) > m;
  if (lb > m) ch |= atomicMin(&lab[b], m) > m;
  if (lc > m) ch |= atomicMin(&lab[c], m) > m;
  if (ch) atomicOr(changed, 1);
}

// pointer jumping: labels only decrease and always name a vertex of the component
__global__ __launch_bounds__(256) void k_lab_jump(int32_t* __restrict__ lab, int64_t nv) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nv) return;
  const int32_t l = lab[i];
  const int32_t ll = lab[l];
  if (ll < l) atomicMin(&lab[i], ll);
}

__global__ __launch_bounds__(256) void k_fill0d(double* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) x[i] = 0.0;
}

// Area per label. A mesh is mostly one or a few components, so the 64
// triangles of a wavefront usually share a label: they are then summed by
// shuffles and added with one atomic instead of 64 on the same address.
__global__ __launch_bounds__(256) void k_comp_area(const int32_t* __restrict__ f, int64_t nf,
                                                   const int32_t* __restrict__ lab, const double* __restrict__ area,
                                                   double* __restrict__ carea) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool ok = i < nf;
  const int l = ok ? lab[f[3 * i]] : -1;
  double a = ok ? area[i] : 0.0;
  const int l0 = __builtin_amdgcn_readfirstlane(l);  // lane 0: the wavefront's first triangle
  if (__all(l == l0 || !ok)) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) a += __shfl_xor(a, d, 64);
    if ((threadIdx.x & 63) == 0 && l0 >= 0) atomicAdd(&carea[l0], a);
  } else if (ok) {
    atomicAdd(&carea[l], a);
  }
}

// the label of greatest area (ties: the lowest label), one workgroup
__global__ __launch_bounds__(256) void k_comp_best(const double* __restrict__ carea, int64_t nv,
                                                   int32_t* __restrict__ best) {
  __shared__ double sa[256];
  __shared__ int64_t sl[256];
  double a = -1.0;
  int64_t l = nv;
  for (int64_t i = threadIdx.x; i < nv; i += 256) {
    if (carea[i] > a) {  // increasing i: the first of equal areas stays
      a = carea[i];
      l = i;
    }
  }
  sa[threadIdx.x] = a;
  sl[threadIdx.x] = l;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) {
      const double ob = sa[threadIdx.x + d];
      const int64_t ol = sl[threadIdx.x + d];
      if (ob > sa[threadIdx.x] || (ob == sa[threadIdx.x] && ol < sl[threadIdx.x])) {
        sa[threadIdx.x] = ob;
        sl[threadIdx.x] = ol;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *best = (int32_t)sl[0];
}

__global__ __launch_bounds__(256) void k_face_mask(const int32_t* __restrict__ f, int64_t nf,
                                                   const int32_t* __restrict__ lab, const int32_t* __restrict__ best,
                                                   float* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nf) return;
  w[i] = lab[f[3 * i]] == *best ? 1.0f : 0.0f;
}

static inline int nb256(int64_t n) { return (int)((n + 255) / 256); }

SampleLayout sample_layout(int64_t nf) {
  SampleLayout L;
  const int64_t nb = (nf + kScanBlock - 1) / kScanBlock;
  L.csum = 0;
  L.bs = align(nf * 8);
  L.total = L.bs + align((nb + 1) * 8);
  return L;
}

int run_sample(const float* v, const float* vn, const int32_t* f, int64_t nf, const float* w, const float* u,
               int64_t m, float* pts, float* nrm, int32_t* face, float* bary, void* ws, hipStream_t s) {
  const SampleLayout L = sample_layout(nf);
  double* a = reinterpret_cast<double*>(static_cast<char*>(ws) + L.csum);
  double* bs = reinterpret_cast<double*>(static_cast<char*>(ws) + L.bs);
  const int nb = (int)((nf + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(k_face_area, dim3(nb256(nf)), dim3(256), 0, s, v, f, nf, w, a);
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(256), 0, s, a, nf, bs);
  hipLaunchKernelGGL(k_scan_tops, dim3(1), dim3(256), 0, s, bs, nb);
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(256), 0, s, a, nf, bs);
  if (m > 0) hipLaunchKernelGGL(k_sample, dim3(nb256(m)), dim3(256), 0, s, v, vn, f, nf, a, u, m, pts, nrm, face, bary);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int run_sample_backward(const int32_t* f, int64_t nv, const int32_t* face, const float* bary, const float* dp,
                        int64_t m, float* dv, hipStream_t s) {
  hipLaunchKernelGGL(k_fill0, dim3(256), dim3(256), 0, s, dv, 3 * nv);
  if (m > 0) hipLaunchKernelGGL(k_sample_bwd, dim3(nb256(m)), dim3(256), 0, s, f, face, bary, dp, m, dv);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

NnLayout nn_layout(int64_t nx, int64_t ny) {
  NnLayout L;
  const int64_t tx = (nx + kNnTile - 1) / kNnTile, ty = (ny + kNnTile - 1) / kNnTile;
  L.cell_bits = nn_cell_bits(nx, ny);
  L.cnt = 0;
  L.srt_x = align(2 * ((int64_t)1 << (3 * L.cell_bits)) * 4);
  L.srt_y = L.srt_x + align(nx * 16);
  L.box_x = L.srt_y + align(ny * 16);
  L.box_y = L.box_x + align(tx * 32);
  L.total = L.box_y + align(ty * 32);
  return L;
}

size_t chamfer_ws(int64_t nx, int64_t ny) { return nn_layout(nx, ny).total; }

int run_chamfer(const float* x, int64_t nx, const float* y, int64_t ny, int32_t* nnx, float* dx, int32_t* nny,
                float* dy, double* loss, void* ws, hipStream_t s) {
  const NnLayout L = nn_layout(nx, ny);
  char* b = static_cast<char*>(ws);
  int* cnt = reinterpret_cast<int*>(b + L.cnt);
  float4* sx = reinterpret_cast<float4*>(b + L.srt_x);
  float4* sy = reinterpret_cast<float4*>(b + L.srt_y);
  float4* bx = reinterpret_cast<float4*>(b + L.box_x);
  float4* by = reinterpret_cast<float4*>(b + L.box_y);
  const int64_t tx = (nx + kNnTile - 1) / kNnTile, ty = (ny + kNnTile - 1) / kNnTile;
  const int cb = L.cell_bits, nc = 1 << (3 * cb);
  static_assert(kNnSmallTiles * kNnTile == 32768, "the small-cloud sort covers the clouds given 16^3 cells");
  if (cb == kNnSmallBits && tx <= kNnSmallTiles && ty <= kNnSmallTiles) {
    hipLaunchKernelGGL(k_nn_sort_small, dim3(2), dim3(1024), 0, s, x, nx, y, ny, cnt, sx, sy, bx, by);
  } else {
    hipLaunchKernelGGL(k_nn_zero, dim3(64), dim3(256), 0, s, cnt, 2 * nc);
    hipLaunchKernelGGL(k_nn_count, dim3(nb256(nx + ny)), dim3(256), 0, s, x, nx, y, ny, cnt, cb);
    hipLaunchKernelGGL(k_nn_scan, dim3(2), dim3(1024), 0, s, cnt, nc);
    hipLaunchKernelGGL(k_nn_scatter, dim3(nb256(nx + ny)), dim3(256), 0, s, x, nx, y, ny, cnt, sx, sy, cb);
    hipLaunchKernelGGL(k_nn_box, dim3(tx + ty), dim3(64), 0, s, sx, nx, sy, ny, tx, bx, by);
  }
  const NnSide A{sx, nx, sy, by, cnt + nc, ny, nnx, dx};  // samples x against the target y
  const NnSide B{sy, ny, sx, bx, cnt, nx, nny, dy};       // and back
  hipLaunchKernelGGL(k_nn_query, dim3(tx + ty), dim3(kNnBlock), 0, s, A, B, tx, cb);
  if (loss) hipLaunchKernelGGL(k_chamfer_loss, dim3(1), dim3(1024), 0, s, dx, nx, dy, ny, loss);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int run_chamfer_backward(const float* x, int64_t nx, const float* y, int64_t ny, const int32_t* nnx,
                         const int32_t* nny, float* g, hipStream_t s) {
  hipLaunchKernelGGL(k_chamfer_bwd_x, dim3(nb256(nx)), dim3(256), 0, s, x, nx, y, nnx, g);
  hipLaunchKernelGGL(k_chamfer_bwd_y, dim3(nb256(ny)), dim3(256), 0, s, x, y, ny, nny, g);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// Adam (Kingma and Ba): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
// p <- p - (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps); the bias
// corrections come from the host in double precision.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, int64_t n, float b1, float b2,
                                              float step, float inv_sqrt_bc2, float eps, int wrap) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  float pi = p[i] - step * mi / (sqrtf(vi) * inv_sqrt_bc2 + eps);
  if (wrap) pi -= floorf(pi);
  p[i] = pi;
}

int run_adam(float* p, float* m, float* v, const float* g, int64_t n, int64_t t, float lr, float b1, float b2,
             float eps, bool wrap, hipStream_t s) {
  const double bc1 = 1.0 - std::pow((double)b1, (double)t), bc2 = 1.0 - std::pow((double)b2, (double)t);
  if (n > 0)
    hipLaunchKernelGGL(k_adam, dim3(nb256(n)), dim3(256), 0, s, p, m, v, g, n, b1, b2, (float)(lr / bc1),
                       (float)(1.0 / std::sqrt(bc2)), eps, wrap ? 1 : 0);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

CompLayout comp_layout(int64_t nv, int64_t nf) {
  CompLayout L;
  L.flag = 0;
  L.best = 256;
  L.carea = 512;
  L.area = L.carea + align(nv * 8);
  L.total = L.area + align(nf * 8);
  return L;
}

int run_components(const float* v, int64_t nv, const int32_t* f, int64_t nf, int32_t* lab, float* w, void* ws,
                   hipStream_t s, int max_iters) {
  const CompLayout L = comp_layout(nv, nf);
  char* b = static_cast<char*>(ws);
  int32_t* flag = reinterpret_cast<int32_t*>(b + L.flag);
  int32_t* best = reinterpret_cast<int32_t*>(b + L.best);
  double* carea = reinterpret_cast<double*>(b + L.carea);
  double* area = reinterpret_cast<double*>(b + L.area);
  hipLaunchKernelGGL(k_lab_init, dim3(nb256(nv)), dim3(256), 0, s, lab, nv);
  int it = 0;
  for (; it < max_iters; ++it) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, flag, 0);
    hipLaunchKernelGGL(k_lab_faces, dim3(nb256(nf)), dim3(256), 0, s, f, nf, lab, flag);
    hipLaunchKernelGGL(k_lab_jump, dim3(nb256(nv)), dim3(256), 0, s, lab, nv);
    int32_t h = 0;
    if (hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return -4;
    if (hipStreamSynchronize(s) != hipSuccess) return -4;
    if (!h) break;
  }
  // a pass that changed nothing leaves one label per component: the smallest
  // vertex index in it, whose own label never changes
  if (it == max_iters) return -5;
  if (w) {
    hipLaunchKernelGGL(k_face_area, dim3(nb256(nf)), dim3(256), 0, s, v, f, nf, nullptr, area);
    hipLaunchKernelGGL(k_fill0d, dim3(256), dim3(256), 0, s, carea, nv);
    hipLaunchKernelGGL(k_comp_area, dim3(nb256(nf)), dim3(256), 0, s, f, nf, lab, area, carea);
    hipLaunchKernelGGL(k_comp_best, dim3(1), dim3(256), 0, s, carea, nv, best);
    hipLaunchKernelGGL(k_face_mask, dim3(nb256(nf)), dim3(256), 0, s, f, nf, lab, best, w);
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace opt
}  // namespace psr
