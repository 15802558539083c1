// gfx950 kernels of the differentiable Poisson solver (Peng et al., NeurIPS 2021).
//
// Pipeline of one forward solve (main Sec. 3.1, Eqs. 2-4; supplement Sec. A):
//   bin      points -> row-tile buckets (count, scan, scatter; below 512^3
//            every scatter workgroup scans the bin counts in LDS)
//   P1       splat normals into LDS rows + real-to-complex FFT along j2
//            (supplement A.1 rasterisation fused with the first FFT axis)
//   P2       FFT along j1 (3 channels in; out v~_0 and the merged channel
//            W = kappa_1 v~_1 + kappa_2 v~_2)
//   P3       FFT along j0, spectral operator of main Eq. 3 summed over the
//            channels, inverse FFT along j0 (one channel out)
//   P4       inverse FFT along j1
//   P5       complex-to-real inverse FFT along j2, write chi', and the
//            trilinear gather of chi' at the points (value + gradient)
//   reduce   FP64 mean at the points, scale c (main Eq. 4), normalise chi
// At 64^3 and 128^3 the plane passes P12 (= P1 + P2) and P45 (= P4 + P5) run
// two axes per kernel with a whole j0 plane on chip; at 256^3 only P45 does.
// The backward runs the adjoint of every step (FP64 sums of G and G*chi, the
// cotangent H, conjugate operator, 3 inverse channels, gather of dL/dv), with
// the same pass structure (B1..B5, B12, B45); on the two-pass path the sums
// ride on a first cotangent pass (B1a) that also transforms the row tiles
// needing no backward scalar. The cotangent's point source -Q delta_0 (the
// derivative through chi'(0,0,0) in Eq. 4) is not transformed: its response
// is read at the points from a table built once per (res, sigma) in FP64
// (a spike of that size would set the FP32 rounding of every spectrum
// element). Planes and row tiles that no point reaches are
// skipped where their values are zero or unused (bitmaps from the bin
// offsets). The splat accumulates 64-bit fixed-point integers in LDS
// (bitwise reproducible at any density).
//
// Layouts (complex64 unless noted; H = r/2 + 1 half-spectrum planes):
//   A[c][k2][j0][j1]   P1 out, P2 in   (3 channels fwd, 1 bwd)
//   B[c][k2][k1][j0]   P2 out, P3 in   (2 fwd, 1 bwd)
//   C[c][j0][k2][k1]   P3 out, P4/P45 in (1 fwd, 2 bwd); P12 out, P3 in
//   D[c][k2][j0][j1]   P4 out, P5 in   (1 fwd, 3 bwd)
// Each pass reads whole contiguous lines or multi-line segments and writes
// the other, so every global access is at least a 128-byte run. FFT data
// stays in registers between the global load, the first and last radix
// stages and the store; LDS carries only the exchange between stages and the
// transposes of segment stores.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fft_device.h"
#include "psr_device.h"
#include "psr_internal.h"

namespace psr {

// Point ranges (in sorted order) whose 2x2 corner lines touch the rows
// j1 in [a0, a0 + SPAN) of plane j0, SPAN a whole number of row tiles:
// floor rows b0 in {j0-1, j0}; in each, both bins of every tile of the span
// and the last-column bin of the tile before it (whose +1 corner reaches
// line a0). These bins are consecutive unless the span starts at tile 0 and
// the previous tile wraps round.
template <int RES, int SPAN>
__device__ __forceinline__ Ranges span_ranges(const int* __restrict__ off, int j0, int a0) {
  constexpr int NT = row_tiles(RES), TR = tile_rows(RES), ST = SPAN / TR;
  static_assert(SPAN % TR == 0 && ST <= NT, "a span is a whole number of row tiles");
  const int tbA = a0 / TR, tbB = tbA + ST;
  Ranges R;
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    const int rb = ((j0 - 1 + o) & (RES - 1)) * 2 * NT;
    int a, b, c, d;
    if constexpr (ST == NT) {
      a = off[rb];
      b = off[rb + 2 * NT];
      c = 0;
      d = 0;
    } else {
      if (tbA > 0) {
        a = off[rb + 2 * tbA - 1];
        b = off[rb + 2 * tbB];
        c = 0;
        d = 0;
      } else {
        a = off[rb + 2 * NT - 1];
        b = off[rb + 2 * NT];
        c = off[rb];
        d = off[rb + 2 * tbB];
      }
    }
    R.lo[2 * o] = a;
    R.n[2 * o] = b - a;
    R.lo[2 * o + 1] = c;
    R.n[2 * o + 1] = d - c;
  }
  R.total = R.n[0] + R.n[1] + R.n[2] + R.n[3];
  return R;
}

// Workgroup -> (row tile T = j0 * row_tiles + tb, channel c < NC) of a row
// pass over NC channels. The NC workgroups of a tile get ids equal mod 8, so
// they run on the same XCD and its L2 serves their repeated reads of the
// tile's point records. The tile count res * row_tiles is a multiple of 8.
template <int NC>
__device__ __forceinline__ void tile_of(int bid, int& T, int& c) {
  const int x = bid & 7, q = bid >> 3;
  c = q % NC;
  T = (q / NC) * 8 + x;
}

template <int RES>
__device__ __forceinline__ Ranges tile_ranges(const int* __restrict__ off, int j0, int tb) {
  return span_ranges<RES, tile_rows(RES)>(off, j0, tb * tile_rows(RES));
}


// Whether any point's corners reach plane j0 (floor planes j0 - 1 and j0).
// A plane no point reaches has zero splat rows, and nothing is gathered from
// it: passes skip reading or writing what only such planes would use.
template <int RES>
__device__ __forceinline__ bool plane_live(const int* __restrict__ off, int j0) {
  constexpr int NB = 2 * row_tiles(RES);  // bins per floor plane
  const int r0 = ((j0 - 1) & (RES - 1)) * NB, r1 = j0 * NB;
  return (off[r0 + NB] - off[r0]) + (off[r1 + NB] - off[r1]) > 0;
}



// ---------------------------------------------------------------------------
// binning: counting sort of the points by row tile (b0, b1 / tile_rows)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void b_init(int* __restrict__ counts, int n, SavedHeader* __restrict__ hdr, int res,
                                       int64_t npoints, float sigma, float m, int reading, int bid, int nblocks) {
  for (int i = bid * blockDim.x + threadIdx.x; i < n; i += nblocks * blockDim.x) counts[i] = 0;
  if (bid == 0 && threadIdx.x == 0) {
    hdr->status = 0;
    hdr->flags = 0;
    hdr->res = res;
    hdr->reading = reading;
    hdr->npoints = npoints;
    hdr->sigma = sigma;
    hdr->m = m;
  }
}

// Each workgroup takes kBinChunk points, counts them per bin in LDS (local
// rank = the LDS atomic's return value), then reserves its slots in every
// bin it touched with one global atomic per bin: few global atomics per bin
// even when a surface crowds the points into a few bins.
constexpr int kBinChunk = 1024;

template <int RES>
__device__ __forceinline__ void b_bin(const float* __restrict__ pts, const float* __restrict__ nrm,
                                      int64_t npoints, int* __restrict__ counts, PointRec* __restrict__ tmp, int2* __restrict__ colrank,
                                      SavedHeader* __restrict__ hdr, int bid) {
  constexpr int NB = num_bins(RES);
  constexpr int PPT = kBinChunk / 256;
  __shared__ int hist[NB];
  const int t = threadIdx.x;
  for (int e = t; e < NB; e += 256) hist[e] = 0;
  __syncthreads();
  int mybin[PPT], myrank[PPT];
  bool anybad = false;
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int64_t i = (int64_t)bid * kBinChunk + u * 256 + t;
    mybin[u] = -1;
    if (i >= npoints) continue;
    float f[3], n[3];
    int b[3];
    bool bad = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float x = pts[3 * i + a];
      n[a] = nrm[3 * i + a];
      if (!isfinite(x)) {
        bad = true;
        x = 0.0f;
      }
      if (!isfinite(n[a])) bad = true;  // the fixed-point splat needs finite values
      float uu = x - floorf(x);  // wrap into [0,1): periodic domain
      if (uu >= 1.0f) uu = 0.0f;
      const float tt = uu * (float)RES;  // exact: RES is a power of two
      int bi = (int)floorf(tt);
      bi = bi < 0 ? 0 : (bi > RES - 1 ? RES - 1 : bi);
      b[a] = bi;
      f[a] = tt - (float)bi;
    }
    if (bad) {
      f[0] = f[1] = f[2] = 0.0f;
      n[0] = n[1] = n[2] = 0.0f;
      anybad = true;
    }
    const int bin = b[0] * 2 * row_tiles(RES) + 2 * (b[1] / tile_rows(RES)) +
                    (b[1] % tile_rows(RES) == tile_rows(RES) - 1 ? 1 : 0);
    mybin[u] = bin;
    myrank[u] = atomicAdd(&hist[bin], 1);
    PointRec r;
    r.f0 = f[0];
    r.f1 = f[1];
    r.f2 = f[2];
    r.b = (uint32_t)b[0] | ((uint32_t)b[1] << 10) | ((uint32_t)b[2] << 20);
    r.n0 = n[0];
    r.n1 = n[1];
    r.n2 = n[2];
    r.idx = (uint32_t)i;
    tmp[i] = r;
  }
  if (anybad) atomicOr(&hdr->flags, 1);
  __syncthreads();
  for (int e = t; e < NB; e += 256) {
    const int cnt = hist[e];
    hist[e] = cnt ? atomicAdd(&counts[e], cnt) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int64_t i = (int64_t)bid * kBinChunk + u * 256 + t;
    if (mybin[u] >= 0) colrank[i] = make_int2(mybin[u], hist[mybin[u]] + myrank[u]);
  }
}

// Exclusive scan of n counts into off[0..n]: one workgroup of 1024 threads,
// coalesced rounds of 1024 elements, wavefront shuffles + a carry.
__device__ __forceinline__ void b_scan(const int* __restrict__ counts, int* __restrict__ off, int n, int bid) {
  __shared__ int wsum[16];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  int carry = 0;
  for (int base = 0; base < n; base += 1024) {
    const int i = base + t;
    const int c = i < n ? counts[i] : 0;
    int v = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(v, d, 64);
      if (lane >= d) v += y;
    }
    if (lane == 63) wsum[wid] = v;
    __syncthreads();
    if (wid == 0) {
      int w = lane < 16 ? wsum[lane] : 0;
#pragma unroll
      for (int d = 1; d < 16; d <<= 1) {
        const int y = __shfl_up(w, d, 64);
        if (lane >= d) w += y;
      }
      if (lane < 16) wsum[lane] = w;
    }
    __syncthreads();
    const int before = (wid ? wsum[wid - 1] : 0) + carry;
    if (i < n) off[i] = before + v - c;
    carry += wsum[15];
    __syncthreads();
  }
  if (t == 0) off[n] = carry;
}

// Bitmap of the planes some point's corners reach (floor planes j0 - 1 and
// j0 hold points), from the finished bin offsets; one workgroup.
template <int RES>
__device__ __forceinline__ void b_live_planes(const int* __restrict__ off, SavedHeader* __restrict__ hdr) {
  constexpr int NB = 2 * row_tiles(RES);  // bins per floor plane
  __shared__ uint32_t bits[16];
  const int t = threadIdx.x;
  if (t < 16) bits[t] = 0;
  __syncthreads();  // also orders this workgroup's offset writes before the reads below
  for (int j0 = t; j0 < RES; j0 += blockDim.x) {
    const int jm = (j0 - 1) & (RES - 1);
    if ((off[j0 * NB + NB] - off[j0 * NB]) + (off[jm * NB + NB] - off[jm * NB]) > 0)
      atomicOr(&bits[j0 >> 5], 1u << (j0 & 31));
  }
  __syncthreads();
  if (t < 16) hdr->live[t] = bits[t];
  // the same per row tile
  constexpr int NT = row_tiles(RES), NTB = RES * NT, NW = (NTB + 31) / 32;
  static_assert(NTB <= 32 * 256 && 32 % NT == 0, "tile bitmap: one word holds the tiles of whole planes");
  __shared__ uint32_t tbits[NW];
  for (int e = t; e < NW; e += blockDim.x) tbits[e] = 0;
  __syncthreads();
  for (int e = t; e < NTB; e += blockDim.x)
    if (tile_ranges<RES>(off, e / NT, e % NT).total > 0) atomicOr(&tbits[e >> 5], 1u << (e & 31));
  __syncthreads();
  for (int e = t; e < NW; e += blockDim.x) hdr->tlive[e] = tbits[e];
}

// The row-tile bits of plane j0 (bit tb), from the tile bitmap.
template <int RES>
__device__ __forceinline__ uint32_t plane_tiles(const uint32_t* __restrict__ tlive, int j0) {
  constexpr int NT = row_tiles(RES);
  const int e = j0 * NT;
  return (tlive[e >> 5] >> (e & 31)) & (NT == 32 ? ~0u : ((1u << NT) - 1u));
}

__device__ __forceinline__ bool live_bit(const uint32_t* live, int j0) { return (live[j0 >> 5] >> (j0 & 31)) & 1u; }

// The plane bitmap held in registers (uniform loads), for per-element tests
// that should not wait on a dependent load.
template <int RES>
struct LiveBits {
  uint32_t w[(RES + 31) / 32];
  __device__ __forceinline__ void load(const uint32_t* __restrict__ p) {
#pragma unroll
    for (int k = 0; k < (RES + 31) / 32; ++k) w[k] = p[k];
  }
  __device__ __forceinline__ bool operator()(int j0) const {
    uint32_t x = w[0];
#pragma unroll
    for (int k = 1; k < (RES + 31) / 32; ++k)
      if ((j0 >> 5) == k) x = w[k];
    return (x >> (j0 & 31)) & 1u;
  }
};

__device__ __forceinline__ void b_scatter(const PointRec* __restrict__ tmp, const int2* __restrict__ colrank,
                          const int* __restrict__ off, PointRec* __restrict__ sorted, int64_t npoints, int bid) {
  const int64_t i = (int64_t)bid * blockDim.x + threadIdx.x;
  if (i >= npoints) return;
  const int2 cr = colrank[i];
  sorted[off[cr.x] + cr.y] = tmp[i];
}

// Grids with at most kLdsBins bins skip the one-workgroup scan kernel: every
// scatter workgroup forms the same exclusive prefix sum of the counts in LDS
// (BLOCK threads, consecutive runs of bins per thread), and workgroup 0 also
// publishes the offsets and the liveness bitmaps.
constexpr int kLdsBins = 4096;

template <int NB, int BLOCK>
__device__ __forceinline__ void scan_to_lds(const int* __restrict__ counts, int* soff) {
  constexpr int PT = (NB + BLOCK - 1) / BLOCK, NW = BLOCK / 64;
  static_assert(BLOCK % 64 == 0, "whole wavefronts");
  __shared__ int wtot[NW];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  int v[PT], sum = 0;
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int i = t * PT + k;
    v[k] = i < NB ? counts[i] : 0;
    sum += v[k];
  }
  int x = sum;  // inclusive scan of the thread sums within the wavefront
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wtot[wid] = x;
  __syncthreads();
  int run = x - sum;
  for (int q = 0; q < wid; ++q) run += wtot[q];
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int i = t * PT + k;
    if (i < NB) soff[i] = run;
    run += v[k];
  }
  if (t == BLOCK - 1) soff[NB] = run;  // the last thread's run ends at NB: the total
  __syncthreads();
}

// ---------------------------------------------------------------------------
// P1 / B1: rasterise one channel into LDS rows, then r2c FFT along j2.
// MODE_SPLAT: v_c = splat of normal component c        [forward, grid x3]
// MODE_BWDH : H = s G + alpha W (1 channel)              [backward]
// MODE_LOADV: v_c loaded from global                     [spectral test hook]
// MODE_VOUT : splat only, rows written to global v_c      [splat test hook]
// MODE_BWDA : the FP64 partials of S_G and S_Gchi per row tile, and H = s G
//             for the row tiles that W does not reach    [backward,
//             before MODE_BWDH, which then takes only the other tiles]
// ---------------------------------------------------------------------------
enum { MODE_SPLAT = 0, MODE_BWDH = 1, MODE_LOADV = 2, MODE_VOUT = 3, MODE_BWDA = 4 };

// blocks of the grid-stride FP64 reduction over RES^3 / 4 float4 (at least 1)
template <int RES>
constexpr int bwd_reduce_blocks() {
  constexpr int64_t n = ((int64_t)RES * RES * RES / 4 + 255) / 256;
  return n > kRedBlocks ? kRedBlocks : (int)n;
}

// The backward's scalars (main Eq. 4 differentiated): Q = sum(G chi) / c,
// g_mu = -s sum(G) + Q (reading B; A drops Q), alpha = g_mu / P, returned as
// (s, Q, alpha). Every workgroup of the cotangent pass sums the same FP64
// per-block partials in the same order; block 0 records them for the final
// pass. Ends with a barrier.
template <int BLOCK>
__device__ __forceinline__ float3 bwd_scalars(const double2* __restrict__ blockpart, int nb,
                                              const SavedHeader* __restrict__ hdr, BwdScalars* __restrict__ bs,
                                              bool record) {
  constexpr int NW = (BLOCK + 63) / 64, W = BLOCK < 64 ? BLOCK : 64;
  __shared__ double wsum[2][NW];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += BLOCK) {
    a += blockpart[i].x;
    b += blockpart[i].y;
  }
#pragma unroll
  for (int d = W / 2; d > 0; d >>= 1) {
    a += __shfl_xor(a, d, W);
    b += __shfl_xor(b, d, W);
  }
  if ((threadIdx.x & 63) == 0) {
    wsum[0][threadIdx.x >> 6] = a;
    wsum[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  double SG = 0.0, SGc = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    SG += wsum[0][w];
    SGc += wsum[1][w];
  }
  const double s = hdr->scale, c = hdr->cscale;
  const double Q = SGc / c;
  const double gmu = -s * SG + (hdr->reading == 0 ? Q : 0.0);
  const float alpha = (float)(gmu / (double)hdr->npoints);
  if (record && threadIdx.x == 0) {
    bs->S_G = SG;
    bs->S_Gchi = SGc;
    bs->Qd = Q;
    bs->gmu = gmu;
    bs->s = (float)s;
    bs->q = (float)Q;
    bs->alpha = alpha;
  }
  return make_float3((float)s, (float)Q, alpha);
}



// Rows [a0, a0 + NROWS) of plane j0: the FP64 sums of G and G chi over them
// into *part (fixed order: per thread, then wavefront shuffles, then
// wavefronts in order), and, when fill, rows H = s G in LDS as fill_rows
// lays them out. Ends with a barrier.
template <int RES, int NROWS, int BLOCK>
__device__ __forceinline__ void bwda_rows(cf* rows, const float* __restrict__ G, const float* __restrict__ chi,
                                          float s, int j0, int a0, double2* __restrict__ part, bool fill) {
  constexpr int M = RES / 2, NV = NROWS * M / 2, IT = (NV + BLOCK - 1) / BLOCK;
  constexpr int NW = (BLOCK + 63) / 64, W = BLOCK < 64 ? BLOCK : 64;
  const int t = threadIdx.x;
  const int64_t base = ((int64_t)j0 * RES + a0) * RES;
  const float4* g4 = reinterpret_cast<const float4*>(G + base);
  const float4* c4 = reinterpret_cast<const float4*>(chi + base);
  float4 gb[IT], cb[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = t + it * BLOCK;
    if (e < NV) {
      gb[it] = g4[e];
      cb[it] = c4[e];
    }
  }
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = t + it * BLOCK;
    if (e < NV) {
      const float4 g = gb[it], c = cb[it];
      a += ((double)g.x + (double)g.y) + ((double)g.z + (double)g.w);
      b += ((double)g.x * c.x + (double)g.y * c.y) + ((double)g.z * c.z + (double)g.w * c.w);
    }
  }
#pragma unroll
  for (int d = W / 2; d > 0; d >>= 1) {
    a += __shfl_xor(a, d, W);
    b += __shfl_xor(b, d, W);
  }
  __shared__ double wsum[2][NW];
  if ((t & 63) == 0) {
    wsum[0][t >> 6] = a;
    wsum[1][t >> 6] = b;
  }
  if (fill) {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * BLOCK;
      if (e < NV) {
        const int mm = (2 * e) % M, l = (2 * e) / M;
        rows[rpos<M>(l, mm)] = cf{gb[it].x * s, gb[it].y * s};
        rows[rpos<M>(l, mm + 1)] = cf{gb[it].z * s, gb[it].w * s};
      }
    }
  }
  __syncthreads();
  if (t == 0) {
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      sa += wsum[0][w];
      sb += wsum[1][w];
    }
    *part = make_double2(sa, sb);
  }
}

template <int RES, int MODE>
__device__ __forceinline__ void b_splat_r2c(const PointRec* __restrict__ sorted,
                                                              const int* __restrict__ off,
                                                              const float* __restrict__ gin,
                                                              BwdScalars* __restrict__ bs,
                                                              const double2* __restrict__ bpart,
                                                              const SavedHeader* __restrict__ hdr,
                                                              const cf* __restrict__ tw, cf* __restrict__ out,
                                                              float* __restrict__ vout, const float* __restrict__ chi_in,
                                                              double2* __restrict__ bpart_w, int bid) {
  constexpr int M = RES / 2, H = M + 1, TR = tile_rows(RES), NT = row_tiles(RES), BR = rows_wg(RES);
  constexpr int TPL = plan_TPL(M), E = plan_E(M), LS = row_ls(M);
  constexpr int64_t N3 = (int64_t)RES * RES * RES;
  __shared__ __align__(16) cf rows[rows_lds(RES) * LS];
  __shared__ cf stw[M];      // FFT table of length M
  __shared__ cf rtw[M + 1];  // W_RES^k, k in [0, M], for the r2c post-processing
  float* rf = reinterpret_cast<float*>(rows);
  constexpr int NC = MODE == MODE_BWDH || MODE == MODE_BWDA ? 1 : 3;  // channels in the grid
  int T, c;
  tile_of<NC>(bid, T, c);
  const int tb = T % NT, j0 = T / NT;
  const int a0 = tb * TR;
  const int t = threadIdx.x;
  Ranges R{};
  if constexpr (MODE != MODE_LOADV) R = tile_ranges<RES>(off, j0, tb);
  const int total = R.total;
  // the row tile of workgroup 0 records the backward scalars for the final pass
  const bool records = T == 0;
  // workgroups with nothing to do leave before staging any table (most row
  // tiles of a large grid hold no point); the test is uniform per workgroup
  if constexpr (MODE == MODE_SPLAT) {
    // no point touches this row tile (of a plane some point may reach): its
    // rows and their spectra are zero; P2 takes them as zero without reading
    if (total == 0) return;
  }
  if constexpr (MODE == MODE_BWDH) {
    if (total == 0 && !records) return;  // done by MODE_BWDA
  }
  if constexpr (MODE != MODE_VOUT) {
    stage_table<BR>(stw, tw + M, M);
    stage_table<BR>(rtw, tw + RES, M + 1);
  }

  if constexpr (MODE == MODE_BWDA) {
    // rows of tiles that W reaches wait for the reductions (MODE_BWDH)
    const bool later = total > 0 || records;
    bwda_rows<RES, TR, BR>(rows, gin, chi_in, (float)hdr->scale, j0, a0, bpart_w + T, !later);
    if (later) return;
  } else {
    float3 sqa = make_float3(1.0f, 0.0f, 1.0f);
    if constexpr (MODE == MODE_BWDH) sqa = bwd_scalars<BR>(bpart, RES * NT, hdr, bs, records);
    fill_rows<RES, TR, BR, MODE == MODE_VOUT ? MODE_SPLAT : MODE>(rows, sorted, R, gin, sqa, j0, a0, c);
  }

  if constexpr (MODE == MODE_VOUT) {
    for (int e = t; e < TR * RES; e += BR) {
      const int nn = e % RES, l = e / RES;
      vout[c * N3 + ((int64_t)j0 * RES + a0 + l) * RES + nn] = rf[2 * rpos<M>(l, nn >> 1) + (nn & 1)];
    }
  } else {
    {
      cf reg[E];
      const int l = t / TPL;
      fft<M, -1, false, false>(reg, rows + l * LS, t % TPL, stw, row_swz(M, l));
    }
    // X[k] = E_k + W_r^k O_k with E = (Z_k + Z*_{M-k})/2, O = (Z_k - Z*_{M-k})/(2i)
    for (int e = t; e < H * (TR / 2); e += BR) {
      const int l = 2 * (e % (TR / 2)), k = e / (TR / 2);
      const cf w = rtw[k];
      float4 o;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const cf zk = rows[rpos<M>(l + h, k == M ? 0 : k)];
        const cf zm = rows[rpos<M>(l + h, k == 0 ? 0 : M - k)];
        const cf Ee{0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y)};
        const cf Oo{0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x)};
        const cf X = cadd(Ee, cmul(w, Oo));
        if (h == 0) {
          o.x = X.x;
          o.y = X.y;
        } else {
          o.z = X.x;
          o.w = X.y;
        }
      }
      *reinterpret_cast<float4*>(out + (((int64_t)c * H + k) * RES + j0) * RES + a0 + l) = o;
    }
  }
}

// Load TC lines stored transposed (element n of line l at src[n * stride_n +
// l], two lines per 16-byte load) into the LDS lines rows[l * LS + pidx(n)].
// All global loads are issued before the LDS writes; ends with a barrier.
template <int RES, int TC>
__device__ __forceinline__ void load_transposed(cf* rows, const cf* __restrict__ src, int64_t stride_n,
                                                const cf* __restrict__ src2 = nullptr) {
  constexpr int BC = TC * plan_TPL(RES), LS = lstride(RES);
  constexpr int NV = RES * (TC / 2), IT = (NV + BC - 1) / BC;
  float4 buf[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * BC;
    if (e < NV) {
      const int l2 = 2 * (e % (TC / 2)), n = e / (TC / 2);
      buf[it] = *reinterpret_cast<const float4*>(src + n * stride_n + l2);
    }
  }
  if (src2) {  // the sum of two channels (uniform)
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = threadIdx.x + it * BC;
      if (e < NV) {
        const int l2 = 2 * (e % (TC / 2)), n = e / (TC / 2);
        const float4 y = *reinterpret_cast<const float4*>(src2 + n * stride_n + l2);
        buf[it] = make_float4(buf[it].x + y.x, buf[it].y + y.y, buf[it].z + y.z, buf[it].w + y.w);
      }
    }
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * BC;
    if (e < NV) {
      const int l2 = 2 * (e % (TC / 2)), n = e / (TC / 2);
      rows[l2 * LS + pidx(n)] = cf{buf[it].x, buf[it].y};
      rows[(l2 + 1) * LS + pidx(n)] = cf{buf[it].z, buf[it].w};
    }
  }
  __syncthreads();
}

// Store the canonical registers of TC lines transposed: out[n][a0 + l] for
// every element n of every line l, two lines per 16-byte store; with masks,
// only the elements n with keep[n] != 0 and the line pairs with a line whose
// keep_line is set.
template <int RES, int TC = tile_cols(RES)>
__device__ __forceinline__ void store_transposed(cf* rows, const cf* reg, cf* __restrict__ dst, int64_t stride_n,
                                                 int l, int lt, const int* keep = nullptr,
                                                 const int* keep_line = nullptr) {
  constexpr int BC = TC * plan_TPL(RES), TPL = plan_TPL(RES), E = plan_E(RES), LS = lstride(RES);
#pragma unroll
  for (int v = 0; v < E; ++v) rows[l * LS + pidx(lt + TPL * v)] = reg[v];
  __syncthreads();
  for (int e = threadIdx.x; e < RES * (TC / 2); e += BC) {
    const int l2 = 2 * (e % (TC / 2)), n = e / (TC / 2);
    if (keep && !keep[n]) continue;
    if (keep_line && !keep_line[l2] && !keep_line[l2 + 1]) continue;
    const cf x0 = rows[l2 * LS + pidx(n)], x1 = rows[(l2 + 1) * LS + pidx(n)];
    *reinterpret_cast<float4*>(dst + n * stride_n + l2) = make_float4(x0.x, x0.y, x1.x, x1.y);
  }
}

// ---------------------------------------------------------------------------
// P2 / B2: forward FFT along j1. A[c][k2][j0][j1] -> B[c'][k2][k1][j0].
// MERGE = false (B2): one channel in, one out.
// MERGE = true (P2): three channels in, two out: v~_0, and
//   W = kappa_1(k1) v~_1 + kappa_2(k2) v~_2, which is all the j0 pass needs of
//   channels 1 and 2 because their operator factors do not vary along j0.
// ---------------------------------------------------------------------------
template <int RES, bool MERGE, bool SKIP>
__device__ __forceinline__ void b_axis1_fwd(const cf* __restrict__ in, cf* __restrict__ out,
                                            const cf* __restrict__ tw, const uint32_t* __restrict__ livebits,
                                            int bid) {
  constexpr int H = RES / 2 + 1, TC = tile_cols(RES), TPL = plan_TPL(RES), E = plan_E(RES), LS = lstride(RES);
  constexpr int64_t CH = (int64_t)H * RES * RES;  // elements per channel
  __shared__ cf rows[TC * LS];
  __shared__ cf stw[RES];
  stage_table<cols_block(RES)>(stw, tw + RES, RES);
  int b = bid;
  const int tb = b % (RES / TC);
  b /= RES / TC;
  const int k2 = b % H;
  // output channel; with MERGE the heavier channel-1 workgroups (two
  // transforms) come first in the grid so that they do not form its tail
  const int c = MERGE ? 1 - b / H : b / H;
  const int a0 = tb * TC;
  const int l = threadIdx.x / TPL, lt = threadIdx.x % TPL;
  const cf* src = in + ((int64_t)k2 * RES + a0 + l) * RES;
  // SKIP: the row-tile segments of a line (element j1 in tile j1 / TR) that no
  // point touches were never written by P1; they are zero. Lines of a plane
  // no point reaches are all zero, and P3 does not read their transforms.
  constexpr int TR = tile_rows(RES);
  __shared__ int line_live[SKIP ? TC : 1];
  const uint32_t tiles = SKIP ? plane_tiles<RES>(livebits, a0 + l) : ~0u;
  const bool live = tiles != 0;
  auto seg = [&](int v) { return !SKIP || ((tiles >> ((lt + TPL * v) / TR)) & 1u); };
  if (SKIP && lt == 0) line_live[l] = live;
  cf reg[E];
  if (!MERGE || c == 0) {
#pragma unroll
    for (int v = 0; v < E; ++v) reg[v] = seg(v) ? src[c * CH + lt + TPL * v] : cf{0.0f, 0.0f};
    fft<RES, -1, true, true>(reg, rows + l * LS, lt, stw);
  } else {
    cf acc[E];
#pragma unroll
    for (int v = 0; v < E; ++v) reg[v] = seg(v) ? src[2 * CH + lt + TPL * v] : cf{0.0f, 0.0f};
    fft<RES, -1, true, true>(reg, rows + l * LS, lt, stw);
    const float k2f = kappa_odd(k2, RES);
#pragma unroll
    for (int v = 0; v < E; ++v) {
      acc[v] = cf{k2f * reg[v].x, k2f * reg[v].y};
      reg[v] = seg(v) ? src[CH + lt + TPL * v] : cf{0.0f, 0.0f};
    }
    fft<RES, -1, true, true>(reg, rows + l * LS, lt, stw);
#pragma unroll
    for (int v = 0; v < E; ++v) {
      const float k1f = kappa_odd(lt + TPL * v, RES);
      reg[v] = cf{acc[v].x + k1f * reg[v].x, acc[v].y + k1f * reg[v].y};
    }
  }
  store_transposed<RES>(rows, reg, out + ((int64_t)c * H + k2) * RES * RES + a0, (int64_t)RES, l, lt, nullptr,
                        SKIP ? line_live : nullptr);
}

// ---------------------------------------------------------------------------
// P3: FFT along j0 of the 3 channels, chi~ = i F(k) sum_d kappa_d^odd v~_d
// with F = g / (-2 pi |kappa|^2) / N (main Eq. 3; the inverse's 1/N folded
// in), then inverse FFT along k0. B[2][k2][k1][j0] (or C[2][j0][k2][k1] after
// a plane pass, IN_C) -> C[1][j0][k2][k1].
// ---------------------------------------------------------------------------

template <int RES, bool IN_C, bool SKIP>
__device__ __forceinline__ void b_fwd_axis0(const cf* __restrict__ in, cf* __restrict__ out,
                                            const cf* __restrict__ tw, float sigma,
                                            const uint32_t* __restrict__ livebits, int bid) {
  constexpr int H = RES / 2 + 1, TC = tile_j0(RES), TPL = plan_TPL(RES), E = plan_E(RES), LS = lstride(RES);
  __shared__ cf rows[TC * LS];
  __shared__ cf stw[RES];
  __shared__ float g1[RES];
  stage_table<j0_block(RES)>(stw, tw + RES, RES);
  gauss_table<RES, j0_block(RES)>(g1, sigma);
  const int tb = bid % (RES / TC);
  const int k2 = bid / (RES / TC);
  const int a0 = tb * TC;
  const int l = threadIdx.x / TPL, lt = threadIdx.x % TPL;
  const int k1 = a0 + l;
  constexpr int64_t CH = (int64_t)H * RES * RES;
  cf acc[E], reg[E];
  // sum_d kappa_d v~_d = kappa_0(k0) FFT_j0(v~_0) + FFT_j0(W)
  // SKIP (two-pass path): elements j0 of planes no point reaches are zero and
  // were not written by P2
  if constexpr (IN_C) {
    const cf* src = in + (int64_t)k2 * RES + a0;  // element j0 of line k1 at src[j0 H RES + l]
    load_transposed<RES, TC>(rows, src, (int64_t)H * RES);
    fft<RES, -1, false, true>(reg, rows + l * LS, lt, stw);
#pragma unroll
    for (int v = 0; v < E; ++v) acc[v] = cscale(reg[v], kappa_odd(lt + TPL * v, RES));
    // W = kappa_1 v~_1 + kappa_2 v~_2, summed on load
    load_transposed<RES, TC>(rows, src + CH, (int64_t)H * RES, src + 2 * CH);
    fft<RES, -1, false, true>(reg, rows + l * LS, lt, stw);
  } else {
    const cf* src = in + ((int64_t)k2 * RES + k1) * RES;
    cf nxt[E];  // W's line is loaded under the first transform
    LiveBits<RES> lb;
    if constexpr (SKIP) lb.load(livebits);
#pragma unroll
    for (int v = 0; v < E; ++v) {
      const bool lv = !SKIP || lb(lt + TPL * v);
      reg[v] = lv ? src[lt + TPL * v] : cf{0.0f, 0.0f};
      nxt[v] = lv ? src[CH + lt + TPL * v] : cf{0.0f, 0.0f};
    }
    // the line transforms synchronise within wavefronts only (a line's
    // threads are lanes of one wavefront, and each touches only its own LDS
    // line until store_transposed's barrier): the tables get a barrier of
    // their own, after the line loads are in flight
    __syncthreads();
    fft<RES, -1, true, true, true>(reg, rows + l * LS, lt, stw);
#pragma unroll
    for (int v = 0; v < E; ++v) {
      acc[v] = cscale(reg[v], kappa_odd(lt + TPL * v, RES));
      reg[v] = nxt[v];
    }
    fft<RES, -1, true, true, true>(reg, rows + l * LS, lt, stw);
  }
  {
    const float g12 = g1[k1] * g1[k2];
    const float q12 = kappa_of(k1, RES) * kappa_of(k1, RES) + kappa_of(k2, RES) * kappa_of(k2, RES);
#pragma unroll
    for (int v = 0; v < E; ++v) {
      const float F = spectral_F<RES>(g1, lt + TPL * v, g12, q12);
      const cf a{acc[v].x + reg[v].x, acc[v].y + reg[v].y};
      reg[v] = cf{-F * a.y, F * a.x};  // i F sum
    }
  }
  fft<RES, +1, true, true, !IN_C>(reg, rows + l * LS, lt, stw);
  store_transposed<RES, TC>(rows, reg, out + (int64_t)k2 * RES + a0, (int64_t)H * RES, l, lt);
}

// B3: FFT along j0 of H^, then the conjugate operator -i F kappa_d H^ and the
// inverse FFT along k0. Channel 0 carries kappa_0(k0); channels 1 and 2 only
// differ by the constants kappa_1(k1), kappa_2(k2) along the line, so one
// unscaled channel U = IFFT_k0(-i F H^) serves both (kappa_1 is applied in
// the k1 pass, kappa_2 in the k2 pass). B[1][k2][k1][j0] (or C[1][j0][k2][k1],
// IN_C) -> C[2][j0][k2][k1].
template <int RES, bool IN_C>
__device__ __forceinline__ void b_bwd_axis0(const cf* __restrict__ in, cf* __restrict__ out,
                                            const cf* __restrict__ tw, float sigma, const int* __restrict__ off,
                                            int bid) {
  constexpr int H = RES / 2 + 1, TC = tile_j0(RES), TPL = plan_TPL(RES), E = plan_E(RES), LS = lstride(RES);
  __shared__ cf rows[TC * LS];
  __shared__ cf stw[RES];
  __shared__ float g1[RES];
  __shared__ int live[RES];  // planes some point reaches: the only ones the next passes read
  stage_table<j0_block(RES)>(stw, tw + RES, RES);
  gauss_table<RES, j0_block(RES)>(g1, sigma);
  for (int e = threadIdx.x; e < RES; e += j0_block(RES)) live[e] = plane_live<RES>(off, e);
  const int tb = bid % (RES / TC);
  const int k2 = bid / (RES / TC);
  const int a0 = tb * TC;
  const int l = threadIdx.x / TPL, lt = threadIdx.x % TPL;
  const int k1 = a0 + l;
  cf h[E], reg[E];
  if constexpr (IN_C) {
    load_transposed<RES, TC>(rows, in + (int64_t)k2 * RES + a0, (int64_t)H * RES);
    fft<RES, -1, false, true>(h, rows + l * LS, lt, stw);
  } else {
    const cf* src = in + ((int64_t)k2 * RES + k1) * RES;
#pragma unroll
    for (int v = 0; v < E; ++v) h[v] = src[lt + TPL * v];
    // wavefront-synchronous line transforms, as in P3: the tables and the
    // live flags get a barrier of their own
    __syncthreads();
    fft<RES, -1, true, true, true>(h, rows + l * LS, lt, stw);
  }
  const float g12 = g1[k1] * g1[k2];
  const float q12 = kappa_of(k1, RES) * kappa_of(k1, RES) + kappa_of(k2, RES) * kappa_of(k2, RES);
#pragma unroll
  for (int v = 0; v < E; ++v) {
    const float F = spectral_F<RES>(g1, lt + TPL * v, g12, q12);
    h[v] = cf{F * h[v].y, -F * h[v].x};  // -i F H^
    const float k0f = kappa_odd(lt + TPL * v, RES);
    reg[v] = cf{k0f * h[v].x, k0f * h[v].y};
  }
  fft<RES, +1, true, true, !IN_C>(reg, rows + l * LS, lt, stw);
  store_transposed<RES, TC>(rows, reg, out + (int64_t)k2 * RES + a0, (int64_t)H * RES, l, lt, live);
  __syncthreads();
  fft<RES, +1, true, true, !IN_C>(h, rows + l * LS, lt, stw);
  store_transposed<RES, TC>(rows, h, out + ((int64_t)RES * H + k2) * RES + a0, (int64_t)H * RES, l, lt, live);
}

// ---------------------------------------------------------------------------
// P4 / B4: inverse FFT along k1. C[c][j0][k2][k1] -> D[c'][k2][j0][j1].
// SPLIT = false (P4): one channel in, one out.
// SPLIT = true (B4): channels (V0, U) in, three out: IFFT(V0),
//   IFFT(kappa_1(k1) U) and IFFT(U) (the last still lacks kappa_2(k2), which
//   the c2r pass applies).
// ---------------------------------------------------------------------------
template <int RES, bool SPLIT>
__device__ __forceinline__ void b_axis1_inv(const cf* __restrict__ in, cf* __restrict__ out,
                                            const cf* __restrict__ tw, const int* __restrict__ off, int bid) {
  constexpr int H = RES / 2 + 1, TC = tile_cols(RES), TPL = plan_TPL(RES), E = plan_E(RES), LS = lstride(RES);
  constexpr int NT = row_tiles(RES), TR = tile_rows(RES);
  constexpr int64_t CH = (int64_t)H * RES * RES;
  __shared__ cf rows[TC * LS];
  __shared__ cf stw[RES];
  __shared__ int tile_live[SPLIT ? TC * NT : 1];
  stage_table<cols_block(RES)>(stw, tw + RES, RES);
  int b = bid;
  const int tb = b % (RES / TC);
  b /= RES / TC;
  const int k2 = b % H;
  // input channel; with SPLIT the heavier channel-1 workgroups (two
  // transforms, two outputs) come first in the grid
  const int c = SPLIT ? 1 - b / H : b / H;
  const int l = threadIdx.x / TPL, lt = threadIdx.x % TPL;
  const int j0 = tb * TC + l;
  const cf* src = in + c * CH + ((int64_t)j0 * H + k2) * RES;
  cf* dst = out + c * CH + ((int64_t)k2 * RES + j0) * RES;
  cf reg[E];
  if constexpr (!SPLIT) {
#pragma unroll
    for (int v = 0; v < E; ++v) reg[v] = src[lt + TPL * v];
    fft<RES, +1, true, true>(reg, rows + l * LS, lt, stw);
#pragma unroll
    for (int v = 0; v < E; ++v) dst[lt + TPL * v] = reg[v];
  } else {
    // backward: B5 reads only row tiles some point touches. Lines of planes
    // no point reaches are neither read nor written; elsewhere only the
    // segments of touched tiles are written (the FFT's barriers publish the
    // flags before the stores read them).
    if (threadIdx.x < TC * NT) {
      const int li = threadIdx.x / NT, ti = threadIdx.x % NT;
      tile_live[threadIdx.x] = tile_ranges<RES>(off, tb * TC + li, ti).total > 0;
    }
    const bool live = plane_live<RES>(off, j0);
    if (c == 0) {
#pragma unroll
      for (int v = 0; v < E; ++v) reg[v] = live ? src[lt + TPL * v] : cf{0.0f, 0.0f};
      fft<RES, +1, true, true>(reg, rows + l * LS, lt, stw);
#pragma unroll
      for (int v = 0; v < E; ++v) {
        const int j1 = lt + TPL * v;
        if (live && tile_live[l * NT + j1 / TR]) dst[j1] = reg[v];
      }
    } else {
      cf u[E];
#pragma unroll
      for (int v = 0; v < E; ++v) {
        u[v] = live ? src[lt + TPL * v] : cf{0.0f, 0.0f};
        reg[v] = cscale(u[v], kappa_odd(lt + TPL * v, RES));
      }
      fft<RES, +1, true, true>(reg, rows + l * LS, lt, stw);
#pragma unroll
      for (int v = 0; v < E; ++v) {
        const int j1 = lt + TPL * v;
        if (live && tile_live[l * NT + j1 / TR]) dst[j1] = reg[v];
      }
      fft<RES, +1, true, true>(u, rows + l * LS, lt, stw);
#pragma unroll
      for (int v = 0; v < E; ++v) {
        const int j1 = lt + TPL * v;
        if (live && tile_live[l * NT + j1 / TR]) dst[CH + j1] = u[v];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// P5 / B5: complex-to-real inverse FFT along k2 of a row tile of one channel,
// then the trilinear gather at the points whose corner lines fall in the tile.
// Per (point, corner line, channel) the partial is (value, d/dc0, d/dc1,
// d/dc2) of the interpolant restricted to that line. Partials are slot-major,
// one array of np float4 per (channel, corner line): part[(c 4 + slot) np + s]
// with slot = 2 o0 + o1, so the lanes of a wavefront, which hold consecutive
// sorted points, store whole lines.
// MODE_FWD: chi' (1 channel): writes chi' rows and the partials.
// MODE_BWD: g_v channel c (grid x3): partials only.
// MODE_DBG: chi' rows only.
// ---------------------------------------------------------------------------
enum { MODE_FWD = 0, MODE_BWD = 1, MODE_DBG = 2 };

template <int RES, int MODE>
__device__ __forceinline__ void b_c2r_gather(const cf* __restrict__ in,
                                                               float* __restrict__ chi_out,
                                                               SavedHeader* __restrict__ hdr,
                                                               const PointRec* __restrict__ sorted,
                                                               const int* __restrict__ off,
                                                               float4* __restrict__ part, int64_t np,
                                                               const cf* __restrict__ tw, int bid) {
  constexpr int M = RES / 2, H = M + 1, TR = tile_rows(RES), NT = row_tiles(RES), BR = rows_wg(RES);
  constexpr int TPL = plan_TPL(M), E = plan_E(M), LS = row_ls(M);
  __shared__ __align__(16) cf rows[rows_lds(RES) * LS];
  __shared__ cf stw[M];      // FFT table of length M
  __shared__ cf rtw[M + 1];  // W_RES^k, k in [0, M], for the c2r pre-processing
  const float* rf = reinterpret_cast<const float*>(rows);
  constexpr int NC = MODE == MODE_BWD ? 3 : 1;  // channels in the grid
  int T, c;
  tile_of<NC>(bid, T, c);
  const int tb = T % NT, j0 = T / NT;
  const int a0 = tb * TR;
  const int t = threadIdx.x;
  Ranges R{};
  if constexpr (MODE != MODE_DBG) R = tile_ranges<RES>(off, j0, tb);
  const int total = R.total;
  if constexpr (MODE != MODE_DBG) {
    // the backward pass only produces per-point partials: a tile that no
    // point touches has nothing to do (uniform across the workgroup; before
    // any table is staged)
    if (MODE == MODE_BWD && total == 0) return;
  }
  stage_table<BR>(stw, tw + M, M);
  stage_table<BR>(rtw, tw + RES, M + 1);
  // the thread's point records are fetched now, under the grid loads
  constexpr int KR = 4;
  Recs<KR> recs;
  if constexpr (MODE != MODE_DBG) fetch_recs<KR, BR>(recs, sorted, R, t);

  {
    constexpr int NV = H * (TR / 2);
    constexpr int IT = (NV + BR - 1) / BR;
    float4 buf[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * BR;
      if (e < NV) {
        const int l = 2 * (e % (TR / 2)), k = e / (TR / 2);
        buf[it] = *reinterpret_cast<const float4*>(in + (((int64_t)c * H + k) * RES + j0) * RES + a0 + l);
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * BR;
      if (e < NV) {
        const int l = 2 * (e % (TR / 2)), k = e / (TR / 2);
        float4 v = buf[it];
        if (MODE == MODE_BWD && c == 2) {  // channel 2 still lacks its kappa_2(k2) factor
          const float k2f = kappa_odd(k, RES);
          v.x *= k2f;
          v.y *= k2f;
          v.z *= k2f;
          v.w *= k2f;
        }
        rows[rpos<M>(l, k)] = cf{v.x, v.y};
        rows[rpos<M>(l + 1, k)] = cf{v.z, v.w};
      }
    }
  }
  __syncthreads();
  // Hermitian half-spectrum X[0..M] -> packed spectrum Z[0..M) of the
  // even/odd samples: Z = (X_k + X*_{M-k}) + i (X_k - X*_{M-k}) e^{+2 pi i k/r}.
  {
    // k in [0, M/2) first, in runs of M/2 per row (whole 16-element blocks of
    // the padded LDS line, so the k reads of a 16-lane group hit distinct
    // banks), then k = M/2, which is its own partner, for every row
    constexpr int NH = M / 2;
    const cf* twr = rtw;
    for (int e = t; e < TR * (NH + 1); e += BR) {
      const int k = e < TR * NH ? e % NH : NH, row = e < TR * NH ? e / NH : e - TR * NH;
      const int ik = rpos<M>(row, k), im = rpos<M>(row, M - k);
      const cf xk = rows[ik], xm = rows[im];
      {
        const cf Ee{xk.x + xm.x, xk.y - xm.y};
        const cf Dd{xk.x - xm.x, xk.y + xm.y};
        const cf w{twr[k].x, -twr[k].y};
        const cf Oo = cmul(Dd, w);
        rows[ik] = cf{Ee.x - Oo.y, Ee.y + Oo.x};
      }
      if (k != 0 && 2 * k != M) {
        const cf Ee{xm.x + xk.x, xm.y - xk.y};
        const cf Dd{xm.x - xk.x, xm.y + xk.y};
        const cf w{twr[M - k].x, -twr[M - k].y};
        const cf Oo = cmul(Dd, w);
        rows[im] = cf{Ee.x - Oo.y, Ee.y + Oo.x};
      }
    }
  }
  __syncthreads();
  {
    cf reg[E];
    fft<M, +1, false, false>(reg, rows + (t / TPL) * LS, t % TPL, stw, row_swz(M, t / TPL));
  }
  // rows now hold real lines, sample n of row l at float slot 2 rpos(l, n/2) + (n&1)
  if constexpr (MODE != MODE_BWD) {
    for (int e = t; e < TR * M; e += BR) {
      const int l = e / M, mm = e % M;
      const cf z = rows[rpos<M>(l, mm)];
      *reinterpret_cast<float2*>(chi_out + ((int64_t)j0 * RES + a0 + l) * RES + 2 * mm) = make_float2(z.x, z.y);
      if (MODE == MODE_FWD && j0 == 0 && a0 == 0 && e == 0) hdr->chi0 = (double)z.x;  // chi'(0,0,0) for Eq. 4
    }
  }
  if constexpr (MODE != MODE_DBG) {
    for_recs<KR, BR, rec_tail(RES)>(recs, sorted, R, t, [&](const float4& p0, const float4& p1, int64_t s) {
      const uint32_t bb = __float_as_uint(p0.w);
      const int b0 = bb & 1023, b1 = (bb >> 10) & 1023, b2 = bb >> 20;
      const int n0 = b2, n1 = (b2 + 1) & (RES - 1);

      const float fz = p0.z;
#pragma unroll
      for (int o0 = 0; o0 < 2; ++o0) {
        if (((b0 + o0) & (RES - 1)) != j0) continue;
        const float wa = o0 ? p0.x : 1.0f - p0.x;
        const float sa = o0 ? 1.0f : -1.0f;
#pragma unroll
        for (int o1 = 0; o1 < 2; ++o1) {
          const int l = (b1 + o1 - a0) & (RES - 1);
          if (l >= TR) continue;
          const float wb = o1 ? p0.y : 1.0f - p0.y;
          const float sb = o1 ? 1.0f : -1.0f;
          const float v0 = rf[2 * rpos<M>(l, n0 >> 1) + (n0 & 1)], v1 = rf[2 * rpos<M>(l, n1 >> 1) + (n1 & 1)];
          const float L = (1.0f - fz) * v0 + fz * v1;
          const float dL = v1 - v0;
          const float4 q = make_float4(wa * wb * L, (float)RES * sa * wb * L, (float)RES * wa * sb * L,
                                       (float)RES * wa * wb * dL);
          const int slot = o0 * 2 + o1;
          part[((MODE == MODE_FWD ? 0 : c * 4) + slot) * np + s] = q;
        }
      }
    });
  }
}

// ---------------------------------------------------------------------------
// Plane passes (res 64, 128, 256). One workgroup owns one j0 plane, or one
// part of it, and runs two transform axes on chip, so the data between the
// j2 and j1 axes never goes through HBM:
//   forward (P12, B12): rows of the plane -> r2c along j2 (LDS) -> FFT along
//     j1 (registers, LDS exchange) -> C[c][j0][k2][k1];
//   inverse (P45, B45): C[c][j0][k2][k1] -> IFFT along k1 (registers) ->
//     c2r along k2 (LDS) -> chi' rows and/or the gather at the points.
// The k2 = 0 and k2 = r/2 columns of a real row's spectrum are both real,
// so they travel through the j1 axis as one packed column X_0 + i X_{r/2}:
// r/2 complex columns per plane. At 256 a plane is split in two parts (k2
// halves forward, j1 halves inverse); each part redoes the other axis.
// ---------------------------------------------------------------------------
template <int RES>
struct Plane {
  static constexpr int M = RES / 2, H = M + 1;
  static constexpr int KP = RES >= PSR_PLANE_SPLIT_MIN ? 2 : 1;  // parts per plane
  static constexpr int NCOL = M / KP;            // packed columns per part (forward) / per round (inverse)
  static constexpr int TPL = plan_TPL(RES);      // threads per j1 line
  static constexpr int BLOCK = NCOL * TPL;
  static constexpr int TPR = plan_TPL(M);        // threads per half-length row
  static constexpr int RC = BLOCK / TPR;         // rows per chunk (forward) = rows per part (inverse)
  static constexpr int NCHUNK = RES / RC;
  static constexpr int LSR = row_ls(M), LSC = lstride(RES);
  static constexpr int SLOTS = RC * LSR > NCOL * LSC ? RC * LSR : NCOL * LSC;
  // waves per SIMD asked of the register allocator: two workgroups per CU
  // where LDS allows it (at most 128 VGPRs then)
  static constexpr int WPE = RES == 256 ? 4 : 2;
  static_assert(plan_E(RES) == 16 && plan_E(M) == 16, "plane passes hold 16 elements per thread");
  static_assert(NCHUNK * RC == RES && RES / KP == RC, "chunks and parts tile the plane");
};

// Where the plane passes pay: at 256 a plane needs all of LDS, one workgroup
// per CU, and each part redoes the other axis; only the inverse forward pass
// (one channel, no point-free skip lost) still gains there.
__host__ __device__ constexpr bool use_plane(int res) { return res >= 64 && res <= 128; }
__host__ __device__ constexpr bool use_plane_p45(int res) { return res >= 64 && res <= 256; }

// Workgroup -> (plane j0, sub-index u < U). The U workgroups of one plane
// get ids equal mod 8, so they are dispatched to the same XCD, close in
// time, and its L2 serves their repeated reads of the plane.
template <int U>
__device__ __forceinline__ void plane_of(int bid, int& j0, int& u) {
  const int x = bid & 7, q = bid >> 3;
  u = q % U;
  j0 = (q / U) * 8 + x;
}

enum { PF_SPLAT = 0, PF_BWDH = 1, PF_LOADV = 2 };

// Rows [a0, a0 + RC) of plane j0 of one channel into LDS (real samples at
// float slot 2 rpos(l, n/2) + (n & 1)), then the half-length FFT of each row in
// place. PF_SPLAT: trilinear splat of normal component ch; PF_BWDH: the
// cotangent H = s G + alpha W; PF_LOADV: v_ch rows from memory.
// Returns false, uniformly and before any barrier, when a splat span holds
// no point (its rows and spectra are zero and LDS is left untouched).
template <int RES, int MODE>
__device__ __forceinline__ bool pf_rows(cf* rows, const cf* stw, const PointRec* __restrict__ sorted,
                                        const int* __restrict__ off, const float* __restrict__ gin,
                                        float3 sqa, int j0, int a0, int ch) {
  using PL = Plane<RES>;
  constexpr int M = PL::M, RC = PL::RC, LSR = PL::LSR, BLOCK = PL::BLOCK;
  const int t = threadIdx.x;
  Ranges R{};
  if constexpr (MODE != PF_LOADV) R = span_ranges<RES, RC>(off, j0, a0);
  if (MODE == PF_SPLAT && R.total == 0) return false;
  fill_rows<RES, RC, BLOCK, MODE>(rows, sorted, R, gin, sqa, j0, a0, ch);
  {
    cf reg[16];
    fft<M, -1, false, false>(reg, rows + (t / PL::TPR) * LSR, t % PL::TPR, stw, row_swz(M, t / PL::TPR));
  }
  return true;
}

// X(a0 + l, k2) of packed column kk from row l's half-length spectrum Z:
// X_k = E_k + W_r^k O_k, E = (Z_k + Z*_{M-k}) / 2, O = (Z_k - Z*_{M-k}) / (2i);
// kk = 0 packs the two real end values, X_0 + i X_M = (Re Z_0 + Im Z_0) +
// i (Re Z_0 - Im Z_0).
template <int RES>
__device__ __forceinline__ cf pf_pick(const cf* rows, const cf* wr, int l, int kk) {
  constexpr int M = RES / 2;
  if (kk == 0) {
    const cf z = rows[rpos<M>(l, 0)];
    return cf{z.x + z.y, z.x - z.y};
  }
  const cf zk = rows[rpos<M>(l, kk)], zm = rows[rpos<M>(l, M - kk)];
  const cf Ee{0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y)};
  const cf Oo{0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x)};
  return cadd(Ee, cmul(wr[kk], Oo));
}

// P12 (MODE PF_SPLAT / PF_LOADV): one channel per workgroup, out v~_0,
// kappa_1(k1) v~_1 and kappa_2(k2) v~_2; the j0 pass sums the last two into
// W (the whole grid runs in one wave at 64^3 and 128^3, so equal workgroups
// beat one doing both W channels). B12 (PF_BWDH): H^ along (j2, j1). Output
// C[set][j0][k2][k1].
template <int RES, int MODE>
__device__ __forceinline__ void b_plane_fwd(const PointRec* __restrict__ sorted, const int* __restrict__ off,
                                            const float* __restrict__ gin, BwdScalars* __restrict__ bs,
                                            const double2* __restrict__ bpart, const SavedHeader* __restrict__ hdr,
                                            const cf* __restrict__ tw, cf* __restrict__ out, int bid) {
  using PL = Plane<RES>;
  constexpr int M = PL::M, H = PL::H, KP = PL::KP, NCOL = PL::NCOL, TPL = PL::TPL, RC = PL::RC;
  constexpr int NCHUNK = PL::NCHUNK, LSC = PL::LSC, BLOCK = PL::BLOCK;
  constexpr int NSET = MODE == PF_BWDH ? 1 : 3;
  constexpr int VPC = 16 / NCHUNK;  // register elements filled per chunk
  constexpr int64_t CH = (int64_t)H * RES * RES;
  __shared__ __align__(16) cf buf[PL::SLOTS];
  __shared__ cf stw[M];    // FFT table of length M (rows)
  __shared__ cf ctw[RES];  // FFT table of length RES (columns); its first M + 1 entries are W_r^k for the r2c
  stage_table<BLOCK>(stw, tw + M, M);
  stage_table<BLOCK>(ctw, tw + RES, RES);
  int j0, u;
  plane_of<KP * NSET>(bid, j0, u);
  const int part = u % KP, set = u / KP;
  const int t = threadIdx.x, col = t / TPL, lt = t % TPL;
  const int kk = part * NCOL + col;  // packed column index; 0 = (k2 = 0, k2 = M)
  cf* const o = out + set * CH + (int64_t)j0 * H * RES;
  if constexpr (MODE == PF_SPLAT) {
    // no point touches the plane: its spectrum is zero
    if (span_ranges<RES, RES>(off, j0, 0).total == 0) {
      const int nout = NCOL + (part == 0 ? 1 : 0);  // output k2 columns of this part (part 0 adds k2 = M)
      for (int e = t; e < nout * (RES / 2); e += BLOCK) {
        const int i = e / (RES / 2), k1 = 2 * (e % (RES / 2));
        const int k2 = i == NCOL ? M : part * NCOL + i;
        *reinterpret_cast<float4*>(o + (int64_t)k2 * RES + k1) = make_float4(0, 0, 0, 0);
      }
      return;
    }
  }
  float3 sqa = make_float3(1.0f, 0.0f, 1.0f);
  if constexpr (MODE == PF_BWDH) sqa = bwd_scalars<BLOCK>(bpart, bwd_reduce_blocks<RES>(), hdr, bs, bid == 0);
  cf reg[16];
  {
    const int ch = set;
#pragma unroll 1
    for (int q = 0; q < NCHUNK; ++q) {
      const int a0 = q * RC;
      const bool any = pf_rows<RES, MODE>(buf, stw, sorted, off, gin, sqa, j0, a0, ch);
#pragma unroll
      for (int w2 = 0; w2 < VPC; ++w2) {
        const cf x = any ? pf_pick<RES>(buf, ctw, lt + TPL * w2, kk) : cf{0.0f, 0.0f};
        // static register indices: chunk q fills reg[q VPC + w2]
#pragma unroll
        for (int qq = 0; qq < NCHUNK; ++qq)
          if (q == qq) reg[qq * VPC + w2] = x;
      }
      __syncthreads();  // the rows are overwritten next
    }
    fft<RES, -1, true, true>(reg, buf + col * LSC, lt, ctw);
  }
  if (set == 1 && kk != 0) {
#pragma unroll
    for (int v = 0; v < 16; ++v) reg[v] = cscale(reg[v], kappa_odd(lt + TPL * v, RES));
  }
  if (set == 2) {
    // kappa_2(k2); zero in the packed column (kappa_2^odd vanishes at k2 = 0 and M)
    const float k2f = kk == 0 ? 0.0f : kappa_odd(kk, RES);
#pragma unroll
    for (int v = 0; v < 16; ++v) reg[v] = cscale(reg[v], k2f);
  }
  // unpack the packed column with its mirror k1 -> -k1:
  // F_0 = (P(k) + P*(-k)) / 2, F_M = (P(k) - P*(-k)) / (2i)
  cf* const line = buf + col * LSC;
  if (kk == 0) {
#pragma unroll
    for (int v = 0; v < 16; ++v) line[pidx(lt + TPL * v)] = reg[v];
  }
  __syncthreads();
  if (kk == 0) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int k = lt + TPL * v;
      const cf pm = line[pidx((RES - k) & (RES - 1))];
      cf f0{0.5f * (reg[v].x + pm.x), 0.5f * (reg[v].y - pm.y)};
      cf fm{0.5f * (reg[v].y + pm.y), -0.5f * (reg[v].x - pm.x)};
      if (set == 1) {
        const float k1f = kappa_odd(k, RES);
        f0 = cscale(f0, k1f);
        fm = cscale(fm, k1f);
      }
      o[k] = f0;
      o[(int64_t)M * RES + k] = fm;
    }
  } else {
#pragma unroll
    for (int v = 0; v < 16; ++v) o[(int64_t)kk * RES + lt + TPL * v] = reg[v];
  }
}

// Splat test hook of the plane passes: the rows that P12 splats for plane
// j0 and channel c (the same fill_rows instantiation and spans), written to
// v_c[j0] instead of being transformed.
template <int RES>
__device__ __forceinline__ void b_plane_splat_dbg(const PointRec* __restrict__ sorted, const int* __restrict__ off,
                                                  float* __restrict__ vout, int bid) {
  using PL = Plane<RES>;
  constexpr int M = PL::M, RC = PL::RC, BLOCK = PL::BLOCK;
  constexpr int64_t N3 = (int64_t)RES * RES * RES;
  __shared__ __align__(16) cf buf[PL::SLOTS];
  const int j0 = bid / 3, c = bid % 3, t = threadIdx.x;
  const float* rf = reinterpret_cast<const float*>(buf);
#pragma unroll 1
  for (int q = 0; q < PL::NCHUNK; ++q) {
    const int a0 = q * RC;
    const Ranges R = span_ranges<RES, RC>(off, j0, a0);
    if (R.total > 0) fill_rows<RES, RC, BLOCK, PF_SPLAT>(buf, sorted, R, nullptr, make_float3(1.0f, 0.0f, 1.0f),
                                                         j0, a0, c);
    for (int e = t; e < RC * RES; e += BLOCK) {
      const int nn = e % RES, l = e / RES;
      vout[c * N3 + ((int64_t)j0 * RES + a0 + l) * RES + nn] =
          R.total > 0 ? rf[2 * rpos<M>(l, nn >> 1) + (nn & 1)] : 0.0f;
    }
    __syncthreads();
  }
}

enum { PI_FWD = 0, PI_BWD = 1, PI_DBG = 2 };

// P45 (PI_FWD): chi' rows and the gather partials at the points (slot-major,
// as in P5 / B5); PI_DBG:
// chi' rows only. B45 (PI_BWD, grid x3): g_v channel c = IFFT of V0, of
// kappa_1 U and of kappa_2 U, gather partials only; a part no point touches
// is skipped. Input C[c][j0][k2][k1]; part p owns rows j1 in [p RC, p RC + RC).
template <int RES, int MODE>
__device__ __forceinline__ void b_plane_inv(const cf* __restrict__ in, float* __restrict__ chi_out,
                                            SavedHeader* __restrict__ hdr,
                                            const PointRec* __restrict__ sorted, const int* __restrict__ off,
                                            float4* __restrict__ part, int64_t np, const cf* __restrict__ tw,
                                            int bid) {
  using PL = Plane<RES>;
  constexpr int M = PL::M, H = PL::H, KP = PL::KP, NCOL = PL::NCOL, TPL = PL::TPL, RC = PL::RC;
  constexpr int LSR = PL::LSR, LSC = PL::LSC, BLOCK = PL::BLOCK, TPR = PL::TPR;
  constexpr int NCH = MODE == PI_BWD ? 3 : 1;
  constexpr int VK = 16 / KP;  // elements kept per round: the part's rows of the column
  constexpr int64_t CH = (int64_t)H * RES * RES;
  constexpr bool WS = RES >= 256;  // wavefront-synchronous transforms
  __shared__ __align__(16) cf buf[PL::SLOTS];
  __shared__ cf stw[M];
  __shared__ cf ctw[RES];
  stage_table<BLOCK>(stw, tw + M, M);
  stage_table<BLOCK>(ctw, tw + RES, RES);
  float* const rf = reinterpret_cast<float*>(buf);
  int j0, u;
  plane_of<KP * NCH>(bid, j0, u);
  const int p = u % KP, c = u / KP;
  const int a0 = p * RC;
  const int t = threadIdx.x, col = t / TPL, lt = t % TPL;
  Ranges R{};
  if constexpr (MODE != PI_DBG) R = span_ranges<RES, RC>(off, j0, a0);
  const int total = R.total;
  if (MODE == PI_BWD && total == 0) return;
  const cf* const src = in + (MODE == PI_BWD && c > 0 ? CH : 0) + (int64_t)j0 * H * RES;
  cf keep[KP][VK];
#pragma unroll
  for (int rd = 0; rd < KP; ++rd) {
    const int kk = rd * NCOL + col;
    cf reg[16];
    if (kk == 0) {
      // pack the real-signal columns k2 = 0 and M: Z = A_0 + i A_M
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const cf a = src[lt + TPL * v], b = src[(int64_t)M * RES + lt + TPL * v];
        reg[v] = cf{a.x - b.y, a.y + b.x};
      }
    } else {
#pragma unroll
      for (int v = 0; v < 16; ++v) reg[v] = src[(int64_t)kk * RES + lt + TPL * v];
    }
    if (MODE == PI_BWD && c == 1) {
#pragma unroll
      for (int v = 0; v < 16; ++v) reg[v] = cscale(reg[v], kappa_odd(lt + TPL * v, RES));
    }
    if (MODE == PI_BWD && c == 2) {
      const float k2f = kk == 0 ? 0.0f : kappa_odd(kk, RES);
#pragma unroll
      for (int v = 0; v < 16; ++v) reg[v] = cscale(reg[v], k2f);
    }
    // at 256 the transforms synchronise within wavefronts only (a line's
    // threads are lanes of one wavefront; 16 wavefronts per workgroup): the
    // tables get a barrier of their own, after the first column loads are in
    // flight (P45 48.4 -> 47.4 us; at 64 and 128 the workgroup barriers cost
    // less than the extra ones here)
    if (WS && rd == 0) __syncthreads();
    fft<RES, +1, true, true, WS>(reg, buf + col * LSC, lt, ctw);
#pragma unroll
    for (int w2 = 0; w2 < VK; ++w2) {
      cf x = reg[w2];
#pragma unroll
      for (int pp = 1; pp < KP; ++pp)
        if (p == pp) x = reg[pp * VK + w2];
      keep[rd][w2] = x;
    }
  }
  // the part's rows into LDS, over the columns: every wavefront must be done
  // reading its columns (the last transform stage ends with a workgroup
  // barrier unless WS); row l = lt + TPL w2, packed column unpacked into
  // k2 = 0, M
  if constexpr (WS) __syncthreads();
#pragma unroll
  for (int rd = 0; rd < KP; ++rd) {
    const int kk = rd * NCOL + col;
#pragma unroll
    for (int w2 = 0; w2 < VK; ++w2) {
      const int l = lt + TPL * w2;
      if (kk == 0) {
        buf[rpos<M>(l, 0)] = cf{keep[rd][w2].x, 0.0f};
        buf[rpos<M>(l, M)] = cf{keep[rd][w2].y, 0.0f};
      } else {
        buf[rpos<M>(l, kk)] = keep[rd][w2];
      }
    }
  }
  // the first gather record of each thread, in flight during the row phase
  float4 pre0 = make_float4(0, 0, 0, 0), pre1 = pre0;
  int64_t pre_s = 0;
  if constexpr (MODE != PI_DBG) {
    if (t < total) {
      pre_s = range_pick(R, t);
      load_rec(sorted, pre_s, pre0, pre1);
    }
  }
  __syncthreads();
  // Hermitian half-spectrum X[0..M] -> packed spectrum Z[0..M) of the
  // even/odd samples: Z = (X_k + X*_{M-k}) + i (X_k - X*_{M-k}) e^{+2 pi i k/r}.
  {
    // k in [0, M/2) in runs of M/2 per row, then k = M/2 for every row (as in
    // the c2r of the row passes)
    constexpr int NH = M / 2;
    for (int e = t; e < RC * (NH + 1); e += BLOCK) {
      const int k = e < RC * NH ? e % NH : NH, row = e < RC * NH ? e / NH : e - RC * NH;
      const int ik = rpos<M>(row, k), im = rpos<M>(row, M - k);
      const cf xk = buf[ik], xm = buf[im];
      {
        const cf Ee{xk.x + xm.x, xk.y - xm.y};
        const cf Dd{xk.x - xm.x, xk.y + xm.y};
        const cf w{ctw[k].x, -ctw[k].y};
        const cf Oo = cmul(Dd, w);
        buf[ik] = cf{Ee.x - Oo.y, Ee.y + Oo.x};
      }
      if (k != 0 && 2 * k != M) {
        const cf Ee{xm.x + xk.x, xm.y - xk.y};
        const cf Dd{xm.x - xk.x, xm.y + xk.y};
        const cf w{ctw[M - k].x, -ctw[M - k].y};
        const cf Oo = cmul(Dd, w);
        buf[im] = cf{Ee.x - Oo.y, Ee.y + Oo.x};
      }
    }
  }
  __syncthreads();
  {
    cf reg[16];
    fft<M, +1, false, false, WS>(reg, buf + (t / TPR) * LSR, t % TPR, stw, row_swz(M, t / TPR));
  }
  if constexpr (WS) __syncthreads();  // the rows are read below across wavefronts
  // rows now hold real lines, sample n of row l at float slot 2 rpos(l, n/2) + (n&1)
  if constexpr (MODE != PI_BWD) {
    for (int e = t; e < RC * M; e += BLOCK) {
      const int l = e / M, mm = e % M;
      const cf z = buf[rpos<M>(l, mm)];
      *reinterpret_cast<float2*>(chi_out + ((int64_t)j0 * RES + a0 + l) * RES + 2 * mm) = make_float2(z.x, z.y);
      if (MODE == PI_FWD && j0 == 0 && a0 == 0 && e == 0) hdr->chi0 = (double)z.x;  // chi'(0,0,0) for Eq. 4
    }
  }
  if constexpr (MODE != PI_DBG) {
    // the thread's first record was fetched before the row phase; the rest
    // come in chunks, their loads in flight together
    Recs<1> first;
    first.a[0] = pre0;
    first.b[0] = pre1;
    first.s[0] = pre_s;
    for_recs<1, BLOCK, rec_tail(RES)>(first, sorted, R, t, [&](const float4& p0, const float4&, int64_t s) {
      const uint32_t bb = __float_as_uint(p0.w);
      const int b0 = bb & 1023, b1 = (bb >> 10) & 1023, b2 = bb >> 20;
      const int n0 = b2, n1 = (b2 + 1) & (RES - 1);
      const float fz = p0.z;
#pragma unroll
      for (int o0 = 0; o0 < 2; ++o0) {
        if (((b0 + o0) & (RES - 1)) != j0) continue;
        const float wa = o0 ? p0.x : 1.0f - p0.x;
        const float sa = o0 ? 1.0f : -1.0f;
#pragma unroll
        for (int o1 = 0; o1 < 2; ++o1) {
          const int l = (b1 + o1 - a0) & (RES - 1);
          if (l >= RC) continue;
          const float wb = o1 ? p0.y : 1.0f - p0.y;
          const float sb = o1 ? 1.0f : -1.0f;
          const float v0 = rf[2 * rpos<M>(l, n0 >> 1) + (n0 & 1)], v1 = rf[2 * rpos<M>(l, n1 >> 1) + (n1 & 1)];
          const float L = (1.0f - fz) * v0 + fz * v1;
          const float dL = v1 - v0;
          const float4 qv = make_float4(wa * wb * L, (float)RES * sa * wb * L, (float)RES * wa * sb * L,
                                        (float)RES * wa * wb * dL);
          const int slot = o0 * 2 + o1;
          part[((MODE == PI_FWD ? 0 : c * 4) + slot) * np + s] = qv;
        }
      }
    });
  }
}

// ---------------------------------------------------------------------------
// FP64 reductions and normalisation (main Eq. 4)
// ---------------------------------------------------------------------------

// Per point: f_i = sum of its 4 corner-line partials (FP64), grad f_i (FP32).
__device__ __forceinline__ void b_fwd_point_reduce(const float4* __restrict__ part, int64_t npoints,
                                                          float4* __restrict__ gradf, double* __restrict__ blockpart, int bid, int nblocks) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t s = (int64_t)bid * blockDim.x + threadIdx.x; s < npoints; s += (int64_t)nblocks * blockDim.x) {
    const float4 q0 = part[s], q1 = part[npoints + s], q2 = part[2 * npoints + s], q3 = part[3 * npoints + s];
    const double f = ((double)q0.x + (double)q1.x) + ((double)q2.x + (double)q3.x);
    gradf[s] = make_float4((q0.y + q1.y) + (q2.y + q3.y), (q0.z + q1.z) + (q2.z + q3.z),
                           (q0.w + q1.w) + (q2.w + q3.w), (float)f);
    acc += f;
  }
  const double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) blockpart[bid] = tot;
}

// mu = (1/P) sum_i f_i, c = chi'(0) - mu (reading B) or chi'(0) (reading A),
// s = m/|c| (main Eq. 4), status; block partials summed in a fixed order.
// mu, c and s (main Eq. 4) from the per-block FP64 sums of f_i; every caller
// sums the same partials in the same order, so all agree bit for bit.
__device__ __forceinline__ void fwd_scalars(const double* __restrict__ blockpart, int nb,
                                            const SavedHeader* __restrict__ hdr, double& mu, double& scale,
                                            double& c, int& status) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) a += blockpart[i];
  const double tot = block_sum(a, sh);
  mu = tot / (double)hdr->npoints;
  const double chi0 = hdr->chi0;
  c = hdr->reading == 0 ? chi0 - mu : chi0;
  status = 0;
  if (hdr->flags & 1) status = -6;  // PSR_ENONFINITE
  else if (!(c != 0.0) || !isfinite(c) || !isfinite(mu)) status = -3;  // PSR_EDEGENERATE
  scale = status ? __longlong_as_double(0x7ff8000000000000LL) : (double)hdr->m / fabs(c);
}

// chi = s (chi' - mu) in place; block 0 also records the scalars and the
// status in the header (chi'(0) was recorded there by the c2r pass).
__device__ __forceinline__ void b_normalize(float* __restrict__ chi, int64_t n, const double* __restrict__ blockpart,
                                            int nb, SavedHeader* __restrict__ hdr, int bid, int nblocks) {
  double mu, s, c;
  int status;
  fwd_scalars(blockpart, nb, hdr, mu, s, c, status);
  if (bid == 0 && threadIdx.x == 0) {
    hdr->status = status;
    hdr->mu = mu;
    hdr->cscale = c;
    hdr->scale = s;
  }
  float4* c4 = reinterpret_cast<float4*>(chi);
  for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n / 4; i += (int64_t)nblocks * blockDim.x) {
    float4 v = c4[i];
    v.x = (float)(((double)v.x - mu) * s);
    v.y = (float)(((double)v.y - mu) * s);
    v.z = (float)(((double)v.z - mu) * s);
    v.w = (float)(((double)v.w - mu) * s);
    c4[i] = v;
  }
}

// Backward: S_G = sum G, S_Gchi = sum G chi (FP64 partials per block).
__device__ __forceinline__ void b_bwd_reduce(const float* __restrict__ G, const float* __restrict__ chi,
                                                    int64_t n, double2* __restrict__ blockpart, int bid, int nblocks) {
  __shared__ double sh[256];
  double sg = 0.0, sgc = 0.0;
  const float4* g4 = reinterpret_cast<const float4*>(G);
  const float4* c4 = reinterpret_cast<const float4*>(chi);
#pragma unroll 4
  for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n / 4; i += (int64_t)nblocks * blockDim.x) {
    const float4 g = g4[i], c = c4[i];
    sg += ((double)g.x + (double)g.y) + ((double)g.z + (double)g.w);
    sgc += ((double)g.x * c.x + (double)g.y * c.y) + ((double)g.z * c.z + (double)g.w * c.w);
  }
  const double a = block_sum(sg, sh);
  const double b = block_sum(sgc, sh);
  if (threadIdx.x == 0) blockpart[bid] = make_double2(a, b);
}

// The response of the backward to the point source -Q delta_0 at a grid
// vertex v, channel d: K_d(v) = Re IFFT(conj(A_d))(v), A_d the operator of
// main Eq. 3 for channel d. K_0 is odd in j0 and even in j1 and j2, and K_d
// is K_0 with axes d and 0 exchanged, so one octant [0, r/2]^3 of K_0
// (ktab[(i0 (h) + i1) h + i2], h = r/2 + 1) serves all three channels.
template <int RES>
__device__ __forceinline__ float ktab_at(const float* __restrict__ kt, int d, int v0, int v1, int v2) {
  constexpr int H = RES / 2, HP = H + 1;
  const int a = d == 0 ? v0 : (d == 1 ? v1 : v2);
  const int b = d == 0 ? v1 : v0;
  const int c = d == 2 ? v1 : v2;
  const bool neg = a > H;
  const int ia = neg ? RES - a : a, ib = b > H ? RES - b : b, ic = c > H ? RES - c : c;
  const float k = kt[((int64_t)ia * HP + ib) * HP + ic];
  return neg ? -k : k;
}

// dn = sum of the 4 corner-line partials of each channel (gather of dL/dv),
// dc = sum over channels of n_d times the weight-gradient partials, plus
// alpha grad chi'(c_i) (the mean term); then the point source -Q delta_0 of
// the cotangent, applied here from the table: -Q K_d gathered at the point
// into dn_d, and -Q sum_d n_d K_d through the weight gradient into dc.
// Eight lanes per point, one per corner o: each reads its corner's three
// table values and (lanes 0-5) two of the twelve partials, and the lanes'
// shares are summed with shuffles in a fixed order.
constexpr int kFinalLanes = 8;

template <int RES>
__device__ __forceinline__ void b_bwd_point_finalize(const float4* __restrict__ part, const float4* __restrict__ gradf,
                                     const PointRec* __restrict__ sorted, const BwdScalars* __restrict__ bs,
                                     const float* __restrict__ ktab, int64_t npoints, float* __restrict__ dpoints,
                                     float* __restrict__ dnormals, int bid) {
  const int64_t s = ((int64_t)bid * blockDim.x + threadIdx.x) / kFinalLanes;
  const int o = threadIdx.x % kFinalLanes;
  const bool live = s < npoints;  // the 8 lanes of a point agree (whole groups only)
  const int64_t sr = live ? s : 0;
  float4 p0, p1;
  load_rec(sorted, sr, p0, p1);
  const float nv[3] = {p1.x, p1.y, p1.z};
  float dn[3] = {0.0f, 0.0f, 0.0f}, dc[3] = {0.0f, 0.0f, 0.0f};
  // partials (c, slot) = (o / 2, 2 (o % 2) + h) for lanes 0-5: channel c, two slots each
  if (o < 6 && live) {
    const int c = o >> 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float4 q = part[(c * 4 + 2 * (o & 1) + h) * npoints + s];
      dn[c] += q.x;
      dc[0] += nv[c] * q.y;
      dc[1] += nv[c] * q.z;
      dc[2] += nv[c] * q.w;
    }
  }
  {
    const float mq = -bs->q;
    const uint32_t bb = __float_as_uint(p0.w);
    const int o0 = o & 1, o1 = (o >> 1) & 1, o2 = o >> 2;
    const int v0 = ((bb & 1023) + o0) & (RES - 1), v1 = (((bb >> 10) & 1023) + o1) & (RES - 1),
              v2 = ((bb >> 20) + o2) & (RES - 1);
    const float w0 = o0 ? p0.x : 1.0f - p0.x, w1 = o1 ? p0.y : 1.0f - p0.y, w2 = o2 ? p0.z : 1.0f - p0.z;
    const float k0 = ktab_at<RES>(ktab, 0, v0, v1, v2), k1 = ktab_at<RES>(ktab, 1, v0, v1, v2),
                k2 = ktab_at<RES>(ktab, 2, v0, v1, v2);
    const float w = (w0 * w1) * w2;
    const float nk = mq * (nv[0] * k0 + nv[1] * k1 + nv[2] * k2);
    dn[0] += mq * (w * k0);
    dn[1] += mq * (w * k1);
    dn[2] += mq * (w * k2);
    dc[0] += (float)RES * ((o0 ? 1.0f : -1.0f) * (w1 * w2) * nk);
    dc[1] += (float)RES * ((o1 ? 1.0f : -1.0f) * (w0 * w2) * nk);
    dc[2] += (float)RES * ((o2 ? 1.0f : -1.0f) * (w0 * w1) * nk);
  }
#pragma unroll
  for (int d = 1; d < kFinalLanes; d <<= 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      dn[k] += __shfl_xor(dn[k], d, kFinalLanes);
      dc[k] += __shfl_xor(dc[k], d, kFinalLanes);
    }
  }
  if (!live || o != 0) return;
  const float alpha = bs->alpha;
  const float4 g = gradf[s];
  dc[0] += alpha * g.x;
  dc[1] += alpha * g.y;
  dc[2] += alpha * g.z;
  const int64_t i = (int64_t)__float_as_uint(p1.w);
  if (dpoints) {
    dpoints[3 * i + 0] = dc[0];
    dpoints[3 * i + 1] = dc[1];
    dpoints[3 * i + 2] = dc[2];
  }
  if (dnormals) {
    dnormals[3 * i + 0] = dn[0];
    dnormals[3 * i + 1] = dn[1];
    dnormals[3 * i + 2] = dn[2];
  }
}

// ---------------------------------------------------------------------------
// Point-source table, built in FP64 once per (res, sigma). With h = r/2 and
// the spectrum folded onto k in [0, h]^3 (K_0 is a sine series along k0 and
// cosine series along k1, k2; wk = 1 at k = 0 and h, 2 between):
//   K_0(j) = -(2/N) sum_{k0=1}^{h-1} sum_{k1,k2=0}^{h} wk1 wk2 g(k) k0 /
//            (2 pi |k|^2) sin(2 pi k0 j0 / r) cos(2 pi k1 j1 / r) cos(2 pi k2 j2 / r)
// (g the Gaussian of main Eq. 3; the Nyquist k0 = h carries no odd factor).
// Three separable passes over the octant, each one output per thread.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ktab_trig(double* __restrict__ cs, double* __restrict__ sn, int r) {
  const int hp = r / 2 + 1;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= hp * hp) return;
  const int k = e / hp, j = e % hp;
  double sv, cv;
  sincospi(2.0 * (double)((k * j) % r) / (double)r, &sv, &cv);
  cs[e] = cv;
  sn[e] = sv;
}

__device__ __forceinline__ double ktab_g1(int k, double sigma, int r) {
  return exp(-2.0 * sigma * sigma * (double)k * (double)k / ((double)r * (double)r));
}

// pass 1: A1[k0][k1][j2] = sum_k2 wk2 g1(k2) cos(k2 j2) / (k0^2 + k1^2 + k2^2)   (k0 >= 1)
__global__ __launch_bounds__(256) void k_ktab_pass1(const double* __restrict__ cs, double* __restrict__ out,
                                                    double sigma, int r) {
  const int h = r / 2, hp = h + 1;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)hp * hp * hp) return;
  const int j2 = (int)(e % hp), k1 = (int)((e / hp) % hp), k0 = (int)(e / ((int64_t)hp * hp));
  double acc = 0.0;
  if (k0 >= 1 && k0 < h) {
    const double q = (double)k0 * k0 + (double)k1 * k1;
    for (int k2 = 0; k2 <= h; ++k2) {
      const double wk = (k2 == 0 || k2 == h) ? 1.0 : 2.0;
      acc += wk * ktab_g1(k2, sigma, r) * cs[k2 * hp + j2] / (q + (double)k2 * k2);
    }
  }
  out[e] = acc;
}

// pass 2: A2[k0][j1][j2] = sum_k1 wk1 g1(k1) cos(k1 j1) A1[k0][k1][j2]
__global__ __launch_bounds__(256) void k_ktab_pass2(const double* __restrict__ cs, const double* __restrict__ in,
                                                    double* __restrict__ out, double sigma, int r) {
  const int h = r / 2, hp = h + 1;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)hp * hp * hp) return;
  const int j2 = (int)(e % hp), j1 = (int)((e / hp) % hp), k0 = (int)(e / ((int64_t)hp * hp));
  double acc = 0.0;
  for (int k1 = 0; k1 <= h; ++k1) {
    const double wk = (k1 == 0 || k1 == h) ? 1.0 : 2.0;
    acc += wk * ktab_g1(k1, sigma, r) * cs[k1 * hp + j1] * in[((int64_t)k0 * hp + k1) * hp + j2];
  }
  out[e] = acc;
}

// pass 3: K_0[j0][j1][j2] = -(2/N) / (2 pi) sum_{k0=1}^{h-1} k0 g1(k0) sin(k0 j0) A2[k0][j1][j2]
__global__ __launch_bounds__(256) void k_ktab_pass3(const double* __restrict__ sn, const double* __restrict__ in,
                                                    float* __restrict__ table, double sigma, int r) {
  const int h = r / 2, hp = h + 1;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)hp * hp * hp) return;
  const int j2 = (int)(e % hp), j1 = (int)((e / hp) % hp), j0 = (int)(e / ((int64_t)hp * hp));
  double acc = 0.0;
  for (int k0 = 1; k0 < h; ++k0)
    acc += (double)k0 * ktab_g1(k0, sigma, r) * sn[k0 * hp + j0] * in[((int64_t)k0 * hp + j1) * hp + j2];
  const double n3 = (double)r * (double)r * (double)r;
  table[e] = (float)(-2.0 / n3 / (2.0 * M_PI) * acc);
}

int build_point_source_table(int res, float sigma, float* table, void* scratch, hipStream_t stream) {
  const size_t hp = (size_t)res / 2 + 1;
  char* b = static_cast<char*>(scratch);
  double* a1 = reinterpret_cast<double*>(b);
  double* a2 = reinterpret_cast<double*>(b + align256(hp * hp * hp * 8));
  double* cs = reinterpret_cast<double*>(b + 2 * align256(hp * hp * hp * 8));
  double* sn = reinterpret_cast<double*>(b + 2 * align256(hp * hp * hp * 8) + align256(hp * hp * 8));
  const int n2 = (int)((hp * hp + 255) / 256), n3 = (int)((hp * hp * hp + 255) / 256);
  hipLaunchKernelGGL(k_ktab_trig, dim3(n2), dim3(256), 0, stream, cs, sn, res);
  hipLaunchKernelGGL(k_ktab_pass1, dim3(n3), dim3(256), 0, stream, cs, a1, (double)sigma, res);
  hipLaunchKernelGGL(k_ktab_pass2, dim3(n3), dim3(256), 0, stream, cs, a1, a2, (double)sigma, res);
  hipLaunchKernelGGL(k_ktab_pass3, dim3(n3), dim3(256), 0, stream, sn, a2, table, (double)sigma, res);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// ---------------------------------------------------------------------------
// __global__ wrappers: resolve the job of this workgroup and its buffers.
// ---------------------------------------------------------------------------
template <int MAXJ>
__device__ __forceinline__ int job_of(const Batch<MAXJ>& B, int blk) {
  if constexpr (MAXJ == 1) {
    return 0;
  } else {
    int lo = 0, hi = B.n - 1;  // last j with start[j] <= blk
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (B.start[mid] <= blk) lo = mid;
      else hi = mid - 1;
    }
    return lo;
  }
}

#define PSR_JOB(RES)                                                  \
  const int j_ = job_of(B, blockIdx.x);                               \
  const int bid = blockIdx.x - B.start[j_];                           \
  const int nbl = B.start[j_ + 1] - B.start[j_];                      \
  const JobArg& J = B.job[j_];                                        \
  const WsView w = ws_view(J.ws, ws_layout(RES, J.P));                \
  const SavedView sv = saved_view(J.sv, saved_layout(RES, J.P));      \
  (void)nbl;                                                          \
  (void)w;                                                            \
  (void)sv

// Backward kernels: the saved state must come from a forward of the same
// resolution and point count (its header records both). Otherwise the saved
// records and the workspace would be indexed with the wrong layout, so every
// backward kernel returns at once; the last one fills the gradients with NaN.
template <int RES>
__device__ __forceinline__ bool saved_mismatch(const SavedHeader* __restrict__ hdr, int64_t P) {
  return hdr->res != RES || hdr->npoints != P;
}
#define PSR_BWD_GUARD(RES) \
  if (saved_mismatch<RES>(sv.hdr, J.P)) return

template <int RES, int MAXJ>
__global__ __launch_bounds__(256) void k_init(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  b_init(w.counts, num_bins(RES), sv.hdr, RES, J.P, J.sigma, B.m, B.reading, bid, nbl);
}

template <int RES, int MAXJ>
__global__ __launch_bounds__(256) void k_bin(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  b_bin<RES>(J.pts, J.nrm, J.P, w.counts, w.tmp, w.colrank, sv.hdr, bid);
}

template <int RES, int MAXJ>
__global__ __launch_bounds__(1024) void k_scan(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  b_scan(w.counts, sv.off, num_bins(RES), bid);
  b_live_planes<RES>(sv.off, sv.hdr);
}

template <int RES, int MAXJ>
__global__ __launch_bounds__(256) void k_scatter(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  b_scatter(w.tmp, w.colrank, sv.off, sv.sorted, J.P, bid);
}

template <int RES, int MAXJ>
__global__ __launch_bounds__(256) void k_scan_scatter(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  constexpr int NB = num_bins(RES);
  static_assert(NB <= kLdsBins, "bins fit in LDS");
  __shared__ int soff[NB + 1];
  scan_to_lds<NB, 256>(w.counts, soff);
  if (bid == 0) {
    for (int e = threadIdx.x; e <= NB; e += 256) sv.off[e] = soff[e];
    b_live_planes<RES>(soff, sv.hdr);
  }
  b_scatter(w.tmp, w.colrank, soff, sv.sorted, J.P, bid);
}

template <int RES, int MODE, int MAXJ>
__global__ __launch_bounds__(rows_wg(RES)) void k_splat_r2c(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  if constexpr (MODE == MODE_BWDH || MODE == MODE_BWDA) { PSR_BWD_GUARD(RES); }
  const float* gin = MODE == MODE_BWDH || MODE == MODE_BWDA ? J.dchi : J.aux_in;
  b_splat_r2c<RES, MODE>(sv.sorted, sv.off, gin, w.bs, (const double2*)w.blockpart, sv.hdr, B.tw, w.X, J.aux_out,
                         J.chi, (double2*)w.blockpart, bid);
}

template <int RES, bool MERGE, bool SKIP, int MAXJ>
__global__ __launch_bounds__(cols_block(RES)) void k_axis1_fwd(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  if constexpr (!MERGE) { PSR_BWD_GUARD(RES); }
  b_axis1_fwd<RES, MERGE, SKIP>(w.X, w.Y, B.tw, sv.hdr->tlive, bid);
}

template <int RES, bool SKIP, int MAXJ>
__global__ __launch_bounds__(j0_block(RES)) void k_fwd_axis0(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  constexpr bool SK = SKIP && !use_plane(RES);
  b_fwd_axis0<RES, use_plane(RES), SK>(w.Y, w.X, B.tw, J.sigma, SK ? sv.hdr->live : nullptr, bid);
}

template <int RES, int MAXJ>
__global__ __launch_bounds__(j0_block(RES)) void k_bwd_axis0(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  PSR_BWD_GUARD(RES);
  b_bwd_axis0<RES, use_plane(RES)>(w.Y, w.X, B.tw, J.sigma, sv.off, bid);
}

template <int RES, bool SPLIT, int MAXJ>
__global__ __launch_bounds__(cols_block(RES)) void k_axis1_inv(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  if constexpr (SPLIT) { PSR_BWD_GUARD(RES); }
  b_axis1_inv<RES, SPLIT>(w.X, w.Y, B.tw, sv.off, bid);
}

template <int RES, int MODE, int MAXJ>
__global__ __launch_bounds__(rows_wg(RES)) void k_c2r_gather(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  if constexpr (MODE == MODE_BWD) { PSR_BWD_GUARD(RES); }
  float* out = MODE == MODE_DBG ? J.aux_out : J.chi;
  b_c2r_gather<RES, MODE>(w.Y, out, sv.hdr, sv.sorted, sv.off, w.part, J.P, B.tw, bid);
}

template <int RES, int MODE, int MAXJ>
__global__ __launch_bounds__(Plane<RES>::BLOCK) __attribute__((amdgpu_waves_per_eu(Plane<RES>::WPE)))
void k_plane_fwd(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  if constexpr (MODE == PF_BWDH) { PSR_BWD_GUARD(RES); }
  const float* gin = MODE == PF_BWDH ? J.dchi : J.aux_in;
  b_plane_fwd<RES, MODE>(sv.sorted, sv.off, gin, w.bs, (const double2*)w.blockpart, sv.hdr, B.tw, w.Y, bid);
}

template <int RES, int MODE, int MAXJ>
__global__ __launch_bounds__(Plane<RES>::BLOCK) __attribute__((amdgpu_waves_per_eu(Plane<RES>::WPE)))
void k_plane_inv(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  if constexpr (MODE == PI_BWD) { PSR_BWD_GUARD(RES); }
  float* outp = MODE == PI_DBG ? J.aux_out : J.chi;
  b_plane_inv<RES, MODE>(w.X, outp, sv.hdr, sv.sorted, sv.off, w.part, J.P, B.tw, bid);
}

template <int RES, int MAXJ>
__global__ __launch_bounds__(Plane<RES>::BLOCK) __attribute__((amdgpu_waves_per_eu(Plane<RES>::WPE)))
void k_plane_splat_dbg(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  b_plane_splat_dbg<RES>(sv.sorted, sv.off, J.aux_out, bid);
}

template <int RES, int MAXJ>
__global__ __launch_bounds__(256) void k_fwd_point_reduce(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  b_fwd_point_reduce(w.part, J.P, sv.gradf, w.blockpart, bid, nbl);
}

template <int RES, int MAXJ>
__global__ __launch_bounds__(256) void k_normalize(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  const int nb = (int)((J.P + 255) / 256) > kRedBlocks ? kRedBlocks : (int)((J.P + 255) / 256);
  b_normalize(J.chi, (int64_t)RES * RES * RES, w.blockpart, nb, sv.hdr, bid, nbl);
}

template <int RES, int MAXJ>
__global__ __launch_bounds__(256) void k_bwd_reduce(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  PSR_BWD_GUARD(RES);
  b_bwd_reduce(J.dchi, J.chi, (int64_t)RES * RES * RES, (double2*)w.blockpart, bid, nbl);
}



template <int RES, int MAXJ>
__global__ __launch_bounds__(256) void k_bwd_point_finalize(const Batch<MAXJ> B) {
  PSR_JOB(RES);
  if (saved_mismatch<RES>(sv.hdr, J.P)) {
    const int64_t s = ((int64_t)bid * blockDim.x + threadIdx.x) / kFinalLanes;
    const float nan = __int_as_float(0x7fc00000);
    for (int k = 0; k < 3 && s < J.P && threadIdx.x % kFinalLanes == 0; ++k) {
      if (J.dpts) J.dpts[3 * s + k] = nan;
      if (J.dnrm) J.dnrm[3 * s + k] = nan;
    }
    return;
  }
  b_bwd_point_finalize<RES>(w.part, sv.gradf, sv.sorted, w.bs, J.ktab, J.P, J.dpts, J.dnrm, bid);
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free forward (psr_forward_static): the workspace
// and the saved state of one solve, in one static array per GPU. Host code
// must not pass the array's name to a kernel (on the host it only stands for
// the symbol); the library takes its device address once per device at
// context creation and passes that.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

int static_scratch_address(void** out) {
  *out = nullptr;
  return hipGetSymbolAddress(out, HIP_SYMBOL(scratch)) == hipSuccess ? 0 : -4;
}

// ---------------------------------------------------------------------------
// host-side launch sequences
// ---------------------------------------------------------------------------
static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }
constexpr int nblk_c(int64_t n, int b) { return (int)((n + b - 1) / b); }

template <int RES>
struct Grid {
  static constexpr int H = RES / 2 + 1;
  static constexpr int rows = RES * row_tiles(RES);        // row-pass workgroups per channel
  static constexpr int cols = H * (RES / tile_cols(RES));  // column-pass workgroups per channel
  static constexpr int j0s = H * (RES / tile_j0(RES));     // workgroups of the fused j0 passes
  static constexpr int BJ = j0_block(RES);
  static constexpr int BR = rows_wg(RES), BC = cols_block(RES);
  static constexpr int64_t N3 = (int64_t)RES * RES * RES;
  static constexpr int init_blocks = nblk_c(num_bins(RES), 256) > 64 ? 64 : nblk_c(num_bins(RES), 256);
  static constexpr int norm_blocks = nblk_c(N3 / 4, 256) > 1024 ? 1024 : nblk_c(N3 / 4, 256);
};

// Launch kernel K once per chunk of up to MAXJ jobs; workgroups per job from nb(job).
template <int MAXJ, typename NB>
static int launch(Exec& x, void (*K)(const Batch<MAXJ>), int block, const JobArg* jobs, int n, NB nb) {
  for (int c0 = 0; c0 < n; c0 += MAXJ) {
    Batch<MAXJ> B;
    B.tw = x.tw;
    B.m = (float)x.m;
    B.reading = x.reading;
    B.n = n - c0 < MAXJ ? n - c0 : MAXJ;
    int total = 0;
    for (int j = 0; j < B.n; ++j) {
      B.job[j] = jobs[c0 + j];
      B.start[j] = total;
      const int nbj = nb(jobs[c0 + j]);
      if (nbj < 1) return -4;  // every stage has work for every job
      total += nbj;
    }
    B.start[B.n] = total;
    hipLaunchKernelGGL(K, dim3(total), dim3(block), 0, x.stream, B);
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

template <int RES, int MAXJ>
static int seq_forward(Exec& x, const JobArg* J, int n) {
  using G = Grid<RES>;
  int rc = 0;
  auto c = [](int v) { return [v](const JobArg&) { return v; }; };
  x.begin(STAGE_BIN);
  rc |= launch<MAXJ>(x, k_init<RES, MAXJ>, 256, J, n, c(G::init_blocks));
  rc |= launch<MAXJ>(x, k_bin<RES, MAXJ>, 256, J, n, [](const JobArg& a) { return nblk(a.P, kBinChunk); });
  if constexpr (num_bins(RES) <= kLdsBins) {
    rc |= launch<MAXJ>(x, k_scan_scatter<RES, MAXJ>, 256, J, n, [](const JobArg& a) { return nblk(a.P, 256); });
  } else {
    rc |= launch<MAXJ>(x, k_scan<RES, MAXJ>, 1024, J, n, c(1));
    rc |= launch<MAXJ>(x, k_scatter<RES, MAXJ>, 256, J, n, [](const JobArg& a) { return nblk(a.P, 256); });
  }
  x.end(STAGE_BIN);
  if constexpr (use_plane(RES)) {
    x.begin(STAGE_P12);
    rc |= launch<MAXJ>(x, k_plane_fwd<RES, PF_SPLAT, MAXJ>, Plane<RES>::BLOCK, J, n, c(RES * Plane<RES>::KP * 3));
    x.end(STAGE_P12);
  } else {
    x.begin(STAGE_P1);
    rc |= launch<MAXJ>(x, k_splat_r2c<RES, MODE_SPLAT, MAXJ>, G::BR, J, n, c(3 * G::rows));
    x.end(STAGE_P1);
    x.begin(STAGE_P2);
    rc |= launch<MAXJ>(x, k_axis1_fwd<RES, true, true, MAXJ>, G::BC, J, n, c(2 * G::cols));
    x.end(STAGE_P2);
  }
  x.begin(STAGE_P3);
  rc |= launch<MAXJ>(x, k_fwd_axis0<RES, true, MAXJ>, G::BJ, J, n, c(G::j0s));
  x.end(STAGE_P3);
  if constexpr (use_plane_p45(RES)) {
    x.begin(STAGE_P45);
    rc |= launch<MAXJ>(x, k_plane_inv<RES, PI_FWD, MAXJ>, Plane<RES>::BLOCK, J, n, c(RES * Plane<RES>::KP));
    x.end(STAGE_P45);
  } else {
    x.begin(STAGE_P4);
    rc |= launch<MAXJ>(x, k_axis1_inv<RES, false, MAXJ>, G::BC, J, n, c(G::cols));
    x.end(STAGE_P4);
    x.begin(STAGE_P5);
    rc |= launch<MAXJ>(x, k_c2r_gather<RES, MODE_FWD, MAXJ>, G::BR, J, n, c(G::rows));
    x.end(STAGE_P5);
  }
  x.begin(STAGE_FWD_REDUCE);
  rc |= launch<MAXJ>(x, k_fwd_point_reduce<RES, MAXJ>, 256, J, n,
                     [](const JobArg& a) { return nblk(a.P, 256) > kRedBlocks ? kRedBlocks : nblk(a.P, 256); });
  x.end(STAGE_FWD_REDUCE);
  x.begin(STAGE_NORMALIZE);
  rc |= launch<MAXJ>(x, k_normalize<RES, MAXJ>, 256, J, n, c(G::norm_blocks));
  x.end(STAGE_NORMALIZE);
  return rc ? -4 : 0;
}

template <int RES, int MAXJ>
static int seq_backward(Exec& x, const JobArg* J, int n) {
  using G = Grid<RES>;
  int rc = 0;
  auto c = [](int v) { return [v](const JobArg&) { return v; }; };
  if constexpr (use_plane(RES)) {
    x.begin(STAGE_BWD_REDUCE);
    rc |= launch<MAXJ>(x, k_bwd_reduce<RES, MAXJ>, 256, J, n, c(bwd_reduce_blocks<RES>()));
    x.end(STAGE_BWD_REDUCE);
    x.begin(STAGE_B12);
    rc |= launch<MAXJ>(x, k_plane_fwd<RES, PF_BWDH, MAXJ>, Plane<RES>::BLOCK, J, n, c(RES * Plane<RES>::KP));
    x.end(STAGE_B12);
  } else {
    // the reductions ride on the first row pass, which also transforms the
    // row tiles that need no backward scalar; the second takes the rest
    x.begin(STAGE_B1A);
    rc |= launch<MAXJ>(x, k_splat_r2c<RES, MODE_BWDA, MAXJ>, G::BR, J, n, c(G::rows));
    x.end(STAGE_B1A);
    x.begin(STAGE_B1);
    rc |= launch<MAXJ>(x, k_splat_r2c<RES, MODE_BWDH, MAXJ>, G::BR, J, n, c(G::rows));
    x.end(STAGE_B1);
    x.begin(STAGE_B2);
    rc |= launch<MAXJ>(x, k_axis1_fwd<RES, false, false, MAXJ>, G::BC, J, n, c(G::cols));
    x.end(STAGE_B2);
  }
  x.begin(STAGE_B3);
  rc |= launch<MAXJ>(x, k_bwd_axis0<RES, MAXJ>, G::BJ, J, n, c(G::j0s));
  x.end(STAGE_B3);
  if constexpr (use_plane(RES)) {
    x.begin(STAGE_B45);
    rc |= launch<MAXJ>(x, k_plane_inv<RES, PI_BWD, MAXJ>, Plane<RES>::BLOCK, J, n, c(RES * Plane<RES>::KP * 3));
    x.end(STAGE_B45);
  } else {
    x.begin(STAGE_B4);
    rc |= launch<MAXJ>(x, k_axis1_inv<RES, true, MAXJ>, G::BC, J, n, c(2 * G::cols));
    x.end(STAGE_B4);
    x.begin(STAGE_B5);
    rc |= launch<MAXJ>(x, k_c2r_gather<RES, MODE_BWD, MAXJ>, G::BR, J, n, c(3 * G::rows));
    x.end(STAGE_B5);
  }
  x.begin(STAGE_BWD_FINAL);
  rc |= launch<MAXJ>(x, k_bwd_point_finalize<RES, MAXJ>, 256, J, n,
                     [](const JobArg& a) { return nblk(a.P * kFinalLanes, 256); });
  x.end(STAGE_BWD_FINAL);
  return rc ? -4 : 0;
}

template <int RES>
static int run_jobs_res(Exec& x, const JobArg* J, int n, int what) {
  if (n == 1) {
    if ((what & RUN_FORWARD) && seq_forward<RES, 1>(x, J, n)) return -4;
    if ((what & RUN_BACKWARD) && seq_backward<RES, 1>(x, J, n)) return -4;
    return 0;
  }
  if ((what & RUN_FORWARD) && seq_forward<RES, kMaxJobs>(x, J, n)) return -4;
  if ((what & RUN_BACKWARD) && seq_backward<RES, kMaxJobs>(x, J, n)) return -4;
  return 0;
}

template <int RES>
static int debug_spectral_res(Exec& x, const JobArg& job) {
  using G = Grid<RES>;
  auto c = [](int v) { return [v](const JobArg&) { return v; }; };
  int rc = 0;
  if constexpr (use_plane(RES)) {
    rc |= launch<1>(x, k_plane_fwd<RES, PF_LOADV, 1>, Plane<RES>::BLOCK, &job, 1, c(RES * Plane<RES>::KP * 3));
  } else {
    rc |= launch<1>(x, k_splat_r2c<RES, MODE_LOADV, 1>, G::BR, &job, 1, c(3 * G::rows));
    rc |= launch<1>(x, k_axis1_fwd<RES, true, false, 1>, G::BC, &job, 1, c(2 * G::cols));
  }
  rc |= launch<1>(x, k_fwd_axis0<RES, false, 1>, G::BJ, &job, 1, c(G::j0s));
  if constexpr (use_plane_p45(RES)) {
    rc |= launch<1>(x, k_plane_inv<RES, PI_DBG, 1>, Plane<RES>::BLOCK, &job, 1, c(RES * Plane<RES>::KP));
  } else {
    rc |= launch<1>(x, k_axis1_inv<RES, false, 1>, G::BC, &job, 1, c(G::cols));
    rc |= launch<1>(x, k_c2r_gather<RES, MODE_DBG, 1>, G::BR, &job, 1, c(G::rows));
  }
  return rc ? -4 : 0;
}

template <int RES>
static int debug_splat_res(Exec& x, const JobArg& job) {
  using G = Grid<RES>;
  auto c = [](int v) { return [v](const JobArg&) { return v; }; };
  int rc = 0;
  rc |= launch<1>(x, k_init<RES, 1>, 256, &job, 1, c(G::init_blocks));
  rc |= launch<1>(x, k_bin<RES, 1>, 256, &job, 1, [](const JobArg& a) { return nblk(a.P, kBinChunk); });
  if constexpr (num_bins(RES) <= kLdsBins) {
    rc |= launch<1>(x, k_scan_scatter<RES, 1>, 256, &job, 1, [](const JobArg& a) { return nblk(a.P, 256); });
  } else {
    rc |= launch<1>(x, k_scan<RES, 1>, 1024, &job, 1, c(1));
    rc |= launch<1>(x, k_scatter<RES, 1>, 256, &job, 1, [](const JobArg& a) { return nblk(a.P, 256); });
  }
  // the splat of the production path: plane passes at 64 and 128, row passes elsewhere
  if constexpr (use_plane(RES))
    rc |= launch<1>(x, k_plane_splat_dbg<RES, 1>, Plane<RES>::BLOCK, &job, 1, c(3 * RES));
  else
    rc |= launch<1>(x, k_splat_r2c<RES, MODE_VOUT, 1>, G::BR, &job, 1, c(3 * G::rows));
  return rc ? -4 : 0;
}

#define PSR_DISPATCH(res, call)     \
  switch (res) {                    \
    case 8: return call(8);         \
    case 16: return call(16);       \
    case 32: return call(32);       \
    case 64: return call(64);       \
    case 128: return call(128);     \
    case 256: return call(256);     \
    case 512: return call(512);     \
    default: return -1;             \
  }

int run_jobs(Exec& x, int res, const JobArg* jobs, int n, int what) {
#define CALL(R) run_jobs_res<R>(x, jobs, n, what)
  PSR_DISPATCH(res, CALL)
#undef CALL
}

int run_debug_spectral(Exec& x, int res, const JobArg& job) {
#define CALL(R) debug_spectral_res<R>(x, job)
  PSR_DISPATCH(res, CALL)
#undef CALL
}

int run_debug_splat(Exec& x, int res, const JobArg& job) {
#define CALL(R) debug_splat_res<R>(x, job)
  PSR_DISPATCH(res, CALL)
#undef CALL
}

}  // namespace psr
