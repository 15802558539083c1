// Slab-decomposed forward solve (main Sec. 3.1, Eqs. 2-4; supplement Sec. A)
// for grids of 16^3 to 1024^3, the large-scene form of the solver (main
// Sec. 5 names the cubic memory of the dense grid as the limit and sliding
// windows as the way round it; here the solve stays global and exact, the
// grid is split into slabs that each pass handles at its own size).
//
// Slab g owns planes [g s, (g+1) s) of j0 (s = r/G). Per slab:
//   S1  splat normals into LDS rows (64-bit fixed point, the row splat of
//       the single-grid solver) + r2c FFT along j2      -> A_g[c][j0][k2 tile][j1]
//   S2  FFT along j1; channels 1, 2 merged into W = kappa_1 v~_1 + kappa_2 v~_2;
//       each k1 range goes to its pencil owner         -> X blocks (h, g)
// Per pencil owner h (k1 in [h q, (h+1) q)):
//   S3  FFT along j0 of v~_0 and W, spectral operator of main Eq. 3, inverse
//       FFT along k0; each j0 range back to its slab   -> Z blocks (g, h)
// Per slab:
//   S4  inverse FFT along k1                           -> Y_g[j0][k2 tile][j1]
//   S5  c2r FFT along k2: chi' rows; the slab's first plane also goes to the
//       previous slab's halo
//   gather: chi' at the points whose floor plane lies in the slab (the top
//       corners of the last floor plane read the halo), FP64, by input index
// Then the FP64 mean over all points (one partial per block, fixed order),
// c and the scale of main Eq. 4, and chi = s (chi' - mu) per slab.
//
// The FFT lines of every pass are the same as in a single-grid solve and the
// splat sums integers, so chi' does not depend on the number of slabs, bit
// for bit.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fft_device.h"
#include "psr_device.h"
#include "psr_internal.h"
#include "psr_slab.h"

namespace psr {
namespace {

constexpr int kScanBlock = 1024;

// Ranges of sorted points whose corners reach rows [a0, a0 + TR) of plane j0:
// points sorted by bin b0 * RES + b1, floor planes j0 - 1 and j0, floor rows
// a0 - 1 (its +1 corner reaches row a0; wraps round at a0 = 0) to a0 + TR - 1.
template <int RES, int TR>
__device__ __forceinline__ Ranges slab_ranges(const int* __restrict__ off, int j0, int a0) {
  Ranges R;
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    const int base = ((j0 - 1 + o) & (RES - 1)) * RES;
    int a, b, c = 0, d = 0;
    if constexpr (TR == RES) {
      a = off[base];
      b = off[base + RES];
    } else {
      if (a0 > 0) {
        a = off[base + a0 - 1];
        b = off[base + a0 + TR];
      } else {
        a = off[base + RES - 1];
        b = off[base + RES];
        c = off[base];
        d = off[base + TR];
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

// Load a column tile of TC lines into LDS: element n of lines l, l + 1 (l
// even) from one 16-byte load at addr(n) + l; lines at or past nvalid read as
// zero. Ends with a barrier.
template <int RES, int TC, typename Addr>
__device__ __forceinline__ void load_cols(cf* rows, Addr addr, int nvalid) {
  constexpr int BC = TC * plan_TPL(RES), LS = lstride(RES), NV = RES * (TC / 2), IT = (NV + BC - 1) / BC;
  float4 buf[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * BC;
    buf[it] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (e < NV) {
      const int l2 = 2 * (e % (TC / 2)), n = e / (TC / 2);
      if (l2 < nvalid) {
        buf[it] = *reinterpret_cast<const float4*>(addr(n) + l2);
        if (l2 + 1 >= nvalid) buf[it].z = buf[it].w = 0.0f;
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

// Store the canonical registers of a column tile: element n of lines l, l + 1
// with one 16-byte store at addr(n) + l; line pairs entirely at or past nvalid
// are not stored (the padding slot of a pair is written, it is never read as
// data). The LDS lines must be free (the transform's last stage ended with a
// barrier).
template <int RES, int TC, typename Addr>
__device__ __forceinline__ void store_cols(cf* rows, const cf* reg, int l, int lt, Addr addr, int nvalid) {
  constexpr int BC = TC * plan_TPL(RES), TPL = plan_TPL(RES), E = plan_E(RES), LS = lstride(RES);
#pragma unroll
  for (int v = 0; v < E; ++v) rows[l * LS + pidx(lt + TPL * v)] = reg[v];
  __syncthreads();
  for (int e = threadIdx.x; e < RES * (TC / 2); e += BC) {
    const int l2 = 2 * (e % (TC / 2)), n = e / (TC / 2);
    if (l2 >= nvalid) continue;
    const cf x0 = rows[l2 * LS + pidx(n)], x1 = rows[(l2 + 1) * LS + pidx(n)];
    *reinterpret_cast<float4*>(addr(n) + l2) = make_float4(x0.x, x0.y, x1.x, x1.y);
  }
}

__device__ __forceinline__ int ilog2(int x) { return 31 - __clz(x); }

// ---------------------------------------------------------------------------
// binning: counting sort of the points by (floor plane b0, floor row b1)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_slab_init(SlabArgs a, int nbins, int res) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nbins; i += gridDim.x * 256) a.counts[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    SlabHeader* h = a.hdr;
    h->status = 0;
    h->flags = 0;
    h->res = res;
    h->slabs = a.G;
    h->npoints = a.P;
    h->sigma = a.sigma;
    h->m = a.m;
    h->reading = a.reading;
    h->pad = 0;
    h->chi0 = 0.0;
  }
}

template <int RES>
__global__ __launch_bounds__(256) void k_slab_bin(SlabArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.P) return;
  float f[3], n[3];
  int b[3];
  bool bad = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float x = a.pts[3 * i + d];
    n[d] = a.nrm[3 * i + d];
    if (!isfinite(x)) {
      bad = true;
      x = 0.0f;
    }
    if (!isfinite(n[d])) bad = true;
    float u = x - floorf(x);  // periodic domain
    if (u >= 1.0f) u = 0.0f;
    const float tt = u * (float)RES;  // exact: RES is a power of two
    int bi = (int)floorf(tt);
    bi = bi < 0 ? 0 : (bi > RES - 1 ? RES - 1 : bi);
    b[d] = bi;
    f[d] = tt - (float)bi;
  }
  if (bad) {
    f[0] = f[1] = f[2] = 0.0f;
    n[0] = n[1] = n[2] = 0.0f;
    atomicOr(&a.hdr->flags, 1);
  }
  const int bin = b[0] * RES + b[1];
  const int rank = atomicAdd(&a.counts[bin], 1);
  PointRec r;
  r.f0 = f[0];
  r.f1 = f[1];
  r.f2 = f[2];
  r.b = (uint32_t)b[0] | ((uint32_t)b[1] << 10) | ((uint32_t)b[2] << 20);
  r.n0 = n[0];
  r.n1 = n[1];
  r.n2 = n[2];
  r.idx = (uint32_t)i;
  a.tmp[i] = r;
  a.colrank[i] = make_int2(bin, rank);
}

// Inclusive scan of v over a workgroup of kScanBlock threads; *total = the sum.
__device__ __forceinline__ int block_incl_scan(int v, int* total) {
  __shared__ int wsum[kScanBlock / 64];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(v, d, 64);
    if (lane >= d) v += y;
  }
  if (lane == 63) wsum[wid] = v;
  __syncthreads();
  if (wid == 0) {
    int w = lane < kScanBlock / 64 ? wsum[lane] : 0;
#pragma unroll
    for (int d = 1; d < kScanBlock / 64; d <<= 1) {
      const int y = __shfl_up(w, d, 64);
      if (lane >= d) w += y;
    }
    if (lane < kScanBlock / 64) wsum[lane] = w;
  }
  __syncthreads();
  *total = wsum[kScanBlock / 64 - 1];
  return v + (wid ? wsum[wid - 1] : 0);
}

// Exclusive scan of the bin counts: per block of kScanBlock bins, then of the
// block sums (at most kScanBlock of them: r^2 <= 2^20), then the block offsets.
__global__ __launch_bounds__(kScanBlock) void k_slab_scan_blocks(SlabArgs a, int n) {
  const int i = blockIdx.x * kScanBlock + threadIdx.x;
  const int c = i < n ? a.counts[i] : 0;
  int tot;
  const int v = block_incl_scan(c, &tot);
  if (i < n) a.off[i] = v - c;
  if (threadIdx.x == 0) a.bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_slab_scan_tops(SlabArgs a, int nb, int n) {
  const int t = threadIdx.x;
  const int c = t < nb ? a.bsum[t] : 0;
  int tot;
  const int v = block_incl_scan(c, &tot);
  if (t < nb) a.bsum[t] = v - c;
  if (t == 0) a.off[n] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_slab_scan_add(SlabArgs a, int n) {
  const int i = blockIdx.x * kScanBlock + threadIdx.x;
  if (i < n) a.off[i] += a.bsum[blockIdx.x];
}

__global__ __launch_bounds__(256) void k_slab_scatter(SlabArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.P) return;
  const int2 cr = a.colrank[i];
  a.sorted[a.off[cr.x] + cr.y] = a.tmp[i];
}

// ---------------------------------------------------------------------------
// S1: rows of one plane of slab g (one channel) -> LDS splat (or the test
// field) -> r2c FFT along j2 -> A_g[c][j0 - g s], k2-tiled rows of r/2 + 1.
// ---------------------------------------------------------------------------
template <int RES, bool LOAD>
__global__ __launch_bounds__(slab_rows_block(RES)) void k_slab_rows_fwd(const SlabArgs a, int g) {
  constexpr int M = RES / 2, H = M + 1, HP = slab_hp(RES), TR = slab_rows(RES), NT = RES / TR;
  constexpr int BR = slab_rows_block(RES), TPL = plan_TPL(M), E = plan_E(M), LS = row_ls(M);
  __shared__ __align__(16) cf rows[TR * LS];
  __shared__ cf stw[M];      // FFT table of length M
  __shared__ cf rtw[M + 1];  // W_RES^k, k in [0, M], for the r2c post-processing
  const int s = RES / a.G;
  const int T = blockIdx.x % (s * NT), c = blockIdx.x / (s * NT);
  const int j0l = T / NT, a0 = (T % NT) * TR, j0 = g * s + j0l;
  constexpr int TC = slab_cols(RES);
  // k2-tiled plane: element (j1, k2) at ((k2 / TC) RES + j1) TC + k2 % TC; the
  // loops below run tile by tile, so each tile's TR rows are one contiguous run
  cf* const out = a.A + ((int64_t)(3 * g + c) * s + j0l) * RES * HP + (int64_t)a0 * TC;
  const int t = threadIdx.x;
  Ranges R{};
  if constexpr (!LOAD) {
    R = slab_ranges<RES, TR>(a.off, j0, a0);
    if (R.total == 0) {  // no point reaches these rows: their spectra are zero
      for (int e = t; e < TR * HP; e += BR) {
        const int kk = e % TC, l = (e / TC) % TR, kt = e / (TC * TR);
        if (kt * TC + kk < H) out[((int64_t)kt * RES + l) * TC + kk] = cf{0.0f, 0.0f};
      }
      return;
    }
  }
  stage_table<BR>(stw, a.tw + M, M);
  stage_table<BR>(rtw, a.tw + RES, M + 1);
  fill_rows<RES, TR, BR, LOAD ? 2 : 0>(rows, a.sorted, R, a.field, make_float3(1.0f, 0.0f, 1.0f), j0, a0, c);
  {
    cf reg[E];
    const int l = t / TPL;
    fft<M, -1, false, false>(reg, rows + l * LS, t % TPL, stw, row_swz(M, l));
  }
  // X[k] = E_k + W_r^k O_k with E = (Z_k + Z*_{M-k})/2, O = (Z_k - Z*_{M-k})/(2i)
  for (int e = t; e < TR * HP; e += BR) {
    const int kk = e % TC, l = (e / TC) % TR, kt = e / (TC * TR), k = kt * TC + kk;
    if (k >= H) continue;
    const cf zk = rows[rpos<M>(l, k == M ? 0 : k)];
    const cf zm = rows[rpos<M>(l, k == 0 ? 0 : M - k)];
    const cf Ee{0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y)};
    const cf Oo{0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x)};
    out[((int64_t)kt * RES + l) * TC + kk] = cadd(Ee, cmul(rtw[k], Oo));
  }
}

// ---------------------------------------------------------------------------
// S2: FFT along j1 of slab g. Output channel 0 = v~_0, channel 1 =
// W = kappa_1(k1) v~_1 + kappa_2(k2) v~_2 (all the j0 pass needs of channels
// 1 and 2); element k1 goes to block (k1 / q, g): [2][s][nt][q][tc].
// ---------------------------------------------------------------------------
template <int RES>
__global__ __launch_bounds__(slab_cols_block(RES)) void k_slab_fft_j1(const SlabArgs a, const BlockPtrs dst, int g) {
  constexpr int H = RES / 2 + 1, HP = slab_hp(RES), TC = slab_cols(RES), NKT = HP / TC;
  constexpr int TPL = plan_TPL(RES), E = plan_E(RES), LS = lstride(RES), BC = slab_cols_block(RES);
  __shared__ cf rows[TC * LS];
  __shared__ cf stw[RES];
  __shared__ cf* dp[kMaxSlabs];
  stage_table<BC>(stw, a.tw + RES, RES);
  for (int e = threadIdx.x; e < a.G; e += BC) dp[e] = dst.p[e];
  const int s = RES / a.G, q = s, lq = ilog2(q);
  int b = blockIdx.x;
  const int kt = b % NKT;
  b /= NKT;
  const int j0l = b % s;
  const int oc = 1 - b / s;  // the heavier channel-1 workgroups first
  const int k2a = kt * TC, nvalid = H - k2a;
  const int l = threadIdx.x / TPL, lt = threadIdx.x % TPL;
  const int64_t CH = (int64_t)s * RES * HP;
  // the tile of channel 0 (k2-tiled planes: one contiguous RES x TC block)
  const cf* src = a.A + ((int64_t)3 * g * s + j0l) * RES * HP + (int64_t)kt * RES * TC;
  cf reg[E];
  if (oc == 0) {
    load_cols<RES, TC>(rows, [&](int n) { return src + (int64_t)n * TC; }, nvalid);
    fft<RES, -1, false, true>(reg, rows + l * LS, lt, stw);
  } else {
    cf acc[E];
    load_cols<RES, TC>(rows, [&](int n) { return src + 2 * CH + (int64_t)n * TC; }, nvalid);
    fft<RES, -1, false, true>(reg, rows + l * LS, lt, stw);
    const float k2f = kappa_odd(k2a + l, RES);
#pragma unroll
    for (int v = 0; v < E; ++v) acc[v] = cscale(reg[v], k2f);
    load_cols<RES, TC>(rows, [&](int n) { return src + CH + (int64_t)n * TC; }, nvalid);
    fft<RES, -1, false, true>(reg, rows + l * LS, lt, stw);
#pragma unroll
    for (int v = 0; v < E; ++v) {
      const float k1f = kappa_odd(lt + TPL * v, RES);
      reg[v] = cf{acc[v].x + k1f * reg[v].x, acc[v].y + k1f * reg[v].y};
    }
  }
  store_cols<RES, TC>(
      rows, reg, l, lt,
      [&](int n) { return dp[n >> lq] + (((int64_t)(oc * s + j0l) * NKT + kt) * q + (n & (q - 1))) * TC; },
      nvalid);
}

// ---------------------------------------------------------------------------
// S3: pencil owner h, line (k1, k2) over all j0: FFT along j0 of v~_0 and W,
// chi~ = i F(k) (kappa_0(k0) v~_0 + W) (main Eq. 3, the inverse's 1/N folded
// into F), inverse FFT along k0; element j0 goes to block (j0 / s, h):
// [s][nt][q][tc].
// ---------------------------------------------------------------------------
template <int RES>
__global__ __launch_bounds__(slab_cols_block(RES)) void k_slab_pencil_j0(const SlabArgs a, const BlockPtrs src,
                                                                         const BlockPtrs dst, int h) {
  constexpr int M = RES / 2, H = M + 1, HP = slab_hp(RES), TC = slab_cols(RES), NKT = HP / TC;
  constexpr int TPL = plan_TPL(RES), E = plan_E(RES), LS = lstride(RES), BC = slab_cols_block(RES);
  __shared__ cf rows[TC * LS];
  __shared__ cf stw[RES];
  __shared__ float g1[RES];
  __shared__ cf* sp[kMaxSlabs];
  __shared__ cf* dp[kMaxSlabs];
  stage_table<BC>(stw, a.tw + RES, RES);
  gauss_table<RES, BC>(g1, a.sigma);
  for (int e = threadIdx.x; e < a.G; e += BC) {
    sp[e] = src.p[e];
    dp[e] = dst.p[e];
  }
  __syncthreads();  // the block tables are read by the first loads
  const int s = RES / a.G, q = s, ls = ilog2(s);
  const int kt = blockIdx.x % NKT, k1l = blockIdx.x / NKT;
  const int k2a = kt * TC, nvalid = H - k2a;
  const int k1 = h * q + k1l;
  const int l = threadIdx.x / TPL, lt = threadIdx.x % TPL;
  cf acc[E], reg[E];
  load_cols<RES, TC>(
      rows, [&](int n) { return sp[n >> ls] + (((int64_t)(n & (s - 1)) * NKT + kt) * q + k1l) * TC; }, nvalid);
  fft<RES, -1, false, true>(reg, rows + l * LS, lt, stw);
#pragma unroll
  for (int v = 0; v < E; ++v) acc[v] = cscale(reg[v], kappa_odd(lt + TPL * v, RES));
  load_cols<RES, TC>(
      rows, [&](int n) { return sp[n >> ls] + (((int64_t)(s + (n & (s - 1))) * NKT + kt) * q + k1l) * TC; },
      nvalid);
  fft<RES, -1, false, true>(reg, rows + l * LS, lt, stw);
  {
    const int k2 = imin(k2a + l, M);  // padding lines are zero; any finite factor will do
    const float g12 = g1[k1] * g1[k2];
    const float q12 = kappa_of(k1, RES) * kappa_of(k1, RES) + kappa_of(k2, RES) * kappa_of(k2, RES);
#pragma unroll
    for (int v = 0; v < E; ++v) {
      const float F = spectral_F<RES>(g1, lt + TPL * v, g12, q12);
      const cf x{acc[v].x + reg[v].x, acc[v].y + reg[v].y};
      reg[v] = cf{-F * x.y, F * x.x};  // i F sum
    }
  }
  fft<RES, +1, true, true>(reg, rows + l * LS, lt, stw);
  store_cols<RES, TC>(
      rows, reg, l, lt, [&](int n) { return dp[n >> ls] + (((int64_t)(n & (s - 1)) * NKT + kt) * q + k1l) * TC; },
      nvalid);
}

// ---------------------------------------------------------------------------
// S4: inverse FFT along k1 of slab g, from blocks (g, h) -> Y_g[j0], k2-tiled.
// ---------------------------------------------------------------------------
template <int RES>
__global__ __launch_bounds__(slab_cols_block(RES)) void k_slab_ifft_k1(const SlabArgs a, const BlockPtrs src, int g) {
  constexpr int H = RES / 2 + 1, HP = slab_hp(RES), TC = slab_cols(RES), NKT = HP / TC;
  constexpr int TPL = plan_TPL(RES), E = plan_E(RES), LS = lstride(RES), BC = slab_cols_block(RES);
  __shared__ cf rows[TC * LS];
  __shared__ cf stw[RES];
  __shared__ cf* sp[kMaxSlabs];
  stage_table<BC>(stw, a.tw + RES, RES);
  for (int e = threadIdx.x; e < a.G; e += BC) sp[e] = src.p[e];
  __syncthreads();
  const int s = RES / a.G, q = s, lq = ilog2(q);
  const int kt = blockIdx.x % NKT, j0l = blockIdx.x / NKT;
  const int k2a = kt * TC, nvalid = H - k2a;
  const int l = threadIdx.x / TPL, lt = threadIdx.x % TPL;
  cf reg[E];
  load_cols<RES, TC>(
      rows, [&](int n) { return sp[n >> lq] + (((int64_t)j0l * NKT + kt) * q + (n & (q - 1))) * TC; }, nvalid);
  fft<RES, +1, false, true>(reg, rows + l * LS, lt, stw);
  cf* const y = a.A + (int64_t)(g * s + j0l) * RES * HP + (int64_t)kt * RES * TC;
  store_cols<RES, TC>(rows, reg, l, lt, [&](int n) { return y + (int64_t)n * TC; }, nvalid);
}

// ---------------------------------------------------------------------------
// S5: rows of one plane of slab g: c2r FFT along k2 -> chi' rows; the slab's
// first plane is also the previous slab's halo; chi'(0,0,0) for main Eq. 4.
// ---------------------------------------------------------------------------
template <int RES>
__global__ __launch_bounds__(slab_rows_block(RES)) void k_slab_rows_inv(const SlabArgs a, int g) {
  constexpr int M = RES / 2, H = M + 1, HP = slab_hp(RES), TR = slab_rows(RES), NT = RES / TR;
  constexpr int BR = slab_rows_block(RES), TPL = plan_TPL(M), E = plan_E(M), LS = row_ls(M);
  __shared__ __align__(16) cf rows[TR * LS];
  __shared__ cf stw[M];
  __shared__ cf rtw[M + 1];
  const int s = RES / a.G;
  const int j0l = blockIdx.x / NT, a0 = (blockIdx.x % NT) * TR, j0 = g * s + j0l;
  const int t = threadIdx.x;
  stage_table<BR>(stw, a.tw + M, M);
  stage_table<BR>(rtw, a.tw + RES, M + 1);
  constexpr int TC = slab_cols(RES);
  const cf* in = a.A + (int64_t)(g * s + j0l) * RES * HP + (int64_t)a0 * TC;  // k2-tiled plane
  for (int e = t; e < TR * HP; e += BR) {
    const int kk = e % TC, l = (e / TC) % TR, kt = e / (TC * TR), k = kt * TC + kk;
    if (k < H) rows[rpos<M>(l, k)] = in[((int64_t)kt * RES + l) * TC + kk];
  }
  __syncthreads();
  // Hermitian half-spectrum X[0..M] -> packed spectrum Z[0..M) of the
  // even/odd samples: Z = (X_k + X*_{M-k}) + i (X_k - X*_{M-k}) e^{+2 pi i k/r};
  // the pairs (k, M - k) of k in [0, M/2] are formed by one thread each
  {
    constexpr int NH = M / 2;
    for (int e = t; e < TR * (NH + 1); e += BR) {
      const int row = e / (NH + 1), k = e % (NH + 1);
      const int ik = rpos<M>(row, k), im = rpos<M>(row, M - k);
      const cf xk = rows[ik], xm = rows[im];
      {
        const cf Ee{xk.x + xm.x, xk.y - xm.y};
        const cf Dd{xk.x - xm.x, xk.y + xm.y};
        const cf Oo = cmul(Dd, cf{rtw[k].x, -rtw[k].y});
        rows[ik] = cf{Ee.x - Oo.y, Ee.y + Oo.x};
      }
      if (k != 0 && 2 * k != M) {
        const cf Ee{xm.x + xk.x, xm.y - xk.y};
        const cf Dd{xm.x - xk.x, xm.y + xk.y};
        const cf Oo = cmul(Dd, cf{rtw[M - k].x, -rtw[M - k].y});
        rows[im] = cf{Ee.x - Oo.y, Ee.y + Oo.x};
      }
    }
  }
  __syncthreads();
  {
    cf reg[E];
    const int l = t / TPL;
    fft<M, +1, false, false>(reg, rows + l * LS, t % TPL, stw, row_swz(M, l));
  }
  float* const dst = a.chi + ((int64_t)j0 * RES + a0) * RES;
  float* const hal = j0l == 0 ? a.halo + (int64_t)((g + a.G - 1) & (a.G - 1)) * RES * RES + (int64_t)a0 * RES
                              : nullptr;
  for (int e = t; e < TR * M; e += BR) {
    const int l = e / M, mm = e % M;
    const cf z = rows[rpos<M>(l, mm)];
    const float2 v = make_float2(z.x, z.y);
    *reinterpret_cast<float2*>(dst + (int64_t)l * RES + 2 * mm) = v;
    if (hal) *reinterpret_cast<float2*>(hal + (int64_t)l * RES + 2 * mm) = v;
    if (j0 == 0 && a0 == 0 && e == 0) a.hdr->chi0 = (double)z.x;
  }
}

// ---------------------------------------------------------------------------
// Gather of chi' at the points of slab g (floor plane in the slab), FP64
// trilinear weights, written by input index.
// ---------------------------------------------------------------------------
template <int RES>
__global__ __launch_bounds__(256) void k_slab_gather(const SlabArgs a, int g) {
  const int s = RES / a.G;
  const int lo = a.off[g * s * RES], hi = a.off[(g + 1) * s * RES];
  const int pend = (g + 1) * s;
  const float* const halo = a.halo + (int64_t)g * RES * RES;
  for (int64_t i = lo + (int64_t)blockIdx.x * 256 + threadIdx.x; i < hi; i += (int64_t)gridDim.x * 256) {
    float4 p0, p1;
    load_rec(a.sorted, i, p0, p1);
    const uint32_t bb = __float_as_uint(p0.w);
    const int b0 = bb & 1023, b1 = (bb >> 10) & 1023, b2 = bb >> 20;
    const double f0 = p0.x, f1 = p0.y, f2 = p0.z;
    double acc = 0.0;
#pragma unroll
    for (int o0 = 0; o0 < 2; ++o0) {
      const int p = b0 + o0;
      const float* pl = p == pend ? halo : a.chi + (int64_t)p * RES * RES;
      const double w0 = o0 ? f0 : 1.0 - f0;
#pragma unroll
      for (int o1 = 0; o1 < 2; ++o1) {
        const float* row = pl + (int64_t)((b1 + o1) & (RES - 1)) * RES;
        const double w01 = w0 * (o1 ? f1 : 1.0 - f1);
        const double v0 = row[b2], v1 = row[(b2 + 1) & (RES - 1)];
        acc += w01 * ((1.0 - f2) * v0 + f2 * v1);
      }
    }
    a.val[__float_as_uint(p1.w)] = acc;
  }
}

// FP64 sum of chi' at the points in input order: one partial per block.
__global__ __launch_bounds__(256) void k_slab_reduce(const SlabArgs a) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.P; i += (int64_t)gridDim.x * 256) acc += a.val[i];
  const double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) a.red[blockIdx.x] = tot;
}

// mu, c and s of main Eq. 4 from the partials (every block sums them in the
// same order), then chi = s (chi' - mu) over the planes of slab g. Block 0 of
// slab 0 records the scalars and the status.
__global__ __launch_bounds__(256) void k_slab_normalize(const SlabArgs a, int g, int nred, int64_t n4) {
  __shared__ double sh[256];
  double x = 0.0;
  for (int i = threadIdx.x; i < nred; i += 256) x += a.red[i];
  const double tot = block_sum(x, sh);
  const SlabHeader* hd = a.hdr;
  const double mu = tot / (double)a.P, chi0 = hd->chi0;
  const double c = a.reading == 0 ? chi0 - mu : chi0;
  int status = 0;
  if (hd->flags & 1) status = -6;  // PSR_ENONFINITE
  else if (!(c != 0.0) || !isfinite(c) || !isfinite(mu)) status = -3;  // PSR_EDEGENERATE
  const double sc = status ? __longlong_as_double(0x7ff8000000000000LL) : (double)a.m / fabs(c);
  if (g == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    a.hdr->status = status;
    if (a.result) {
      a.result->mu = mu;
      a.result->cscale = c;
      a.result->scale = sc;
      a.result->chi0 = chi0;
      a.result->status = status;
      a.result->flags = hd->flags;
    }
  }
  float4* c4 = reinterpret_cast<float4*>(a.chi) + (int64_t)g * n4;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256) {
    float4 v = c4[i];
    v.x = (float)(((double)v.x - mu) * sc);
    v.y = (float)(((double)v.y - mu) * sc);
    v.z = (float)(((double)v.z - mu) * sc);
    v.w = (float)(((double)v.w - mu) * sc);
    c4[i] = v;
  }
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <int RES>
int slab_sequence(Exec& x, const SlabArgs& a) {
  constexpr int HP = slab_hp(RES), TR = slab_rows(RES), NT = RES / TR, NKT = HP / slab_cols(RES);
  constexpr int BR = slab_rows_block(RES), BC = slab_cols_block(RES);
  const bool load = a.field != nullptr;
  const int G = a.G, s = RES / G, q = s;
  const int64_t blkX = (int64_t)2 * s * q * HP, blkZ = (int64_t)s * q * HP;
  const hipStream_t st = x.stream;
  const int nbins = RES * RES;

  x.begin(STAGE_SLAB_BIN);
  hipLaunchKernelGGL(k_slab_init, dim3((unsigned)imin(1024, (int)cdiv(nbins, 256))), dim3(256), 0, st, a, nbins,
                     RES);
  if (!load) {
    const unsigned pb = (unsigned)cdiv(a.P, 256);
    const int nsb = (int)cdiv(nbins, kScanBlock);
    hipLaunchKernelGGL(k_slab_bin<RES>, dim3(pb), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_slab_scan_blocks, dim3(nsb), dim3(kScanBlock), 0, st, a, nbins);
    hipLaunchKernelGGL(k_slab_scan_tops, dim3(1), dim3(kScanBlock), 0, st, a, nsb, nbins);
    hipLaunchKernelGGL(k_slab_scan_add, dim3(nsb), dim3(kScanBlock), 0, st, a, nbins);
    hipLaunchKernelGGL(k_slab_scatter, dim3(pb), dim3(256), 0, st, a);
  }
  x.end(STAGE_SLAB_BIN);

  x.begin(STAGE_S1);
  for (int g = 0; g < G; ++g) {
    if (load) hipLaunchKernelGGL((k_slab_rows_fwd<RES, true>), dim3(3 * s * NT), dim3(BR), 0, st, a, g);
    else hipLaunchKernelGGL((k_slab_rows_fwd<RES, false>), dim3(3 * s * NT), dim3(BR), 0, st, a, g);
  }
  x.end(STAGE_S1);

  x.begin(STAGE_S2);
  for (int g = 0; g < G; ++g) {
    BlockPtrs d{};
    for (int h = 0; h < G; ++h) d.p[h] = a.X + (int64_t)(h * G + g) * blkX;
    hipLaunchKernelGGL(k_slab_fft_j1<RES>, dim3(2 * s * NKT), dim3(BC), 0, st, a, d, g);
  }
  x.end(STAGE_S2);

  x.begin(STAGE_S3);
  for (int h = 0; h < G; ++h) {
    BlockPtrs sp{}, dp{};
    for (int g = 0; g < G; ++g) {
      sp.p[g] = a.X + (int64_t)(h * G + g) * blkX;
      dp.p[g] = a.Z + (int64_t)(g * G + h) * blkZ;
    }
    hipLaunchKernelGGL(k_slab_pencil_j0<RES>, dim3(q * NKT), dim3(BC), 0, st, a, sp, dp, h);
  }
  x.end(STAGE_S3);

  x.begin(STAGE_S4);
  for (int g = 0; g < G; ++g) {
    BlockPtrs sp{};
    for (int h = 0; h < G; ++h) sp.p[h] = a.Z + (int64_t)(g * G + h) * blkZ;
    hipLaunchKernelGGL(k_slab_ifft_k1<RES>, dim3(s * NKT), dim3(BC), 0, st, a, sp, g);
  }
  x.end(STAGE_S4);

  x.begin(STAGE_S5);
  for (int g = 0; g < G; ++g) hipLaunchKernelGGL(k_slab_rows_inv<RES>, dim3(s * NT), dim3(BR), 0, st, a, g);
  x.end(STAGE_S5);

  if (!load) {
    x.begin(STAGE_SLAB_GATHER);
    const int gb = (int)imin(1024, (int)cdiv(a.P, 256));
    for (int g = 0; g < G; ++g) hipLaunchKernelGGL(k_slab_gather<RES>, dim3(gb), dim3(256), 0, st, a, g);
    const int nred = (int)imin(kRedBlocks, (int)cdiv(a.P, 256));
    hipLaunchKernelGGL(k_slab_reduce, dim3(nred), dim3(256), 0, st, a);
    x.end(STAGE_SLAB_GATHER);
    x.begin(STAGE_SLAB_NORM);
    const int64_t n4 = (int64_t)s * RES * RES / 4;
    const int nb = (int)imin(1024, (int)cdiv(n4, 256));
    for (int g = 0; g < G; ++g) hipLaunchKernelGGL(k_slab_normalize, dim3(nb), dim3(256), 0, st, a, g, nred, n4);
    x.end(STAGE_SLAB_NORM);
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace

int run_slab(Exec& x, int res, const SlabArgs& a) {
  switch (res) {
    case 16: return slab_sequence<16>(x, a);
    case 32: return slab_sequence<32>(x, a);
    case 64: return slab_sequence<64>(x, a);
    case 128: return slab_sequence<128>(x, a);
    case 256: return slab_sequence<256>(x, a);
    case 512: return slab_sequence<512>(x, a);
    case 1024: return slab_sequence<1024>(x, a);
    default: return -1;
  }
}

}  // namespace psr
