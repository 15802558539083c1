// gfx950 kernels of the differentiable Poisson solver (Peng et al., NeurIPS 2021).
//
// Pipeline of one forward solve (main Sec. 3.1, Eqs. 2-4; supplement Sec. A):
//   bin      points -> column (b0, b1) buckets (count, scan, scatter)
//   P1       splat normals into LDS rows + real-to-complex FFT along j2
//            (supplement A.1 rasterisation fused with the first FFT axis)
//   P2       FFT along j1 (3 channels)
//   P3       FFT along j0, spectral operator of main Eq. 3 summed over the 3
//            channels, inverse FFT along j0 (one channel out)
//   P4       inverse FFT along j1
//   P5       complex-to-real inverse FFT along j2, write chi', and the
//            trilinear gather of chi' at the points (value + gradient)
//   reduce   FP64 mean at the points, scale c (main Eq. 4), normalise chi
// The backward runs the adjoint of every step (FP64 sums of G and G*chi, the
// cotangent H, conjugate operator, 3 inverse channels, gather of dL/dv).
//
// Layouts (complex64 unless noted; H = r/2 + 1 half-spectrum planes):
//   A[c][k2][j0][j1]   P1 out, P2 in
//   B[c][k1][k2][j0]   P2 out, P3 in
//   C[c][j0][k2][k1]   P3 out, P4 in
//   D[c][k2][j0][j1]   P4 out, P5 in
// Each pass reads whole contiguous lines or 16-line segments and writes the
// other, so every global access is at least a 128-byte run.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fft_device.h"
#include "psr_internal.h"

namespace psr {

__host__ __device__ constexpr int tile_lines(int res) { return res >= 512 ? 8 : (res >= 16 ? 16 : res); }

__device__ __forceinline__ float kappa_of(int k, int res) { return (float)(k < res / 2 ? k : k - res); }
// odd (first-derivative) factor: zero at the Nyquist index
__device__ __forceinline__ float kappa_odd(int k, int res) { return k == res / 2 ? 0.0f : kappa_of(k, res); }

__device__ __forceinline__ void load_rec(const PointRec* __restrict__ s, int64_t i, float4& a, float4& b) {
  const float4* p = reinterpret_cast<const float4*>(s + i);
  a = p[0];
  b = p[1];
}

// Point ranges (in sorted order) whose 2x2 corner lines can touch the tile of
// lines (j0, j1 in [a0, a0+T)): floor columns b0 in {j0-1, j0},
// b1 in [a0-1, a0+T-1] (mod res). Up to 4 disjoint ranges.
template <int RES, int T>
__device__ __forceinline__ int tile_ranges(const int* __restrict__ off, int j0, int a0, int* lo, int* hi) {
  int nr = 0;
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    const int b0 = (j0 - 1 + o) & (RES - 1);
    const int rb = b0 * RES;
    if constexpr (T == RES) {
      lo[nr] = off[rb];
      hi[nr] = off[rb + RES];
      ++nr;
    } else {
      if (a0 > 0) {
        lo[nr] = off[rb + a0 - 1];
        hi[nr] = off[rb + a0 + T];
        ++nr;
      } else {
        lo[nr] = off[rb + RES - 1];
        hi[nr] = off[rb + RES];
        ++nr;
        lo[nr] = off[rb];
        hi[nr] = off[rb + T];
        ++nr;
      }
    }
  }
  return nr;
}

__device__ __forceinline__ int64_t range_pick(const int* lo, const int* hi, int nr, int q) {
  for (int r = 0; r < nr; ++r) {
    const int n = hi[r] - lo[r];
    if (q < n) return lo[r] + q;
    q -= n;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// binning (counting sort of the points by floor column (b0, b1))
// ---------------------------------------------------------------------------
__global__ void k_init(int* __restrict__ counts, int n, SavedHeader* __restrict__ hdr, int res,
                       int64_t npoints, float sigma, float m, int reading) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) counts[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hdr->status = 0;
    hdr->flags = 0;
    hdr->res = res;
    hdr->reading = reading;
    hdr->npoints = npoints;
    hdr->sigma = sigma;
    hdr->m = m;
  }
}

template <int RES>
__global__ void k_bin(const float* __restrict__ pts, const float* __restrict__ nrm, int64_t npoints,
                      int* __restrict__ counts, PointRec* __restrict__ tmp, int2* __restrict__ colrank,
                      SavedHeader* __restrict__ hdr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npoints) return;
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
    float u = x - floorf(x);  // wrap into [0,1): periodic domain
    if (u >= 1.0f) u = 0.0f;
    const float t = u * (float)RES;  // exact: RES is a power of two
    int bi = (int)floorf(t);
    bi = bi < 0 ? 0 : (bi > RES - 1 ? RES - 1 : bi);
    b[a] = bi;
    f[a] = t - (float)bi;
  }
  if (bad) {
    f[0] = f[1] = f[2] = 0.0f;
    n[0] = n[1] = n[2] = 0.0f;
    atomicOr(&hdr->flags, 1);
  }
  const int col = b[0] * RES + b[1];
  const int rank = atomicAdd(&counts[col], 1);
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
  colrank[i] = make_int2(col, rank);
}

// Exclusive scan of n counts into off[0..n] with one workgroup of 1024.
__global__ __launch_bounds__(1024) void k_scan(const int* __restrict__ counts, int* __restrict__ off, int n) {
  __shared__ int sums[1024];
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int lo = t * chunk;
  const int hi = min(lo + chunk, n);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += counts[i];
  sums[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int v = t >= d ? sums[t - d] : 0;
    __syncthreads();
    sums[t] += v;
    __syncthreads();
  }
  int run = t == 0 ? 0 : sums[t - 1];
  for (int i = lo; i < hi; ++i) {
    off[i] = run;
    run += counts[i];
  }
  if (t == 1023) off[n] = sums[1023];
}

__global__ void k_scatter(const PointRec* __restrict__ tmp, const int2* __restrict__ colrank,
                          const int* __restrict__ off, PointRec* __restrict__ sorted, int64_t npoints) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npoints) return;
  const int2 cr = colrank[i];
  sorted[off[cr.x] + cr.y] = tmp[i];
}

// ---------------------------------------------------------------------------
// P1 / B1: rasterise into LDS rows, then r2c FFT along j2.
// MODE_SPLAT: v = splat of normals (3 channels)         [forward]
// MODE_BWDH : H = s G + alpha W - Q delta_0 (1 channel)   [backward]
// MODE_LOADV: v loaded from global (3 channels)         [spectral test hook]
// MODE_VOUT : splat only, rows written to global v       [splat test hook]
// ---------------------------------------------------------------------------
enum { MODE_SPLAT = 0, MODE_BWDH = 1, MODE_LOADV = 2, MODE_VOUT = 3 };

template <int RES, int MODE>
__global__ __launch_bounds__(kBlock) void k_splat_r2c(const PointRec* __restrict__ sorted,
                                                      const int* __restrict__ off,
                                                      const float* __restrict__ gin,
                                                      const BwdScalars* __restrict__ bs,
                                                      const cf* __restrict__ tw, cf* __restrict__ out,
                                                      float* __restrict__ vout) {
  constexpr int M = RES / 2, H = M + 1, T = tile_lines(RES);
  constexpr int C = MODE == MODE_BWDH ? 1 : 3;
  constexpr int LS = lstride(M);
  constexpr int64_t N3 = (int64_t)RES * RES * RES;
  __shared__ cf rows[C * T * LS];
  float* rf = reinterpret_cast<float*>(rows);
  const int tb = blockIdx.x % (RES / T);
  const int j0 = blockIdx.x / (RES / T);
  const int a0 = tb * T;

  if constexpr (MODE == MODE_SPLAT || MODE == MODE_VOUT) {
    for (int e = threadIdx.x; e < C * T * LS; e += kBlock) rows[e] = cf{0.0f, 0.0f};
  } else {
    float sg = 1.0f, q = 0.0f;
    if constexpr (MODE == MODE_BWDH) {
      sg = bs->s;
      q = bs->q;
    }
    for (int e = threadIdx.x; e < C * T * M; e += kBlock) {
      const int mm = e % M, l = (e / M) % T, c = e / (M * T);
      const int64_t gi = c * N3 + ((int64_t)j0 * RES + a0 + l) * RES + 2 * mm;
      const float2 v = *reinterpret_cast<const float2*>(gin + gi);
      cf z{v.x * sg, v.y * sg};
      if constexpr (MODE == MODE_BWDH) {
        if (j0 == 0 && a0 + l == 0 && mm == 0) z.x -= q;
      }
      rows[(c * T + l) * LS + pidx(mm)] = z;
    }
  }

  if constexpr (MODE != MODE_LOADV) {
    float alpha = 0.0f;
    if constexpr (MODE == MODE_BWDH) alpha = bs->alpha;
    __syncthreads();
    int lo[4], hi[4];
    const int nr = tile_ranges<RES, T>(off, j0, a0, lo, hi);
    int total = 0;
    for (int r = 0; r < nr; ++r) total += hi[r] - lo[r];
    for (int qd = threadIdx.x; qd < total; qd += kBlock) {
      const int64_t s = range_pick(lo, hi, nr, qd);
      float4 p0, p1;
      load_rec(sorted, s, p0, p1);
      const uint32_t bb = __float_as_uint(p0.w);
      const int b0 = bb & 1023, b1 = (bb >> 10) & 1023, b2 = bb >> 20;
      const float nv[3] = {p1.x, p1.y, p1.z};
#pragma unroll
      for (int o0 = 0; o0 < 2; ++o0) {
        if (((b0 + o0) & (RES - 1)) != j0) continue;
        const float w0 = o0 ? p0.x : 1.0f - p0.x;
#pragma unroll
        for (int o1 = 0; o1 < 2; ++o1) {
          const int l = (b1 + o1 - a0) & (RES - 1);
          if (l >= T) continue;
          const float w01 = w0 * (o1 ? p0.y : 1.0f - p0.y);
#pragma unroll
          for (int o2 = 0; o2 < 2; ++o2) {
            const int nn = (b2 + o2) & (RES - 1);
            const float w = w01 * (o2 ? p0.z : 1.0f - p0.z);
            const int addr = 2 * pidx(nn >> 1) + (nn & 1);
            if constexpr (MODE == MODE_BWDH) {
              atomicAdd(&rf[l * LS * 2 + addr], w * alpha);
            } else {
#pragma unroll
              for (int c = 0; c < 3; ++c) atomicAdd(&rf[(c * T + l) * LS * 2 + addr], w * nv[c]);
            }
          }
        }
      }
    }
  }
  __syncthreads();

  if constexpr (MODE == MODE_VOUT) {
    for (int e = threadIdx.x; e < C * T * RES; e += kBlock) {
      const int nn = e % RES, l = (e / RES) % T, c = e / (RES * T);
      vout[c * N3 + ((int64_t)j0 * RES + a0 + l) * RES + nn] = rf[(c * T + l) * LS * 2 + 2 * pidx(nn >> 1) + (nn & 1)];
    }
    return;
  } else {
    fft_lines<M, -1>(rows, C * T, LS, tw + M);
    const cf* twr = tw + RES;
    for (int e = threadIdx.x; e < C * H * T; e += kBlock) {
      const int l = e % T, k = (e / T) % H, c = e / (T * H);
      const cf* row = rows + (c * T + l) * LS;
      const cf zk = row[pidx(k == M ? 0 : k)];
      const cf zm = row[pidx(k == 0 ? 0 : M - k)];
      const cf E{0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y)};
      const cf O{0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x)};
      const cf X = cadd(E, cmul(twr[k], O));
      out[(((int64_t)c * H + k) * RES + j0) * RES + a0 + l] = X;
    }
  }
}

// ---------------------------------------------------------------------------
// P2 / B2: forward FFT along j1. A[c][k2][j0][j1] -> B[c][k1][k2][j0].
// ---------------------------------------------------------------------------
template <int RES>
__global__ __launch_bounds__(kBlock) void k_axis1_fwd(const cf* __restrict__ in, cf* __restrict__ out,
                                                      const cf* __restrict__ tw) {
  constexpr int H = RES / 2 + 1, T = tile_lines(RES), LS = lstride(RES);
  __shared__ cf rows[T * LS];
  int b = blockIdx.x;
  const int tb = b % (RES / T);
  b /= RES / T;
  const int k2 = b % H;
  const int c = b / H;
  const int a0 = tb * T;
  const cf* src = in + (((int64_t)c * H + k2) * RES + a0) * RES;
  for (int e = threadIdx.x; e < T * RES; e += kBlock) rows[(e / RES) * LS + pidx(e % RES)] = src[e];
  __syncthreads();
  fft_lines<RES, -1>(rows, T, LS, tw + RES);
  for (int e = threadIdx.x; e < T * RES; e += kBlock) {
    const int l = e % T, n = e / T;
    out[(((int64_t)c * RES + n) * H + k2) * RES + a0 + l] = rows[l * LS + pidx(n)];
  }
}

// ---------------------------------------------------------------------------
// P3: FFT along j0 of the 3 channels, chi~ = i F(k) sum_d kappa_d^odd v~_d
// with F = g / (-2 pi |kappa|^2) / N (main Eq. 3; the inverse's 1/N folded
// in), then inverse FFT along k0. B[3][k1][k2][j0] -> C[j0][k2][k1].
// ---------------------------------------------------------------------------
template <int RES>
__device__ __forceinline__ float spectral_F(int k0, int k1, int k2, float sigma) {
  const float q0 = kappa_of(k0, RES), q1 = kappa_of(k1, RES), q2 = kappa_of(k2, RES);
  const float K2 = q0 * q0 + q1 * q1 + q2 * q2;
  if (K2 == 0.0f) return 0.0f;
  constexpr float invN = 1.0f / ((float)RES * (float)RES * (float)RES);
  constexpr float inv_r2 = 1.0f / ((float)RES * (float)RES);
  const float g = expf(-2.0f * sigma * sigma * K2 * inv_r2);
  return g * invN / (-6.283185307179586f * K2);
}

template <int RES>
__global__ __launch_bounds__(kBlock) void k_fwd_axis0(const cf* __restrict__ in, cf* __restrict__ out,
                                                      const cf* __restrict__ tw, float sigma) {
  constexpr int H = RES / 2 + 1, T = tile_lines(RES), LS = lstride(RES);
  constexpr int EPT = (T * RES + kBlock - 1) / kBlock;
  __shared__ cf rows[T * LS];
  const int tb = blockIdx.x % (RES / T);
  const int k2 = blockIdx.x / (RES / T);
  const int a0 = tb * T;
  cf acc[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) acc[u] = cf{0.0f, 0.0f};
  for (int c = 0; c < 3; ++c) {
    for (int e = threadIdx.x; e < T * RES; e += kBlock) {
      const int l = e / RES, n = e % RES;
      rows[l * LS + pidx(n)] = in[(((int64_t)c * RES + a0 + l) * H + k2) * RES + n];
    }
    __syncthreads();
    fft_lines<RES, -1>(rows, T, LS, tw + RES);
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * kBlock;
      if (e < T * RES) {
        const int l = e / RES, n = e % RES;
        const float kap = c == 0 ? kappa_odd(n, RES) : (c == 1 ? kappa_odd(a0 + l, RES) : kappa_odd(k2, RES));
        const cf x = rows[l * LS + pidx(n)];
        acc[u].x += kap * x.x;
        acc[u].y += kap * x.y;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = threadIdx.x + u * kBlock;
    if (e < T * RES) {
      const int l = e / RES, n = e % RES;
      const float F = spectral_F<RES>(n, a0 + l, k2, sigma);
      rows[l * LS + pidx(n)] = cf{-F * acc[u].y, F * acc[u].x};  // i F acc
    }
  }
  __syncthreads();
  fft_lines<RES, +1>(rows, T, LS, tw + RES);
  for (int e = threadIdx.x; e < T * RES; e += kBlock) {
    const int l = e % T, n = e / T;
    out[((int64_t)n * H + k2) * RES + a0 + l] = rows[l * LS + pidx(n)];
  }
}

// B3: FFT along j0 of H^, then for each channel d: -i F kappa_d H^ (the
// conjugate operator), inverse FFT along k0. B[k1][k2][j0] -> C[3][j0][k2][k1].
template <int RES>
__global__ __launch_bounds__(kBlock) void k_bwd_axis0(const cf* __restrict__ in, cf* __restrict__ out,
                                                      const cf* __restrict__ tw, float sigma) {
  constexpr int H = RES / 2 + 1, T = tile_lines(RES), LS = lstride(RES);
  constexpr int EPT = (T * RES + kBlock - 1) / kBlock;
  __shared__ cf rows[T * LS];
  const int tb = blockIdx.x % (RES / T);
  const int k2 = blockIdx.x / (RES / T);
  const int a0 = tb * T;
  for (int e = threadIdx.x; e < T * RES; e += kBlock) {
    const int l = e / RES, n = e % RES;
    rows[l * LS + pidx(n)] = in[(((int64_t)a0 + l) * H + k2) * RES + n];
  }
  __syncthreads();
  fft_lines<RES, -1>(rows, T, LS, tw + RES);
  cf h[EPT];
  float F[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = threadIdx.x + u * kBlock;
    if (e < T * RES) {
      const int l = e / RES, n = e % RES;
      h[u] = rows[l * LS + pidx(n)];
      F[u] = spectral_F<RES>(n, a0 + l, k2, sigma);
    }
  }
  __syncthreads();
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * kBlock;
      if (e < T * RES) {
        const int l = e / RES, n = e % RES;
        const float kap = c == 0 ? kappa_odd(n, RES) : (c == 1 ? kappa_odd(a0 + l, RES) : kappa_odd(k2, RES));
        const float fk = F[u] * kap;
        rows[l * LS + pidx(n)] = cf{fk * h[u].y, -fk * h[u].x};  // -i F kappa H^
      }
    }
    __syncthreads();
    fft_lines<RES, +1>(rows, T, LS, tw + RES);
    for (int e = threadIdx.x; e < T * RES; e += kBlock) {
      const int l = e % T, n = e / T;
      out[(((int64_t)c * RES + n) * H + k2) * RES + a0 + l] = rows[l * LS + pidx(n)];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// P4 / B4: inverse FFT along k1. C[c][j0][k2][k1] -> D[c][k2][j0][j1].
// ---------------------------------------------------------------------------
template <int RES>
__global__ __launch_bounds__(kBlock) void k_axis1_inv(const cf* __restrict__ in, cf* __restrict__ out,
                                                      const cf* __restrict__ tw) {
  constexpr int H = RES / 2 + 1, T = tile_lines(RES), LS = lstride(RES);
  __shared__ cf rows[T * LS];
  int b = blockIdx.x;
  const int tb = b % (RES / T);
  b /= RES / T;
  const int k2 = b % H;
  const int c = b / H;
  const int a0 = tb * T;
  for (int e = threadIdx.x; e < T * RES; e += kBlock) {
    const int l = e / RES, n = e % RES;
    rows[l * LS + pidx(n)] = in[(((int64_t)c * RES + a0 + l) * H + k2) * RES + n];
  }
  __syncthreads();
  fft_lines<RES, +1>(rows, T, LS, tw + RES);
  cf* dst = out + (((int64_t)c * H + k2) * RES + a0) * RES;
  for (int e = threadIdx.x; e < T * RES; e += kBlock) dst[e] = rows[(e / RES) * LS + pidx(e % RES)];
}

// ---------------------------------------------------------------------------
// P5 / B5: complex-to-real inverse FFT along k2 of a tile of lines, then the
// trilinear gather at the points whose corner lines fall in the tile.
// MODE_FWD: 1 channel; writes chi' rows and per (point, corner-line) partials
//           (value, d/dc0, d/dc1, d/dc2) of the interpolant.
// MODE_BWD: 3 channels g_v; partials of dL/dn (3) and dL/dc (3).
// MODE_DBG: 1 channel; writes chi' rows only.
// ---------------------------------------------------------------------------
enum { MODE_FWD = 0, MODE_BWD = 1, MODE_DBG = 2 };

template <int RES, int MODE>
__global__ __launch_bounds__(kBlock) void k_c2r_gather(const cf* __restrict__ in, float* __restrict__ chi_out,
                                                       const PointRec* __restrict__ sorted,
                                                       const int* __restrict__ off, float4* __restrict__ part,
                                                       const cf* __restrict__ tw) {
  constexpr int M = RES / 2, H = M + 1, T = tile_lines(RES);
  constexpr int C = MODE == MODE_BWD ? 3 : 1;
  constexpr int LS = lstride(M);
  __shared__ cf rows[C * T * LS];
  const float* rf = reinterpret_cast<const float*>(rows);
  const int tb = blockIdx.x % (RES / T);
  const int j0 = blockIdx.x / (RES / T);
  const int a0 = tb * T;

  for (int e = threadIdx.x; e < C * H * T; e += kBlock) {
    const int l = e % T, k = (e / T) % H, c = e / (T * H);
    rows[(c * T + l) * LS + pidx(k)] = in[(((int64_t)c * H + k) * RES + j0) * RES + a0 + l];
  }
  __syncthreads();
  // Hermitian half-spectrum X[0..M] -> packed spectrum Z[0..M) of the
  // even/odd samples: Z = (X_k + X*_{M-k}) + i (X_k - X*_{M-k}) e^{+2 pi i k/r}.
  {
    constexpr int NP = M / 2 + 1;
    const cf* twr = tw + RES;
    for (int e = threadIdx.x; e < C * T * NP; e += kBlock) {
      const int k = e % NP, row = e / NP;
      cf* rp = rows + row * LS;
      const cf xk = rp[pidx(k)], xm = rp[pidx(M - k)];
      {
        const cf Ee{xk.x + xm.x, xk.y - xm.y};
        const cf Dd{xk.x - xm.x, xk.y + xm.y};
        const cf w{twr[k].x, -twr[k].y};
        const cf Oo = cmul(Dd, w);
        rp[pidx(k)] = cf{Ee.x - Oo.y, Ee.y + Oo.x};
      }
      if (k != 0 && 2 * k != M) {
        const cf Ee{xm.x + xk.x, xm.y - xk.y};
        const cf Dd{xm.x - xk.x, xm.y + xk.y};
        const cf w{twr[M - k].x, -twr[M - k].y};
        const cf Oo = cmul(Dd, w);
        rp[pidx(M - k)] = cf{Ee.x - Oo.y, Ee.y + Oo.x};
      }
    }
  }
  __syncthreads();
  fft_lines<M, +1>(rows, C * T, LS, tw + M);
  // rows now hold real lines, sample n at float slot 2 pidx(n/2) + (n&1)
  if constexpr (MODE != MODE_BWD) {
    for (int e = threadIdx.x; e < T * RES; e += kBlock) {
      const int l = e / RES, n = e % RES;
      chi_out[((int64_t)j0 * RES + a0 + l) * RES + n] = rf[l * LS * 2 + 2 * pidx(n >> 1) + (n & 1)];
    }
  }
  if constexpr (MODE != MODE_DBG) {
    int lo[4], hi[4];
    const int nr = tile_ranges<RES, T>(off, j0, a0, lo, hi);
    int total = 0;
    for (int r = 0; r < nr; ++r) total += hi[r] - lo[r];
    for (int qd = threadIdx.x; qd < total; qd += kBlock) {
      const int64_t s = range_pick(lo, hi, nr, qd);
      float4 p0, p1;
      load_rec(sorted, s, p0, p1);
      const uint32_t bb = __float_as_uint(p0.w);
      const int b0 = bb & 1023, b1 = (bb >> 10) & 1023, b2 = bb >> 20;
      const int n0 = b2, n1 = (b2 + 1) & (RES - 1);
      const int s0 = 2 * pidx(n0 >> 1) + (n0 & 1), s1 = 2 * pidx(n1 >> 1) + (n1 & 1);
      const float fz = p0.z;
#pragma unroll
      for (int o0 = 0; o0 < 2; ++o0) {
        if (((b0 + o0) & (RES - 1)) != j0) continue;
        const float wa = o0 ? p0.x : 1.0f - p0.x;
        const float sa = o0 ? 1.0f : -1.0f;
#pragma unroll
        for (int o1 = 0; o1 < 2; ++o1) {
          const int l = (b1 + o1 - a0) & (RES - 1);
          if (l >= T) continue;
          const float wb = o1 ? p0.y : 1.0f - p0.y;
          const float sb = o1 ? 1.0f : -1.0f;
          const int slot = o0 * 2 + o1;
          if constexpr (MODE == MODE_FWD) {
            const float v0 = rf[l * LS * 2 + s0], v1 = rf[l * LS * 2 + s1];
            const float L = (1.0f - fz) * v0 + fz * v1;
            const float dL = v1 - v0;
            part[s * 4 + slot] = make_float4(wa * wb * L, (float)RES * sa * wb * L, (float)RES * wa * sb * L,
                                             (float)RES * wa * wb * dL);
          } else {
            float Lc[3], dLc[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const float v0 = rf[(c * T + l) * LS * 2 + s0], v1 = rf[(c * T + l) * LS * 2 + s1];
              Lc[c] = (1.0f - fz) * v0 + fz * v1;
              dLc[c] = v1 - v0;
            }
            const float Ln = p1.x * Lc[0] + p1.y * Lc[1] + p1.z * Lc[2];
            const float dLn = p1.x * dLc[0] + p1.y * dLc[1] + p1.z * dLc[2];
            const float ww = wa * wb;
            part[(s * 4 + slot) * 2 + 0] = make_float4(ww * Lc[0], ww * Lc[1], ww * Lc[2], (float)RES * sa * wb * Ln);
            part[(s * 4 + slot) * 2 + 1] = make_float4((float)RES * wa * sb * Ln, (float)RES * ww * dLn, 0.0f, 0.0f);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 reductions and normalisation (main Eq. 4)
// ---------------------------------------------------------------------------
template <typename Tv>
__device__ __forceinline__ Tv block_sum(Tv v, Tv* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = blockDim.x / 2; d > 0; d >>= 1) {
    if (t < d) sh[t] += sh[t + d];
    __syncthreads();
  }
  const Tv r = sh[0];
  __syncthreads();
  return r;
}

// per point: f_i = sum of its 4 corner-line partials (FP64), grad f_i (FP32)
__global__ __launch_bounds__(256) void k_fwd_point_reduce(const float4* __restrict__ part, int64_t npoints,
                                                          float4* __restrict__ gradf, double* __restrict__ blockpart) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < npoints; s += (int64_t)gridDim.x * blockDim.x) {
    const float4 q0 = part[s * 4 + 0], q1 = part[s * 4 + 1], q2 = part[s * 4 + 2], q3 = part[s * 4 + 3];
    const double f = ((double)q0.x + (double)q1.x) + ((double)q2.x + (double)q3.x);
    gradf[s] = make_float4((q0.y + q1.y) + (q2.y + q3.y), (q0.z + q1.z) + (q2.z + q3.z),
                           (q0.w + q1.w) + (q2.w + q3.w), (float)f);
    acc += f;
  }
  const double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) blockpart[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_fwd_scalars(const double* __restrict__ blockpart, int nb,
                                                     const float* __restrict__ chi, SavedHeader* __restrict__ hdr) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) a += blockpart[i];
  const double tot = block_sum(a, sh);
  if (threadIdx.x == 0) {
    const double mu = tot / (double)hdr->npoints;
    const double chi0 = (double)chi[0];
    const double c = hdr->reading == 0 ? chi0 - mu : chi0;
    int status = 0;
    if (hdr->flags & 1) status = -6;  // PSR_ENONFINITE
    else if (!(c != 0.0) || !isfinite(c) || !isfinite(mu)) status = -3;  // PSR_EDEGENERATE
    hdr->status = status;
    hdr->mu = mu;
    hdr->chi0 = chi0;
    hdr->cscale = c;
    hdr->scale = status ? __longlong_as_double(0x7ff8000000000000LL) : (double)hdr->m / fabs(c);
  }
}

__global__ void k_normalize(float* __restrict__ chi, int64_t n, const SavedHeader* __restrict__ hdr) {
  const double mu = hdr->mu, s = hdr->scale;
  float4* c4 = reinterpret_cast<float4*>(chi);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n / 4; i += (int64_t)gridDim.x * blockDim.x) {
    float4 v = c4[i];
    v.x = (float)(((double)v.x - mu) * s);
    v.y = (float)(((double)v.y - mu) * s);
    v.z = (float)(((double)v.z - mu) * s);
    v.w = (float)(((double)v.w - mu) * s);
    c4[i] = v;
  }
}

// backward: S_G = sum G, S_Gchi = sum G chi (FP64 partials per block)
__global__ __launch_bounds__(256) void k_bwd_reduce(const float* __restrict__ G, const float* __restrict__ chi,
                                                    int64_t n, double2* __restrict__ blockpart) {
  __shared__ double sh[256];
  double sg = 0.0, sgc = 0.0;
  const float4* g4 = reinterpret_cast<const float4*>(G);
  const float4* c4 = reinterpret_cast<const float4*>(chi);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n / 4; i += (int64_t)gridDim.x * blockDim.x) {
    const float4 g = g4[i], c = c4[i];
    sg += ((double)g.x + (double)g.y) + ((double)g.z + (double)g.w);
    sgc += ((double)g.x * c.x + (double)g.y * c.y) + ((double)g.z * c.z + (double)g.w * c.w);
  }
  const double a = block_sum(sg, sh);
  const double b = block_sum(sgc, sh);
  if (threadIdx.x == 0) blockpart[blockIdx.x] = make_double2(a, b);
}

__global__ __launch_bounds__(256) void k_bwd_scalars(const double2* __restrict__ blockpart, int nb,
                                                     const SavedHeader* __restrict__ hdr, BwdScalars* __restrict__ bs) {
  __shared__ double sh[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    a += blockpart[i].x;
    b += blockpart[i].y;
  }
  const double SG = block_sum(a, sh);
  const double SGc = block_sum(b, sh);
  if (threadIdx.x == 0) {
    const double s = hdr->scale, c = hdr->cscale;
    const double Q = SGc / c;
    const double gmu = -s * SG + (hdr->reading == 0 ? Q : 0.0);
    bs->S_G = SG;
    bs->S_Gchi = SGc;
    bs->Qd = Q;
    bs->gmu = gmu;
    bs->s = (float)s;
    bs->q = (float)Q;
    bs->alpha = (float)(gmu / (double)hdr->npoints);
  }
}

__global__ void k_bwd_point_finalize(const float4* __restrict__ part, const float4* __restrict__ gradf,
                                     const PointRec* __restrict__ sorted, const BwdScalars* __restrict__ bs,
                                     int64_t npoints, float* __restrict__ dpoints, float* __restrict__ dnormals) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= npoints) return;
  float dn[3] = {0, 0, 0}, dc[3] = {0, 0, 0};
#pragma unroll
  for (int slot = 0; slot < 4; ++slot) {
    const float4 a = part[(s * 4 + slot) * 2 + 0], b = part[(s * 4 + slot) * 2 + 1];
    dn[0] += a.x;
    dn[1] += a.y;
    dn[2] += a.z;
    dc[0] += a.w;
    dc[1] += b.x;
    dc[2] += b.y;
  }
  const float alpha = bs->alpha;
  const float4 g = gradf[s];
  dc[0] += alpha * g.x;
  dc[1] += alpha * g.y;
  dc[2] += alpha * g.z;
  const uint32_t i = sorted[s].idx;
  if (dpoints) {
    dpoints[3 * (int64_t)i + 0] = dc[0];
    dpoints[3 * (int64_t)i + 1] = dc[1];
    dpoints[3 * (int64_t)i + 2] = dc[2];
  }
  if (dnormals) {
    dnormals[3 * (int64_t)i + 0] = dn[0];
    dnormals[3 * (int64_t)i + 1] = dn[1];
    dnormals[3 * (int64_t)i + 2] = dn[2];
  }
}

// ---------------------------------------------------------------------------
// host-side launchers, one instantiation per resolution
// ---------------------------------------------------------------------------
#define PSR_CHECK_LAUNCH()                       \
  do {                                           \
    if (hipGetLastError() != hipSuccess) return -4; \
  } while (0)

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

template <int RES>
static int launch_bin(Exec& x, const float* pts, const float* nrm, int64_t P, const WsView& w, const SavedView& sv) {
  constexpr int N2 = RES * RES;
  x.begin(STAGE_BIN);
  hipLaunchKernelGGL(k_init, dim3(nblk(N2, 256) > 1024 ? 1024 : nblk(N2, 256)), dim3(256), 0, x.stream, w.counts, N2,
                     sv.hdr, RES, P, x.sigma, (float)x.m, x.reading);
  hipLaunchKernelGGL(k_bin<RES>, dim3(nblk(P, 256)), dim3(256), 0, x.stream, pts, nrm, P, w.counts, w.tmp, w.colrank,
                     sv.hdr);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, x.stream, w.counts, sv.off, N2);
  hipLaunchKernelGGL(k_scatter, dim3(nblk(P, 256)), dim3(256), 0, x.stream, w.tmp, w.colrank, sv.off, sv.sorted, P);
  x.end(STAGE_BIN);
  PSR_CHECK_LAUNCH();
  return 0;
}

template <int RES>
static int launch_forward(Exec& x, const float* pts, const float* nrm, int64_t P, float* chi, const WsView& w,
                          const SavedView& sv) {
  constexpr int H = RES / 2 + 1, T = tile_lines(RES);
  constexpr int64_t N3 = (int64_t)RES * RES * RES;
  if (int rc = launch_bin<RES>(x, pts, nrm, P, w, sv)) return rc;
  x.begin(STAGE_P1);
  hipLaunchKernelGGL((k_splat_r2c<RES, MODE_SPLAT>), dim3(RES * (RES / T)), dim3(kBlock), 0, x.stream, sv.sorted,
                     sv.off, (const float*)nullptr, (const BwdScalars*)nullptr, x.tw, w.X, (float*)nullptr);
  x.end(STAGE_P1);
  x.begin(STAGE_P2);
  hipLaunchKernelGGL(k_axis1_fwd<RES>, dim3(3 * H * (RES / T)), dim3(kBlock), 0, x.stream, w.X, w.Y, x.tw);
  x.end(STAGE_P2);
  x.begin(STAGE_P3);
  hipLaunchKernelGGL(k_fwd_axis0<RES>, dim3(H * (RES / T)), dim3(kBlock), 0, x.stream, w.Y, w.X, x.tw, x.sigma);
  x.end(STAGE_P3);
  x.begin(STAGE_P4);
  hipLaunchKernelGGL(k_axis1_inv<RES>, dim3(H * (RES / T)), dim3(kBlock), 0, x.stream, w.X, w.Y, x.tw);
  x.end(STAGE_P4);
  x.begin(STAGE_P5);
  hipLaunchKernelGGL((k_c2r_gather<RES, MODE_FWD>), dim3(RES * (RES / T)), dim3(kBlock), 0, x.stream, w.Y, chi,
                     sv.sorted, sv.off, w.part, x.tw);
  x.end(STAGE_P5);
  const int nb = nblk(P, 256) > kRedBlocks ? kRedBlocks : nblk(P, 256);
  x.begin(STAGE_FWD_REDUCE);
  hipLaunchKernelGGL(k_fwd_point_reduce, dim3(nb), dim3(256), 0, x.stream, w.part, P, sv.gradf, w.blockpart);
  hipLaunchKernelGGL(k_fwd_scalars, dim3(1), dim3(256), 0, x.stream, w.blockpart, nb, chi, sv.hdr);
  x.end(STAGE_FWD_REDUCE);
  x.begin(STAGE_NORMALIZE);
  hipLaunchKernelGGL(k_normalize, dim3(nblk(N3 / 4, 256) > 4096 ? 4096 : nblk(N3 / 4, 256)), dim3(256), 0, x.stream,
                     chi, N3, sv.hdr);
  x.end(STAGE_NORMALIZE);
  PSR_CHECK_LAUNCH();
  return 0;
}

template <int RES>
static int launch_backward(Exec& x, int64_t P, const float* chi, const float* dchi, float* dpts, float* dnrm,
                           const WsView& w, const SavedView& sv) {
  constexpr int H = RES / 2 + 1, T = tile_lines(RES);
  constexpr int64_t N3 = (int64_t)RES * RES * RES;
  const int nbr = kRedBlocks;
  x.begin(STAGE_BWD_REDUCE);
  hipLaunchKernelGGL(k_bwd_reduce, dim3(nbr), dim3(256), 0, x.stream, dchi, chi, N3, (double2*)w.blockpart);
  hipLaunchKernelGGL(k_bwd_scalars, dim3(1), dim3(256), 0, x.stream, (const double2*)w.blockpart, nbr,
                     (const SavedHeader*)sv.hdr, w.bs);
  x.end(STAGE_BWD_REDUCE);
  x.begin(STAGE_B1);
  hipLaunchKernelGGL((k_splat_r2c<RES, MODE_BWDH>), dim3(RES * (RES / T)), dim3(kBlock), 0, x.stream, sv.sorted,
                     sv.off, dchi, (const BwdScalars*)w.bs, x.tw, w.X, (float*)nullptr);
  x.end(STAGE_B1);
  x.begin(STAGE_B2);
  hipLaunchKernelGGL(k_axis1_fwd<RES>, dim3(1 * H * (RES / T)), dim3(kBlock), 0, x.stream, w.X, w.Y, x.tw);
  x.end(STAGE_B2);
  x.begin(STAGE_B3);
  hipLaunchKernelGGL(k_bwd_axis0<RES>, dim3(H * (RES / T)), dim3(kBlock), 0, x.stream, w.Y, w.X, x.tw, x.sigma);
  x.end(STAGE_B3);
  x.begin(STAGE_B4);
  hipLaunchKernelGGL(k_axis1_inv<RES>, dim3(3 * H * (RES / T)), dim3(kBlock), 0, x.stream, w.X, w.Y, x.tw);
  x.end(STAGE_B4);
  x.begin(STAGE_B5);
  hipLaunchKernelGGL((k_c2r_gather<RES, MODE_BWD>), dim3(RES * (RES / T)), dim3(kBlock), 0, x.stream, w.Y,
                     (float*)nullptr, sv.sorted, sv.off, w.part, x.tw);
  x.end(STAGE_B5);
  x.begin(STAGE_BWD_FINAL);
  hipLaunchKernelGGL(k_bwd_point_finalize, dim3(nblk(P, 256)), dim3(256), 0, x.stream, (const float4*)w.part,
                     (const float4*)sv.gradf, (const PointRec*)sv.sorted, (const BwdScalars*)w.bs, P, dpts, dnrm);
  x.end(STAGE_BWD_FINAL);
  PSR_CHECK_LAUNCH();
  return 0;
}

template <int RES>
static int launch_debug_spectral(Exec& x, const float* v, float* chi_prime, const WsView& w) {
  constexpr int H = RES / 2 + 1, T = tile_lines(RES);
  hipLaunchKernelGGL((k_splat_r2c<RES, MODE_LOADV>), dim3(RES * (RES / T)), dim3(kBlock), 0, x.stream,
                     (const PointRec*)nullptr, (const int*)nullptr, v, (const BwdScalars*)nullptr, x.tw, w.X,
                     (float*)nullptr);
  hipLaunchKernelGGL(k_axis1_fwd<RES>, dim3(3 * H * (RES / T)), dim3(kBlock), 0, x.stream, w.X, w.Y, x.tw);
  hipLaunchKernelGGL(k_fwd_axis0<RES>, dim3(H * (RES / T)), dim3(kBlock), 0, x.stream, w.Y, w.X, x.tw, x.sigma);
  hipLaunchKernelGGL(k_axis1_inv<RES>, dim3(H * (RES / T)), dim3(kBlock), 0, x.stream, w.X, w.Y, x.tw);
  hipLaunchKernelGGL((k_c2r_gather<RES, MODE_DBG>), dim3(RES * (RES / T)), dim3(kBlock), 0, x.stream, w.Y,
                     chi_prime, (const PointRec*)nullptr, (const int*)nullptr, (float4*)nullptr, x.tw);
  PSR_CHECK_LAUNCH();
  return 0;
}

template <int RES>
static int launch_debug_splat(Exec& x, const float* pts, const float* nrm, int64_t P, float* v, const WsView& w,
                              const SavedView& sv) {
  constexpr int T = tile_lines(RES);
  if (int rc = launch_bin<RES>(x, pts, nrm, P, w, sv)) return rc;
  hipLaunchKernelGGL((k_splat_r2c<RES, MODE_VOUT>), dim3(RES * (RES / T)), dim3(kBlock), 0, x.stream, sv.sorted,
                     sv.off, (const float*)nullptr, (const BwdScalars*)nullptr, x.tw, (cf*)nullptr, v);
  PSR_CHECK_LAUNCH();
  return 0;
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

int run_forward(Exec& x, int res, const float* pts, const float* nrm, int64_t P, float* chi, const WsView& w,
                const SavedView& sv) {
#define CALL(R) launch_forward<R>(x, pts, nrm, P, chi, w, sv)
  PSR_DISPATCH(res, CALL)
#undef CALL
}

int run_backward(Exec& x, int res, int64_t P, const float* chi, const float* dchi, float* dpts, float* dnrm,
                 const WsView& w, const SavedView& sv) {
#define CALL(R) launch_backward<R>(x, P, chi, dchi, dpts, dnrm, w, sv)
  PSR_DISPATCH(res, CALL)
#undef CALL
}

int run_debug_spectral(Exec& x, int res, const float* v, float* chi_prime, const WsView& w) {
#define CALL(R) launch_debug_spectral<R>(x, v, chi_prime, w)
  PSR_DISPATCH(res, CALL)
#undef CALL
}

int run_debug_splat(Exec& x, int res, const float* pts, const float* nrm, int64_t P, float* v, const WsView& w,
                    const SavedView& sv) {
#define CALL(R) launch_debug_splat<R>(x, pts, nrm, P, v, w, sv)
  PSR_DISPATCH(res, CALL)
#undef CALL
}

}  // namespace psr
