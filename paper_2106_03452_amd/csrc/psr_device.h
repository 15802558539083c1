// Device helpers shared by the solver's passes and the slab solve: wave
// numbers, sorted point records and their ranges, the fixed-point LDS splat
// of rows, the spectral factor of main Eq. 3 and block reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fft_device.h"
#include "psr_internal.h"

namespace psr {

__device__ __forceinline__ float kappa_of(int k, int res) { return (float)(k < res / 2 ? k : k - res); }
// odd (first-derivative) factor: zero at the Nyquist index
__device__ __forceinline__ float kappa_odd(int k, int res) { return k == res / 2 ? 0.0f : kappa_of(k, res); }

__device__ __forceinline__ void load_rec(const PointRec* __restrict__ s, int64_t i, float4& a, float4& b) {
  const float4* p = reinterpret_cast<const float4*>(s + i);
  a = p[0];
  b = p[1];
}

// Up to four disjoint ranges of sorted point records (unused ones empty),
// kept in named scalars so nothing is indexed dynamically.
struct Ranges {
  int lo[4], n[4];
  int total;
};

// LDS layout of the half-length rows of the row passes: row l starts at
// l * row_ls(M), element i sits at pidx(i) ^ row_swz(M, l). At M = 128 the
// XOR skew puts the rows one wavefront touches together on different banks,
// both in the FFT stages (8 rows x 8 threads) and in the line-pair transposes
// of the loads and stores (32 rows, one element).
__host__ __device__ constexpr int row_ls(int M) { return M == 128 ? 152 : lstride(M); }
__host__ __device__ constexpr int row_swz(int M, int l) { return M == 128 ? (l >> 1) & 15 : 0; }
template <int M>
__device__ __forceinline__ int rpos(int l, int i) {
  return l * row_ls(M) + (pidx(i) ^ row_swz(M, l));
}

// Sorted index of the q-th point of the ranges (q < R.total).
__device__ __forceinline__ int64_t range_pick(const Ranges& R, int q) {
  int64_t s = R.lo[3] + (q - R.n[0] - R.n[1] - R.n[2]);
  if (q < R.n[0] + R.n[1] + R.n[2]) s = R.lo[2] + (q - R.n[0] - R.n[1]);
  if (q < R.n[0] + R.n[1]) s = R.lo[1] + (q - R.n[0]);
  if (q < R.n[0]) s = R.lo[0] + q;
  return s;
}

// Up to K point records per thread fetched ahead (thread t takes points t,
// t + BLOCK, ... of the ranges), so the splat and gather loops find them in
// registers instead of waiting on a dependent global load each turn.
template <int K>
struct Recs {
  float4 a[K], b[K];
  int64_t s[K];
};

template <int K, int BLOCK>
__device__ __forceinline__ void fetch_recs(Recs<K>& r, const PointRec* __restrict__ sorted, const Ranges& R,
                                           int t) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int q = t + k * BLOCK;
    r.s[k] = 0;
    r.a[k] = make_float4(0, 0, 0, 0);
    r.b[k] = r.a[k];
    if (q < R.total) {
      r.s[k] = range_pick(R, q);
      load_rec(sorted, r.s[k], r.a[k], r.b[k]);
    }
  }
}

// f(a, b, s) for every point this thread takes: the fetched ones, then any
// beyond K * BLOCK loaded on the way, KT at a time (their loads in flight
// together; KT = 0: one at a time, for kernels without registers to spare).
template <int K, int BLOCK, int KT = 0, typename F>
__device__ __forceinline__ void for_recs(const Recs<K>& r, const PointRec* __restrict__ sorted, const Ranges& R,
                                         int t, F&& f) {
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (t + k * BLOCK < R.total) f(r.a[k], r.b[k], r.s[k]);
  if constexpr (KT == 0) {
    for (int q = t + K * BLOCK; q < R.total; q += BLOCK) {
      float4 a, b;
      const int64_t s = range_pick(R, q);
      load_rec(sorted, s, a, b);
      f(a, b, s);
    }
  } else {
    for (int q0 = t + K * BLOCK; q0 < R.total; q0 += KT * BLOCK) {
      Recs<KT> c;
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        const int q = q0 + k * BLOCK;
        c.s[k] = 0;
        c.a[k] = make_float4(0, 0, 0, 0);
        c.b[k] = c.a[k];
        if (q < R.total) {
          c.s[k] = range_pick(R, q);
          load_rec(sorted, c.s[k], c.a[k], c.b[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < KT; ++k)
        if (q0 + k * BLOCK < R.total) f(c.a[k], c.b[k], c.s[k]);
    }
  }
}

// Records fetched together in the tail of the splat's and gathers' point
// loops (beyond the first K * BLOCK, so only where a span is dense): none at
// 256^3 and 512^3, whose row passes have no registers to spare below the
// 128 that two workgroups per CU allow; eight at 64^3 and below, whose
// plane and row passes (a few hundred workgroups, registers to spare) walk
// the longest lists (10^6 points: 64^3 1.78 -> 1.35 ms, 32^3 1.53 -> 1.15 ms);
// at 128^3 eight cost more in register pressure than they save (the
// 64-shape batch 33.1k -> 31.3k shapes/s).
__host__ __device__ constexpr int rec_tail(int res) { return res >= 256 ? 0 : (res == 64 || res <= 32 ? 8 : 2); }

// Fixed-point splat. LDS float atomics are several times slower than integer
// ones on gfx950, and their result depends on the order of the adds, so the
// splat accumulates integers: each corner contribution w * value becomes
// rintf(w * value * 2^S) with 2^S * maxabs <= 2^30, where maxabs bounds the
// |value| of the span's points. Every contribution then fits in 31 bits and
// is added to a 64-bit LDS accumulator; at most 2^30 points (the library's
// limit) keep any partial sum below 2^60. The rounding error of one
// contribution is at most 2^-S / 2 <= maxabs * 2^-30, independent of how
// many points share the span or how their contributions cancel (opposite
// normals of a thin wall in one cell). Integer sums do not depend on the
// order of the adds: the splat is bitwise reproducible.
//
// Returns 2^S for maxabs and sets inv = 2^-S (both built from exponent bits).
__device__ __forceinline__ float splat_scale(float maxabs, float& inv) {
  int S = 0;
  if (maxabs > 0.0f) {
    // maxabs < 2^e with e = biased exponent - 126 (also for subnormal
    // maxabs); an infinite maxabs (absurd normals) takes the smallest scale
    const int e = ((__float_as_int(maxabs) >> 23) & 0xff) - 126;
    S = 30 - e;
    S = S > 126 ? 126 : (S < -126 || e > 128 ? -126 : S);
  }
  inv = __int_as_float((127 - S) << 23);
  return __int_as_float((127 + S) << 23);
}

// Maximum of m over a workgroup of BLOCK threads: each wavefront's maximum
// goes to wmax[wave] (BLOCK < 64: one partial wavefront, shuffles stay within
// its BLOCK lanes); block_max reads them back after the next barrier.
template <int BLOCK>
__device__ __forceinline__ void wave_max_store(float* wmax, float m) {
  constexpr int W = BLOCK < 64 ? BLOCK : 64;
#pragma unroll
  for (int d = W / 2; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, W));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
}
template <int BLOCK>
__device__ __forceinline__ float block_max(const float* wmax) {
  float m = wmax[0];
#pragma unroll
  for (int w = 1; w < (BLOCK + 63) / 64; ++w) m = fmaxf(m, wmax[w]);
  return m;
}

// Copy the twiddle table of length L (exp(-2 pi i e / L), e in [0, n)) into
// LDS; the first barrier of the caller makes it visible. Loaded at kernel
// start so the copy overlaps the data loads instead of stalling a stage.
template <int BLOCK>
__device__ __forceinline__ void stage_table(cf* dst, const cf* __restrict__ src, int n) {
  for (int e = threadIdx.x; e < n; e += BLOCK) dst[e] = src[e];
}

// Rows [a0, a0 + NROWS) of plane j0 of one channel into LDS as float samples
// (row l, sample n at float slot 2 rpos(l, n/2) + (n & 1)). KIND 0: splat of
// normal component ch over the points of R; KIND 1: the cotangent without
// its point source at vertex 0, H = s G + alpha W (W = splat of ones, G from
// gin; the -Q delta_0 term is applied at the points from the point-source
// table, see b_bwd_point_finalize); KIND 2: rows of v_ch from gin. Ends with a
// barrier.
template <int RES, int NROWS, int BLOCK, int KIND>
__device__ __forceinline__ void fill_rows(cf* rows, const PointRec* __restrict__ sorted, const Ranges& R,
                                          const float* __restrict__ gin, float3 sqa, int j0, int a0, int ch) {
  constexpr int M = RES / 2;
  constexpr int64_t N3 = (int64_t)RES * RES * RES;
  const int t = threadIdx.x;
  // the NROWS rows are one contiguous run of NROWS * RES floats
  constexpr int NV = NROWS * M / 2;  // float4 = two complex slots
  constexpr int IT = (NV + BLOCK - 1) / BLOCK;
  if (KIND == 2 || (KIND == 1 && R.total == 0)) {
    // rows straight from memory: v_ch (KIND 2), or s G where no point adds
    // to W (KIND 1; uniform over the workgroup)
    const float sg = KIND == 1 ? sqa.x : 1.0f;
    const float4* g4 = reinterpret_cast<const float4*>(gin + (KIND == 2 ? ch * N3 : 0) + ((int64_t)j0 * RES + a0) * RES);
    float4 buf[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * BLOCK;
      if (e < NV) buf[it] = g4[e];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * BLOCK;
      if (e < NV) {
        const int mm = (2 * e) % M, l = (2 * e) / M;
        rows[rpos<M>(l, mm)] = cf{buf[it].x * sg, buf[it].y * sg};
        rows[rpos<M>(l, mm + 1)] = cf{buf[it].z * sg, buf[it].w * sg};
      }
    }
  } else if constexpr (KIND != 2) {
    // splat of normal component ch (or of unit weights: W in the backward)
    // in 64-bit fixed point, then back to floats, and in the backward
    // H = s G + alpha W. A complex LDS slot (8 bytes) holds two
    // samples as floats but one as a 64-bit integer, so the samples are
    // accumulated in two rounds in place: even samples (the real parts),
    // then odd samples; the even sums wait in registers meanwhile.
    __shared__ float wmax[(BLOCK + 63) / 64];
    constexpr int KR = 4;
    Recs<KR> recs;
    fetch_recs<KR, BLOCK>(recs, sorted, R, t);
    unsigned long long* const r64 = reinterpret_cast<unsigned long long*>(rows);
    float4 gbuf[KIND == 1 ? IT : 1];
    if constexpr (KIND == 1) {
      const float4* g4 = reinterpret_cast<const float4*>(gin + ((int64_t)j0 * RES + a0) * RES);
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int e = t + it * BLOCK;
        if (e < NV) gbuf[it] = g4[e];
      }
    }
    // each thread owns the two slots (l, mm), (l, mm + 1) of its float4s:
    // every slot the splat touches has one owner, which zeroes it before
    // each round and converts it after
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * BLOCK;
      if (e < NV) {
        const int mm = (2 * e) % M, l = (2 * e) / M;
        r64[rpos<M>(l, mm)] = 0ull;
        r64[rpos<M>(l, mm + 1)] = 0ull;
      }
    }
    float m = 1.0f;
    if constexpr (KIND == 0) {
      m = 0.0f;
      for_recs<KR, BLOCK, rec_tail(RES)>(recs, sorted, R, t, [&](const float4&, const float4& p1, int64_t) {
        m = fmaxf(m, fabsf(ch == 0 ? p1.x : (ch == 1 ? p1.y : p1.z)));
      });
    }
    wave_max_store<BLOCK>(wmax, m);
    __syncthreads();
    float inv = 1.0f;
    const float sc = splat_scale(block_max<BLOCK>(wmax), inv);
    float2 even[IT];  // the finished even samples (l, 2 mm) and (l, 2 mm + 2) of each owned float4
    const float alpha = KIND == 1 ? sqa.z : 1.0f;
#pragma unroll 1
    for (int par = 0; par < 2; ++par) {
      for_recs<KR, BLOCK, rec_tail(RES)>(recs, sorted, R, t, [&](const float4& p0, const float4& p1, int64_t) {
        const uint32_t bb = __float_as_uint(p0.w);
        const int b0 = bb & 1023, b1 = (bb >> 10) & 1023, b2 = bb >> 20;
        float val;
        if constexpr (KIND == 1) val = 1.0f;
        else val = ch == 0 ? p1.x : (ch == 1 ? p1.y : p1.z);
        // the corner along j2 whose sample index has this round's parity
        // (r is even, so the wrap keeps the parity)
        const int o2 = (b2 & 1) ^ par;
        const int nn = (b2 + o2) & (RES - 1);
        const float w2 = o2 ? p0.z : 1.0f - p0.z;
#pragma unroll
        for (int o0 = 0; o0 < 2; ++o0) {
          if (((b0 + o0) & (RES - 1)) != j0) continue;
          const float w0 = o0 ? p0.x : 1.0f - p0.x;
#pragma unroll
          for (int o1 = 0; o1 < 2; ++o1) {
            const int l = (b1 + o1 - a0) & (RES - 1);
            if (l >= NROWS) continue;
            // w2 first: every product depends on the round, so nothing of it
            // is hoisted out of the round loop into registers
            const float w = ((w2 * w0) * (o1 ? p0.y : 1.0f - p0.y)) * val;
            atomicAdd(&r64[rpos<M>(l, nn >> 1)], (unsigned long long)(long long)(int)rintf(w * sc));
          }
        }
      });
      __syncthreads();
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int e = t + it * BLOCK;
        if (e < NV) {
          const int mm = (2 * e) % M, l = (2 * e) / M;
          const int i0 = rpos<M>(l, mm), i1 = rpos<M>(l, mm + 1);
          float x0 = (float)(long long)r64[i0] * inv, x1 = (float)(long long)r64[i1] * inv;
          if constexpr (KIND == 1) {
            // H = s G + alpha W
            x0 = alpha * x0 + sqa.x * (par ? gbuf[it].y : gbuf[it].x);
            x1 = alpha * x1 + sqa.x * (par ? gbuf[it].w : gbuf[it].z);
          }
          if (par == 0) {
            even[it] = make_float2(x0, x1);
            r64[i0] = 0ull;
            r64[i1] = 0ull;
          } else {
            rows[i0] = cf{even[it].x, x0};
            rows[i1] = cf{even[it].y, x1};
          }
        }
      }
      if (par == 0) __syncthreads();  // the odd round's adds reach slots other threads own
    }
  }
  __syncthreads();
}

// Separable Gaussian of main Eq. 3: g(k) = g1(k0) g1(k1) g1(k2) with
// g1(k) = exp(-2 sigma^2 kappa(k)^2 / r^2); one table of RES floats per
// workgroup in LDS (the Nyquist index keeps kappa^2 = (r/2)^2).
template <int RES, int BLOCK>
__device__ __forceinline__ void gauss_table(float* g1, float sigma) {
  constexpr float inv_r2 = 1.0f / ((float)RES * (float)RES);
  for (int e = threadIdx.x; e < RES; e += BLOCK) {
    const float q = kappa_of(e, RES);
    g1[e] = expf(-2.0f * sigma * sigma * q * q * inv_r2);
  }
}

// F(k) = g(k) / (-2 pi |kappa|^2) / N, and 0 at k = 0 (the inverse's 1/N folded in).
template <int RES>
__device__ __forceinline__ float spectral_F(const float* g1, int k0, float g12, float q12) {
  const float q0 = kappa_of(k0, RES);
  const float K2 = q0 * q0 + q12;
  constexpr float c = -1.0f / (6.283185307179586f * (float)RES * (float)RES * (float)RES);
  // the hardware reciprocal (1 ulp) instead of a full-precision division:
  // it is per element of the j0 passes, where VALU time is half the kernel
  return K2 == 0.0f ? 0.0f : (g1[k0] * g12 * c) * __builtin_amdgcn_rcpf(K2);
}

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

}  // namespace psr
