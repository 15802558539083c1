// Device building blocks for the gfx950 FFT passes: complex arithmetic,
// register DFT codelets of size 2/4/8/16 and Stockham autosort stages that
// run on lines held in LDS.
//
// The transforms are the discrete Fourier transforms the supplement (Sec. A.2,
// FT and inverse FT) writes with e^{-2 pi i x.u} forward and e^{+2 pi i x.u}
// inverse; all transforms here are unnormalised (the 1/N of the inverse is
// folded into the spectral operator by the caller).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "psr_geometry.h"

namespace psr {


struct cf {
  float x, y;
};

__device__ __forceinline__ cf cadd(cf a, cf b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cf cmul(cf a, cf b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cf cscale(cf a, float s) { return {a.x * s, a.y * s}; }

// a * (DIR * i): DIR = -1 multiplies by -i, DIR = +1 by +i.
template <int DIR>
__device__ __forceinline__ cf mul_i(cf a) {
  return DIR < 0 ? cf{a.y, -a.x} : cf{-a.y, a.x};
}

// a * exp(DIR * 2 pi i q / 16) for a compile-time-foldable q.
template <int DIR>
__device__ __forceinline__ cf rot16(cf a, int q) {
  constexpr float C1 = 0.92387953251128674f;  // cos(pi/8)
  constexpr float S1 = 0.38268343236508978f;  // sin(pi/8)
  constexpr float HH = 0.70710678118654752f;  // cos(pi/4)
  q &= 15;
  float c, s;
  switch (q) {
    case 0: return a;
    case 4: return mul_i<DIR>(a);
    case 8: return {-a.x, -a.y};
    case 12: return mul_i<-DIR>(a);
    case 1: c = C1; s = S1; break;
    case 2: c = HH; s = HH; break;
    case 3: c = S1; s = C1; break;
    case 5: c = -S1; s = C1; break;
    case 6: c = -HH; s = HH; break;
    case 7: c = -C1; s = S1; break;
    case 9: c = -C1; s = -S1; break;
    case 10: c = -HH; s = -HH; break;
    case 11: c = -S1; s = -C1; break;
    case 13: c = S1; s = -C1; break;
    case 14: c = HH; s = -HH; break;
    default: c = C1; s = -S1; break;  // 15
  }
  s = DIR < 0 ? -s : s;
  return {a.x * c - a.y * s, a.x * s + a.y * c};
}

// In-register DFTs, natural order in and out: X[k] = sum_n a[n] exp(DIR 2 pi i nk/R).
template <int DIR>
__device__ __forceinline__ void dft2(cf* a) {
  cf t = a[0];
  a[0] = cadd(t, a[1]);
  a[1] = csub(t, a[1]);
}

template <int DIR>
__device__ __forceinline__ void dft4(cf* a) {
  cf t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
  cf t2 = cadd(a[1], a[3]), t3 = mul_i<DIR>(csub(a[1], a[3]));
  a[0] = cadd(t0, t2);
  a[2] = csub(t0, t2);
  a[1] = cadd(t1, t3);
  a[3] = csub(t1, t3);
}

// 8 = 4 x 2: n = 2 n1 + n2, k = k1 + 4 k2.
template <int DIR>
__device__ __forceinline__ void dft8(cf* a) {
  cf b0[4] = {a[0], a[2], a[4], a[6]};
  cf b1[4] = {a[1], a[3], a[5], a[7]};
  dft4<DIR>(b0);
  dft4<DIR>(b1);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cf t = rot16<DIR>(b1[k1], 2 * k1);
    a[k1] = cadd(b0[k1], t);
    a[k1 + 4] = csub(b0[k1], t);
  }
}

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2, twiddle W16^{n2 k1}.
template <int DIR>
__device__ __forceinline__ void dft16(cf* a) {
  cf b[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) b[n2][n1] = a[4 * n1 + n2];
    dft4<DIR>(b[n2]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) b[n2][k1] = rot16<DIR>(b[n2][k1], n2 * k1);
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cf c[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
    dft4<DIR>(c);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = c[k2];
  }
}

template <int R, int DIR>
__device__ __forceinline__ void dft(cf* a) {
  if constexpr (R == 2) dft2<DIR>(a);
  else if constexpr (R == 4) dft4<DIR>(a);
  else if constexpr (R == 8) dft8<DIR>(a);
  else if constexpr (R == 16) dft16<DIR>(a);
}

// LDS line layout: element i of a line lives at pidx(i) (one spare slot per
// 16 elements breaks the power-of-two strides of the Stockham writes across
// LDS banks). A line of length L needs lstride(L) slots (index L included,
// used by the r2c/c2r Nyquist slot).
__host__ __device__ constexpr int lstride(int L) { return L + L / 16 + 1; }
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }

// Canonical register layout of a line (plan_TPL(L) threads, plan_E(L)
// elements each): reg[v] holds element lt + TPL * v of the line (lt = the
// thread's index within its line). Every radix plan below reads its first
// stage from, and writes its last stage to, exactly that set.

// One Stockham autosort radix-R stage of a length-L line. Butterfly j
// (j = lt + TPL u) reads elements j + m L/R, multiplies them by the twiddles
// exp(DIR 2 pi i m k / (NS R)) with k = j mod NS (NS = product of the earlier
// radices), does a radix-R DFT and writes element (j - k) R + k + q NS.
// IN_REG: inputs come from the canonical registers (first stage only),
// otherwise from the LDS line. OUT_REG: outputs go to the canonical
// registers (last stage only), otherwise to the LDS line. A stage that reads
// LDS ends its reads with a barrier; one that writes LDS ends with a barrier.
// A first stage that writes LDS assumes the line is no longer being read.
// `tw` is the table exp(-2 pi i e / L), e in [0, L).
// WS (wavefront-synchronous): the TPL threads of a line are consecutive lanes
// of one wavefront and only they touch the line, so the barriers order the
// wavefront's own LDS accesses (in order in hardware; a fence keeps the
// compiler from moving them) instead of the workgroup's. The caller then
// synchronises the workgroup where other threads read or write the lines.
__device__ __forceinline__ void fft_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <bool WS>
__device__ __forceinline__ void fft_sync() {
  if constexpr (WS) fft_wave_sync();
  else __syncthreads();
}

template <int L, int R, int NS, int DIR, bool IN_REG, bool OUT_REG, bool WS = false>
__device__ __forceinline__ void stage(cf* reg, cf* line, int lt, const cf* __restrict__ tw, int swz) {
  constexpr int E = plan_E(L), TPL = plan_TPL(L);
  static_assert(!WS || 64 % TPL == 0, "a wavefront-synchronous line lies within one wavefront");
  constexpr int NB = E / R;
  constexpr int STRIDE = L / R;
  cf a[NB][R];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int j = lt + TPL * u;
#pragma unroll
    for (int m = 0; m < R; ++m) a[u][m] = IN_REG ? reg[u + m * NB] : line[pidx(j + m * STRIDE) ^ swz];
  }
  if constexpr (!IN_REG) fft_sync<WS>();
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int j = lt + TPL * u;
    const int k = j & (NS - 1);
    if constexpr (NS > 1) {
#pragma unroll
      for (int m = 1; m < R; ++m) {
        cf w = tw[m * k * (L / (NS * R))];
        if constexpr (DIR > 0) w.y = -w.y;
        a[u][m] = cmul(a[u][m], w);
      }
    }
    dft<R, DIR>(a[u]);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if constexpr (OUT_REG) reg[u + q * NB] = a[u][q];
      else line[pidx(base + q * NS) ^ swz] = a[u][q];
    }
  }
  if constexpr (!OUT_REG) fft_sync<WS>();
}

// Whole length-L transform. IN_REG / OUT_REG select where the first stage
// reads and the last stage writes (canonical registers or the LDS line).
template <int L, int DIR, bool IN_REG, bool OUT_REG, bool WS = false>
__device__ __forceinline__ void fft(cf* reg, cf* line, int lt, const cf* __restrict__ tw, int swz = 0) {
  if constexpr (L == 4) {
    stage<4, 4, 1, DIR, IN_REG, OUT_REG, WS>(reg, line, lt, tw, swz);
  } else if constexpr (L == 8) {
    stage<8, 8, 1, DIR, IN_REG, OUT_REG, WS>(reg, line, lt, tw, swz);
  } else if constexpr (L == 16) {
    stage<16, 16, 1, DIR, IN_REG, OUT_REG, WS>(reg, line, lt, tw, swz);
  } else if constexpr (L == 32) {
    stage<32, 8, 1, DIR, IN_REG, false, WS>(reg, line, lt, tw, swz);
    stage<32, 4, 8, DIR, false, OUT_REG, WS>(reg, line, lt, tw, swz);
  } else if constexpr (L == 64) {
    stage<64, 8, 1, DIR, IN_REG, false, WS>(reg, line, lt, tw, swz);
    stage<64, 8, 8, DIR, false, OUT_REG, WS>(reg, line, lt, tw, swz);
  } else if constexpr (L == 128) {
    stage<128, 16, 1, DIR, IN_REG, false, WS>(reg, line, lt, tw, swz);
    stage<128, 8, 16, DIR, false, OUT_REG, WS>(reg, line, lt, tw, swz);
  } else if constexpr (L == 256) {
    stage<256, 16, 1, DIR, IN_REG, false, WS>(reg, line, lt, tw, swz);
    stage<256, 16, 16, DIR, false, OUT_REG, WS>(reg, line, lt, tw, swz);
  } else if constexpr (L == 512) {
    stage<512, 8, 1, DIR, IN_REG, false, WS>(reg, line, lt, tw, swz);
    stage<512, 8, 8, DIR, false, false, WS>(reg, line, lt, tw, swz);
    stage<512, 8, 64, DIR, false, OUT_REG, WS>(reg, line, lt, tw, swz);
  } else if constexpr (L == 1024) {
    stage<1024, 16, 1, DIR, IN_REG, false, WS>(reg, line, lt, tw, swz);
    stage<1024, 16, 16, DIR, false, false, WS>(reg, line, lt, tw, swz);
    stage<1024, 4, 256, DIR, false, OUT_REG, WS>(reg, line, lt, tw, swz);
  }
}

}  // namespace psr
