// Slab-decomposed forward solve: work decomposition, workspace layout and
// kernel arguments shared by the host launch code and the kernels.
//
// The grid is cut along j0 into G slabs of s = r/G planes; slab g owns planes
// [g s, (g+1) s). The transform along j0 needs every plane, so between the
// per-slab passes the spectrum is exchanged in blocks: after the j1 pass,
// slab g holds (for its planes) every k1; the pencil owner h takes k1 in
// [h q, (h+1) q) (q = r/G) for every plane. Block (h, g) is what slab g
// sends to owner h, and owner h sends block (g, h) back after the j0 pass.
// The kernels address every block through a table of base pointers, so a
// block may live in another process's memory; here all blocks sit in one
// workspace.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "psr_internal.h"

namespace psr {

constexpr int kMaxSlabs = 64;
constexpr int kSlabMinRes = 16;
constexpr int kSlabMaxRes = 1024;  // the packed floor vertex of a point record holds 10 bits per axis

// Row passes of a slab (splat + r2c along j2, c2r along k2): slab_rows(res)
// consecutive j1 rows of one plane per workgroup, plan_TPL(res/2) threads
// per row.
__host__ __device__ constexpr int slab_rows(int res) { return imin(res, PSR_ROW_THREADS / plan_TPL(res / 2)); }
__host__ __device__ constexpr int slab_rows_block(int res) { return slab_rows(res) * plan_TPL(res / 2); }
// Column passes (FFT along j1, j0 and k1): slab_cols(res) neighbouring k2
// lines per workgroup, so every global access is a run of slab_cols(res)
// complex values (64 or 128 bytes).
__host__ __device__ constexpr int slab_cols(int res) { return res >= 512 ? 8 : 16; }
__host__ __device__ constexpr int slab_cols_block(int res) { return slab_cols(res) * plan_TPL(res); }
// Row length of the half spectrum (res/2 + 1 values) padded to whole column
// tiles; the padding columns are never read as data.
__host__ __device__ constexpr int slab_hp(int res) {
  return (res / 2 + 1 + slab_cols(res) - 1) / slab_cols(res) * slab_cols(res);
}

// Head of the slab workspace.
struct SlabHeader {
  int32_t status;
  int32_t flags;  // bit 0: a non-finite coordinate or normal was seen
  int32_t res;
  int32_t slabs;
  int64_t npoints;
  float sigma;
  float m;
  int32_t reading;
  int32_t pad;
  double chi0;  // chi'(0,0,0)
};

// What the forward reports to its caller (same layout as psr_slab_result).
struct SlabResult {
  double mu, cscale, scale, chi0;
  int32_t status, flags;
};

struct SlabLayout {
  size_t hdr, counts, off, bsum, tmp, colrank, sorted, val, red, A, X, Z, halo, total;
};

// Spectra are k2-tiled: k2 in tiles of tc = slab_cols(r) values, nt = hp / tc
// tiles, the tc values of a tile innermost, so that a column pass's tile of
// tc lines is one contiguous block (or a few long runs).
// A: the three splat channels after the row pass, A_g[c][j0 - g s][nt][j1][tc]
//    per slab (3 s r hp complex each), later the rows before the c2r pass,
//    Y_g[j0 - g s][nt][j1][tc] (s r hp each, in the first third of A_g's room);
// X: blocks (h, g), h-major: [2][s][nt][q][tc] (v~_0 and the merged channel W);
// Z: blocks (g, h), g-major: [s][nt][q][tc];
// halo: per slab, chi' of the first plane of the next slab (r r floats).
__host__ __device__ inline SlabLayout slab_layout(int res, int64_t P, int G) {
  const size_t hp = (size_t)slab_hp(res), bins = (size_t)res * res, plane = (size_t)res * hp;
  SlabLayout L;
  size_t o = 0;
  L.hdr = o;
  o += align256(sizeof(SlabHeader));
  L.counts = o;
  o += align256(bins * 4);
  L.off = o;
  o += align256((bins + 1) * 4);
  L.bsum = o;
  o += align256(1024 * 4);
  L.tmp = o;
  o += align256((size_t)P * sizeof(PointRec));
  L.colrank = o;
  o += align256((size_t)P * 8);
  L.sorted = o;
  o += align256((size_t)P * sizeof(PointRec));
  L.val = o;
  o += align256((size_t)P * 8);
  L.red = o;
  o += align256((size_t)kRedBlocks * 8);
  L.A = o;
  o += align256(3 * (size_t)res * plane * 8);
  L.X = o;
  o += align256(2 * (size_t)res * plane * 8);
  L.Z = o;
  o += align256((size_t)res * plane * 8);
  L.halo = o;
  o += align256((size_t)G * bins * 4);
  L.total = o;
  return L;
}

// Base pointers of the exchange blocks a pass reads or writes, indexed by the
// other side's slab (or owner) number.
struct BlockPtrs {
  cf* p[kMaxSlabs];
};

struct SlabArgs {
  const cf* tw;            // twiddle tables (table of length L at offset L)
  const float* pts;        // [P][3]
  const float* nrm;        // [P][3]
  const float* field;      // test hook: v [3][r][r][r] instead of the splat
  float* chi;              // [r][r][r]: chi', then chi
  SlabResult* result;      // may be null (test hook)
  SlabHeader* hdr;
  int* counts;
  int* off;
  int* bsum;
  PointRec* tmp;
  int2* colrank;
  PointRec* sorted;
  double* val;             // chi' at the points, by input index
  double* red;             // FP64 block partials of the mean
  cf* A;
  cf* X;
  cf* Z;
  float* halo;
  int64_t P;
  float sigma;
  float m;
  int reading;
  int G;
};

// Enqueue the slab forward (or, with a field, the solve of that field without
// normalisation) on x.stream. Returns 0 or -4 (launch failure).
int run_slab(Exec& x, int res, const SlabArgs& a);

}  // namespace psr
