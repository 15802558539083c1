// Shared host/device definitions of the solver library: per-solve state
// layouts, workspace layout and the launch context.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "psr_geometry.h"

namespace psr {

struct cf;

// Sorted point record (32 bytes): fractional cell offsets f, packed floor
// vertex b (10 bits per axis), normal n, original index.
struct __align__(16) PointRec {
  float f0, f1, f2;
  uint32_t b;
  float n0, n1, n2;
  uint32_t idx;
};

// Head of the `saved` buffer: the forward's status and FP64 scalars.
struct SavedHeader {
  int32_t status;   // PSR_OK / PSR_EDEGENERATE / PSR_ENONFINITE
  int32_t flags;    // bit 0: a non-finite coordinate was seen
  int32_t res;
  int32_t reading;  // 0 = B, 1 = A
  int64_t npoints;
  float sigma;
  float m;
  double mu;        // mean of chi' at the points
  double cscale;    // c (reading B: chi'(0) - mu; reading A: chi'(0))
  double scale;     // m / |c|
  double chi0;      // chi'(0,0,0)
  uint32_t live[16];  // bit j0: some point's corners reach plane j0 (j0 < 512)
  // bit j0 * row_tiles(res) + tb: some point's corners reach row tile tb of
  // plane j0 (res * row_tiles(res) <= 8192)
  uint32_t tlive[256];
};

// Backward scalars computed on the device from the FP64 reductions.
struct BwdScalars {
  double S_G, S_Gchi, Qd, gmu;
  float s, q, alpha, pad;
};

enum Stage {
  STAGE_BIN = 0,
  STAGE_P1,
  STAGE_P2,
  STAGE_P3,
  STAGE_P4,
  STAGE_P5,
  STAGE_FWD_REDUCE,
  STAGE_NORMALIZE,
  STAGE_BWD_REDUCE,
  STAGE_B1,
  STAGE_B2,
  STAGE_B3,
  STAGE_B4,
  STAGE_B5,
  STAGE_BWD_FINAL,
  STAGE_P12,  // plane pass: P1 + P2 in one kernel
  STAGE_P45,  // plane pass: P4 + P5
  STAGE_B12,  // plane pass: B1 + B2
  STAGE_B45,  // plane pass: B4 + B5
  STAGE_B1A,  // two-pass path: backward reductions + r2c of point-free row tiles
  STAGE_SLAB_BIN,     // slab solve: binning by floor plane and row
  STAGE_S1,           // slab solve: splat + r2c along j2, per slab
  STAGE_S2,           // slab solve: FFT along j1, per slab, into the exchange blocks
  STAGE_S3,           // slab solve: j0 pencils, spectral operator, per owner
  STAGE_S4,           // slab solve: inverse FFT along k1, per slab
  STAGE_S5,           // slab solve: c2r along k2 + halo plane, per slab
  STAGE_SLAB_GATHER,  // slab solve: gather at the points + FP64 mean
  STAGE_SLAB_NORM,    // slab solve: normalisation, per slab
  NUM_STAGES
};

constexpr int kRedBlocks = 1024;  // fixed block count of the FP64 reductions (deterministic order)

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
  size_t bs, blockpart, X, Y, counts, tmp, colrank, part, total;
};

__host__ __device__ inline WsLayout ws_layout(int res, int64_t P) {
  const size_t H = (size_t)res / 2 + 1;
  const size_t spec = 3 * H * (size_t)res * (size_t)res * 8;
  WsLayout L;
  size_t o = 0;
  L.bs = o;
  o += align256(sizeof(BwdScalars));
  L.blockpart = o;
  {
    // FP64 block partials: the grid-stride reductions (kRedBlocks) or one
    // per row tile of the backward's first row pass
    const size_t tiles = (size_t)res * (size_t)row_tiles(res);
    o += align256((tiles > (size_t)kRedBlocks ? tiles : (size_t)kRedBlocks) * 16);
  }
  L.X = o;
  o += align256(spec);
  L.Y = o;
  o += align256(spec);
  L.counts = o;
  o += align256((size_t)num_bins(res) * 4);
  L.tmp = o;
  o += align256((size_t)P * sizeof(PointRec));
  L.colrank = o;
  o += align256((size_t)P * 8);
  L.part = o;
  o += align256((size_t)P * 4 * 3 * 16);  // per point, corner line and channel: 4 floats
  L.total = o;
  return L;
}

struct SavedLayout {
  size_t hdr, off, sorted, gradf, total;
};

__host__ __device__ inline SavedLayout saved_layout(int res, int64_t P) {
  SavedLayout L;
  size_t o = 0;
  L.hdr = o;
  o += align256(sizeof(SavedHeader));
  L.off = o;
  o += align256(((size_t)num_bins(res) + 1) * 4);
  L.sorted = o;
  o += align256((size_t)P * sizeof(PointRec));
  L.gradf = o;
  o += align256((size_t)P * 16);
  L.total = o;
  return L;
}

struct WsView {
  cf* X;
  cf* Y;
  int* counts;
  PointRec* tmp;
  int2* colrank;
  float4* part;
  double* blockpart;
  BwdScalars* bs;
};

struct SavedView {
  SavedHeader* hdr;
  int* off;
  PointRec* sorted;
  float4* gradf;
};

__host__ __device__ inline WsView ws_view(void* base, const WsLayout& L) {
  char* b = static_cast<char*>(base);
  WsView w;
  w.X = reinterpret_cast<cf*>(b + L.X);
  w.Y = reinterpret_cast<cf*>(b + L.Y);
  w.counts = reinterpret_cast<int*>(b + L.counts);
  w.tmp = reinterpret_cast<PointRec*>(b + L.tmp);
  w.colrank = reinterpret_cast<int2*>(b + L.colrank);
  w.part = reinterpret_cast<float4*>(b + L.part);
  w.blockpart = reinterpret_cast<double*>(b + L.blockpart);
  w.bs = reinterpret_cast<BwdScalars*>(b + L.bs);
  return w;
}

__host__ __device__ inline SavedView saved_view(void* base, const SavedLayout& L) {
  char* b = static_cast<char*>(base);
  SavedView s;
  s.hdr = reinterpret_cast<SavedHeader*>(b + L.hdr);
  s.off = reinterpret_cast<int*>(b + L.off);
  s.sorted = reinterpret_cast<PointRec*>(b + L.sorted);
  s.gradf = reinterpret_cast<float4*>(b + L.gradf);
  return s;
}

// One solve as the kernels see it (passed by value inside a Batch).
struct JobArg {
  const float* pts;
  const float* nrm;
  float* chi;
  const float* dchi;
  float* dpts;
  float* dnrm;
  void* ws;
  void* sv;
  const float* aux_in;  // test hooks: field v in
  float* aux_out;       // test hooks: field v out
  const float* ktab;    // backward: point-source table of (res, sigma)
  int64_t P;
  float sigma;
  int pad;
};

// Up to MAXJ solves of one resolution in one launch: workgroups
// [start[j], start[j+1]) belong to job j.
template <int MAXJ>
struct Batch {
  const cf* tw;
  float m;
  int reading;
  int n;
  int start[MAXJ + 1];
  JobArg job[MAXJ];
};

constexpr int kMaxJobs = 24;  // jobs per batched launch (kernel argument stays under 4 KiB)

struct Timers;
void timer_begin(Timers* t, int stage, hipStream_t s);
void timer_end(Timers* t, int stage, hipStream_t s);

// Everything a launch sequence needs besides its buffers.
struct Exec {
  hipStream_t stream;
  const cf* tw;  // twiddle tables: table of length L at offset L
  double m;
  int reading;
  Timers* timers;  // null when timing is off
  void begin(int st) {
    if (timers) timer_begin(timers, st, stream);
  }
  void end(int st) {
    if (timers) timer_end(timers, st, stream);
  }
};

enum RunWhat { RUN_FORWARD = 1, RUN_BACKWARD = 2 };

// Point-source table of the backward (see build_point_source_table): floats
// on the octant [0, res/2]^3, and the FP64 scratch its build needs.
__host__ __device__ inline size_t ktab_floats(int res) {
  const size_t h = (size_t)res / 2 + 1;
  return h * h * h;
}
__host__ __device__ inline size_t ktab_scratch_bytes(int res) {
  const size_t h = (size_t)res / 2 + 1;
  return 2 * align256(h * h * h * 8) + 2 * align256(h * h * 8);
}
// Build the table of (res, sigma) into `table` (ktab_floats(res) floats) with
// `scratch` (ktab_scratch_bytes(res) bytes) as FP64 temporaries; enqueued on
// `stream`. Returns 0 or -4 (launch failure).
int build_point_source_table(int res, float sigma, float* table, void* scratch, hipStream_t stream);

// The allocation-free forward (psr_forward_static) carves its workspace and
// saved state out of one static device array of this size per GPU.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
// Device address of that array on the current device (hipGetSymbolAddress);
// 0 on success, -4 on failure.
int static_scratch_address(void** out);

// Run forward and/or backward for n jobs of one resolution.
int run_jobs(Exec& x, int res, const JobArg* jobs, int n, int what);
int run_debug_spectral(Exec& x, int res, const JobArg& job);
int run_debug_splat(Exec& x, int res, const JobArg& job);

}  // namespace psr
