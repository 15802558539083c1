// Host-side declarations of the optimisation-loop kernels (mesh sampling,
// Chamfer loss, mesh components) and their workspace layouts.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace psr {
namespace opt {

inline size_t align(int64_t x) { return ((size_t)x + 255) & ~(size_t)255; }

struct SampleLayout {
  size_t csum, bs, total;  // FP64 running face areas, FP64 scan-block sums
};
SampleLayout sample_layout(int64_t nfaces);

// Chamfer workspace: per cloud (x, y) the cell counts / offsets of the
// counting sort, the sorted points (x, y, z, original index bits) and the
// bounding box of every tile of kNnTile sorted points.
constexpr int kNnTile = 64;  // sorted points per tile
// 2^b cells per axis (Morton-ordered): about four or more points per cell
inline int nn_cell_bits(int64_t nx, int64_t ny) {
  const int64_t n = nx > ny ? nx : ny;
  return n <= 32768 ? 4 : (n <= 262144 ? 5 : 6);
}
struct NnLayout {
  int cell_bits;
  size_t cnt, srt_x, srt_y, box_x, box_y, total;
};
NnLayout nn_layout(int64_t nx, int64_t ny);
size_t chamfer_ws(int64_t nx, int64_t ny);

struct CompLayout {
  size_t flag, best, carea, area, total;
};
CompLayout comp_layout(int64_t nverts, int64_t nfaces);

int run_sample(const float* v, const float* vn, const int32_t* f, int64_t nf, const float* w, const float* u,
               int64_t m, float* pts, float* nrm, int32_t* face, float* bary, void* ws, hipStream_t s);
int run_sample_backward(const int32_t* f, int64_t nv, const int32_t* face, const float* bary, const float* dp,
                        int64_t m, float* dv, hipStream_t s);
int run_chamfer(const float* x, int64_t nx, const float* y, int64_t ny, int32_t* nnx, float* dx, int32_t* nny,
                float* dy, double* loss, void* ws, hipStream_t s);
int run_chamfer_backward(const float* x, int64_t nx, const float* y, int64_t ny, const int32_t* nnx,
                         const int32_t* nny, float* g, hipStream_t s);
// Adam on n values (moments m, v in place), then p -= floor(p) when wrap
int run_adam(float* p, float* m, float* v, const float* g, int64_t n, int64_t t, float lr, float b1, float b2,
             float eps, bool wrap, hipStream_t s);
int run_components(const float* v, int64_t nv, const int32_t* f, int64_t nf, int32_t* lab, float* w, void* ws,
                   hipStream_t s, int max_iters);

}  // namespace opt
}  // namespace psr
