// gfx950 kernels of the optimisation-based reconstruction loop around the
// solver (Peng et al., "Shape As Points", main Sec. 3.2): points sampled on
// the Marching Cubes mesh (the p_mesh of Eq. 5) with their backward, the
// bidirectional Chamfer loss of Eq. 5 with its gradient, and the connected
// components of the mesh for the resampling from the largest component.
//
// Sampling: FP64 face areas, an FP64 inclusive scan (block sums, their scan,
// block-local scans), then per sample a binary search of u0 * total and the
// barycentric weights (1 - sqrt(u1), sqrt(u1) (1 - u2), sqrt(u1) u2).
// Chamfer: brute-force nearest neighbours, every query against a chunk of the
// reference cloud staged through LDS per workgroup (enough chunks that the
// grid fills the chip), the chunks' minima reduced in index order (equal
// distances go to the lower index); FP64 sums for the loss.
// Components: label propagation over the triangles (atomic minimum) with
// pointer jumping until no label changes, FP64 areas per label, and the
// label with the greatest area (ties: the lowest label).
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// nearest reference point of each query within one chunk of the references
__global__ __launch_bounds__(256) void k_nn_chunk(const float* __restrict__ q, int64_t nq, const float* __restrict__ r,
                                                  int64_t nr, int64_t chunk, float* __restrict__ pd,
                                                  int32_t* __restrict__ pi) {
  __shared__ float4 tile[256];
  const int64_t qi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t c = blockIdx.y;
  const int64_t r0 = c * chunk, r1 = r0 + chunk < nr ? r0 + chunk : nr;
  float qx = 0.0f, qy = 0.0f, qz = 0.0f;
  if (qi < nq) {
    qx = q[3 * qi];
    qy = q[3 * qi + 1];
    qz = q[3 * qi + 2];
  }
  float best = __int_as_float(0x7f800000);
  int32_t bi = -1;
  for (int64_t t0 = r0; t0 < r1; t0 += 256) {
    const int64_t j = t0 + threadIdx.x;
    __syncthreads();
    tile[threadIdx.x] = j < r1 ? make_float4(r[3 * j], r[3 * j + 1], r[3 * j + 2], 0.0f) : make_float4(0, 0, 0, 0);
    __syncthreads();
    const int n = r1 - t0 < 256 ? (int)(r1 - t0) : 256;
    for (int k = 0; k < n; ++k) {
      const float4 p = tile[k];
      const float dx = qx - p.x, dy = qy - p.y, dz = qz - p.z;
      const float d = dx * dx + dy * dy + dz * dz;
      if (d < best) {
        best = d;
        bi = (int32_t)(t0 + k);
      }
    }
  }
  if (qi < nq) {
    pd[c * nq + qi] = best;
    pi[c * nq + qi] = bi;
  }
}

__global__ __launch_bounds__(256) void k_nn_reduce(const float* __restrict__ pd, const int32_t* __restrict__ pi,
                                                   int64_t nq, int nchunks, int32_t* __restrict__ nn,
                                                   float* __restrict__ dist) {
  const int64_t qi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (qi >= nq) return;
  float best = pd[qi];
  int32_t bi = pi[qi];
  for (int c = 1; c < nchunks; ++c) {
    const float d = pd[(int64_t)c * nq + qi];
    if (d < best) {
      best = d;
      bi = pi[(int64_t)c * nq + qi];
    }
  }
  nn[qi] = bi;
  dist[qi] = best;
}

// loss = mean(d_x) + mean(d_y), FP64 sums in a fixed order (one workgroup)
__global__ __launch_bounds__(256) void k_chamfer_loss(const float* __restrict__ dx, int64_t nx,
                                                      const float* __restrict__ dy, int64_t ny,
                                                      double* __restrict__ loss) {
  __shared__ double sh[256];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < nx; i += 256) a += dx[i];
  for (int64_t i = threadIdx.x; i < ny; i += 256) b += dy[i];
  double tot;
  block_excl_scan(a / (double)nx + b / (double)ny, sh, tot);
  if (threadIdx.x == 0) *loss = tot;
}

__global__ __launch_bounds__(256) void k_chamfer_bwd_x(const float* __restrict__ x, int64_t nx,
                                                       const float* __restrict__ y, const int32_t* __restrict__ nnx,
                                                       float* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nx) return;
  const int64_t j = nnx[i];
  const float s = 2.0f / (float)nx;
#pragma unroll
  for (int d = 0; d < 3; ++d) g[3 * i + d] = s * (x[3 * i + d] - y[3 * j + d]);
}

__global__ __launch_bounds__(256) void k_chamfer_bwd_y(const float* __restrict__ x, const float* __restrict__ y,
                                                       int64_t ny, const int32_t* __restrict__ nny,
                                                       float* __restrict__ g) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= ny) return;
  const int64_t i = nny[j];
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

__global__ __launch_bounds__(256) void k_comp_area(const int32_t* __restrict__ f, int64_t nf,
                                                   const int32_t* __restrict__ lab, const double* __restrict__ area,
                                                   double* __restrict__ carea) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nf) return;
  atomicAdd(&carea[lab[f[3 * i]]], area[i]);
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

// chunks of the reference cloud per query block: enough workgroups to fill the chip
static int nn_chunks(int64_t nq, int64_t nr) {
  const int64_t qb = (nq + 255) / 256;
  int64_t c = (2048 + qb - 1) / qb;
  const int64_t maxc = (nr + 255) / 256;
  if (c > maxc) c = maxc;
  if (c < 1) c = 1;
  return (int)c;
}

NnLayout nn_layout(int64_t nq, int64_t nr) {
  NnLayout L;
  const int64_t c = nn_chunks(nq, nr);
  L.chunks = (int)c;
  L.pd = 0;
  L.pi = align(c * nq * 4);
  L.total = L.pi + align(c * nq * 4);
  return L;
}

static int run_nn(const float* q, int64_t nq, const float* r, int64_t nr, int32_t* nn, float* dist, void* ws,
                  hipStream_t s) {
  const NnLayout L = nn_layout(nq, nr);
  float* pd = reinterpret_cast<float*>(static_cast<char*>(ws) + L.pd);
  int32_t* pi = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + L.pi);
  int64_t chunk = (nr + L.chunks - 1) / L.chunks;
  chunk = (chunk + 255) / 256 * 256;
  const int nchunks = (int)((nr + chunk - 1) / chunk);
  hipLaunchKernelGGL(k_nn_chunk, dim3(nb256(nq), nchunks), dim3(256), 0, s, q, nq, r, nr, chunk, pd, pi);
  hipLaunchKernelGGL(k_nn_reduce, dim3(nb256(nq)), dim3(256), 0, s, pd, pi, nq, nchunks, nn, dist);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

size_t chamfer_ws(int64_t nx, int64_t ny) {
  const size_t a = nn_layout(nx, ny).total, b = nn_layout(ny, nx).total;
  return a > b ? a : b;
}

int run_chamfer(const float* x, int64_t nx, const float* y, int64_t ny, int32_t* nnx, float* dx, int32_t* nny,
                float* dy, double* loss, void* ws, hipStream_t s) {
  int rc = run_nn(x, nx, y, ny, nnx, dx, ws, s);  // the two directions reuse the workspace in stream order
  rc |= run_nn(y, ny, x, nx, nny, dy, ws, s);
  if (loss) hipLaunchKernelGGL(k_chamfer_loss, dim3(1), dim3(256), 0, s, dx, nx, dy, ny, loss);
  return rc || hipGetLastError() != hipSuccess ? -4 : 0;
}

int run_chamfer_backward(const float* x, int64_t nx, const float* y, int64_t ny, const int32_t* nnx,
                         const int32_t* nny, float* g, hipStream_t s) {
  hipLaunchKernelGGL(k_chamfer_bwd_x, dim3(nb256(nx)), dim3(256), 0, s, x, nx, y, nnx, g);
  hipLaunchKernelGGL(k_chamfer_bwd_y, dim3(nb256(ny)), dim3(256), 0, s, x, y, ny, nny, g);
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
