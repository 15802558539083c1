// gfx950 kernels of the Marching Cubes layer and its inverse-normal gradient
// (Peng et al., "Shape As Points", main Sec. 3.2, Eqs. 5-6; Marching Cubes
// after Lorensen and Cline 1987, case table in mc_table.h).
//
// Forward, over the r^3 grid vertices j (cells (j, j + 1) for j in
// [0, r - 2]^3; vertex j owns the grid edges from j along +axis 0, 1, 2):
//   count  per vertex: crossing edges it owns and triangles of its cell,
//          summed per 256-vertex workgroup
//   scan   exclusive offsets of the workgroup sums (one workgroup)
//   emit   per vertex again: its mesh vertices (position by linear zero along
//          the edge, normal from the central-difference gradient), the base
//          index of its vertices, and its cell's triangles as global edge ids
//   link   edge ids of the triangles -> vertex indices
// Mesh vertices are numbered by global edge id 3 * j + axis, triangles by
// cell (row-major) and table order: the same order a serial sweep gives.
// The grid is read twice (count and emit): the emit pass must know where its
// workgroup's output starts, which only the scan over all workgroups gives.
//
// Backward (main Eq. 6): dp/dchi = -n, spread onto the two ends of each
// vertex's edge with its interpolation weights (1 - t, t); one thread per
// grid vertex sums the contributions of the up to six edges that meet there
// in a fixed order, so the result is deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mc_table.h"
#include "psr_mc.h"

namespace psr {
namespace mc {

__device__ __forceinline__ float ld(const float* __restrict__ chi, int64_t i) { return chi[i]; }

// central-difference gradient of the periodic grid at vertex (a, b, c), in domain units
template <int R>
__device__ __forceinline__ float3 grad_at(const float* __restrict__ chi, int a, int b, int c) {
  constexpr int M = R - 1;
  auto at = [&](int x, int y, int z) { return ld(chi, ((int64_t)(x & M) * R + (y & M)) * R + (z & M)); };
  const float h = 0.5f * (float)R;
  return make_float3((at(a + 1, b, c) - at(a - 1, b, c)) * h, (at(a, b + 1, c) - at(a, b - 1, c)) * h,
                     (at(a, b, c + 1) - at(a, b, c - 1)) * h);
}

struct Cell {
  int j0, j1, j2;
  int mask;  // bit a: the edge from j along axis a crosses the level
  int cs;    // sign pattern of the cell at j (0 when the cell does not exist)
  float c0;  // chi at j
  float ce[3];  // chi at j + e_a
};

template <int R>
__device__ __forceinline__ Cell classify(const float* __restrict__ chi, int64_t e, float iso) {
  constexpr int L = __builtin_ctz(R);
  Cell q;
  q.j2 = (int)(e & (R - 1));
  q.j1 = (int)((e >> L) & (R - 1));
  q.j0 = (int)(e >> (2 * L));
  const bool v0 = q.j0 < R - 1, v1 = q.j1 < R - 1, v2 = q.j2 < R - 1;
  float c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int o0 = k & 1, o1 = (k >> 1) & 1, o2 = k >> 2;
    const bool ok = (!o0 || v0) && (!o1 || v1) && (!o2 || v2);
    c[k] = ok ? ld(chi, e + (int64_t)o0 * R * R + o1 * R + o2) : iso;
  }
  q.c0 = c[0];
  q.ce[0] = c[1];
  q.ce[1] = c[2];
  q.ce[2] = c[4];
  const bool in0 = c[0] < iso;
  q.mask = (v0 && (in0 != (c[1] < iso)) ? 1 : 0) | (v1 && (in0 != (c[2] < iso)) ? 2 : 0) |
           (v2 && (in0 != (c[4] < iso)) ? 4 : 0);
  int cs = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) cs |= (c[k] < iso ? 1 : 0) << k;
  q.cs = (v0 && v1 && v2) ? cs : 0;
  return q;
}

// inclusive prefix over a 256-thread workgroup of two counters
__device__ __forceinline__ int2 block_scan2(int2 v, int2* wtot, int2& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int x = __shfl_up(v.x, d, 64), y = __shfl_up(v.y, d, 64);
    if (lane >= d) {
      v.x += x;
      v.y += y;
    }
  }
  if (lane == 63) wtot[wid] = v;
  __syncthreads();
  int2 base = make_int2(0, 0);
  total = make_int2(0, 0);
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    if (w < wid) {
      base.x += wtot[w].x;
      base.y += wtot[w].y;
    }
    total.x += wtot[w].x;
    total.y += wtot[w].y;
  }
  return make_int2(v.x + base.x, v.y + base.y);
}

template <int R>
__global__ __launch_bounds__(256) void k_mc_count(const float* __restrict__ chi, float iso, McState st) {
  __shared__ int8_t ntri[256];
  __shared__ int2 wtot[4];
  ntri[threadIdx.x] = kTable.ntri[threadIdx.x];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const Cell q = classify<R>(chi, e, iso);
  int2 tot;
  block_scan2(make_int2(__popc(q.mask), ntri[q.cs]), wtot, tot);
  if (threadIdx.x == 0) st.blk[blockIdx.x] = tot;
}

// Exclusive offsets of the per-workgroup counts, in place; the totals and
// the grid size go to the header.
__global__ __launch_bounds__(1024) void k_mc_scan(McState st, int nblocks, int res, float iso) {
  __shared__ int2 wtot[16];
  const int t = threadIdx.x, per = (nblocks + 1023) / 1024;
  const int lo = t * per, hi = lo + per < nblocks ? lo + per : nblocks;
  int2 s = make_int2(0, 0);
  for (int i = lo; i < hi; ++i) {
    s.x += st.blk[i].x;
    s.y += st.blk[i].y;
  }
  const int lane = t & 63, wid = t >> 6;
  int2 v = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int x = __shfl_up(v.x, d, 64), y = __shfl_up(v.y, d, 64);
    if (lane >= d) {
      v.x += x;
      v.y += y;
    }
  }
  if (lane == 63) wtot[wid] = v;
  __syncthreads();
  int2 base = make_int2(0, 0), total = make_int2(0, 0);
  for (int w = 0; w < 16; ++w) {
    if (w < wid) {
      base.x += wtot[w].x;
      base.y += wtot[w].y;
    }
    total.x += wtot[w].x;
    total.y += wtot[w].y;
  }
  int2 run = make_int2(base.x + v.x - s.x, base.y + v.y - s.y);  // exclusive start of this thread's chunk
  for (int i = lo; i < hi; ++i) {
    const int2 c = st.blk[i];
    st.blk[i] = run;
    run.x += c.x;
    run.y += c.y;
  }
  if (t == 0) {
    st.hdr->nv = total.x;
    st.hdr->nt = total.y;
    st.hdr->res = res;
    st.hdr->iso = iso;
    st.hdr->status = total.x >= (1 << 29) ? -1 : 0;
  }
}

template <int R>
__global__ __launch_bounds__(256) void k_mc_emit(const float* __restrict__ chi, float iso, McState st, McOut out) {
  __shared__ int8_t ntri[256];
  __shared__ int8_t edges[256][kMaxTri * 3];
  __shared__ int2 wtot[4];
  ntri[threadIdx.x] = kTable.ntri[threadIdx.x];
  for (int i = 0; i < kMaxTri * 3; ++i) edges[threadIdx.x][i] = kTable.edge[threadIdx.x][i];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const Cell q = classify<R>(chi, e, iso);
  const int nv = __popc(q.mask), nt = ntri[q.cs];
  int2 tot;
  const int2 incl = block_scan2(make_int2(nv, nt), wtot, tot);
  const int2 b = st.blk[blockIdx.x];
  const int vo = b.x + incl.x - nv, to = b.y + incl.y - nt;
  if (q.mask) st.vbase[e] = ((uint32_t)vo << 3) | (uint32_t)q.mask;
  const float inv_r = 1.0f / (float)R;
  int v = vo;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!((q.mask >> a) & 1)) continue;
    if (v < out.vcap) {
      const float t = (q.c0 - iso) / (q.c0 - q.ce[a]);
      const float p0 = ((float)q.j0 + (a == 0 ? t : 0.0f)) * inv_r;
      const float p1 = ((float)q.j1 + (a == 1 ? t : 0.0f)) * inv_r;
      const float p2 = ((float)q.j2 + (a == 2 ? t : 0.0f)) * inv_r;
      const float3 ga = grad_at<R>(chi, q.j0, q.j1, q.j2);
      const float3 gb = grad_at<R>(chi, q.j0 + (a == 0), q.j1 + (a == 1), q.j2 + (a == 2));
      float n0 = (1.0f - t) * ga.x + t * gb.x, n1 = (1.0f - t) * ga.y + t * gb.y, n2 = (1.0f - t) * ga.z + t * gb.z;
      const float il = rsqrtf(n0 * n0 + n1 * n1 + n2 * n2);
      n0 *= il;
      n1 *= il;
      n2 *= il;
      out.verts[3 * (int64_t)v + 0] = p0;
      out.verts[3 * (int64_t)v + 1] = p1;
      out.verts[3 * (int64_t)v + 2] = p2;
      out.normals[3 * (int64_t)v + 0] = n0;
      out.normals[3 * (int64_t)v + 1] = n1;
      out.normals[3 * (int64_t)v + 2] = n2;
      if (out.edges) out.edges[v] = (int32_t)(3 * e + a);
    }
    ++v;
  }
  for (int i = 0; i < nt; ++i) {
    const int64_t tri = (int64_t)to + i;
    if (tri >= out.tcap) break;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int le = edges[q.cs][3 * i + m];
      const int a = edge_axis(le);
      // owner of the edge: j plus the lower corner of local edge le
      const int64_t owner = e + (int64_t)edge_lo(le, 0) * R * R + edge_lo(le, 1) * R + edge_lo(le, 2);
      out.tris[3 * tri + m] = (int32_t)(3 * owner + a);
    }
  }
}

// triangle corners: global edge id -> vertex index (base of the owner + rank
// of the axis among the owner's crossing edges)
__global__ __launch_bounds__(256) void k_mc_link(McState st, McOut out) {
  const int64_t nt = st.hdr->nt < out.tcap ? st.hdr->nt : out.tcap;
  const int64_t n = 3 * nt;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int32_t ge = out.tris[i];
    const int64_t j = ge / 3;
    const int a = ge - 3 * (int32_t)j;
    const uint32_t vb = st.vbase[j];
    out.tris[i] = (int32_t)((vb >> 3) + __popc(vb & 7u & ((1u << a) - 1u)));
  }
}

template <int R>
__global__ __launch_bounds__(256) void k_mc_backward(const float* __restrict__ chi, float iso, McState st,
                                                     const float* __restrict__ normals,
                                                     const float* __restrict__ dverts, int64_t nverts,
                                                     float* __restrict__ dchi) {
  constexpr int L = __builtin_ctz(R);
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (st.hdr->res != R || st.hdr->iso != iso) {
    // the state comes from another grid size or level: no valid vertex map
    dchi[e] = __int_as_float(0x7fc00000);
    return;
  }
  const int j[3] = {(int)(e >> (2 * L)), (int)((e >> L) & (R - 1)), (int)(e & (R - 1))};
  const int64_t stride[3] = {(int64_t)R * R, R, 1};
  const float cj = chi[e];
  const bool inj = cj < iso;
  float g = 0.0f;
  // -(dL/dp . n) of the vertex on edge (owner, a), 0 beyond nverts
  auto gv = [&](int64_t owner, int a) {
    const uint32_t vb = st.vbase[owner];
    const int64_t v = (int64_t)(vb >> 3) + __popc(vb & 7u & ((1u << a) - 1u));
    if (v >= nverts) return 0.0f;
    return -(dverts[3 * v] * normals[3 * v] + dverts[3 * v + 1] * normals[3 * v + 1] +
             dverts[3 * v + 2] * normals[3 * v + 2]);
  };
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (j[a] < R - 1) {  // the edge j -> j + e_a: this vertex is its lower end, weight 1 - t
      const float cb = chi[e + stride[a]];
      if (inj != (cb < iso)) {
        const float t = (cj - iso) / (cj - cb);
        g += (1.0f - t) * gv(e, a);
      }
    }
    if (j[a] > 0) {  // the edge j - e_a -> j: this vertex is its upper end, weight t
      const float ca = chi[e - stride[a]];
      if ((ca < iso) != inj) {
        const float t = (ca - iso) / (ca - cj);
        g += t * gv(e - stride[a], a);
      }
    }
  }
  dchi[e] = g;
}

template <int R>
static int forward_res(const float* chi, float iso, const McState& st, const McOut& out, hipStream_t s) {
  const int nb = (int)((int64_t)R * R * R / 256);
  hipLaunchKernelGGL(k_mc_count<R>, dim3(nb), dim3(256), 0, s, chi, iso, st);
  hipLaunchKernelGGL(k_mc_scan, dim3(1), dim3(1024), 0, s, st, nb, R, iso);
  hipLaunchKernelGGL(k_mc_emit<R>, dim3(nb), dim3(256), 0, s, chi, iso, st, out);
  hipLaunchKernelGGL(k_mc_link, dim3(1024), dim3(256), 0, s, st, out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

template <int R>
static int backward_res(const float* chi, float iso, const McState& st, const float* normals, const float* dverts,
                        int64_t nverts, float* dchi, hipStream_t s) {
  const int nb = (int)((int64_t)R * R * R / 256);
  hipLaunchKernelGGL(k_mc_backward<R>, dim3(nb), dim3(256), 0, s, chi, iso, st, normals, dverts, nverts, dchi);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

#define PSR_MC_DISPATCH(res, call) \
  switch (res) {                   \
    case 8: return call(8);        \
    case 16: return call(16);      \
    case 32: return call(32);      \
    case 64: return call(64);      \
    case 128: return call(128);    \
    case 256: return call(256);    \
    case 512: return call(512);    \
    default: return -1;            \
  }

int run_forward(int res, const float* chi, float iso, const McState& st, const McOut& out, hipStream_t s) {
#define CALL(R) forward_res<R>(chi, iso, st, out, s)
  PSR_MC_DISPATCH(res, CALL)
#undef CALL
}

int run_backward(int res, const float* chi, float iso, const McState& st, const float* normals,
                 const float* dverts, int64_t nverts, float* dchi, hipStream_t s) {
#define CALL(R) backward_res<R>(chi, iso, st, normals, dverts, nverts, dchi, s)
  PSR_MC_DISPATCH(res, CALL)
#undef CALL
}

void case_table(int8_t* ntri, int8_t* edge) {
  for (int c = 0; c < 256; ++c) {
    if (ntri) ntri[c] = kTable.ntri[c];
    if (edge)
      for (int i = 0; i < kMaxTri * 3; ++i) edge[c * kMaxTri * 3 + i] = kTable.edge[c][i];
  }
}

}  // namespace mc
}  // namespace psr
