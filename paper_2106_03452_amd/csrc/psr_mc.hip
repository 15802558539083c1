// gfx950 kernels of the Marching Cubes layer and its inverse-normal gradient
// (Peng et al., "Shape As Points", main Sec. 3.2, Eqs. 5-6; Marching Cubes
// after Lorensen and Cline 1987, case table in mc_table.h).
//
// Forward, over the r^3 grid vertices j (cells (j, j + 1) for j in
// [0, r - 2]^3; vertex j owns the grid edges from j along +axis 0, 1, 2):
//   count  per vertex: crossing edges it owns and triangles of its cell,
//          summed per workgroup (1024 vertices: 4 consecutive ones along j2
//          per thread, read as float4 rows)
//   scan   exclusive offsets of the workgroup sums, in two levels
//   emit   per vertex again, in the workgroups that hold surface only: its
//          mesh vertices (position by linear zero along the edge, normal from
//          the central-difference gradient), the base index of its vertices,
//          and its cell's triangles as global edge ids
//   link   edge ids of the triangles -> vertex indices
// Mesh vertices are numbered by global edge id 3 * j + axis, triangles by
// cell (row-major) and table order: the same order a serial sweep gives.
// The grid is read once in full (count) and again only where the surface is
// (emit): the emit pass must know where its workgroup's output starts, which
// only the scan over all workgroups gives.
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

// central-difference gradient of the periodic grid at vertex (a, b, c), in domain units
template <int R>
__device__ __forceinline__ float3 grad_at(const float* __restrict__ chi, int a, int b, int c) {
  constexpr int M = R - 1;
  auto at = [&](int x, int y, int z) { return chi[((int64_t)(x & M) * R + (y & M)) * R + (z & M)]; };
  const float h = 0.5f * (float)R;
  return make_float3((at(a + 1, b, c) - at(a - 1, b, c)) * h, (at(a, b + 1, c) - at(a, b - 1, c)) * h,
                     (at(a, b, c + 1) - at(a, b, c - 1)) * h);
}

// The kMcVpt vertices (j0, j1, j2 .. j2 + 3) of one thread: chi at the corners
// of their cells. A thread reads its own run on rows (j0, j1) and (j0 + 1, j1)
// as float4; the runs on row j1 + 1 are those of thread t + R / kMcVpt, passed
// through LDS (read from memory only where that thread is in the next
// workgroup), and the value one past the run is the next lane's first (read
// from memory only where that lane is in the next wavefront, i.e. rows longer
// than a wavefront's 256 vertices). Each grid row is so fetched about twice
// per workgroup instead of eight times.
template <int R>
struct Run {
  int j0, j1, j2;
  float v[2][2][kMcVpt + 1];  // [o0][o1][k]: chi(j0 + o0, j1 + o1, j2 + k)
  bool ok0, ok1;              // rows j0 + 1 / j1 + 1 exist

  // Called by every thread of the workgroup (it holds a workgroup barrier);
  // live: e is a grid vertex; xs: 2 * kMcThreads float4 of LDS.
  __device__ __forceinline__ void load(const float* __restrict__ chi, int64_t e, bool live, float iso,
                                       float4* xs) {
    constexpr int L = __builtin_ctz(R);
    constexpr int D = R / kMcVpt;  // threads per grid row
    constexpr int64_t S0 = (int64_t)R * R;
    j2 = (int)(e & (R - 1));
    j1 = (int)((e >> L) & (R - 1));
    j0 = (int)(e >> (2 * L));
    ok0 = live && j0 < R - 1;
    ok1 = live && j1 < R - 1;
    const int t = threadIdx.x, lane = t & 63;
    const float4 none = make_float4(iso, iso, iso, iso);
    auto ld4 = [&](int64_t i) { return *reinterpret_cast<const float4*>(chi + i); };
    float4 q[2][2];
    q[0][0] = live ? ld4(e) : none;
    q[1][0] = ok0 ? ld4(e + S0) : none;
    xs[t] = q[0][0];
    xs[kMcThreads + t] = q[1][0];
    __syncthreads();
    // thread t + D holds (j0, j1 + 1, j2) whenever j1 + 1 exists
    if (!ok1) {
      q[0][1] = none;
      q[1][1] = none;
    } else if (t + D < kMcThreads) {
      q[0][1] = xs[t + D];
      q[1][1] = xs[kMcThreads + t + D];
    } else {
      q[0][1] = ld4(e + R);
      q[1][1] = ok0 ? ld4(e + S0 + R) : none;
    }
#pragma unroll
    for (int o0 = 0; o0 < 2; ++o0)
#pragma unroll
      for (int o1 = 0; o1 < 2; ++o1) {
        v[o0][o1][0] = q[o0][o1].x;
        v[o0][o1][1] = q[o0][o1].y;
        v[o0][o1][2] = q[o0][o1].z;
        v[o0][o1][3] = q[o0][o1].w;
        // the next lane's run continues this one when j2 + kMcVpt < R; otherwise
        // the value is never read (mask and cell test j2 + k < R - 1)
        v[o0][o1][kMcVpt] = __shfl_down(q[o0][o1].x, 1, 64);
      }
    if constexpr (R > 64 * kMcVpt) {
      if (lane == 63 && live && j2 + kMcVpt < R) {
#pragma unroll
        for (int o0 = 0; o0 < 2; ++o0)
#pragma unroll
          for (int o1 = 0; o1 < 2; ++o1) {
            const bool ok = (!o0 || ok0) && (!o1 || ok1);
            v[o0][o1][kMcVpt] = ok ? chi[e + o0 * S0 + o1 * R + kMcVpt] : iso;
          }
      }
    }
  }
  // crossing mask of the three edges owned by vertex j2 + k
  __device__ __forceinline__ int mask(int k, float iso) const {
    const bool in0 = v[0][0][k] < iso;
    return (ok0 && (in0 != (v[1][0][k] < iso)) ? 1 : 0) | (ok1 && (in0 != (v[0][1][k] < iso)) ? 2 : 0) |
           (j2 + k < R - 1 && (in0 != (v[0][0][k + 1] < iso)) ? 4 : 0);
  }
  // sign pattern of the cell at j2 + k (0 when the cell does not exist)
  __device__ __forceinline__ int cell(int k, float iso) const {
    if (!ok0 || !ok1 || j2 + k >= R - 1) return 0;
    int cs = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) cs |= (v[c & 1][(c >> 1) & 1][k + (c >> 2)] < iso ? 1 : 0) << c;
    return cs;
  }
};

// inclusive prefix over a workgroup of NT threads of two counters; total too
template <int NT>
__device__ __forceinline__ int2 block_scan2(int2 v, int2* wtot, int2& total) {
  constexpr int NW = NT / 64;
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
  for (int w = 0; w < NW; ++w) {
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
__global__ __launch_bounds__(kMcThreads) void k_mc_count(const float* __restrict__ chi, float iso, McState st) {
  static_assert(kMcThreads == 256, "one table entry per thread");
  __shared__ float4 xs[2 * kMcThreads];
  __shared__ int8_t ntri[256];  // triangles per cell case, read from LDS rather than from memory
  __shared__ int wsum[kMcThreads / 64];
  ntri[threadIdx.x] = kTable.ntri[threadIdx.x];  // visible after the barrier in load
  const int64_t e = ((int64_t)blockIdx.x * kMcThreads + threadIdx.x) * kMcVpt;
  const bool live = e < (int64_t)R * R * R;
  int nv = 0, nt = 0;
  Run<R> q;
  q.load(chi, e, live, iso, xs);
  if (live) {
#pragma unroll
    for (int k = 0; k < kMcVpt; ++k) {
      nv += __popc(q.mask(k, iso));
      nt += ntri[q.cell(k, iso)];
    }
  }
  // workgroup totals, both counters in one word: at most 3 * 1024 crossing
  // edges and kMaxTri * 1024 triangles per workgroup, each below 2^16
  static_assert(3 * kMcBlock < (1 << 16) && kMaxTri * kMcBlock < (1 << 15), "packed counters");
  int sum = nv | (nt << 16);
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) sum += __shfl_down(sum, d, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int w = 0;
#pragma unroll
    for (int i = 0; i < kMcThreads / 64; ++i) w += wsum[i];
    const int2 tot = make_int2(w & 0xffff, w >> 16);
    st.blk[blockIdx.x] = tot;
    st.cnt[blockIdx.x] = tot;
  }
}

// first level: exclusive offsets of the workgroup counts within groups of
// kMcGroup, and each group's total
__global__ __launch_bounds__(kMcGroup) void k_mc_scan1(McState st, int nblocks) {
  __shared__ int2 wtot[kMcGroup / 64];
  const int i = blockIdx.x * kMcGroup + threadIdx.x;
  const int2 c = i < nblocks ? st.blk[i] : make_int2(0, 0);
  int2 tot;
  const int2 incl = block_scan2<kMcGroup>(c, wtot, tot);
  if (i < nblocks) st.blk[i] = make_int2(incl.x - c.x, incl.y - c.y);
  if (threadIdx.x == 0) st.tops[blockIdx.x] = tot;
}

// second level: exclusive offsets of the groups (one workgroup); totals to the header
__global__ __launch_bounds__(kMcGroup) void k_mc_scan2(McState st, int ngroups, int res, float iso) {
  __shared__ int2 wtot[kMcGroup / 64];
  int2 carry = make_int2(0, 0);
  for (int g0 = 0; g0 < ngroups; g0 += kMcGroup) {
    const int g = g0 + threadIdx.x;
    const int2 c = g < ngroups ? st.tops[g] : make_int2(0, 0);
    int2 tot;
    const int2 incl = block_scan2<kMcGroup>(c, wtot, tot);
    __syncthreads();  // wtot is reused by the next chunk
    if (g < ngroups) st.tops[g] = make_int2(carry.x + incl.x - c.x, carry.y + incl.y - c.y);
    carry.x += tot.x;
    carry.y += tot.y;
  }
  if (threadIdx.x == 0) {
    st.hdr->nv = carry.x;
    st.hdr->nt = carry.y;
    st.hdr->res = res;
    st.hdr->iso = iso;
    st.hdr->status = carry.x >= (1 << 29) ? -1 : 0;
  }
}

template <int R>
__global__ __launch_bounds__(kMcThreads) void k_mc_emit(const float* __restrict__ chi, float iso, McState st,
                                                        McOut out) {
  __shared__ int2 wtot[kMcThreads / 64];
  {
    // no surface in this workgroup: nothing to emit, and its part of the
    // grid is not read again (uniform over the workgroup)
    const int2 c = st.cnt[blockIdx.x];
    if (c.x == 0 && c.y == 0) return;
  }
  const int64_t e = ((int64_t)blockIdx.x * kMcThreads + threadIdx.x) * kMcVpt;
  const bool live = e < (int64_t)R * R * R;
  __shared__ float4 xs[2 * kMcThreads];
  __shared__ int8_t ntri[256];  // triangles per cell case (visible after the barrier in load)
  ntri[threadIdx.x] = kTable.ntri[threadIdx.x];
  Run<R> q;
  int m[kMcVpt], cs[kMcVpt], nv = 0, nt = 0;
  q.load(chi, e, live, iso, xs);
#pragma unroll
  for (int k = 0; k < kMcVpt; ++k) {
    m[k] = live ? q.mask(k, iso) : 0;
    cs[k] = live ? q.cell(k, iso) : 0;
    nv += __popc(m[k]);
    nt += ntri[cs[k]];
  }
  int2 tot;
  const int2 incl = block_scan2<kMcThreads>(make_int2(nv, nt), wtot, tot);
  const int2 b = st.blk[blockIdx.x], g = st.tops[blockIdx.x / kMcGroup];
  // The workgroup's mesh vertices and triangles are numbered in thread order
  // (then run position, then axis or table order); they are handed out one
  // per thread, so that a thread with many does not hold up the workgroup.
  // Each thread publishes its first indices and its masks / cell cases.
  __shared__ int pv[kMcThreads], pt[kMcThreads], pm[kMcThreads], pc[kMcThreads];
  const int t = threadIdx.x;
  pv[t] = incl.x - nv;
  pt[t] = incl.y - nt;
  pm[t] = m[0] | (m[1] << 3) | (m[2] << 6) | (m[3] << 9);
  pc[t] = cs[0] | (cs[1] << 8) | (cs[2] << 16) | (cs[3] << 24);
  {
    int v = g.x + b.x + incl.x - nv;
#pragma unroll
    for (int k = 0; k < kMcVpt; ++k) {
      if (m[k]) st.vbase[e + k] = ((uint32_t)v << 3) | (uint32_t)m[k];
      v += __popc(m[k]);
    }
  }
  __syncthreads();
  static_assert(kMcVpt == 4 && kMcThreads == 256, "masks and cases packed for 4 vertices per thread");
  // the thread whose range [p[o], p[o] + count) holds local index x: the last
  // o with p[o] <= x (threads with nothing share their successor's start)
  auto owner = [](const int* p, int x) {
    int lo = 0;
#pragma unroll
    for (int step = kMcThreads / 2; step > 0; step >>= 1)
      if (p[lo + step] <= x) lo += step;
    return lo;
  };
  const float inv_r = 1.0f / (float)R;
  constexpr int L = __builtin_ctz(R);
  const int64_t e_blk = (int64_t)blockIdx.x * kMcThreads * kMcVpt;
  for (int x = t; x < tot.x; x += kMcThreads) {
    const int v = g.x + b.x + x;
    if (v >= out.vcap) break;
    const int o = owner(pv, x);
    int r = x - pv[o], k = 0, a = 0;
    const int mo = pm[o];
    // the r-th crossing edge of the owner, in run-position then axis order
#pragma unroll
    for (int kk = 0; kk < kMcVpt; ++kk)
#pragma unroll
      for (int aa = 0; aa < 3; ++aa)
        if ((mo >> (3 * kk + aa)) & 1) {
          if (r == 0) {
            k = kk;
            a = aa;
          }
          --r;
        }
    const int64_t ek = e_blk + (int64_t)o * kMcVpt + k;
    const int j2 = (int)(ek & (R - 1)), j1 = (int)((ek >> L) & (R - 1)), j0 = (int)(ek >> (2 * L));
    const int64_t stride = a == 0 ? (int64_t)R * R : (a == 1 ? R : 1);
    const float c0 = chi[ek], cb = chi[ek + stride];
    const float tt = (c0 - iso) / (c0 - cb);
    const float3 ga = grad_at<R>(chi, j0, j1, j2);
    const float3 gb = grad_at<R>(chi, j0 + (a == 0), j1 + (a == 1), j2 + (a == 2));
    const float n0 = (1.0f - tt) * ga.x + tt * gb.x, n1 = (1.0f - tt) * ga.y + tt * gb.y,
                n2 = (1.0f - tt) * ga.z + tt * gb.z;
    const float il = rsqrtf(n0 * n0 + n1 * n1 + n2 * n2);
    out.verts[3 * (int64_t)v + 0] = ((float)j0 + (a == 0 ? tt : 0.0f)) * inv_r;
    out.verts[3 * (int64_t)v + 1] = ((float)j1 + (a == 1 ? tt : 0.0f)) * inv_r;
    out.verts[3 * (int64_t)v + 2] = ((float)j2 + (a == 2 ? tt : 0.0f)) * inv_r;
    out.normals[3 * (int64_t)v + 0] = n0 * il;
    out.normals[3 * (int64_t)v + 1] = n1 * il;
    out.normals[3 * (int64_t)v + 2] = n2 * il;
    if (out.edges) out.edges[v] = (int32_t)(3 * ek + a);
  }
  for (int x = t; x < tot.y; x += kMcThreads) {
    const int64_t tri = (int64_t)g.y + b.y + x;
    if (tri >= out.tcap) break;
    const int o = owner(pt, x);
    const int co = pc[o];
    // the cell and the table triangle of the owner's (x - pt[o])-th triangle
    int cell = 0, i = x - pt[o];
#pragma unroll
    for (int kk = 0; kk < kMcVpt - 1; ++kk) {
      const int n = ntri[(co >> (8 * kk)) & 255];
      if (cell == kk && i >= n) {
        i -= n;
        cell = kk + 1;
      }
    }
    const int csk = (co >> (8 * cell)) & 255;
    const int64_t ek = e_blk + (int64_t)o * kMcVpt + cell;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int le = kTable.edge[csk][3 * i + c];
      // owner of the edge: this vertex plus the lower corner of local edge le
      const int64_t own = ek + (int64_t)edge_lo(le, 0) * R * R + edge_lo(le, 1) * R + edge_lo(le, 2);
      out.tris[3 * tri + c] = (int32_t)(3 * own + edge_axis(le));
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

// one thread per kMcVpt consecutive grid vertices; each sums, in a fixed
// order, the contributions of the up to six crossing edges that meet there.
// A workgroup none of whose vertices, nor their lower neighbours along the
// three axes, owns a crossing edge (the forward's per-workgroup counts tell)
// writes zeros without reading chi. Elsewhere rows j1 -/+ 1 come from the
// threads R / kMcVpt before and after through LDS, and chi at j2 - 1 and
// j2 + kMcVpt from the neighbouring lanes.
template <int R>
__global__ __launch_bounds__(kMcThreads) void k_mc_backward(const float* __restrict__ chi, float iso, McState st,
                                                            const float* __restrict__ normals,
                                                            const float* __restrict__ dverts, int64_t nverts,
                                                            float* __restrict__ dchi) {
  constexpr int L = __builtin_ctz(R);
  constexpr int D = R / kMcVpt;  // threads per grid row
  static_assert(R <= kMcBlock, "a row and its predecessor lie in this and the previous workgroup");
  __shared__ float4 xs[kMcThreads];
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int64_t e = ((int64_t)b * kMcThreads + tid) * kMcVpt;
  const bool live = e < (int64_t)R * R * R;
  const int64_t s0 = (int64_t)R * R, s1 = R;
  if (st.hdr->res != R || st.hdr->iso != iso) {
    // the state comes from another grid size or level: no valid vertex map
    const float nan = __int_as_float(0x7fc00000);
    if (live) *reinterpret_cast<float4*>(dchi + e) = make_float4(nan, nan, nan, nan);
    return;
  }
  {
    // owners of the edges that end in this workgroup: its own vertices, e - 1
    // and e - R (this workgroup or the previous one), e - R^2 (the workgroup
    // R^2 vertices back, R^2 being a multiple of the workgroup's vertices or
    // below them)
    const int64_t eb = (int64_t)b * kMcBlock;
    const bool any = st.cnt[b].x != 0 || (b > 0 && st.cnt[b - 1].x != 0) ||
                     (eb >= s0 && st.cnt[(eb - s0) / kMcBlock].x != 0);
    if (!any) {
      if (live) *reinterpret_cast<float4*>(dchi + e) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      return;
    }
  }
  const int j2 = (int)(e & (R - 1)), j1 = (int)((e >> L) & (R - 1)), j0 = (int)(e >> (2 * L));
  // chi along the run (j2 - 1 .. j2 + 4) and on the four neighbouring rows
  float c[kMcVpt + 2], xm[kMcVpt], xp[kMcVpt], ym[kMcVpt], yp[kMcVpt];
  {
    const float4 none = make_float4(iso, iso, iso, iso);
    auto ld4 = [&](int64_t i) { return *reinterpret_cast<const float4*>(chi + i); };
    const float4 q = live ? ld4(e) : none;
    const float4 rxm = live && j0 > 0 ? ld4(e - s0) : none;
    const float4 rxp = live && j0 < R - 1 ? ld4(e + s0) : none;
    xs[tid] = q;
    __syncthreads();
    // threads tid -/+ D hold (j0, j1 -/+ 1, j2) whenever that row exists
    const float4 rym = !live || j1 == 0 ? none : (tid >= D ? xs[tid - D] : ld4(e - s1));
    const float4 ryp = !live || j1 == R - 1 ? none : (tid + D < kMcThreads ? xs[tid + D] : ld4(e + s1));
    const float pw = __shfl_up(q.w, 1, 64), nx = __shfl_down(q.x, 1, 64);
    c[0] = live && j2 > 0 ? (lane > 0 ? pw : chi[e - 1]) : iso;
    c[1] = q.x;
    c[2] = q.y;
    c[3] = q.z;
    c[4] = q.w;
    c[5] = live && j2 + kMcVpt < R ? (lane < 63 ? nx : chi[e + kMcVpt]) : iso;
    auto put = [](const float4& r, float* d) {
      d[0] = r.x;
      d[1] = r.y;
      d[2] = r.z;
      d[3] = r.w;
    };
    put(rxm, xm);
    put(rxp, xp);
    put(rym, ym);
    put(ryp, yp);
  }
  auto gv = [&](int64_t owner, int a) {
    const uint32_t vb = st.vbase[owner];
    const int64_t v = (int64_t)(vb >> 3) + __popc(vb & 7u & ((1u << a) - 1u));
    if (v >= nverts) return 0.0f;
    return -(dverts[3 * v] * normals[3 * v] + dverts[3 * v + 1] * normals[3 * v + 1] +
             dverts[3 * v + 2] * normals[3 * v + 2]);
  };
  if (!live) return;
  float out[kMcVpt];
#pragma unroll
  for (int k = 0; k < kMcVpt; ++k) {
    const int64_t ek = e + k;
    const float cj = c[k + 1];
    const bool inj = cj < iso;
    const int jj[3] = {j0, j1, j2 + k};
    const float up[3] = {xp[k], yp[k], c[k + 2]}, dn[3] = {xm[k], ym[k], c[k]};
    const int64_t stride[3] = {s0, s1, 1};
    float g = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (jj[a] < R - 1 && inj != (up[a] < iso)) {  // edge j -> j + e_a: weight 1 - t
        const float t = (cj - iso) / (cj - up[a]);
        g += (1.0f - t) * gv(ek, a);
      }
      if (jj[a] > 0 && (dn[a] < iso) != inj) {  // edge j - e_a -> j: weight t
        const float t = (dn[a] - iso) / (dn[a] - cj);
        g += t * gv(ek - stride[a], a);
      }
    }
    out[k] = g;
  }
  *reinterpret_cast<float4*>(dchi + e) = make_float4(out[0], out[1], out[2], out[3]);
}

template <int R>
static int forward_res(const float* chi, float iso, const McState& st, const McOut& out, hipStream_t s) {
  const int nb = (int)mc_blocks(R), ng = (int)mc_groups(R);
  hipLaunchKernelGGL(k_mc_count<R>, dim3(nb), dim3(kMcThreads), 0, s, chi, iso, st);
  hipLaunchKernelGGL(k_mc_scan1, dim3(ng), dim3(kMcGroup), 0, s, st, nb);
  hipLaunchKernelGGL(k_mc_scan2, dim3(1), dim3(kMcGroup), 0, s, st, ng, R, iso);
  hipLaunchKernelGGL(k_mc_emit<R>, dim3(nb), dim3(kMcThreads), 0, s, chi, iso, st, out);
  hipLaunchKernelGGL(k_mc_link, dim3(1024), dim3(256), 0, s, st, out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

template <int R>
static int backward_res(const float* chi, float iso, const McState& st, const float* normals, const float* dverts,
                        int64_t nverts, float* dchi, hipStream_t s) {
  const int nb = (int)mc_blocks(R);
  hipLaunchKernelGGL(k_mc_backward<R>, dim3(nb), dim3(kMcThreads), 0, s, chi, iso, st, normals, dverts, nverts,
                     dchi);
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
