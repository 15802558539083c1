// Host/device definitions of the Marching Cubes layer: the state buffer
// layout (header, per-workgroup counts, per-vertex base indices) and the
// launch entry points.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace psr {
namespace mc {

struct McHeader {
  int64_t nv;      // mesh vertices in total (may exceed the caller's capacity)
  int64_t nt;      // triangles in total
  int32_t res;     // grid size the state was made for
  int32_t status;  // 0, or -1 when nv reaches 2^29 (vertex bases no longer fit)
  float iso;       // level the state was made for
  int32_t pad;
};

constexpr int kMcThreads = 256;                 // threads per workgroup of the sweeps
constexpr int kMcVpt = 4;                       // consecutive grid vertices (along j2) per thread
constexpr int kMcBlock = kMcThreads * kMcVpt;   // grid vertices per workgroup
constexpr int kMcGroup = 1024;                  // workgroup counts per first-level scan group

struct McState {
  McHeader* hdr;
  int2* blk;        // per workgroup of the sweeps: counts, then offsets within its scan group (vertices, triangles)
  int2* cnt;        // per workgroup of the sweeps: its counts (kept through the scan)
  int2* tops;       // per scan group: exclusive offsets
  uint32_t* vbase;  // per grid vertex with a crossing edge: first vertex index << 3 | crossing mask
};

struct McOut {
  float* verts;    // [vcap][3]
  float* normals;  // [vcap][3]
  int32_t* edges;  // [vcap] global edge id 3 j + axis, or null
  int32_t* tris;   // [tcap][3]
  int64_t vcap, tcap;
};

inline size_t mc_align(size_t x) { return (x + 255) & ~(size_t)255; }

struct McLayout {
  size_t hdr, blk, cnt, tops, vbase, total;
};

inline size_t mc_blocks(int res) { return ((size_t)res * res * res + kMcBlock - 1) / kMcBlock; }
inline size_t mc_groups(int res) { return (mc_blocks(res) + kMcGroup - 1) / kMcGroup; }

inline McLayout state_layout(int res) {
  const size_t n = (size_t)res * res * res;
  McLayout L;
  L.hdr = 0;
  L.blk = mc_align(sizeof(McHeader));
  L.cnt = L.blk + mc_align(mc_blocks(res) * sizeof(int2));
  L.tops = L.cnt + mc_align(mc_blocks(res) * sizeof(int2));
  L.vbase = L.tops + mc_align(mc_groups(res) * sizeof(int2));
  L.total = L.vbase + mc_align(n * 4);
  return L;
}

inline McState state_view(void* base, int res) {
  const McLayout L = state_layout(res);
  char* b = static_cast<char*>(base);
  McState s;
  s.hdr = reinterpret_cast<McHeader*>(b + L.hdr);
  s.blk = reinterpret_cast<int2*>(b + L.blk);
  s.cnt = reinterpret_cast<int2*>(b + L.cnt);
  s.tops = reinterpret_cast<int2*>(b + L.tops);
  s.vbase = reinterpret_cast<uint32_t*>(b + L.vbase);
  return s;
}

int run_forward(int res, const float* chi, float iso, const McState& st, const McOut& out, hipStream_t s);
int run_backward(int res, const float* chi, float iso, const McState& st, const float* normals,
                 const float* dverts, int64_t nverts, float* dchi, hipStream_t s);
void case_table(int8_t* ntri, int8_t* edge);

}  // namespace mc
}  // namespace psr
