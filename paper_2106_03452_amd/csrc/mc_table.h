// Marching Cubes case table (Lorensen and Cline, SIGGRAPH 1987), generated
// by the compiler from the rule below rather than typed in.
//
// Cell corner k sits at offset (k & 1, (k >> 1) & 1, (k >> 2) & 1) along grid
// axes (0, 1, 2); bit k of a case is set when corner k is inside (chi < iso).
// Edge 4a + u + 2v runs along axis a from the corner whose other two
// coordinates, in increasing axis order, are (u, v). An edge carries a mesh
// vertex when exactly one of its corners is inside.
//
// Per cell face: two crossing edges are joined by one segment; four crossing
// edges (inside corners on a diagonal) are joined so that each inside corner
// is cut off on its own (neighbouring cells see the same face signs and cut
// it the same way, so the mesh is closed). A segment is directed so that,
// seen from outside the cell, the inside corner lies to its right. The
// directed segments chain into loops, each started at its smallest edge id;
// a loop is split into a fan from the first of its vertices whose diagonals
// all cross the cell's interior (a diagonal within a face could be drawn by
// the neighbouring cell too). The triangles then run counter-clockwise seen
// from the outside (the chi > iso side).
#pragma once
#include <stdint.h>

namespace psr {
namespace mc {

constexpr int kMaxTri = 5;  // at most 5 triangles per cell under this rule (static_assert below)

struct Table {
  int8_t ntri[256];
  int8_t edge[256][kMaxTri * 3];
};

constexpr int corner_coord(int k, int a) { return (k >> a) & 1; }

// axis of edge e and the coordinate of its lower corner along axis b
constexpr int edge_axis(int e) { return e / 4; }
constexpr int edge_lo(int e, int b) {
  const int a = e / 4, uv = e % 4;
  if (b == a) return 0;
  const int first = a == 0 ? 1 : 0;  // the lower-numbered of the other two axes
  return b == first ? (uv & 1) : ((uv >> 1) & 1);
}
constexpr int edge_corner(int e, int hi) {
  int k = 0;
  for (int b = 0; b < 3; ++b) k |= (b == edge_axis(e) ? hi : edge_lo(e, b)) << b;
  return k;
}
// edge e lies on face (b, side) when b is not its axis and its lower corner has coordinate side along b
constexpr bool edge_on_face(int e, int b, int side) { return edge_axis(e) != b && edge_lo(e, b) == side; }
constexpr bool edges_share_face(int e1, int e2) {
  for (int b = 0; b < 3; ++b)
    for (int side = 0; side < 2; ++side)
      if (edge_on_face(e1, b, side) && edge_on_face(e2, b, side)) return true;
  return false;
}

constexpr Table build() {
  Table T{};
  for (int cs = 0; cs < 256; ++cs) {
    bool in[8] = {};
    for (int k = 0; k < 8; ++k) in[k] = (cs >> k) & 1;
    bool cross[12] = {};
    for (int e = 0; e < 12; ++e) cross[e] = in[edge_corner(e, 0)] != in[edge_corner(e, 1)];
    int next[12] = {};
    for (int e = 0; e < 12; ++e) next[e] = -1;
    for (int a = 0; a < 3; ++a) {
      for (int side = 0; side < 2; ++side) {
        int fe[4] = {}, nf = 0, ce[4] = {}, nc = 0;
        for (int e = 0; e < 12; ++e)
          if (edge_on_face(e, a, side)) {
            fe[nf++] = e;
            if (cross[e]) ce[nc++] = e;
          }
        // segments (e1, e2, inside corner q) of this face
        int seg[2][3] = {}, ns = 0;
        if (nc == 2) {
          int q = -1;
          for (int k = 0; k < 8 && q < 0; ++k)
            if (corner_coord(k, a) == side && in[k]) q = k;
          seg[0][0] = ce[0];
          seg[0][1] = ce[1];
          seg[0][2] = q;
          ns = 1;
        } else if (nc == 4) {
          for (int k = 0; k < 8; ++k) {
            if (corner_coord(k, a) != side || !in[k]) continue;
            int adj[2] = {}, na = 0;
            for (int i = 0; i < 4; ++i)
              if (edge_corner(fe[i], 0) == k || edge_corner(fe[i], 1) == k) adj[na++] = fe[i];
            seg[ns][0] = adj[0];
            seg[ns][1] = adj[1];
            seg[ns][2] = k;
            ++ns;
          }
        }
        for (int i = 0; i < ns; ++i) {
          int e1 = seg[i][0], e2 = seg[i][1];
          const int q = seg[i][2];
          // doubled coordinates: edge midpoints and the corner are integers
          int A[3] = {}, B[3] = {}, Q[3] = {};
          for (int b = 0; b < 3; ++b) {
            A[b] = b == edge_axis(e1) ? 1 : 2 * edge_lo(e1, b);
            B[b] = b == edge_axis(e2) ? 1 : 2 * edge_lo(e2, b);
            Q[b] = 2 * corner_coord(q, b);
          }
          const int u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
          const int v[3] = {Q[0] - A[0], Q[1] - A[1], Q[2] - A[2]};
          const int cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
          // outward face normal is (2 side - 1) along a; the corner must lie to the right
          if (cr[a] * (2 * side - 1) > 0) {
            const int tmp = e1;
            e1 = e2;
            e2 = tmp;
          }
          next[e1] = e2;
        }
      }
    }
    bool seen[12] = {};
    int nt = 0;
    for (int e0 = 0; e0 < 12; ++e0) {
      if (next[e0] < 0 || seen[e0]) continue;
      int loop[12] = {}, n = 0;
      for (int e = e0; !seen[e]; e = next[e]) {
        seen[e] = true;
        loop[n++] = e;
      }
      int s = 0;
      for (; s < n; ++s) {
        bool ok = true;
        for (int i = 0; i < n; ++i) {
          if (i == s || i == (s + 1) % n || i == (s + n - 1) % n) continue;
          if (edges_share_face(loop[s], loop[i])) ok = false;
        }
        if (ok) break;
      }
      if (s == n) {  // no interior apex (never happens under this rule; fits() rejects it)
        T.ntri[cs] = -1;
        break;
      }
      for (int i = 1; i + 1 < n; ++i) {
        T.edge[cs][3 * nt + 0] = (int8_t)loop[s];
        T.edge[cs][3 * nt + 1] = (int8_t)loop[(s + i) % n];
        T.edge[cs][3 * nt + 2] = (int8_t)loop[(s + i + 1) % n];
        ++nt;
      }
    }
    if (T.ntri[cs] == 0) T.ntri[cs] = (int8_t)nt;
  }
  return T;
}

constexpr Table kTable = build();

constexpr bool fits() {
  for (int c = 0; c < 256; ++c)
    if (kTable.ntri[c] > kMaxTri || kTable.ntri[c] < 0) return false;
  return true;
}
static_assert(fits(), "a cell with more than kMaxTri triangles or without an interior fan apex");

}  // namespace mc
}  // namespace psr
