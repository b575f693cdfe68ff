// Host-side layout of a mesh for the LDS-tiled element-by-element kernels.
//
// 1. Elements are ordered along a Morton (Z-order) curve of their centroids,
//    which groups spatial neighbours whatever the input numbering.
// 2. Consecutive elements form tiles, closed when the next element would
//    exceed TILE_MAX_NODES distinct nodes or TILE_MAX_ELEMS elements, so a
//    tile's node values and accumulators fit in one workgroup's LDS.
// 3. Nodes are renumbered: every tile's interior nodes (touched by no other
//    tile), tile by tile, then all shared nodes in the order tiles first
//    touch them.  A tile's interior nodes are thus one contiguous id range
//    (plain coalesced stores, and overwritten by every pass, so never
//    cleared); only shared nodes, one range at the end, need atomics and
//    clearing.
// 4. Inside a tile, elements are interleaved (stride S along the curve) so
//    that the elements of one wavefront rarely share nodes.
// 5. Element connectivity is stored as 16-bit indices into the tile's node
//    list; boundary faces are attached to the tile of their owning element.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#include "sw_layout.h"

namespace sw {

static inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

void build_layout(int64_t n_nodes, int64_t n_tets, int64_t n_faces, const double* xyz, const int32_t* tet10,
                  const int32_t* tri6, const int32_t* face_tet, const uint8_t* face_role, HostLayout& L,
                  int max_nodes, int max_elems) {
  L = HostLayout();
  L.n_nodes = n_nodes;
  L.n_tets = n_tets;
  L.n_faces = n_faces;
  // --- Morton order of element centroids
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = 0; i < n_nodes; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], xyz[3 * i + d]);
      hi[d] = std::max(hi[d], xyz[3 * i + d]);
    }
  double span = 0.0;
  for (int d = 0; d < 3; ++d) span = std::max(span, hi[d] - lo[d]);
  const double scale = span > 0.0 ? (double)((1 << 21) - 1) / span : 0.0;
  std::vector<std::pair<uint64_t, int32_t>> key(n_tets);
  for (int64_t e = 0; e < n_tets; ++e) {
    double c[3] = {0, 0, 0};
    for (int k = 0; k < 4; ++k)
      for (int d = 0; d < 3; ++d) c[d] += 0.25 * xyz[3 * (int64_t)tet10[10 * e + k] + d];
    uint64_t m = 0;
    for (int d = 0; d < 3; ++d) m |= spread3((uint64_t)((c[d] - lo[d]) * scale)) << d;
    key[e] = {m, (int32_t)e};
  }
  std::sort(key.begin(), key.end());
  // --- tiles (node-capped)
  std::vector<int32_t> mark(n_nodes, -1);
  L.elem_order.resize(n_tets);
  L.tile_elem_off.push_back(0);
  int32_t tile = 0, tile_nodes = 0, tile_elems = 0;
  for (int64_t i = 0; i < n_tets; ++i) {
    const int32_t e = key[i].second;
    int add = 0;
    for (int k = 0; k < 10; ++k) {
      const int32_t n = tet10[10 * (int64_t)e + k];
      bool dup = mark[n] == tile;
      for (int j = 0; j < k && !dup; ++j) dup = tet10[10 * (int64_t)e + j] == n;
      add += dup ? 0 : 1;
    }
    if (tile_elems > 0 && (tile_nodes + add > max_nodes || tile_elems + 1 > max_elems)) {
      L.tile_elem_off.push_back((int32_t)i);
      ++tile;
      tile_nodes = 0;
      tile_elems = 0;
      add = 10;  // recount for the new tile
      int distinct = 0;
      for (int k = 0; k < 10; ++k) {
        bool dup = false;
        for (int j = 0; j < k && !dup; ++j) dup = tet10[10 * (int64_t)e + j] == tet10[10 * (int64_t)e + k];
        distinct += dup ? 0 : 1;
      }
      add = distinct;
    }
    for (int k = 0; k < 10; ++k) mark[tet10[10 * (int64_t)e + k]] = tile;
    tile_nodes += add;
    ++tile_elems;
    L.elem_order[i] = e;
  }
  L.tile_elem_off.push_back((int32_t)n_tets);
  const int32_t n_tiles = tile + 1;
  L.n_tiles = n_tiles;
  // --- element order inside each tile: position j holds the tile's
  // (j * S mod n)-th element along the Morton curve, S coprime to n.  The
  // kernels hand consecutive positions to consecutive lanes (coalesced
  // loads), and those elements lie S apart along the curve, so they rarely
  // share a node and the LDS atomics of one instruction seldom collide.
  {
    std::vector<int32_t> tmp;
    for (int32_t t = 0; t < n_tiles; ++t) {
      const int32_t e0 = L.tile_elem_off[t], n_e = L.tile_elem_off[t + 1] - e0;
      // n_e <= TILE_MAX_ELEMS < 7 * 11 * 13 * 17, so one of these is coprime
      const int S = (n_e % 7) ? 7 : ((n_e % 11) ? 11 : ((n_e % 13) ? 13 : 17));
      tmp.assign(L.elem_order.begin() + e0, L.elem_order.begin() + e0 + n_e);
      for (int32_t j = 0; j < n_e; ++j) L.elem_order[e0 + j] = tmp[(int32_t)(((int64_t)j * S) % n_e)];
    }
  }
  // --- how many tiles touch each node
  std::vector<int32_t> ntouch(n_nodes, 0);
  std::fill(mark.begin(), mark.end(), -1);
  for (int32_t t = 0; t < n_tiles; ++t)
    for (int32_t i = L.tile_elem_off[t]; i < L.tile_elem_off[t + 1]; ++i) {
      const int32_t e = L.elem_order[i];
      for (int k = 0; k < 10; ++k) {
        const int32_t n = tet10[10 * (int64_t)e + k];
        if (mark[n] != t) {
          mark[n] = t;
          ++ntouch[n];
        }
      }
    }
  // --- node renumbering: every tile's interior nodes, tile by tile (one
  // contiguous range per tile), then all shared nodes in the order tiles
  // first touch them (one contiguous range at the end)
  L.node_u2i.assign(n_nodes, -1);
  int32_t next = 0;
  L.tile_int_base.resize(n_tiles);
  L.tile_nint.resize(n_tiles);
  for (int pass = 0; pass < 2; ++pass) {
    for (int32_t t = 0; t < n_tiles; ++t) {
      if (pass == 0) L.tile_int_base[t] = next;
      for (int32_t i = L.tile_elem_off[t]; i < L.tile_elem_off[t + 1]; ++i) {
        const int32_t e = L.elem_order[i];
        for (int k = 0; k < 10; ++k) {
          const int32_t n = tet10[10 * (int64_t)e + k];
          if (L.node_u2i[n] >= 0) continue;
          if ((pass == 0) == (ntouch[n] == 1)) L.node_u2i[n] = next++;
        }
      }
      if (pass == 0) L.tile_nint[t] = next - L.tile_int_base[t];
    }
    if (pass == 0) L.n_interior = next;
  }
  for (int64_t n = 0; n < n_nodes; ++n)
    if (L.node_u2i[n] < 0) L.node_u2i[n] = next++;  // nodes of no element
  L.node_i2u.resize(n_nodes);
  for (int64_t n = 0; n < n_nodes; ++n) L.node_i2u[L.node_u2i[n]] = (int32_t)n;
  // --- tile node lists (interior ascending, then shared ascending) and local connectivity
  L.tile_node_off.assign(n_tiles + 1, 0);
  L.tet_stride = (n_tets + 63) / 64 * 64;
  L.conn_loc.assign(10 * (size_t)L.tet_stride, 0);
  L.elem_u2i.resize(n_tets);
  std::vector<int32_t> loc(n_nodes, -1), shared;
  for (int32_t t = 0; t < n_tiles; ++t) {
    const int32_t base = L.tile_int_base[t], nint = L.tile_nint[t];
    for (int32_t j = 0; j < nint; ++j) {
      L.tile_nodes.push_back(base + j);
      loc[L.node_i2u[base + j]] = j;
    }
    shared.clear();
    for (int32_t i = L.tile_elem_off[t]; i < L.tile_elem_off[t + 1]; ++i) {
      const int32_t e = L.elem_order[i];
      for (int k = 0; k < 10; ++k) {
        const int32_t n = tet10[10 * (int64_t)e + k];
        if (ntouch[n] > 1 && loc[n] == -1) {
          loc[n] = -2;  // seen
          shared.push_back(L.node_u2i[n]);
        }
      }
    }
    std::sort(shared.begin(), shared.end());
    for (size_t j = 0; j < shared.size(); ++j) {
      L.tile_nodes.push_back(shared[j]);
      loc[L.node_i2u[shared[j]]] = nint + (int32_t)j;
    }
    const int32_t nt = nint + (int32_t)shared.size();
    L.tile_node_off[t + 1] = L.tile_node_off[t] + nt;
    L.max_tile_nodes = std::max(L.max_tile_nodes, nt);
    for (int32_t i = L.tile_elem_off[t]; i < L.tile_elem_off[t + 1]; ++i) {
      const int32_t e = L.elem_order[i];
      L.elem_u2i[e] = i;
      for (int k = 0; k < 10; ++k)
        L.conn_loc[k * (size_t)L.tet_stride + i] = (uint16_t)(3 * loc[tet10[10 * (int64_t)e + k]]);
    }
    // reset loc for this tile's nodes
    for (int32_t j = L.tile_node_off[t]; j < L.tile_node_off[t + 1]; ++j) loc[L.node_i2u[L.tile_nodes[j]]] = -1;
  }
  // --- coordinates in internal order
  L.xyz.resize(3 * (size_t)n_nodes);
  for (int64_t i = 0; i < n_nodes; ++i)
    for (int d = 0; d < 3; ++d) L.xyz[3 * i + d] = xyz[3 * (int64_t)L.node_i2u[i] + d];
  // --- element count per node (for element-to-node averages)
  {
    std::vector<int32_t> cnt(n_nodes, 0);
    for (int64_t e = 0; e < n_tets; ++e)
      for (int k = 0; k < 10; ++k) cnt[L.node_u2i[tet10[10 * e + k]]] += 1;
    L.inv_valence.resize(n_nodes);
    for (int64_t i = 0; i < n_nodes; ++i) L.inv_valence[i] = cnt[i] > 0 ? 1.0f / (float)cnt[i] : 0.0f;
  }
  // --- faces grouped by the tile of their owner; local and global node ids
  std::vector<int32_t> forder(n_faces);
  std::iota(forder.begin(), forder.end(), 0);
  std::stable_sort(forder.begin(), forder.end(),
                   [&](int32_t a, int32_t b) { return L.elem_u2i[face_tet[a]] < L.elem_u2i[face_tet[b]]; });
  L.face_stride = (std::max<int64_t>(n_faces, 1) + 63) / 64 * 64;
  L.fconn.assign(6 * (size_t)L.face_stride, 0);
  L.fconn_loc.assign(6 * (size_t)L.face_stride, 0);
  L.face_elem.assign(L.face_stride, 0);
  L.face_role.assign(L.face_stride, 0);
  L.tile_face_off.assign(n_tiles + 1, 0);
  {
    int32_t f = 0;
    for (int32_t t = 0; t < n_tiles; ++t) {
      // local index map of this tile
      for (int32_t j = L.tile_node_off[t]; j < L.tile_node_off[t + 1]; ++j)
        loc[L.node_i2u[L.tile_nodes[j]]] = j - L.tile_node_off[t];
      while (f < n_faces && L.elem_u2i[face_tet[forder[f]]] < L.tile_elem_off[t + 1]) {
        const int32_t uf = forder[f];
        for (int k = 0; k < 6; ++k) {
          const int32_t n = tri6[6 * (int64_t)uf + k];
          L.fconn[k * (size_t)L.face_stride + f] = L.node_u2i[n];
          L.fconn_loc[k * (size_t)L.face_stride + f] = (uint16_t)loc[n];
        }
        L.face_elem[f] = L.elem_u2i[face_tet[uf]];
        L.face_role[f] = face_role[uf];
        ++f;
      }
      L.tile_face_off[t + 1] = f;
      for (int32_t j = L.tile_node_off[t]; j < L.tile_node_off[t + 1]; ++j) loc[L.node_i2u[L.tile_nodes[j]]] = -1;
    }
  }
}

void build_incidence(const HostLayout& L, Incidence& I) {
  const int64_t nn = L.n_nodes;
  // element slots: slot e * 10 + k of internal element e's node k
  I.elem_off.assign(nn + 1, 0);
  auto node_of = [&](int32_t t, int64_t e, int k) {
    return L.tile_nodes[L.tile_node_off[t] + L.conn_loc[k * (size_t)L.tet_stride + e] / 3];
  };
  for (int32_t t = 0; t < L.n_tiles; ++t)
    for (int64_t e = L.tile_elem_off[t]; e < L.tile_elem_off[t + 1]; ++e)
      for (int k = 0; k < 10; ++k) ++I.elem_off[node_of(t, e, k) + 1];
  for (int64_t i = 0; i < nn; ++i) I.elem_off[i + 1] += I.elem_off[i];
  I.elem.assign(I.elem_off[nn], 0);
  std::vector<int32_t> pos(I.elem_off.begin(), I.elem_off.end() - 1);
  // elements in increasing order, so every node's list is sorted
  for (int32_t t = 0; t < L.n_tiles; ++t)
    for (int64_t e = L.tile_elem_off[t]; e < L.tile_elem_off[t + 1]; ++e)
      for (int k = 0; k < 10; ++k) I.elem[pos[node_of(t, e, k)]++] = (int32_t)(e * 10 + k);
  // face slots: f * 6 + k
  I.face_off.assign(nn + 1, 0);
  for (int64_t f = 0; f < L.n_faces; ++f)
    for (int k = 0; k < 6; ++k) ++I.face_off[L.fconn[k * (size_t)L.face_stride + f] + 1];
  for (int64_t i = 0; i < nn; ++i) I.face_off[i + 1] += I.face_off[i];
  I.face.assign(std::max<int32_t>(I.face_off[nn], 1), 0);
  pos.assign(I.face_off.begin(), I.face_off.end() - 1);
  for (int64_t f = 0; f < L.n_faces; ++f)
    for (int k = 0; k < 6; ++k) I.face[pos[L.fconn[k * (size_t)L.face_stride + f]]++] = (int32_t)(f * 6 + k);
}

}  // namespace sw
