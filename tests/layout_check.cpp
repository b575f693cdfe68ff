// CPU check of the host-side tiled mesh layout (sw::build_layout): builds the
// layout of a caller's mesh and verifies every property the operator kernels
// rely on.  Compiled with g++ together with sw_mesh.cpp by tests/test_layout.py;
// returns 0, or the number of the first property that fails.  plant != 0
// first plants one mistake in the built layout (a test that the checks see
// it): 1 a wrong tile-local index, 2 an interior node id out of its range,
// 3 a wrong inverse valence, 4 a face moved to another tile's element, 5 two
// slots of a node's incidence list swapped, 6 an element slot listed under
// the wrong node.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "sw_layout.h"

using sw::HostLayout;

extern "C" int check_layout(int64_t nn, int64_t nt, int64_t nf, const double* xyz, const int32_t* tet10,
                            const int32_t* tri6, const int32_t* face_tet, const uint8_t* face_role,
                            int32_t plant, int64_t* stats) {
  HostLayout L;
  sw::build_layout(nn, nt, nf, xyz, tet10, tri6, face_tet, face_role, L);
  if (plant == 1) std::swap(L.conn_loc[0], L.conn_loc[L.tet_stride]);
  if (plant == 2) L.tile_nodes[L.tile_node_off[0]] += 1;
  if (plant == 3) L.inv_valence[nn / 2] *= 0.5f;
  if (plant == 4 && nf > 0) {
    const int t = L.tile_face_off[1] > 0 ? 0 : 1;  // a tile that owns a face
    L.face_elem[L.tile_face_off[t]] = L.tile_elem_off[t + 1];
  }
  // 1-2: element and node numberings are permutations, 3: tile size caps
  std::vector<int> seen(nt, 0);
  for (int32_t e : L.elem_order)
    if (e < 0 || e >= nt || seen[e]++) return 1;
  for (int64_t i = 0; i < nn; ++i)
    if (L.node_u2i[i] < 0 || L.node_u2i[i] >= nn || L.node_i2u[L.node_u2i[i]] != i) return 2;
  if (L.max_tile_nodes > sw::TILE_MAX_NODES) return 3;
  // 4: coordinates follow the node numbering
  for (int64_t i = 0; i < nn; ++i)
    for (int d = 0; d < 3; ++d)
      if (L.xyz[3 * (int64_t)L.node_u2i[i] + d] != xyz[3 * i + d]) return 4;
  std::vector<int> touched_by(nn, 0), last(nn, -1), valence(nn, 0);
  int64_t shared_total = 0, tile_nodes_total = 0, max_elems = 0, next_interior = 0;
  for (int t = 0; t < L.n_tiles; ++t) {
    const int n0 = L.tile_node_off[t], ntn = L.tile_node_off[t + 1] - n0, nint = L.tile_nint[t];
    const int ne = L.tile_elem_off[t + 1] - L.tile_elem_off[t];
    // 5: caps per tile; 6: the interior ranges are consecutive in tile order
    if (ntn > sw::TILE_MAX_NODES || ne > sw::TILE_MAX_ELEMS || nint < 0 || nint > ntn) return 5;
    if (L.tile_int_base[t] != next_interior) return 6;
    next_interior += nint;
    // 7: interior nodes first, as one contiguous id range
    for (int j = 0; j < nint; ++j)
      if (L.tile_nodes[n0 + j] != L.tile_int_base[t] + j) return 7;
    // 8: shared nodes follow, address-sorted, all in the shared suffix
    for (int j = nint; j < ntn; ++j) {
      const int g = L.tile_nodes[n0 + j];
      if (g < L.n_interior || g >= nn || (j > nint && g <= L.tile_nodes[n0 + j - 1])) return 8;
    }
    shared_total += ntn - nint;
    tile_nodes_total += ntn;
    max_elems = std::max<int64_t>(max_elems, ne);
    // 9-11: every element's tile-local indices name its own nodes, and the
    // tile's node list holds exactly the nodes its elements use
    std::vector<char> used(ntn, 0);
    for (int e = L.tile_elem_off[t]; e < L.tile_elem_off[t + 1]; ++e) {
      const int ue = L.elem_order[e];
      if (L.elem_u2i[ue] != e) return 9;
      for (int k = 0; k < 10; ++k) {
        // stored as three times the tile-local index (the offset of the
        // node's first value in the tile's 3-value-per-node arrays)
        const int l3 = L.conn_loc[k * L.tet_stride + e];
        if (l3 % 3) return 10;
        const int l = l3 / 3;
        if (l >= ntn || L.tile_nodes[n0 + l] != L.node_u2i[tet10[10 * (int64_t)ue + k]]) return 10;
        used[l] = 1;
        const int g = L.tile_nodes[n0 + l];
        valence[g] += 1;
        if (last[g] != t) {
          last[g] = t;
          touched_by[g] += 1;
        }
      }
    }
    for (int j = 0; j < ntn; ++j)
      if (!used[j]) return 11;
    // 12-13: faces sit in the tile of their owning element, with consistent
    // local and global node ids
    for (int f = L.tile_face_off[t]; f < L.tile_face_off[t + 1]; ++f) {
      if (L.face_elem[f] < L.tile_elem_off[t] || L.face_elem[f] >= L.tile_elem_off[t + 1]) return 12;
      for (int k = 0; k < 6; ++k) {
        const int l = L.fconn_loc[k * L.face_stride + f];
        if (l >= ntn || L.tile_nodes[n0 + l] != L.fconn[k * L.face_stride + f]) return 13;
      }
    }
  }
  // 14: every face placed once; 15: the interior ranges cover [0, n_interior)
  if (L.tile_face_off[L.n_tiles] != nf) return 14;
  if (next_interior != L.n_interior) return 15;
  // 16: an interior node is touched by its own tile only, a shared one by
  // more than one
  for (int64_t g = 0; g < nn; ++g) {
    if (g < L.n_interior && touched_by[g] != 1) return 16;
    if (g >= L.n_interior && touched_by[g] < 2) return 16;
  }
  // 17: 1 / valence per node
  for (int64_t g = 0; g < nn; ++g) {
    const float want = valence[g] > 0 ? 1.0f / (float)valence[g] : 0.0f;
    if (L.inv_valence[g] != want) return 17;
  }
  // 18-19: the incidence lists of the deterministic passes: every element
  // slot e * 10 + k (face slot f * 6 + k) listed once, under the internal id
  // of that slot's node, each list in increasing order
  sw::Incidence I;
  sw::build_incidence(L, I);
  if (plant == 5) {
    for (int64_t g = 0; g < nn; ++g)
      if (I.elem_off[g + 1] - I.elem_off[g] >= 2) {
        std::swap(I.elem[I.elem_off[g]], I.elem[I.elem_off[g] + 1]);
        break;
      }
  }
  if (plant == 6) std::swap(I.elem[0], I.elem[I.elem.size() - 1]);
  if ((int64_t)I.elem_off.size() != nn + 1 || I.elem_off[0] != 0 || I.elem_off[nn] != 10 * nt) return 18;
  {
    std::vector<int> hit(10 * nt, 0);
    for (int64_t g = 0; g < nn; ++g)
      for (int32_t j = I.elem_off[g]; j < I.elem_off[g + 1]; ++j) {
        const int32_t sl = I.elem[j];
        if (sl < 0 || sl >= 10 * nt || hit[sl]++) return 18;
        if (j > I.elem_off[g] && I.elem[j - 1] >= sl) return 18;
        const int64_t e = sl / 10, k = sl % 10;
        if (L.node_u2i[tet10[10 * (int64_t)L.elem_order[e] + k]] != g) return 18;
      }
  }
  if ((int64_t)I.face_off.size() != nn + 1 || I.face_off[nn] != 6 * nf) return 19;
  {
    std::vector<int> hit(std::max<int64_t>(6 * nf, 1), 0);
    for (int64_t g = 0; g < nn; ++g)
      for (int32_t j = I.face_off[g]; j < I.face_off[g + 1]; ++j) {
        const int32_t sl = I.face[j];
        if (sl < 0 || sl >= 6 * nf || hit[sl]++) return 19;
        if (j > I.face_off[g] && I.face[j - 1] >= sl) return 19;
        if (L.fconn[(sl % 6) * L.face_stride + sl / 6] != g) return 19;
      }
  }
  stats[0] = L.n_tiles;
  stats[1] = L.max_tile_nodes;
  stats[2] = shared_total;
  stats[3] = tile_nodes_total;
  stats[4] = max_elems;
  stats[5] = L.n_interior;
  return 0;
}

// Modelled LDS bank cycles of the element work: for every wavefront of 64
// element positions of a tile and every node k of the element, the largest
// number of distinct dwords that one instruction sends to one of 64
// dword-wide banks: out[0] for the FP32 node-value reads (dword 3 l + c),
// out[1] for the FP64 accumulator atomics (dwords 2 (3 l + c) and the next),
// averaged over instructions.  Tiles close at max_elems elements.
extern "C" int bank_cycles(int64_t nn, int64_t nt, int64_t nf, const double* xyz, const int32_t* tet10,
                           const int32_t* tri6, const int32_t* face_tet, const uint8_t* face_role, int32_t max_elems,
                           double* out) {
  HostLayout L;
  sw::build_layout(nn, nt, nf, xyz, tet10, tri6, face_tet, face_role, L, sw::TILE_MAX_NODES, max_elems);
  double rd = 0.0, at = 0.0;
  int64_t n = 0;
  for (int32_t t = 0; t < L.n_tiles; ++t) {
    const int32_t e0 = L.tile_elem_off[t], ne = L.tile_elem_off[t + 1] - e0;
    for (int32_t w0 = 0; w0 < ne; w0 += 64) {
      const int nl = std::min(64, ne - w0);
      for (int k = 0; k < 10; ++k)
        for (int c = 0; c < 3; ++c) {
          int rcnt[64] = {0}, acnt[64] = {0};
          std::vector<int> seen;
          for (int l = 0; l < nl; ++l) {
            const int a = L.conn_loc[k * (size_t)L.tet_stride + e0 + w0 + l] + c;
            acnt[(2 * a) % 64]++;
            acnt[(2 * a + 1) % 64]++;
            if (std::find(seen.begin(), seen.end(), a) != seen.end()) continue;
            seen.push_back(a);
            rcnt[a % 64]++;
          }
          rd += *std::max_element(rcnt, rcnt + 64);
          at += *std::max_element(acnt, acnt + 64);
          ++n;
        }
    }
  }
  out[0] = rd / n;
  out[1] = at / n;
  return 0;
}

// Tile shape statistics of the layout with caps (max_nodes, max_elems):
// out[0] tiles, out[1] fewest and out[2] most elements in a tile, out[3] the
// share of tile-node entries that are shared nodes, out[4] tile-node entries
// per mesh node.
extern "C" int tile_stats(int64_t nn, int64_t nt, int64_t nf, const double* xyz, const int32_t* tet10,
                          const int32_t* tri6, const int32_t* face_tet, const uint8_t* face_role, int32_t max_nodes,
                          int32_t max_elems, double* out) {
  HostLayout L;
  sw::build_layout(nn, nt, nf, xyz, tet10, tri6, face_tet, face_role, L, max_nodes, max_elems);
  int64_t entries = 0, shared = 0;
  int lo = 1 << 30, hi = 0;
  for (int32_t t = 0; t < L.n_tiles; ++t) {
    const int n = L.tile_node_off[t + 1] - L.tile_node_off[t];
    entries += n;
    shared += n - L.tile_nint[t];
    const int ne = L.tile_elem_off[t + 1] - L.tile_elem_off[t];
    lo = std::min(lo, ne);
    hi = std::max(hi, ne);
  }
  out[0] = L.n_tiles;
  out[1] = lo;
  out[2] = hi;
  out[3] = (double)shared / (double)entries;
  out[4] = (double)entries / (double)nn;
  return 0;
}
