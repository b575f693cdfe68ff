// Host-side layout of a mesh for the LDS-tiled element-by-element kernels.
//
// 1. Elements are ordered along a Morton (Z-order) curve of their centroids,
//    which groups spatial neighbours whatever the input numbering.
// 2. Tiles come from recursive coordinate bisection of the element
//    centroids into compact parts of at most TILE_MAX_ELEMS elements and
//    TILE_MAX_NODES distinct nodes, so a tile's node values and accumulators
//    fit in one workgroup's LDS; each part keeps the Morton order.
// 3. Nodes are renumbered: every tile's interior nodes (touched by no other
//    tile), tile by tile, then all shared nodes in the order tiles first
//    touch them.  A tile's interior nodes are thus one contiguous id range
//    (plain coalesced stores, and overwritten by every pass, so never
//    cleared); only shared nodes, one range at the end, need atomics and
//    clearing.
// 4. Inside a tile, elements are interleaved (stride S along the curve) so
//    that the elements of one wavefront rarely share nodes; then elements are
//    grouped into half-wavefronts and the tile's interior nodes relabelled so
//    that the nodes one LDS instruction reaches fall into different banks
//    (spread_banks).
// 5. Element connectivity is stored as 16-bit indices into the tile's node
//    list; boundary faces are attached to the tile of their owning element.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <system_error>
#include <thread>
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

// LDS bank spreading of one tile.  A work-item handles the tile's elements
// i, i + 256, ...; so element position p runs in wavefront p / 64 (64 lanes)
// and half-wavefront p / 32, and the k-th node of every element of a
// wavefront is read (three FP32 values at dword 3 l + c of the tile's node
// arrays) and accumulated (three FP64 atomics at dwords 2 (3 l + c), +1) by
// one LDS instruction each.  Two lanes of one instruction at different
// addresses in one bank serialise: for the FP32 reads when their local
// indices l agree mod 64 (3 is invertible mod 64), for the FP64 atomics when
// they agree mod 32.  The tile's shared nodes keep their local indices (the
// address-sorted suffix); two greedy passes spread the rest:
//  * elements, in the interleaved order, each go to the half-wavefront
//    (with room) where their shared nodes collide least with those already
//    there (node k against node k: collisions mod 64 over the wavefront plus
//    mod 32 over the half), a node repeated at the same k costing most;
//  * interior nodes, most-referenced first, each take the residue mod 64
//    (with a free slot in [0, nint)) that collides least over the groups it
//    appears in, and the slots of each residue are handed out in order.
// Reorders the tile's elements (conn columns, elem_order) and returns the new
// local index of each interior node in newloc.
static_assert(TILE_MAX_ELEMS <= 32 * 32, "a tile's half-wavefronts must fit the 32-bit group mask");
static void spread_banks(int32_t e0, int32_t ne, int32_t nint, int32_t nt, int64_t stride, std::vector<uint16_t>& conn,
                         std::vector<int32_t>& elem_order, std::vector<int32_t>& newloc) {
  const int nh = (ne + 31) / 32, nw = (ne + 63) / 64;
  auto node = [&](int i, int k) { return (int)(conn[k * (size_t)stride + e0 + i] / 3); };
  // --- elements into half-wavefronts
  std::vector<int32_t> pos(ne), fill(nh, 0);
  std::vector<uint32_t> inhalf((size_t)nt * 10, 0);  // bit h: node at position k in half h
  std::vector<int32_t> c64((size_t)nw * 10 * 64, 0), c32((size_t)nh * 10 * 32, 0);
  for (int i = 0; i < ne; ++i) {
    int best = -1;
    int64_t bc = INT64_MAX;
    for (int h = 0; h < nh; ++h) {
      if (fill[h] >= std::min(32, ne - 32 * h)) continue;
      const int w = h / 2;
      int64_t c = 0;
      for (int k = 0; k < 10; ++k) {
        const int j = node(i, k);
        if ((inhalf[(size_t)j * 10 + k] >> h) & 1u)
          c += 8;
        else if (j >= nint)
          c += c64[((size_t)w * 10 + k) * 64 + j % 64] + c32[((size_t)h * 10 + k) * 32 + j % 32];
      }
      if (c < bc) {
        bc = c;
        best = h;
      }
    }
    const int h = best, w = h / 2;
    pos[i] = 32 * h + fill[h]++;
    for (int k = 0; k < 10; ++k) {
      const int j = node(i, k);
      inhalf[(size_t)j * 10 + k] |= 1u << h;
      if (j >= nint) {
        c64[((size_t)w * 10 + k) * 64 + j % 64]++;
        c32[((size_t)h * 10 + k) * 32 + j % 32]++;
      }
    }
  }
  std::vector<int32_t> tmp(ne);
  std::vector<uint16_t> col(ne);
  for (int k = 0; k < 10; ++k) {
    uint16_t* ck = conn.data() + k * (size_t)stride + e0;
    std::copy(ck, ck + ne, col.begin());
    for (int i = 0; i < ne; ++i) ck[pos[i]] = col[i];
  }
  std::copy(elem_order.begin() + e0, elem_order.begin() + e0 + ne, tmp.begin());
  for (int i = 0; i < ne; ++i) elem_order[e0 + pos[i]] = tmp[i];
  // --- interior nodes onto residues
  std::vector<int32_t> goff(nt + 1, 0), gw, gh;
  for (int i = 0; i < ne; ++i)
    for (int k = 0; k < 10; ++k) ++goff[node(i, k) + 1];
  for (int j = 0; j < nt; ++j) goff[j + 1] += goff[j];
  gw.resize(goff[nt]);
  gh.resize(goff[nt]);
  {
    std::vector<int32_t> at(goff.begin(), goff.end() - 1);
    for (int i = 0; i < ne; ++i)
      for (int k = 0; k < 10; ++k) {
        const int j = node(i, k);
        gw[at[j]] = (i / 64) * 10 + k;
        gh[at[j]++] = (i / 32) * 10 + k;
      }
  }
  std::fill(c64.begin(), c64.end(), 0);
  std::fill(c32.begin(), c32.end(), 0);
  for (int j = nint; j < nt; ++j)
    for (int q = goff[j]; q < goff[j + 1]; ++q) {
      c64[(size_t)gw[q] * 64 + j % 64]++;
      c32[(size_t)gh[q] * 32 + j % 32]++;
    }
  int cap[64] = {0};
  for (int j = 0; j < nint; ++j) ++cap[j % 64];
  std::vector<int32_t> ord(nint), res(nint);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int a, int b) { return goff[a + 1] - goff[a] > goff[b + 1] - goff[b]; });
  int32_t cost[64];
  for (int j : ord) {
    std::fill(cost, cost + 64, 0);
    for (int q = goff[j]; q < goff[j + 1]; ++q) {
      const int32_t* a = &c64[(size_t)gw[q] * 64];
      const int32_t* b = &c32[(size_t)gh[q] * 32];
      for (int r = 0; r < 64; ++r) cost[r] += a[r] + b[r & 31];
    }
    int best = -1;
    int32_t bc = INT32_MAX;
    for (int r = 0; r < 64; ++r)
      if (cap[r] && cost[r] < bc) {
        bc = cost[r];
        best = r;
      }
    res[j] = best;
    --cap[best];
    for (int q = goff[j]; q < goff[j + 1]; ++q) {
      c64[(size_t)gw[q] * 64 + best]++;
      c32[(size_t)gh[q] * 32 + best % 32]++;
    }
  }
  int next[64];
  for (int r = 0; r < 64; ++r) next[r] = r;
  newloc.resize(nint);
  for (int j = 0; j < nint; ++j) {
    newloc[j] = next[res[j]];
    next[res[j]] += 64;
  }
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
  // --- tiles: recursive coordinate bisection of the element centroids.  A
  // range is cut across its longest extent at the multiple of max_elems
  // nearest its middle, so parts are compact blocks of max_elems elements
  // (fewer nodes shared between tiles than runs of the Morton curve); a part
  // over the node cap is halved again.  Parts are emitted depth first
  // (neighbouring tiles stay neighbours in the list), each in Morton order.
  std::vector<int32_t> mark(n_nodes, -1);
  {
    std::vector<float> cen(3 * (size_t)n_tets);
    std::vector<uint64_t> mkey(n_tets);
    std::vector<int32_t> ids(n_tets);
    for (int64_t i = 0; i < n_tets; ++i) {
      const int32_t e = key[i].second;
      ids[i] = e;
      mkey[e] = key[i].first;
      for (int d = 0; d < 3; ++d) {
        double c = 0.0;
        for (int k = 0; k < 4; ++k) c += 0.25 * xyz[3 * (int64_t)tet10[10 * (int64_t)e + k] + d];
        cen[3 * (size_t)e + d] = (float)c;
      }
    }
    int32_t stamp = 0;
    auto distinct_nodes = [&](int64_t a, int64_t b) {
      ++stamp;
      int cnt = 0;
      for (int64_t i = a; i < b; ++i)
        for (int k = 0; k < 10; ++k) {
          const int32_t n = tet10[10 * (int64_t)ids[i] + k];
          if (mark[n] != stamp) {
            mark[n] = stamp;
            ++cnt;
          }
        }
      return cnt;
    };
    L.elem_order.reserve(n_tets);
    L.tile_elem_off.push_back(0);
    std::vector<std::pair<int64_t, int64_t>> todo{{0, n_tets}};
    while (!todo.empty()) {
      const int64_t a = todo.back().first, b = todo.back().second;
      todo.pop_back();
      const int64_t n = b - a;
      if (n == 1 || (n <= max_elems && distinct_nodes(a, b) <= max_nodes)) {
        std::sort(ids.begin() + a, ids.begin() + b, [&](int32_t x, int32_t y) { return mkey[x] < mkey[y]; });
        L.elem_order.insert(L.elem_order.end(), ids.begin() + a, ids.begin() + b);
        L.tile_elem_off.push_back((int32_t)L.elem_order.size());
        continue;
      }
      float lo3[3] = {3e38f, 3e38f, 3e38f}, hi3[3] = {-3e38f, -3e38f, -3e38f};
      for (int64_t i = a; i < b; ++i)
        for (int d = 0; d < 3; ++d) {
          lo3[d] = std::min(lo3[d], cen[3 * (size_t)ids[i] + d]);
          hi3[d] = std::max(hi3[d], cen[3 * (size_t)ids[i] + d]);
        }
      int ax = 0;
      for (int d = 1; d < 3; ++d)
        if (hi3[d] - lo3[d] > hi3[ax] - lo3[ax]) ax = d;
      int64_t cut = n / 2;
      if (n > max_elems) {
        cut = (cut + max_elems / 2) / max_elems * max_elems;
        cut = std::min<int64_t>(std::max<int64_t>(cut, max_elems), n - 1);
      }
      std::nth_element(ids.begin() + a, ids.begin() + a + cut, ids.begin() + b, [&](int32_t x, int32_t y) {
        return cen[3 * (size_t)x + ax] < cen[3 * (size_t)y + ax];
      });
      todo.push_back({a + cut, b});
      todo.push_back({a, a + cut});
    }
  }
  const int32_t n_tiles = (int32_t)L.tile_elem_off.size() - 1;
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
      for (int k = 0; k < 10; ++k)
        L.conn_loc[k * (size_t)L.tet_stride + i] = (uint16_t)(3 * loc[tet10[10 * (int64_t)e + k]]);
    }
    // reset loc for this tile's nodes
    for (int32_t j = L.tile_node_off[t]; j < L.tile_node_off[t + 1]; ++j) loc[L.node_i2u[L.tile_nodes[j]]] = -1;
  }
  // --- bank spreading, tile by tile on host threads (a tile touches only its
  // own elements' positions and connectivity and its interior node ids): the
  // new element order, and the interior nodes' new local indices, which
  // their ids follow (id = tile_int_base + local index)
  {
    auto run = [&](int32_t t_lo, int32_t t_hi) {
      std::vector<int32_t> newloc, moved;
      for (int32_t t = t_lo; t < t_hi; ++t) {
        const int32_t base = L.tile_int_base[t], nint = L.tile_nint[t];
        const int32_t nt = L.tile_node_off[t + 1] - L.tile_node_off[t];
        const int32_t e0 = L.tile_elem_off[t], ne = L.tile_elem_off[t + 1] - e0;
        spread_banks(e0, ne, nint, nt, L.tet_stride, L.conn_loc, L.elem_order, newloc);
        for (int32_t i = e0; i < e0 + ne; ++i) {
          L.elem_u2i[L.elem_order[i]] = i;
          for (int k = 0; k < 10; ++k) {
            uint16_t& v = L.conn_loc[k * (size_t)L.tet_stride + i];
            if (v / 3 < nint) v = (uint16_t)(3 * newloc[v / 3]);
          }
        }
        moved.resize(nint);
        for (int32_t j = 0; j < nint; ++j) moved[newloc[j]] = L.node_i2u[base + j];
        for (int32_t j = 0; j < nint; ++j) {
          L.node_i2u[base + j] = moved[j];
          L.node_u2i[moved[j]] = base + j;
        }
      }
    };
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    // chunk k of nth; a chunk whose thread cannot be started runs here
    auto lo = [&](int k) { return (int32_t)((int64_t)n_tiles * k / nth); };
    std::vector<std::thread> pool;
    int started = 0;
    if (n_tiles >= 4 * nth) {
      for (; started < nth; ++started) {
        try {
          pool.emplace_back(run, lo(started), lo(started + 1));
        } catch (const std::system_error&) {
          break;
        }
      }
    }
    run(lo(started), n_tiles);
    for (auto& th : pool) th.join();
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
