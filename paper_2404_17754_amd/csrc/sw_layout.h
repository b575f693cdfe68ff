// Host-side tiled mesh layout (built by sw_mesh.cpp, uploaded by sw_api.cpp).
#pragma once

#include <cstdint>
#include <vector>

namespace sw {

// A tile's node values and accumulators live in LDS: FP64 accumulators (24
// bytes per node; LDS FP32 atomics measured 2.3x slower), the input values
// (12 bytes in FP32, 24 in FP64) and a 4-byte node id.  At 1280 nodes an FP32
// pass takes 51 KB, so three workgroups share a compute unit's 160 KB (the
// FP32 kernel's registers allow three waves per SIMD), and an FP64 pass
// 67 KB (two workgroups; its registers allow two waves per SIMD).  Measured
// on the 9.6 M-tet mesh: FP32 pass 787 us at 1536 nodes, 655 us at 1280,
// 670 us at 1152.
constexpr int TILE_MAX_NODES = 1280;
constexpr int TILE_MAX_ELEMS = 1024;
// Default element cap: two per work-item of a 256-wide workgroup.  At the
// 1280-node cap alone tiles of P2 tets close at about 570 elements, so the
// work-items of a workgroup take two or three elements and the third round
// runs mostly idle; closing tiles at 512 elements (about 1150 nodes) gives
// every work-item two.  Measured on the 9.6 M-tet mesh, FP32 pass: 0.409 ms
// at 512 elements against 0.424 ms at 1024 (node-limited).
constexpr int TILE_DEFAULT_ELEMS = 512;

struct HostLayout {
  int64_t n_nodes = 0, n_tets = 0, n_faces = 0;
  int32_t n_tiles = 0;
  int32_t max_tile_nodes = 0;
  int64_t n_interior = 0;              // nodes [0, n_interior) are interior to one tile
  int64_t tet_stride = 0, face_stride = 0;
  std::vector<int32_t> elem_order;     // internal element i = user element elem_order[i]
  std::vector<int32_t> elem_u2i;       // user element -> internal
  std::vector<int32_t> node_u2i, node_i2u;
  std::vector<int32_t> tile_elem_off;  // [n_tiles + 1]
  std::vector<int32_t> tile_node_off;  // [n_tiles + 1]
  std::vector<int32_t> tile_nodes;     // internal node ids, per tile: interior then shared
  std::vector<int32_t> tile_int_base;  // first interior node id of each tile
  std::vector<int32_t> tile_nint;      // interior node count of each tile
  std::vector<int32_t> tile_face_off;  // [n_tiles + 1]
  std::vector<uint16_t> conn_loc;      // [10][tet_stride] 3 x tile-local node index (offset of the node's
                                       // first value in 3-value-per-node tile arrays)
  std::vector<double> xyz;             // [n_nodes][3] internal order
  std::vector<int32_t> fconn;          // [6][face_stride] internal node ids
  std::vector<uint16_t> fconn_loc;     // [6][face_stride] tile-local node index
  std::vector<int32_t> face_elem;      // internal element owning each face
  std::vector<uint8_t> face_role;
  std::vector<float> inv_valence;      // [n_nodes] 1 / elements containing the node (0 if none)
};

// Per node, the element slots (internal element e's node k: e * 10 + k) and
// face slots (f * 6 + k) that touch it, each list in increasing order: a
// node sums the contributions in this fixed order in deterministic passes.
struct Incidence {
  std::vector<int32_t> elem_off, elem;  // [n_nodes + 1], [10 n_tets]
  std::vector<int32_t> face_off, face;  // [n_nodes + 1], [6 n_faces]
};

void build_incidence(const HostLayout& L, Incidence& I);

// Tiles close at max_nodes distinct nodes or max_elems elements (at most
// TILE_MAX_NODES / TILE_MAX_ELEMS; smaller tiles are a tuning and test knob).
void build_layout(int64_t n_nodes, int64_t n_tets, int64_t n_faces, const double* xyz, const int32_t* tet10,
                  const int32_t* tri6, const int32_t* face_tet, const uint8_t* face_role, HostLayout& L,
                  int max_nodes = TILE_MAX_NODES, int max_elems = TILE_MAX_ELEMS);

}  // namespace sw
