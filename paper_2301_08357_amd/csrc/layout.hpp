// Host-side mesh ingest for the P1 pressure operator: validation,
// orientation, Morton renumbering, element ordering and node-to-element
// lists.  Integer work only (plus the sign of each element volume).
#pragma once

#include <cstdint>
#include <vector>

#include "pressure_cg.h"

namespace pm {

struct Layout {
    int dim = 0;
    int64_t n_nodes = 0, n_elems = 0, n_free = 0;
    std::vector<int32_t> node_new2old;   // internal node -> caller node
    std::vector<int32_t> elem_new2old;   // internal element -> caller element
    std::vector<int32_t> conn;           // n_elems * 4, internal ids, oriented (slot 3 = 0 in 2D)
    std::vector<int32_t> n2e_off;        // n_nodes + 1
    std::vector<int32_t> n2e_ent;        // 4*e + a, ascending e
    std::vector<uint8_t> dirichlet;      // internal order
    std::vector<double> coords;          // internal order, SoA: coords[ax * n_nodes + i]
    bool periodic = false;               // some period[ax] > 0
    double period[3] = {0.0, 0.0, 0.0};  // 0 = open axis
};

// Validate, orient and renumber.  Returns a PM_* status.
int build_layout(const pm_mesh *m, Layout *L);

// Morton tiles: runs of `tile_nodes` consecutive internal nodes.  A tile
// holds every element touching one of its nodes (its "instances", ascending
// element id: first those whose smallest vertex lies in an earlier tile,
// then the contiguous run the tile owns) and the outside vertices those
// elements reach (its halo, ascending).  Each instance is one record of four
// 16-bit fields, one per vertex (the fourth is 0 for a triangle):
//   bits 0 .. lvb-1   tile-local index: own node i -> i - first node,
//                     halo node -> tile_nodes + rank in the halo list;
//   bits lvb .. 15    for an own node, the rank of the instance among that
//                     node's instances ("row"); max_deg for a halo vertex.
// Node i's k-th element in ascending order is the instance whose vertex i
// has row k.  lvb = 10 for tiles of up to 256 nodes, 11 for larger ones.
struct Tiles {
    int tile_nodes = 0;                   // largest tile
    std::vector<int32_t> node_off;        // n_tiles + 1: tile t owns nodes [node_off[t], node_off[t+1])
    int lvb = 0;
    int64_t n_tiles = 0;
    int max_inst = 0;                     // largest instance count of a tile
    int max_halo = 0;                     // largest halo of a tile
    int max_deg = 0;                      // largest number of elements at one node
    std::vector<int32_t> halo_off;        // n_tiles + 1
    std::vector<int32_t> halo;            // global node ids
    std::vector<int32_t> inst_off;        // n_tiles + 1
    std::vector<int32_t> inst_elem;       // element id of each instance
    std::vector<uint16_t> inst;           // 4 fields per instance
};

// Returned by build_tiles when a node has more elements, or a tile more
// own and halo nodes, than a record can name at this tile size.
constexpr int TILES_TOO_WIDE = 100;

// n_tiles = 0: runs of tile_nodes nodes (the last one shorter); n_tiles > 0:
// that many runs of equal length (floor(t N / n_tiles) boundaries), each at
// most tile_nodes long, so that a grid of B resident blocks gets exactly
// n_tiles / B tiles per block.
int build_tiles(const Layout &L, int tile_nodes, Tiles *T, int64_t n_tiles = 0);

// Dual cells of the face-type staggered mesh: one per face (3D) or edge
// (2D) of the primal mesh.  Faces are numbered by the sorted tuples of the
// node ids of the mesh passed in, in lexicographic order.  A face belongs to
// one element (boundary) or two (interior; with merged periodic vertices
// the two images of a seam face are one interior face).
struct Faces {
    int dim = 0;
    int64_t n_faces = 0, n_boundary = 0;
    std::vector<int32_t> vertices;    // n_faces * dim, ascending node ids
    std::vector<int32_t> elems;       // n_faces * 2 element ids, ascending; -1 = none
    std::vector<int32_t> elem_face;   // n_elems * (dim+1): face opposite local vertex a
};

// Returns PM_EINVAL for a face shared by more than two elements.
int build_faces(const pm_mesh *m, Faces *F);

}  // namespace pm
