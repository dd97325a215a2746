// Host-side mesh, node numbering, hanging-node constraints, node-graph sparsity and the
// node-centric assembly tables.
#pragma once
#include <cstdint>
#include <array>
#include <vector>

#include "../../include/fracture.h"

namespace fr {

struct HostMesh {
    int dim = 2, nv = 4;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    double h_min = 0;                   // edge of the finest cell (lattice unit)
    int64_t n_nodes = 0, n_cells = 0, n_free = 0, n_hanging = 0;
    std::vector<double> coords;         // [n_nodes][dim]
    std::vector<int64_t> lattice;       // [n_nodes][dim], units of h_min
    std::vector<int32_t> cells;         // [n_cells][nv], vertex a at lower corner + bits(a) * size
    std::vector<double> cell_lo;        // [n_cells][dim]
    std::vector<double> cell_h;         // [n_cells]
    std::vector<uint8_t> dirichlet;     // [n_nodes]
    std::vector<int32_t> free_of_node;  // [n_nodes], -1 for hanging nodes
    std::vector<int32_t> node_of_free;  // [n_free]
    // Conformity: value(node) = sum_j con_w[j] * value(free con_master[j]), j in [con_ptr[n], con_ptr[n+1]).
    std::vector<int32_t> con_ptr, con_master;
    std::vector<double> con_w;
    // Independent instances stored as a disjoint union (instance-major numbering of nodes,
    // cells and free nodes); one instance: n_inst = 1 and the offsets are {0, total}.
    int n_inst = 1;
    std::vector<int64_t> node_off, cell_off, free_off;   // [n_inst+1]
    std::vector<double> inst_h_min;                        // [n_inst]
    // The descriptor this mesh was built from (one instance) and its number of levels (the
    // lattice unit is the base cell edge / 2^levels); a refined mesh records its own.
    fr_mesh_desc desc{};
    int levels = 0;
};

// Node-graph pattern in SELL-C layout plus the tables of the node-centric assembly.
struct Pattern {
    int C = 64;
    int64_t n_rows = 0, n_slices = 0, n_slots = 0, nnz = 0;
    int max_row = 0;
    std::vector<int32_t> slice_ptr;   // [n_slices+1] first slot of each slice
    std::vector<int32_t> row_len;     // [n_rows]
    std::vector<int32_t> col;         // [n_slots] column (free node); padding points at the row itself
    // Row entries: the cells (and local vertex) where the row's basis function lives.
    std::vector<int32_t> ent_ptr;     // [n_rows+1]
    std::vector<int32_t> ent_cell;    // [n_ent]
    std::vector<uint8_t> ent_a;       // [n_ent] local vertex of the row node (or of its hanging dependent)
    std::vector<double> ent_w;        // [n_ent] weight of the row's basis function at that vertex
    std::vector<uint8_t> ent_k;       // [n_ent][nv] position of vertex b's node in the row, 255 = hanging
    // Hanging vertices (ent_k == 255): row positions of their masters, in the order the row
    // meets them (entries, then vertices b, then the vertex's constraint masters).  Empty
    // without hanging nodes.
    std::vector<int32_t> hang_ptr;    // [n_rows+1]
    std::vector<uint8_t> hang_k;      // [hang_ptr[n_rows]]
};

// Cells to split on top of a descriptor's base grid: every cell of level l whose lattice
// origin is listed in split[l] is split (origins in units of the finest cell of a mesh with L
// levels); the 2:1 closure then runs as for the descriptor's own rule, which the seed replaces.
struct RefineSeed {
    int L = 0;
    std::vector<std::vector<uint64_t>> split;   // [L] packed origins (21 bits per axis) of split cells
};

HostMesh build_mesh(const fr_mesh_desc& d, const RefineSeed* seed = nullptr);

// The mesh obtained from `old` (one instance) by splitting every cell c with flags[c] != 0,
// then the 2:1 closure.  loc_cell[n] / loc_xi[n*dim + k]: a cell of `old` that contains node n
// of the result and the node's local coordinates in it (in [0, 1]).
HostMesh refine_mesh(const HostMesh& old, const uint8_t* flags, std::vector<int32_t>& loc_cell,
                     std::vector<double>& loc_xi);
// Disjoint union of n independent meshes of the same dimension.
HostMesh build_mesh_batch(const fr_mesh_desc* d, int n);

// Face neighbours of every cell (one instance or a batch): for face j = 2k + side (axis k,
// side 0 = low, 1 = high) of cell c the cells across it are nbr[ptr[2 dim c + j] ..
// ptr[2 dim c + j + 1]): none on the domain boundary, one of the same or the next coarser level,
// or the 2^(dim-1) cells of the next finer level (2:1 balance).
void face_neighbors(const HostMesh& m, std::vector<int32_t>& ptr, std::vector<int32_t>& nbr);
Pattern build_pattern(const HostMesh& m, int C);

}  // namespace fr
