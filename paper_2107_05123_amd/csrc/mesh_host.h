// Host-side octree mesh: leaves, independent nodes, hanging constraints and
// the brick decomposition that the device kernels stream over.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "chns.h"

namespace chns {

// Bricks are aligned cubes of B^d leaves of one level.  Class c holds
// bricks with B = 8 >> c (c = 3: single leaves).
constexpr int kBrickClasses = 4;
inline int brick_side(int c) { return 8 >> c; }

struct BrickClass {
  int B = 0;                    // leaves per brick edge
  int64_t count = 0;            // number of bricks
  int nodes_per_brick = 0;      // (B+1)^d
  int bnd_per_brick = 0;        // brick-boundary node positions
  int64_t slot_base = 0;        // first slot of this class
  std::vector<int32_t> table;   // count * nodes_per_brick gather entries
  std::vector<int8_t> level;    // count
  std::vector<int32_t> anchor;  // count * 3 (integer lower corner)
  std::vector<int32_t> rank;    // nodes_per_brick: boundary rank or -1 (interior)
  // 3D 8^3 bricks of a blocked node order: per brick the node numbers of the
  // 2x2x2 aligned 8^3 point blocks it touches, such that its node at
  // (jx, jy, jz) is base[(jx>>3) | (jy>>3)<<1 | (jz>>3)<<2] + (jx&7) +
  // 8 (jy&7) + 64 (jz&7) for all 9^3 of them; base[0] = -1 where that does
  // not hold (the table is used); empty for other classes
  std::vector<int32_t> abase;   // count * 8
};

struct HostMesh {
  int dim = 3;
  int max_level = 0;
  bool uniform = false;
  int node_order = 0;  // 0 lexicographic, 1 Morton, 2 blocked (8^d blocks in Morton order)

  // leaves in Morton order
  std::vector<int8_t> leaf_level;
  std::vector<int32_t> leaf_anchor;  // E * 3

  // independent nodes in vector order
  int64_t n_indep = 0;
  std::vector<int32_t> indep_coords;  // n_indep * 3

  // hanging nodes: coordinates and up to 4 parents (independent ids, -1 pad)
  int64_t n_hanging = 0;
  std::vector<int32_t> hang_coords;   // n_hanging * 3
  std::vector<int32_t> hang_parents;  // n_hanging * 4
  std::vector<int8_t> hang_npar;      // n_hanging

  BrickClass cls[kBrickClasses];
  int64_t n_slots = 0;

  // deterministic combine: shared node -> (slot | weight code) list
  std::vector<int32_t> comb_node;   // rows
  std::vector<int32_t> comb_ptr;    // rows + 1
  std::vector<uint32_t> comb_ent;   // slot (30 bits) | code << 30 (0: 1, 1: 1/2, 2: 1/4)
  // every independent node is either interior to exactly one brick or a combine row
  // node colours for probing the exact diagonal
  int n_colors = 0;
  std::vector<uint8_t> color;  // n_indep
  // Dirichlet wall mask (1 on the domain boundary)
  std::vector<uint8_t> wall;   // n_indep
  // domain: the box [0, box_hi[d]] (units of 2^-max_level); the whole cube
  // unless the octree is carved (carve_level > 0: the box is a union of
  // level-carve_level octants)
  int carve_level = 0;
  int32_t box_hi[3] = {0, 0, 0};

  int64_t n_elems() const { return (int64_t)leaf_level.size(); }
};

// Build everything from a spec; returns CHNS_OK or an error with msg set.
int build_host_mesh(const chns_mesh_spec& spec, HostMesh& m, std::string& msg);
// Build from an explicit leaf list (levels and anchors in units of 2^-max_level)
// inside the domain of `like` (its carving, rescaled to this max_level).
int build_host_mesh_from_leaves(int dim, int max_level, const std::vector<int8_t>& level,
                                const std::vector<int32_t>& anchor, HostMesh& m, std::string& msg,
                                const HostMesh* like = nullptr);
// Leaves of `fine` with every leaf deeper than k replaced by its level-k
// ancestor, in units of 2^-k (truncation keeps 2:1 balance).
void truncate_leaves(const HostMesh& fine, int k, std::vector<int8_t>& level, std::vector<int32_t>& anchor);

// Grid transfer between two meshes one level apart (coarse = fine truncated):
// P (fine rows) evaluates the coarse Q1 field, hanging constraints of both
// meshes included; R = P^T (coarse rows); I injects a fine nodal field into
// the coarse nodes (value of the fine field at the coarse node).
struct Transfer {
  std::vector<int32_t> P_ptr, P_col;
  std::vector<double> P_val;
  std::vector<int32_t> R_ptr, R_col;
  std::vector<double> R_val;
  std::vector<int32_t> I_ptr, I_col;
  std::vector<double> I_val;
};
int build_transfer(const HostMesh& fine, const HostMesh& coarse, Transfer& t, std::string& msg);

// Remeshing by the phase field: a new octree of the same dimension and
// max_level, refined to max_level wherever the nodal values of phi (old
// mesh, vector order) inside an octant's half-open box span a range meeting
// [-thr, thr], and to min_level elsewhere; 2:1 balanced.
int build_host_mesh_remesh(const HostMesh& old, const double* phi, int min_level, double thr, int brick_max,
                           HostMesh& out, std::string& msg);
// Intergrid transfer of nodal fields: row i (destination node i) evaluates
// the source Q1 field, hanging constraints included, at the node's
// position.  CSR with dst.n_indep rows and src.n_indep columns.
int build_interp(const HostMesh& src, const HostMesh& dst, std::vector<int32_t>& ptr, std::vector<int32_t>& col,
                 std::vector<double>& val, std::string& msg);

// Transfers between a 3D octree on the whole cube and the uniform node grid
// of level g ((2^g + 1)^3 points in lexicographic order, x fastest):
//   P (mesh nodes x grid points): the grid's Q1 field at every mesh node;
//   R = P^T (grid points x mesh nodes);
//   Q (grid points x mesh nodes): the mesh's Q1 field, hanging constraints
//   included, at every grid point.
struct GridTransfer {
  int level = 0;
  std::vector<int32_t> P_ptr, P_col, R_ptr, R_col, Q_ptr, Q_col;
  std::vector<double> P_val, R_val, Q_val;
};
int build_grid_transfer(const HostMesh& m, int g, GridTransfer& t, std::string& msg);

}  // namespace chns
