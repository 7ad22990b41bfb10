// Host-side plan of the hierarchical domain decomposition tree.
//
// The tree follows the HDD tree definition (Section 2.1): the root is the
// unit square, every node has two sons that split it into halves with a
// small shared interface gamma = d(omega_1) \ d(omega) (eq. gamma_def), and
// the construction recurses.  The split rule (the paper only asks for halves
// with a small interface) cuts the longer side at its midpoint, ties cut
// vertically, so the root interface is the midline x = 1/2.  Below the leaf
// size of the tree the recursion continues down to m x m-cell micro-blocks,
// which eliminate the leaf interior by nested dissection; the leaf level only
// matters to the caller as a granularity of the tree.
//
// Every node carries a dense "frame": the son-union index set ordered as
// [gamma ; Gamma ; rhs] (Gamma = boundary nodes of the node, outer Dirichlet
// nodes dropped above the micro level; rhs = one extra row holding the
// condensed load), size U+1 with U = |gamma| + |Gamma|.  This is the block
// system of eq. block_equation4 with the interface ordered first and the
// right-hand side appended as a row.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace hdd {

struct PlanOptions {
  int n = 0;            // interior nodes per side
  int leaf = 0;         // leaf size in cells
  int micro = 2;        // micro-block size in cells (2 or 4)
  bool keep_dirichlet = false;  // keep outer-boundary nodes in every Gamma
};

struct PlanNode {
  int x0, y0, w, h;     // rectangle in cells
  int depth;
  int index;            // index within its depth
  bool micro;           // micro-block (no sons)
  bool vertical;        // cut direction (sons: left/right if vertical)
  std::vector<int32_t> gam;  // global node ids of gamma (micro: interior)
  std::vector<int32_t> bnd;  // global node ids of Gamma, counter-clockwise from (x0, y0)
  int U() const { return int(gam.size() + bnd.size()); }
  int ld = 0;                 // leading dimension of the frame (>= U+1)
  int64_t frame_off = 0;      // offset (elements) within the level's per-sample block
  int64_t map_off = -1;       // offset into the level's map array (2 * (U+1) ints)
  int64_t ids_off = 0;        // offset into the level's id array (U ints)
};

struct PlanLevel {
  int depth;
  int gam;                    // |gamma| (same for all nodes of a level)
  int max_U;
  int max_bnd;
  int64_t frame_elems;        // per-sample elements of all frames of this level
  std::vector<PlanNode> nodes;
  std::vector<int32_t> maps;  // for node k: mapA[0..U], mapB[0..U] (son [Gamma;rhs] index or -1)
  std::vector<int32_t> ids;   // for node k: global ids of [gamma ; Gamma]
};

struct Plan {
  PlanOptions opt;
  int nc = 0;                 // cells per side
  int depth_micro = 0;        // depth of the micro-blocks
  int depth_leaf = 0;         // depth of the L x L leaves
  std::vector<PlanLevel> levels;  // index = depth (0 = root)
  std::string error;

  int node_id(int i, int j) const { return j * (nc + 1) + i; }
  bool dirichlet(int i, int j) const { return i == 0 || j == 0 || i == nc || j == nc; }
};

// Builds the plan; returns false with plan.error set on invalid options.
bool build_plan(const PlanOptions& opt, Plan& plan);

// Depth and index of the node whose rectangle is exactly the given cell
// rectangle, or false.
bool find_node(const Plan& plan, int x0, int y0, int w, int h, int* depth, int* index);

}  // namespace hdd
