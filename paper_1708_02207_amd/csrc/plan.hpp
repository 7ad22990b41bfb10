// Host-side plan of the hierarchical domain decomposition tree.
//
// The tree follows the HDD tree definition (Section 2.1): the root is the
// unit square, every node has two sons that split it into halves with a
// small shared interface gamma = d(omega_1) \ d(omega) (eq. gamma_def), and
// the construction recurses.  The split rule (the paper only asks for halves
// with a small interface) cuts the longer side at its midpoint, ties cut
// vertically, so the root interface is the midline x = 1/2.
//
// The global plan stops at s x s-cell "block" nodes (s = min(16, leaf)).
// Below a block the recursion continues down to 2 x 2-cell micro-blocks, but
// all blocks share one local template: inside a block every boundary node is
// kept (outer Dirichlet nodes included), so the block's sub-tree, its index
// maps and its storage offsets are identical for every block.  One workgroup
// eliminates (and later solves) a whole block in LDS; this is the in-leaf
// nested dissection that eliminates a leaf's interior.
//
// Every node carries a dense "frame": the son-union index set ordered as
// [gamma ; Gamma ; rhs] (Gamma = boundary nodes of the node, outer Dirichlet
// nodes dropped above the block level; rhs = one extra row holding the
// condensed load), size U+1 with U = |gamma| + |Gamma|.  This is the block
// system of eq. block_equation4 with the interface ordered first and the
// right-hand side appended as a row.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace hdd {

struct PlanOptions {
  int n = 0;                    // interior nodes per side
  int leaf = 0;                 // leaf size in cells
  int block = 16;               // largest block handled in LDS (cells per side)
  bool keep_dirichlet = false;  // keep outer-boundary nodes in every Gamma
};

struct PlanNode {
  int x0, y0, w, h;     // rectangle in cells
  int depth;
  int index;            // index within its depth
  bool block;           // block node (deepest global level)
  bool vertical;        // cut direction (sons: left/right if vertical)
  std::vector<int32_t> gam;  // global node ids of gamma
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

// Local sub-tree of one s x s block (level 0 = the block, last = micro-blocks).
struct SubLevel {
  int n;          // nodes on this level
  int gam, bnd;   // |gamma|, |Gamma| (uniform on the level, Dirichlet kept)
  int U;          // gam + bnd
  int fsz;        // frame elements in LDS: U+1 rows, packed lower triangle
  int cst_off;    // offset of the level's retained blocks in a block's compact store
  int vec_off;    // offset of the level's z values in a block's vector store
  int map_off;    // into maps: node t uses maps[map_off + t*2*(U+1) ...] (levels above micro)
  int lid_off;    // into lids: node t uses lids[lid_off + t*U ...]
};

struct SubTemplate {
  int s = 0;                    // cells per side
  std::vector<SubLevel> lv;     // 0 = block root
  std::vector<int32_t> maps;    // son [Gamma;rhs] index (or -1) per father frame row
  std::vector<int32_t> lids;    // local node id b*(s+1)+a of [gamma ; Gamma] per node
  std::vector<int32_t> micro_xy;// micro-blocks: local lower-left corner (a0, b0) pairs
  int cst_size = 0;             // compact elements per block: sum n (U+1) gam
  int vec_size = 0;             // z elements per block: sum n gam = (s-1)^2
  int max_buf = 0;              // max over levels of n * fsz
  int max_gam_nodes = 0;        // max over levels of n * gam
  int max_bnd_nodes = 0;        // max over levels of n * (U)
};

struct Plan {
  PlanOptions opt;
  int nc = 0;                 // cells per side
  int depth_block = 0;        // depth of the blocks (deepest global level)
  int depth_leaf = 0;         // depth of the L x L leaves
  std::vector<PlanLevel> levels;  // index = depth (0 = root)
  SubTemplate sub;
  std::string error;

  int node_id(int i, int j) const { return j * (nc + 1) + i; }
  bool dirichlet(int i, int j) const { return i == 0 || j == 0 || i == nc || j == nc; }
};

// Builds the plan; returns false with plan.error set on invalid options.
bool build_plan(const PlanOptions& opt, Plan& plan);

// Algorithmic flops of one build: sum over all nodes of the tree down to the
// 2 x 2-cell micro-blocks (outer Dirichlet nodes dropped) of
// g^3/3 + g^2 G + g G^2 (interface factorization, solve, Schur update).
double algorithmic_flops(int n);

}  // namespace hdd
