// Device-side data structures and helpers shared by the HDD kernels.
//
// Frame layout (one per tree node and parameter sample): a dense row-major
// (U+1) x ld block whose rows and columns are ordered [gamma ; Gamma ; rhs].
// Only the lower triangle is meaningful.  After the elimination of a node the
// frame holds, in place:
//   rows/cols [0, g)          L, the Cholesky factor of the interface block
//   rows [g, U), cols [0, g)  P = S_Gamma,gamma L^-T
//   row U, cols [0, g)        z = L^-1 (condensed interface load)
//   rows/cols [g, U]          S_omega (Schur complement on Gamma) and, in row
//                             U, the condensed boundary load g_omega
// which is the retained map Phi of the node (Section 2.4: Phi^g = -A22^-1 A21,
// Phi^f = A22^-1 F2, here kept in factored form) and the map Psi passed to
// the father (Psi^g = A11 - A12 A22^-1 A21, Psi^f = F1 - A12 A22^-1 F2).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hdd {

struct DevNode {
  long long frame_off;  // elements within the level's per-sample block
  long long map_off;    // into the level's map array (2 * (U+1) ints), -1 at micro level
  int U;                // |gamma| + |Gamma|
  int bnd;              // |Gamma|
  int ld;               // frame leading dimension
  int ids_off;          // into the level's id array ([gamma ; Gamma] global node ids)
  int x0, y0;           // lower-left cell of the node's rectangle
  long long panel_off;  // elements within the level's per-sample panel block (levels with a panel store)
  int cw, ch;           // width and height of the rectangle in cells
};

struct DevLevel {
  void* frames;          // float* or double*
  long long stride;      // per-sample elements of this level
  // Panel store: the retained columns [L ; P ; z] of every node, (U+1) x
  // gamma per node with row stride panel_ld (zero above the diagonal of L), kept
  // after the build while the frames are reused; the sweeps read contiguous
  // rows.  nullptr for the block level, and, in handles that keep all frames,
  // for the levels whose frames hold the retained columns.
  void* panel;
  long long panel_stride;  // per-sample elements of the panel store
  int panel_ld;            // row stride of the panel store: gamma rounded up to 4 (16-byte rows)
  // Block low-rank copy of the maps P of the level (HDD_FLAG_LOWRANK), used
  // by the refinement sweeps; lr_store is nullptr on levels without it.
  const int* lr_perm;    // parallel to ids: at ids_off + gamma + k the Gamma position of row k (perimeter order)
  const int* lr_node;    // [n_nodes + 1]: first block of every node (blocks row-major over 64 x 64 blocks)
  const int4* lr_blk;    // per block: (0 dense / 1 low rank, offset in a sample's store, node, bi << 16 | bj)
  void* lr_store;        // [sample][...] float or double: dense blocks 64 x 64, low-rank U (64 x kr) then V (kr x 64)
  long long lr_stride;   // per-sample elements of lr_store
  int* lr_rank;          // [sample][block] rank of the low-rank blocks
  int lr_nblk;           // blocks of the level
  const DevNode* nodes;
  const int* maps;
  const int* ids;
  double* vec;           // forward-pass vectors [sample][sum U] (refinement)
  long long vec_stride;  // per-sample elements of vec
  int n_nodes;
  int gam;
  int max_U;
  int is_double;
  int depth;
  int node_base;         // global index of this level's first node (for error reports)
};

// One level of the shared s x s block sub-tree (level 0 = the block).
struct DevSubLevel {
  int n, gam, bnd, U, fsz, cst_off, vec_off, map_off, lid_off;
};
constexpr int kMaxSubLevels = 12;

// Everything the block kernels need: the sub-tree template, the compact
// stores and the global level of the blocks.
struct DevBlocks {
  DevSubLevel lv[kMaxSubLevels];
  int nlev;           // sub-tree levels
  int s;              // cells per block side
  int nb;             // blocks per sample
  int cst_size;       // compact elements per block
  int vec_size;       // z values per block
  int max_buf;        // LDS frame elements per buffer
  int max_gam_nodes;  // max n * gam over levels
  int max_bnd_nodes;  // max n * U over levels
  int no_mfma;        // in-block Schur updates without matrix cores (cross-check)
  const int* maps;
  const int* lids;
  const int* micro_xy;
  const unsigned* ext;  // merge tables of the block build and forward kernels (see k_block_ext)
  const int* origin;  // [nb][2] lower-left cell of every block
  void* cst;          // [sample][block][cst_size], float or double
  long long cst_stride;
  double* vec;        // [sample][block][vec_size]
  long long vec_stride;
  DevLevel top;       // the global level made of the blocks
};

template <typename T> __device__ __forceinline__ T* frame_ptr(const DevLevel& L, int node, int s) {
  return reinterpret_cast<T*>(L.frames) + (long long)s * L.stride + L.nodes[node].frame_off;
}

// A node's block of the level's panel store ((U+1) x gamma, row stride panel_ld).
template <typename T> __device__ __forceinline__ T* panel_ptr(const DevLevel& L, int node, int s) {
  return reinterpret_cast<T*>(L.panel) + (long long)s * L.panel_stride + L.nodes[node].panel_off;
}

// Retained columns [L ; P ; z] of a node and their row stride: the panel
// store when the level has one, else the frame's first gamma columns.
template <typename T> __device__ __forceinline__ T* retained_ptr(const DevLevel& L, int node, int s, int& ld) {
  if (L.panel) {
    ld = L.panel_ld;
    return reinterpret_cast<T*>(L.panel) + (long long)s * L.panel_stride + L.nodes[node].panel_off;
  }
  ld = L.nodes[node].ld;
  return frame_ptr<T>(L, node, s);
}

__device__ __forceinline__ int tri_row(long long e) {
  // row r of the lower-triangle element with flat index e (row-major lower order)
  int r = int((sqrt(8.0 * double(e) + 1.0) - 1.0) * 0.5);
  while ((long long)(r + 1) * (r + 2) / 2 <= e) ++r;
  while ((long long)r * (r + 1) / 2 > e) --r;
  return r;
}

}  // namespace hdd
