// In-LDS nested dissection of s x s-cell blocks (the leaf interior).
//
// One workgroup handles one (block, sample).  All blocks share one local
// sub-tree (outer Dirichlet nodes are kept inside a block), so every level
// has n nodes of identical shape, known at compile time from the block size
// S, and the whole level is processed in parallel with workgroup barriers.
// Level k (0 = the block) has 2^k nodes of (S >> ((k+1)/2)) x (S >> (k/2))
// cells; the last level holds the 2 x 2-cell micro-blocks.
//
//  k_block_build     Section 3.1 (leaf assembly, eq. coefA, eq. coefc) and
//                    Sections 2.4 / 3.3 (Schur elimination and merge of
//                    sons) for every level of the block, bottom-up.  Frames
//                    live in two ping-pong LDS buffers; from each node's
//                    factored columns [L ; P ; z] the kernel forms the node's
//                    local operators M = A_gg^-1, W = A_gg^-1 A_gG and
//                    y = A_gg^-1 b_gamma and writes them to a compact HBM
//                    store; the block root's full frame (with S_omega and
//                    g_omega) goes to the global frame store.
//  k_block_topdown   Root to Leaves inside the block (Section 3.4): from u on
//                    the block boundary, every interface of the block, one
//                    GEMV per level (u_gamma = y - W u_Gamma).
//  k_block_forward   bottom-up propagation of a new load (the residual of the
//                    refinement) through the block's operators.
#include <algorithm>
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace hdd {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int NT = 256;   // threads of the top-down / forward kernels
constexpr int NTB = 512;  // threads of the build kernel

// ---------------------------------------------------------------------------
// Local systems of the micro-blocks (Section 3.1): 2 x 2 cells, 8 triangles,
// 9 nodes numbered in the frame as
//      y=2:  7 6 5
//      y=1:  8 0 4        (0 = the micro-block's interface node)
//      y=0:  1 2 3
// Every entry of the packed 10-row frame (rows 0..8 the nodes, row 9 the
// load) is a fixed combination of the 8 triangle coefficients (eq. coefA:
// kappa_T (grad phi_a . grad phi_b) |T|, in cell units) or of the nodal load
// (eq. coefc, vertex rule: |T| / 3 per triangle at the node).  The
// combinations are tabulated at compile time; triangle tr = (cb*2 + ca)*2 + tri
// of cell (ca, cb) has the vertices (0,0),(1,0),(1,1) (tri 0) or
// (0,0),(1,1),(0,1) (tri 1) relative to the cell corner.
struct MicroTable {
  int nt[45];         // nonzero terms of stiffness entry e (packed (r, c), c <= r < 9)
  int tr[45][6];      // their triangles
  double co[45][6];   // and coefficients
  int cnt[9];         // triangles at node c
  int nx[9], ny[9];   // local coordinates of node c
};

constexpr MicroTable make_micro_table() {
  MicroTable m{};
  const int fidx[3][3] = {{1, 2, 3}, {8, 0, 4}, {7, 6, 5}};  // [y][x]
  for (int y = 0; y < 3; ++y)
    for (int x = 0; x < 3; ++x) {
      m.nx[fidx[y][x]] = x;
      m.ny[fidx[y][x]] = y;
    }
  for (int cb = 0; cb < 2; ++cb)
    for (int ca = 0; ca < 2; ++ca)
      for (int tri = 0; tri < 2; ++tri) {
        const int tr = (cb * 2 + ca) * 2 + tri;
        const int vx[3] = {ca, ca + 1, tri == 0 ? ca + 1 : ca};
        const int vy[3] = {cb, tri == 0 ? cb : cb + 1, cb + 1};
        const int det = (vx[1] - vx[0]) * (vy[2] - vy[0]) - (vx[2] - vx[0]) * (vy[1] - vy[0]);
        const int gx[3] = {vy[1] - vy[2], vy[2] - vy[0], vy[0] - vy[1]};
        const int gy[3] = {vx[2] - vx[1], vx[0] - vx[2], vx[1] - vx[0]};
        for (int a = 0; a < 3; ++a) {
          const int ia = fidx[vy[a]][vx[a]];
          m.cnt[ia] += 1;
          for (int b = 0; b < 3; ++b) {
            const int ib = fidx[vy[b]][vx[b]];
            const int num = gx[a] * gx[b] + gy[a] * gy[b];
            if (ib <= ia && num != 0) {
              const int e = ia * (ia + 1) / 2 + ib;
              m.tr[e][m.nt[e]] = tr;
              m.co[e][m.nt[e]] = double(num) / (2.0 * double(det < 0 ? -det : det));
              m.nt[e] += 1;
            }
          }
        }
      }
  return m;
}
constexpr MicroTable kMicro = make_micro_table();

template <int E, int Q> __device__ __forceinline__ double micro_sum(const double (&kap)[8]) {
  constexpr double c = kMicro.co[E][Q];
  constexpr int tr = kMicro.tr[E][Q];
  if constexpr (Q + 1 < kMicro.nt[E]) return c * kap[tr] + micro_sum<E, Q + 1>(kap);
  else return c * kap[tr];
}

// Entries E, E + NW, ... of the frame of micro-block t (wave wv takes the
// entries with E % NW == wv, one micro-block per lane).
template <typename T, int S, int E>
__device__ __forceinline__ void micro_entries(T* F, const double (&kap)[8], const double* fL, int a0, int b0,
                                              double area3, bool act, int wv) {
  if constexpr (E < 55) {
    if (E % (NTB / 64) == wv) {
      double v = 0.0;
      if constexpr (E < 45) {
        if constexpr (kMicro.nt[E] > 0) v = micro_sum<E, 0>(kap);
      } else if constexpr (E < 54) {
        constexpr int c = E - 45;
        v = double(kMicro.cnt[c]) * area3 * fL[(b0 + kMicro.ny[c]) * (S + 1) + a0 + kMicro.nx[c]];
      }
      if (act) F[E] = T(v);
    }
    micro_entries<T, S, E + 1>(F, kap, fL, a0, b0, area3, act, wv);
  }
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

template <int S, int K> struct Lv {
  static constexpr int Lm = 2 * ilog2c(S / 2);  // micro level
  static constexpr int w = S >> ((K + 1) / 2);
  static constexpr int h = S >> (K / 2);
  static constexpr int n = 1 << K;
  static constexpr int gam = (K == Lm) ? 1 : (w >= h ? h - 1 : w - 1);
  static constexpr int bnd = 2 * (w + h);
  static constexpr int U = gam + bnd;
  static constexpr int ld = U + 1;              // frame rows
  static constexpr int fsz = ld * (ld + 1) / 2;   // LDS elements per frame: packed lower triangle
  __host__ __device__ static constexpr int row(int r) { return r * (r + 1) / 2; }  // start of row r
  static constexpr int per = ld * gam;            // compact elements per node
};


// Extend-add gather table of the build kernel.  Every block shares the
// sub-tree, so the LDS addresses of the extend-add are the same for all of
// them.  Entry e of level K (K above the micro level) is element e of the
// level's packed frames (node t, row r, column c <= r, in that order) and
// holds the two son elements merged into it, a | b << 16, as element offsets
// from the start of the kernel's LDS frame buffers: a (b) the son-A (son-B)
// element, or the zero slot 2 * max_buf when the row or column is not in that
// son (Section 2.4, eq. S_omega).  Level K's frames live in buffer
// (Lm - K) & 1.
template <int S, int K> constexpr int ext_count() {
  using L = Lv<S, K>;
  return (K < L::Lm) ? L::n * L::ld * (L::ld + 1) / 2 : 0;
}
template <int S, int K> constexpr int ext_off() {
  if constexpr (K == 0) return 0;
  else return ext_off<S, K - 1>() + ext_count<S, K - 1>();
}
template <int S> constexpr int ext_total() { return ext_off<S, Lv<S, 0>::Lm>(); }

template <int S, int K>
__device__ __forceinline__ void ext_entry(const DevBlocks& B, int e, unsigned* out) {
  using L = Lv<S, K>;
  if constexpr (K < L::Lm) {
    if (e >= ext_count<S, K>()) {
      ext_entry<S, K + 1>(B, e - ext_count<S, K>(), out);
      return;
    }
    using C = Lv<S, K + 1>;
    constexpr int tri = L::ld * (L::ld + 1) / 2;
    const int t = e / tri, rc = e % tri;
    const int r = tri_row(rc), c = rc - r * (r + 1) / 2;
    const int zero = 2 * B.max_buf;
    const int prev = ((L::Lm - K + 1) & 1) * B.max_buf;
    const int* mA = B.maps + B.lv[K].map_off + t * 2 * L::ld;
    const int* mB = mA + L::ld;
    const int sa = prev + (2 * t) * C::fsz + C::gam, sb = sa + C::fsz;  // + row(gam + r') + c' of S~
    const int ar = mA[r], ac = mA[c], br = mB[r], bc = mB[c];
    const int a = (ar >= 0 && ac >= 0) ? sa + C::row(C::gam + max(ar, ac)) + min(ar, ac) : zero;
    const int b = (br >= 0 && bc >= 0) ? sb + C::row(C::gam + max(br, bc)) + min(br, bc) : zero;
    out[ext_off<S, K>() + e] = unsigned(a) | (unsigned(b) << 16);
  }
}

// Merge table of the forward sweep: entry e = t * U + i of level K adds the
// sons' condensed loads, a | b << 16 as offsets from the start of the
// kernel's two LDS value buffers (max_bnd_nodes each; level K's values live
// in buffer (Lm - K) & 1), the zero slot 2 * max_bnd_nodes where row i is not
// in that son.  Stored after the build's table.
template <int S, int K> constexpr int fext_count() {
  using L = Lv<S, K>;
  return (K < L::Lm) ? L::n * L::U : 0;
}
template <int S, int K> constexpr int fext_off() {
  if constexpr (K == 0) return 0;
  else return fext_off<S, K - 1>() + fext_count<S, K - 1>();
}
template <int S> constexpr int fext_total() { return fext_off<S, Lv<S, 0>::Lm>(); }

template <int S, int K>
__device__ __forceinline__ void fext_entry(const DevBlocks& B, int e, unsigned* out) {
  using L = Lv<S, K>;
  if constexpr (K < L::Lm) {
    if (e >= fext_count<S, K>()) {
      fext_entry<S, K + 1>(B, e - fext_count<S, K>(), out);
      return;
    }
    using C = Lv<S, K + 1>;
    const int t = e / L::U, i = e % L::U;
    const int zero = 2 * B.max_bnd_nodes;
    const int prev = ((L::Lm - K + 1) & 1) * B.max_bnd_nodes;
    const int* mA = B.maps + B.lv[K].map_off + t * 2 * L::ld;
    const int* mB = mA + L::ld;
    const int a = mA[i] >= 0 ? prev + (2 * t) * C::U + C::gam + mA[i] : zero;
    const int b = mB[i] >= 0 ? prev + (2 * t + 1) * C::U + C::gam + mB[i] : zero;
    out[ext_total<S>() + fext_off<S, K>() + e] = unsigned(a) | (unsigned(b) << 16);
  }
}

template <int S> __global__ void k_block_ext(DevBlocks B, unsigned* __restrict__ ext) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ext_total<S>()) ext_entry<S, 0>(B, e, ext);
  else if (e < ext_total<S>() + fext_total<S>()) fext_entry<S, 0>(B, e - ext_total<S>(), ext);
}


template <typename T> __device__ __forceinline__ T* cst_block(const DevBlocks& B, int q, int s) {
  return reinterpret_cast<T*>(B.cst) + (long long)s * B.cst_stride + (long long)q * B.cst_size;
}

// Largest n * gam^2 over the levels of a block (the X = L_gg^-1 blocks).
template <int S, int K> constexpr int inv_size_from() {
  using L = Lv<S, K>;
  constexpr int m = L::n * L::gam * L::gam;
  if constexpr (K < L::Lm) {
    constexpr int rest = inv_size_from<S, K + 1>();
    return m > rest ? m : rest;
  } else {
    return m;
  }
}


// ---------------------------------------------------------------------------
// Partial Cholesky of the first gam columns of every frame of a level in
// registers (Section 2.4, eq. SchurC1 with the pivots of eq. Phi): a group
// of GS lanes per node, lane j holding row j (first gam entries).
// Right-looking: column J is scaled by 1 / L_JJ, then the later columns k of
// every row take A_rk -= L_rJ L_kJ, with L_JJ and L_kJ sent to the group by
// cross-lane reads (rows J, k < gam sit in the group's first lanes).  The
// same lanes then form X = L_gg^-1 row by row (X_kk = 1 / L_kk,
// X_ic = -(sum_k L_ik X_kc) / L_ii) and leave it in xs[node][gam][gam].
// No barriers inside; frames are read from and written back to LDS.  A
// frame of more than 64 rows (the block root) has its remaining rows done
// by chol_tail.
template <typename L> struct CholCfg {
  static constexpr int R = L::U + 1;  // rows: gamma, Gamma, load
  static constexpr int GS = R > 32 ? 64 : (R > 16 ? 32 : (R > 8 ? 16 : (R > 4 ? 8 : 4)));
  static constexpr int RR = R < 64 ? R : 64;  // rows held in registers (one per lane)
  static constexpr int NPW = 64 / GS;         // nodes per wave
  static constexpr int WAVES = (L::n + NPW - 1) / NPW;
};

template <typename T, int GS>
__device__ __forceinline__ T group_read(T v, int src_lane) {
  if constexpr (GS == 64) {  // wave-uniform source: through the scalar unit
    if constexpr (sizeof(T) == 8) {
      const long long b = __double_as_longlong(double(v));
      const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), src_lane);
      const int hi = __builtin_amdgcn_readlane(int(b >> 32), src_lane);
      return T(__longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo)));
    } else {
      return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(float(v)), src_lane));
    }
  } else {
    return __shfl(v, src_lane);
  }
}

template <typename T, typename L>
__device__ __forceinline__ void chol_regs(T* cur, T* xs, int& bad_pivot) {
  using C = CholCfg<L>;
  constexpr int g = L::gam, GS = C::GS;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = lane % GS;
  const int gbase = lane - j;
  for (int w0 = 0; w0 < C::WAVES; w0 += NTB / 64) {  // uniform
    const int t = (w0 + wv) * C::NPW + lane / GS;
    if (w0 + wv >= C::WAVES) break;  // wave-uniform
    const bool act = t < L::n;
    T* F = cur + (act ? t : 0) * L::fsz;
    const int r = min(j, C::RR - 1);
    T a[g];
#pragma unroll
    for (int c = 0; c < g; ++c) a[c] = F[L::row(r) + c];  // c > r: unused
    // Entries above the diagonal (a[c], c > j) are updated like the others
    // but never read back or written out, so no masks are needed.
    T rdj = T(1);  // 1 / L_jj in lane j < g
#pragma unroll
    for (int J = 0; J < g; ++J) {
      const T p = group_read<T, GS>(a[J], GS == 64 ? J : gbase + J);
      const bool ok = (p > T(0)) && (p < T(1e300));
      if (!ok && act) bad_pivot = 1;
      const T d = ok ? T(sqrt(p)) : T(1);  // correctly rounded: the refinement's
      const T rd = T(1) / d;               // contraction depends on these pivots
      if (j == J) rdj = rd;
      a[J] = j == J ? d : a[J] * rd;
#pragma unroll
      for (int k = J + 1; k < g; ++k) {
        const T lk = group_read<T, GS>(a[J], GS == 64 ? k : gbase + k);  // L_kJ
        a[k] -= a[J] * lk;
      }
    }
    if (act && j < C::RR) {
#pragma unroll
      for (int c = 0; c < g; ++c)
        if (c <= j) F[L::row(j) + c] = a[c];
    }
    // X = L_gg^-1: lane i accumulates v_c = -sum_{k<i} L_ik X_kc, finishes
    // its row at step k = i and stores it then (later updates of a finished
    // row are harmless)
    T v[g];
#pragma unroll
    for (int c = 0; c < g; ++c) v[c] = T(0);
    T* X = xs + (act ? t : 0) * g * g + min(j, g - 1) * g;
#pragma unroll
    for (int k = 0; k < g; ++k) {
      if (j == k) {
        v[k] += T(1);
#pragma unroll
        for (int c = 0; c <= k; ++c) v[c] *= rdj;
        if (act) {
#pragma unroll
          for (int c = 0; c < g; ++c) X[c] = c <= k ? v[c] : T(0);
        }
      }
#pragma unroll
      for (int c = 0; c <= k; ++c) {
        const T xk = group_read<T, GS>(v[c], GS == 64 ? k : gbase + k);  // X_kc
        v[c] -= a[k] * xk;
      }
    }
  }
  __syncthreads();
}

// Rows 64 .. U of a frame with more than 64 rows: L_rJ = sum_{l<=J} A_rl X_Jl
// (one output per thread, written after a barrier since the row is read).
template <typename T, typename L>
__device__ __forceinline__ void chol_tail(T* cur, const T* xs) {
  constexpr int g = L::gam, R = L::U + 1;
  if constexpr (R > 64) {
    static_assert(L::n == 1, "frames of more than 64 rows: one node per level");
    constexpr int NO = (R - 64) * g;
    static_assert(NO <= NTB, "tail rows fit the workgroup");
    const int e = threadIdx.x;
    T val = T(0);
    const int r = 64 + min(e, NO - 1) / g, J = min(e, NO - 1) % g;
    if (e < NO) {
      for (int l = 0; l <= J; ++l) val += cur[L::row(r) + l] * xs[J * g + l];
    }
    __syncthreads();
    if (e < NO) cur[L::row(r) + J] = val;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Build: one level (extend-add from the sons in `prev`, eliminate in `cur`).
template <typename T, int S, int K> constexpr int ext_regs() {
  return ext_count<S, K>() > 0 ? (ext_count<S, K>() + NTB - 1) / NTB : 1;
}

// Build: one level (extend-add from the sons in `prev`, eliminate in `cur`).
// `tab` holds this thread's entries of the level's gather table, loaded into
// registers while the level below was being eliminated.
template <typename T, int S, int K>
__device__ __forceinline__ void build_level(T* base, T* cur, T* cst, const DevBlocks& B, T* xs, int& bad_pivot,
                                            const unsigned (&tab)[ext_regs<T, S, K>()]) {
  using L = Lv<S, K>;
  const int tid = threadIdx.x;
  constexpr int NB = NTB;
  if constexpr (K < L::Lm) {
    // S_omega = S~_A + S~_B (eq. S_omega): all gathers of the thread, then
    // all stores (the table's elements of one level never overlap)
    constexpr int E = ext_count<S, K>(), NP = ext_regs<T, S, K>();
    T v[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) v[j] = base[tab[j] & 0xffffu] + base[tab[j] >> 16];
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (j + 1 < NP || tid + NB * j < E) cur[tid + NB * j] = v[j];
    __syncthreads();
  }
  // Partial Cholesky of the first gam columns: L (interface rows), P
  // (boundary rows) and z (load row) of every node.
  constexpr int g = L::gam;
  chol_regs<T, L>(cur, xs, bad_pivot);
  chol_tail<T, L>(cur, xs);
  // Schur update of the boundary block and the load row (rank-g, eq.
  // SchurC1): S[i][l] -= sum_k P[i][k] P[l][k], g <= l <= i <= U.
  // One thread per row i >= g: its P entries in registers, the columns
  // l = g .. i unrolled (compile-time offsets; P rows l read by every thread
  // of the node at once).
  auto schur_rows = [&]() {
    constexpr int nr = L::U + 1 - g;
    for (int e = tid; e < L::n * nr; e += NB) {
      const int t = e / nr, i = g + e % nr;
      T* F = cur + t * L::fsz;
      T* Fi = F + L::row(i);
      T pi[g];
#pragma unroll
      for (int k = 0; k < g; ++k) pi[k] = Fi[k];
#pragma unroll
      for (int l = g; l <= L::U; ++l) {
        if (l <= i) {
          T acc = T(0);
#pragma unroll
          for (int k = 0; k < g; ++k) acc += pi[k] * F[L::row(l) + k];
          Fi[l] -= acc;
        }
      }
    }
  };
  if constexpr (std::is_same<T, float>::value && g >= 7) {
    if (!B.no_mfma) {  // uniform
      // matrix cores: 32 x 32 tiles of the lower triangle, one wave per tile,
      // K = g padded to even with zeros; P read from the frame in LDS
      constexpr int nr = L::U + 1 - g;
      constexpr int nt = (nr + 31) / 32;
      constexpr int tiles = L::n * nt * (nt + 1) / 2;
      const int lane = tid & 63, wv = tid >> 6;
      for (int q = wv; q < tiles; q += NB / 64) {
        const int t = q / (nt * (nt + 1) / 2), tq = q % (nt * (nt + 1) / 2);
        const int ti = tri_row(tq), tj = tq - ti * (ti + 1) / 2;
        T* F = cur + t * L::fsz;
        // rows beyond U are clamped: they only feed accumulator rows and
        // columns that are not written back
        const int ra = g + ti * 32 + (lane & 31), rb = g + tj * 32 + (lane & 31);
        const T* pa = F + L::row(min(ra, L::U)) + (lane >> 5);
        const T* pb = F + L::row(min(rb, L::U)) + (lane >> 5);
        floatx16 acc;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
        for (int kk = 0; kk < g; kk += 2) {
          float av = pa[kk], bv = pb[kk];
          if (kk + 1 == g) av = (lane >> 5) ? 0.f : av;  // odd g: column g is not in P
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
        }
        // accumulator v of this lane: row i0 + d(v), column l
        const int l = g + tj * 32 + (lane & 31);
        const int i0 = g + ti * 32 + (lane >> 5) * 4;
        T* Fl = F + L::row(i0) + l;
        const bool edge = ti == tj || g + ti * 32 + 31 > L::U;  // wave-uniform
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int d = (v >> 2) * 8 + (v & 3);
          // row(i0 + d) = row(i0) + d * i0 + d (d + 1) / 2
          T* p = Fl + d * i0 + d * (d + 1) / 2;
          if (!edge || (i0 + d <= L::U && l <= i0 + d)) *p -= acc[v];
        }
      }
    } else {
      schur_rows();
    }
  } else {
    schur_rows();
  }
  __syncthreads();
  // Local operators of every node -> compact store, g values per row
  // (Section 3.4: the interface values of a node follow from its boundary
  // values and its load as u_gamma = A_gg^-1 (b_gamma - A_gG u_Gamma)).  With
  // X = L_gg^-1 (lower):
  //   rows 0 .. g-1   M = A_gg^-1 = X^T X
  //   rows g .. U-1   W^T with W = A_gg^-1 A_gG = X^T P^T (row j: X^T p_j)
  //   row  U          y = A_gg^-1 b_gamma = X^T z
  // every entry a dot product over k (X is stored with zeros above its
  // diagonal, so the full-length sums are exact), one entry per thread.
  T* out = cst + B.lv[K].cst_off;
  for (int e = tid; e < L::n * L::per; e += NB) {
    const int t = e / L::per, rc = e % L::per;
    const int r = rc / g, i = rc % g;
    const T* Xi = xs + t * g * g + i;
    const T* V = r < g ? xs + t * g * g + r : nullptr;  // column r of X, or row r of the frame
    const T* Fr = cur + t * L::fsz + L::row(r);
    T val = T(0);
    if (r < g) {
#pragma unroll
      for (int k = 0; k < g; ++k) val += V[k * g] * Xi[k * g];
    } else {
#pragma unroll
      for (int k = 0; k < g; ++k) val += Fr[k] * Xi[k * g];
    }
    out[e] = val;
  }
  __syncthreads();
}

// Loads this thread's entries of level K's gather table.
template <typename T, int S, int K>
__device__ __forceinline__ void load_ext(const DevBlocks& B, unsigned (&tab)[ext_regs<T, S, K>()]) {
  constexpr int E = ext_count<S, K>();
  if constexpr (E > 0) {
    const unsigned* src = B.ext + ext_off<S, K>();
#pragma unroll
    for (int j = 0; j < ext_regs<T, S, K>(); ++j) tab[j] = src[min(int(threadIdx.x) + NTB * j, E - 1)];
  }
}

template <typename T, int S, int K>
__device__ __forceinline__ void build_levels(T* base, T* cur, T* prev, T* cst, const DevBlocks& B, T* xs,
                                             int& bad_pivot, const unsigned (&tab)[ext_regs<T, S, K>()]) {
  if constexpr (K > 0) {
    unsigned nxt[ext_regs<T, S, K - 1>()];
    load_ext<T, S, K - 1>(B, nxt);
    build_level<T, S, K>(base, cur, cst, B, xs, bad_pivot, tab);
    build_levels<T, S, K - 1>(base, prev, cur, cst, B, xs, bad_pivot, nxt);
  } else {
    build_level<T, S, K>(base, cur, cst, B, xs, bad_pivot, tab);
  }
}

template <typename T, int S>
__global__ void __launch_bounds__(NTB) k_block_build(DevBlocks B, int n_samples, int nc,
                                                    const double* __restrict__ kappa, const double* __restrict__ f,
                                                    int* __restrict__ bad, int* __restrict__ info) {
  using M = Lv<S, Lv<S, 0>::Lm>;
  constexpr int Lm = M::Lm;
  extern __shared__ __align__(16) unsigned char smem[];
  T* buf0 = reinterpret_cast<T*>(smem);
  T* buf1 = buf0 + B.max_buf;
  __shared__ int bad_pivot;
  __shared__ T xs[inv_size_from<S, 0>()];  // X = L_gg^-1 of every node of the current level
  const int q = blockIdx.x / n_samples;
  const int s = blockIdx.x % n_samples;
  const int X0 = B.origin[2 * q], Y0 = B.origin[2 * q + 1];
  const int tid = threadIdx.x;
  // the first extend-add's gather entries are in flight during the assembly
  unsigned first[ext_regs<T, S, (Lm > 0 ? Lm - 1 : 0)>()];
  if constexpr (Lm > 0) load_ext<T, S, Lm - 1>(B, first);
  if (tid == 0) {
    bad_pivot = 0;
    buf0[2 * B.max_buf] = T(0);  // zero slot of the gather table
  }
  // The block's coefficients (S x S cells x 2 triangles) and nodal load
  // ((S+1)^2) are staged in the still unused second frame buffer.
  constexpr int S1 = S + 1;
  double* kL = reinterpret_cast<double*>(buf1);
  double* fL = kL + 2 * S * S;
  {
    const double* ks = kappa + (long long)s * nc * nc * 2;
    for (int e = tid; e < 2 * S * S; e += NTB) {
      const int row = e / (2 * S), col = e % (2 * S);
      kL[e] = ks[((long long)(Y0 + row) * nc + X0) * 2 + col];
    }
    for (int e = tid; e < S1 * S1; e += NTB) fL[e] = f[(long long)(Y0 + e / S1) * (nc + 1) + X0 + e % S1];
  }
  __syncthreads();
  // micro-blocks: every entry of the packed 10-row frames (lower triangle and
  // load row) written once, one micro-block per lane
  {
    static_assert(M::n <= 64 && M::fsz == 55, "micro-block frames");
    const double h = 1.0 / nc;
    const double area3 = 0.5 * h * h / 3.0;
    const int lane = tid & 63, wv = tid >> 6;
    const bool act = lane < M::n;
    const int t = act ? lane : 0;
    const int a0 = B.micro_xy[2 * t], b0 = B.micro_xy[2 * t + 1];  // local corner
    double kap[8];
    bool ok = true;
#pragma unroll
    for (int tr = 0; tr < 8; ++tr) {
      const int cb = tr >> 2, ca = (tr >> 1) & 1, tri = tr & 1;
      kap[tr] = kL[(b0 + cb) * 2 * S + (a0 + ca) * 2 + tri];
      ok = ok && (kap[tr] > 0.0) && (kap[tr] < 1.0e300);
    }
    micro_entries<T, S, 0>(buf0 + t * M::fsz, kap, fL, a0, b0, area3, act, wv);
    if (wv == 0 && act && !ok && bad) atomicCAS(bad + s, 0, 1);
  }
  __syncthreads();
  T* cst = cst_block<T>(B, q, s);
  int bp = 0;
  {
    const unsigned none[1] = {0u};
    build_level<T, S, Lm>(buf0, buf0, cst, B, xs, bp, none);
    if constexpr (Lm > 0) build_levels<T, S, Lm - 1>(buf0, buf1, buf0, cst, B, xs, bp, first);
  }
  if (bp) bad_pivot = 1;
  __syncthreads();
  // block root frame -> global frame store (lower triangle)
  {
    using R = Lv<S, 0>;
    const T* root = (Lm % 2 == 0) ? buf0 : buf1;
    const DevNode nd = B.top.nodes[q];
    T* G = reinterpret_cast<T*>(B.top.frames) + (long long)s * B.top.stride + nd.frame_off;
    const int lane = tid & 63;
    for (int r = tid >> 6; r < R::ld; r += NTB / 64)  // one row per wave
      for (int c = lane; c <= r; c += 64) G[(long long)r * nd.ld + c] = root[R::row(r) + c];
  }
  if (tid == 0 && bad_pivot && info) atomicCAS(info + s, 0, B.top.node_base + q + 1);
}

// ---------------------------------------------------------------------------
// Block solves.  Both run on the local operators the build leaves in the
// compact store (M, W^T, y per node), so every level is one matrix-vector
// product with no substitution chain.  Each thread's operator entries for
// ALL levels are loaded from HBM into registers when the kernel starts; LDS
// holds only the node values.

// Lanes per dot product of a level's GEMV: the largest power of two (at most
// 16) such that work * P threads fit in the workgroup (1 if work > NT).
constexpr int gemv_split(int work) {
  int p = 1;
  while (p < 16 && work * p * 2 <= NT) p *= 2;
  return p;
}

// ---------------------------------------------------------------------------
// Top-down (Root to Leaves inside the block, Section 3.4): from u on the
// block boundary, every level's interfaces in one GEMV per node,
//   u_gamma = y - W u_Gamma            (the build's load), or
//   u_gamma = M g_gamma - W u_Gamma    (a load propagated by k_block_forward,
//                                       g_gamma read from the vector store).
// Thread (w = t * g + i, p) of a level sums the columns j = p (mod P).
template <typename T, int S, int K> struct TdLevel {
  using L = Lv<S, K>;
  static constexpr int g = L::gam, nbd = L::bnd, U = L::U;
  static constexpr int P = gemv_split(L::n * g);
  static constexpr int NJ = (nbd + P - 1) / P;
  static constexpr int NL = (g + P - 1) / P;
  static constexpr int act = L::n * g * P;
  static_assert(act <= NT, "level GEMV does not fit the workgroup");
};

template <typename T, int S, int K> struct TdRegs {
  using C = TdLevel<T, S, K>;
  T w[C::NJ];
  int lj[C::NJ];
  T m[C::NL];
  double z[C::NL];
  T y;
  int li;
};

template <typename T, int S, int K, bool Last = (K == Lv<S, 0>::Lm)> struct TdAll;
template <typename T, int S, int K> struct TdAll<T, S, K, true> {
  TdRegs<T, S, K> r;
};
template <typename T, int S, int K> struct TdAll<T, S, K, false> {
  TdRegs<T, S, K> r;
  TdAll<T, S, K + 1> next;
};

template <typename T, int S, int K, bool FV>
__device__ __forceinline__ void td_load(const DevBlocks& B, const T* cst, const double* vz, TdAll<T, S, K>& a) {
  using C = TdLevel<T, S, K>;
  using L = Lv<S, K>;
  constexpr int g = C::g, P = C::P;
  const int tid = threadIdx.x;
  const int w = min(tid / P, L::n * g - 1);  // idle threads load a valid entry
  const int p = tid % P;
  const int t = w / g, i = w % g;
  const T* blk = cst + B.lv[K].cst_off + t * L::per;
  const int* lid = B.lids + B.lv[K].lid_off + t * C::U;
  // loaded values are masked where they are used, never here: a select on a
  // loaded value would wait for that load and serialise the whole prologue
#pragma unroll
  for (int jj = 0; jj < C::NJ; ++jj) {
    const int jc = min(p + P * jj, C::nbd - 1);
    a.r.w[jj] = blk[(g + jc) * g + i];
    a.r.lj[jj] = lid[g + jc];
  }
  if constexpr (FV) {
    const double* zt = vz + B.lv[K].vec_off + t * g;
#pragma unroll
    for (int ll = 0; ll < C::NL; ++ll) {
      const int lc = min(p + P * ll, g - 1);
      a.r.m[ll] = blk[lc * g + i];
      a.r.z[ll] = zt[lc];
    }
  } else {
    a.r.y = blk[C::U * g + i];
  }
  a.r.li = lid[i];
  if constexpr (K < L::Lm) td_load<T, S, K + 1, FV>(B, cst, vz, a.next);
}

template <typename T, int S, int K, bool FV>
__device__ __forceinline__ void td_solve(const TdAll<T, S, K>& a, double* uL) {
  using C = TdLevel<T, S, K>;
  const int tid = threadIdx.x;
  if (tid < C::act) {
    const int p = tid % C::P;
    double acc = 0.0;
    if constexpr (FV) {
#pragma unroll
      for (int ll = 0; ll < C::NL; ++ll)
        if (p + C::P * ll < C::g) acc += double(a.r.m[ll]) * a.r.z[ll];
    } else {
      if (p == 0) acc = double(a.r.y);
    }
#pragma unroll
    for (int jj = 0; jj < C::NJ; ++jj)
      if (p + C::P * jj < C::nbd) acc -= double(a.r.w[jj]) * uL[a.r.lj[jj]];
    // the P lanes of an entry are consecutive and P divides 64
#pragma unroll
    for (int o = C::P / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (p == 0) uL[a.r.li] = acc;  // gamma of this node: read by no other node of the level
  }
  __syncthreads();
  if constexpr (K < Lv<S, 0>::Lm) td_solve<T, S, K + 1, FV>(a.next, uL);
}

template <typename T, int S, bool FV>
__global__ void __launch_bounds__(NT) k_block_topdown(DevBlocks B, const int* __restrict__ list, int n_samples,
                                                      int nc, double* __restrict__ u, long long ustride) {
  constexpr int S1 = S + 1;
  __shared__ double uL[S1 * S1];
  const int q = list[blockIdx.x / n_samples];
  const int s = blockIdx.x % n_samples;
  const int X0 = B.origin[2 * q], Y0 = B.origin[2 * q + 1];
  const int tid = threadIdx.x;
  double* us = u + (long long)s * ustride;
  const double* vz = FV ? B.vec + (long long)s * B.vec_stride + (long long)q * B.vec_size : nullptr;
  TdAll<T, S, 0> a;
  td_load<T, S, 0, FV>(B, cst_block<T>(B, q, s), vz, a);
  for (int e = tid; e < S1 * S1; e += NT) uL[e] = us[(long long)(Y0 + e / S1) * (nc + 1) + X0 + e % S1];
  __syncthreads();
  td_solve<T, S, 0, FV>(a, uL);
  constexpr int si = S - 1;
  for (int e = tid; e < si * si; e += NT) {
    const int a0 = 1 + e % si, b0 = 1 + e / si;
    us[(long long)(Y0 + b0) * (nc + 1) + X0 + a0] = uL[b0 * S1 + a0];
  }
}

// ---------------------------------------------------------------------------
// Forward: a new load (the refinement's residual) propagated bottom-up
// through the block.  Per level: the sons' condensed loads are merged
// (g = [g_gamma ; g_Gamma], eq. g_omega of Section 2.4, with the gather table
// of k_block_ext), g_gamma goes to the block vector store for the top-down,
// and the condensed load is g_omega = g_Gamma - W^T g_gamma.
// Output j of a level is summed by P lanes, lane p taking i = p (mod P).
template <typename T, int S, int K> struct FwLevel {
  using L = Lv<S, K>;
  static constexpr int g = L::gam, nbd = L::bnd, U = L::U;
  static constexpr int P = gemv_split(L::n * nbd);
  static constexpr int NI = (g + P - 1) / P;
  static constexpr int R = (L::n * nbd * P + NT - 1) / NT;  // rounds of NT / P outputs
  static constexpr int NE = (K < L::Lm) ? (L::n * U + NT - 1) / NT : 1;  // merge entries
};

template <typename T, int S, int K> struct FwRegs {
  using C = FwLevel<T, S, K>;
  T w[C::R][C::NI];
  unsigned e[C::NE];
};

template <typename T, int S, int K, bool First = (K == 0)> struct FwAll;
template <typename T, int S, int K> struct FwAll<T, S, K, true> {
  FwRegs<T, S, K> r;
};
template <typename T, int S, int K> struct FwAll<T, S, K, false> {
  FwRegs<T, S, K> r;
  FwAll<T, S, K - 1> next;
};


template <typename T, int S, int K>
__device__ __forceinline__ void fw_load(const DevBlocks& B, const T* cst, FwAll<T, S, K>& a) {
  using C = FwLevel<T, S, K>;
  using L = Lv<S, K>;
  constexpr int g = C::g, P = C::P;
  const int tid = threadIdx.x;
  const T* base = cst + B.lv[K].cst_off;
#pragma unroll
  for (int rr = 0; rr < C::R; ++rr) {
    const int o = min(tid / P + rr * (NT / P), L::n * C::nbd - 1);
    const int p = tid % P;
    const int t = o / C::nbd, j = o % C::nbd;
    const T* row = base + t * L::per + (g + j) * g;
#pragma unroll
    for (int ii = 0; ii < C::NI; ++ii) a.r.w[rr][ii] = row[min(p + P * ii, g - 1)];  // masked at use
  }
  if constexpr (K < L::Lm) {
    const unsigned* src = B.ext + ext_total<S>() + fext_off<S, K>();
#pragma unroll
    for (int k = 0; k < C::NE; ++k) a.r.e[k] = src[min(tid + NT * k, fext_count<S, K>() - 1)];
  }
  if constexpr (K > 0) fw_load<T, S, K - 1>(B, cst, a.next);
}

template <typename T, int S, int K>
__device__ __forceinline__ void fw_level(const FwAll<T, S, K>& a, const DevBlocks& B, double* gb, double* vz) {
  using C = FwLevel<T, S, K>;
  using L = Lv<S, K>;
  constexpr int g = C::g, U = C::U, P = C::P;
  const int tid = threadIdx.x;
  double* cur = gb + ((L::Lm - K) & 1) * B.max_bnd_nodes;
  if constexpr (K < L::Lm) {
    double v[C::NE];
#pragma unroll
    for (int k = 0; k < C::NE; ++k) v[k] = gb[a.r.e[k] & 0xffffu] + gb[a.r.e[k] >> 16];
#pragma unroll
    for (int k = 0; k < C::NE; ++k)
      if (k + 1 < C::NE || tid + NT * k < L::n * U) cur[tid + NT * k] = v[k];
    __syncthreads();
  }
  for (int e = tid; e < L::n * g; e += NT) vz[B.lv[K].vec_off + e] = cur[(e / g) * U + e % g];
#pragma unroll
  for (int rr = 0; rr < C::R; ++rr) {
    const int o = tid / P + rr * (NT / P), p = tid % P;
    const int oc = min(o, L::n * C::nbd - 1);
    const int t = oc / C::nbd, j = oc % C::nbd;
    const double* x = cur + t * U;
    double acc = 0.0;
#pragma unroll
    for (int ii = 0; ii < C::NI; ++ii)
      if (p + P * ii < g) acc += double(a.r.w[rr][ii]) * x[p + P * ii];
#pragma unroll
    for (int sh = P / 2; sh > 0; sh >>= 1) acc += __shfl_xor(acc, sh);
    // own slot: other threads read only x[0 .. g)
    if (p == 0 && o < L::n * C::nbd) cur[t * U + g + j] = x[g + j] - acc;
  }
  __syncthreads();
  if constexpr (K > 0) fw_level<T, S, K - 1>(a.next, B, gb, vz);
}

template <typename T, int S>
__global__ void __launch_bounds__(NT) k_block_forward(DevBlocks B, int n_samples, int nc,
                                                      const double* __restrict__ res, long long rstride) {
  using M = Lv<S, Lv<S, 0>::Lm>;
  constexpr int Lm = M::Lm;
  constexpr int S1 = S + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  double* gb = reinterpret_cast<double*>(smem);  // two buffers of max_bnd_nodes, then the zero slot
  const int q = blockIdx.x / n_samples;
  const int s = blockIdx.x % n_samples;
  const int X0 = B.origin[2 * q], Y0 = B.origin[2 * q + 1];
  const int tid = threadIdx.x;
  // micro-blocks: node (i, j) of the residual belongs to the micro-block that
  // contains cell (i, j), so each global entry is counted exactly once.  The
  // index loads go first, the operator loads next, the residual loads (which
  // need the indices) last, so the prologue waits for memory once.
  constexpr int NM = (M::n * M::U + NT - 1) / NT;
  int lid[NM], ax[NM], by[NM];
  {
    const int* lids = B.lids + B.lv[Lm].lid_off;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const int e = min(tid + NT * k, M::n * M::U - 1);
      const int t = e / M::U;
      lid[k] = lids[e];
      ax[k] = B.micro_xy[2 * t];
      by[k] = B.micro_xy[2 * t + 1];
    }
  }
  FwAll<T, S, Lm> a;
  fw_load<T, S, Lm>(B, cst_block<T>(B, q, s), a);
  double* vz = B.vec + (long long)s * B.vec_stride + (long long)q * B.vec_size;
  const double* rs = res + (long long)s * rstride;
  if (tid == 0) gb[2 * B.max_bnd_nodes] = 0.0;
  {
    double v[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const int a0 = lid[k] % S1, b0 = lid[k] / S1;
      const bool own = a0 >= ax[k] && a0 < ax[k] + 2 && b0 >= by[k] && b0 < by[k] + 2;
      v[k] = own ? rs[(long long)(Y0 + b0) * (nc + 1) + X0 + a0] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < NM; ++k)
      if (tid + NT * k < M::n * M::U) gb[tid + NT * k] = v[k];
  }
  __syncthreads();
  fw_level<T, S, Lm>(a, B, gb, vz);
  // block root [g_gamma ; g_omega] -> the global vector store of the block level
  using R = Lv<S, 0>;
  const double* root = gb + (Lm & 1) * B.max_bnd_nodes;
  const DevNode nd = B.top.nodes[q];
  double* out = B.top.vec + (long long)s * B.top.vec_stride + nd.ids_off;
  for (int e = tid; e < R::U; e += NT) out[e] = root[e];
}

// ---------------------------------------------------------------------------
// two frame buffers and the gather table's zero slot
size_t block_build_lds(const DevBlocks& B, bool dbl) { return (size_t(2) * B.max_buf + 2) * (dbl ? 8 : 4); }

size_t block_ext_entries(int s) {
  switch (s) {
    case 2: return ext_total<2>() + fext_total<2>();
    case 4: return ext_total<4>() + fext_total<4>();
    case 8: return ext_total<8>() + fext_total<8>();
    case 16: return ext_total<16>() + fext_total<16>();
    default: return 0;
  }
}

template <int S> static void launch_ext_t(const DevBlocks& B, unsigned* ext, hipStream_t st) {
  constexpr int n = ext_total<S>() + fext_total<S>();
  if (n > 0) hipLaunchKernelGGL((k_block_ext<S>), dim3((n + 255) / 256), dim3(256), 0, st, B, ext);
}

hipError_t launch_block_ext(const DevBlocks& B, unsigned* ext, hipStream_t st) {
  // every offset (and the zero slots) must fit the tables' 16-bit fields
  if (2 * B.max_buf >= 65536 || 2 * B.max_bnd_nodes >= 65536) return hipErrorInvalidValue;
  switch (B.s) {
    case 2: launch_ext_t<2>(B, ext, st); break;
    case 4: launch_ext_t<4>(B, ext, st); break;
    case 8: launch_ext_t<8>(B, ext, st); break;
    case 16: launch_ext_t<16>(B, ext, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t block_topdown_lds(const DevBlocks& B, bool) { return sizeof(double) * size_t((B.s + 1) * (B.s + 1)); }

// two buffers of node values and the gather table's zero slot
size_t block_forward_lds(const DevBlocks& B, bool) { return sizeof(double) * size_t(2 * B.max_bnd_nodes + 1); }

template <int S, int K> static bool shape_ok_from(const DevBlocks& B) {
  using L = Lv<S, K>;
  const bool ok = B.lv[K].n == L::n && B.lv[K].gam == L::gam && B.lv[K].bnd == L::bnd && B.lv[K].fsz == L::fsz;
  if constexpr (K < Lv<S, 0>::Lm) return ok && shape_ok_from<S, K + 1>(B);
  return ok;
}

template <int S> static bool shape_ok(const DevBlocks& B) {
  return B.nlev == Lv<S, 0>::Lm + 1 && shape_ok_from<S, 0>(B);
}

bool block_shape_ok(const DevBlocks& B) {
  switch (B.s) {
    case 2: return shape_ok<2>(B);
    case 4: return shape_ok<4>(B);
    case 8: return shape_ok<8>(B);
    case 16: return shape_ok<16>(B);
    default: return false;
  }
}

template <typename T, int S>
static void launch_build_t(const DevBlocks& B, int n_samples, int nc, const double* kappa, const double* f, int* bad,
                           int* info, hipStream_t st) {
  const size_t lds = block_build_lds(B, sizeof(T) == 8);
  hipLaunchKernelGGL((k_block_build<T, S>), dim3(B.nb * n_samples), dim3(NTB), lds, st, B, n_samples, nc, kappa, f,
                     bad, info);
}

template <typename T, int S>
static void launch_topdown_t(const DevBlocks& B, const int* list, int n_list, int n_samples, int nc, double* u,
                             long long ustride, bool from_vec, hipStream_t st) {
  if (from_vec)
    hipLaunchKernelGGL((k_block_topdown<T, S, true>), dim3(n_list * n_samples), dim3(NT), 0, st, B, list, n_samples,
                       nc, u, ustride);
  else
    hipLaunchKernelGGL((k_block_topdown<T, S, false>), dim3(n_list * n_samples), dim3(NT), 0, st, B, list, n_samples,
                       nc, u, ustride);
}

template <typename T, int S>
static void launch_forward_t(const DevBlocks& B, int n_samples, int nc, const double* r, long long rstride,
                             hipStream_t st) {
  const size_t lds = block_forward_lds(B, sizeof(T) == 8);
  hipLaunchKernelGGL((k_block_forward<T, S>), dim3(B.nb * n_samples), dim3(NT), lds, st, B, n_samples, nc, r,
                     rstride);
}

#define HDD_BLOCK_DISPATCH(FN, ...)                                   \
  do {                                                                \
    const bool dbl_ = B.top.is_double != 0;                           \
    switch (B.s) {                                                    \
      case 2: dbl_ ? FN<double, 2>(__VA_ARGS__) : FN<float, 2>(__VA_ARGS__); break;    \
      case 4: dbl_ ? FN<double, 4>(__VA_ARGS__) : FN<float, 4>(__VA_ARGS__); break;    \
      case 8: dbl_ ? FN<double, 8>(__VA_ARGS__) : FN<float, 8>(__VA_ARGS__); break;    \
      case 16: dbl_ ? FN<double, 16>(__VA_ARGS__) : FN<float, 16>(__VA_ARGS__); break; \
      default: return hipErrorInvalidValue;                           \
    }                                                                 \
  } while (0)

hipError_t launch_block_build(const DevBlocks& B, int n_samples, int nc, const double* kappa, const double* f,
                              int* bad, int* info, hipStream_t st) {
  HDD_BLOCK_DISPATCH(launch_build_t, B, n_samples, nc, kappa, f, bad, info, st);
  return hipGetLastError();
}

hipError_t launch_block_topdown(const DevBlocks& B, const int* list, int n_list, int n_samples, int nc, double* u,
                                long long ustride, bool from_vec, hipStream_t st) {
  if (n_list <= 0) return hipSuccess;
  HDD_BLOCK_DISPATCH(launch_topdown_t, B, list, n_list, n_samples, nc, u, ustride, from_vec, st);
  return hipGetLastError();
}

hipError_t launch_block_forward(const DevBlocks& B, int n_samples, int nc, const double* r, long long rstride,
                                hipStream_t st) {
  HDD_BLOCK_DISPATCH(launch_forward_t, B, n_samples, nc, r, rstride, st);
  return hipGetLastError();
}

}  // namespace hdd
