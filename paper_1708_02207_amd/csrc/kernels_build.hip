// HDD "Leaves to Root" kernels above the block level (Sections 3.2-3.4): the
// extend-add of two sons' Schur complements into the father's frame, and the
// elimination of the father's interface by a partial Cholesky factorization
// of its frame (panel factorization + triangular solve, then a symmetric
// rank-k update on the MFMA matrix cores).
#include <algorithm>
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace hdd {

// Tiles (ti, tj) with tj <= ti and tj < tc of a tr x tc tile grid, numbered
// row by row: the tiles on or below the diagonal of a Schur update whose
// rows and columns start at the same index.  Only these are launched (empty
// workgroups for the tiles above the diagonal cost 2.6 ms per step of the
// 128 x 128 updates at 1023^2 x 128).
__host__ __device__ inline int lower_tile_count(int tr, int tc) {
  return tc >= tr ? tr * (tr + 1) / 2 : tc * (tc + 1) / 2 + (tr - tc) * tc;
}
__device__ __forceinline__ void lower_tile(int t, int tc, int& ti, int& tj) {
  const int tri = tc * (tc + 1) / 2;  // rows 0 .. tc - 1 hold ti + 1 tiles
  if (t < tri) {
    ti = tri_row(t);
    tj = t - ti * (ti + 1) / 2;
  } else {
    ti = tc + (t - tri) / tc;
    tj = (t - tri) % tc;
  }
}

// ---------------------------------------------------------------------------
// Extend-add (eq. Psi_sum and the block system eq. block_equation4): the
// father's frame is the sum of both sons' [Gamma;rhs] blocks embedded in the
// father's [gamma;Gamma;rhs] ordering.  Gather form: every lower-triangle
// element (r, c) of the father reads at most one element of each son.
// One dimension, in the XCD-aware order of the Schur-update tiles: the tiles
// of one (node, sample) frame follow each other on one XCD, so the cache
// lines that neighbouring tiles share in a son's rows (Gamma starts at an
// odd column of the son frame) are read from HBM once (17.5 -> 16.2 ms per
// step at 1023^2 x 128 against a (pair, tile) grid).
// ---------------------------------------------------------------------------
template <typename Ts, typename Tf>
__global__ void __launch_bounds__(256) k_extend_add(DevLevel F, DevLevel S, int n_samples) {
  // One 64 x 64 tile of the father's lower triangle per workgroup: lanes run
  // over the 64 columns (coalesced stores), the 4 waves over 16 rows each.
  // The tile's row and column maps are staged in LDS; every son read goes
  // through an address that is valid even when the entry is absent (then the
  // value is dropped), so all 32 reads of a thread are issued together.
  __shared__ int mrow[2][64], mcol[2][64];
  const int nt = (F.max_U + 1 + 63) / 64;
  const int n_tiles = nt * (nt + 1) / 2;
  const int loc = blockIdx.x >> 3;
  const int pair = (loc / n_tiles) * 8 + (blockIdx.x & 7);
  if (pair >= F.n_nodes * n_samples) return;
  const int node = pair / n_samples;
  const int s = pair % n_samples;
  const DevNode nd = F.nodes[node];
  const int n = nd.U + 1;
  const int t = loc % n_tiles;
  const int ti = tri_row(t), tj = t - ti * (ti + 1) / 2;
  const int r0 = ti * 64, c0 = tj * 64;
  if (r0 >= n) return;  // uniform
  const int* mA = F.maps + nd.map_off;
  const int* mB = mA + n;
  const int tid = threadIdx.x;
  if (tid < 128) {
    const int q = tid & 63, which = tid >> 6;
    const int r = r0 + q, c = c0 + q;
    const int* m = which ? mB : mA;
    mrow[which][q] = r < n ? m[r] : -1;
    mcol[which][q] = c < n ? m[c] : -1;
  }
  __syncthreads();
  const int sonA = 2 * node, sonB = 2 * node + 1;
  const DevNode na = S.nodes[sonA], nb = S.nodes[sonB];
  const int ga = na.U - na.bnd, gb = nb.U - nb.bnd;
  const Ts* SA = frame_ptr<Ts>(S, sonA, s) + (long long)ga * na.ld + ga;
  const Ts* SB = frame_ptr<Ts>(S, sonB, s) + (long long)gb * nb.ld + gb;
  Tf* out = frame_ptr<Tf>(F, node, s);
  const int lane = tid & 63, w = tid >> 6;
  const int c = c0 + lane;
  const int ac = mcol[0][lane], bc = mcol[1][lane];
  Ts va[16], vb[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int rr = w + 4 * q;
    const int ar = mrow[0][rr], br = mrow[1][rr];
    const long long ia = (ar >= 0 && ac >= 0) ? (long long)max(ar, ac) * na.ld + min(ar, ac) : 0;
    const long long ib = (br >= 0 && bc >= 0) ? (long long)max(br, bc) * nb.ld + min(br, bc) : 0;
    va[q] = SA[ia];
    vb[q] = SB[ib];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int rr = w + 4 * q;
    const int r = r0 + rr;
    if (r < n && c <= r) {
      const int ar = mrow[0][rr], br = mrow[1][rr];
      Tf v = Tf(0);
      if (ar >= 0 && ac >= 0) v += Tf(va[q]);
      if (br >= 0 && bc >= 0) v += Tf(vb[q]);
      out[(long long)r * nd.ld + c] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Panel step of the partial Cholesky (the elimination of eq. SchurMinus1 on
// the interface block; the paper's M = -(sum of the sons' interface blocks)
// of eq. gamma is factored as -M = L L^T, which is positive definite).
//
// k_panel_diag: one wave per (node, sample) factors the kb x kb diagonal
//   block at (k0, k0), kb <= 64, in registers (lane i holds row i); the
//   scaled pivot column is exchanged through LDS, so no workgroup barrier is
//   needed.  A non-positive or non-finite pivot is recorded in info[sample]
//   and replaced by 1 so that no NaN spreads.
// k_panel_rows: solves X L^T = A[r, k0:k0+kb] for the rows r below the block
//   (interface rows, boundary rows and the rhs row), one row per thread in
//   registers against L in LDS; rows are staged through LDS with coalesced
//   loads and stores.  grid = (node x sample, row chunks of RW).
// ---------------------------------------------------------------------------
template <typename T> struct PanelCfg {
  static constexpr int RW = sizeof(T) == 8 ? 64 : 128;  // rows (= threads) per workgroup
};

__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <typename T, int NB>
__global__ void __launch_bounds__(64) k_panel_diag(DevLevel L, int k0, int kb, int n_samples, int* info) {
  const int pair = blockIdx.x;
  const int node = pair / n_samples;
  const int s = pair % n_samples;
  const DevNode nd = L.nodes[node];
  const int ld = nd.ld;
  T* Dg = frame_ptr<T>(L, node, s) + (long long)k0 * ld + k0;
  const int lane = threadIdx.x;
  T a[NB];
  const int lc = min(lane, kb - 1);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const T v = Dg[(long long)lc * ld + min(k, lc)];
    a[k] = (lane < kb && k <= lane) ? v : T(0);
  }
  int bp = 0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < kb) {
      T d = lane_value(a[j], j);
      if (!(d > T(0)) || !(d < T(1e300))) {
        if (!bp) bp = k0 + j + 1;
        d = T(1);
      }
      d = sqrt(d);
      a[j] = lane == j ? d : (lane > j ? a[j] / d : a[j]);
#pragma unroll
      for (int k = j + 1; k < NB; ++k) {
        const T ck = lane_value(a[j], k);  // L_kj (zero on lanes >= kb)
        if (k <= lane) a[k] -= a[j] * ck;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (lane < kb && k <= lane) Dg[(long long)lane * ld + k] = a[k];
  if (L.panel) {  // the final columns also go to the level's panel store
    T* Pp = panel_ptr<T>(L, node, s) + (long long)(k0 + lane) * L.panel_ld + k0;
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (lane < kb && k <= lane) Pp[k] = a[k];
  }
  if (lane == 0 && bp && info) atomicCAS(info + s, 0, L.node_base + node + 1);
}

template <typename T, int NB>
__global__ void __launch_bounds__(PanelCfg<T>::RW) k_panel_rows(DevLevel L, int k0, int kb, int n_samples) {
  constexpr int RW = PanelCfg<T>::RW;
  __shared__ T D[NB][NB + 1];
  __shared__ T X[RW][NB + 1];
  __shared__ T rD[NB];  // reciprocal pivots 1 / L_jj
  const int pair = blockIdx.x;
  const int node = pair / n_samples;
  const int s = pair % n_samples;
  const DevNode nd = L.nodes[node];
  const int U = nd.U, ld = nd.ld;
  const int r0 = k0 + kb + blockIdx.y * RW;
  if (r0 > U) return;  // uniform
  T* F = frame_ptr<T>(L, node, s);
  const int tid = threadIdx.x;
  const int nrows = min(RW, U + 1 - r0);
  const int total = nrows * NB;  // row e / NB, column e % NB (used where < kb)
  // every staging load of the thread is issued before any LDS store (one
  // memory latency): the diagonal block (NB x NB, valid below and on the
  // diagonal within kb) and the panel rows (nrows x kb), consecutive
  // threads on consecutive columns; addresses are clamped into the panel.
  // Entries are numbered with the compile-time width NB, so no index needs
  // a division by the run-time kb.
  constexpr int DPT = (NB * NB + RW - 1) / RW;
  T dv[DPT], xv[NB];
#pragma unroll
  for (int u = 0; u < DPT; ++u) {
    const int e = tid + u * RW;
    const int i = min(e / NB, kb - 1), j = min(e % NB, i);
    dv[u] = F[(long long)(k0 + i) * ld + k0 + j];
  }
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int e = min(tid + u * RW, total - 1);
    xv[u] = F[(long long)(r0 + e / NB) * ld + k0 + min(e % NB, kb - 1)];
  }
#pragma unroll
  for (int u = 0; u < DPT; ++u) {
    const int e = tid + u * RW;
    const int i = e / NB, j = e % NB;
    if (i < kb && j <= i) D[i][j] = dv[u];
  }
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int e = tid + u * RW;
    if (e < total) X[e / NB][e % NB] = xv[u];
  }
  __syncthreads();
  if (tid < kb) rD[tid] = T(1) / D[tid][tid];
  __syncthreads();
  if (tid < nrows) {
    T x[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) x[k] = k < kb ? X[tid][k] : T(0);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (j < kb) {
        T v = x[j];
#pragma unroll
        for (int l = 0; l < j; ++l) v -= x[l] * D[j][l];
        x[j] = v * rD[j];
      }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (k < kb) X[tid][k] = x[k];
  }
  __syncthreads();
  // the finished columns go to the level's panel store, which the Schur
  // updates read them from (else back to the frame)
  T* Pp = L.panel ? panel_ptr<T>(L, node, s) : F;
  const int pld = L.panel ? L.panel_ld : ld;
  for (int e = tid; e < total; e += RW)
    if (e % NB < kb) Pp[(long long)(r0 + e / NB) * pld + k0 + e % NB] = X[e / NB][e % NB];
}

// ---------------------------------------------------------------------------
// Symmetric rank-k update of a lower-triangular region of the frame:
//   C[i][j] -= sum_{k in [k0,k1)} F[i][k] F[j][k],   r0 <= i <= U,
//   c0 <= j < c1 (c1 < 0: U+1), j <= i.
// Used for the trailing update inside the interface (K = one panel) and for
// the Schur update S_omega = S~ - P P^T (K = |gamma|), i.e. Psi^g of
// Section 2.4, together with the boundary load g_omega = g~ - P z (rhs row).
// 64 x 64 output tile per workgroup of 256 threads (4 waves, 32 x 32 each).
// ---------------------------------------------------------------------------
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> struct SyrkCfg;
template <> struct SyrkCfg<float> { static constexpr int KC = 32; };
template <> struct SyrkCfg<double> { static constexpr int KC = 16; };

struct SyrkArgs {
  int k0, k1, r0, c0, c1;
  int tiles_c;  // number of tile columns
  int tiles_r;  // number of tile rows
  int sep;      // 1: matrix-core tiles (rows <= U - 1; the load row U by the diagonal tiles)
};

// One K chunk of the A rows (rowA0..) and B rows (rowB0..) into LDS.  Rows
// past U are clamped to U (they only feed outputs that are never stored);
// columns past k1 read a clamped address and are replaced by zero, so the
// loads carry no branches.
template <typename T, bool WZ = false>
__device__ __forceinline__ void syrk_load_chunk(T (*As)[SyrkCfg<T>::KC + 1], T (*Bs)[SyrkCfg<T>::KC + 1],
                                                const T* F, int ld, int U, int rowA0, int rowB0, int kbeg,
                                                int k1) {
  constexpr int KC = SyrkCfg<T>::KC;
  constexpr int PER = 64 * KC / 256;  // elements per thread per matrix
  const int tid = threadIdx.x;
  const int row = tid / (KC / PER);
  const int col0 = (tid % (KC / PER)) * PER;
  const T* pa = F + (long long)min(rowA0 + row, U) * ld;
  const T* pb = F + (long long)min(rowB0 + row, U) * ld;
  T va[PER], vb[PER], vz = T(0);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int k = kbeg + col0 + q;
    const int kc = min(k, k1 - 1);
    va[q] = pa[kc];
    vb[q] = pb[kc];
  }
  // WZ: row 64 of As receives the chunk of the load row U (z)
  if (WZ && tid < KC) vz = F[(long long)U * ld + min(kbeg + tid, k1 - 1)];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const bool kin = kbeg + col0 + q < k1;
    As[row][col0 + q] = kin ? va[q] : T(0);
    Bs[row][col0 + q] = kin ? vb[q] : T(0);
  }
  if (WZ && tid < KC) As[64][tid] = kbeg + tid < k1 ? vz : T(0);
}
// Rows of the operand columns [k0, k1) of a node's update: the level's panel
// store, where the panel kernels leave the finished columns [L ; P ; z]
// (the frame keeps only the columns still to be updated), else the frame.
template <typename T>
__device__ __forceinline__ const T* syrk_operands(const DevLevel& L, int node, int s, const T* F, int ld, int& pl) {
  if (L.panel) {
    pl = L.panel_ld;
    return panel_ptr<T>(L, node, s);
  }
  pl = ld;
  return F;
}

// Output element (i, j) of the update belongs to this call's region.
__device__ __forceinline__ bool syrk_in(int U, int i, int j, const SyrkArgs& a, int c1e) {
  return i <= U && i >= a.r0 && j >= a.c0 && j < c1e && j <= i;
}

template <typename T>
__device__ __forceinline__ void syrk_store(T* F, int ld, int U, int i, int j, const SyrkArgs& a, int c1e, T v) {
  if (syrk_in(U, i, j, a, c1e)) F[(long long)i * ld + j] -= v;
}

// Current value at (i, j) read through an address clamped into the frame,
// so that all reads of a tile can be issued before any store.
template <typename T>
__device__ __forceinline__ T syrk_old(const T* F, int ld, int U, int i, int j) {
  return F[(long long)min(i, U) * ld + min(j, U)];
}

// The 64 x 64 matrix-core tiles leave the load row U to the diagonal tiles'
// idle wave: in a diagonal tile the upper-right 32 x 32 wave block lies
// strictly above the diagonal, so that wave instead forms the update of the
// load row, F[U][j] -= sum_k z_k F[j][k] (g_omega = g~ - P z, eq. SchurC1),
// for the tile's 64 columns from the B rows in LDS and z staged as row 64 of
// As.  Without this the single row U would cost a whole row of tiles.
// Workgroup order as in the 128 x 128 tile: workgroup b runs on XCD b % 8
// and the tiles of one (node, sample) frame follow each other on one XCD,
// so their operand rows are shared in its L2 (float64 updates 7.6 -> 7.0 ms
// per step at 1023^2 x 128 against the (pair, tile) grid).
__global__ void __launch_bounds__(256) k_syrk_mfma_f32(DevLevel L, SyrkArgs a, int n_samples) {
  constexpr int KC = SyrkCfg<float>::KC;
  __shared__ float As[65][KC + 1];
  __shared__ float Bs[64][KC + 1];
  const int n_tiles = lower_tile_count(a.tiles_r, a.tiles_c);
  const int loc = blockIdx.x >> 3;
  const int pair = (loc / n_tiles) * 8 + (blockIdx.x & 7);
  if (pair >= L.n_nodes * n_samples) return;
  const int node = pair / n_samples, s = pair % n_samples;
  const DevNode nd = L.nodes[node];
  const int U = nd.U;
  const int Ue = U - 1;  // last row of the tiles; row U is the load row
  const int c1e = min(a.c1 < 0 ? U + 1 : a.c1, U);
  int ti, tj;
  lower_tile(loc % n_tiles, a.tiles_c, ti, tj);
  const int i0 = a.r0 + ti * 64, j0 = a.c0 + tj * 64;
  if (i0 > Ue || j0 >= c1e) return;
  float* F = frame_ptr<float>(L, node, s);
  const int ld = nd.ld;
  int pl;
  const float* Pb = syrk_operands<float>(L, node, s, F, ld, pl);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
  const bool diag = i0 == j0;
  const bool rhs_wave = diag && wr == 0 && wc == 1;  // wave-uniform
  floatx16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  float racc = 0.f;
  // the current values of the wave's 32 x 32 block are read before the K loop
  // (their latency overlaps the first chunk's) and kept apart from the
  // accumulators, so S~ - P P^T is still rounded once
  float old[16];
  if (!rhs_wave) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = i0 + wr * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
      const int j = j0 + wc * 32 + (lane & 31);
      old[v] = syrk_old(F, ld, U, i, j);
    }
  }
  for (int kb = a.k0; kb < a.k1; kb += KC) {
    __syncthreads();
    syrk_load_chunk<float, true>(As, Bs, Pb, pl, U, i0, j0, kb, a.k1);
    __syncthreads();
    if (rhs_wave) {
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) racc += As[64][kk] * Bs[lane][kk];
    } else {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 2) {
        const float av = As[wr * 32 + (lane & 31)][kk + (lane >> 5)];
        const float bv = Bs[wc * 32 + (lane & 31)][kk + (lane >> 5)];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
      }
    }
  }
  if (rhs_wave) {
    const int j = j0 + lane;
    if (j < c1e) F[(long long)U * ld + j] -= racc;
    return;
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = i0 + wr * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
    const int j = j0 + wc * 32 + (lane & 31);
    if (syrk_in(Ue, i, j, a, c1e)) F[(long long)i * ld + j] = old[v] - acc[v];
  }
}

// Tall tile for updates of at most 32 columns (the panel-to-panel updates
// at the bottom of the recursive interface factorization): 128 rows x 32
// columns per workgroup, wave w on rows i0 + 32 w .. + 31, one 32 x 32 x 2
// MFMA accumulator each, K chunks of 32 through LDS.  The load row U is an
// ordinary row here (its A operand row is z).  A 64 x 64 tile over 32
// columns would read and multiply twice the columns it stores.
__global__ void __launch_bounds__(256) k_syrk_tall_f32(DevLevel L, SyrkArgs a, int n_samples) {
  constexpr int KC = 32;
  __shared__ float As[128][KC + 1];
  __shared__ float Bs[32][KC + 1];
  const int pair = blockIdx.x;
  const int node = pair / n_samples, s = pair % n_samples;
  const DevNode nd = L.nodes[node];
  const int U = nd.U;
  const int c1e = a.c1 < 0 ? U + 1 : a.c1;
  const int ti = blockIdx.y / a.tiles_c, tj = blockIdx.y % a.tiles_c;
  const int i0 = a.r0 + ti * 128, j0 = a.c0 + tj * 32;
  if (i0 > U || j0 >= c1e || i0 + 127 < j0) return;
  float* F = frame_ptr<float>(L, node, s);
  const int ld = nd.ld;
  int pl;
  const float* Pb = syrk_operands<float>(L, node, s, F, ld, pl);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // loaders: A row tid / 2 (16 consecutive k), B row tid / 8 (4 consecutive
  // k); rows past U clamped to U, columns past k1 read clamped and zeroed
  const int ar = tid >> 1, ak = (tid & 1) * 16;
  const int br = tid >> 3, bk = (tid & 7) * 4;
  const float* rowA = Pb + (long long)min(i0 + ar, U) * pl;
  const float* rowB = Pb + (long long)min(j0 + br, U) * pl;
  floatx16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  // current values read before the K loop, kept apart from the accumulators
  const int j = j0 + (lane & 31);
  const int ib = i0 + w * 32 + (lane >> 5) * 4;
  float old[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) old[v] = syrk_old(F, ld, U, ib + (v >> 2) * 8 + (v & 3), j);
  for (int kb = a.k0; kb < a.k1; kb += KC) {
    float va[16], vb[4];
#pragma unroll
    for (int q = 0; q < 16; ++q) va[q] = rowA[min(kb + ak + q, a.k1 - 1)];
#pragma unroll
    for (int q = 0; q < 4; ++q) vb[q] = rowB[min(kb + bk + q, a.k1 - 1)];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) As[ar][ak + q] = kb + ak + q < a.k1 ? va[q] : 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) Bs[br][bk + q] = kb + bk + q < a.k1 ? vb[q] : 0.f;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[w * 32 + (lane & 31)][kk + (lane >> 5)],
                                                 Bs[lane & 31][kk + (lane >> 5)], acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = ib + (v >> 2) * 8 + (v & 3);
    if (syrk_in(U, i, j, a, c1e)) F[(long long)i * ld + j] = old[v] - acc[v];
  }
}

// float64 version of the same tile (16 x 16 x 4 MFMA, 2 x 2 per wave).
__global__ void __launch_bounds__(256) k_syrk_mfma_f64(DevLevel L, SyrkArgs a, int n_samples) {
  constexpr int KC = SyrkCfg<double>::KC;
  __shared__ double As[65][KC + 1];
  __shared__ double Bs[64][KC + 1];
  const int n_tiles = lower_tile_count(a.tiles_r, a.tiles_c);
  const int loc = blockIdx.x >> 3;
  const int pair = (loc / n_tiles) * 8 + (blockIdx.x & 7);
  if (pair >= L.n_nodes * n_samples) return;
  const int node = pair / n_samples, s = pair % n_samples;
  const DevNode nd = L.nodes[node];
  const int U = nd.U;
  const int Ue = U - 1;  // last row of the tiles; row U is the load row
  const int c1e = min(a.c1 < 0 ? U + 1 : a.c1, U);
  int ti, tj;
  lower_tile(loc % n_tiles, a.tiles_c, ti, tj);
  const int i0 = a.r0 + ti * 64, j0 = a.c0 + tj * 64;
  if (i0 > Ue || j0 >= c1e) return;
  double* F = frame_ptr<double>(L, node, s);
  const int ld = nd.ld;
  int pl;
  const double* Pb = syrk_operands<double>(L, node, s, F, ld, pl);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
  const bool rhs_wave = i0 == j0 && wr == 0 && wc == 1;  // wave-uniform
  doublex4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[x][y][v] = 0.0;
  double racc = 0.0;
  for (int kb = a.k0; kb < a.k1; kb += KC) {
    __syncthreads();
    syrk_load_chunk<double, true>(As, Bs, Pb, pl, U, i0, j0, kb, a.k1);
    __syncthreads();
    if (rhs_wave) {
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) racc += As[64][kk] * Bs[lane][kk];
    } else {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        double av[2], bv[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) av[x] = As[wr * 32 + x * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int y = 0; y < 2; ++y) bv[y] = Bs[wc * 32 + y * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
      }
    }
  }
  if (rhs_wave) {
    const int j = j0 + lane;
    if (j < c1e) F[(long long)U * ld + j] -= racc;
    return;
  }
  double old[2][2][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wr * 32 + x * 16 + 4 * v + (lane >> 4);  // f64 16x16x4: row 4v + lane/16
        const int j = j0 + wc * 32 + y * 16 + (lane & 15);
        old[x][y][v] = syrk_old(F, ld, U, i, j);
      }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wr * 32 + x * 16 + 4 * v + (lane >> 4);
        const int j = j0 + wc * 32 + y * 16 + (lane & 15);
        if (syrk_in(Ue, i, j, a, c1e)) F[(long long)i * ld + j] = old[x][y][v] - acc[x][y][v];
      }
}

// Large-tile version for the upper levels: 128 x 128 output tile per
// workgroup (4 waves, 64 x 64 each as 2 x 2 blocks of 32 x 32 x 2 MFMA),
// K chunks of KC staged through two LDS buffers, one barrier per chunk.  The
// next chunk's global loads are in flight while the current chunk is
// multiplied: the loop body has no branch, every chunk is read at addresses
// clamped into the node's frame (rows past U to U, columns to the last
// column of the row), and entries outside [k0, k1) are zeroed when the chunk
// is stored to LDS, after the MFMAs, so no load result is waited for before
// the MFMAs of the chunk it is prefetched behind.  The last chunk is peeled
// so that its MFMAs overlap the epilogue's first reads.  In diagonal tiles
// the blocks above the diagonal issue no MFMAs, and the wave whose block
// lies wholly above it forms the load row U instead (the tiles stop at row
// U - 1, so a frame of 128 m + 1 rows needs no further row of tiles).  V4:
// 16-byte operand loads (operand row stride pl % 4 == 0 and k0 % 4 == 0).
template <bool V4, int KC>
__device__ __forceinline__ void syrk128_tile(float (*As)[128][KC + 1], float (*Bs)[128][KC + 1], float* F, int ld,
                                             const float* Pb, int pl, int U, int Ue, int i0, int j0,
                                             const SyrkArgs& a, int c1e) {
  constexpr int NQ = KC / 8;  // float4 groups per thread and operand
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  // loader mapping: thread -> (row lr, KC / 2 consecutive k) for A and B.  Rows
  // past U are clamped to U: they only feed outputs that are never stored.
  const int lr = tid >> 1, lk = (tid & 1) * (KC / 2);
  const float* rowA = Pb + (long long)min(i0 + lr, U) * pl;
  const float* rowB = Pb + (long long)min(j0 + lr, U) * pl;
  float4 pa[NQ], pb[NQ];
  auto load = [&](int kb) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = kb + lk + 4 * q;
      if constexpr (V4) {
        const int kc = min(k, pl - 4);  // pl % 4 == 0: stays 16-byte aligned
        pa[q] = *reinterpret_cast<const float4*>(rowA + kc);
        pb[q] = *reinterpret_cast<const float4*>(rowB + kc);
      } else {
        float ta[4], tb[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int kc = min(k + x, pl - 1);
          ta[x] = rowA[kc];
          tb[x] = rowB[kc];
        }
        pa[q] = make_float4(ta[0], ta[1], ta[2], ta[3]);
        pb[q] = make_float4(tb[0], tb[1], tb[2], tb[3]);
      }
    }
  };
  auto store = [&](int buf, int kb) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = kb + lk + 4 * q;
      // select, not multiply: entries past k1 may hold any bit pattern
      const bool m0 = k + 0 < a.k1, m1 = k + 1 < a.k1, m2 = k + 2 < a.k1, m3 = k + 3 < a.k1;
      As[buf][lr][lk + 4 * q + 0] = m0 ? pa[q].x : 0.f;
      As[buf][lr][lk + 4 * q + 1] = m1 ? pa[q].y : 0.f;
      As[buf][lr][lk + 4 * q + 2] = m2 ? pa[q].z : 0.f;
      As[buf][lr][lk + 4 * q + 3] = m3 ? pa[q].w : 0.f;
      Bs[buf][lr][lk + 4 * q + 0] = m0 ? pb[q].x : 0.f;
      Bs[buf][lr][lk + 4 * q + 1] = m1 ? pb[q].y : 0.f;
      Bs[buf][lr][lk + 4 * q + 2] = m2 ? pb[q].z : 0.f;
      Bs[buf][lr][lk + 4 * q + 3] = m3 ? pb[q].w : 0.f;
    }
  };
  floatx16 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[x][y][v] = 0.f;
  // MODE 2: all four 32 x 32 blocks of the wave; 1: not the block (x, y) =
  // (0, 1), which lies above the diagonal in the diagonal waves of a
  // diagonal tile; 0: none (the wave's 64 x 64 block lies above the
  // diagonal).  Each mode is its own branch-free copy of the K loop.
  auto mma = [&](auto mode, int buf) {
    constexpr int MODE = decltype(mode)::value;
    if constexpr (MODE > 0) {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 2) {
        float av[2], bv[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) av[x] = As[buf][wr * 64 + x * 32 + (lane & 31)][kk + (lane >> 5)];
#pragma unroll
        for (int y = 0; y < 2; ++y) bv[y] = Bs[buf][wc * 64 + y * 32 + (lane & 31)][kk + (lane >> 5)];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            if (MODE == 2 || x != 0 || y != 1)
              acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[x], bv[y], acc[x][y], 0, 0, 0);
      }
    }
  };
  // epilogue reads of accumulator tile q = 2 x + y (issued ahead of use)
  auto load_old = [&](int q, float* o) {
    const int x = q >> 1, y = q & 1;
    const int ib = i0 + wr * 64 + x * 32 + (lane >> 5) * 4;
    const int j = j0 + wc * 64 + y * 32 + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) o[v] = syrk_old(F, ld, U, ib + (v >> 2) * 8 + (v & 3), j);
  };
  auto store_new = [&](int q, const float* o, const floatx16& c) {
    const int x = q >> 1, y = q & 1;
    const int ib = i0 + wr * 64 + x * 32 + (lane >> 5) * 4;
    const int j = j0 + wc * 64 + y * 32 + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = ib + (v >> 2) * 8 + (v & 3);
      if (syrk_in(Ue, i, j, a, c1e)) F[(long long)i * ld + j] = o[v] - c[v];
    }
  };
  // The load row U (g_omega = g~ - P z) is not part of the tiles (rows r0 ..
  // U - 1): the wave of a diagonal tile whose 64 x 64 block lies above the
  // diagonal forms it for the tile's 128 columns from the B rows in LDS and
  // z, row U of the operand, read from global memory one chunk ahead.
  const float* zrow = Pb + (long long)U * pl;
  // lane q < KC holds z[kb + q] (one load per chunk), read back by lane reads
  auto zload = [&](int kb) {
    const int k = kb + lane;
    const float v = zrow[min(k, pl - 1)];
    return (lane < KC && k < a.k1) ? v : 0.f;  // select: entries past k1 may hold any bit pattern
  };
  float rz0 = 0.f, rz1 = 0.f;
  auto rowdot = [&](int buf, float zv) {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const float z = lane_value(zv, kk);
      rz0 += z * Bs[buf][lane][kk];
      rz1 += z * Bs[buf][64 + lane][kk];
    }
  };
  auto run = [&](auto mode) {
    constexpr int MODE = decltype(mode)::value;
    float zc = 0.f, zn = 0.f;
    if constexpr (MODE == 0) zc = zload(a.k0);
    load(a.k0);
    store(0, a.k0);
    __syncthreads();
    int buf = 0, kb = a.k0;
    for (; kb + KC < a.k1; kb += KC) {
      load(kb + KC);
      if constexpr (MODE == 0) zn = zload(kb + KC);
      // keep the prefetch ahead of the MFMAs (the scheduler would otherwise
      // sink the loads next to their LDS stores)
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (MODE == 0)
        rowdot(buf, zc);
      else
        mma(mode, buf);
      __builtin_amdgcn_sched_barrier(0);
      store(buf ^ 1, kb + KC);
      __syncthreads();
      buf ^= 1;
      if constexpr (MODE == 0) zc = zn;
    }
    if constexpr (MODE == 0) {
      rowdot(buf, zc);
      const int ja = j0 + lane, jb = j0 + 64 + lane;
      if (ja >= a.c0 && ja < c1e && ja <= U) F[(long long)U * ld + ja] -= rz0;
      if (jb >= a.c0 && jb < c1e && jb <= U) F[(long long)U * ld + jb] -= rz1;
      return;
    }
    float o0[16];
    load_old(0, o0);  // the first epilogue reads overlap the last chunk's MFMAs
    __builtin_amdgcn_sched_barrier(0);
    mma(mode, buf);
    store_new(0, o0, acc[0][0]);
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      if (MODE == 1 && q == 1) continue;
      load_old(q, o0);
      store_new(q, o0, acc[q >> 1][q & 1]);
    }
  };
  // wave-uniform: which of the wave's 32 x 32 blocks hold stored elements
  // (block (x, y) lies above the diagonal when its first column exceeds its
  // last row)
  const int ri = i0 + wr * 64, cj = j0 + wc * 64;
  if (cj > ri + 63)
    run(std::integral_constant<int, 0>{});
  else if (cj >= ri && cj <= ri + 31)  // only (0, 1) above the diagonal
    run(std::integral_constant<int, 1>{});
  else
    run(std::integral_constant<int, 2>{});
}

// Three workgroups per CU: K chunks of 16 (34 KiB of LDS) and at most 168
// VGPRs per lane, so that one workgroup's epilogue and first loads overlap
// the others' MFMAs (two per CU with 32-wide chunks: 2.3 ms per step more).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_syrk128_f32(DevLevel L, SyrkArgs a, int n_samples) {
  constexpr int TM = 128, KC = 16;
  __shared__ float As[2][TM][KC + 1];
  __shared__ float Bs[2][TM][KC + 1];
  // XCD-aware order: workgroup b runs on XCD b % 8; all tiles of one (node,
  // sample) frame go to the same XCD in consecutive order, so its panel
  // columns stay in that XCD's L2 while its tiles are computed.
  const int n_pairs = L.n_nodes * n_samples;
  const int n_tiles = lower_tile_count(a.tiles_r, a.tiles_c);
  const int b = blockIdx.x;
  const int loc = b >> 3;
  const int pair = (loc / n_tiles) * 8 + (b & 7);
  if (pair >= n_pairs) return;
  int ti, tj;
  lower_tile(loc % n_tiles, a.tiles_c, ti, tj);
  const int node = pair / n_samples, s = pair % n_samples;
  const DevNode nd = L.nodes[node];
  const int U = nd.U;
  const int Ue = U - 1;  // tiles cover rows r0 .. U - 1; row U is formed in the diagonal tiles
  const int c1e = a.c1 < 0 ? U + 1 : a.c1;
  const int i0 = a.r0 + ti * TM, j0 = a.c0 + tj * TM;
  if (i0 > Ue || j0 >= c1e) return;
  float* F = frame_ptr<float>(L, node, s);
  const int ld = nd.ld;
  int pl;
  const float* Pb = syrk_operands<float>(L, node, s, F, ld, pl);
  if ((pl % 4) == 0 && (a.k0 % 4) == 0)  // uniform per workgroup
    syrk128_tile<true, KC>(As, Bs, F, ld, Pb, pl, U, Ue, i0, j0, a, c1e);
  else
    syrk128_tile<false, KC>(As, Bs, F, ld, Pb, pl, U, Ue, i0, j0, a, c1e);
}


// ---------------------------------------------------------------------------
// Fused merge of one node for narrow interfaces (gamma <= GP - 1, float32,
// matrix cores): extend-add, partial Cholesky and Schur update in one pass,
// one workgroup per (node, sample), so every frame entry is written once and
// the sons' Schur complements are read once.
//  1. the first gamma columns of every frame row (the panel) are gathered
//     from the sons (eq. Psi_sum) into LDS;
//  2. wave 0 factors the gamma x gamma block in registers (eq. gamma,
//     eq. SchurMinus1), then each thread solves one panel row: P = S L^-T
//     and z = L^-1 g (the rhs row);
//  3. the panel [L ; P ; z] goes to the frame;
//  4. S_omega = S~ - P P^T and g_omega = g~ - P z (eq. SchurC1) for the lower
//     triangle of rows / columns gamma..U in 32 x 32 matrix-core tiles, with
//     S~ gathered from the sons in the tile epilogue.
// Dynamic LDS: 2 nr ints (maps) + nr (GP + 1) floats (panel) + GP floats
// (reciprocal pivots), with
// nr = gamma + 32 ceil((U + 1 - gamma) / 32) rows (tile overhang is zero).
// ---------------------------------------------------------------------------
__host__ __device__ inline int merge_rows(int g, int n) { return g + ((n - g + 31) / 32) * 32; }

size_t merge_small_lds(int max_U, int g, int GP) {
  const int nr = merge_rows(g, max_U + 1);
  return size_t(2) * nr * 4 + size_t(nr) * (GP + 1) * 4 + size_t(GP) * 4;
}

template <int GP, int NT>
__global__ void __launch_bounds__(NT) k_merge_small(DevLevel F, DevLevel S, int n_samples, int* info) {
  constexpr int KP = GP + 1;
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int bad_pivot;
  const int pair = blockIdx.x;
  const int node = pair / n_samples;
  const int s = pair % n_samples;
  const DevNode nd = F.nodes[node];
  const int U = nd.U, n = U + 1, g = F.gam, ld = nd.ld;
  const int nr = merge_rows(g, n);
  int* mA = reinterpret_cast<int*>(smem);
  int* mB = mA + nr;
  float* P = reinterpret_cast<float*>(mB + nr);  // [nr][KP]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  {
    const int* gA = F.maps + nd.map_off;
    const int* gB = gA + n;
    for (int r = tid; r < nr; r += NT) {
      mA[r] = r < n ? gA[r] : -1;
      mB[r] = r < n ? gB[r] : -1;
    }
  }
  if (tid == 0) bad_pivot = 0;
  const DevNode na = S.nodes[2 * node], nb = S.nodes[2 * node + 1];
  const int ga = na.U - na.bnd, gb = nb.U - nb.bnd;
  const float* SA = frame_ptr<float>(S, 2 * node, s) + (long long)ga * na.ld + ga;
  const float* SB = frame_ptr<float>(S, 2 * node + 1, s) + (long long)gb * nb.ld + gb;
  float* Fo = frame_ptr<float>(F, node, s);
  __syncthreads();
  // S~(r, c) from the sons; addresses are valid for absent entries too
  auto gather = [&](int r, int c, float& va, float& vb) {
    const int ar = mA[r], ac = mA[c], br = mB[r], bc = mB[c];
    const long long ia = (ar >= 0 && ac >= 0) ? (long long)max(ar, ac) * na.ld + min(ar, ac) : 0;
    const long long ib = (br >= 0 && bc >= 0) ? (long long)max(br, bc) * nb.ld + min(br, bc) : 0;
    const float xa = SA[ia], xb = SB[ib];
    va = (ar >= 0 && ac >= 0) ? xa : 0.f;
    vb = (br >= 0 && bc >= 0) ? xb : 0.f;
  };
  // 1. panel gather (rows past U and columns past gamma are zero)
  {
    constexpr int UNR = 8;
    const int total = nr * GP;
    for (int base = 0; base < total; base += NT * UNR) {
      float va[UNR], vb[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int e = min(base + u * NT + tid, total - 1);
        gather(e / GP, e % GP, va[u], vb[u]);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int e = base + u * NT + tid;
        const int r = e / GP, c = e % GP;
        if (e < total) P[r * KP + c] = (r < n && c < g && c <= r) ? va[u] + vb[u] : 0.f;
      }
    }
  }
  __syncthreads();
  // 2a. Cholesky of the gamma x gamma block by wave 0 (lane i holds row i)
  if (tid < 64) {
    float a[GP];
    const int lc = min(lane, g - 1);
#pragma unroll
    for (int k = 0; k < GP; ++k) a[k] = (lane < g && k <= lane) ? P[lc * KP + k] : 0.f;
    int bp = 0;
#pragma unroll
    for (int j = 0; j < GP; ++j) {
      if (j < g) {
        float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a[j]), j));
        if (!(d > 0.f) || !(d < 3.0e38f)) {
          if (!bp) bp = j + 1;
          d = 1.f;
        }
        d = sqrtf(d);
        a[j] = lane == j ? d : (lane > j ? a[j] / d : a[j]);
#pragma unroll
        for (int k = j + 1; k < GP; ++k) {
          const float ck = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a[j]), k));  // L_kj
          if (k <= lane) a[k] -= a[j] * ck;
        }
      }
    }
    if (lane < g) {
#pragma unroll
      for (int k = 0; k < GP; ++k)
        if (k <= lane) P[lane * KP + k] = a[k];
    }
    if (lane == 0) bad_pivot = bp;
  }
  __syncthreads();
  if (tid == 0 && bad_pivot && info) atomicCAS(info + s, 0, F.node_base + node + 1);
  // 2b. panel rows below the block: x L^T = a, pivots applied as reciprocals
  float* rP = P + nr * KP;  // [GP]
  if (tid < g) rP[tid] = 1.f / P[tid * KP + tid];
  __syncthreads();
  for (int r = g + tid; r < n; r += NT) {
    float x[GP];
#pragma unroll
    for (int k = 0; k < GP; ++k) x[k] = P[r * KP + k];
#pragma unroll
    for (int j = 0; j < GP; ++j) {
      if (j < g) {
        float v = x[j];
#pragma unroll
        for (int l = 0; l < j; ++l) v -= x[l] * P[j * KP + l];
        x[j] = v * rP[j];
      }
    }
#pragma unroll
    for (int k = 0; k < GP; ++k) P[r * KP + k] = x[k];
  }
  __syncthreads();
  // 3. panel -> the level's panel store, (U+1) x gamma dense (zeros above the
  // diagonal of L), or the frame's first gamma columns
  if (F.panel) {
    float* Po = reinterpret_cast<float*>(F.panel) + (long long)s * F.panel_stride + nd.panel_off;
    const int pld = F.panel_ld;
    for (int e = tid; e < n * GP; e += NT) {
      const int r = e / GP, c = e % GP;
      if (c < g) Po[(long long)r * pld + c] = P[r * KP + c];
    }
  } else {
    for (int e = tid; e < n * GP; e += NT) {
      const int r = e / GP, c = e % GP;
      if (c < g && c <= r) Fo[(long long)r * ld + c] = P[r * KP + c];
    }
  }
  // 4. Schur update tiles over rows / columns g..U-1 (lower tiles only); the
  // load row U follows in step 5 (as its own tile row it would cost a whole
  // row of tiles)
  const int nt = (n - 1 - g + 31) / 32;
  for (int t = wv; t < nt * (nt + 1) / 2; t += NW) {
    const int ti = tri_row(t), tj = t - ti * (ti + 1) / 2;
    const int i0 = g + ti * 32, j0 = g + tj * 32;
    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
    for (int kk = 0; kk < GP; kk += 2) {
      const float av = P[(i0 + (lane & 31)) * KP + kk + (lane >> 5)];
      const float bv = P[(j0 + (lane & 31)) * KP + kk + (lane >> 5)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
    const int j = j0 + (lane & 31);
    float va[16], vb[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = i0 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
      gather(i, j, va[v], vb[v]);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = i0 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
      if (i < n - 1 && j <= i) Fo[(long long)i * ld + j] = va[v] + vb[v] - acc[v];
    }
  }
  // 5. the load row: g_omega = g~ - P z (eq. SchurC1), one column per thread
  for (int j = g + tid; j < n; j += NT) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < GP; ++k) acc += P[U * KP + k] * P[j * KP + k];
    float va, vb;
    gather(U, j, va, vb);
    Fo[(long long)U * ld + j] = va + vb - acc;
  }
}

static constexpr size_t kMaxDynLds = 160 * 1024 - 1024;  // LDS per workgroup minus the static part

// gamma <= 31 only: with 64-column panels the in-register factorization
// loses accuracy (the second refinement correction doubles at 1023^2) and
// the level runs at one workgroup per CU for no net gain.
bool merge_small_ok(const DevLevel& F, bool mfma) {
  if (!mfma || F.is_double || F.gam < 1 || F.gam > 31) return false;
  const int GP = F.gam <= 15 ? 16 : 32;
  return merge_small_lds(F.max_U, F.gam, GP) <= kMaxDynLds;
}

hipError_t launch_merge_small(const DevLevel& F, const DevLevel& S, int n_samples, int* info, hipStream_t st) {
  if (!merge_small_ok(F, true) || S.is_double) return hipErrorInvalidValue;
  dim3 grid(F.n_nodes * n_samples);
  if (F.gam <= 15) {
    const size_t lds = merge_small_lds(F.max_U, F.gam, 16);
    hipLaunchKernelGGL((k_merge_small<16, 256>), grid, dim3(256), lds, st, F, S, n_samples, info);
  } else {
    const size_t lds = merge_small_lds(F.max_U, F.gam, 32);
    hipLaunchKernelGGL((k_merge_small<32, 256>), grid, dim3(256), lds, st, F, S, n_samples, info);
  }
  return hipGetLastError();
}



// ---------------------------------------------------------------------------
// Fused elimination of one node with an interface of 63 nodes (float32,
// matrix cores), one workgroup per (node, sample), on the frame that the
// extend-add has filled (eq. Psi_sum):
//  1. wave 0 reads the first 32 x 32 diagonal block into registers and
//     factors it (eq. gamma, eq. SchurMinus1) while the other waves bring
//     the rest of the panel (the first 63 columns of every frame row) to
//     LDS, row r at P[r * 63 + k] (an odd row length: one column read by
//     consecutive lanes hits distinct banks), zero above the diagonal;
//  2. every thread solves panel rows against the first block, the other 31
//     columns take the rank-32 update on matrix cores, wave 0 factors the
//     second diagonal block while the other waves write the finished first
//     32 columns out, and every thread solves the rows below it;
//  3. the rest of the panel [L ; P ; z] goes to the level's panel store (or
//     the frame);
//  4. S_omega = S~ - P P^T (eq. SchurC1) on rows / columns 63..U-1 in
//     32 x 32 matrix-core tiles, each tile's old values loaded from the frame
//     before its products;
//  5. the load row, g_omega = g~ - P z, one column per thread.
// Operand rows past U are read clamped to row U: they only feed outputs
// that are not stored.  Each frame entry is read and written once; the
// panel is read once.  Pivots are applied as reciprocals.
// ---------------------------------------------------------------------------
constexpr int kMidGam = 63;

size_t eliminate_mid_lds(int max_U) { return size_t(max_U + 1) * kMidGam * 4 + 64 * 4; }

// Right-looking Cholesky of the m x m block (m <= 32) that wave 0 holds one
// row per lane (lane i: a[k] = A_ik for k <= i); pivots and multipliers by
// cross-lane reads.  Entries above the diagonal are updated like the others
// but never read, so no masks are needed.  Leaves 1 / L_ii in rd of lane i;
// returns 1 + the first failing pivot (a non-positive or non-finite pivot
// is replaced by 1), 0 if none.
__device__ __forceinline__ int chol_block32(float (&a)[32], int m, int lane, float& rd) {
  int bp = 0;
  rd = 1.f;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    if (j < m) {
      float d = lane_value(a[j], j);
      if (!(d > 0.f) || !(d < 3.0e38f)) {
        if (!bp) bp = j + 1;
        d = 1.f;
      }
      d = sqrtf(d);
      const float r = 1.f / d;
      if (lane == j) rd = r;
      a[j] = lane == j ? d : a[j] * r;
#pragma unroll
      for (int k = j + 1; k < 32; ++k) a[k] -= a[j] * lane_value(a[j], k);  // L_kj
    }
  }
  return bp;
}

// One panel row r against a diagonal block of width W starting at column c0:
// x L^T = a for x = P[r, c0 .. c0+W), with the rows of L at D[j * G + l] and
// the reciprocal pivots in rd.
template <int W>
__device__ __forceinline__ void solve_row(float* P, const float* D, const float* rd, int r) {
  constexpr int G = kMidGam;
  float x[W];
#pragma unroll
  for (int k = 0; k < W; ++k) x[k] = P[r * G + k];
#pragma unroll
  for (int j = 0; j < W; ++j) {
    float v = x[j];
#pragma unroll
    for (int l = 0; l < j; ++l) v -= x[l] * D[j * G + l];
    x[j] = v * rd[j];
  }
#pragma unroll
  for (int k = 0; k < W; ++k) P[r * G + k] = x[k];
}

// 4 waves per SIMD: two 512-thread workgroups (or one of 1024) per CU.
template <int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
k_eliminate_mid(DevLevel F, int n_samples, int* info) {
  constexpr int NW = NT / 64;
  constexpr int G = kMidGam, G2 = G - 32;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int bad_pivot;
  const int pair = blockIdx.x;
  const int node = pair / n_samples;
  const int s = pair % n_samples;
  const DevNode nd = F.nodes[node];
  const int U = nd.U, ld = nd.ld;
  float* P = reinterpret_cast<float*>(smem);  // [U+1][G]
  float* rdg = P + (U + 1) * G;               // [64] reciprocal pivots
  float* Fo = frame_ptr<float>(F, node, s);
  float* Po = F.panel ? panel_ptr<float>(F, node, s) : nullptr;
  const int pld = F.panel_ld;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // panel entry (r, k) -> the panel store, or the frame's first G columns
  auto put = [&](int r, int k, float v) {
    if (Po) Po[(long long)r * pld + k] = v;
    else Fo[(long long)r * ld + k] = v;
  };
  if (wv == 0) {
    // 1a. first diagonal block straight from the frame, factored in registers
    float a[32];
    const int lc = min(lane, 31);
#pragma unroll
    for (int k = 0; k < 32; ++k) a[k] = Fo[(long long)lc * ld + min(k, lc)];
    float rd;
    const int bp = chol_block32(a, 32, lane, rd);
    if (lane < 32) {
#pragma unroll
      for (int k = 0; k < 32; ++k) P[lane * G + k] = k <= lane ? a[k] : 0.f;
      rdg[lane] = rd;
    }
    if (lane == 0) bad_pivot = bp;
  } else {
    // 1b. the rest of the panel -> LDS (all loads of a batch before its stores)
    constexpr int UNR = 8;
    const int t0 = tid - 64;
    const int total = (U + 1) * G;
    for (int base = 0; base < total; base += (NT - 64) * UNR) {
      float v[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int e = min(base + u * (NT - 64) + t0, total - 1);
        const int r = e / G, k = e % G;
        v[u] = Fo[(long long)r * ld + min(k, r)];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int e = base + u * (NT - 64) + t0;
        const int r = e / G, k = e % G;
        if (e < total && (r >= 32 || k >= 32)) P[e] = (k <= r) ? v[u] : 0.f;
      }
    }
  }
  __syncthreads();
  // 2a. rows 32..U, columns 0..31 (one row per thread)
  for (int r = 32 + tid; r <= U; r += NT) solve_row<32>(P, P, rdg, r);
  __syncthreads();
  // 2b. columns 32..62 of rows 32..U: A(r, c) -= sum_{k<32} A(r, k) A(c, k)
  // on matrix cores, 32-row tiles, columns 32..63 (c = 63 is not stored)
  for (int t = wv; 32 + t * 32 <= U; t += NW) {
    const int i0 = 32 + t * 32;
    const int ra = min(i0 + (lane & 31), U), rb = min(32 + (lane & 31), U);
    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
    for (int kk = 0; kk < 32; kk += 2) {
      const int k = kk + (lane >> 5);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(P[ra * G + k], P[rb * G + k], acc, 0, 0, 0);
    }
    const int c = 32 + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = i0 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
      if (c < G && c <= i && i <= U) P[i * G + c] -= acc[v];
    }
  }
  __syncthreads();
  if (wv == 0) {
    // 2c. second diagonal block (31 x 31) by wave 0
    float a[32];
    const int lc = 32 + min(lane, G2 - 1);
#pragma unroll
    for (int k = 0; k < 32; ++k) a[k] = k < G2 ? P[lc * G + 32 + min(k, lane)] : 0.f;
    float rd;
    const int bp = chol_block32(a, G2, lane, rd);
    if (lane < G2) {
#pragma unroll
      for (int k = 0; k < G2; ++k)
        if (k <= lane) P[(32 + lane) * G + 32 + k] = a[k];
      rdg[32 + lane] = rd;
    }
    if (lane == 0 && bp && !bad_pivot) bad_pivot = 32 + bp;
  } else {
    // 3a. meanwhile: the finished columns 0..31 of every row go out
    for (int e = tid - 64; e < (U + 1) * 32; e += NT - 64) {
      const int r = e >> 5, k = e & 31;
      if (k <= r) put(r, k, P[r * G + k]);
    }
  }
  __syncthreads();
  // 2d. rows 63..U, columns 32..62 (one row per thread)
  for (int r = G + tid; r <= U; r += NT) solve_row<G2>(P + 32, P + 32 * G + 32, rdg + 32, r);
  __syncthreads();
  if (tid == 0 && bad_pivot && info) atomicCAS(info + s, 0, F.node_base + node + 1);
  // 3b. columns 32..62 of rows 32..U
  for (int e = tid; e < (U - 31) * G2; e += NT) {
    const int r = 32 + e / G2, k = 32 + e % G2;
    if (k <= r) put(r, k, P[r * G + k]);
  }
  // 4. Schur update tiles over rows / columns G..U-1 (lower tiles only); the
  // old values of a wave's next tile are loaded while its current tile is
  // multiplied
  const int nt = (U - G + 31) / 32;
  const int ntiles = nt * (nt + 1) / 2;
  auto load_old = [&](int t, float (&o)[16]) {
    const int ti = tri_row(t), tj = t - ti * (ti + 1) / 2;
    const int i0 = G + ti * 32, j = G + tj * 32 + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = i0 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
      o[v] = Fo[(long long)min(i, U - 1) * ld + min(j, U - 1)];
    }
  };
  float nxt[16];
  if (wv < ntiles) load_old(wv, nxt);
  for (int t = wv; t < ntiles; t += NW) {
    const int ti = tri_row(t), tj = t - ti * (ti + 1) / 2;
    const int i0 = G + ti * 32, j0 = G + tj * 32;
    const int j = j0 + (lane & 31);
    float old[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) old[v] = nxt[v];
    if (t + NW < ntiles) load_old(t + NW, nxt);
    const float* pa = P + min(i0 + (lane & 31), U) * G + (lane >> 5);
    const float* pb = P + min(j, U) * G + (lane >> 5);
    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
    for (int kk = 0; kk < G - 1; kk += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(pa[kk], pb[kk], acc, 0, 0, 0);
    {  // k = 62 (lanes 0..31) and the zero column 63 (lanes 32..63)
      const int q = (lane >> 5) ? 0 : G - 1;
      const float av = pa[q];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32((lane >> 5) ? 0.f : av, pb[q], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = i0 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
      if (i < U && j <= i) Fo[(long long)i * ld + j] = old[v] - acc[v];
    }
  }
  // 5. the load row: g_omega = g~ - P z (eq. SchurC1), one column per thread
  for (int j = G + tid; j <= U; j += NT) {
    const float o = Fo[(long long)U * ld + j];
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < G; ++k) acc += P[U * G + k] * P[j * G + k];
    Fo[(long long)U * ld + j] = o - acc;
  }
}

// Interfaces of 63 nodes on float32 matrix-core levels whose panel fits in
// LDS.  Two workgroups share a CU while the panel takes at most half of its
// LDS; larger panels get 1024 threads.
bool eliminate_mid_ok(const DevLevel& L, bool mfma) {
  if (!mfma || L.is_double || L.gam != kMidGam || L.max_U <= L.gam) return false;
  return eliminate_mid_lds(L.max_U) <= kMaxDynLds;
}

hipError_t launch_eliminate_mid(const DevLevel& L, int n_samples, int* info, hipStream_t st) {
  if (!eliminate_mid_ok(L, true)) return hipErrorInvalidValue;
  const size_t lds = eliminate_mid_lds(L.max_U);
  dim3 grid(L.n_nodes * n_samples);
  if (lds <= 80 * 1024)
    hipLaunchKernelGGL(k_eliminate_mid<512>, grid, dim3(512), lds, st, L, n_samples, info);
  else
    hipLaunchKernelGGL(k_eliminate_mid<1024>, grid, dim3(1024), lds, st, L, n_samples, info);
  return hipGetLastError();
}

// Plain FMA version of the same update (no matrix cores), kept as a
// cross-check of the MFMA lane layouts.
template <typename T>
__global__ void __launch_bounds__(256) k_syrk_simple(DevLevel L, SyrkArgs a, int n_samples) {
  constexpr int KC = SyrkCfg<T>::KC;
  __shared__ T As[64][KC + 1];
  __shared__ T Bs[64][KC + 1];
  const int pair = blockIdx.x;
  const int node = pair / n_samples, s = pair % n_samples;
  const DevNode nd = L.nodes[node];
  const int U = nd.U;
  const int c1e = a.c1 < 0 ? U + 1 : a.c1;
  int ti, tj;
  lower_tile(blockIdx.y, a.tiles_c, ti, tj);
  const int i0 = a.r0 + ti * 64, j0 = a.c0 + tj * 64;
  if (i0 > U || j0 >= c1e) return;
  T* F = frame_ptr<T>(L, node, s);
  const int ld = nd.ld;
  int pl;
  const T* Pb = syrk_operands<T>(L, node, s, F, ld, pl);
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  T acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = T(0);
  for (int kb = a.k0; kb < a.k1; kb += KC) {
    __syncthreads();
    syrk_load_chunk<T>(As, Bs, Pb, pl, U, i0, j0, kb, a.k1);
    __syncthreads();
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] += As[tr + 16 * x][kk] * Bs[tc + 16 * y][kk];
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) syrk_store<T>(F, ld, U, i0 + tr + 16 * x, j0 + tc + 16 * y, a, c1e, acc[x][y]);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static int ceil_div(long long a, long long b) { return int((a + b - 1) / b); }

hipError_t launch_extend_add(const DevLevel& F, const DevLevel& S, int n_samples, hipStream_t st) {
  const long long nt = ((long long)F.max_U + 1 + 63) / 64;  // 64 x 64 tiles per side
  const long long nwg = (long long)ceil_div(F.n_nodes * n_samples, 8) * 8 * (nt * (nt + 1) / 2);
  if (nwg > 0x7fffffffll) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(nwg)), block(256);
  if (F.is_double && S.is_double)
    hipLaunchKernelGGL((k_extend_add<double, double>), grid, block, 0, st, F, S, n_samples);
  else if (F.is_double)
    hipLaunchKernelGGL((k_extend_add<float, double>), grid, block, 0, st, F, S, n_samples);
  else if (!S.is_double)
    hipLaunchKernelGGL((k_extend_add<float, float>), grid, block, 0, st, F, S, n_samples);
  else
    return hipErrorInvalidValue;  // a double son under a float father is never planned
  return hipGetLastError();
}

template <typename T, int NB>
static void launch_panel_t(const DevLevel& L, int k0, int kb, int n_samples, int* info, hipStream_t st) {
  const int pairs = L.n_nodes * n_samples;
  const int rows = L.max_U + 1 - (k0 + kb);
  hipLaunchKernelGGL((k_panel_diag<T, NB>), dim3(pairs), dim3(64), 0, st, L, k0, kb, n_samples, info);
  if (rows > 0) {
    constexpr int RW = PanelCfg<T>::RW;
    hipLaunchKernelGGL((k_panel_rows<T, NB>), dim3(pairs, ceil_div(rows, RW)), dim3(RW), 0, st, L, k0, kb,
                       n_samples);
  }
}

hipError_t launch_panel(const DevLevel& L, int k0, int kb, int n_samples, int* info, hipStream_t st) {
  if (kb < 1 || kb > kPanelNB) return hipErrorInvalidValue;
  // the smallest compiled panel width that holds kb columns
  if (L.is_double) {
    if (kb <= 16) launch_panel_t<double, 16>(L, k0, kb, n_samples, info, st);
    else if (kb <= 32) launch_panel_t<double, 32>(L, k0, kb, n_samples, info, st);
    else launch_panel_t<double, 64>(L, k0, kb, n_samples, info, st);
  } else {
    if (kb <= 16) launch_panel_t<float, 16>(L, k0, kb, n_samples, info, st);
    else if (kb <= 32) launch_panel_t<float, 32>(L, k0, kb, n_samples, info, st);
    else launch_panel_t<float, 64>(L, k0, kb, n_samples, info, st);
  }
  return hipGetLastError();
}

// Large frames (16-byte aligned rows) with enough work per tile use the
// 128 x 128 matrix-core tile: K >= 96 and at least 96 output columns (a
// 127-column half of a 255-column interface fills one tile column).
// Narrow updates (K < 96) go to the 64 x 64 tile: with two K chunks per
// tile the 128 x 128 tile's read-modify-write dominates (measured at
// 1023^2, 448-row frames, K = 63: 1.5 ms instead of 2.3 ms; no gain at 320
// rows).
bool syrk_uses_big_tile(const DevLevel& L, int k0, int k1, int r0, int c0, int c1, bool mfma, int tile) {
  if (!mfma || L.is_double || k1 <= k0) return false;  // the 128 x 128 tile is float32 matrix-core only
  if (tile == 64 || r0 != c0) return false;  // diagonal tiles of the 128 x 128 grid form the load row
  if (tile == 128) return true;
  const int rows = L.max_U + 1 - r0;
  const int cols = (c1 < 0 ? L.max_U + 1 : c1) - c0;
  if (k1 - k0 < 96) return false;
  return rows >= 192 && cols >= 96 && (k0 % 4) == 0 && L.max_U + 1 >= 64;
}

hipError_t launch_syrk(const DevLevel& L, int k0, int k1, int r0, int c0, int c1, int n_samples, bool mfma,
                       int tile, hipStream_t st) {
  if (r0 != c0) return hipErrorInvalidValue;  // the tile grids hold the tiles on or below the diagonal
  if (k1 <= k0) return hipSuccess;
  SyrkArgs a{k0, k1, r0, c0, c1, 0, 0, 0};
  const int rows = L.max_U + 1 - r0;
  const int cols = (c1 < 0 ? L.max_U + 1 : c1) - c0;
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const bool big = syrk_uses_big_tile(L, k0, k1, r0, c0, c1, mfma, tile);
  if (!big && mfma && !L.is_double && c1 >= 0 && cols <= 32 && tile != 64) {
    // tall 128 x 32 tiles, rows r0 .. U (the load row included)
    a.sep = 0;
    a.tiles_r = ceil_div(rows, 128);
    a.tiles_c = 1;
    dim3 grid(L.n_nodes * n_samples, a.tiles_r);
    hipLaunchKernelGGL(k_syrk_tall_f32, grid, dim3(256), 0, st, L, a, n_samples);
    return hipGetLastError();
  }
  const int TM = big ? 128 : 64;
  // the matrix-core tiles cover rows r0 .. U-1; the load row U is formed by
  // the idle wave of the diagonal tiles
  a.sep = mfma ? 1 : 0;
  const int tr = ceil_div(rows - a.sep, TM);
  a.tiles_c = ceil_div(c1 < 0 ? cols - a.sep : cols, TM);
  a.tiles_r = tr;
  if (tr > 0 && a.tiles_c > 0) {
    const int n_low = lower_tile_count(tr, a.tiles_c);
    dim3 grid(L.n_nodes * n_samples, n_low), block(256);
    // matrix-core tiles: one dimension, (node, sample) pairs padded to a
    // multiple of 8 for the XCD-aware order
    const long long nwg = (long long)ceil_div(L.n_nodes * n_samples, 8) * 8 * n_low;
    if (mfma && nwg > 0x7fffffffll) return hipErrorInvalidValue;
    if (big)
      hipLaunchKernelGGL(k_syrk128_f32, dim3(unsigned(nwg)), block, 0, st, L, a, n_samples);
    else if (L.is_double && mfma)
      hipLaunchKernelGGL(k_syrk_mfma_f64, dim3(unsigned(nwg)), block, 0, st, L, a, n_samples);
    else if (L.is_double)
      hipLaunchKernelGGL(k_syrk_simple<double>, grid, block, 0, st, L, a, n_samples);
    else if (mfma)
      hipLaunchKernelGGL(k_syrk_mfma_f32, dim3(unsigned(nwg)), block, 0, st, L, a, n_samples);
    else
      hipLaunchKernelGGL(k_syrk_simple<float>, grid, block, 0, st, L, a, n_samples);
  }
  return hipGetLastError();
}

}  // namespace hdd
