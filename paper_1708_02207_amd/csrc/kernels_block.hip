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
//                    live in two ping-pong LDS buffers; each node's retained
//                    columns [L ; P ; z] (the factored Phi of the node) go to
//                    a compact HBM store; the block root's full frame (with
//                    S_omega and g_omega) goes to the global frame store.
//  k_block_topdown   Root to Leaves inside the block (Section 3.4): from u on
//                    the block boundary, solve every interface of the block.
//  k_block_forward   bottom-up propagation of a new load (the residual of the
//                    refinement) through the block's factors.
#include <algorithm>
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace hdd {

typedef float floatx16 __attribute__((ext_vector_type(16)));

__constant__ int c_mb_local[3][3] = {  // micro-block local node (a, b) -> frame index
    {1, 2, 3},
    {8, 0, 4},
    {7, 6, 5}};

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

template <int S, int K> struct Lv {
  static constexpr int Lm = 2 * ilog2c(S / 2);  // micro level
  static constexpr int w = S >> ((K + 1) / 2);
  static constexpr int h = S >> (K / 2);
  static constexpr int n = 1 << K;
  static constexpr int gam = (K == Lm) ? 1 : (w >= h ? h - 1 : w - 1);
  static constexpr int bnd = 2 * (w + h);
  static constexpr int U = gam + bnd;
  static constexpr int ld = U + 1;              // logical frame size
  static constexpr int ldp = ld | 1;              // odd LDS row stride (no bank conflicts on columns)
  static constexpr int fsz = ld * ldp;            // LDS elements per frame
  static constexpr int per = ld * gam;            // compact elements per node
};

// Largest per-level index table (maps: n * 2 * (U+1), local ids: n * U).
template <int S, int K> constexpr int idx_max_from() {
  using L = Lv<S, K>;
  constexpr int a = (K < L::Lm) ? L::n * 2 * L::ld : 0;
  constexpr int b = L::n * L::U;
  constexpr int m = a > b ? a : b;
  if constexpr (K < L::Lm) {
    constexpr int rest = idx_max_from<S, K + 1>();
    return m > rest ? m : rest;
  } else {
    return m;
  }
}
template <int S> constexpr int kIdxMax = idx_max_from<S, 0>();

// Extend-add gather table of the build kernel.  Every block shares the
// sub-tree, so the LDS addresses of the extend-add are the same for all of
// them: entry e of level K (K above the micro level) names one lower-triangle
// element (t, r, c) of the level's frames and the two son elements merged into
// it, as element offsets from the start of the kernel's LDS frame buffers:
// x = dst | a << 16, y = b, with a (b) the son-A (son-B) element or the zero
// slot 2 * max_buf when the row or column is not in that son (Section 2.4,
// eq. S_omega).  Level K's frames live in buffer (Lm - K) & 1.
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
__device__ __forceinline__ void ext_entry(const DevBlocks& B, int e, uint2* out) {
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
    const int cur = ((L::Lm - K) & 1) * B.max_buf, prev = ((L::Lm - K + 1) & 1) * B.max_buf;
    const int* mA = B.maps + B.lv[K].map_off + t * 2 * L::ld;
    const int* mB = mA + L::ld;
    const int sa = prev + (2 * t) * C::fsz + C::gam * C::ldp + C::gam, sb = sa + C::fsz;
    const int ar = mA[r], ac = mA[c], br = mB[r], bc = mB[c];
    const int a = (ar >= 0 && ac >= 0) ? sa + max(ar, ac) * C::ldp + min(ar, ac) : zero;
    const int b = (br >= 0 && bc >= 0) ? sb + max(br, bc) * C::ldp + min(br, bc) : zero;
    const int dst = cur + t * L::fsz + r * L::ldp + c;
    out[ext_off<S, K>() + e] = make_uint2(unsigned(dst) | (unsigned(a) << 16), unsigned(b));
  }
}

template <int S> __global__ void k_block_ext(DevBlocks B, uint2* __restrict__ ext) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ext_total<S>()) ext_entry<S, 0>(B, e, ext);
}

__device__ __forceinline__ void stage_ints(int* dst, const int* src, int n) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
}

template <typename T> __device__ __forceinline__ T* cst_block(const DevBlocks& B, int q, int s) {
  return reinterpret_cast<T*>(B.cst) + (long long)s * B.cst_stride + (long long)q * B.cst_size;
}

constexpr int NT = 256;   // threads of the top-down / forward kernels
constexpr int NTB = 512;  // threads of the build kernel

// ---------------------------------------------------------------------------
// Column J of the left-looking partial Cholesky for all n frames of a level,
// one barrier per column: every thread of a node recomputes the pivot
// L_JJ = sqrt(A_JJ - sum_l L_Jl^2) from row J (whose diagonal entry is left
// untouched until the end), the thread of row J records it in dg, and the
// rows below (interface, boundary and load rows) take
// L_iJ = (A_iJ - sum_l L_il L_Jl) / L_JJ.  The recorded pivots are written to
// the diagonal after the last column.  Unrolled over the (compile-time)
// columns so every inner loop has a fixed length.
template <typename T, typename L, int J>
__device__ __forceinline__ void crout_columns(T* cur, T* dg, int& bad_pivot) {
  if constexpr (J < L::gam) {
    constexpr int ld = L::ldp;
    constexpr int m = L::U + 1 - J;  // rows J .. U
    for (int e = threadIdx.x; e < L::n * m; e += NTB) {
      const int t = e / m, i = J + e % m;
      T* F = cur + t * L::fsz;
      T d = F[J * ld + J];
#pragma unroll
      for (int l = 0; l < J; ++l) d -= F[J * ld + l] * F[J * ld + l];
      const bool ok = (d > T(0)) && (d < T(1e300));
      d = ok ? sqrt(d) : T(1);
      if (i == J) {
        if (!ok) bad_pivot = 1;
        dg[t * L::gam + J] = d;
      } else {
        T v = F[i * ld + J];
#pragma unroll
        for (int l = 0; l < J; ++l) v -= F[i * ld + l] * F[J * ld + l];
        F[i * ld + J] = v / d;
      }
    }
    __syncthreads();
    crout_columns<T, L, J + 1>(cur, dg, bad_pivot);
  } else {
    for (int e = threadIdx.x; e < L::n * L::gam; e += NTB) {
      const int t = e / L::gam, j = e % L::gam;
      cur[t * L::fsz + j * L::ldp + j] = dg[e];
    }
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
__device__ __forceinline__ void build_level(T* base, T* cur, T* cst, const DevBlocks& B, T* dg, int& bad_pivot,
                                            const uint2 (&tab)[ext_regs<T, S, K>()]) {
  using L = Lv<S, K>;
  const int tid = threadIdx.x;
  constexpr int NB = NTB;
  if constexpr (K < L::Lm) {
    // S_omega = S~_A + S~_B (eq. S_omega): all gathers of the thread, then
    // all stores (the table's elements of one level never overlap)
    constexpr int E = ext_count<S, K>(), NP = ext_regs<T, S, K>();
    T v[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) v[j] = base[tab[j].x >> 16] + base[tab[j].y];
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (j + 1 < NP || tid + NB * j < E) base[tab[j].x & 0xffffu] = v[j];
    __syncthreads();
  }
  // Partial Cholesky of the first gam columns (left-looking, column by
  // column): L_jj = sqrt(A_jj - sum_l L_jl^2), then every row below
  // (interface, boundary and load rows) L_ij = (A_ij - sum_l L_il L_jl) / L_jj.
  constexpr int g = L::gam, ld = L::ldp;
  crout_columns<T, L, 0>(cur, dg, bad_pivot);
  // Schur update of the boundary block and the load row (rank-g, eq.
  // SchurC1): S[i][l] -= sum_k P[i][k] P[l][k], g <= l <= i <= U.
  if constexpr (std::is_same<T, float>::value && g >= 7) {
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
      const int ra = g + ti * 32 + (lane & 31), rb = g + tj * 32 + (lane & 31);
      const T* pa = F + min(ra, L::U) * ld;
      const T* pb = F + min(rb, L::U) * ld;
      floatx16 acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
      for (int kk = 0; kk < g; kk += 2) {
        const int k = kk + (lane >> 5);
        const float av = (k < g && ra <= L::U) ? pa[k] : 0.f;
        const float bv = (k < g && rb <= L::U) ? pb[k] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
      }
      const int l = g + tj * 32 + (lane & 31);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = g + ti * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        if (i <= L::U && l <= i) F[i * ld + l] -= acc[v];
      }
    }
  } else {
    constexpr int nr = L::U + 1 - g;
    for (int e = tid; e < L::n * nr * nr; e += NB) {
      const int t = e / (nr * nr), p = e % (nr * nr);
      const int i = g + p / nr, l = g + p % nr;
      if (l > i) continue;
      T* F = cur + t * L::fsz;
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < g; ++k) acc += F[i * ld + k] * F[l * ld + k];
      F[i * ld + l] -= acc;
    }
  }
  __syncthreads();
  // retained columns [L ; P ; z] of every node -> compact store
  T* out = cst + B.lv[K].cst_off;
  for (int e = tid; e < L::n * L::per; e += NB) {
    const int t = e / L::per, rc = e % L::per;
    const int r = rc / g, c = rc % g;
    out[e] = (c <= r) ? cur[t * L::fsz + r * ld + c] : T(0);  // ld = physical stride here
  }
  __syncthreads();
}

// Loads this thread's entries of level K's gather table.
template <typename T, int S, int K>
__device__ __forceinline__ void load_ext(const DevBlocks& B, uint2 (&tab)[ext_regs<T, S, K>()]) {
  constexpr int E = ext_count<S, K>();
  if constexpr (E > 0) {
    const uint2* src = B.ext + ext_off<S, K>();
#pragma unroll
    for (int j = 0; j < ext_regs<T, S, K>(); ++j) tab[j] = src[min(int(threadIdx.x) + NTB * j, E - 1)];
  }
}

template <typename T, int S, int K>
__device__ __forceinline__ void build_levels(T* base, T* cur, T* prev, T* cst, const DevBlocks& B, T* dg,
                                             int& bad_pivot, const uint2 (&tab)[ext_regs<T, S, K>()]) {
  if constexpr (K > 0) {
    uint2 nxt[ext_regs<T, S, K - 1>()];
    load_ext<T, S, K - 1>(B, nxt);
    build_level<T, S, K>(base, cur, cst, B, dg, bad_pivot, tab);
    build_levels<T, S, K - 1>(base, prev, cur, cst, B, dg, bad_pivot, nxt);
  } else {
    build_level<T, S, K>(base, cur, cst, B, dg, bad_pivot, tab);
  }
}

// Largest n * gam over the levels of a block (pivots recorded per column).
template <int S, int K> constexpr int gam_nodes_from() {
  using L = Lv<S, K>;
  constexpr int m = L::n * L::gam;
  if constexpr (K < L::Lm) {
    constexpr int rest = gam_nodes_from<S, K + 1>();
    return m > rest ? m : rest;
  } else {
    return m;
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
  __shared__ T dg[gam_nodes_from<S, 0>()];
  const int q = blockIdx.x / n_samples;
  const int s = blockIdx.x % n_samples;
  const int X0 = B.origin[2 * q], Y0 = B.origin[2 * q + 1];
  const int tid = threadIdx.x;
  // the first extend-add's gather entries are in flight during the assembly
  uint2 first[ext_regs<T, S, (Lm > 0 ? Lm - 1 : 0)>()];
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
  // micro-blocks: assemble the 9 x 9 local systems (lower triangle + load row)
  for (int e = tid; e < M::n * M::fsz; e += NTB) buf0[e] = T(0);
  __syncthreads();
  {
    const double h = 1.0 / nc;
    const double area = 0.5 * h * h;
    for (int t = tid; t < M::n; t += NTB) {
      T* F = buf0 + t * M::fsz;
      const int a0 = B.micro_xy[2 * t], b0 = B.micro_xy[2 * t + 1];  // local corner
      bool ok = true;
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int ca = 0; ca < 2; ++ca)
#pragma unroll
          for (int tri = 0; tri < 2; ++tri) {
            // T-: (0,0),(1,0),(1,1); T+: (0,0),(1,1),(0,1) relative to the cell corner
            const int vx[3] = {ca, ca + 1, tri == 0 ? ca + 1 : ca};
            const int vy[3] = {cb, tri == 0 ? cb : cb + 1, cb + 1};
            const double kap = kL[(b0 + cb) * 2 * S + (a0 + ca) * 2 + tri];
            ok = ok && (kap > 0.0) && (kap < 1.0e300);
            const double det = double((vx[1] - vx[0]) * (vy[2] - vy[0]) - (vx[2] - vx[0]) * (vy[1] - vy[0]));
            const double gx[3] = {double(vy[1] - vy[2]), double(vy[2] - vy[0]), double(vy[0] - vy[1])};
            const double gy[3] = {double(vx[2] - vx[1]), double(vx[0] - vx[2]), double(vx[1] - vx[0])};
            const double scale = kap / (2.0 * fabs(det));
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const int ia = c_mb_local[vy[a]][vx[a]];
#pragma unroll
              for (int b = 0; b < 3; ++b) {
                const int ib = c_mb_local[vy[b]][vx[b]];
                if (ib <= ia) F[ia * M::ldp + ib] += T(scale * (gx[a] * gx[b] + gy[a] * gy[b]));
              }
              const double fv = fL[(b0 + vy[a]) * S1 + (a0 + vx[a])];
              F[9 * M::ldp + ia] += T(area * fv / 3.0);
            }
          }
      if (!ok && bad) atomicCAS(bad + s, 0, 1);
    }
  }
  __syncthreads();
  T* cst = cst_block<T>(B, q, s);
  int bp = 0;
  {
    const uint2 none[1] = {make_uint2(0u, 0u)};
    build_level<T, S, Lm>(buf0, buf0, cst, B, dg, bp, none);
    if constexpr (Lm > 0) build_levels<T, S, Lm - 1>(buf0, buf1, buf0, cst, B, dg, bp, first);
  }
  if (bp) bad_pivot = 1;
  __syncthreads();
  // block root frame -> global frame store (lower triangle)
  {
    using R = Lv<S, 0>;
    const T* root = (Lm % 2 == 0) ? buf0 : buf1;
    const DevNode nd = B.top.nodes[q];
    T* G = reinterpret_cast<T*>(B.top.frames) + (long long)s * B.top.stride + nd.frame_off;
    for (int e = tid; e < R::ld * R::ld; e += NTB) {
      const int r = e / R::ld, c = e % R::ld;
      if (c <= r) G[(long long)r * nd.ld + c] = root[r * R::ldp + c];
    }
  }
  if (tid == 0 && bad_pivot && info) atomicCAS(info + s, 0, B.top.node_base + q + 1);
}

// ---------------------------------------------------------------------------
// Shared pieces of the block solves.
//
// Staging of a block's compact factors into LDS with 16-byte loads (the
// per-block store is a multiple of 16 bytes whenever cst_size * sizeof(T) is).
template <typename T>
__device__ __forceinline__ void stage_factors(T* dst, const T* src, int n_elems) {
  const int bytes = n_elems * int(sizeof(T));
  if ((bytes & 15) == 0 && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
    const uint4* s4 = reinterpret_cast<const uint4*>(src);
    uint4* d4 = reinterpret_cast<uint4*>(dst);
    for (int e = threadIdx.x; e < bytes / 16; e += NT) d4[e] = s4[e];
  } else {
    for (int e = threadIdx.x; e < n_elems; e += NT) dst[e] = src[e];
  }
}

// Lanes per dot product of a level's GEMV: the largest power of two (at most
// 16) such that n * gam * P threads fit in the workgroup.
constexpr int gemv_split(int work) {
  int p = 1;
  while (p < 16 && work * p * 2 <= NT) p *= 2;
  return p;
}

// The triangular solves of a level run one node per group of gam lanes,
// floor(64 / gam) groups per wave, with the pivot values broadcast by shuffles.
template <int G> struct Groups {
  static constexpr int per_wave = 64 / G;
};

// ---------------------------------------------------------------------------
// Top-down: the block's compact factors are staged in LDS, u on the block's
// (S+1)^2 nodes lives in LDS; levels are solved root first.
template <typename T, int S, int K>
__device__ __forceinline__ void topdown_level(const DevBlocks& B, const T* cst, const double* vz, double* uL,
                                              double* rb, int* idx) {
  using L = Lv<S, K>;
  constexpr int g = L::gam, U = L::U, nbd = L::bnd;
  constexpr int P = gemv_split(L::n * g);
  static_assert(L::n * g * P <= NT, "level GEMV does not fit the workgroup");
  const int tid = threadIdx.x;
  const T* base = cst + B.lv[K].cst_off;
  // idx holds this level's local ids (staged by the caller or the level above)
  const int* lids = idx;
  // rb = z - P^T u_Gamma: P lanes per entry, reduced by shuffles (the P lanes
  // of an entry are consecutive and P divides 64, so they share a wave)
  if (tid < L::n * g * P) {
    const int w = tid / P, p = tid % P;
    const int t = w / g, i = w % g;
    const T* blk = base + t * L::per;
    const int* lid = lids + t * U;
    double acc = 0.0;
#pragma unroll
    for (int j = p; j < nbd; j += P) acc += double(blk[(g + j) * g + i]) * uL[lid[g + j]];
#pragma unroll
    for (int o = P / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (p == 0) rb[w] = (vz ? vz[B.lv[K].vec_off + w] : double(blk[U * g + i])) - acc;
  }
  __syncthreads();
  // the next level's local ids are loaded into registers now, so their
  // latency overlaps the triangular solves
  constexpr int NN = (K < L::Lm) ? Lv<S, (K < L::Lm ? K + 1 : K)>::n * Lv<S, (K < L::Lm ? K + 1 : K)>::U : 1;
  constexpr int NP = (NN + NT - 1) / NT;
  int pre[NP];
  if constexpr (K < L::Lm) {
    const int* src = B.lids + B.lv[K + 1].lid_off;
#pragma unroll
    for (int j = 0; j < NP; ++j) pre[j] = src[min(tid + NT * j, NN - 1)];
  }
  // back substitution L^T x = rb, one node per group of g lanes
  {
    constexpr int GPW = Groups<g>::per_wave;
    constexpr int NW = (L::n + GPW - 1) / GPW;
    static_assert(NW * 64 <= NT, "level solve does not fit the workgroup");
    const int wv = tid >> 6, lane = tid & 63;
    const int grp = lane / g, i = lane % g;
    const int t = wv * GPW + grp;
    const bool act = grp < GPW && t < L::n;
    if (wv < NW) {
      const T* blk = base + (act ? t : 0) * L::per;
      const int gb = grp * g;
      double v = act ? rb[t * g + i] : 0.0;
#pragma unroll
      for (int l = g - 1; l >= 0; --l) {
        const double xl = __shfl(v, gb + l) / double(blk[l * g + l]);
        if (i == l) v = xl;
        else if (i < l) v -= double(blk[l * g + i]) * xl;
      }
      if (act) uL[lids[t * U + i]] = v;
    }
  }
  __syncthreads();
  if constexpr (K < L::Lm) {
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (tid + NT * j < NN) idx[tid + NT * j] = pre[j];
    __syncthreads();
  }
}

template <typename T, int S, int K>
__device__ __forceinline__ void topdown_levels(const DevBlocks& B, const T* cst, const double* vz, double* uL,
                                               double* rb, int* idx) {
  topdown_level<T, S, K>(B, cst, vz, uL, rb, idx);
  if constexpr (K < Lv<S, 0>::Lm) topdown_levels<T, S, K + 1>(B, cst, vz, uL, rb, idx);
}

template <typename T, int S>
__global__ void __launch_bounds__(NT) k_block_topdown(DevBlocks B, const int* __restrict__ list, int n_samples,
                                                      int nc, double* __restrict__ u, long long ustride,
                                                      int from_vec) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int S1 = S + 1;
  T* cs = reinterpret_cast<T*>(smem);                                    // cst_size
  double* uL = reinterpret_cast<double*>(smem + ((size_t(B.cst_size) * sizeof(T) + 15) / 16) * 16);
  double* rb = uL + S1 * S1;                                             // max n * gam
  __shared__ int idx[kIdxMax<S>];
  const int q = list[blockIdx.x / n_samples];
  const int s = blockIdx.x % n_samples;
  const int X0 = B.origin[2 * q], Y0 = B.origin[2 * q + 1];
  const int tid = threadIdx.x;
  double* us = u + (long long)s * ustride;
  stage_factors<T>(cs, cst_block<T>(B, q, s), B.cst_size);
  for (int e = tid; e < S1 * S1; e += NT) uL[e] = us[(long long)(Y0 + e / S1) * (nc + 1) + X0 + e % S1];
  stage_ints(idx, B.lids + B.lv[0].lid_off, Lv<S, 0>::n * Lv<S, 0>::U);
  __syncthreads();
  const double* vz = from_vec ? B.vec + (long long)s * B.vec_stride + (long long)q * B.vec_size : nullptr;
  topdown_levels<T, S, 0>(B, cs, vz, uL, rb, idx);
  constexpr int si = S - 1;
  for (int e = tid; e < si * si; e += NT) {
    const int a = 1 + e % si, b = 1 + e / si;
    us[(long long)(Y0 + b) * (nc + 1) + X0 + a] = uL[b * S1 + a];
  }
}

// ---------------------------------------------------------------------------
// Forward: new load propagated bottom-up through the block's factors.
template <typename T, int S, int K>
__device__ __forceinline__ void forward_level(const DevBlocks& B, const T* cst, double* vz, double* cur,
                                              const double* prev, int* idx) {
  using L = Lv<S, K>;
  constexpr int g = L::gam, U = L::U;
  const int tid = threadIdx.x;
  // the next (upper) level's extend-add maps are loaded into registers now
  // and written to idx once this level no longer needs it
  constexpr int NN = (K > 0) ? Lv<S, (K > 0 ? K - 1 : 0)>::n * 2 * (Lv<S, (K > 0 ? K - 1 : 0)>::U + 1) : 1;
  constexpr int NP = (NN + NT - 1) / NT;
  int pre[NP];
  if constexpr (K > 0) {
    const int* src = B.maps + B.lv[K - 1].map_off;
#pragma unroll
    for (int j = 0; j < NP; ++j) pre[j] = src[min(tid + NT * j, NN - 1)];
  }
  if constexpr (K < L::Lm) {
    using C = Lv<S, K + 1>;
    const int* maps = idx;  // this level's maps, staged by the level below
    for (int e = tid; e < L::n * U; e += NT) {
      const int t = e / U, i = e % U;
      const int* mA = maps + t * 2 * (U + 1);
      const int* mB = mA + (U + 1);
      double v = 0.0;
      if (mA[i] >= 0) v += prev[(2 * t) * C::U + C::gam + mA[i]];
      if (mB[i] >= 0) v += prev[(2 * t + 1) * C::U + C::gam + mB[i]];
      cur[e] = v;
    }
    __syncthreads();
  }
  const T* base = cst + B.lv[K].cst_off;
  // z = L^-1 g_gamma, one node per group of g lanes
  {
    constexpr int GPW = Groups<g>::per_wave;
    constexpr int NW = (L::n + GPW - 1) / GPW;
    static_assert(NW * 64 <= NT, "level solve does not fit the workgroup");
    const int wv = tid >> 6, lane = tid & 63;
    const int grp = lane / g, i = lane % g;
    const int t = wv * GPW + grp;
    const bool act = grp < GPW && t < L::n;
    if (wv < NW) {
      const T* blk = base + (act ? t : 0) * L::per;
      const int gb = grp * g;
      double v = act ? cur[t * U + i] : 0.0;
#pragma unroll
      for (int l = 0; l < g; ++l) {
        const double xl = __shfl(v, gb + l) / double(blk[l * g + l]);
        if (i == l) v = xl;
        else if (i > l) v -= double(blk[i * g + l]) * xl;
      }
      if (act) {
        cur[t * U + i] = v;
        vz[B.lv[K].vec_off + t * g + i] = v;
      }
    }
  }
  if constexpr (K > 0) {  // idx is free: this level's extend-add is done
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (tid + NT * j < NN) idx[tid + NT * j] = pre[j];
  }
  __syncthreads();
  for (int e = tid; e < L::n * L::bnd; e += NT) {  // g_omega = g_Gamma - P z
    const int t = e / L::bnd, j = e % L::bnd;
    const T* blk = base + t * L::per;
    const double* x = cur + t * U;
    double v = x[g + j];
#pragma unroll
    for (int i = 0; i < g; ++i) v -= double(blk[(g + j) * g + i]) * x[i];
    cur[t * U + g + j] = v;  // own slot; other threads read only x[0..g)
  }
  __syncthreads();
}

template <typename T, int S, int K>
__device__ __forceinline__ void forward_levels(const DevBlocks& B, const T* cst, double* vz, double* cur,
                                               double* prev, int* idx) {
  forward_level<T, S, K>(B, cst, vz, cur, prev, idx);
  if constexpr (K > 0) forward_levels<T, S, K - 1>(B, cst, vz, prev, cur, idx);
}

template <typename T, int S>
__global__ void __launch_bounds__(NT) k_block_forward(DevBlocks B, int n_samples, int nc,
                                                      const double* __restrict__ res, long long rstride) {
  using M = Lv<S, Lv<S, 0>::Lm>;
  constexpr int Lm = M::Lm;
  constexpr int S1 = S + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  T* cs = reinterpret_cast<T*>(smem);
  double* g0 = reinterpret_cast<double*>(smem + ((size_t(B.cst_size) * sizeof(T) + 15) / 16) * 16);
  double* g1 = g0 + B.max_bnd_nodes;
  __shared__ int idx[kIdxMax<S>];
  const int q = blockIdx.x / n_samples;
  const int s = blockIdx.x % n_samples;
  const int X0 = B.origin[2 * q], Y0 = B.origin[2 * q + 1];
  const int tid = threadIdx.x;
  stage_factors<T>(cs, cst_block<T>(B, q, s), B.cst_size);
  double* vz = B.vec + (long long)s * B.vec_stride + (long long)q * B.vec_size;
  const double* rs = res + (long long)s * rstride;
  // micro-blocks: node (i, j) of the residual belongs to the micro-block that
  // contains cell (i, j), so each global entry is counted exactly once
  {
    stage_ints(idx, B.lids + B.lv[Lm].lid_off, M::n * M::U);
    __syncthreads();
    const int* lids = idx;
    for (int e = tid; e < M::n * M::U; e += NT) {
      const int t = e / M::U;
      const int lid = lids[e];
      const int a = lid % S1, b = lid / S1;
      const int a0 = B.micro_xy[2 * t], b0 = B.micro_xy[2 * t + 1];
      const bool own = a >= a0 && a < a0 + 2 && b >= b0 && b < b0 + 2;
      g0[e] = own ? rs[(long long)(Y0 + b) * (nc + 1) + X0 + a] : 0.0;
    }
  }
  __syncthreads();
  forward_levels<T, S, Lm>(B, cs, vz, g0, g1, idx);
  // block root [z ; g_omega] -> the global vector store of the block level
  using R = Lv<S, 0>;
  const double* root = (Lm % 2 == 0) ? g0 : g1;
  const DevNode nd = B.top.nodes[q];
  double* out = B.top.vec + (long long)s * B.top.vec_stride + nd.ids_off;
  for (int e = tid; e < R::U; e += NT) out[e] = root[e];
}

// ---------------------------------------------------------------------------
// two frame buffers and the gather table's zero slot
size_t block_build_lds(const DevBlocks& B, bool dbl) { return (size_t(2) * B.max_buf + 2) * (dbl ? 8 : 4); }

size_t block_ext_entries(int s) {
  switch (s) {
    case 2: return ext_total<2>();
    case 4: return ext_total<4>();
    case 8: return ext_total<8>();
    case 16: return ext_total<16>();
    default: return 0;
  }
}

template <int S> static void launch_ext_t(const DevBlocks& B, uint2* ext, hipStream_t st) {
  constexpr int n = ext_total<S>();
  if (n > 0) hipLaunchKernelGGL((k_block_ext<S>), dim3((n + 255) / 256), dim3(256), 0, st, B, ext);
}

hipError_t launch_block_ext(const DevBlocks& B, uint2* ext, hipStream_t st) {
  // every offset (and the zero slot) must fit the table's 16-bit fields
  if (2 * B.max_buf >= 65536) return hipErrorInvalidValue;
  switch (B.s) {
    case 2: launch_ext_t<2>(B, ext, st); break;
    case 4: launch_ext_t<4>(B, ext, st); break;
    case 8: launch_ext_t<8>(B, ext, st); break;
    case 16: launch_ext_t<16>(B, ext, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static size_t stage_bytes(const DevBlocks& B, bool dbl) { return (size_t(B.cst_size) * (dbl ? 8 : 4) + 15) / 16 * 16; }

size_t block_topdown_lds(const DevBlocks& B, bool dbl) {
  return stage_bytes(B, dbl) + sizeof(double) * size_t((B.s + 1) * (B.s + 1) + B.max_gam_nodes);
}

size_t block_forward_lds(const DevBlocks& B, bool dbl) {
  return stage_bytes(B, dbl) + sizeof(double) * size_t(2 * B.max_bnd_nodes);
}

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
  const size_t lds = block_topdown_lds(B, sizeof(T) == 8);
  hipLaunchKernelGGL((k_block_topdown<T, S>), dim3(n_list * n_samples), dim3(NT), lds, st, B, list, n_samples, nc, u,
                     ustride, from_vec ? 1 : 0);
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
