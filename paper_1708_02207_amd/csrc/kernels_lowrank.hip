// Block low-rank (H-matrix style) storage of the maps P = S_Gamma,gamma L^-T
// of the wide levels (Section 4: the maps Phi and Psi of every node admit
// H-matrix approximations, dense blocks near the diagonal and low-rank blocks
// elsewhere; Fig. Hg and Fig. Hrhs).
//
// P of a node (|Gamma| x |gamma|) is cut into 64 x 64 blocks, rows taken
// in the order of the node's boundary (a permutation of Gamma sorted along
// the perimeter), columns in the order of the cut.  A block whose boundary
// segment lies at least its own extent away from its interface segment is
// stored as U V (U: 64 x r, V: r x 64, r <= kr, slots of 2 x 64 x kr), the
// others densely.  The low-rank factors come from a randomized range finder
// with one power iteration: Y = B (B^T (B Omega)), Q = orth(Y) by twice
// modified Gram-Schmidt, V = Q^T B; the rank is the number of columns of Q
// whose Gram-Schmidt norm, taken to the power 1/3, is above tol times the
// first one's (the power iteration cubes the singular values), at most kr
// (a block that needs more is truncated to kr; the refinement absorbs the
// difference like any other approximation of the maps).  Omega is a fixed
// pseudo-random +-1 matrix (a hash of the row and column).
//
// The compressed maps replace the dense P in the products of Root to Leaves
// (r = z - P^T u_Gamma) and of the forward pass (g_omega = g~ - P z) of the
// refinement sweeps; the float64 residual of every sweep measures the exact
// operator, so the refined field still converges to the discrete solution.
#include <cstdint>

#include "device.hpp"
#include "kernels.hpp"

namespace hdd {

namespace {

constexpr int LB = kLowRankBlock;  // block edge
constexpr int KR = kLowRankMax;    // rank slots

__device__ __forceinline__ double omega_entry(int c, int k) {
  unsigned h = unsigned(c) * 0x9E3779B1u ^ unsigned(k) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return (h & 1u) ? 1.0 : -1.0;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <typename T> __device__ __forceinline__ T* lr_ptr(const DevLevel& L, int s, long long off) {
  return reinterpret_cast<T*>(L.lr_store) + (long long)s * L.lr_stride + off;
}

// Row r of block row bi of node nd: the Gamma position (index into Gamma).
__device__ __forceinline__ int lr_row(const DevLevel& L, const DevNode& nd, int bi, int r) {
  return L.lr_perm[nd.ids_off + L.gam + bi * LB + r];
}

}  // namespace

// One wave per (block, sample).  Dynamic LDS: B (64 x 65), Y or Q (64 x KR),
// Z (64 x KR), all float64.
template <typename T>
__global__ void __launch_bounds__(64) k_lr_compress(DevLevel L, int n_samples, double tol) {
  extern __shared__ double lds[];
  double* B = lds;                  // [64][65]
  double* Y = B + LB * (LB + 1);    // [64][KR]
  double* Z = Y + LB * KR;          // [64][KR]
  const int b = blockIdx.x / n_samples, s = blockIdx.x % n_samples;
  const int4 blk = L.lr_blk[b];     // type, offset, node, bi << 16 | bj
  const DevNode nd = L.nodes[blk.z];
  const int g = L.gam, G = nd.bnd;
  const int bi = blk.w >> 16, bj = blk.w & 0xffff;
  const int R = min(LB, G - bi * LB), C = min(LB, g - bj * LB);
  int ld;
  const T* F = retained_ptr<T>(L, blk.z, s, ld);
  const int lane = threadIdx.x;
  T* out = lr_ptr<T>(L, s, blk.y);
  // the block, rows in perimeter order; coalesced along the columns
  for (int r = 0; r < LB; ++r) {
    double v = 0.0;
    if (r < R && lane < C) v = double(F[(long long)(g + lr_row(L, nd, bi, r)) * ld + bj * LB + lane]);
    B[r * (LB + 1) + lane] = v;
  }
  __syncthreads();
  if (blk.x == 0) {  // dense block
    for (int r = 0; r < LB; ++r) out[r * LB + lane] = T(B[r * (LB + 1) + lane]);
    return;
  }
  // Z = B Omega (lane r: row r)
  double t[KR];
#pragma unroll
  for (int k = 0; k < KR; ++k) t[k] = 0.0;
  for (int c = 0; c < LB; ++c) {
    const double brc = B[lane * (LB + 1) + c];
#pragma unroll
    for (int k = 0; k < KR; ++k) t[k] += brc * omega_entry(c, k);
  }
#pragma unroll
  for (int k = 0; k < KR; ++k) Z[lane * KR + k] = t[k];
  __syncthreads();
  // Y = B^T Z (lane c: row c of Y)
#pragma unroll
  for (int k = 0; k < KR; ++k) t[k] = 0.0;
  for (int r = 0; r < LB; ++r) {
    const double brc = B[r * (LB + 1) + lane];
#pragma unroll
    for (int k = 0; k < KR; ++k) t[k] += brc * Z[r * KR + k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KR; ++k) Y[lane * KR + k] = t[k];
  __syncthreads();
  // Z = B Y (lane r): the sample of the range of B
#pragma unroll
  for (int k = 0; k < KR; ++k) t[k] = 0.0;
  for (int c = 0; c < LB; ++c) {
    const double brc = B[lane * (LB + 1) + c];
#pragma unroll
    for (int k = 0; k < KR; ++k) t[k] += brc * Y[c * KR + k];
  }
  // twice modified Gram-Schmidt on the columns of t (distributed over lanes)
  double nrm[KR];
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
      for (int j = 0; j < k; ++j) {
        const double d = wave_sum(t[j] * t[k]);
        t[k] -= d * t[j];
      }
    }
    const double n2 = wave_sum(t[k] * t[k]);
    nrm[k] = sqrt(n2);
    t[k] = n2 > 0.0 ? t[k] / nrm[k] : 0.0;
  }
  int rank = 0;
  const double lead = nrm[0];
#pragma unroll
  for (int k = 0; k < KR; ++k)
    if (lead > 0.0 && cbrt(nrm[k] / lead) > tol) rank = k + 1;
  // U = Q[:, :rank] (lane r), V = Q^T B (lane c)
  T* U = out;
  T* V = out + LB * KR;
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    U[lane * KR + k] = T(k < rank ? t[k] : 0.0);
    Z[lane * KR + k] = k < rank ? t[k] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KR; ++k) t[k] = 0.0;
  for (int r = 0; r < LB; ++r) {
    const double brc = B[r * (LB + 1) + lane];
#pragma unroll
    for (int k = 0; k < KR; ++k) t[k] += Z[r * KR + k] * brc;
  }
#pragma unroll
  for (int k = 0; k < KR; ++k) V[k * LB + lane] = T(t[k]);
  if (lane == 0) L.lr_rank[(long long)s * L.lr_nblk + b] = rank;
}

// r_i = z_i - (P^T u_Gamma)_i for the 64 columns i of block column bj, with
// the compressed P; written to the gamma slots of u (as k_topdown_gemv).
// grid = (entry x sample, block columns), 64 threads.
template <typename T>
__global__ void __launch_bounds__(64) k_lr_topdown_gemv(DevLevel L, const int* __restrict__ list, int n_samples,
                                                       double* __restrict__ u, long long ustride, int z_from_vec) {
  __shared__ double xs[LB];
  __shared__ double ts[KR];
  const int e = blockIdx.x;
  const int node = list[e / n_samples];
  const int s = e % n_samples;
  const DevNode nd = L.nodes[node];
  const int g = L.gam, G = nd.bnd, U = nd.U;
  const int bj = blockIdx.y;
  if (bj * LB >= g) return;  // uniform
  const int nbr = (G + LB - 1) / LB, nbc = (g + LB - 1) / LB;
  const int* ids = L.ids + nd.ids_off;
  double* us = u + (long long)s * ustride;
  const int lane = threadIdx.x;
  double acc = 0.0;
  for (int bi = 0; bi < nbr; ++bi) {
    const int b = L.lr_node[node] + bi * nbc + bj;
    const int4 blk = L.lr_blk[b];
    const int row = bi * LB + lane;
    __syncthreads();
    xs[lane] = row < G ? us[ids[g + lr_row(L, nd, bi, lane)]] : 0.0;
    __syncthreads();
    const T* D = lr_ptr<T>(L, s, blk.y);
    const int rank = blk.x == 0 ? -1 : L.lr_rank[(long long)s * L.lr_nblk + b];  // -1: dense block
    if (rank < 0) {
      for (int r = 0; r < LB; ++r) acc += double(D[r * LB + lane]) * xs[r];
    } else {
      if (lane < rank) {
        double tk = 0.0;
        for (int r = 0; r < LB; ++r) tk += double(D[r * KR + lane]) * xs[r];
        ts[lane] = tk;
      }
      __syncthreads();
      const T* V = D + LB * KR;
      for (int k = 0; k < rank; ++k) acc += double(V[k * LB + lane]) * ts[k];
    }
  }
  const int i = bj * LB + lane;
  if (i < g) {
    int ld;
    const T* F = retained_ptr<T>(L, node, s, ld);
    const double z = z_from_vec ? L.vec[(long long)s * L.vec_stride + nd.ids_off + i] : double(F[(long long)U * ld + i]);
    us[ids[i]] = z - acc;
  }
}

// g_omega -= P z for the 64 rows of block row bi, with the compressed P
// (vec[node] = [z ; g_omega] as left by k_forward with the product deferred).
// grid = (node x sample, block rows), 64 threads.
template <typename T>
__global__ void __launch_bounds__(64) k_lr_forward_gemv(DevLevel L, int n_samples) {
  __shared__ double zs[LB];
  __shared__ double ts[KR];
  __shared__ double Ds[LB][LB + 1];
  const int e = blockIdx.x;
  const int node = e / n_samples;
  const int s = e % n_samples;
  const DevNode nd = L.nodes[node];
  const int g = L.gam, G = nd.bnd;
  const int bi = blockIdx.y;
  if (bi * LB >= G) return;  // uniform
  const int nbc = (g + LB - 1) / LB;
  double* out = L.vec + (long long)s * L.vec_stride + nd.ids_off;
  const int lane = threadIdx.x;
  double acc = 0.0;
  for (int bj = 0; bj < nbc; ++bj) {
    const int b = L.lr_node[node] + bi * nbc + bj;
    const int4 blk = L.lr_blk[b];
    const int col = bj * LB + lane;
    __syncthreads();
    zs[lane] = col < g ? out[col] : 0.0;
    const T* D = lr_ptr<T>(L, s, blk.y);
    const int rank = blk.x == 0 ? -1 : L.lr_rank[(long long)s * L.lr_nblk + b];  // -1: dense block
    if (rank < 0) {
      for (int r = 0; r < LB; ++r) Ds[r][lane] = double(D[r * LB + lane]);
      __syncthreads();
      for (int c = 0; c < LB; ++c) acc += Ds[lane][c] * zs[c];
    } else {
      __syncthreads();
      const T* V = D + LB * KR;
      if (lane < rank) {
        double tk = 0.0;
        for (int c = 0; c < LB; ++c) tk += double(V[lane * LB + c]) * zs[c];
        ts[lane] = tk;
      }
      __syncthreads();
      for (int k = 0; k < rank; ++k) acc += double(D[lane * KR + k]) * ts[k];
    }
  }
  const int row = bi * LB + lane;
  if (row < G) out[g + lr_row(L, nd, bi, lane)] -= acc;
}

hipError_t launch_lr_compress(const DevLevel& L, int n_samples, double tol, hipStream_t st) {
  if (!L.lr_store || L.lr_nblk <= 0) return hipSuccess;
  const size_t lds = sizeof(double) * (size_t(LB) * (LB + 1) + 2 * size_t(LB) * KR);
  const dim3 grid(unsigned(L.lr_nblk) * unsigned(n_samples));
  if (L.is_double)
    hipLaunchKernelGGL(k_lr_compress<double>, grid, dim3(64), lds, st, L, n_samples, tol);
  else
    hipLaunchKernelGGL(k_lr_compress<float>, grid, dim3(64), lds, st, L, n_samples, tol);
  return hipGetLastError();
}

hipError_t launch_lr_topdown_gemv(const DevLevel& L, const int* list, int n_list, int n_samples, double* u,
                                  long long ustride, bool z_from_vec, hipStream_t st) {
  const dim3 grid(unsigned(n_list) * unsigned(n_samples), unsigned((L.gam + LB - 1) / LB));
  if (L.is_double)
    hipLaunchKernelGGL(k_lr_topdown_gemv<double>, grid, dim3(64), 0, st, L, list, n_samples, u, ustride,
                       z_from_vec ? 1 : 0);
  else
    hipLaunchKernelGGL(k_lr_topdown_gemv<float>, grid, dim3(64), 0, st, L, list, n_samples, u, ustride,
                       z_from_vec ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_lr_forward_gemv(const DevLevel& L, int n_samples, hipStream_t st) {
  const dim3 grid(unsigned(L.n_nodes) * unsigned(n_samples), unsigned((L.max_U - L.gam + LB - 1) / LB));
  if (L.is_double)
    hipLaunchKernelGGL(k_lr_forward_gemv<double>, grid, dim3(64), 0, st, L, n_samples);
  else
    hipLaunchKernelGGL(k_lr_forward_gemv<float>, grid, dim3(64), 0, st, L, n_samples);
  return hipGetLastError();
}

}  // namespace hdd
