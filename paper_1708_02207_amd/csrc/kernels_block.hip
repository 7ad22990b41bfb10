// In-LDS nested dissection of s x s-cell blocks (the leaf interior).
//
// One workgroup handles one (block, sample).  All blocks share one local
// sub-tree (outer Dirichlet nodes are kept inside a block), so every level
// has n nodes of identical shape and the whole level is processed in
// parallel with workgroup-wide barriers.
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

#include "device.hpp"
#include "kernels.hpp"

namespace hdd {

__constant__ int c_mb_local[3][3] = {  // micro-block local node (a, b) -> frame index
    {1, 2, 3},
    {8, 0, 4},
    {7, 6, 5}};

template <typename T> __device__ __forceinline__ T* cst_block(const DevBlocks& B, int q, int s) {
  return reinterpret_cast<T*>(B.cst) + (long long)s * B.cst_stride + (long long)q * B.cst_size;
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_block_build(DevBlocks B, int n_samples, int nc,
                                                     const double* __restrict__ kappa, const double* __restrict__ f,
                                                     int* __restrict__ bad, int* __restrict__ info) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* buf0 = reinterpret_cast<T*>(smem);
  T* buf1 = buf0 + B.max_buf;
  __shared__ int bad_pivot;
  const int q = blockIdx.x / n_samples;
  const int s = blockIdx.x % n_samples;
  const int X0 = B.origin[2 * q], Y0 = B.origin[2 * q + 1];
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  const int Lm = B.nlev - 1;
  if (tid == 0) bad_pivot = 0;
  // ---- micro-blocks: assemble the 9 x 9 local systems (lower triangle + load row)
  {
    const DevSubLevel M = B.lv[Lm];
    for (int e = tid; e < M.n * M.fsz; e += NT) buf0[e] = T(0);
    __syncthreads();
    const double h = 1.0 / nc;
    const double area = 0.5 * h * h;
    const double* ks = kappa + (long long)s * nc * nc * 2;
    for (int t = tid; t < M.n; t += NT) {
      T* F = buf0 + t * M.fsz;
      const int a0 = X0 + B.micro_xy[2 * t], b0 = Y0 + B.micro_xy[2 * t + 1];
      bool ok = true;
      for (int cb = 0; cb < 2; ++cb)
        for (int ca = 0; ca < 2; ++ca)
          for (int tri = 0; tri < 2; ++tri) {
            // T-: (0,0),(1,0),(1,1); T+: (0,0),(1,1),(0,1) relative to the cell corner
            const int vx[3] = {ca, ca + 1, tri == 0 ? ca + 1 : ca};
            const int vy[3] = {cb, tri == 0 ? cb : cb + 1, cb + 1};
            const double kap = ks[((long long)(b0 + cb) * nc + (a0 + ca)) * 2 + tri];
            ok = ok && (kap > 0.0) && (kap < 1.0e300);
            const double det = double((vx[1] - vx[0]) * (vy[2] - vy[0]) - (vx[2] - vx[0]) * (vy[1] - vy[0]));
            const double gx[3] = {double(vy[1] - vy[2]), double(vy[2] - vy[0]), double(vy[0] - vy[1])};
            const double gy[3] = {double(vx[2] - vx[1]), double(vx[0] - vx[2]), double(vx[1] - vx[0])};
            const double scale = kap / (2.0 * fabs(det));
            for (int a = 0; a < 3; ++a) {
              const int ia = c_mb_local[vy[a]][vx[a]];
              for (int b = 0; b < 3; ++b) {
                const int ib = c_mb_local[vy[b]][vx[b]];
                if (ib <= ia) F[ia * 10 + ib] += T(scale * (gx[a] * gx[b] + gy[a] * gy[b]));
              }
              const double fv = f[(long long)(b0 + vy[a]) * (nc + 1) + (a0 + vx[a])];
              F[9 * 10 + ia] += T(area * fv / 3.0);
            }
          }
      if (!ok && bad) atomicCAS(bad + s, 0, 1);
    }
    __syncthreads();
  }
  T* cur = buf0;
  T* prev = buf1;
  for (int k = Lm; k >= 0; --k) {
    const DevSubLevel L = B.lv[k];
    const int ld = L.U + 1;
    if (k < Lm) {
      // extend-add of the sons' [Gamma ; rhs] blocks (in `prev`) into the frames (in `cur`)
      const DevSubLevel C = B.lv[k + 1];
      const int lds = C.U + 1;
      for (int e = tid; e < L.n * L.fsz; e += NT) {
        const int t = e / L.fsz, rc = e % L.fsz;
        const int r = rc / ld, c = rc % ld;
        if (c > r) continue;
        const int* mA = B.maps + L.map_off + t * 2 * ld;
        const int* mB = mA + ld;
        T v = T(0);
        const T* SA = prev + (2 * t) * C.fsz + C.gam * lds + C.gam;
        const T* SB = prev + (2 * t + 1) * C.fsz + C.gam * lds + C.gam;
        const int ar = mA[r], ac = mA[c];
        if (ar >= 0 && ac >= 0) v += ar >= ac ? SA[ar * lds + ac] : SA[ac * lds + ar];
        const int br = mB[r], bc = mB[c];
        if (br >= 0 && bc >= 0) v += br >= bc ? SB[br * lds + bc] : SB[bc * lds + br];
        cur[e] = v;
      }
      __syncthreads();
    }
    // partial Cholesky of the first gam columns of every frame of the level
    for (int j = 0; j < L.gam; ++j) {
      for (int t = tid; t < L.n; t += NT) {
        T d = cur[t * L.fsz + j * ld + j];
        if (!(d > T(0)) || !(d < T(1e300))) {
          bad_pivot = 1;
          d = T(1);
        }
        cur[t * L.fsz + j * ld + j] = sqrt(d);
      }
      __syncthreads();
      const int m = L.U - j;  // rows j+1 .. U
      for (int e = tid; e < L.n * m; e += NT) {
        const int t = e / m, i = j + 1 + e % m;
        cur[t * L.fsz + i * ld + j] /= cur[t * L.fsz + j * ld + j];
      }
      __syncthreads();
      for (int e = tid; e < L.n * m * m; e += NT) {
        const int t = e / (m * m), rr = e % (m * m);
        const int i = j + 1 + rr / m, l = j + 1 + rr % m;
        if (l <= i) {
          T* F = cur + t * L.fsz;
          F[i * ld + l] -= F[i * ld + j] * F[l * ld + j];
        }
      }
      __syncthreads();
    }
    // retained columns [L ; P ; z] of every node -> compact store
    T* out = cst_block<T>(B, q, s) + L.cst_off;
    const int per = ld * L.gam;
    for (int e = tid; e < L.n * per; e += NT) {
      const int t = e / per, rc = e % per;
      const int r = rc / L.gam, c = rc % L.gam;
      out[e] = (c <= r) ? cur[t * L.fsz + r * ld + c] : T(0);
    }
    __syncthreads();
    T* tmp = cur;
    cur = prev;
    prev = tmp;
  }
  // block root frame (now in `prev`) -> global frame store (lower triangle)
  {
    const DevSubLevel R = B.lv[0];
    const int ld = R.U + 1;
    const DevNode nd = B.top.nodes[q];
    T* G = reinterpret_cast<T*>(B.top.frames) + (long long)s * B.top.stride + nd.frame_off;
    for (int e = tid; e < R.fsz; e += NT) {
      const int r = e / ld, c = e % ld;
      if (c <= r) G[(long long)r * nd.ld + c] = prev[e];
    }
  }
  if (tid == 0 && bad_pivot && info) atomicCAS(info + s, 0, B.top.node_base + q + 1);
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_block_topdown(DevBlocks B, const int* __restrict__ list, int n_samples,
                                                       int nc, double* __restrict__ u, long long ustride,
                                                       int from_vec) {
  extern __shared__ double dsm[];
  const int S1 = B.s + 1;
  double* uL = dsm;               // (s+1)^2 local nodal values
  double* rb = dsm + S1 * S1;     // n * gam work values of one level
  const int q = list[blockIdx.x / n_samples];
  const int s = blockIdx.x % n_samples;
  const int X0 = B.origin[2 * q], Y0 = B.origin[2 * q + 1];
  const int tid = threadIdx.x, NT = blockDim.x;
  double* us = u + (long long)s * ustride;
  for (int e = tid; e < S1 * S1; e += NT) uL[e] = us[(long long)(Y0 + e / S1) * (nc + 1) + X0 + e % S1];
  __syncthreads();
  const T* cst = cst_block<T>(B, q, s);
  const double* vz = from_vec ? B.vec + (long long)s * B.vec_stride + (long long)q * B.vec_size : nullptr;
  for (int k = 0; k < B.nlev; ++k) {
    const DevSubLevel L = B.lv[k];
    const int g = L.gam, per = (L.U + 1) * g;
    for (int e = tid; e < L.n * g; e += NT) {
      const int t = e / g, i = e % g;
      const T* blk = cst + L.cst_off + t * per;
      const int* lid = B.lids + L.lid_off + t * L.U;
      double acc = from_vec ? vz[L.vec_off + e] : double(blk[L.U * g + i]);
      for (int j = 0; j < L.bnd; ++j) acc -= double(blk[(g + j) * g + i]) * uL[lid[g + j]];
      rb[e] = acc;
    }
    __syncthreads();
    for (int t = tid; t < L.n; t += NT) {
      const T* blk = cst + L.cst_off + t * per;
      const int* lid = B.lids + L.lid_off + t * L.U;
      double* x = rb + t * g;
      for (int i = g - 1; i >= 0; --i) {
        double v = x[i];
        for (int l = i + 1; l < g; ++l) v -= double(blk[l * g + i]) * x[l];
        v /= double(blk[i * g + i]);
        x[i] = v;
        uL[lid[i]] = v;
      }
    }
    __syncthreads();
  }
  const int si = B.s - 1;
  for (int e = tid; e < si * si; e += NT) {
    const int a = 1 + e % si, b = 1 + e / si;
    us[(long long)(Y0 + b) * (nc + 1) + X0 + a] = uL[b * S1 + a];
  }
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_block_forward(DevBlocks B, int n_samples, int nc,
                                                       const double* __restrict__ res, long long rstride) {
  extern __shared__ double dsm[];
  double* g0 = dsm;                       // per level: n * U values
  double* g1 = dsm + B.max_bnd_nodes;
  const int S1 = B.s + 1;
  const int q = blockIdx.x / n_samples;
  const int s = blockIdx.x % n_samples;
  const int X0 = B.origin[2 * q], Y0 = B.origin[2 * q + 1];
  const int tid = threadIdx.x, NT = blockDim.x;
  const int Lm = B.nlev - 1;
  const T* cst = cst_block<T>(B, q, s);
  double* vz = B.vec + (long long)s * B.vec_stride + (long long)q * B.vec_size;
  const double* rs = res + (long long)s * rstride;
  double* cur = g0;
  double* prev = g1;
  for (int k = Lm; k >= 0; --k) {
    const DevSubLevel L = B.lv[k];
    const int g = L.gam, U = L.U, per = (U + 1) * g;
    if (k == Lm) {
      // micro-blocks: the residual node (i, j) belongs to the micro-block
      // that contains cell (i, j), so each global entry is counted once
      for (int e = tid; e < L.n * U; e += NT) {
        const int t = e / U, i = e % U;
        const int lid = B.lids[L.lid_off + e];
        const int a = lid % S1, b = lid / S1;
        const int a0 = B.micro_xy[2 * t], b0 = B.micro_xy[2 * t + 1];
        const bool own = a >= a0 && a < a0 + 2 && b >= b0 && b < b0 + 2;
        cur[e] = own ? rs[(long long)(Y0 + b) * (nc + 1) + X0 + a] : 0.0;
        (void)i;
      }
    } else {
      const DevSubLevel C = B.lv[k + 1];
      for (int e = tid; e < L.n * U; e += NT) {
        const int t = e / U, i = e % U;
        const int* mA = B.maps + L.map_off + t * 2 * (U + 1);
        const int* mB = mA + (U + 1);
        double v = 0.0;
        if (mA[i] >= 0) v += prev[(2 * t) * C.U + C.gam + mA[i]];
        if (mB[i] >= 0) v += prev[(2 * t + 1) * C.U + C.gam + mB[i]];
        cur[e] = v;
      }
    }
    __syncthreads();
    // z = L^-1 g_gamma, one thread per node
    for (int t = tid; t < L.n; t += NT) {
      const T* blk = cst + L.cst_off + t * per;
      double* x = cur + t * U;
      for (int i = 0; i < g; ++i) {
        double v = x[i];
        for (int l = 0; l < i; ++l) v -= double(blk[i * g + l]) * x[l];
        x[i] = v / double(blk[i * g + i]);
        vz[L.vec_off + t * g + i] = x[i];
      }
    }
    __syncthreads();
    // g_omega = g_Gamma - P z
    for (int e = tid; e < L.n * L.bnd; e += NT) {
      const int t = e / L.bnd, j = e % L.bnd;
      const T* blk = cst + L.cst_off + t * per;
      const double* x = cur + t * U;
      double v = x[g + j];
      for (int i = 0; i < g; ++i) v -= double(blk[(g + j) * g + i]) * x[i];
      cur[t * U + g + j] = v;  // own slot only: rows g+j are not read by other threads
    }
    __syncthreads();
    double* tmp = cur;
    cur = prev;
    prev = tmp;
  }
  // block root [z ; g_omega] -> the global vector store of the block level
  const DevSubLevel R = B.lv[0];
  const DevNode nd = B.top.nodes[q];
  double* out = B.top.vec + (long long)s * B.top.vec_stride + nd.ids_off;
  for (int e = tid; e < R.U; e += NT) out[e] = prev[e];
}

// ---------------------------------------------------------------------------
static int ceil_div_b(long long a, long long b) { return int((a + b - 1) / b); }

size_t block_build_lds(const DevBlocks& B, bool dbl) { return size_t(2) * B.max_buf * (dbl ? 8 : 4); }

hipError_t launch_block_build(const DevBlocks& B, int n_samples, int nc, const double* kappa, const double* f,
                              int* bad, int* info, hipStream_t st) {
  dim3 grid(B.nb * n_samples), block(256);
  const bool dbl = B.top.is_double != 0;
  const size_t lds = block_build_lds(B, dbl);
  if (dbl)
    hipLaunchKernelGGL(k_block_build<double>, grid, block, lds, st, B, n_samples, nc, kappa, f, bad, info);
  else
    hipLaunchKernelGGL(k_block_build<float>, grid, block, lds, st, B, n_samples, nc, kappa, f, bad, info);
  return hipGetLastError();
}

hipError_t launch_block_topdown(const DevBlocks& B, const int* list, int n_list, int n_samples, int nc, double* u,
                                long long ustride, bool from_vec, hipStream_t st) {
  if (n_list <= 0) return hipSuccess;
  dim3 grid(n_list * n_samples), block(256);
  const size_t lds = sizeof(double) * size_t((B.s + 1) * (B.s + 1) + B.max_gam_nodes);
  if (B.top.is_double)
    hipLaunchKernelGGL(k_block_topdown<double>, grid, block, lds, st, B, list, n_samples, nc, u, ustride,
                       from_vec ? 1 : 0);
  else
    hipLaunchKernelGGL(k_block_topdown<float>, grid, block, lds, st, B, list, n_samples, nc, u, ustride,
                       from_vec ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_block_forward(const DevBlocks& B, int n_samples, int nc, const double* r, long long rstride,
                                hipStream_t st) {
  dim3 grid(B.nb * n_samples), block(256);
  const size_t lds = sizeof(double) * size_t(2 * B.max_bnd_nodes);
  if (B.top.is_double)
    hipLaunchKernelGGL(k_block_forward<double>, grid, block, lds, st, B, n_samples, nc, r, rstride);
  else
    hipLaunchKernelGGL(k_block_forward<float>, grid, block, lds, st, B, n_samples, nc, r, rstride);
  (void)ceil_div_b;
  return hipGetLastError();
}

}  // namespace hdd
