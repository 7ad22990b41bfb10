// HDD "Root to Leaves" kernels (Section 3.4) and the measurement operators.
//
// Top-down per node (eq. SchurC1, second line, with the retained factors):
//   u_gamma = L^-T (z - P^T u_Gamma),
// where u_Gamma is gathered from the values its ancestors already wrote into
// the nodal field (the data d_omega built from the father, Root-to-Leaves
// step 3).  The forward pass propagates a new right-hand side bottom-up with
// the same factors (z = L^-1 g~_gamma, g_omega = g~_Gamma - P z), which is
// what the iterative refinement of the FP32 path needs.
#include <algorithm>

#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace hdd {

static int ceil_div(long long a, long long b) { return int((a + b - 1) / b); }

template <typename T> __device__ __forceinline__ double ldd(const T* p) { return double(*p); }

// ---------------------------------------------------------------------------
// Shared pieces of the per-node solves.  Dynamic LDS layout (doubles):
//   v[U+1] (work vector), part[...] (GEMV partial sums).  The triangular
// solves go in diagonal blocks of nb = min(64, gam) rows.
// ---------------------------------------------------------------------------
__host__ __device__ inline int solve_nb(int g) { return g < 64 ? g : 64; }

// Lanes that share one row of a wave-level dot product: the columns of a row
// are spread over `lanes_for(n)` consecutive lanes (a power of two, at most
// 64), so a wave covers 64 / lanes_for(n) rows per step.
__host__ __device__ inline int lanes_for(int n) {
  int p = 1;
  while (p < n && p < 64) p <<= 1;
  return p;
}

// Partial sums of the transposed GEMV: one row of g per lane group.
__host__ __device__ inline int solve_part(int g, int bs) { return g < 64 ? bs : (bs / 64) * g; }

size_t solve_lds(int max_U, int gam, int bs, bool need_part = true) {
  return sizeof(double) * (size_t(max_U + 1) + (need_part ? size_t(solve_part(gam, bs)) : 0));
}

// Value of lane l (wave-uniform l) in every lane, through the scalar unit.
__device__ __forceinline__ double bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Diagonal-block solves by one wave, nb <= 64 rows, in chunks of 16 rows
// held in registers (one column, resp. row, of the chunk per lane) so that
// the only serial dependency is the broadcast of each solved entry.
//   back:    L^T x = v  (lane i holds column i: c[q] = L[j0 + q][i], j >= i)
//   forward: L z = v    (lane i holds row i:    c[q] = L[i][j0 + q], j <= i)
// The next chunk's 16 values are loaded while the current chunk is solved
// (addresses clamped into the block, unused values masked at use).
template <typename T>
__device__ __forceinline__ double diag_back(const T* D, int ld, int nb, double v) {
  const int lane = threadIdx.x & 63;
  const int lc = min(lane, nb - 1);
  const double rinv = 1.0 / double(D[(long long)lc * (ld + 1)]);  // lane j: 1 / L_jj
  auto load = [&](int j0, T (&c)[16]) {
#pragma unroll
    for (int q = 0; q < 16; ++q) c[q] = D[(long long)min(j0 + q, nb - 1) * ld + lc];
  };
  int j0 = ((nb - 1) >> 4) << 4;
  T c[16], cn[16];
  load(j0, c);
  for (; j0 >= 0; j0 -= 16) {
    if (j0 >= 16) load(j0 - 16, cn);
#pragma unroll
    for (int q = 15; q >= 0; --q) {
      const int j = j0 + q;
      if (j < nb) {
        const double xj = bcast(v * rinv, j);
        if (lane == j) v = xj;
        else if (lane < j) v -= double(c[q]) * xj;
      }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) c[q] = cn[q];
  }
  return v;
}

template <typename T>
__device__ __forceinline__ double diag_forward(const T* D, int ld, int nb, double v) {
  const int lane = threadIdx.x & 63;
  const int lc = min(lane, nb - 1);
  const double rinv = 1.0 / double(D[(long long)lc * (ld + 1)]);  // lane j: 1 / L_jj
  auto load = [&](int j0, T (&c)[16]) {
#pragma unroll
    for (int q = 0; q < 16; ++q) c[q] = D[(long long)lc * ld + min(j0 + q, nb - 1)];
  };
  T c[16], cn[16];
  load(0, c);
  for (int j0 = 0; j0 < nb; j0 += 16) {
    if (j0 + 16 < nb) load(j0 + 16, cn);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = j0 + q;
      if (j < nb) {
        const double zj = bcast(v * rinv, j);
        if (lane == j) v = zj;
        else if (lane > j) v -= double(c[q]) * zj;
      }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) c[q] = cn[q];
  }
  return v;
}

// y_r = sum_c F[r][c0 + c] x[c] for rows r0 <= r < r1 and 0 <= c < nc (F row
// major with stride ld), by all waves of the workgroup: the columns of a row
// are read by consecutive lanes (coalesced), reduced with shuffles, and
// fn(r, y_r) is called by the first lane of the row.  RB row steps are
// loaded before any reduction so that many loads are in flight.
template <typename T, int BS, typename Fn>
__device__ __forceinline__ void rows_dot(const T* F, int ld, int r0, int r1, int c0, int nc, const double* x, Fn&& fn) {
  constexpr int NW = BS / 64;
  constexpr int RB = 16;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int gp = lanes_for(nc);
  const int rpi = 64 / gp;
  const int sub = lane / gp, c = lane % gp;
  const int step = NW * rpi;
  for (int rb = r0 + wv * rpi; rb < r1; rb += step * RB) {  // uniform within a wave
    double acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = 0.0;
    for (int cb = 0; cb < nc; cb += gp) {
      const int cc = cb + c;
      const bool cok = cc < nc;
      T v[RB];
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int r = rb + q * step + sub;
        v[q] = (cok && r < r1) ? F[(long long)r * ld + c0 + cc] : T(0);
      }
      const double xv = cok ? x[cc] : 0.0;
#pragma unroll
      for (int q = 0; q < RB; ++q) acc[q] += double(v[q]) * xv;
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      double v = acc[q];
      for (int o = gp >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
      const int r = rb + q * step + sub;
      if (c == 0 && r < r1) fn(r, v);
    }
  }
}

// Same product with one thread per row: the row's nc values are read as
// 16-byte vectors where the row is aligned (scalar tail), x from LDS, no
// cross-lane reduction.  For workgroups of 256 or more threads, where the
// shuffle reductions of rows_dot saturate the cross-lane network.
template <typename T, int BS, typename Fn>
__device__ __forceinline__ void rows_dot_thread(const T* F, int ld, int r0, int r1, int c0, int nc, const double* x,
                                                Fn&& fn) {
  constexpr int V = 16 / sizeof(T);  // elements per 16-byte vector
  using Vec = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
  for (int r = r0 + int(threadIdx.x); r < r1; r += BS) {
    const T* row = F + (long long)r * ld + c0;
    double acc = 0.0;
    int k = 0;
    if ((reinterpret_cast<uintptr_t>(row) & 15) == 0) {
      const Vec* rv = reinterpret_cast<const Vec*>(row);
#pragma unroll 4
      for (; k + V <= nc; k += V) {
        const Vec v = rv[k / V];
        const T* ve = reinterpret_cast<const T*>(&v);
#pragma unroll
        for (int e = 0; e < V; ++e) acc += double(ve[e]) * x[k + e];
      }
    }
    for (; k < nc; ++k) acc += double(row[k]) * x[k];
    fn(r, acc);
  }
}

// General form for one wave: TR rows per tile, any number of columns (in
// chunks of 64).  tile: TR x 65 elements private to the wave.
template <typename T, int TR, typename Fn>
__device__ __forceinline__ void rows_dot_tile(const T* F, int ld, int r0, int r1, int c0, int nc, const double* x,
                                              T* tile, Fn&& fn) {
  static_assert(TR % 16 == 0 && TR <= 64, "tile rows");
  const int lane = threadIdx.x & 63;
  for (int rb = r0; rb < r1; rb += TR) {
    double acc = 0.0;
    for (int cb = 0; cb < nc; cb += 64) {
      const int cl = cb + lane;
      const bool cok = cl < nc;
      const int cc = c0 + min(cl, nc - 1);
#pragma unroll
      for (int b = 0; b < TR / 16; ++b) {
        T v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int r = min(rb + b * 16 + q, r1 - 1);
          v[q] = F[(long long)r * ld + cc];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) tile[(b * 16 + q) * 65 + lane] = cok ? v[q] : T(0);
      }
      if (lane < TR) {
        const T* row = tile + lane * 65;
        const int m = min(64, nc - cb);
#pragma unroll 16
        for (int c = 0; c < m; ++c) acc += double(row[c]) * x[cb + c];
      }
    }
    if (lane < TR && rb + lane < r1) fn(rb + lane, acc);
  }
}

// Top-down solve of the nodes in `list` (indices within the level) for all
// samples: u_gamma = L^-T (z - P^T u_Gamma).  grid.x = entry * n_samples + s.
template <typename T, int BS>
__global__ void __launch_bounds__(BS) k_topdown(DevLevel L, const int* __restrict__ list, int n_samples,
                                                double* __restrict__ u, long long ustride, int z_from_vec,
                                                int r_ready) {
  extern __shared__ double dyn[];
  constexpr int NW = BS / 64;
  const int e = blockIdx.x;
  const int node = list[e / n_samples];
  const int s = e % n_samples;
  const DevNode nd = L.nodes[node];
  const int g = L.gam, G = nd.bnd, U = nd.U;
  const int nbm = solve_nb(g);
  double* r = dyn;                 // [g]
  double* ub = dyn + g;            // [G]
  double* part = dyn + (L.max_U + 1);
  int ld;
  const T* F = retained_ptr<T>(L, node, s, ld);
  const int* ids = L.ids + nd.ids_off;
  double* us = u + (long long)s * ustride;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double* vz = z_from_vec ? L.vec + (long long)s * L.vec_stride + nd.ids_off : nullptr;
  if (r_ready) {  // r = z - P^T u_Gamma was left in the gamma slots of u by k_topdown_gemv
    for (int i = tid; i < g; i += BS) r[i] = us[ids[i]];
  } else {
    for (int i = tid; i < g; i += BS) r[i] = z_from_vec ? vz[i] : ldd(F + (long long)U * ld + i);
    for (int j = tid; j < G; j += BS) ub[j] = us[ids[g + j]];
  }
  __syncthreads();
  // r -= P^T u_Gamma, P[j][i] = F[(g + j) * ld + i]: a group of gp lanes
  // covers consecutive i, the 64 / gp groups of a wave and the waves split j
  if (G > 0 && !r_ready) {
    const int gp = lanes_for(g);
    const int rpw = 64 / gp;
    const int jg = wv * rpw + lane / gp, JG = NW * rpw;
    for (int i0 = 0; i0 < g; i0 += gp) {
      const int i = i0 + lane % gp;
      if (i < g) {
        double acc = 0.0;
        const T* col = F + (long long)g * ld + i;
#pragma unroll 16
        for (int j = jg; j < G; j += JG) acc += ldd(col + (long long)j * ld) * ub[j];
        part[jg * g + i] = acc;
      }
    }
    __syncthreads();
    for (int i = tid; i < g; i += BS) {
      double acc = 0.0;
      for (int w = 0; w < JG; ++w) acc += part[w * g + i];
      r[i] -= acc;
    }
    __syncthreads();
  }
  // back substitution L^T x = r in blocks of nbm rows from the bottom
  for (int b1 = g; b1 > 0; b1 -= nbm) {
    const int b0 = b1 > nbm ? b1 - nbm : 0;
    const int nb = b1 - b0;
    if (tid < 64) {
      const double v = diag_back<T>(F + (long long)b0 * ld + b0, ld, nb, tid < nb ? r[b0 + tid] : 0.0);
      if (tid < nb) r[b0 + tid] = v;
    }
    __syncthreads();
    if (b0 > 0) {
      for (int i = tid; i < b0; i += BS) {
        double acc = 0.0;
        const T* col = F + (long long)b0 * ld + i;
#pragma unroll 16
        for (int k = 0; k < nb; ++k) acc += ldd(col + (long long)k * ld) * r[b0 + k];
        r[i] -= acc;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < g; i += BS) us[ids[i]] = r[i];
}

// The GEMV of the top-down for wide interfaces, spread over 64-column
// chunks of gamma: r_i = z_i - sum_j P[j][i] u_Gamma[j] for the chunk's i,
// left in the gamma slots of u for k_topdown (r_ready) to solve.
// grid = (entry x sample, gamma / 64); dynamic LDS: G_max + 256 doubles.
template <typename T>
__global__ void __launch_bounds__(256) k_topdown_gemv(DevLevel L, const int* __restrict__ list, int n_samples,
                                                      double* __restrict__ u, long long ustride, int z_from_vec) {
  extern __shared__ double dyn[];
  const int e = blockIdx.x;
  const int node = list[e / n_samples];
  const int s = e % n_samples;
  const DevNode nd = L.nodes[node];
  const int g = L.gam, G = nd.bnd, U = nd.U;
  const int i0 = blockIdx.y * 64;
  if (i0 >= g) return;  // uniform
  double* ub = dyn;                  // [G]
  double* part = dyn + (L.max_U - L.gam);    // [4][64]
  int ld;
  const T* F = retained_ptr<T>(L, node, s, ld);
  const int* ids = L.ids + nd.ids_off;
  double* us = u + (long long)s * ustride;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int j = tid; j < G; j += 256) ub[j] = us[ids[g + j]];
  __syncthreads();
  const int i = i0 + lane;
  double acc = 0.0;
  if (i < g) {
    const T* col = F + (long long)g * ld + i;
#pragma unroll 16
    for (int j = wv; j < G; j += 4) acc += ldd(col + (long long)j * ld) * ub[j];
  }
  part[wv * 64 + lane] = acc;
  __syncthreads();
  if (wv == 0 && i < g) {
    const double z = z_from_vec ? L.vec[(long long)s * L.vec_stride + nd.ids_off + i] : ldd(F + (long long)U * ld + i);
    us[ids[i]] = z - (part[lane] + part[64 + lane] + part[128 + lane] + part[192 + lane]);
  }
}

// Forward (bottom-up) propagation of a right-hand side for all nodes of a
// level above the blocks: the load is the extend-add of the sons' condensed
// loads; z = L^-1 g~_gamma, g_omega = g~_Gamma - P z.
// vec[node] = [z (gamma) ; g_omega (Gamma)].
template <typename T, int BS>
__global__ void __launch_bounds__(BS) k_forward(DevLevel L, DevLevel C, int n_samples, int defer_gemv) {
  extern __shared__ double dyn[];
  const int e = blockIdx.x;
  const int node = e / n_samples;
  const int s = e % n_samples;
  const DevNode nd = L.nodes[node];
  const int g = L.gam, G = nd.bnd, U = nd.U;
  const int nbm = solve_nb(g);
  double* gt = dyn;  // [U]
  int ld;
  const T* F = retained_ptr<T>(L, node, s, ld);
  const int tid = threadIdx.x;
  {
    const int* mA = L.maps + nd.map_off;
    const int* mB = mA + (U + 1);
    const DevNode na = C.nodes[2 * node], nb = C.nodes[2 * node + 1];
    const double* va = C.vec + (long long)s * C.vec_stride + na.ids_off + (na.U - na.bnd);
    const double* vb = C.vec + (long long)s * C.vec_stride + nb.ids_off + (nb.U - nb.bnd);
    for (int t = tid; t < U; t += BS) {
      double v = 0.0;
      const int a = mA[t], b = mB[t];
      if (a >= 0) v += va[a];
      if (b >= 0) v += vb[b];
      gt[t] = v;
    }
  }
  __syncthreads();
  // forward substitution L z = gt[0:g] in blocks of nbm rows from the top
  for (int b0 = 0; b0 < g; b0 += nbm) {
    const int b1 = b0 + nbm < g ? b0 + nbm : g;
    const int nb = b1 - b0;
    if (tid < 64) {
      const double v = diag_forward<T>(F + (long long)b0 * ld + b0, ld, nb, tid < nb ? gt[b0 + tid] : 0.0);
      if (tid < nb) gt[b0 + tid] = v;
    }
    __syncthreads();
    if (b1 < g) {  // rows below the block: gt[i] -= L[i][b0:b1] z[b0:b1]
      if constexpr (BS >= 256)
        rows_dot_thread<T, BS>(F, ld, b1, g, b0, nb, gt + b0, [&](int i, double y) { gt[i] -= y; });
      else
        rows_dot<T, BS>(F, ld, b1, g, b0, nb, gt + b0, [&](int i, double y) { gt[i] -= y; });
      __syncthreads();
    }
  }
  // g_omega[j] = gt[g + j] - sum_i P[j][i] z_i (or only gt, with the product
  // left to k_forward_gemv)
  double* out = L.vec + (long long)s * L.vec_stride + nd.ids_off;
  if (defer_gemv) {
    for (int j = tid; j < G; j += BS) out[g + j] = gt[g + j];
  } else if constexpr (BS == 64) {
    T* tile = reinterpret_cast<T*>(dyn + (L.max_U + 1));  // 32 x 65
    if (G > 0) rows_dot_tile<T, 32>(F, ld, g, g + G, 0, g, gt, tile, [&](int r, double y) { out[r] = gt[r] - y; });
  } else {
    rows_dot_thread<T, BS>(F, ld, g, g + G, 0, g, gt, [&](int r, double y) { out[r] = gt[r] - y; });
  }
  for (int i = tid; i < g; i += BS) out[i] = gt[i];
}

// g_omega -= P z for wide interfaces, spread over 128-row chunks of Gamma.
// grid = (node x sample, Gamma / 128); dynamic LDS: gamma doubles.
template <typename T>
__global__ void __launch_bounds__(256) k_forward_gemv(DevLevel L, int n_samples) {
  extern __shared__ double dyn[];
  const int e = blockIdx.x;
  const int node = e / n_samples;
  const int s = e % n_samples;
  const DevNode nd = L.nodes[node];
  const int g = L.gam, G = nd.bnd;
  const int j0 = blockIdx.y * 128;
  if (j0 >= G) return;  // uniform
  int ld;
  const T* F = retained_ptr<T>(L, node, s, ld);
  double* out = L.vec + (long long)s * L.vec_stride + nd.ids_off;
  double* z = dyn;
  T* tile = reinterpret_cast<T*>(dyn + g) + (threadIdx.x >> 6) * 32 * 65;  // per wave 32 x 65
  for (int i = threadIdx.x; i < g; i += 256) z[i] = out[i];
  __syncthreads();
  // wave w takes rows j0 + 32 w .. j0 + 32 w + 31 of the chunk
  const int rw = g + j0 + (threadIdx.x >> 6) * 32;
  const int re = g + min(G, j0 + 128);
  if (rw < re)
    rows_dot_tile<T, 32>(F, ld, rw, min(rw + 32, re), 0, g, z, tile, [&](int r, double y) { out[r] -= y; });
}

// ---------------------------------------------------------------------------
// Full-field kernels
// ---------------------------------------------------------------------------
__global__ void k_fill(double* p, long long n, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_i32(int* p, long long n, int v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// Residual r = b - A u at every interior node, FP64, assembled on the fly
// from the six triangles around the node with the element matrices of
// eq. coefA and the vertex-rule load of eq. coefc.  Zero on the boundary.
__global__ void k_residual(int nc, int n_samples, const double* __restrict__ kappa, const double* __restrict__ f,
                           const double* __restrict__ u, double* __restrict__ r) {
  const long long nn = (long long)(nc + 1) * (nc + 1);
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nn * n_samples) return;
  const int s = int(t / nn);
  const int id = int(t % nn);
  const int i = id % (nc + 1), j = id / (nc + 1);
  double* rs = r + (long long)s * nn;
  if (i == 0 || j == 0 || i == nc || j == nc) {
    rs[id] = 0.0;
    return;
  }
  const double* us = u + (long long)s * nn;
  const double* ks = kappa + (long long)s * nc * nc * 2;
  const double h = 1.0 / nc;
  const double area = 0.5 * h * h;
  double au = 0.0, b = 0.0;
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) {
    const int ca = i - (cc == 1 || cc == 2 ? 1 : 0);
    const int cb = j - (cc >= 2 ? 1 : 0);
#pragma unroll
    for (int tri = 0; tri < 2; ++tri) {
      const int vx[3] = {ca, ca + 1, tri == 0 ? ca + 1 : ca};
      const int vy[3] = {cb, tri == 0 ? cb : cb + 1, cb + 1};
      int a = -1;
#pragma unroll
      for (int q = 0; q < 3; ++q)
        if (vx[q] == i && vy[q] == j) a = q;
      if (a < 0) continue;
      const double kap = ks[((long long)cb * nc + ca) * 2 + tri];
      const double det = double((vx[1] - vx[0]) * (vy[2] - vy[0]) - (vx[2] - vx[0]) * (vy[1] - vy[0]));
      const double gx[3] = {double(vy[1] - vy[2]), double(vy[2] - vy[0]), double(vy[0] - vy[1])};
      const double gy[3] = {double(vx[2] - vx[1]), double(vx[0] - vx[2]), double(vx[1] - vx[0])};
      const double scale = kap / (2.0 * fabs(det));
#pragma unroll
      for (int q = 0; q < 3; ++q)
        au += scale * (gx[a] * gx[q] + gy[a] * gy[q]) * us[(long long)vy[q] * (nc + 1) + vx[q]];
      b += area * f[id] / 3.0;
    }
  }
  rs[id] = b - au;
}

// Start of a solve with Dirichlet data: u = g on the outer boundary (g
// nodal, shared by all samples; nullptr = zero) and 0 inside, so that the
// residual b - A u is the lifted load b_I - A_ID g_D at the interior nodes.
__global__ void k_lift_init(int nc, int n_samples, const double* __restrict__ g, double* __restrict__ u) {
  const long long nn = (long long)(nc + 1) * (nc + 1);
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nn * n_samples) return;
  const int id = int(t % nn);
  const int i = id % (nc + 1), j = id / (nc + 1);
  const bool bnd = i == 0 || j == 0 || i == nc || j == nc;
  u[t] = (bnd && g) ? g[id] : 0.0;
}

// Fine-mesh nodal values of a P1 function given on the mesh of twice the
// step (both meshes split every cell along its SW-NE diagonal): a fine node
// is a coarse node or the midpoint of a coarse edge (horizontal, vertical or
// diagonal) and takes the coarse value or the mean of the edge's two ends.
// vc: [nc/2 + 1]^2, vf: [nc + 1]^2.
__global__ void k_prolong(int nc, const double* __restrict__ vc, double* __restrict__ vf) {
  const long long nn = (long long)(nc + 1) * (nc + 1);
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nn) return;
  const int i = int(t % (nc + 1)), j = int(t / (nc + 1));
  const int m1 = nc / 2 + 1;
  const int I0 = i / 2, J0 = j / 2;
  const int I1 = (i + 1) / 2, J1 = (j + 1) / 2;  // the other end of the edge (or the node itself)
  vf[t] = 0.5 * (vc[(long long)J0 * m1 + I0] + vc[(long long)J1 * m1 + I1]);
}

// Values of the field at the nodes of the mesh of twice the step.
__global__ void k_inject(int nc, const double* __restrict__ u, double* __restrict__ out) {
  const int m1 = nc / 2 + 1;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)m1 * m1) return;
  const int I = int(t % m1), J = int(t / m1);
  out[t] = u[(long long)(2 * J) * (nc + 1) + 2 * I];
}

__device__ __forceinline__ void atomic_max_abs(unsigned long long* p, double v) {
  atomicMax(p, (unsigned long long)__double_as_longlong(fabs(v)));
}

// u += d and per-sample max |d|, max |u| (as ordered bit patterns of
// non-negative doubles, so the maximum is exact and order independent).
// One atomic per workgroup and quantity: the waves reduce through LDS first.
// Samples with active[s] == 0 (a sample whose refinement has stopped) keep
// their field; active == nullptr updates every sample.
__global__ void __launch_bounds__(256) k_axpy_maxabs(int nc, int n_samples, double* __restrict__ u,
                                                     const double* __restrict__ d,
                                                     unsigned long long* __restrict__ maxbits,
                                                     const int* __restrict__ active) {
  __shared__ double red[2][4];
  const long long nn = (long long)(nc + 1) * (nc + 1);
  const int s = blockIdx.y;
  if (active && !active[s]) return;  // uniform over the workgroup
  double* us = u + (long long)s * nn;
  const double* ds = d + (long long)s * nn;
  double md = 0.0, mu = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (long long)gridDim.x * blockDim.x) {
    const double dv = ds[i];
    const double nv = us[i] + dv;
    us[i] = nv;
    md = fmax(md, fabs(dv));
    mu = fmax(mu, fabs(nv));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    md = fmax(md, __shfl_xor(md, o));
    mu = fmax(mu, __shfl_xor(mu, o));
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = md;
    red[1][wv] = mu;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const double m = fmax(fmax(red[threadIdx.x][0], red[threadIdx.x][1]), fmax(red[threadIdx.x][2], red[threadIdx.x][3]));
    atomic_max_abs(maxbits + 2 * s + threadIdx.x, m);
  }
}

// P1 interpolation at points (measurement "u in a few points", Section 1.2).
__global__ void k_points(int nc, int n_samples, int n_pts, const double* __restrict__ xy, const double* __restrict__ u,
                         double* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n_pts * n_samples) return;
  const int s = int(t / n_pts), p = int(t % n_pts);
  const long long nn = (long long)(nc + 1) * (nc + 1);
  const double* us = u + (long long)s * nn;
  const double x = xy[2 * p] * nc, y = xy[2 * p + 1] * nc;
  int ci = int(floor(x)), cj = int(floor(y));
  ci = ci < 0 ? 0 : (ci > nc - 1 ? nc - 1 : ci);
  cj = cj < 0 ? 0 : (cj > nc - 1 ? nc - 1 : cj);
  const double fx = x - ci, fy = y - cj;
  const double u00 = us[(long long)cj * (nc + 1) + ci];
  const double u11 = us[(long long)(cj + 1) * (nc + 1) + ci + 1];
  double v;
  if (fx >= fy) v = (1.0 - fx) * u00 + (fx - fy) * us[(long long)cj * (nc + 1) + ci + 1] + fy * u11;
  else v = (1.0 - fy) * u00 + fx * u11 + (fy - fx) * us[(long long)(cj + 1) * (nc + 1) + ci];
  out[t] = v;
}

// The same interpolation for sample-specific point sets: point t belongs to
// sample smp[t].
__global__ void k_points_ragged(int nc, int n_total, const double* __restrict__ xy, const int* __restrict__ smp,
                                const double* __restrict__ u, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_total) return;
  const long long nn = (long long)(nc + 1) * (nc + 1);
  const double* us = u + (long long)smp[t] * nn;
  const double x = xy[2 * t] * nc, y = xy[2 * t + 1] * nc;
  int ci = int(floor(x)), cj = int(floor(y));
  ci = ci < 0 ? 0 : (ci > nc - 1 ? nc - 1 : ci);
  cj = cj < 0 ? 0 : (cj > nc - 1 ? nc - 1 : cj);
  const double fx = x - ci, fy = y - cj;
  const double u00 = us[(long long)cj * (nc + 1) + ci];
  const double u11 = us[(long long)(cj + 1) * (nc + 1) + ci + 1];
  double v;
  if (fx >= fy) v = (1.0 - fx) * u00 + (fx - fy) * us[(long long)cj * (nc + 1) + ci + 1] + fy * u11;
  else v = (1.0 - fy) * u00 + fx * u11 + (fy - fx) * us[(long long)(cj + 1) * (nc + 1) + ci];
  out[t] = v;
}

// u at a list of global node ids, for every sample: out[s][k] = u_s(ids[k]).
__global__ void k_gather(int n_ids, int n_samples, const int* __restrict__ ids, const double* __restrict__ u,
                         long long ustride, double* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n_ids * n_samples) return;
  const int s = int(t / n_ids), k = int(t % n_ids);
  out[t] = u[(long long)s * ustride + ids[k]];
}

// eq. mean: sum over triangles of (|t|/3)(u1+u2+u3) / |R|, one block per
// sample, fixed reduction order.
__global__ void __launch_bounds__(256) k_mean(int nc, int i0, int i1, int j0, int j1, const double* __restrict__ u,
                                              double* __restrict__ out) {
  __shared__ double part[256];
  const int s = blockIdx.x;
  const double* us = u + (long long)s * (nc + 1) * (nc + 1);
  const double h = 1.0 / nc;
  const double at = 0.5 * h * h;
  const int w = i1 - i0;
  const long long ncell = (long long)w * (j1 - j0);
  double acc = 0.0;
  for (long long c = threadIdx.x; c < ncell; c += 256) {
    const int i = i0 + int(c % w), j = j0 + int(c / w);
    const double a = us[(long long)j * (nc + 1) + i], b = us[(long long)j * (nc + 1) + i + 1];
    const double cc = us[(long long)(j + 1) * (nc + 1) + i + 1], d = us[(long long)(j + 1) * (nc + 1) + i];
    acc += at / 3.0 * (a + b + cc) + at / 3.0 * (a + cc + d);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[s] = part[0] / (double(ncell) * h * h);
}

// Gaussian log-likelihood (product of noise densities, Section 1.2):
// -sum (y - Hu)^2 / (2 sigma^2), optionally - n_y log(sigma sqrt(2 pi)).
// Log-likelihood per sample over its own observations y[off[s] .. off[s+1])
// with its own noise level sigma[s]; one block per sample, fixed order.
__global__ void __launch_bounds__(256) k_loglik_ragged(const int* __restrict__ off, const double* __restrict__ hu,
                                                       const double* __restrict__ y, const double* __restrict__ sigma,
                                                       int normalized, double* __restrict__ out) {
  __shared__ double part[256];
  const int s = blockIdx.x;
  const int i0 = off[s], i1 = off[s + 1];
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += 256) {
    const double r = y[i] - hu[i];
    acc += r * r;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double sg = sigma[s];
    double v = -part[0] / (2.0 * sg * sg);
    if (normalized) v -= (i1 - i0) * log(sg * sqrt(2.0 * M_PI));
    out[s] = v;
  }
}

__global__ void __launch_bounds__(256) k_loglik(int n_y, const double* __restrict__ hu, const double* __restrict__ y,
                                                double sigma, int normalized, double* __restrict__ out) {
  __shared__ double part[256];
  const int s = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n_y; i += 256) {
    const double r = y[i] - hu[(long long)s * n_y + i];
    acc += r * r;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double v = -part[0] / (2.0 * sigma * sigma);
    if (normalized) v -= n_y * log(sigma * sqrt(2.0 * M_PI));
    out[s] = v;
  }
}

// Matrix-core layout check: C = A B^T for A, B = fixed 32 x 8 / 16 x 8
// patterns through the same builtins and fragment mapping as the Schur
// update.  out: 32*32 (f32) or 16*16 (f64) doubles.
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
__global__ void k_mfma_selftest(int dtype, double* out) {
  const int lane = threadIdx.x;
  if (dtype == 0) {
    floatx16 acc;
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
    for (int kk = 0; kk < 8; kk += 2) {
      const int i = lane & 31, k = kk + (lane >> 5);
      const float a = float((i * 7 + k * 3) % 11) - 5.f;
      const float b = float((i * 5 + k * 2) % 13) - 6.f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    for (int v = 0; v < 16; ++v) {
      const int i = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3), j = lane & 31;
      out[i * 32 + j] = acc[v];
    }
  } else {
    doublex4 acc;
    for (int v = 0; v < 4; ++v) acc[v] = 0.0;
    for (int kk = 0; kk < 8; kk += 4) {
      const int i = lane & 15, k = kk + (lane >> 4);
      const double a = double((i * 7 + k * 3) % 11) - 5.0;
      const double b = double((i * 5 + k * 2) % 13) - 6.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * v + (lane >> 4), j = lane & 15;
      out[i * 16 + j] = acc[v];
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Interfaces at least this wide run the solves' matrix-vector products as
// separate launches spread over many workgroups.
constexpr int kSplitGamma = 127;

hipError_t launch_topdown(const DevLevel& L, const int* list, int n_list, int n_samples, double* u, long long ustride,
                          bool z_from_vec, hipStream_t st) {
  if (n_list <= 0) return hipSuccess;
  dim3 grid(n_list * n_samples);
  const int zv = z_from_vec ? 1 : 0;
  const int split = (L.gam >= kSplitGamma && (L.max_U - L.gam) > 0) ? 1 : 0;
  if (split && L.lr_store) {
    const hipError_t e = launch_lr_topdown_gemv(L, list, n_list, n_samples, u, ustride, z_from_vec, st);
    if (e != hipSuccess) return e;
  } else if (split) {
    dim3 g2(n_list * n_samples, ceil_div(L.gam, 64));
    const size_t lds = sizeof(double) * (size_t((L.max_U - L.gam)) + 256);
    if (L.is_double)
      hipLaunchKernelGGL(k_topdown_gemv<double>, g2, dim3(256), lds, st, L, list, n_samples, u, ustride, zv);
    else
      hipLaunchKernelGGL(k_topdown_gemv<float>, g2, dim3(256), lds, st, L, list, n_samples, u, ustride, zv);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const bool no_part = split || L.max_U == L.gam;  // no transposed GEMV in this kernel
  if (L.gam > 64 && no_part && n_list * n_samples < 256) {  // few workgroups: 16 waves each
    const size_t lds = solve_lds(L.max_U, L.gam, 1024, false);
    if (L.is_double)
      hipLaunchKernelGGL((k_topdown<double, 1024>), grid, dim3(1024), lds, st, L, list, n_samples, u, ustride, zv,
                         split);
    else
      hipLaunchKernelGGL((k_topdown<float, 1024>), grid, dim3(1024), lds, st, L, list, n_samples, u, ustride, zv,
                         split);
  } else if (L.gam <= 64) {
    const size_t lds = solve_lds(L.max_U, L.gam, 64);
    if (L.is_double)
      hipLaunchKernelGGL((k_topdown<double, 64>), grid, dim3(64), lds, st, L, list, n_samples, u, ustride, zv, split);
    else
      hipLaunchKernelGGL((k_topdown<float, 64>), grid, dim3(64), lds, st, L, list, n_samples, u, ustride, zv, split);
  } else {
    const size_t lds = solve_lds(L.max_U, L.gam, 256);
    if (L.is_double)
      hipLaunchKernelGGL((k_topdown<double, 256>), grid, dim3(256), lds, st, L, list, n_samples, u, ustride, zv,
                         split);
    else
      hipLaunchKernelGGL((k_topdown<float, 256>), grid, dim3(256), lds, st, L, list, n_samples, u, ustride, zv,
                         split);
  }
  return hipGetLastError();
}

hipError_t launch_forward(const DevLevel& L, const DevLevel& child, int n_samples, hipStream_t st) {
  dim3 grid(L.n_nodes * n_samples);
  const int split = (L.gam >= kSplitGamma && (L.max_U - L.gam) > 0) ? 1 : 0;
  if (L.gam > 64 && L.n_nodes * n_samples < 256) {  // few workgroups: 16 waves each
    const size_t lds = solve_lds(L.max_U, L.gam, 1024, false);
    if (L.is_double)
      hipLaunchKernelGGL((k_forward<double, 1024>), grid, dim3(1024), lds, st, L, child, n_samples, split);
    else
      hipLaunchKernelGGL((k_forward<float, 1024>), grid, dim3(1024), lds, st, L, child, n_samples, split);
  } else if (L.gam <= 64) {
    const size_t tile = size_t(32) * 65 * (L.is_double ? 8 : 4);
    const size_t lds = sizeof(double) * size_t(L.max_U + 1) + tile;
    if (L.is_double)
      hipLaunchKernelGGL((k_forward<double, 64>), grid, dim3(64), lds, st, L, child, n_samples, split);
    else
      hipLaunchKernelGGL((k_forward<float, 64>), grid, dim3(64), lds, st, L, child, n_samples, split);
  } else {
    const size_t lds = solve_lds(L.max_U, L.gam, 256);
    if (L.is_double)
      hipLaunchKernelGGL((k_forward<double, 256>), grid, dim3(256), lds, st, L, child, n_samples, split);
    else
      hipLaunchKernelGGL((k_forward<float, 256>), grid, dim3(256), lds, st, L, child, n_samples, split);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !split) return e;
  if (L.lr_store) return launch_lr_forward_gemv(L, n_samples, st);
  dim3 g2(L.n_nodes * n_samples, ceil_div((L.max_U - L.gam), 128));
  const size_t lds = sizeof(double) * size_t(L.gam) + size_t(4) * 32 * 65 * (L.is_double ? 8 : 4);
  if (L.is_double)
    hipLaunchKernelGGL(k_forward_gemv<double>, g2, dim3(256), lds, st, L, n_samples);
  else
    hipLaunchKernelGGL(k_forward_gemv<float>, g2, dim3(256), lds, st, L, n_samples);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, long long n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  dim3 grid(std::max(1, std::min(ceil_div(n, 256), 65536))), block(256);
  hipLaunchKernelGGL(k_fill, grid, block, 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, long long n, int v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  dim3 grid(std::max(1, std::min(ceil_div(n, 256), 65536))), block(256);
  hipLaunchKernelGGL(k_fill_i32, grid, block, 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_prolong(int nc, const double* vc, double* vf, hipStream_t st) {
  const long long n = (long long)(nc + 1) * (nc + 1);
  hipLaunchKernelGGL(k_prolong, dim3(ceil_div(n, 256)), dim3(256), 0, st, nc, vc, vf);
  return hipGetLastError();
}

hipError_t launch_inject(int nc, const double* u, double* out, hipStream_t st) {
  const long long n = (long long)(nc / 2 + 1) * (nc / 2 + 1);
  hipLaunchKernelGGL(k_inject, dim3(ceil_div(n, 256)), dim3(256), 0, st, nc, u, out);
  return hipGetLastError();
}

hipError_t launch_lift_init(int nc, int n_samples, const double* g, double* u, hipStream_t st) {
  const long long n = (long long)(nc + 1) * (nc + 1) * n_samples;
  hipLaunchKernelGGL(k_lift_init, dim3(ceil_div(n, 256)), dim3(256), 0, st, nc, n_samples, g, u);
  return hipGetLastError();
}

hipError_t launch_residual(int nc, int n_samples, const double* kappa, const double* f, const double* u, double* r,
                           hipStream_t st) {
  const long long n = (long long)(nc + 1) * (nc + 1) * n_samples;
  hipLaunchKernelGGL(k_residual, dim3(ceil_div(n, 256)), dim3(256), 0, st, nc, n_samples, kappa, f, u, r);
  return hipGetLastError();
}

hipError_t launch_axpy_maxabs(int nc, int n_samples, double* u, const double* d, unsigned long long* maxbits,
                              const int* active, hipStream_t st) {
  const long long nn = (long long)(nc + 1) * (nc + 1);
  // about 16 elements per thread: 4096 / n_samples workgroups per sample at most
  const int per = std::max(1, std::min(ceil_div(nn, 256 * 16), std::max(16, 4096 / std::max(n_samples, 1))));
  dim3 grid(per, n_samples);
  hipLaunchKernelGGL(k_axpy_maxabs, grid, dim3(256), 0, st, nc, n_samples, u, d, maxbits, active);
  return hipGetLastError();
}

hipError_t launch_points(int nc, int n_samples, int n_pts, const double* xy, const double* u, double* out,
                         hipStream_t st) {
  const long long n = (long long)n_pts * n_samples;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_points, dim3(ceil_div(n, 128)), dim3(128), 0, st, nc, n_samples, n_pts, xy, u, out);
  return hipGetLastError();
}

hipError_t launch_gather(int n_ids, int n_samples, const int* ids, const double* u, long long ustride, double* out,
                         hipStream_t st) {
  const long long n = (long long)n_ids * n_samples;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3(ceil_div(n, 256)), dim3(256), 0, st, n_ids, n_samples, ids, u, ustride, out);
  return hipGetLastError();
}

hipError_t launch_mean(int nc, int n_samples, int i0, int i1, int j0, int j1, const double* u, double* out,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_mean, dim3(n_samples), dim3(256), 0, st, nc, i0, i1, j0, j1, u, out);
  return hipGetLastError();
}

hipError_t launch_points_ragged(int nc, int n_total, const double* xy, const int* smp, const double* u, double* out,
                                hipStream_t st) {
  if (n_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_points_ragged, dim3(ceil_div(n_total, 128)), dim3(128), 0, st, nc, n_total, xy, smp, u, out);
  return hipGetLastError();
}

hipError_t launch_loglik_ragged(int n_samples, const int* off, const double* hu, const double* y, const double* sigma,
                                int normalized, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_loglik_ragged, dim3(n_samples), dim3(256), 0, st, off, hu, y, sigma, normalized, out);
  return hipGetLastError();
}

hipError_t launch_loglik(int n_samples, int n_y, const double* hu, const double* y, double sigma, int normalized,
                         double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_loglik, dim3(n_samples), dim3(256), 0, st, n_y, hu, y, sigma, normalized, out);
  return hipGetLastError();
}

hipError_t launch_mfma_selftest(int dtype, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_mfma_selftest, dim3(1), dim3(64), 0, st, dtype, out);
  return hipGetLastError();
}

}  // namespace hdd
