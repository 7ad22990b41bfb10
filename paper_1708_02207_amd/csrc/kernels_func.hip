// Means of u_h over every subdomain of the tree (Section 5.1, the example
// after Lemma Func1, and the algorithms of Section 5.2).
//
// The integral of u_h over a node omega is a linear functional of the node's
// data, (l^f, f) + (l^g, u_Gamma) (eq. prop1); the integrals of the two sons
// add up to the father's (eq. prop2 with c_1 = c_2 = 1; the means follow by
// dividing by |omega|).  Lemma Func1 builds the father's representation from
// the sons': with the son-union frame [gamma ; Gamma] and the sons'
// functionals summed into it (l~),
//   l^g_omega   = l~_Gamma + (Phi^g)^T l~_gamma = l~_Gamma - P L^-1 l~_gamma
//   (l^f, f)    = (l^f_1, f_1) + (l^f_2, f_2) + l~_gamma . Phi^f f
// where Phi^f f = S~_gg^-1 g~_gamma is the node's interface solution for zero
// boundary values, so the last term is (L^-1 l~_gamma) . z with the retained
// z = L^-1 g~_gamma of the build (inside a block: l~_gamma . y with the
// retained y = A_gg^-1 b_gamma).  The l^g recursion has exactly the form of
// the bottom-up load elimination, so the forward-pass kernels build it from a
// nodal weight vector; the scalars mu_omega = (l^f_omega, f_omega) are the
// dot products below, summed over the subtree.
//
// Quadrature weights.  The forward pass hands every mesh node's load to the
// micro-block that holds the cell whose lower-left corner the node is, so
// with the weight vector h^2 at every node it propagates, for every node, the
// functional sum over the nodes "owned" by omega of h^2 u_p.  It differs from
// the integral (each node p weighted by (h^2/6) times the number of omega's
// triangles at p) only on Gamma; the readout adds that difference, so no
// block interior is ever solved.
//
// When the whole field is already known (after refinement), the integrals
// are summed directly from it (eq. mean per block, then sons into fathers).
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace hdd {
namespace {

constexpr int FT = 256;

// Sum of one value per thread in a fixed order; the result is valid in
// thread 0.
__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < FT / 64; ++k) t += red[k];
  return t;
}

// mu of every block: sum over the nodes t of its sub-tree of
// l~_gamma(t) . y_t, where l~_gamma(t) is the functional's interface load left
// in the vector store by the forward pass and y_t = A_gg^-1 b_gamma is the
// build's interface solution for zero boundary values (compact store row U).
template <typename T>
__global__ void __launch_bounds__(FT) k_block_mu(DevBlocks B, int n_samples, double* __restrict__ mu,
                                                 long long mu_stride) {
  __shared__ double red[FT / 64];
  const int q = blockIdx.x / n_samples;
  const int s = blockIdx.x % n_samples;
  const T* cst = reinterpret_cast<const T*>(B.cst) + (long long)s * B.cst_stride + (long long)q * B.cst_size;
  const double* vz = B.vec + (long long)s * B.vec_stride + (long long)q * B.vec_size;
  // one entry of the store per thread (the levels' entries are contiguous,
  // level K at vec_off[K]), every load issued before any is used
  double acc = 0.0;
  for (int e0 = 0; e0 < B.vec_size; e0 += FT) {
    const int e = e0 + int(threadIdx.x);
    int K = 0;
    for (int k = 1; k < B.nlev; ++k)
      if (e >= B.lv[k].vec_off) K = k;
    const DevSubLevel l = B.lv[K];
    const int r = min(e, B.vec_size - 1) - l.vec_off;
    const int t = r / l.gam, i = r % l.gam;
    const double a = vz[l.vec_off + r];
    const double y = double(cst[l.cst_off + (long long)t * (l.U + 1) * l.gam + (long long)l.U * l.gam + i]);
    if (e < B.vec_size) acc += a * y;
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) mu[(long long)s * mu_stride + B.top.node_base + q] = tot;
}

// mu of the nodes of a level above the blocks: (L^-1 l~_gamma) . z plus the
// sons' mu.
template <typename T>
__global__ void __launch_bounds__(FT) k_level_mu(DevLevel L, DevLevel C, int n_samples, double* __restrict__ mu,
                                                 long long mu_stride) {
  __shared__ double red[FT / 64];
  const int node = blockIdx.x / n_samples;
  const int s = blockIdx.x % n_samples;
  const DevNode nd = L.nodes[node];
  const int g = L.gam;
  int ld;
  const T* F = retained_ptr<T>(L, node, s, ld);
  const T* z = F + (long long)nd.U * ld;
  const double* v = L.vec + (long long)s * L.vec_stride + nd.ids_off;
  double acc = 0.0;
  for (int i = threadIdx.x; i < g; i += FT) acc += v[i] * double(z[i]);
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) {
    double* m = mu + (long long)s * mu_stride;
    m[L.node_base + node] = tot + m[C.node_base + 2 * node] + m[C.node_base + 2 * node + 1];
  }
}

// Mean of every node of a level from its functional and u on its boundary:
// integral = mu + sum_j (l'_j + c_j) u_j, with l' the propagated functional
// on Gamma and c_j = (h^2/6) (triangles of omega at node j) - h^2 [node j
// owned by omega].  Outer Dirichlet nodes (kept in block boundaries) hold
// u = 0.
__global__ void __launch_bounds__(FT) k_node_means(DevLevel L, int n_samples, int nc, const double* __restrict__ u,
                                                   long long ustride, const double* __restrict__ mu,
                                                   long long mu_stride, double* __restrict__ out,
                                                   long long out_stride) {
  __shared__ double red[FT / 64];
  const int node = blockIdx.x / n_samples;
  const int s = blockIdx.x % n_samples;
  const DevNode nd = L.nodes[node];
  const int g = nd.U - nd.bnd, G = nd.bnd;
  const int* ids = L.ids + nd.ids_off + g;
  const double* lam = L.vec + (long long)s * L.vec_stride + nd.ids_off + g;
  const double* us = u + (long long)s * ustride;
  const double h = 1.0 / nc;
  const double h2 = h * h;
  double acc = 0.0;
  for (int j = threadIdx.x; j < G; j += FT) {
    const int id = ids[j];
    const int a = id % (nc + 1) - nd.x0, b = id / (nc + 1) - nd.y0;  // node in the rectangle's cell frame
    const int c00 = (a >= 0 && a < nd.cw && b >= 0 && b < nd.ch) ? 1 : 0;          // cell (a, b): T- and T+
    const int c10 = (a >= 1 && a <= nd.cw && b >= 0 && b < nd.ch) ? 1 : 0;         // cell (a-1, b): T-
    const int c01 = (a >= 0 && a < nd.cw && b >= 1 && b <= nd.ch) ? 1 : 0;         // cell (a, b-1): T+
    const int c11 = (a >= 1 && a <= nd.cw && b >= 1 && b <= nd.ch) ? 1 : 0;        // cell (a-1, b-1): T- and T+
    const double c = h2 * double(2 * c00 + c10 + c01 + 2 * c11) / 6.0 - h2 * double(c00);
    acc += (lam[j] + c) * us[id];
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) {
    const int k = L.node_base + node;
    out[(long long)s * out_stride + k] = (mu[(long long)s * mu_stride + k] + tot) / (double(nd.cw) * nd.ch * h2);
  }
}

// Integral of u_h over every block from the field (eq. mean), fixed order.
__global__ void __launch_bounds__(FT) k_block_integral(DevLevel L, int n_samples, int nc, const double* __restrict__ u,
                                                       long long ustride, double* __restrict__ mu,
                                                       long long mu_stride, double* __restrict__ out,
                                                       long long out_stride) {
  __shared__ double red[FT / 64];
  const int node = blockIdx.x / n_samples;
  const int s = blockIdx.x % n_samples;
  const DevNode nd = L.nodes[node];
  const double* us = u + (long long)s * ustride;
  const double h = 1.0 / nc;
  const double t3 = 0.5 * h * h / 3.0;  // |t| / 3
  const int n1 = nc + 1;
  double acc = 0.0;
  for (int c = threadIdx.x; c < nd.cw * nd.ch; c += FT) {
    const int i = nd.x0 + c % nd.cw, j = nd.y0 + c / nd.cw;
    const double a = us[(long long)j * n1 + i], b = us[(long long)j * n1 + i + 1];
    const double cc = us[(long long)(j + 1) * n1 + i + 1], d = us[(long long)(j + 1) * n1 + i];
    acc += t3 * (a + b + cc) + t3 * (a + cc + d);
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) {
    const int k = L.node_base + node;
    mu[(long long)s * mu_stride + k] = tot;
    out[(long long)s * out_stride + k] = tot / (double(nd.cw) * nd.ch * h * h);
  }
}

// Father integral = sum of the sons' (the means average with c_i = |omega_i| / |omega|).
__global__ void __launch_bounds__(FT) k_level_sum(DevLevel L, DevLevel C, int n_samples, int nc,
                                                  double* __restrict__ mu, long long mu_stride,
                                                  double* __restrict__ out, long long out_stride) {
  const long long t = (long long)blockIdx.x * FT + threadIdx.x;
  if (t >= (long long)L.n_nodes * n_samples) return;
  const int node = int(t / n_samples);
  const int s = int(t % n_samples);
  const DevNode nd = L.nodes[node];
  const double h = 1.0 / nc;
  double* m = mu + (long long)s * mu_stride;
  const double v = m[C.node_base + 2 * node] + m[C.node_base + 2 * node + 1];
  m[L.node_base + node] = v;
  out[(long long)s * out_stride + L.node_base + node] = v / (double(nd.cw) * nd.ch * h * h);
}

}  // namespace

hipError_t launch_block_mu(const DevBlocks& B, int n_samples, double* mu, long long mu_stride, hipStream_t st) {
  const dim3 grid(unsigned(B.nb) * unsigned(n_samples));
  if (B.top.is_double)
    hipLaunchKernelGGL(k_block_mu<double>, grid, dim3(FT), 0, st, B, n_samples, mu, mu_stride);
  else
    hipLaunchKernelGGL(k_block_mu<float>, grid, dim3(FT), 0, st, B, n_samples, mu, mu_stride);
  return hipGetLastError();
}

hipError_t launch_level_mu(const DevLevel& L, const DevLevel& child, int n_samples, double* mu, long long mu_stride,
                           hipStream_t st) {
  const dim3 grid(unsigned(L.n_nodes) * unsigned(n_samples));
  if (L.is_double)
    hipLaunchKernelGGL(k_level_mu<double>, grid, dim3(FT), 0, st, L, child, n_samples, mu, mu_stride);
  else
    hipLaunchKernelGGL(k_level_mu<float>, grid, dim3(FT), 0, st, L, child, n_samples, mu, mu_stride);
  return hipGetLastError();
}

hipError_t launch_node_means(const DevLevel& L, int n_samples, int nc, const double* u, long long ustride,
                             const double* mu, long long mu_stride, double* out, long long out_stride,
                             hipStream_t st) {
  const dim3 grid(unsigned(L.n_nodes) * unsigned(n_samples));
  hipLaunchKernelGGL(k_node_means, grid, dim3(FT), 0, st, L, n_samples, nc, u, ustride, mu, mu_stride, out,
                     out_stride);
  return hipGetLastError();
}

hipError_t launch_block_integral(const DevLevel& L, int n_samples, int nc, const double* u, long long ustride,
                                 double* mu, long long mu_stride, double* out, long long out_stride, hipStream_t st) {
  const dim3 grid(unsigned(L.n_nodes) * unsigned(n_samples));
  hipLaunchKernelGGL(k_block_integral, grid, dim3(FT), 0, st, L, n_samples, nc, u, ustride, mu, mu_stride, out,
                     out_stride);
  return hipGetLastError();
}

hipError_t launch_level_sum(const DevLevel& L, const DevLevel& child, int n_samples, int nc, double* mu,
                            long long mu_stride, double* out, long long out_stride, hipStream_t st) {
  const long long n = (long long)L.n_nodes * n_samples;
  hipLaunchKernelGGL(k_level_sum, dim3(unsigned((n + FT - 1) / FT)), dim3(FT), 0, st, L, child, n_samples, nc, mu,
                     mu_stride, out, out_stride);
  return hipGetLastError();
}

}  // namespace hdd
