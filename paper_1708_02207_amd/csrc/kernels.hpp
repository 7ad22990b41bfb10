// Host-side launchers of the HDD kernels (all launches are asynchronous on
// the given stream; they return the launch status only).
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "hdd.h"

namespace hdd {

// hdd_create with an extra mode: no_alloc takes the caller's workspace and
// stream (null: the null stream) and makes no device, pinned-host or event
// allocation, at creation or later.
int create_handle(const hdd_opts* o, int32_t max_samples, void* stream, void* workspace, size_t workspace_bytes,
                  bool no_alloc, hdd_handle* out);

constexpr int kPanelNB = 32;  // panel width of the interface factorization

// Leaves to Root
hipError_t launch_extend_add(const DevLevel& F, const DevLevel& S, int n_samples, hipStream_t st);
hipError_t launch_panel(const DevLevel& L, int k0, int kb, int n_samples, int* info, hipStream_t st);
// Rank-K update C[r0.., c0..c1) -= F[.., k0..k1) F[.., k0..k1)^T of every
// node's frame (lower triangle; r0 == c0, else hipErrorInvalidValue).  tile:
// 0 = the built-in rule (128 x 128 tiles for float32
// updates with K >= 96 on large frames, else 64 x 64), 64 or 128 to force a
// tile (128 only on float32 matrix-core levels).
hipError_t launch_syrk(const DevLevel& L, int k0, int k1, int r0, int c0, int c1, int n_samples, bool mfma,
                       int tile, hipStream_t st);
bool syrk_uses_big_tile(const DevLevel& L, int k0, int k1, int r0, int c0, int c1, bool mfma, int tile);
// Fused extend-add + factorization + Schur update of a float32 level with
// gamma <= 31 (matrix cores), one workgroup per node and sample, when the
// node's panel fits in LDS.
bool merge_small_ok(const DevLevel& F, bool mfma);
hipError_t launch_merge_small(const DevLevel& F, const DevLevel& S, int n_samples, int* info, hipStream_t st);
// Fused factorization + Schur update of a float32 level with gamma = 63
// (matrix cores), one workgroup per node and sample, on the frame filled by
// the extend-add, when the node's panel fits in LDS.
bool eliminate_mid_ok(const DevLevel& L, bool mfma);
hipError_t launch_eliminate_mid(const DevLevel& L, int n_samples, int* info, hipStream_t st);

// Blocks (in-LDS nested dissection of the leaf interior)
size_t block_build_lds(const DevBlocks& B, bool dbl);
size_t block_topdown_lds(const DevBlocks& B, bool dbl);
size_t block_forward_lds(const DevBlocks& B, bool dbl);
bool block_shape_ok(const DevBlocks& B);  // template sizes match the compiled shapes
size_t block_ext_entries(int s);          // entries of the extend-add gather table
hipError_t launch_block_ext(const DevBlocks& B, unsigned* ext, hipStream_t st);
hipError_t launch_block_build(const DevBlocks& B, int n_samples, int nc, const double* kappa, const double* f,
                              int* bad, int* info, hipStream_t st);
hipError_t launch_block_topdown(const DevBlocks& B, const int* list, int n_list, int n_samples, int nc, double* u,
                                long long ustride, bool from_vec, hipStream_t st);
hipError_t launch_block_forward(const DevBlocks& B, int n_samples, int nc, const double* r, long long rstride,
                                hipStream_t st);

// Root to Leaves and right-hand-side propagation
hipError_t launch_topdown(const DevLevel& L, const int* list, int n_list, int n_samples, double* u,
                          long long ustride, bool z_from_vec, hipStream_t st);
hipError_t launch_forward(const DevLevel& L, const DevLevel& child, int n_samples, hipStream_t st);

// Full-field and readout kernels (FP64)
hipError_t launch_fill(double* p, long long n, double v, hipStream_t st);
hipError_t launch_fill_i32(int* p, long long n, int v, hipStream_t st);
hipError_t launch_prolong(int nc, const double* vc, double* vf, hipStream_t st);
hipError_t launch_inject(int nc, const double* u, double* out, hipStream_t st);
hipError_t launch_lift_init(int nc, int n_samples, const double* g, double* u, hipStream_t st);
hipError_t launch_residual(int nc, int n_samples, const double* kappa, const double* f, const double* u,
                           double* r, hipStream_t st);
hipError_t launch_axpy_maxabs(int nc, int n_samples, double* u, const double* d, unsigned long long* maxbits,
                              const int* active, hipStream_t st);
hipError_t launch_points(int nc, int n_samples, int n_pts, const double* xy, const double* u, double* out,
                         hipStream_t st);
hipError_t launch_gather(int n_ids, int n_samples, const int* ids, const double* u, long long ustride, double* out,
                         hipStream_t st);
hipError_t launch_mean(int nc, int n_samples, int i0, int i1, int j0, int j1, const double* u, double* out,
                       hipStream_t st);
hipError_t launch_points_ragged(int nc, int n_total, const double* xy, const int* smp, const double* u, double* out,
                                hipStream_t st);
hipError_t launch_loglik_ragged(int n_samples, const int* off, const double* hu, const double* y, const double* sigma,
                                int normalized, double* out, hipStream_t st);
hipError_t launch_loglik(int n_samples, int n_y, const double* hu, const double* y, double sigma, int normalized,
                         double* out, hipStream_t st);
hipError_t launch_mfma_selftest(int dtype, double* out, hipStream_t st);

// Block low-rank maps P (kernels_lowrank.hip): blocks of kLowRankBlock x
// kLowRankBlock, low-rank blocks with at most kLowRankMax rank slots.
constexpr int kLowRankBlock = 64;
constexpr int kLowRankMax = 16;
hipError_t launch_lr_compress(const DevLevel& L, int n_samples, double tol, hipStream_t st);
hipError_t launch_lr_topdown_gemv(const DevLevel& L, const int* list, int n_list, int n_samples, double* u,
                                  long long ustride, bool z_from_vec, hipStream_t st);
hipError_t launch_lr_forward_gemv(const DevLevel& L, int n_samples, hipStream_t st);

// Means over every subdomain of the tree (functional propagation, or the
// direct sum when the whole field is known).  mu / out: [sample][global node].
hipError_t launch_block_mu(const DevBlocks& B, int n_samples, double* mu, long long mu_stride, hipStream_t st);
hipError_t launch_level_mu(const DevLevel& L, const DevLevel& child, int n_samples, double* mu, long long mu_stride,
                           hipStream_t st);
hipError_t launch_node_means(const DevLevel& L, int n_samples, int nc, const double* u, long long ustride,
                             const double* mu, long long mu_stride, double* out, long long out_stride,
                             hipStream_t st);
hipError_t launch_block_integral(const DevLevel& L, int n_samples, int nc, const double* u, long long ustride,
                                 double* mu, long long mu_stride, double* out, long long out_stride, hipStream_t st);
hipError_t launch_level_sum(const DevLevel& L, const DevLevel& child, int n_samples, int nc, double* mu,
                            long long mu_stride, double* out, long long out_stride, hipStream_t st);

}  // namespace hdd
