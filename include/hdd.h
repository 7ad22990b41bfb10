/*
 * hdd.h -- C ABI of the MI355X hierarchical domain decomposition (HDD)
 * partial inverse for -div(kappa(x, Z) grad u) = f on the unit square with
 * P1 finite elements and zero Dirichlet data (problem statement, eq.
 * elliptic; notation of Section 2.1).
 *
 * The library builds, for many parameter samples Z at once, the HDD tree
 * bottom-up ("Leaves to Root", Section 3.4): leaf assembly (Section 3.1,
 * eq. coefA and eq. coefc), elimination of every subdomain's interface by the
 * Schur complement (Section 2.4, eq. SchurMinus1 / eq. SchurC1; merge of two
 * sons, Section 3.2-3.3, eq. block_equation4 and eq. gamma), keeping the maps
 * Phi of every node in factored form.  Queries then run "Root to Leaves"
 * only along the paths they need (Section 5.3) and apply the measurement
 * operators of Section 1.2 (point values; integral / mean over a subdomain,
 * eq. mean) and the Gaussian likelihood L(z) = prod pi_eps(y_i - S_i(z)).
 *
 * Conventions (all entry points):
 *  - Every call returns an int status: HDD_OK (0) or a negative HDD_E* code;
 *    no exception crosses the ABI.  hdd_strerror() names a code.
 *  - Mesh: N interior nodes per side, Nc = N + 1 cells, h = 1/Nc; Nc must be
 *    leaf * 2^p and leaf must be 2 * 2^q.  Cell (i, j) is split along its
 *    SW-NE diagonal into T- (index 0) and T+ (index 1).
 *  - kappa: float64 [n_samples][Nc][Nc][2], per triangle, [j][i][T-/T+],
 *    strictly positive and finite.  f: float64 [N+2][N+2] nodal, [j][i]
 *    (boundary entries are read by the leaf assembly but multiply zero data).
 *  - Pointer kind: arguments documented "(mem)" are host pointers when the
 *    call's `mem` argument is HDD_MEM_HOST and device pointers (HBM) when it
 *    is HDD_MEM_DEVICE.  Other pointers are host pointers.  Inputs are read
 *    during the call only (device inputs: before the call's work on the
 *    handle's stream completes); outputs are caller-allocated.
 *  - Work is issued on the handle's stream.  Calls that return host data
 *    synchronize that stream; device-output calls do not.
 *  - A handle is not thread safe; calls on one handle are ordered.
 */
#ifndef HDD_H_
#define HDD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* largest total number of sites of one ragged query (all samples together) */
#define HDD_MAX_QUERY_POINTS 4096

/* status codes */
#define HDD_OK 0
#define HDD_EINVAL (-1)         /* bad argument, shape or non-positive/non-finite kappa */
#define HDD_ENOMEM (-2)         /* workspace too small / device allocation failed */
#define HDD_ENOTSPD (-3)        /* non-positive pivot in an interface factorization; see hdd_last_node */
#define HDD_ENOTCONVERGED (-4)  /* iterative refinement did not reach refine_tol in max_refine sweeps */
#define HDD_EDEVICE (-5)        /* HIP runtime error */
#define HDD_ESTATE (-6)         /* call out of order (e.g. query before build) */

/* precision modes */
#define HDD_FP64 0          /* every level factored in float64 */
#define HDD_FP32_REFINE 1   /* float32 levels (matrix-core Schur updates), the top
                               fp64_top_levels levels in float64, then float64
                               iterative refinement of the full field against the
                               assembled operator */

/* pointer kinds */
#define HDD_MEM_HOST 0
#define HDD_MEM_DEVICE 1

/* option flags */
#define HDD_FLAG_NO_MFMA 1        /* Schur updates and fused merges without matrix cores (plain FMA), in
                                     the blocks too: a cross-check of the matrix-core lane layouts */
#define HDD_FLAG_KEEP_DIRICHLET 2 /* plan only: keep outer-boundary nodes in every Gamma */
#define HDD_FLAG_BLOCK8 4         /* eliminate leaf interiors in 8 x 8-cell blocks (default 16 x 16) */
#define HDD_FLAG_NO_GRAPH 16      /* issue every launch eagerly instead of replaying captured HIP graphs */
#define HDD_FLAG_LOWRANK 32       /* block low-rank (H-matrix style, Section 4) copies of the maps P of the
                                     levels with |gamma| >= 255, applied by the refinement sweeps and further
                                     loads; needs refinement (HDD_FP32_REFINE, or max_refine > 0) */
#define HDD_FLAG_KEEP_FRAMES 8    /* keep every node's whole frame (its Schur complement S_omega) after the
                                     build, for hdd_debug_node_schur / hdd_debug_frame.  By default only
                                     the retained factors of every node stay (Section 3.4: the sons' Schur
                                     complements are not needed once the father is built) and frame memory
                                     is reused by every second level */
#define HDD_FLAG_NO_FUSED 64      /* factor every float32 level by separate extend-add, panel and Schur-
                                     update launches (no fused merge of gamma <= 31, no fused elimination
                                     of 33 <= gamma <= 63): a cross-check of the fused kernels */

typedef struct hdd_opts {
  int32_t n;               /* N, interior nodes per side */
  int32_t leaf;            /* leaf size in cells (tree granularity); default 2 * 2^q <= Nc */
  int32_t precision;       /* HDD_FP64 or HDD_FP32_REFINE */
  int32_t fp64_top_levels; /* HDD_FP32_REFINE: levels (from the root) kept in float64; default 2
                              (0 changed neither the sweep count nor the refined error from
                              255^2 to 2047^2, and is about 5% faster at 1023^2) */
  int32_t max_refine;      /* refinement sweeps allowed (HDD_FP32_REFINE default 6; HDD_FP64 default 0) */
  int32_t flags;           /* HDD_FLAG_* */
  double refine_tol;       /* stop once the predicted relative error of the field,
                              c r / (1 - r) with c = max|du| / max|u| of the last
                              sweep and r = c / (c of the sweep before), is
                              <= refine_tol for every sample (so at least two
                              sweeps; r >= 1/2 never stops; default 2e-9) */
  int32_t reserved[8];     /* must be zero */
} hdd_opts;

typedef struct hdd_tree* hdd_handle;

/* Fill *opts with defaults for mesh size n and the given precision. */
int hdd_default_opts(int32_t n, int32_t precision, hdd_opts* opts);

/* Bytes of device workspace a handle for max_samples samples needs. */
int hdd_workspace_size(const hdd_opts* opts, int32_t max_samples, size_t* bytes);

/*
 * Create a handle: plan the tree (Section 2.1) and lay out device memory for
 * up to max_samples parameter samples.
 *   stream     hipStream_t to issue all work on (NULL: a stream the handle owns)
 *   workspace  device buffer of at least hdd_workspace_size() bytes, owned by
 *              the caller and kept alive until hdd_destroy (NULL: the handle
 *              allocates and owns it)
 * Errors: HDD_EINVAL (options), HDD_ENOMEM (workspace too small or
 * allocation failure), HDD_EDEVICE.
 */
int hdd_create(const hdd_opts* opts, int32_t max_samples, void* stream, void* workspace, size_t workspace_bytes,
               hdd_handle* out);

/*
 * hdd_create for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * workspace is a static device array of the library, HDD_STATIC_WORKSPACE_BYTES
 * per GPU (held by every GPU the library runs on until the process ends), so
 * neither this call nor any later call on the handle makes a device,
 * pinned-host or event allocation.  Everything else is as hdd_create: same
 * plan, kernels and results.
 *   stream  hipStream_t for all work (NULL: the null stream)
 * Limits and sharing:
 *  - hdd_workspace_size(opts, max_samples) must be at most
 *    HDD_STATIC_WORKSPACE_BYTES (64 MiB: e.g. 127^2 with 5 samples in float64
 *    or 10 in float32 + refinement, 255^2 with 1 or 2), else HDD_ENOMEM and
 *    nothing is created.
 *  - All static handles of one GPU share its array, so at most one lives per
 *    GPU at a time: HDD_ESTATE while another exists (after hdd_destroy the
 *    next one may be created).  The array keeps the previous handle's
 *    contents; creation clears the part the new handle uses to zero.  Work of
 *    the handle that overlaps other users of the array would race; the
 *    single-owner rule prevents that within the library.
 *  - hdd_timing_enable with a non-zero mask is refused (HDD_EINVAL): timing
 *    events would be allocations.
 * Errors: HDD_EINVAL (options), HDD_ENOMEM (too large), HDD_ESTATE (array in
 * use), HDD_EDEVICE.
 */
#define HDD_STATIC_WORKSPACE_BYTES (64 << 20)
int hdd_create_static(const hdd_opts* opts, int32_t max_samples, void* stream, hdd_handle* out);

/*
 * Leaves to Root for n_samples (<= max_samples) samples: assemble every leaf,
 * eliminate every interface, keep all factors (Section 3.4).
 *   kappa  (mem) float64 [n_samples][Nc][Nc][2]
 *   f      (mem) float64 [N+2][N+2], shared by all samples
 *   g      must be NULL (zero Dirichlet data)
 * Invalidates earlier query results.  Errors: HDD_EINVAL (shape, g != NULL,
 * kappa <= 0 or non-finite: detected on the device and reported by the next
 * synchronizing call), HDD_ENOTSPD (reported by the next synchronizing call),
 * HDD_EDEVICE.
 */
int hdd_build(hdd_handle h, int32_t n_samples, const double* kappa, const double* f, const double* g, int32_t mem);

/*
 * Point values u_h(x) for all built samples (measurement example b,
 * Section 1.2), by P1 interpolation in the triangle that holds x.  Runs Root
 * to Leaves only on the nodes whose interfaces bound the micro-blocks that
 * hold the points (Section 5.3), unless the full field is already solved
 * (always the case in HDD_FP32_REFINE mode, whose refinement needs it).
 *   xy     host float64 [n_pts][2] in [0,1]^2
 *   u_out  (mem) float64 [n_samples][n_pts]
 */
int hdd_query_points(hdd_handle h, int32_t n_pts, const double* xy, double* u_out, int32_t mem);

/*
 * u on the interface gamma_omega of one tree node (eq. gamma_def: the cut
 * that splits omega into its two sons, without the cut's two end points;
 * Section 2.1), for every built sample.  The node is (depth, index) as in
 * hdd_plan_node, 0 <= depth <= the depth of the blocks; (0, 0) is the root,
 * whose gamma is the vertical midline x = 1/2 (setup (a) of Fig. HDDidea).
 *   u_out (mem) float64 [n_samples][|gamma|], entry k at the global node
 *         ids[k] of hdd_plan_node (nodes along the cut, increasing
 *         coordinate); *len (may be NULL) = |gamma|.
 * Without the full field (HDD_FP64 with max_refine = 0, before
 * hdd_solve_full) only the interfaces on the path root -> node are solved
 * (Root to Leaves restricted to that path, Section 5.3).  Errors: HDD_EINVAL
 * (no such node), HDD_ESTATE before a build.
 */
int hdd_query_interface(hdd_handle h, int32_t depth, int32_t index, double* u_out, int32_t* len, int32_t mem);

/*
 * u_h on a coarse mesh made of interfaces (setup (c) of Fig. HDDidea and the
 * remark that HDD gives u_h restricted to a coarser grid with reduced
 * effort; Section 3.5): the fine-mesh solution at every node of the
 * interfaces gamma of all tree nodes of depth < depth (1 <= depth <= the
 * depth of the blocks), i.e. on the grid lines that bound the cells of
 * `depth`.  u_out (mem) float64 [n_samples][*len], nodes in plan order (the
 * root's gamma first, then depth by depth, each node's gamma along its cut;
 * the ids of hdd_plan_node).  Without the full field (HDD_FP64 with
 * max_refine = 0, before hdd_solve_full) Root to Leaves stops above
 * `depth`: no interface below it and no block interior is solved.  Errors:
 * HDD_EINVAL (depth), HDD_ESTATE before a build.
 */
int hdd_query_skeleton(hdd_handle h, int32_t depth, double* u_out, int32_t* len, int32_t mem);

/*
 * Status of every built sample of the batch (host int32 [n_samples]):
 * HDD_EINVAL (its kappa was non-positive or non-finite), HDD_ENOTSPD (an
 * interface factorization of this sample met a non-positive pivot; its
 * values are not usable), HDD_ENOTCONVERGED (its refinement did not reach
 * refine_tol in max_refine sweeps; values still usable), else HDD_OK.
 * Samples are independent: one sample's status never changes another's
 * values.  The calls above return the first non-OK code of the batch.
 * Synchronizes.  Errors: HDD_ESTATE before a build.
 */
int hdd_sample_status(hdd_handle h, int32_t* status);

/*
 * Mean of u over the cell-aligned rectangle rect = {x0, x1, y0, y1} (eq. mean;
 * measurement example a divided by |R|): out (mem) float64 [n_samples].
 * Solves only the subtree nodes that touch the rectangle and their ancestors.
 */
int hdd_query_mean(hdd_handle h, const double rect[4], double* out, int32_t mem);

/*
 * Mean of u over every subdomain of the tree down to the blocks (the example
 * after Lemma Func1, Section 5.1: mean values in all subdomains):
 *   out (mem) float64 [n_samples][n_nodes], n_nodes = hdd_plan_summary()
 *   out[1]; node order root first, then depth by depth, node k of a depth as
 *   in hdd_plan_node(depth, k) (the sons of node k are 2k and 2k+1 of the
 *   next depth).
 * Without the full field (HDD_FP64 with max_refine = 0, before
 * hdd_solve_full) the means come from functional propagation (Lemma Func1;
 * the algorithms of Section 5.2 in factored form): a bottom-up pass builds
 * every node's functional l^g on its boundary and the scalar (l^f, f) from
 * the retained factors, Root to Leaves solves the interfaces above the
 * blocks only, and each mean is (l^f, f) + (l^g, u_Gamma) divided by |omega|;
 * no block interior is solved.  With the full field (always in
 * HDD_FP32_REFINE mode, whose refinement needs it) the means are summed from
 * the field (eq. mean per block, sons into fathers).  Overwrites the
 * forward-pass vectors of the handle.  Errors: HDD_ESTATE before a build.
 */
int hdd_query_node_means(hdd_handle h, double* out, int32_t mem);

/*
 * Log-likelihood of observations y at sites xy for every built sample:
 *   out[s] = -sum_i (y_i - u_s(x_i))^2 / (2 sigma^2)
 *            [- n_y log(sigma sqrt(2 pi)) if normalized]
 * (the likelihood L(z) = prod_i pi_eps(y_i - S_i(z)) of Section 1.2 with
 * Gaussian noise).  xy: host float64 [n_y][2]; y (mem) float64 [n_y];
 * out (mem) float64 [n_samples].
 */
int hdd_loglik(hdd_handle h, int32_t n_y, const double* xy, const double* y, double sigma, int32_t normalized,
               double* out, int32_t mem);

/*
 * Sample-specific observation sites (each sample of the batch has its own
 * points, e.g. independent requests batched together).  Sample s owns points
 * offsets[s] .. offsets[s+1]-1 of xy; offsets: host int32 [n_samples+1] with
 * offsets[0] = 0, non-decreasing, total at most HDD_MAX_QUERY_POINTS.
 * hdd_query_points_ragged: u_out (mem) float64 [offsets[n_samples]], the P1
 *   interpolated values in the order of xy.
 * hdd_loglik_ragged: out (mem) float64 [n_samples], sample s's Gaussian
 *   log-likelihood of its own y (host float64, indexed like xy) with its own
 *   noise level sigma[s] (host float64 [n_samples], > 0), as hdd_loglik.
 * Host arrays are read during the call only.  EINVAL for bad offsets, points
 * outside the unit square or non-positive sigma.
 */
int hdd_query_points_ragged(hdd_handle h, const int32_t* offsets, const double* xy, double* u_out, int32_t mem);
int hdd_loglik_ragged(hdd_handle h, const int32_t* offsets, const double* xy, const double* y, const double* sigma,
                      int32_t normalized, double* out, int32_t mem);

/* Root to Leaves on every node (Section 3.4), plus refinement in
 * HDD_FP32_REFINE mode.  Errors: HDD_ENOTCONVERGED (values still usable). */
int hdd_solve_full(hdd_handle h);

/*
 * The field for another load and Dirichlet data on the built operators: the
 * maps of every node (Phi^f and Phi^g in factored form) are computed once by
 * hdd_build and applied here again (u_h = F_h f_h + G_h g_h, eq.
 * oper_represent2; the advantage for many right-hand sides and Dirichlet data
 * noted after it).  For every built sample, u_h solves the problem of eq.
 * elliptic_det with load f and u = g on the outer boundary:
 *   f  (mem) float64 [N+2][N+2] nodal, shared by all samples (boundary
 *      entries unused)
 *   g  (mem) float64 [N+2][N+2] nodal, only the outer-boundary entries are
 *      read, shared by all samples; NULL: zero Dirichlet data
 * Starting from u = g on the boundary and 0 inside, the lifted load
 * b(f) - A u is eliminated bottom-up (the forward pass), then a full Root to
 * Leaves solves every node; in HDD_FP32_REFINE mode (max_refine > 0) the
 * refinement sweeps follow with the stopping test of refine_tol.  Later
 * queries (points, interface, means, likelihood, hdd_get_solution) read this
 * field until the next hdd_build.  hdd_error_estimate reports the sweeps,
 * the solve sweep included.  Errors: HDD_ESTATE before a build, HDD_EINVAL
 * (non-finite host data), HDD_ENOTCONVERGED (values still usable).
 */
int hdd_solve_rhs(hdd_handle h, const double* f, const double* g, int32_t mem);

/*
 * Two-grid data (Section 3.5, multiple scales): a smooth load given on the
 * mesh of twice the step, H = 2h, and the solution read on that mesh.
 * hdd_solve_rhs_coarse: as hdd_solve_rhs with the fine load taken as the P1
 *   interpolant of f_coarse (mem, float64 [Nc/2+1][Nc/2+1] nodal, both meshes
 *   split along SW-NE diagonals, so a fine node takes the coarse value or the
 *   mean of a coarse edge's two ends); g as in hdd_solve_rhs (fine mesh).
 * hdd_get_solution_coarse: the field of sample `sample` at the nodes of the
 *   coarse mesh, u_out (mem) float64 [Nc/2+1][Nc/2+1] (requires the full
 *   field: after hdd_solve_full, hdd_solve_rhs(_coarse), or any query in
 *   HDD_FP32_REFINE mode; HDD_ESTATE otherwise).
 */
int hdd_solve_rhs_coarse(hdd_handle h, const double* f_coarse, const double* g, int32_t mem);
int hdd_get_solution_coarse(hdd_handle h, int32_t sample, double* u_out, int32_t mem);

/* The nodal field of one sample, u_out (mem) float64 [N+2][N+2]; requires
 * hdd_solve_full. */
int hdd_get_solution(hdd_handle h, int32_t sample, double* u_out, int32_t mem);

/* Last refinement correction max|du| / max|u| per sample (0 if none ran); it
 * bounds the error left after the sweep before it:
 * rel_est host float64 [n_samples]; *sweeps = the most sweeps any sample
 * ran.  Each sample stops refining on its own once its predicted error is
 * below refine_tol (later corrections of the batch are not applied to it). */
int hdd_error_estimate(hdd_handle h, double* rel_est, int32_t* sweeps);

/*
 * Autotuner for the Schur updates (a6): on the kappa and load of the last
 * hdd_build, every float32 matrix-core level's updates are timed with HIP
 * events on the 64 x 64 tile kernel and on the 128 x 128 tile kernel, reps
 * builds each, and each level keeps the faster for later builds (replacing
 * the built-in rule: 128 x 128 for K >= 96 on large frames).  The handle is
 * left built with the chosen tiles.  choices (host int32 [levels], may be
 * NULL): per level 64 or 128, or 0 where the level has no choice (float64
 * levels, fused narrow merges, the blocks).  Errors: HDD_ESTATE before a
 * build, HDD_EINVAL (reps < 1, or a handle from hdd_create_static).
 */
int hdd_autotune(hdd_handle h, int32_t reps, int32_t* choices);

/*
 * Block low-rank maps (HDD_FLAG_LOWRANK; Section 4, the Proposition that the
 * maps of every node admit H-matrix approximations).  After a build, the
 * map P = S_Gamma,gamma L^-T of every level with |gamma| >= 255 is also kept
 * as 64 x 64 blocks (rows in the order of the node's perimeter, columns
 * along the cut): blocks whose boundary and interface segments lie at least
 * their extent apart as factors U V of rank <= 16 (randomized range
 * finder, rank by a relative tolerance of 1e-5 in float32 and 1e-8 in
 * float64, the H-matrix accuracies of the paper's experiments), the others
 * dense.  The refinement sweeps and further loads apply these blocks
 * instead of the dense P; the float64 residual keeps the refined result
 * exact.  out (host float64 [6]), per sample over the compressed levels:
 * bytes of the dense maps, bytes of the block store (64 x 64 per dense
 * block, 2 x 64 x 16 per low-rank block), bytes the chosen ranks need
 * (2 x 64 x rank per low-rank block), blocks stored at low rank, blocks
 * stored dense, mean rank of the low-rank blocks (all 0 without the flag).
 * The dense maps stay in the retained factors (the build's Schur updates
 * write them); the sweeps read only the block store.  Synchronizes.  Errors: HDD_ESTATE before a build.
 */
int hdd_lowrank_info(hdd_handle h, double out[6]);

/*
 * Captured launch sequences: the build, the first full Root to Leaves and
 * each refinement sweep are captured once per sample count as HIP graphs and
 * replayed (unless HDD_FLAG_NO_GRAPH, timing is enabled, or the handle comes
 * from hdd_create_static).  out (host int64 [4]): nodes of the build graph,
 * of the full Root to Leaves graph and of the sweep graph for the current
 * sample count (0 if not captured), and graph launches so far.
 */
int hdd_graph_info(hdd_handle h, int64_t out[4]);

/* Wait for the handle's stream and report deferred device-side errors. */
int hdd_sync(hdd_handle h);

/* Global node index + 1 of the first failing interface factorization, 0 if none. */
int hdd_last_node(hdd_handle h);

int hdd_destroy(hdd_handle h);
const char* hdd_strerror(int code);

/* ---- inspection (tests, benchmark) ---- */

/* Plan summary: out[0] global tree levels (root .. blocks), out[1] global
 * nodes, out[2] depth of the leaves, out[3] depth of the blocks (s x s cells,
 * s = min(16, leaf), whose interior is eliminated in LDS), out[4] per-sample
 * stored factor elements, out[5] algorithmic build flops per sample (sum over
 * every node of the tree down to 2 x 2-cell micro-blocks, outer Dirichlet
 * nodes dropped, of g^3/3 + g^2 G + g G^2).  Host-only; needs no GPU. */
int hdd_plan_summary(const hdd_opts* opts, int64_t out[6]);

/* One node of the global plan (depth <= depth of the blocks): info[0] x0, info[1] y0, info[2] w, info[3] h (cells),
 * info[4] |gamma|, info[5] |Gamma|; ids (may be NULL, else room for
 * |gamma|+|Gamma|) receives global node ids (j*(Nc+1)+i) of [gamma ; Gamma].
 * Host-only; needs no GPU. */
int hdd_plan_node(const hdd_opts* opts, int32_t depth, int32_t index, int32_t info[6], int32_t* ids);

/* Per-level plan: out[0] nodes, out[1] |gamma|, out[2] max U = |gamma|+max|Gamma|,
 * out[3] 1 if the level is float64 in this precision mode.  Host-only. */
int hdd_plan_level(const hdd_opts* opts, int32_t depth, int32_t out[4]);

/* Schur complement data of one built node (handles created with
 * HDD_FLAG_KEEP_FRAMES; HDD_ESTATE otherwise): S (host float64 [|Gamma|+1]^2,
 * row-major, full symmetric, last row/column = condensed load g_omega and
 * its transpose, corner undefined) and ids (host, |Gamma| global node ids).
 * After the build S is the Schur complement S_omega = Psi^g_omega on the
 * node's boundary (Section 2.4).  Synchronizes. */
int hdd_debug_node_schur(hdd_handle h, int32_t sample, int32_t depth, int32_t index, double* S, int32_t* ids);

/* Raw frame of one built node (HDD_FLAG_KEEP_FRAMES; HDD_ESTATE otherwise)
 * (lower triangle, [gamma ; Gamma ; rhs] order,
 * upper triangle returned as zeros): out host float64 [(U+1)^2] with room for
 * the largest frame of the level; *U_out = U.  The first gamma columns are the
 * retained [L ; P ; z] (read from the level's panel store where it has one).
 * Synchronizes. */
int hdd_debug_frame(hdd_handle h, int32_t sample, int32_t depth, int32_t index, double* out, int32_t* U_out);

/* Timing of kernel classes with HIP events around every launch of the class
 * on the handle's stream.  kind: 0 Schur update (rank-k, matrix cores) on
 * float32 levels, 1 interface factorization (diagonal + row solves),
 * 2 extend-add, 3 block build (leaf assembly and in-LDS elimination of the
 * leaf interior), 4 top-down, 5 forward pass, 6 residual, 7 Schur update on
 * float64 levels, 8 the 128 x 128-tile float32 Schur update kernel (launches
 * of kind 8 are not counted in kind 0), 9 fused merge of narrow float32
 * levels (extend-add, factorization and Schur update in one launch),
 * 10 the functional and readout kernels of hdd_query_node_means, 11 the
 * compression of the block low-rank maps, 12 fused elimination of float32
 * levels with 33 <= gamma <= 63 (factorization and Schur update in one
 * launch after the extend-add).
 * hdd_timing_enable(h, mask): bit k enables kind k (0 disables and clears).
 * hdd_timing_get: total milliseconds, number of launches and summed
 * algorithmic flops of the timed launches (Schur update: 2 K per lower-
 * triangle output element; 0 for other kinds).  Synchronizes. */
int hdd_timing_enable(hdd_handle h, int32_t mask);
int hdd_timing_get(hdd_handle h, int32_t kind, double* ms, int64_t* launches, double* flops);
/* Same, restricted to launches on tree level `level` (depth; -1: all), and
 * with the summed algorithmic HBM bytes of the launches in *bytes (Schur
 * update: the panel rows read once plus the output region read and written
 * once; 0 for other kinds).  Any output pointer may be NULL. */
int hdd_timing_get_level(hdd_handle h, int32_t kind, int32_t level, double* ms, int64_t* launches, double* flops,
                         double* bytes);

/* Matrix-core lane-layout self check: dtype 0 (f32 32x32x2) writes 32*32,
 * dtype 1 (f64 16x16x4) writes 16*16 products C = A B^T of fixed integer
 * patterns into out (host).  Needs a GPU. */
int hdd_mfma_selftest(int32_t dtype, double* out);


/* ------------------------------------------------------------------------
 * Likelihood server with continuous batching (the serving loop around the
 * calls above; implementation in serve.hip).
 *
 * One handle, one stream and one worker thread per mesh size.  A request is
 * one parameter sample (kappa of its mesh), its observation sites and
 * optional observations; the answer is the P1 values at the sites and the
 * unnormalized Gaussian log-likelihood (0 without observations).  Requests
 * queue per mesh; a free mesh takes the waiting requests in order, up to
 * its slot count and HDD_MAX_QUERY_POINTS sites in total, as one batch
 * (Leaves to Root, then hdd_query_points_ragged and
 * hdd_loglik_ragged), so requests arriving while others run are admitted as
 * soon as a slot frees up, and batches of different meshes overlap on the
 * GPU.  Every launch sequence of a batch size is captured once and replayed
 * (HIP graphs) when there is no HBM budget.
 * HBM admission: a mesh's device workspace (a full batch) is allocated when
 * its first batch is admitted and counted against hbm_budget bytes (0: no
 * limit).  A batch whose workspace does not fit releases idle meshes'
 * workspaces, least recently used first, or waits until running batches
 * finish (its requests stay queued).  Slots per mesh (default 32) are halved
 * while one mesh's full-batch workspace alone exceeds the budget; ENOMEM at
 * creation if a single sample's does.  With a budget the handles launch
 * eagerly (a workspace release may synchronize the device).
 * ------------------------------------------------------------------------ */
#define HDD_SERVER_MAX_MESHES 8
#define HDD_SERVER_MAX_POINTS 256

typedef struct hdd_server* hdd_server_t;

typedef struct {
  int32_t n_meshes;                      /* 1 .. HDD_SERVER_MAX_MESHES */
  int32_t n[HDD_SERVER_MAX_MESHES];      /* interior nodes per side of each mesh */
  int32_t leaf[HDD_SERVER_MAX_MESHES];   /* leaf size in cells (0: default) */
  int32_t precision;                     /* HDD_FP64 or HDD_FP32_REFINE */
  int32_t slots;                         /* samples per batch per mesh (0: 32) */
  double hbm_budget;                     /* bytes for all device workspaces (0: no limit) */
  int32_t max_refine;                    /* refinement sweeps allowed per batch (0: the default of hdd_default_opts) */
  int32_t reserved[7];                   /* must be zero */
} hdd_server_opts;

/* f: per mesh host float64 [(n+2)^2] nodal right-hand side copied at
 * creation, or NULL (f = 1 on every mesh); an entry may also be NULL. */
int hdd_server_create(const hdd_server_opts* opts, const double* const* f, hdd_server_t* out);
/* Samples per batch (the smallest over the meshes, after the budget). */
int hdd_server_slots(hdd_server_t s, int32_t* slots);
/* HBM admission state, out int64 [4]: bytes of resident workspaces, meshes
 * resident, workspaces released to admit another mesh, workspaces created. */
int hdd_server_memory(hdd_server_t s, int64_t* out);
/* Queue a request on mesh `mesh` (index into opts.n): kappa host float64
 * [n+1][n+1][2] (positive, finite), xy host float64 [n_pts][2] in the unit
 * square (1 <= n_pts <= HDD_SERVER_MAX_POINTS), y host float64 [n_pts] or
 * NULL, sigma > 0.  Inputs are copied; *id identifies the request. */
int hdd_server_submit(hdd_server_t s, int32_t mesh, const double* kappa, int32_t n_pts, const double* xy,
                      const double* y, double sigma, int64_t* id);
/* *done = 1 once the request's batch has finished (non-blocking). */
int hdd_server_poll(hdd_server_t s, int64_t id, int32_t* done);
/* Wait for a request, copy its values (host float64 [n_pts]) and
 * log-likelihood, and release it.  times (host float64 [4], may be NULL):
 * queue wait, batch time, submit-to-done seconds, and the batch size.
 * Returns the request's own status: its sample's code from
 * hdd_sample_status (HDD_ENOTCONVERGED: values and log-likelihood still
 * delivered), or the batch's code when the batch failed as a whole. */
int hdd_server_result(hdd_server_t s, int64_t id, double* values, double* loglik, double* times);
/* out int64 [4]: submitted, completed, batches run, queued now. */
int hdd_server_stats(hdd_server_t s, int64_t* out);
/* Stops the workers after their running batches; queued requests fail with
 * HDD_ESTATE. */
int hdd_server_destroy(hdd_server_t s);
#ifdef __cplusplus
}
#endif
#endif /* HDD_H_ */
