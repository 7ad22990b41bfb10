// C ABI of the HDD library (declarations and documentation in include/hdd.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hdd.h"
#include "kernels.hpp"
#include "plan.hpp"
#include "trace.hpp"

using hdd::DevLevel;
using hdd::DevNode;
using hdd::Plan;

// Workspace of hdd_create_static: one array per GPU that the library runs
// on, held until the process ends.  Host code never uses the name as an
// address (on the host it is only a stand-in): the device address of each
// GPU's copy is resolved once per device with hipGetSymbolAddress and kept
// per device (static_slots below).
static __device__ __align__(256) unsigned char scratch[HDD_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kKinds = 13;
enum Kind {
  K_SYRK = 0, K_FACTOR = 1, K_EXTEND = 2, K_ASSEMBLE = 3, K_TOPDOWN = 4, K_FORWARD = 5, K_RESIDUAL = 6, K_SYRK64 = 7,
  K_SYRK128 = 8, K_MERGE = 9, K_FUNCTIONAL = 10, K_LOWRANK = 11, K_ELIMINATE = 12
};

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }


bool refinement_possible(const hdd_opts& o) { return o.precision == HDD_FP32_REFINE || o.max_refine > 0; }

bool level_double(const hdd_opts& o, int depth) {
  return o.precision == HDD_FP64 || depth < o.fp64_top_levels;
}

int validate_opts(const hdd_opts* o) {
  if (!o) return HDD_EINVAL;
  if (o->precision != HDD_FP64 && o->precision != HDD_FP32_REFINE) return HDD_EINVAL;
  if (o->fp64_top_levels < 0 || o->max_refine < 0 || !(o->refine_tol >= 0.0)) return HDD_EINVAL;
  // the compressed maps are only applied under refinement against the exact operator
  if ((o->flags & HDD_FLAG_LOWRANK) && !(o->precision == HDD_FP32_REFINE || o->max_refine > 0)) return HDD_EINVAL;
  for (int i = 0; i < 8; ++i)
    if (o->reserved[i] != 0) return HDD_EINVAL;
  return HDD_OK;
}

// Levels above the blocks that the fused merge builds (float32 with float32
// sons, gamma <= 31, the node's panel in LDS); they keep their retained
// columns in a dense panel store.
bool merge_level(const Plan& p, const hdd_opts& o, int d) {
  const int D = int(p.levels.size()) - 1;  // the block level
  if (d < 0 || d >= D || (o.flags & (HDD_FLAG_NO_MFMA | HDD_FLAG_NO_FUSED))) return false;
  hdd::DevLevel t{};
  t.gam = p.levels[d].gam;
  t.max_U = p.levels[d].max_U;
  t.is_double = level_double(o, d) ? 1 : 0;
  return hdd::merge_small_ok(t, true) && !level_double(o, d + 1);
}

bool keep_frames(const hdd_opts& o) { return (o.flags & HDD_FLAG_KEEP_FRAMES) != 0; }

// Levels whose maps P get a block low-rank copy: |gamma| >= 255 above the
// blocks, with a boundary (HDD_FLAG_LOWRANK).
constexpr int kLowRankMinGamma = 255;
bool lowrank_level(const Plan& p, const hdd_opts& o, int d) {
  const int D = int(p.levels.size()) - 1;
  return (o.flags & HDD_FLAG_LOWRANK) && d < D && p.levels[d].gam >= kLowRankMinGamma &&
         p.levels[d].max_U > p.levels[d].gam;
}

// Block tables of a low-rank level: per node the boundary positions sorted
// along the node's perimeter (counter-clockwise from its lower-left
// corner), and its 64 x 64 blocks row-major, each dense or low rank by the
// admissibility of its two segments: their bounding boxes (in cells) lie at
// least the larger box edge apart.
struct LowRankTables {
  std::vector<int> perm;      // parallel to the level's ids
  std::vector<int> node;      // first block of every node, n_nodes + 1
  std::vector<int> blk;       // 4 ints per block
  int64_t elems = 0;          // per-sample store elements
  int64_t dense_p = 0;        // per-sample elements of the dense maps P
  int n_lr = 0, n_dense = 0;
};

LowRankTables lowrank_tables(const Plan& p, int d) {
  const auto& lv = p.levels[d];
  const int LB = hdd::kLowRankBlock, KR = hdd::kLowRankMax;
  const int nc = p.nc;
  LowRankTables t;
  t.perm.assign(lv.ids.size(), 0);
  t.node.push_back(0);
  auto coords = [&](int id, int& i, int& j) {
    i = id % (nc + 1);
    j = id / (nc + 1);
  };
  for (size_t k = 0; k < lv.nodes.size(); ++k) {
    const auto& nd = lv.nodes[k];
    const int g = int(nd.gam.size()), G = int(nd.bnd.size());
    // perimeter parameter of a boundary node of the rectangle
    std::vector<std::pair<double, int>> key(G);
    for (int q = 0; q < G; ++q) {
      int i, j;
      coords(nd.bnd[q], i, j);
      double tp;
      if (j == nd.y0) tp = i - nd.x0;
      else if (i == nd.x0 + nd.w) tp = nd.w + (j - nd.y0);
      else if (j == nd.y0 + nd.h) tp = nd.w + nd.h + (nd.x0 + nd.w - i);
      else tp = 2.0 * nd.w + nd.h + (nd.y0 + nd.h - j);
      key[q] = {tp, q};
    }
    std::sort(key.begin(), key.end());
    for (int q = 0; q < G; ++q) t.perm[nd.ids_off + g + q] = key[q].second;
    const int nbr = (G + LB - 1) / LB, nbc = (g + LB - 1) / LB;
    auto box = [&](const int32_t* idv, const int* order, int b0, int n, int bb[4]) {
      bb[0] = bb[2] = 1 << 30;
      bb[1] = bb[3] = -1;
      for (int q = b0; q < b0 + n; ++q) {
        int i, j;
        coords(idv[order ? order[q] : q], i, j);
        bb[0] = std::min(bb[0], i); bb[1] = std::max(bb[1], i);
        bb[2] = std::min(bb[2], j); bb[3] = std::max(bb[3], j);
      }
    };
    std::vector<int> ord(G);
    for (int q = 0; q < G; ++q) ord[q] = key[q].second;
    for (int bi = 0; bi < nbr; ++bi)
      for (int bj = 0; bj < nbc; ++bj) {
        int rb[4], cb[4];
        box(nd.bnd.data(), ord.data(), bi * LB, std::min(LB, G - bi * LB), rb);
        box(nd.gam.data(), nullptr, bj * LB, std::min(LB, g - bj * LB), cb);
        const int dx = std::max(0, std::max(rb[0] - cb[1], cb[0] - rb[1]));
        const int dy = std::max(0, std::max(rb[2] - cb[3], cb[2] - rb[3]));
        const int ext = std::max({rb[1] - rb[0], rb[3] - rb[2], cb[1] - cb[0], cb[3] - cb[2]});
        const bool far = std::max(dx, dy) >= std::max(ext, 1);
        t.blk.push_back(far ? 1 : 0);
        t.blk.push_back(int(t.elems));
        t.blk.push_back(int(k));
        t.blk.push_back((bi << 16) | bj);
        t.elems += far ? 2LL * LB * KR : int64_t(LB) * LB;
        (far ? t.n_lr : t.n_dense) += 1;
      }
    t.node.push_back(int(t.blk.size() / 4));
    t.dense_p += int64_t(g) * G;
  }
  return t;
}

// Row stride of a panel store: gamma rounded up to 4 elements (16-byte rows).
int panel_ld(int g) { return (g + 3) / 4 * 4; }

int64_t panel_elems(const Plan& p, int d) {
  int64_t e = 0;
  for (const auto& nd : p.levels[d].nodes) e += int64_t(nd.U() + 1) * panel_ld(p.levels[d].gam);
  return e;
}

bool make_plan(const hdd_opts& o, Plan& p) {
  hdd::PlanOptions po;
  po.n = o.n;
  po.leaf = o.leaf;
  po.block = (o.flags & HDD_FLAG_BLOCK8) ? 8 : 16;
  po.keep_dirichlet = (o.flags & HDD_FLAG_KEEP_DIRICHLET) != 0;
  return hdd::build_plan(po, p);
}

// Byte offsets of everything the handle keeps in its device workspace.
struct Layout {
  std::vector<int64_t> frames, nodes, maps, ids, vec, panel;
  std::vector<int64_t> lr_perm, lr_node, lr_blk, lr_store, lr_rank;  // low-rank levels (-1 elsewhere)
  int64_t kappa, f, u, d, r, info, bad, act, maxbits, qout, qxy, qy, qsmp, qoff, qsig, lists, iota;
  int64_t cst, bvec, tmaps, tlids, tmicro, origin, text;
  int64_t wts, mu, nmean;  // node means: weight vector, subtree functionals, output staging
  int64_t max_q;
  int64_t total;
};

Layout make_layout(const Plan& p, const hdd_opts& o, int ms) {
  Layout L;
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t at = off;
    off += align256(std::max<int64_t>(bytes, 0));
    return at;
  };
  const int nd = int(p.levels.size());
  L.frames.resize(nd); L.nodes.resize(nd); L.maps.resize(nd); L.ids.resize(nd); L.vec.resize(nd); L.panel.resize(nd);
  L.lr_perm.resize(nd); L.lr_node.resize(nd); L.lr_blk.resize(nd); L.lr_store.resize(nd); L.lr_rank.resize(nd);
  const bool refine = refinement_possible(o);
  const bool keep = keep_frames(o);
  // Frames: by default two buffers, level d in buffer d % 2.  A level's
  // frames are written by its extend-add (or the block build) and read by
  // its own elimination and by the father's extend-add; by the time level
  // d - 2 writes the buffer, level d is consumed.  Every level above the
  // blocks keeps its retained columns [L ; P ; z] in its panel store.
  int64_t pingpong[2] = {-1, -1};
  if (!keep) {
    int64_t need[2] = {0, 0};
    for (int d = 0; d < nd; ++d)
      need[d % 2] = std::max<int64_t>(need[d % 2], p.levels[d].frame_elems * (level_double(o, d) ? 8 : 4) * ms);
    pingpong[0] = take(need[0]);
    pingpong[1] = take(need[1]);
  }
  int64_t total_nodes = 0, max_nodes = 0;
  for (int d = 0; d < nd; ++d) {
    const auto& lv = p.levels[d];
    const int64_t esz = level_double(o, d) ? 8 : 4;
    L.frames[d] = keep ? take(lv.frame_elems * esz * ms) : pingpong[d % 2];
    L.nodes[d] = take(int64_t(lv.nodes.size()) * int64_t(sizeof(DevNode)));
    L.maps[d] = take(int64_t(lv.maps.size()) * 4);
    L.ids[d] = take(int64_t(lv.ids.size()) * 4);
    // forward-pass vectors: refinement, and the functional propagation of the node means
    L.vec[d] = take(int64_t(lv.ids.size()) * 8 * ms);
    const bool store = d < nd - 1 && (!keep || merge_level(p, o, d));
    L.panel[d] = store ? take(panel_elems(p, d) * esz * ms) : -1;
    if (lowrank_level(p, o, d)) {
      const LowRankTables t = lowrank_tables(p, d);
      L.lr_perm[d] = take(int64_t(t.perm.size()) * 4);
      L.lr_node[d] = take(int64_t(t.node.size()) * 4);
      L.lr_blk[d] = take(int64_t(t.blk.size()) * 4);
      L.lr_store[d] = take(t.elems * esz * ms);
      L.lr_rank[d] = take(int64_t(t.blk.size() / 4) * 4 * ms);
    } else {
      L.lr_perm[d] = L.lr_node[d] = L.lr_blk[d] = L.lr_store[d] = L.lr_rank[d] = -1;
    }
    total_nodes += int64_t(lv.nodes.size());
    max_nodes = std::max<int64_t>(max_nodes, int64_t(lv.nodes.size()));
  }
  const int64_t nc = p.nc;
  const int64_t nn = (nc + 1) * (nc + 1);
  L.max_q = std::max<int64_t>(4096, nc);
  L.kappa = take(int64_t(ms) * nc * nc * 2 * 8);
  L.f = take(nn * 8);
  L.u = take(int64_t(ms) * nn * 8);
  // correction and residual fields: refinement, and solves for further loads
  L.d = take(int64_t(ms) * nn * 8);
  L.r = take(int64_t(ms) * nn * 8);
  L.info = take(int64_t(ms) * 4);
  L.bad = take(int64_t(ms) * 4);
  L.act = take(int64_t(ms) * 4);
  L.maxbits = take(int64_t(ms) * 16);
  L.qout = take((int64_t(ms) + 1) * L.max_q * 8);
  L.qxy = take(L.max_q * 16);
  L.qy = take(L.max_q * 8);
  L.qsmp = take(L.max_q * 4);
  L.qoff = take((int64_t(ms) + 1) * 4);
  L.qsig = take(int64_t(ms) * 8);
  L.lists = take(total_nodes * 4);
  L.iota = take(max_nodes * 4);
  const auto& T = p.sub;
  const int64_t nb = int64_t(p.levels.back().nodes.size());
  const int64_t besz = level_double(o, int(p.levels.size()) - 1) ? 8 : 4;
  L.cst = take(int64_t(ms) * nb * T.cst_size * besz);
  L.bvec = take(int64_t(ms) * nb * T.vec_size * 8);
  L.wts = take(nn * 8);
  L.mu = take(int64_t(ms) * total_nodes * 8);
  L.nmean = take(int64_t(ms) * total_nodes * 8);
  L.tmaps = take(int64_t(T.maps.size()) * 4);
  L.tlids = take(int64_t(T.lids.size()) * 4);
  L.tmicro = take(int64_t(T.micro_xy.size()) * 4);
  L.origin = take(nb * 8);
  L.text = take(int64_t(hdd::block_ext_entries(T.s)) * 4);
  L.total = off;
  return L;
}

}  // namespace

struct hdd_tree {
  hdd_opts opt{};
  Plan plan;
  Layout lay;
  hipStream_t st = nullptr;
  bool own_stream = false;
  int device = 0;
  int max_samples = 0, n_samples = 0;
  char* ws = nullptr;
  bool own_ws = false;
  std::vector<DevLevel> lev;
  hdd::DevBlocks blk{};
  std::vector<int64_t> lev_list_off;  // offset (in ints) of each level's node list
  long long nn = 0;
  double *kappa = nullptr, *f = nullptr, *u = nullptr, *d = nullptr, *r = nullptr;
  int *info = nullptr, *bad = nullptr;
  unsigned long long* maxbits = nullptr;
  double *qout = nullptr, *qxy = nullptr, *qy = nullptr, *qsig = nullptr;
  int *qsmp = nullptr, *qoff = nullptr;
  int *lists = nullptr, *iota = nullptr;
  double *wts = nullptr, *mu = nullptr, *nmean = nullptr;
  long long total_nodes = 0;
  bool wts_ready = false;
  int* pinned_lists = nullptr;       // host staging of the node lists (pinned, or lists_host)
  hipEvent_t lists_done = nullptr;   // the last list upload has completed (null: synchronize instead)
  std::vector<int> lists_host;       // pageable staging when the handle may not allocate
  bool no_alloc = false;             // no device, pinned or event allocation after creation
  int static_dev = -1;               // device whose static scratch this handle owns (hdd_create_static)
  bool built = false, full = false;
  std::vector<std::vector<uint8_t>> solved;
  std::vector<double> est;
  int sweeps = 0;                 // most sweeps any sample ran
  std::vector<int> sweeps_s;      // sweeps per sample
  std::vector<int> sstat;         // per-sample refinement status (HDD_OK / HDD_ENOTCONVERGED)
  std::vector<int> act_host;      // samples still refining
  int* act = nullptr;             // device copy of act_host
  // captured launch sequences (HIP graphs), replayed while n_samples and the
  // tile choices are unchanged: the build, the first full Root to Leaves, one
  // refinement sweep
  struct Graph {
    hipGraphExec_t exec = nullptr;
    int64_t nodes = 0;
  };
  using Graphs = std::map<int, Graph>;  // by sample count (a server batch varies it)
  Graphs g_build, g_solve, g_sweep;
  int64_t graph_launches = 0;
  std::vector<int> tile;          // per level: Schur-update tile (0 rule, 64, 128), set by hdd_autotune
  int last_node = 0;
  int deferred = HDD_OK;
  // timing
  int timing_mask = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Rec { int kind, level; hipEvent_t a, b; double flops, bytes; };
  int cur_level = -1;  // level of the launches being recorded
  std::vector<Rec> recs;
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? HDD_OK : HDD_EDEVICE; }

#define HDD_TRY(expr)                      \
  do {                                     \
    const int _st = (expr);                \
    if (_st != HDD_OK) return _st;         \
  } while (0)
#define HIP_TRY(expr) HDD_TRY(hip_status(expr))

hipEvent_t next_event(hdd_tree* h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

// Runs `launch` and, when the kind is being timed, brackets it with events.
template <typename F>
int timed(hdd_tree* h, int kind, double flops, F&& launch, double bytes = 0.0) {
  if (!(h->timing_mask & (1 << kind))) return hip_status(launch());
  hipEvent_t a = next_event(h), b = next_event(h);
  if (!a || !b) return HDD_EDEVICE;
  HIP_TRY(hipEventRecord(a, h->st));
  HIP_TRY(launch());
  HIP_TRY(hipEventRecord(b, h->st));
  h->recs.push_back({kind, h->cur_level, a, b, flops, bytes});
  return HDD_OK;
}

bool graphs_on(const hdd_tree* h) {
  // timing brackets launches with events; a handle that may not allocate
  // does not instantiate graphs; capture needs a stream other than the null one
  return !(h->opt.flags & HDD_FLAG_NO_GRAPH) && h->timing_mask == 0 && !h->no_alloc && h->st != nullptr;
}

void drop_graphs(hdd_tree::Graphs& gs) {
  for (auto& kv : gs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  gs.clear();
}

void drop_graphs(hdd_tree* h) {
  drop_graphs(h->g_build);
  drop_graphs(h->g_solve);
  drop_graphs(h->g_sweep);
}

// Runs `body` (device work on h->st only: kernel launches, no host
// synchronization or host copies) through a captured HIP graph, captured on
// the first call for the current sample count and replayed afterwards; eager
// when graphs are off.
template <typename F>
int run_graph(hdd_tree* h, hdd_tree::Graphs& gs, F&& body) {
  if (!graphs_on(h)) return body();
  auto it = gs.find(h->n_samples);
  if (it == gs.end()) {
    if (gs.size() >= 64) drop_graphs(gs);  // bounded cache
    HIP_TRY(hipStreamBeginCapture(h->st, hipStreamCaptureModeRelaxed));
    const int rc = body();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(h->st, &graph);
    if (rc != HDD_OK || e != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc != HDD_OK ? rc : HDD_EDEVICE;
    }
    size_t n = 0;
    (void)hipGraphGetNodes(graph, nullptr, &n);
    hdd_tree::Graph g;
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return HDD_EDEVICE;
    g.nodes = int64_t(n);
    it = gs.emplace(h->n_samples, g).first;
  }
  ++h->graph_launches;
  return hip_status(hipGraphLaunch(it->second.exec, h->st));
}

// lower-triangle elements (i, j) with r0 <= i <= U, c0 <= j < c1e, j <= i
double lower_count(int r0, int U, int c0, int c1e) {
  double n = 0;
  for (int i = r0; i <= U; ++i) {
    const int hi = std::min(c1e - 1, i);
    if (hi >= c0) n += hi - c0 + 1;
  }
  return n;
}

double syrk_flops(const hdd_tree* h, int d, int k0, int k1, int r0, int c0, int c1) {
  double tot = 0;
  for (const auto& nd : h->plan.levels[d].nodes) {
    const int U = nd.U();
    tot += lower_count(r0, U, c0, c1 < 0 ? U + 1 : c1);
  }
  return tot * 2.0 * (k1 - k0) * h->n_samples;
}

// Algorithmic HBM bytes of the same update: the panel rows it reads once
// (rows min(r0, c0) .. U, columns k0 .. k1) and the output region read and
// written once.
double syrk_bytes(const hdd_tree* h, int d, int k0, int k1, int r0, int c0, int c1) {
  const double esz = h->lev[d].is_double ? 8.0 : 4.0;
  double tot = 0;
  for (const auto& nd : h->plan.levels[d].nodes) {
    const int U = nd.U();
    const int rlo = std::min(r0, c0);
    tot += double(U + 1 - rlo) * (k1 - k0) + 2.0 * lower_count(r0, U, c0, c1 < 0 ? U + 1 : c1);
  }
  return tot * esz * h->n_samples;
}

void reset_refine_state(hdd_tree* h) {
  const int ns = h->n_samples;
  h->sweeps = 0;
  h->est.assign(ns, 0.0);
  h->sweeps_s.assign(ns, 0);
  h->sstat.assign(ns, HDD_OK);
}

int check_deferred(hdd_tree* h) {
  HIP_TRY(hipStreamSynchronize(h->st));
  if (!h->built) return h->deferred;
  std::vector<int> info(h->n_samples), bad(h->n_samples);
  // copies on the handle's stream: no legacy-stream operation that could
  // disturb a capture running on another handle's stream
  HIP_TRY(hipMemcpyAsync(info.data(), h->info, sizeof(int) * h->n_samples, hipMemcpyDeviceToHost, h->st));
  HIP_TRY(hipMemcpyAsync(bad.data(), h->bad, sizeof(int) * h->n_samples, hipMemcpyDeviceToHost, h->st));
  HIP_TRY(hipStreamSynchronize(h->st));
  for (int s = 0; s < h->n_samples; ++s)
    if (bad[s]) return HDD_EINVAL;
  for (int s = 0; s < h->n_samples; ++s)
    if (info[s]) {
      h->last_node = info[s];
      return HDD_ENOTSPD;
    }
  return h->deferred;
}

int run_topdown_level(hdd_tree* h, int d, const int* list_dev, int n_list, double* target, bool from_vec) {
  const DevLevel& L = h->lev[d];
  h->cur_level = d;
  return timed(h, K_TOPDOWN, 0.0, [&] {
    return hdd::launch_topdown(L, list_dev, n_list, h->n_samples, target, h->nn, from_vec, h->st);
  });
}

int run_block_topdown(hdd_tree* h, const int* list_dev, int n_list, double* target, bool from_vec) {
  h->cur_level = int(h->lev.size()) - 1;
  return timed(h, K_TOPDOWN, 0.0, [&] {
    return hdd::launch_block_topdown(h->blk, list_dev, n_list, h->n_samples, h->plan.nc, target, h->nn, from_vec,
                                     h->st);
  });
}

int full_topdown(hdd_tree* h, double* target, bool from_vec) {
  const int DB = int(h->lev.size()) - 1;
  for (int d = 0; d < DB; ++d) HDD_TRY(run_topdown_level(h, d, h->iota, h->lev[d].n_nodes, target, from_vec));
  return run_block_topdown(h, h->iota, h->blk.nb, target, from_vec);
}

// Up to max_it correction sweeps u += d, with d from the bottom-up
// elimination of the residual r = b - A u (forward pass) and a full top-down
// on it, stopped per sample by the predicted-error test below.  With u
// holding only boundary data the first sweep is the solve itself.  A sample
// that has passed the test keeps its field (its later corrections are
// computed but not applied), so its result does not depend on the other
// samples of the batch.  With `test` false the sweeps never report
// non-convergence (a single solve sweep has nothing to compare with).
int correction_sweeps(hdd_tree* h, int max_it, bool test) {
  const int D = int(h->lev.size()) - 1;
  const int nc = h->plan.nc;
  const int ns = h->n_samples;
  std::vector<unsigned long long> mb(2 * ns);
  std::vector<double> prev(ns, 0.0);
  h->act_host.assign(ns, 1);
  int n_active = ns;
  for (int it = 0; it < max_it && n_active > 0; ++it) {
    hdd::Range rg("refinement sweep %d: %d of %d samples", it + 1, n_active, ns);
    // which samples still refine; read by the update at the end of the sweep
    HIP_TRY(hipMemcpyAsync(h->act, h->act_host.data(), sizeof(int) * ns, hipMemcpyHostToDevice, h->st));
    HDD_TRY(run_graph(h, h->g_sweep, [&]() -> int {
      h->cur_level = -1;
      HDD_TRY(timed(h, K_RESIDUAL, 0.0,
                    [&] { return hdd::launch_residual(nc, ns, h->kappa, h->f, h->u, h->r, h->st); }));
      h->cur_level = D;
      HDD_TRY(timed(h, K_FORWARD, 0.0, [&] { return hdd::launch_block_forward(h->blk, ns, nc, h->r, h->nn, h->st); }));
      for (int d = D - 1; d >= 0; --d) {
        h->cur_level = d;
        HDD_TRY(timed(h, K_FORWARD, 0.0, [&] { return hdd::launch_forward(h->lev[d], h->lev[d + 1], ns, h->st); }));
      }
      HIP_TRY(hdd::launch_fill(h->d, (long long)ns * h->nn, 0.0, h->st));
      HDD_TRY(full_topdown(h, h->d, true));
      // all-zero bits are +0.0: the fill kernel clears the max-norm words
      HIP_TRY(hdd::launch_fill(reinterpret_cast<double*>(h->maxbits), 2LL * ns, 0.0, h->st));
      return hip_status(hdd::launch_axpy_maxabs(nc, ns, h->u, h->d, h->maxbits, h->act, h->st));
    }));
    HIP_TRY(hipMemcpyAsync(mb.data(), h->maxbits, sizeof(unsigned long long) * 2 * ns, hipMemcpyDeviceToHost, h->st));
    HIP_TRY(hipStreamSynchronize(h->st));
    h->sweeps = it + 1;
    // Stopping test on the predicted error of the refined field: for a
    // linearly convergent correction sequence with contraction r the error
    // left after a correction of size c is at most c r / (1 - r); r is the
    // observed ratio of the last two corrections.  A sample whose ratio is
    // not below 1/2 (or that has only one correction) does not stop.
    for (int s = 0; s < ns; ++s) {
      if (!h->act_host[s]) continue;
      double md, mu;
      std::memcpy(&md, &mb[2 * s], 8);
      std::memcpy(&mu, &mb[2 * s + 1], 8);
      const double c = mu > 0 ? md / mu : md;
      double pred = std::numeric_limits<double>::infinity();
      if (c == 0.0) {
        pred = 0.0;
      } else if (it > 0 && prev[s] > 0.0) {
        const double r = c / prev[s];
        if (r < 0.5) pred = c * r / (1.0 - r);
      }
      h->est[s] = c;
      h->sweeps_s[s] = it + 1;
      prev[s] = c;
      if (pred <= h->opt.refine_tol) {
        h->act_host[s] = 0;
        --n_active;
      }
    }
  }
  if (test)
    for (int s = 0; s < ns; ++s)
      if (h->act_host[s]) {
        h->sstat[s] = HDD_ENOTCONVERGED;
        h->deferred = HDD_ENOTCONVERGED;
      }
  return HDD_OK;
}

int ensure_full(hdd_tree* h) {
  if (h->full) return HDD_OK;
  hdd::Range rg("full Root to Leaves");
  HDD_TRY(run_graph(h, h->g_solve, [&] { return full_topdown(h, h->u, false); }));
  for (auto& v : h->solved) std::fill(v.begin(), v.end(), 1);
  h->full = true;
  reset_refine_state(h);
  if (h->opt.max_refine <= 0) return HDD_OK;
  return correction_sweeps(h, h->opt.max_refine, true);
}

// Solve, root first, the nodes marked in `need` that are not solved yet.
int partial_topdown(hdd_tree* h, const std::vector<std::vector<uint8_t>>& need) {
  hdd::Range rg("partial Root to Leaves");
  if (h->lists_done) HIP_TRY(hipEventSynchronize(h->lists_done));
  else HIP_TRY(hipStreamSynchronize(h->st));
  int64_t total = 0;
  std::vector<int> counts(h->lev.size(), 0);
  for (size_t d = 0; d < h->lev.size(); ++d) {
    int* dst = h->pinned_lists + h->lev_list_off[d];
    int c = 0;
    for (size_t k = 0; k < need[d].size(); ++k)
      if (need[d][k] && !h->solved[d][k]) dst[c++] = int(k);
    counts[d] = c;
    total += c;
  }
  if (total == 0) return HDD_OK;
  HIP_TRY(hipMemcpyAsync(h->lists, h->pinned_lists, sizeof(int) * (h->lev_list_off.back() + h->lev.back().n_nodes),
                         hipMemcpyHostToDevice, h->st));
  if (h->lists_done) HIP_TRY(hipEventRecord(h->lists_done, h->st));
  const size_t DB = h->lev.size() - 1;
  for (size_t d = 0; d < h->lev.size(); ++d) {
    if (!counts[d]) continue;
    if (d < DB)
      HDD_TRY(run_topdown_level(h, int(d), h->lists + h->lev_list_off[d], counts[d], h->u, false));
    else
      HDD_TRY(run_block_topdown(h, h->lists + h->lev_list_off[d], counts[d], h->u, false));
    for (size_t k = 0; k < need[d].size(); ++k)
      if (need[d][k]) h->solved[d][k] = 1;
  }
  return HDD_OK;
}

// Mark the path root -> block holding cell (ci, cj).
void mark_cell_path(const hdd_tree* h, int ci, int cj, std::vector<std::vector<uint8_t>>& need) {
  int k = 0;
  for (size_t d = 0; d < h->plan.levels.size(); ++d) {
    const auto& nd = h->plan.levels[d].nodes[k];
    need[d][k] = 1;
    if (nd.block) break;
    int s;
    if (nd.vertical) s = ci >= nd.x0 + nd.w / 2 ? 1 : 0;
    else s = cj >= nd.y0 + nd.h / 2 ? 1 : 0;
    k = 2 * k + s;
  }
}

std::vector<std::vector<uint8_t>> empty_need(const hdd_tree* h) {
  std::vector<std::vector<uint8_t>> need(h->lev.size());
  for (size_t d = 0; d < h->lev.size(); ++d) need[d].assign(h->lev[d].n_nodes, 0);
  return need;
}

int prepare_values(hdd_tree* h, const std::vector<std::vector<uint8_t>>& need) {
  if (h->full) return HDD_OK;
  if (h->opt.max_refine > 0) return ensure_full(h);
  return partial_topdown(h, need);
}

hipMemcpyKind copy_kind(int mem) { return mem == HDD_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice; }

// The full field for the load already in h->f and Dirichlet data g (nodal,
// outer-boundary entries read; nullptr = zero): u = g on the boundary and 0
// inside, then the correction sweeps, the first of which is the solve.  g is
// staged in the residual field, which the first sweep overwrites.
int solve_loaded_rhs(hdd_tree* h, const double* g, int mem) {
  if (g) HIP_TRY(hipMemcpyAsync(h->r, g, size_t(h->nn) * 8, copy_kind(mem), h->st));
  HIP_TRY(hdd::launch_lift_init(h->plan.nc, h->n_samples, g ? h->r : nullptr, h->u, h->st));
  for (auto& v : h->solved) std::fill(v.begin(), v.end(), 1);
  h->full = true;
  reset_refine_state(h);
  const int refine = std::max(0, h->opt.max_refine);
  HDD_TRY(correction_sweeps(h, 1 + refine, refine > 0));
  return check_deferred(h);
}

int copy_out(hdd_tree* h, double* dst, const double* src_dev, size_t n, int mem) {
  if (mem == HDD_MEM_DEVICE) return hip_status(hipMemcpyAsync(dst, src_dev, n * 8, hipMemcpyDeviceToDevice, h->st));
  HIP_TRY(hipMemcpyAsync(dst, src_dev, n * 8, hipMemcpyDeviceToHost, h->st));
  return check_deferred(h);
}

}  // namespace

extern "C" {

int hdd_default_opts(int32_t n, int32_t precision, hdd_opts* o) {
  if (!o || n < 1) return HDD_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->n = n;
  const int nc = n + 1;
  int leaf = 32;
  while (leaf > 2 && (nc % leaf != 0 || leaf > nc)) leaf >>= 1;
  o->leaf = leaf;
  o->precision = precision;
  o->fp64_top_levels = 2;
  o->max_refine = precision == HDD_FP32_REFINE ? 6 : 0;
  o->refine_tol = 2e-9;
  return validate_opts(o);
}

int hdd_workspace_size(const hdd_opts* o, int32_t max_samples, size_t* bytes) {
  HDD_TRY(validate_opts(o));
  if (max_samples < 1 || !bytes) return HDD_EINVAL;
  Plan p;
  if (!make_plan(*o, p)) return HDD_EINVAL;
  *bytes = size_t(make_layout(p, *o, max_samples).total);
  return HDD_OK;
}

}  // extern "C"

namespace {

// hdd_create; with no_alloc the handle takes a caller workspace and a stream
// (null: the null stream) and makes no device, pinned-host or event
// allocation, now or later (node lists are staged in pageable memory).
int create_impl(const hdd_opts* o, int32_t max_samples, void* stream, void* workspace, size_t workspace_bytes,
                bool no_alloc, hdd_handle* out) {
  HDD_TRY(validate_opts(o));
  if (no_alloc && !workspace) return HDD_EINVAL;
  if (max_samples < 1 || !out) return HDD_EINVAL;
  hdd_tree* h = new (std::nothrow) hdd_tree();
  if (!h) return HDD_ENOMEM;
  h->opt = *o;
  if (!make_plan(*o, h->plan)) {
    delete h;
    return HDD_EINVAL;
  }
  h->max_samples = max_samples;
  h->lay = make_layout(h->plan, *o, max_samples);
  auto fail = [&](int code) {
    hdd_destroy(h);
    return code;
  };
  if (hipGetDevice(&h->device) != hipSuccess) return fail(HDD_EDEVICE);
  h->no_alloc = no_alloc;
  if (stream || no_alloc) {
    h->st = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking) != hipSuccess) return fail(HDD_EDEVICE);
    h->own_stream = true;
  }
  if (workspace) {
    if (workspace_bytes < size_t(h->lay.total)) return fail(HDD_ENOMEM);
    h->ws = static_cast<char*>(workspace);
  } else {
    if (hipMalloc(&h->ws, size_t(h->lay.total)) != hipSuccess) {
      h->ws = nullptr;
      return fail(HDD_ENOMEM);
    }
    h->own_ws = true;
  }
  if (no_alloc) {
    // a reused workspace keeps the previous handle's contents: start from zeros
    if (hdd::launch_fill(reinterpret_cast<double*>(h->ws), h->lay.total / 8, 0.0, h->st) != hipSuccess ||
        hipStreamSynchronize(h->st) != hipSuccess)
      return fail(HDD_EDEVICE);
  }
  // host tables to the device on the handle's stream (the source vectors are
  // live until the copy has completed)
  auto upload = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->st);
    return e != hipSuccess ? e : hipStreamSynchronize(h->st);
  };
  const Layout& L = h->lay;
  const int nd = int(h->plan.levels.size());
  h->lev.resize(nd);
  h->lev_list_off.resize(nd);
  h->solved.resize(nd);
  int64_t list_off = 0, node_base = 0;
  for (int d = 0; d < nd; ++d) {
    const auto& pl = h->plan.levels[d];
    std::vector<DevNode> dn(pl.nodes.size());
    int64_t poff = 0;
    for (size_t k = 0; k < pl.nodes.size(); ++k) {
      const auto& p = pl.nodes[k];
      dn[k].panel_off = poff;
      poff += int64_t(p.U() + 1) * panel_ld(pl.gam);
      dn[k].frame_off = p.frame_off;
      dn[k].map_off = p.map_off;
      dn[k].U = p.U();
      dn[k].bnd = int(p.bnd.size());
      dn[k].ld = p.ld;
      dn[k].ids_off = int(p.ids_off);
      dn[k].x0 = p.x0;
      dn[k].y0 = p.y0;
      dn[k].cw = p.w;
      dn[k].ch = p.h;
    }
    DevLevel& lv = h->lev[d];
    lv.frames = h->ws + L.frames[d];
    lv.stride = pl.frame_elems;
    lv.panel = L.panel[d] >= 0 ? h->ws + L.panel[d] : nullptr;
    lv.panel_stride = L.panel[d] >= 0 ? panel_elems(h->plan, d) : 0;
    lv.panel_ld = panel_ld(pl.gam);
    if (L.lr_store[d] >= 0) {
      const LowRankTables t = lowrank_tables(h->plan, d);
      lv.lr_perm = reinterpret_cast<const int*>(h->ws + L.lr_perm[d]);
      lv.lr_node = reinterpret_cast<const int*>(h->ws + L.lr_node[d]);
      lv.lr_blk = reinterpret_cast<const int4*>(h->ws + L.lr_blk[d]);
      lv.lr_store = h->ws + L.lr_store[d];
      lv.lr_stride = t.elems;
      lv.lr_rank = reinterpret_cast<int*>(h->ws + L.lr_rank[d]);
      lv.lr_nblk = int(t.blk.size() / 4);
      if (upload(h->ws + L.lr_perm[d], t.perm.data(), t.perm.size() * 4) != hipSuccess ||
          upload(h->ws + L.lr_node[d], t.node.data(), t.node.size() * 4) != hipSuccess ||
          upload(h->ws + L.lr_blk[d], t.blk.data(), t.blk.size() * 4) != hipSuccess)
        return fail(HDD_EDEVICE);
    }
    lv.nodes = reinterpret_cast<const DevNode*>(h->ws + L.nodes[d]);
    lv.maps = reinterpret_cast<const int*>(h->ws + L.maps[d]);
    lv.ids = reinterpret_cast<const int*>(h->ws + L.ids[d]);
    lv.vec = L.vec[d] >= 0 ? reinterpret_cast<double*>(h->ws + L.vec[d]) : nullptr;
    lv.vec_stride = (long long)pl.ids.size();
    lv.n_nodes = int(pl.nodes.size());
    lv.gam = pl.gam;
    lv.max_U = pl.max_U;
    lv.is_double = level_double(*o, d) ? 1 : 0;
    lv.depth = d;
    lv.node_base = int(node_base);
    node_base += lv.n_nodes;
    if (upload(h->ws + L.nodes[d], dn.data(), dn.size() * sizeof(DevNode)) != hipSuccess ||
        upload(h->ws + L.maps[d], pl.maps.data(), pl.maps.size() * 4) != hipSuccess ||
        upload(h->ws + L.ids[d], pl.ids.data(), pl.ids.size() * 4) != hipSuccess)
      return fail(HDD_EDEVICE);
    h->lev_list_off[d] = list_off;
    list_off += lv.n_nodes;
    h->solved[d].assign(lv.n_nodes, 0);
  }
  {
    const auto& T = h->plan.sub;
    if (int(T.lv.size()) > hdd::kMaxSubLevels) return fail(HDD_EINVAL);
    hdd::DevBlocks& B = h->blk;
    B.nlev = int(T.lv.size());
    for (int k = 0; k < B.nlev; ++k) {
      const auto& sl = T.lv[k];
      B.lv[k] = hdd::DevSubLevel{sl.n, sl.gam, sl.bnd, sl.U, sl.fsz, sl.cst_off, sl.vec_off, sl.map_off, sl.lid_off};
    }
    B.s = T.s;
    B.nb = h->lev.back().n_nodes;
    B.cst_size = T.cst_size;
    B.vec_size = T.vec_size;
    B.max_buf = T.max_buf;
    B.max_gam_nodes = T.max_gam_nodes;
    B.max_bnd_nodes = T.max_bnd_nodes;
    B.no_mfma = (o->flags & HDD_FLAG_NO_MFMA) ? 1 : 0;
    B.maps = reinterpret_cast<const int*>(h->ws + L.tmaps);
    B.lids = reinterpret_cast<const int*>(h->ws + L.tlids);
    B.micro_xy = reinterpret_cast<const int*>(h->ws + L.tmicro);
    B.ext = reinterpret_cast<const unsigned*>(h->ws + L.text);
    B.origin = reinterpret_cast<const int*>(h->ws + L.origin);
    B.cst = h->ws + L.cst;
    B.cst_stride = (long long)B.nb * T.cst_size;
    B.vec = L.bvec >= 0 ? reinterpret_cast<double*>(h->ws + L.bvec) : nullptr;
    B.vec_stride = (long long)B.nb * T.vec_size;
    B.top = h->lev.back();
    std::vector<int> org;
    for (const auto& nd : h->plan.levels.back().nodes) {
      org.push_back(nd.x0);
      org.push_back(nd.y0);
    }
    if (upload(h->ws + L.tmaps, T.maps.data(), T.maps.size() * 4) != hipSuccess ||
        upload(h->ws + L.tlids, T.lids.data(), T.lids.size() * 4) != hipSuccess ||
        upload(h->ws + L.tmicro, T.micro_xy.data(), T.micro_xy.size() * 4) != hipSuccess ||
        upload(h->ws + L.origin, org.data(), org.size() * 4) != hipSuccess)
      return fail(HDD_EDEVICE);
    const bool bdbl = B.top.is_double != 0;
    if (!hdd::block_shape_ok(B)) return fail(HDD_EINVAL);
    if (hdd::launch_block_ext(B, const_cast<unsigned*>(B.ext), h->st) != hipSuccess ||
        hipStreamSynchronize(h->st) != hipSuccess)
      return fail(HDD_EDEVICE);
    // the build stages the block's coefficients and load in its second frame buffer
    if (size_t(2 * B.s * B.s + (B.s + 1) * (B.s + 1)) * 8 > size_t(B.max_buf) * (bdbl ? 8 : 4))
      return fail(HDD_EINVAL);
    if (hdd::block_build_lds(B, bdbl) > 160 * 1024 || hdd::block_topdown_lds(B, bdbl) > 160 * 1024 ||
        hdd::block_forward_lds(B, bdbl) > 160 * 1024)
      return fail(HDD_EINVAL);
  }
  // panel stores: the entries above the diagonal of L are never written by a
  // build and must read as zero
  for (int d = 0; d < nd; ++d)
    if (L.panel[d] >= 0) {
      const int64_t bytes = panel_elems(h->plan, d) * (h->lev[d].is_double ? 8 : 4) * max_samples;
      if (hdd::launch_fill(reinterpret_cast<double*>(h->ws + L.panel[d]), (bytes + 7) / 8, 0.0, h->st) !=
          hipSuccess)
        return fail(HDD_EDEVICE);
    }
  if (hipStreamSynchronize(h->st) != hipSuccess) return fail(HDD_EDEVICE);
  h->nn = (long long)(h->plan.nc + 1) * (h->plan.nc + 1);
  h->kappa = reinterpret_cast<double*>(h->ws + L.kappa);
  h->f = reinterpret_cast<double*>(h->ws + L.f);
  h->u = reinterpret_cast<double*>(h->ws + L.u);
  h->d = L.d >= 0 ? reinterpret_cast<double*>(h->ws + L.d) : nullptr;
  h->r = L.r >= 0 ? reinterpret_cast<double*>(h->ws + L.r) : nullptr;
  h->info = reinterpret_cast<int*>(h->ws + L.info);
  h->bad = reinterpret_cast<int*>(h->ws + L.bad);
  h->act = reinterpret_cast<int*>(h->ws + L.act);
  h->maxbits = reinterpret_cast<unsigned long long*>(h->ws + L.maxbits);
  h->qout = reinterpret_cast<double*>(h->ws + L.qout);
  h->qxy = reinterpret_cast<double*>(h->ws + L.qxy);
  h->qy = reinterpret_cast<double*>(h->ws + L.qy);
  h->qsmp = reinterpret_cast<int*>(h->ws + L.qsmp);
  h->qoff = reinterpret_cast<int*>(h->ws + L.qoff);
  h->qsig = reinterpret_cast<double*>(h->ws + L.qsig);
  h->lists = reinterpret_cast<int*>(h->ws + L.lists);
  h->iota = reinterpret_cast<int*>(h->ws + L.iota);
  h->wts = reinterpret_cast<double*>(h->ws + L.wts);
  h->mu = reinterpret_cast<double*>(h->ws + L.mu);
  h->nmean = reinterpret_cast<double*>(h->ws + L.nmean);
  h->total_nodes = 0;
  for (auto& lv : h->lev) h->total_nodes += lv.n_nodes;
  if (no_alloc) {
    h->lists_host.assign(size_t(std::max<int64_t>(list_off, 1)), 0);
    h->pinned_lists = h->lists_host.data();
  } else if (hipHostMalloc(&h->pinned_lists, sizeof(int) * size_t(std::max<int64_t>(list_off, 1))) != hipSuccess) {
    h->pinned_lists = nullptr;
    return fail(HDD_ENOMEM);
  }
  {
    int64_t mx = 0;
    for (auto& lv : h->lev) mx = std::max<int64_t>(mx, lv.n_nodes);
    std::vector<int> io(mx);
    for (int64_t k = 0; k < mx; ++k) io[k] = int(k);
    if (upload(h->iota, io.data(), io.size() * 4) != hipSuccess) return fail(HDD_EDEVICE);
  }
  if (!no_alloc) {
    if (hipEventCreateWithFlags(&h->lists_done, hipEventDisableTiming) != hipSuccess) {
      h->lists_done = nullptr;
      return fail(HDD_EDEVICE);
    }
    if (hipEventRecord(h->lists_done, h->st) != hipSuccess) return fail(HDD_EDEVICE);
  }
  *out = h;
  return HDD_OK;
}

constexpr int kMaxStaticDevices = 64;
struct StaticSlot {
  void* ptr = nullptr;       // device address of this GPU's scratch
  bool resolved = false;
  hdd_tree* owner = nullptr; // the live static handle on this GPU, if any
};
std::mutex static_mu;
StaticSlot static_slots[kMaxStaticDevices];

}  // namespace

namespace hdd {
int create_handle(const hdd_opts* o, int32_t max_samples, void* stream, void* workspace, size_t workspace_bytes,
                  bool no_alloc, hdd_handle* out) {
  return create_impl(o, max_samples, stream, workspace, workspace_bytes, no_alloc, out);
}
}  // namespace hdd

extern "C" {

int hdd_create(const hdd_opts* o, int32_t max_samples, void* stream, void* workspace, size_t workspace_bytes,
               hdd_handle* out) {
  return create_impl(o, max_samples, stream, workspace, workspace_bytes, false, out);
}

int hdd_create_static(const hdd_opts* o, int32_t max_samples, void* stream, hdd_handle* out) {
  HDD_TRY(validate_opts(o));
  if (max_samples < 1 || !out) return HDD_EINVAL;
  size_t need = 0;
  HDD_TRY(hdd_workspace_size(o, max_samples, &need));
  if (need > size_t(HDD_STATIC_WORKSPACE_BYTES)) return HDD_ENOMEM;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxStaticDevices) return HDD_EDEVICE;
  std::lock_guard<std::mutex> lock(static_mu);
  StaticSlot& slot = static_slots[dev];
  if (!slot.resolved) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HDD_EDEVICE;
    slot.ptr = p;
    slot.resolved = true;
  }
  if (slot.owner) return HDD_ESTATE;
  hdd_handle h = nullptr;
  HDD_TRY(create_impl(o, max_samples, stream, slot.ptr, size_t(HDD_STATIC_WORKSPACE_BYTES), true, &h));
  h->static_dev = dev;
  slot.owner = h;
  *out = h;
  return HDD_OK;
}

}  // extern "C"

namespace {

// The device part of Leaves to Root for h->n_samples samples whose kappa and
// load are in the workspace: kernel launches on h->st only (captured as one
// HIP graph by run_graph).
int build_device(hdd_tree* h) {
  const int n_samples = h->n_samples;
  const int nc = h->plan.nc;
  HIP_TRY(hdd::launch_fill_i32(h->info, n_samples, 0, h->st));
  HIP_TRY(hdd::launch_fill_i32(h->bad, n_samples, 0, h->st));
  const int D = int(h->lev.size()) - 1;
  const bool mfma = !(h->opt.flags & HDD_FLAG_NO_MFMA);
  auto eliminate = [&](int d) -> int {
    h->cur_level = d;
    const DevLevel& L = h->lev[d];
    const int g = L.gam;
    const int syrk_kind = L.is_double ? K_SYRK64 : K_SYRK;
    const int tile_final = h->tile.empty() ? 0 : h->tile[d];
    // interfaces of 33..63 nodes: factorization and Schur update in one launch
    if (!(h->opt.flags & HDD_FLAG_NO_FUSED) && hdd::eliminate_mid_ok(L, mfma))
      return timed(h, K_ELIMINATE, 0.0, [&] { return hdd::launch_eliminate_mid(L, n_samples, h->info, h->st); });
    // Rank-K update C[r0.., c0..c1) -= F[.., k0..k1) F[.., k0..k1)^T, timed;
    // the autotuned tile applies to the Schur update of Gamma, the trailing
    // updates inside the interface follow the built-in rule.
    auto syrk = [&](int k0, int k1, int r0, int c1) -> int {
      const int tile = c1 < 0 ? tile_final : 0;
      const double fl = h->timing_mask ? syrk_flops(h, d, k0, k1, r0, r0, c1) : 0.0;
      const double by = h->timing_mask ? syrk_bytes(h, d, k0, k1, r0, r0, c1) : 0.0;
      const int kind = hdd::syrk_uses_big_tile(L, k0, k1, r0, r0, c1, mfma, tile) ? K_SYRK128 : syrk_kind;
      return timed(
          h, kind, fl, [&] { return hdd::launch_syrk(L, k0, k1, r0, r0, c1, n_samples, mfma, tile, h->st); }, by);
    };
    // Recursive blocked partial Cholesky of the first g columns: the
    // columns [c0, c1) are halved (at a multiple of kPanelNB), the left half
    // is factored, the right half takes its update from the left half in one
    // rank-K launch, then the right half is factored; kPanelNB-column panels
    // at the bottom.  Every column is rewritten once per halving, with the
    // widest K available for each update.
    std::function<int(int, int)> factor_range = [&](int c0, int c1) -> int {
      if (c1 - c0 <= hdd::kPanelNB)
        return timed(h, K_FACTOR, 0.0, [&] { return hdd::launch_panel(L, c0, c1 - c0, n_samples, h->info, h->st); });
      const int half = ((c1 - c0) / 2 + hdd::kPanelNB - 1) / hdd::kPanelNB * hdd::kPanelNB;
      const int mid = c0 + half;
      HDD_TRY(factor_range(c0, mid));
      HDD_TRY(syrk(c0, mid, mid, c1));
      return factor_range(mid, c1);
    };
    HDD_TRY(factor_range(0, g));
    if (L.max_U > g) HDD_TRY(syrk(0, g, g, -1));  // Schur update of Gamma (and the boundary load row)
    return HDD_OK;
  };
  h->cur_level = D;
  hdd::Range rg("Leaves to Root: blocks");
  HDD_TRY(timed(h, K_ASSEMBLE, 0.0, [&] {
    return hdd::launch_block_build(h->blk, n_samples, nc, h->kappa, h->f, h->bad, h->info, h->st);
  }));
  for (int d = D - 1; d >= 0; --d) {
    h->cur_level = d;
    hdd::Range rg("Leaves to Root depth %d", d);
    if (merge_level(h->plan, h->opt, d)) {
      HDD_TRY(timed(h, K_MERGE, 0.0, [&] {
        return hdd::launch_merge_small(h->lev[d], h->lev[d + 1], n_samples, h->info, h->st);
      }));
      continue;
    }
    HDD_TRY(timed(h, K_EXTEND, 0.0, [&] { return hdd::launch_extend_add(h->lev[d], h->lev[d + 1], n_samples, h->st); }));
    HDD_TRY(eliminate(d));
  }
  // block low-rank copies of the wide levels' maps P (refinement sweeps)
  for (int d = 0; d < D; ++d)
    if (h->lev[d].lr_store) {
      h->cur_level = d;
      // relative accuracy of the blocks: 1e-5 in float32, 1e-8 in float64
      const double tol = h->lev[d].is_double ? 1e-8 : 1e-5;
      HDD_TRY(timed(h, K_LOWRANK, 0.0, [&] { return hdd::launch_lr_compress(h->lev[d], n_samples, tol, h->st); }));
    }
  return hip_status(hdd::launch_fill(h->u, (long long)n_samples * h->nn, 0.0, h->st));
}

// Leaves to Root on the kappa and load already in the workspace.
int build_resident(hdd_tree* h, int n_samples) {
  hdd::Range rg("hdd_build n=%d samples=%d", h->opt.n, n_samples);
  h->n_samples = n_samples;
  h->built = false;
  h->full = false;
  h->deferred = HDD_OK;
  h->last_node = 0;
  reset_refine_state(h);
  for (auto& v : h->solved) std::fill(v.begin(), v.end(), 0);
  HDD_TRY(run_graph(h, h->g_build, [&] { return build_device(h); }));
  h->built = true;
  return HDD_OK;
}

}  // namespace

extern "C" {

int hdd_build(hdd_handle h, int32_t n_samples, const double* kappa, const double* f, const double* g, int32_t mem) {
  if (!h || !kappa || !f || g != nullptr || n_samples < 1 || n_samples > h->max_samples) return HDD_EINVAL;
  if (mem != HDD_MEM_HOST && mem != HDD_MEM_DEVICE) return HDD_EINVAL;
  const int nc = h->plan.nc;
  const size_t kbytes = size_t(n_samples) * nc * nc * 2 * 8;
  const size_t fbytes = size_t(h->nn) * 8;
  if (mem == HDD_MEM_HOST) {
    for (size_t i = 0; i < kbytes / 8; ++i)
      if (!(kappa[i] > 0.0) || !std::isfinite(kappa[i])) return HDD_EINVAL;
    HIP_TRY(hipMemcpyAsync(h->kappa, kappa, kbytes, hipMemcpyHostToDevice, h->st));
    HIP_TRY(hipMemcpyAsync(h->f, f, fbytes, hipMemcpyHostToDevice, h->st));
  } else {
    HIP_TRY(hipMemcpyAsync(h->kappa, kappa, kbytes, hipMemcpyDeviceToDevice, h->st));
    HIP_TRY(hipMemcpyAsync(h->f, f, fbytes, hipMemcpyDeviceToDevice, h->st));
  }
  return build_resident(h, n_samples);
}

int hdd_autotune(hdd_handle h, int32_t reps, int32_t* choices) {
  if (!h || reps < 1) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  if (h->no_alloc) return HDD_EINVAL;  // timing events would be allocations
  hdd::Range rg("hdd_autotune");
  const int nd = int(h->lev.size());
  const int ns = h->n_samples;
  const int saved_mask = h->timing_mask;
  // per level: event time of its Schur update of Gamma on the 64 x 64 tile,
  // then on the 128 x 128 tile (the trailing updates inside the interface
  // keep the built-in rule and are timed under another kind)
  std::vector<double> ms[2];
  const int cand[2] = {64, 128};
  for (int c = 0; c < 2; ++c) {
    ms[c].assign(nd, 0.0);
    h->tile.assign(nd, cand[c]);
    for (int r = 0; r < reps; ++r) {
      HDD_TRY(hdd_timing_enable(h, (1 << K_SYRK) | (1 << K_SYRK64) | (1 << K_SYRK128)));
      HDD_TRY(build_resident(h, ns));
      for (int d = 0; d < nd; ++d)
        for (int k : {K_SYRK, K_SYRK128}) {
          double t = 0.0;
          HDD_TRY(hdd_timing_get_level(h, k, d, &t, nullptr, nullptr, nullptr));
          ms[c][d] += t;
        }
    }
  }
  std::vector<int> pick(nd, 0);
  for (int d = 0; d < nd; ++d) {
    const bool choice = !h->lev[d].is_double && !merge_level(h->plan, h->opt, d) && d < nd - 1 &&
                        h->lev[d].max_U > 0 && !(h->opt.flags & HDD_FLAG_NO_MFMA);
    if (choice && ms[0][d] + ms[1][d] > 0.0) pick[d] = ms[1][d] < ms[0][d] ? 128 : 64;
    if (choices) choices[d] = pick[d];
  }
  h->tile = pick;
  HDD_TRY(hdd_timing_enable(h, saved_mask));
  drop_graphs(h);
  return build_resident(h, ns);  // the handle is left built with the chosen tiles
}

int hdd_lowrank_info(hdd_handle h, double out[6]) {
  if (!h || !out) return HDD_EINVAL;
  for (int q = 0; q < 6; ++q) out[q] = 0.0;
  if (!h->built) return HDD_ESTATE;
  const int LB = hdd::kLowRankBlock, KR = hdd::kLowRankMax;
  const int ns = h->n_samples;
  double rank_sum = 0.0, used = 0.0, lr_count = 0.0;
  for (size_t d = 0; d < h->lev.size(); ++d) {
    const DevLevel& L = h->lev[d];
    if (!L.lr_store) continue;
    const LowRankTables t = lowrank_tables(h->plan, int(d));
    const double esz = L.is_double ? 8.0 : 4.0;
    std::vector<int> rk(size_t(L.lr_nblk) * ns);
    HIP_TRY(hipMemcpyAsync(rk.data(), L.lr_rank, rk.size() * 4, hipMemcpyDeviceToHost, h->st));
    HIP_TRY(hipStreamSynchronize(h->st));
    out[0] += double(t.dense_p) * esz;
    out[1] += double(t.elems) * esz;
    for (int s = 0; s < ns; ++s)
      for (int b = 0; b < L.lr_nblk; ++b) {
        const int r = t.blk[4 * b] == 1 ? rk[size_t(s) * L.lr_nblk + b] : -1;  // -1: dense
        used += (r >= 0 ? 2.0 * LB * r : double(LB) * LB) * esz / ns;
        if (r >= 0) rank_sum += r, lr_count += 1;
      }
    out[4] += t.n_dense + t.n_lr;
  }
  out[2] = used;
  out[3] = lr_count / ns;   // blocks stored at low rank (per sample)
  out[4] -= out[3];         // blocks stored dense
  out[5] = lr_count > 0 ? rank_sum / lr_count : 0.0;
  (void)KR;
  return HDD_OK;
}

int hdd_graph_info(hdd_handle h, int64_t out[4]) {
  if (!h || !out) return HDD_EINVAL;
  auto nodes = [&](const hdd_tree::Graphs& gs) -> int64_t {
    auto it = gs.find(h->n_samples);
    return it == gs.end() ? 0 : it->second.nodes;
  };
  out[0] = nodes(h->g_build);
  out[1] = nodes(h->g_solve);
  out[2] = nodes(h->g_sweep);
  out[3] = h->graph_launches;
  return HDD_OK;
}

int hdd_query_points(hdd_handle h, int32_t n_pts, const double* xy, double* u_out, int32_t mem) {
  if (!h || n_pts < 1 || !xy || !u_out || n_pts > h->lay.max_q) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  const int nc = h->plan.nc;
  auto need = empty_need(h);
  for (int p = 0; p < n_pts; ++p) {
    const double x = xy[2 * p], y = xy[2 * p + 1];
    if (!(x >= 0.0 && x <= 1.0 && y >= 0.0 && y <= 1.0)) return HDD_EINVAL;
    const int ci = std::min(int(std::floor(x * nc)), nc - 1), cj = std::min(int(std::floor(y * nc)), nc - 1);
    mark_cell_path(h, ci, cj, need);
  }
  HDD_TRY(prepare_values(h, need));
  HIP_TRY(hipMemcpyAsync(h->qxy, xy, size_t(n_pts) * 16, hipMemcpyHostToDevice, h->st));
  double* dst = mem == HDD_MEM_DEVICE ? u_out : h->qout;
  HIP_TRY(hdd::launch_points(nc, h->n_samples, n_pts, h->qxy, h->u, dst, h->st));
  if (mem == HDD_MEM_DEVICE) return HDD_OK;
  return copy_out(h, u_out, h->qout, size_t(n_pts) * h->n_samples, HDD_MEM_HOST);
}

// Marks the paths to every point of a ragged set, uploads the points and
// their sample index, and interpolates into dst (device).
static int ragged_points(hdd_tree* h, const int32_t* off, const double* xy, double* dst) {
  const int ns = h->n_samples;
  if (!off || !xy || off[0] != 0) return HDD_EINVAL;
  for (int s = 0; s < ns; ++s)
    if (off[s + 1] < off[s]) return HDD_EINVAL;
  const int n_total = off[ns];
  if (n_total < 1 || n_total > h->lay.max_q) return HDD_EINVAL;
  const int nc = h->plan.nc;
  auto need = empty_need(h);
  std::vector<int> smp(n_total);
  for (int s = 0; s < ns; ++s)
    for (int p = off[s]; p < off[s + 1]; ++p) {
      const double x = xy[2 * p], y = xy[2 * p + 1];
      if (!(x >= 0.0 && x <= 1.0 && y >= 0.0 && y <= 1.0)) return HDD_EINVAL;
      const int ci = std::min(int(std::floor(x * nc)), nc - 1), cj = std::min(int(std::floor(y * nc)), nc - 1);
      mark_cell_path(h, ci, cj, need);
      smp[p] = s;
    }
  HDD_TRY(prepare_values(h, need));
  HIP_TRY(hipMemcpyAsync(h->qxy, xy, size_t(n_total) * 16, hipMemcpyHostToDevice, h->st));
  HIP_TRY(hipMemcpyAsync(h->qsmp, smp.data(), size_t(n_total) * 4, hipMemcpyHostToDevice, h->st));
  HIP_TRY(hdd::launch_points_ragged(nc, n_total, h->qxy, h->qsmp, h->u, dst, h->st));
  // the pageable sources above must stay valid until the copies complete
  HIP_TRY(hipStreamSynchronize(h->st));
  return HDD_OK;
}

int hdd_query_points_ragged(hdd_handle h, const int32_t* offsets, const double* xy, double* u_out, int32_t mem) {
  if (!h || !u_out) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  double* dst = mem == HDD_MEM_DEVICE ? u_out : h->qout;
  HDD_TRY(ragged_points(h, offsets, xy, dst));
  if (mem == HDD_MEM_DEVICE) return HDD_OK;
  return copy_out(h, u_out, h->qout, size_t(offsets[h->n_samples]), HDD_MEM_HOST);
}

int hdd_loglik_ragged(hdd_handle h, const int32_t* offsets, const double* xy, const double* y, const double* sigma,
                      int32_t normalized, double* out, int32_t mem) {
  if (!h || !y || !sigma || !out || !offsets) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  const int ns = h->n_samples;
  for (int s = 0; s < ns; ++s)
    if (!(sigma[s] > 0.0)) return HDD_EINVAL;
  HDD_TRY(ragged_points(h, offsets, xy, h->qout));
  const int n_total = offsets[ns];
  HIP_TRY(hipMemcpyAsync(h->qy, y, size_t(n_total) * 8, hipMemcpyHostToDevice, h->st));
  HIP_TRY(hipMemcpyAsync(h->qoff, offsets, size_t(ns + 1) * 4, hipMemcpyHostToDevice, h->st));
  HIP_TRY(hipMemcpyAsync(h->qsig, sigma, size_t(ns) * 8, hipMemcpyHostToDevice, h->st));
  double* dst = mem == HDD_MEM_DEVICE ? out : h->qout + n_total;
  HIP_TRY(hdd::launch_loglik_ragged(ns, h->qoff, h->qout, h->qy, h->qsig, normalized, dst, h->st));
  if (mem == HDD_MEM_DEVICE) return hip_status(hipStreamSynchronize(h->st));  // host sources stay valid until here
  return copy_out(h, out, dst, size_t(ns), HDD_MEM_HOST);
}

int hdd_query_interface(hdd_handle h, int32_t depth, int32_t index, double* u_out, int32_t* len, int32_t mem) {
  if (!h || !u_out || (mem != HDD_MEM_HOST && mem != HDD_MEM_DEVICE)) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  if (depth < 0 || depth >= int(h->lev.size()) || index < 0 || index >= h->lev[depth].n_nodes) return HDD_EINVAL;
  const auto& nd = h->plan.levels[depth].nodes[index];
  // the path root -> node: the node's gamma is solved once its ancestors'
  // interfaces (its boundary data) are known
  auto need = empty_need(h);
  int k = index;
  for (int d = depth; d >= 0; --d, k >>= 1) need[d][k] = 1;
  HDD_TRY(prepare_values(h, need));
  const int g = int(nd.gam.size());
  if (len) *len = g;
  double* dst = mem == HDD_MEM_DEVICE ? u_out : h->qout;
  const int* ids = h->lev[depth].ids + nd.ids_off;  // [gamma ; Gamma] global ids, gamma first
  HIP_TRY(hdd::launch_gather(g, h->n_samples, ids, h->u, h->nn, dst, h->st));
  if (mem == HDD_MEM_DEVICE) return HDD_OK;
  return copy_out(h, u_out, h->qout, size_t(g) * h->n_samples, HDD_MEM_HOST);
}

int hdd_query_skeleton(hdd_handle h, int32_t depth, double* u_out, int32_t* len, int32_t mem) {
  if (!h || !u_out || (mem != HDD_MEM_HOST && mem != HDD_MEM_DEVICE)) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  hdd::Range rg("hdd_query_skeleton depth=%d", depth);
  const int D = int(h->lev.size()) - 1;
  if (depth < 1 || depth > D) return HDD_EINVAL;
  // every interface above `depth`; without the full field only these are
  // solved (Root to Leaves stops at the coarse cells)
  auto need = empty_need(h);
  std::vector<int> ids;
  for (int d = 0; d < depth; ++d) {
    std::fill(need[d].begin(), need[d].end(), 1);
    for (const auto& nd : h->plan.levels[d].nodes) ids.insert(ids.end(), nd.gam.begin(), nd.gam.end());
  }
  HDD_TRY(prepare_values(h, need));
  const int n = int(ids.size());
  if (len) *len = n;
  // the id list is staged in the residual field (free outside the sweeps)
  int* ids_dev = reinterpret_cast<int*>(h->r);
  HIP_TRY(hipMemcpyAsync(ids_dev, ids.data(), size_t(n) * 4, hipMemcpyHostToDevice, h->st));
  double* dst = u_out;
  if (mem == HDD_MEM_HOST) {
    if (size_t(n) * h->n_samples > size_t(h->nn) * h->n_samples) return HDD_EINVAL;
    dst = h->d;  // staging (the correction field is free outside the sweeps)
  }
  HIP_TRY(hdd::launch_gather(n, h->n_samples, ids_dev, h->u, h->nn, dst, h->st));
  if (mem == HDD_MEM_DEVICE) return hip_status(hipStreamSynchronize(h->st));  // the host id list stays valid until here
  return copy_out(h, u_out, h->d, size_t(n) * h->n_samples, HDD_MEM_HOST);
}

int hdd_sample_status(hdd_handle h, int32_t* status) {
  if (!h || !status) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  HIP_TRY(hipStreamSynchronize(h->st));
  const int ns = h->n_samples;
  std::vector<int> info(ns), bad(ns);
  HIP_TRY(hipMemcpyAsync(info.data(), h->info, sizeof(int) * ns, hipMemcpyDeviceToHost, h->st));
  HIP_TRY(hipMemcpyAsync(bad.data(), h->bad, sizeof(int) * ns, hipMemcpyDeviceToHost, h->st));
  HIP_TRY(hipStreamSynchronize(h->st));
  for (int s = 0; s < ns; ++s)
    status[s] = bad[s] ? HDD_EINVAL : info[s] ? HDD_ENOTSPD : h->sstat.empty() ? HDD_OK : h->sstat[s];
  return HDD_OK;
}

int hdd_query_mean(hdd_handle h, const double rect[4], double* out, int32_t mem) {
  if (!h || !rect || !out) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  const int nc = h->plan.nc;
  int b[4];
  for (int q = 0; q < 4; ++q) {
    const double v = rect[q] * nc;
    b[q] = int(std::lround(v));
    if (!(rect[q] >= 0.0 && rect[q] <= 1.0) || std::fabs(v - b[q]) > 1e-9) return HDD_EINVAL;
  }
  if (b[1] <= b[0] || b[3] <= b[2]) return HDD_EINVAL;
  auto need = empty_need(h);
  const int m = h->plan.sub.s;
  for (int cj = b[2]; cj < b[3]; ++cj)
    for (int ci = b[0]; ci < b[1]; ++ci)
      if (ci % m == 0 || ci == b[0])
        if (cj % m == 0 || cj == b[2]) mark_cell_path(h, ci, cj, need);
  HDD_TRY(prepare_values(h, need));
  double* dst = mem == HDD_MEM_DEVICE ? out : h->qout;
  HIP_TRY(hdd::launch_mean(nc, h->n_samples, b[0], b[1], b[2], b[3], h->u, dst, h->st));
  if (mem == HDD_MEM_DEVICE) return HDD_OK;
  return copy_out(h, out, h->qout, size_t(h->n_samples), HDD_MEM_HOST);
}

int hdd_query_node_means(hdd_handle h, double* out, int32_t mem) {
  if (!h || !out || (mem != HDD_MEM_HOST && mem != HDD_MEM_DEVICE)) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  hdd::Range rg("hdd_query_node_means");
  if (!h->full && h->opt.max_refine > 0) HDD_TRY(ensure_full(h));
  const int ns = h->n_samples, nc = h->plan.nc;
  const int D = int(h->lev.size()) - 1;
  const long long tn = h->total_nodes;
  double* dst = mem == HDD_MEM_DEVICE ? out : h->nmean;
  if (h->full) {
    // the field is known: eq. mean per block, then every father sums its sons
    h->cur_level = D;
    HDD_TRY(timed(h, K_FUNCTIONAL, 0.0, [&] {
      return hdd::launch_block_integral(h->lev[D], ns, nc, h->u, h->nn, h->mu, tn, dst, tn, h->st);
    }));
    for (int d = D - 1; d >= 0; --d) {
      h->cur_level = d;
      HDD_TRY(timed(h, K_FUNCTIONAL, 0.0, [&] {
        return hdd::launch_level_sum(h->lev[d], h->lev[d + 1], ns, nc, h->mu, tn, dst, tn, h->st);
      }));
    }
  } else {
    // Lemma Func1 bottom-up: the functional of every node from the nodal
    // weight vector h^2 (shared by all samples), then mu of every subtree
    if (!h->wts_ready) {
      const double hc = 1.0 / nc;
      HIP_TRY(hdd::launch_fill(h->wts, h->nn, hc * hc, h->st));
      h->wts_ready = true;
    }
    h->cur_level = D;
    HDD_TRY(timed(h, K_FORWARD, 0.0, [&] { return hdd::launch_block_forward(h->blk, ns, nc, h->wts, 0, h->st); }));
    for (int d = D - 1; d >= 0; --d) {
      h->cur_level = d;
      HDD_TRY(timed(h, K_FORWARD, 0.0, [&] { return hdd::launch_forward(h->lev[d], h->lev[d + 1], ns, h->st); }));
    }
    h->cur_level = D;
    HDD_TRY(timed(h, K_FUNCTIONAL, 0.0, [&] { return hdd::launch_block_mu(h->blk, ns, h->mu, tn, h->st); }));
    for (int d = D - 1; d >= 0; --d) {
      h->cur_level = d;
      HDD_TRY(timed(h, K_FUNCTIONAL, 0.0, [&] {
        return hdd::launch_level_mu(h->lev[d], h->lev[d + 1], ns, h->mu, tn, h->st);
      }));
    }
    // Root to Leaves on the interfaces above the blocks only: every node's
    // boundary is then known, and no block interior is solved
    auto need = empty_need(h);
    for (int d = 0; d < D; ++d) std::fill(need[d].begin(), need[d].end(), 1);
    HDD_TRY(partial_topdown(h, need));
    for (int d = 0; d <= D; ++d) {
      h->cur_level = d;
      HDD_TRY(timed(h, K_FUNCTIONAL, 0.0, [&] {
        return hdd::launch_node_means(h->lev[d], ns, nc, h->u, h->nn, h->mu, tn, dst, tn, h->st);
      }));
    }
  }
  if (mem == HDD_MEM_DEVICE) return HDD_OK;
  return copy_out(h, out, h->nmean, size_t(ns) * size_t(tn), HDD_MEM_HOST);
}

int hdd_loglik(hdd_handle h, int32_t n_y, const double* xy, const double* y, double sigma, int32_t normalized,
               double* out, int32_t mem) {
  if (!h || n_y < 1 || !xy || !y || !out || !(sigma > 0.0) || n_y >= h->lay.max_q) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  HDD_TRY(hdd_query_points(h, n_y, xy, h->qout, HDD_MEM_DEVICE));
  const double* ydev = y;
  if (mem == HDD_MEM_HOST) {
    HIP_TRY(hipMemcpyAsync(h->qy, y, size_t(n_y) * 8, hipMemcpyHostToDevice, h->st));
    ydev = h->qy;
  }
  double* dst = mem == HDD_MEM_DEVICE ? out : h->qout + size_t(n_y) * h->n_samples;
  HIP_TRY(hdd::launch_loglik(h->n_samples, n_y, h->qout, ydev, sigma, normalized, dst, h->st));
  if (mem == HDD_MEM_DEVICE) return HDD_OK;
  return copy_out(h, out, dst, size_t(h->n_samples), HDD_MEM_HOST);
}

int hdd_solve_full(hdd_handle h) {
  if (!h) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  HDD_TRY(ensure_full(h));
  return check_deferred(h);
}

int hdd_solve_rhs(hdd_handle h, const double* f, const double* g, int32_t mem) {
  if (!h || !f || (mem != HDD_MEM_HOST && mem != HDD_MEM_DEVICE)) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  hdd::Range rg("hdd_solve_rhs");
  const size_t fbytes = size_t(h->nn) * 8;
  if (mem == HDD_MEM_HOST) {
    for (long long i = 0; i < h->nn; ++i)
      if (!std::isfinite(f[i]) || (g && !std::isfinite(g[i]))) return HDD_EINVAL;
  }
  // the new load replaces the build's (the residual reads it)
  HIP_TRY(hipMemcpyAsync(h->f, f, fbytes, copy_kind(mem), h->st));
  return solve_loaded_rhs(h, g, mem);
}

int hdd_solve_rhs_coarse(hdd_handle h, const double* f_coarse, const double* g, int32_t mem) {
  if (!h || !f_coarse || (mem != HDD_MEM_HOST && mem != HDD_MEM_DEVICE)) return HDD_EINVAL;
  if (!h->built) return HDD_ESTATE;
  hdd::Range rg("hdd_solve_rhs_coarse");
  const long long m1 = h->plan.nc / 2 + 1;
  if (mem == HDD_MEM_HOST) {
    for (long long i = 0; i < m1 * m1; ++i)
      if (!std::isfinite(f_coarse[i])) return HDD_EINVAL;
    if (g)
      for (long long i = 0; i < h->nn; ++i)
        if (!std::isfinite(g[i])) return HDD_EINVAL;
  }
  // coarse values staged in the correction field, prolonged into the load
  HIP_TRY(hipMemcpyAsync(h->d, f_coarse, size_t(m1 * m1) * 8, copy_kind(mem), h->st));
  HIP_TRY(hdd::launch_prolong(h->plan.nc, h->d, h->f, h->st));
  return solve_loaded_rhs(h, g, mem);
}

int hdd_get_solution_coarse(hdd_handle h, int32_t sample, double* u_out, int32_t mem) {
  if (!h || !u_out || sample < 0 || sample >= h->n_samples || (mem != HDD_MEM_HOST && mem != HDD_MEM_DEVICE))
    return HDD_EINVAL;
  if (!h->built || !h->full) return HDD_ESTATE;
  const long long m1 = h->plan.nc / 2 + 1;
  double* dst = mem == HDD_MEM_DEVICE ? u_out : h->d;
  HIP_TRY(hdd::launch_inject(h->plan.nc, h->u + (long long)sample * h->nn, dst, h->st));
  if (mem == HDD_MEM_DEVICE) return HDD_OK;
  return copy_out(h, u_out, h->d, size_t(m1 * m1), HDD_MEM_HOST);
}

int hdd_get_solution(hdd_handle h, int32_t sample, double* u_out, int32_t mem) {
  if (!h || !u_out || sample < 0 || sample >= h->n_samples) return HDD_EINVAL;
  if (!h->built || !h->full) return HDD_ESTATE;
  return copy_out(h, u_out, h->u + (long long)sample * h->nn, size_t(h->nn), mem);
}

int hdd_error_estimate(hdd_handle h, double* rel_est, int32_t* sweeps) {
  if (!h || !rel_est) return HDD_EINVAL;
  for (int s = 0; s < h->n_samples; ++s) rel_est[s] = h->est.empty() ? 0.0 : h->est[s];
  if (sweeps) *sweeps = h->sweeps;
  return HDD_OK;
}

int hdd_sync(hdd_handle h) {
  if (!h) return HDD_EINVAL;
  return check_deferred(h);
}

int hdd_last_node(hdd_handle h) { return h ? h->last_node : 0; }

int hdd_destroy(hdd_handle h) {
  if (!h) return HDD_OK;
  if (h->st) (void)hipStreamSynchronize(h->st);
  drop_graphs(h);
  for (auto e : h->ev_pool) (void)hipEventDestroy(e);
  if (h->lists_done) (void)hipEventDestroy(h->lists_done);
  if (h->pinned_lists && !h->no_alloc) (void)hipHostFree(h->pinned_lists);
  if (h->own_ws && h->ws) (void)hipFree(h->ws);
  if (h->own_stream && h->st) (void)hipStreamDestroy(h->st);
  if (h->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(static_mu);
    if (static_slots[h->static_dev].owner == h) static_slots[h->static_dev].owner = nullptr;
  }
  delete h;
  return HDD_OK;
}

const char* hdd_strerror(int code) {
  switch (code) {
    case HDD_OK: return "ok";
    case HDD_EINVAL: return "invalid argument";
    case HDD_ENOMEM: return "out of device memory / workspace too small";
    case HDD_ENOTSPD: return "interface block not positive definite";
    case HDD_ENOTCONVERGED: return "iterative refinement did not converge";
    case HDD_EDEVICE: return "HIP runtime error";
    case HDD_ESTATE: return "call out of order";
    default: return "unknown error";
  }
}

int hdd_plan_summary(const hdd_opts* o, int64_t out[6]) {
  HDD_TRY(validate_opts(o));
  if (!out) return HDD_EINVAL;
  Plan p;
  if (!make_plan(*o, p)) return HDD_EINVAL;
  int64_t nodes = 0, elems = 0;
  for (const auto& L : p.levels) {
    nodes += int64_t(L.nodes.size());
    elems += L.frame_elems;
  }
  elems += int64_t(p.levels.back().nodes.size()) * p.sub.cst_size;
  out[0] = int64_t(p.levels.size());
  out[1] = nodes;
  out[2] = p.depth_leaf;
  out[3] = p.depth_block;
  out[4] = elems;
  out[5] = int64_t(hdd::algorithmic_flops(o->n));
  return HDD_OK;
}

int hdd_plan_node(const hdd_opts* o, int32_t depth, int32_t index, int32_t info[6], int32_t* ids) {
  HDD_TRY(validate_opts(o));
  if (!info) return HDD_EINVAL;
  Plan p;
  if (!make_plan(*o, p)) return HDD_EINVAL;
  if (depth < 0 || depth >= int(p.levels.size())) return HDD_EINVAL;
  const auto& L = p.levels[depth];
  if (index < 0 || index >= int(L.nodes.size())) return HDD_EINVAL;
  const auto& nd = L.nodes[index];
  info[0] = nd.x0; info[1] = nd.y0; info[2] = nd.w; info[3] = nd.h;
  info[4] = int(nd.gam.size()); info[5] = int(nd.bnd.size());
  if (ids) {
    std::copy(nd.gam.begin(), nd.gam.end(), ids);
    std::copy(nd.bnd.begin(), nd.bnd.end(), ids + nd.gam.size());
  }
  return HDD_OK;
}

int hdd_plan_level(const hdd_opts* o, int32_t depth, int32_t out[4]) {
  HDD_TRY(validate_opts(o));
  if (!out) return HDD_EINVAL;
  Plan p;
  if (!make_plan(*o, p)) return HDD_EINVAL;
  if (depth < 0 || depth >= int(p.levels.size())) return HDD_EINVAL;
  const auto& L = p.levels[depth];
  out[0] = int(L.nodes.size());
  out[1] = L.gam;
  out[2] = L.max_U;
  out[3] = level_double(*o, depth) ? 1 : 0;
  return HDD_OK;
}

int hdd_debug_node_schur(hdd_handle h, int32_t sample, int32_t depth, int32_t index, double* S, int32_t* ids) {
  if (!h || !S || !ids) return HDD_EINVAL;
  if (!h->built || !keep_frames(h->opt)) return HDD_ESTATE;
  if (sample < 0 || sample >= h->n_samples || depth < 0 || depth >= int(h->lev.size())) return HDD_EINVAL;
  const auto& pl = h->plan.levels[depth];
  if (index < 0 || index >= int(pl.nodes.size())) return HDD_EINVAL;
  HIP_TRY(hipStreamSynchronize(h->st));  // read back even after a failed pivot (diagnostics)
  const auto& nd = pl.nodes[index];
  const int U = nd.U(), g = int(nd.gam.size()), G = int(nd.bnd.size()), ld = nd.ld;
  const bool dbl = h->lev[depth].is_double != 0;
  const size_t esz = dbl ? 8 : 4;
  std::vector<char> buf(size_t(U + 1) * ld * esz);
  const char* src = static_cast<const char*>(h->lev[depth].frames) +
                    (size_t(sample) * h->lev[depth].stride + size_t(nd.frame_off)) * esz;
  HIP_TRY(hipMemcpy(buf.data(), src, buf.size(), hipMemcpyDeviceToHost));
  auto at = [&](int r, int c) -> double {
    if (r < c) std::swap(r, c);
    const size_t k = size_t(r) * ld + c;
    return dbl ? reinterpret_cast<const double*>(buf.data())[k] : double(reinterpret_cast<const float*>(buf.data())[k]);
  };
  for (int a = 0; a <= G; ++a)
    for (int b = 0; b <= G; ++b) S[size_t(a) * (G + 1) + b] = at(g + a, g + b);
  std::copy(nd.bnd.begin(), nd.bnd.end(), ids);
  (void)U;
  return HDD_OK;
}

int hdd_debug_frame(hdd_handle h, int32_t sample, int32_t depth, int32_t index, double* out, int32_t* U_out) {
  if (!h || !out || !U_out) return HDD_EINVAL;
  if (!h->built || !keep_frames(h->opt)) return HDD_ESTATE;
  if (sample < 0 || sample >= h->n_samples || depth < 0 || depth >= int(h->lev.size())) return HDD_EINVAL;
  const auto& pl = h->plan.levels[depth];
  if (index < 0 || index >= int(pl.nodes.size())) return HDD_EINVAL;
  HIP_TRY(hipStreamSynchronize(h->st));
  const auto& nd = pl.nodes[index];
  const int n = nd.U() + 1, ld = nd.ld;
  const bool dbl = h->lev[depth].is_double != 0;
  const size_t esz = dbl ? 8 : 4;
  std::vector<char> buf(size_t(n) * ld * esz);
  const char* src = static_cast<const char*>(h->lev[depth].frames) +
                    (size_t(sample) * h->lev[depth].stride + size_t(nd.frame_off)) * esz;
  HIP_TRY(hipMemcpy(buf.data(), src, buf.size(), hipMemcpyDeviceToHost));
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      const size_t k = size_t(r) * ld + c;
      out[size_t(r) * n + c] = (c <= r) ? (dbl ? reinterpret_cast<const double*>(buf.data())[k]
                                                  : double(reinterpret_cast<const float*>(buf.data())[k]))
                                          : 0.0;
    }
  if (h->lev[depth].panel) {  // retained columns kept in the level's panel store
    const int g = pl.gam, pld = panel_ld(g);
    int64_t poff = 0;
    for (int k = 0; k < index; ++k) poff += int64_t(pl.nodes[k].U() + 1) * pld;
    std::vector<char> pan(size_t(n) * pld * esz);
    const char* psrc = static_cast<const char*>(h->lev[depth].panel) +
                       (size_t(sample) * h->lev[depth].panel_stride + size_t(poff)) * esz;
    HIP_TRY(hipMemcpy(pan.data(), psrc, pan.size(), hipMemcpyDeviceToHost));
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < g && c <= r; ++c) {
        const size_t k = size_t(r) * pld + c;
        out[size_t(r) * n + c] = dbl ? reinterpret_cast<const double*>(pan.data())[k]
                                     : double(reinterpret_cast<const float*>(pan.data())[k]);
      }
  }
  *U_out = n - 1;
  return HDD_OK;
}

int hdd_timing_enable(hdd_handle h, int32_t mask) {
  if (!h || (h->no_alloc && mask != 0)) return HDD_EINVAL;  // timing events would be allocations
  HIP_TRY(hipStreamSynchronize(h->st));
  h->timing_mask = mask;
  h->recs.clear();
  h->ev_used = 0;
  return HDD_OK;
}

int hdd_timing_get(hdd_handle h, int32_t kind, double* ms, int64_t* launches, double* flops) {
  return hdd_timing_get_level(h, kind, -1, ms, launches, flops, nullptr);
}

int hdd_timing_get_level(hdd_handle h, int32_t kind, int32_t level, double* ms, int64_t* launches, double* flops,
                         double* bytes) {
  if (!h || kind < 0 || kind >= kKinds) return HDD_EINVAL;
  HIP_TRY(hipStreamSynchronize(h->st));
  double tot = 0, fl = 0, by = 0;
  int64_t n = 0;
  for (const auto& r : h->recs) {
    if (r.kind != kind || (level >= 0 && r.level != level)) continue;
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
    tot += t;
    fl += r.flops;
    by += r.bytes;
    ++n;
  }
  if (ms) *ms = tot;
  if (launches) *launches = n;
  if (flops) *flops = fl;
  if (bytes) *bytes = by;
  return HDD_OK;
}

int hdd_mfma_selftest(int32_t dtype, double* out) {
  if (!out || (dtype != 0 && dtype != 1)) return HDD_EINVAL;
  const size_t n = dtype == 0 ? 32 * 32 : 16 * 16;
  double* dev = nullptr;
  HIP_TRY(hipMalloc(&dev, n * 8));
  hipError_t e = hdd::launch_mfma_selftest(dtype, dev, nullptr);
  if (e == hipSuccess) e = hipMemcpy(out, dev, n * 8, hipMemcpyDeviceToHost);
  (void)hipFree(dev);
  return hip_status(e);
}

}  // extern "C"
