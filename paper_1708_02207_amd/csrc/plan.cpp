// Host-side HDD tree plan (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <unordered_map>

namespace hdd {
namespace {

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Leading dimension of a frame with U+1 rows: small frames are packed, large
// ones padded to 8 elements so that rows start on 32-byte boundaries.
int frame_ld(int rows) { return rows < 64 ? rows : int(align_up(rows, 8)); }

}  // namespace

bool build_plan(const PlanOptions& opt, Plan& plan) {
  plan = Plan();
  plan.opt = opt;
  const int nc = opt.n + 1;
  plan.nc = nc;
  if (opt.n < 1 || opt.leaf < 1 || opt.micro < 2) {
    plan.error = "n, leaf must be positive and micro >= 2";
    return false;
  }
  if (!is_pow2(opt.micro) || opt.micro > 8) {
    plan.error = "micro-block size must be 2, 4 or 8";
    return false;
  }
  if (nc % opt.leaf != 0 || !is_pow2(nc / opt.leaf)) {
    plan.error = "n+1 must be leaf * 2^p";
    return false;
  }
  if (opt.leaf % opt.micro != 0 || !is_pow2(opt.leaf / opt.micro)) {
    plan.error = "leaf must be micro * 2^q";
    return false;
  }
  int lg = 0;
  while ((opt.micro << lg) < nc) ++lg;
  plan.depth_micro = 2 * lg;
  int lq = 0;
  while ((opt.leaf << lq) < nc) ++lq;
  plan.depth_leaf = 2 * lq;
  plan.levels.resize(plan.depth_micro + 1);

  // Breadth-first construction: sons of node k at depth d are 2k and 2k+1.
  std::vector<PlanNode> cur(1);
  cur[0] = PlanNode{};
  cur[0].x0 = 0; cur[0].y0 = 0; cur[0].w = nc; cur[0].h = nc;
  for (int d = 0; d <= plan.depth_micro; ++d) {
    PlanLevel& L = plan.levels[d];
    L.depth = d;
    std::vector<PlanNode> next;
    for (size_t k = 0; k < cur.size(); ++k) {
      PlanNode nd = cur[k];
      nd.depth = d;
      nd.index = int(k);
      nd.micro = (d == plan.depth_micro);
      if (nd.micro && (nd.w != opt.micro || nd.h != opt.micro)) {
        plan.error = "internal: micro-block shape mismatch";
        return false;
      }
      const bool keep = opt.keep_dirichlet || nd.micro;
      // Gamma: boundary nodes counter-clockwise from (x0, y0).
      auto push_b = [&](int i, int j) {
        if (keep || !plan.dirichlet(i, j)) nd.bnd.push_back(plan.node_id(i, j));
      };
      for (int t = 0; t < nd.w; ++t) push_b(nd.x0 + t, nd.y0);
      for (int t = 0; t < nd.h; ++t) push_b(nd.x0 + nd.w, nd.y0 + t);
      for (int t = 0; t < nd.w; ++t) push_b(nd.x0 + nd.w - t, nd.y0 + nd.h);
      for (int t = 0; t < nd.h; ++t) push_b(nd.x0, nd.y0 + nd.h - t);
      if (nd.micro) {
        for (int b = 1; b < nd.h; ++b)
          for (int a = 1; a < nd.w; ++a) nd.gam.push_back(plan.node_id(nd.x0 + a, nd.y0 + b));
      } else {
        nd.vertical = nd.w >= nd.h;
        PlanNode s0{}, s1{};
        if (nd.vertical) {
          const int xc = nd.x0 + nd.w / 2;
          for (int t = 1; t < nd.h; ++t) nd.gam.push_back(plan.node_id(xc, nd.y0 + t));
          s0.x0 = nd.x0; s0.y0 = nd.y0; s0.w = nd.w / 2; s0.h = nd.h;
          s1.x0 = xc; s1.y0 = nd.y0; s1.w = nd.w / 2; s1.h = nd.h;
        } else {
          const int yc = nd.y0 + nd.h / 2;
          for (int t = 1; t < nd.w; ++t) nd.gam.push_back(plan.node_id(nd.x0 + t, yc));
          s0.x0 = nd.x0; s0.y0 = nd.y0; s0.w = nd.w; s0.h = nd.h / 2;
          s1.x0 = nd.x0; s1.y0 = yc; s1.w = nd.w; s1.h = nd.h / 2;
        }
        next.push_back(s0);
        next.push_back(s1);
      }
      L.nodes.push_back(std::move(nd));
    }
    cur.swap(next);
  }

  // Frame offsets, ids, maps.
  for (int d = 0; d <= plan.depth_micro; ++d) {
    PlanLevel& L = plan.levels[d];
    L.gam = int(L.nodes[0].gam.size());
    L.max_U = 0;
    L.max_bnd = 0;
    int64_t off = 0, ids_off = 0;
    for (auto& nd : L.nodes) {
      if (int(nd.gam.size()) != L.gam) {
        plan.error = "internal: interface size differs within a level";
        return false;
      }
      const int U = nd.U();
      L.max_U = std::max(L.max_U, U);
      L.max_bnd = std::max(L.max_bnd, int(nd.bnd.size()));
      nd.ld = frame_ld(U + 1);
      nd.frame_off = off;
      off += align_up(int64_t(nd.ld) * nd.ld, nd.ld < 64 ? 16 : 64);
      nd.ids_off = ids_off;
      ids_off += U;
      L.ids.insert(L.ids.end(), nd.gam.begin(), nd.gam.end());
      L.ids.insert(L.ids.end(), nd.bnd.begin(), nd.bnd.end());
    }
    L.frame_elems = align_up(off, 64);
  }
  for (int d = 0; d < plan.depth_micro; ++d) {
    PlanLevel& L = plan.levels[d];
    const PlanLevel& C = plan.levels[d + 1];
    int64_t moff = 0;
    for (auto& nd : L.nodes) {
      const int U = nd.U();
      nd.map_off = moff;
      std::unordered_map<int32_t, int> pos;
      for (int t = 0; t < U; ++t) pos[t < int(nd.gam.size()) ? nd.gam[t] : nd.bnd[t - nd.gam.size()]] = t;
      for (int s = 0; s < 2; ++s) {
        const PlanNode& son = C.nodes[2 * nd.index + s];
        std::vector<int32_t> m(U + 1, -1);
        for (size_t a = 0; a < son.bnd.size(); ++a) {
          auto it = pos.find(son.bnd[a]);
          if (it == pos.end()) {
            const int gi = son.bnd[a] % (nc + 1), gj = son.bnd[a] / (nc + 1);
            if (!plan.dirichlet(gi, gj)) {
              plan.error = "internal: son boundary node missing from father frame";
              return false;
            }
            continue;
          }
          m[it->second] = int32_t(a);
        }
        m[U] = int32_t(son.bnd.size());  // rhs row
        L.maps.insert(L.maps.end(), m.begin(), m.end());
      }
      moff += 2 * int64_t(U + 1);
    }
  }
  return true;
}

bool find_node(const Plan& plan, int x0, int y0, int w, int h, int* depth, int* index) {
  for (const auto& L : plan.levels)
    for (const auto& nd : L.nodes)
      if (nd.x0 == x0 && nd.y0 == y0 && nd.w == w && nd.h == h) {
        *depth = L.depth;
        *index = nd.index;
        return true;
      }
  return false;
}

}  // namespace hdd
