// Host-side HDD tree plan (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <functional>
#include <unordered_map>

namespace hdd {
namespace {

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }
int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Leading dimension of a global frame with U+1 rows: small frames are packed,
// large ones padded to 8 elements so that rows start on 32-byte boundaries.
int frame_ld(int rows) { return rows < 64 ? rows : int(align_up(rows, 8)); }

struct Coord {
  int i, j;
};

struct RawNode {
  int x0, y0, w, h;
  bool vertical = false;
  std::vector<Coord> gam, bnd;
};

// Nodes of the tree over the rectangle (x0, y0, W, H), level by level, down
// to `stop` x `stop` nodes.  A stop-sized node's gamma is its own cut unless
// stop == 2 (micro-block: gamma = the centre node).  `keep(i, j, last)`
// decides whether a boundary node stays in Gamma.
std::vector<std::vector<RawNode>> enumerate(int x0, int y0, int W, int H, int stop,
                                            const std::function<bool(int, int, bool)>& keep) {
  std::vector<std::vector<RawNode>> out;
  std::vector<RawNode> cur(1);
  cur[0].x0 = x0; cur[0].y0 = y0; cur[0].w = W; cur[0].h = H;
  while (!cur.empty()) {
    std::vector<RawNode> next;
    for (auto& nd : cur) {
      const bool last = nd.w == stop && nd.h == stop;
      auto push_b = [&](int i, int j) {
        if (keep(i, j, last)) nd.bnd.push_back({i, j});
      };
      for (int t = 0; t < nd.w; ++t) push_b(nd.x0 + t, nd.y0);
      for (int t = 0; t < nd.h; ++t) push_b(nd.x0 + nd.w, nd.y0 + t);
      for (int t = 0; t < nd.w; ++t) push_b(nd.x0 + nd.w - t, nd.y0 + nd.h);
      for (int t = 0; t < nd.h; ++t) push_b(nd.x0, nd.y0 + nd.h - t);
      nd.vertical = nd.w >= nd.h;
      if (last && stop == 2) {
        nd.gam.push_back({nd.x0 + 1, nd.y0 + 1});
      } else if (nd.vertical) {
        const int xc = nd.x0 + nd.w / 2;
        for (int t = 1; t < nd.h; ++t) nd.gam.push_back({xc, nd.y0 + t});
      } else {
        const int yc = nd.y0 + nd.h / 2;
        for (int t = 1; t < nd.w; ++t) nd.gam.push_back({nd.x0 + t, yc});
      }
      if (!last) {
        RawNode s0, s1;
        if (nd.vertical) {
          const int xc = nd.x0 + nd.w / 2;
          s0.x0 = nd.x0; s0.y0 = nd.y0; s0.w = nd.w / 2; s0.h = nd.h;
          s1.x0 = xc; s1.y0 = nd.y0; s1.w = nd.w / 2; s1.h = nd.h;
        } else {
          const int yc = nd.y0 + nd.h / 2;
          s0.x0 = nd.x0; s0.y0 = nd.y0; s0.w = nd.w; s0.h = nd.h / 2;
          s1.x0 = nd.x0; s1.y0 = yc; s1.w = nd.w; s1.h = nd.h / 2;
        }
        next.push_back(s0);
        next.push_back(s1);
      }
    }
    out.push_back(std::move(cur));
    cur.swap(next);
  }
  return out;
}

// Son [Gamma;rhs] index of every father frame row, or -1; false if a kept
// son boundary node is missing from the father's frame.
bool son_map(const std::vector<int32_t>& fgam, const std::vector<int32_t>& fbnd, const std::vector<int32_t>& sbnd,
             const std::function<bool(int32_t)>& droppable, std::vector<int32_t>& m) {
  const int U = int(fgam.size() + fbnd.size());
  std::unordered_map<int32_t, int> pos;
  for (int t = 0; t < U; ++t) pos[t < int(fgam.size()) ? fgam[t] : fbnd[t - fgam.size()]] = t;
  m.assign(U + 1, -1);
  for (size_t a = 0; a < sbnd.size(); ++a) {
    auto it = pos.find(sbnd[a]);
    if (it == pos.end()) {
      if (!droppable(sbnd[a])) return false;
      continue;
    }
    m[it->second] = int32_t(a);
  }
  m[U] = int32_t(sbnd.size());
  return true;
}

bool build_template(int s, SubTemplate& T, std::string& err) {
  T = SubTemplate();
  T.s = s;
  const auto raw = enumerate(0, 0, s, s, 2, [](int, int, bool) { return true; });
  auto lid = [&](const Coord& c) { return int32_t(c.j * (s + 1) + c.i); };
  int cst = 0, vec = 0;
  for (size_t k = 0; k < raw.size(); ++k) {
    const auto& nodes = raw[k];
    SubLevel L{};
    L.n = int(nodes.size());
    L.gam = int(nodes[0].gam.size());
    L.bnd = int(nodes[0].bnd.size());
    L.U = L.gam + L.bnd;
    L.fsz = (L.U + 1) * (L.U + 2) / 2;  // LDS frame: U+1 rows, packed lower triangle
    L.cst_off = cst;
    L.vec_off = vec;
    L.lid_off = int(T.lids.size());
    for (const auto& nd : nodes) {
      if (int(nd.gam.size()) != L.gam || int(nd.bnd.size()) != L.bnd) {
        err = "internal: block template level is not uniform";
        return false;
      }
      for (const auto& c : nd.gam) T.lids.push_back(lid(c));
      for (const auto& c : nd.bnd) T.lids.push_back(lid(c));
    }
    cst += L.n * (L.U + 1) * L.gam;
    vec += L.n * L.gam;
    T.max_buf = std::max(T.max_buf, L.n * L.fsz);
    T.max_gam_nodes = std::max(T.max_gam_nodes, L.n * L.gam);
    T.max_bnd_nodes = std::max(T.max_bnd_nodes, L.n * L.U);
    T.lv.push_back(L);
  }
  for (size_t k = 0; k + 1 < raw.size(); ++k) {
    SubLevel& L = T.lv[k];
    L.map_off = int(T.maps.size());
    for (size_t t = 0; t < raw[k].size(); ++t) {
      std::vector<int32_t> fg, fb;
      for (const auto& c : raw[k][t].gam) fg.push_back(lid(c));
      for (const auto& c : raw[k][t].bnd) fb.push_back(lid(c));
      for (int sidx = 0; sidx < 2; ++sidx) {
        std::vector<int32_t> sb, m;
        for (const auto& c : raw[k + 1][2 * t + sidx].bnd) sb.push_back(lid(c));
        if (!son_map(fg, fb, sb, [](int32_t) { return false; }, m)) {
          err = "internal: block template map";
          return false;
        }
        T.maps.insert(T.maps.end(), m.begin(), m.end());
      }
    }
  }
  T.lv.back().map_off = -1;
  for (const auto& nd : raw.back()) {
    T.micro_xy.push_back(nd.x0);
    T.micro_xy.push_back(nd.y0);
  }
  T.cst_size = cst;
  T.vec_size = vec;
  return true;
}

}  // namespace

bool build_plan(const PlanOptions& opt, Plan& plan) {
  plan = Plan();
  plan.opt = opt;
  const int nc = opt.n + 1;
  plan.nc = nc;
  if (opt.n < 1 || opt.leaf < 2 || !is_pow2(opt.leaf)) {
    plan.error = "n must be positive and leaf a power of two >= 2";
    return false;
  }
  if (nc % opt.leaf != 0 || !is_pow2(nc / opt.leaf)) {
    plan.error = "n+1 must be leaf * 2^p";
    return false;
  }
  if (opt.block < 2 || !is_pow2(opt.block)) {
    plan.error = "block size must be a power of two >= 2";
    return false;
  }
  const int s = std::min(opt.block, opt.leaf);
  plan.depth_block = 2 * ilog2(nc / s);
  plan.depth_leaf = 2 * ilog2(nc / opt.leaf);
  if (!build_template(s, plan.sub, plan.error)) return false;

  auto gid = [&](const Coord& c) { return int32_t(plan.node_id(c.i, c.j)); };
  const bool keepd = opt.keep_dirichlet;
  const auto raw = enumerate(0, 0, nc, nc, s, [&](int i, int j, bool last) {
    return keepd || last || !plan.dirichlet(i, j);
  });
  if (int(raw.size()) != plan.depth_block + 1) {
    plan.error = "internal: depth mismatch";
    return false;
  }
  plan.levels.resize(raw.size());
  // Boundary order: above the block level a son lists its boundary nodes in
  // the order of its father's frame [gamma ; Gamma], so the father-to-son map
  // is increasing and a lower-triangle element of the father always reads a
  // lower-triangle element of the son along a son row (contiguous).  Blocks
  // keep the order of the compiled block template.
  std::vector<std::vector<std::vector<int32_t>>> bnd_of(raw.size());
  for (size_t d = 0; d < raw.size(); ++d) {
    bnd_of[d].resize(raw[d].size());
    for (size_t k = 0; k < raw[d].size(); ++k)
      for (const auto& c : raw[d][k].bnd) bnd_of[d][k].push_back(gid(c));
  }
  for (size_t d = 0; d + 2 < raw.size(); ++d)
    for (size_t k = 0; k < raw[d].size(); ++k) {
      std::unordered_map<int32_t, int> pos;
      int q = 0;
      for (const auto& c : raw[d][k].gam) pos[gid(c)] = q++;
      for (const int32_t g : bnd_of[d][k]) pos[g] = q++;
      for (int sidx = 0; sidx < 2; ++sidx) {
        auto& sb = bnd_of[d + 1][2 * k + sidx];
        for (const int32_t g : sb)
          if (!pos.count(g)) {
            plan.error = "internal: son boundary node missing from father frame";
            return false;
          }
        std::stable_sort(sb.begin(), sb.end(), [&](int32_t a, int32_t b) { return pos[a] < pos[b]; });
      }
    }
  for (size_t d = 0; d < raw.size(); ++d) {
    PlanLevel& L = plan.levels[d];
    L.depth = int(d);
    L.max_U = 0;
    L.max_bnd = 0;
    int64_t off = 0, ids_off = 0;
    for (size_t k = 0; k < raw[d].size(); ++k) {
      const RawNode& r = raw[d][k];
      PlanNode nd{};
      nd.x0 = r.x0; nd.y0 = r.y0; nd.w = r.w; nd.h = r.h;
      nd.depth = int(d);
      nd.index = int(k);
      nd.block = d + 1 == raw.size();
      nd.vertical = r.vertical;
      for (const auto& c : r.gam) nd.gam.push_back(gid(c));
      nd.bnd = bnd_of[d][k];
      const int U = nd.U();
      if (k == 0) L.gam = int(nd.gam.size());
      if (int(nd.gam.size()) != L.gam) {
        plan.error = "internal: interface size differs within a level";
        return false;
      }
      L.max_U = std::max(L.max_U, U);
      L.max_bnd = std::max(L.max_bnd, int(nd.bnd.size()));
      nd.ld = frame_ld(U + 1);
      nd.frame_off = off;
      off += align_up(int64_t(nd.ld) * nd.ld, nd.ld < 64 ? 16 : 64);
      nd.ids_off = ids_off;
      ids_off += U;
      L.ids.insert(L.ids.end(), nd.gam.begin(), nd.gam.end());
      L.ids.insert(L.ids.end(), nd.bnd.begin(), nd.bnd.end());
      L.nodes.push_back(std::move(nd));
    }
    L.frame_elems = align_up(off, 64);
  }
  for (size_t d = 0; d + 1 < plan.levels.size(); ++d) {
    PlanLevel& L = plan.levels[d];
    const PlanLevel& C = plan.levels[d + 1];
    int64_t moff = 0;
    for (auto& nd : L.nodes) {
      nd.map_off = moff;
      for (int sidx = 0; sidx < 2; ++sidx) {
        std::vector<int32_t> m;
        if (!son_map(nd.gam, nd.bnd, C.nodes[2 * nd.index + sidx].bnd,
                     [&](int32_t g) { return plan.dirichlet(g % (nc + 1), g / (nc + 1)); }, m)) {
          plan.error = "internal: son boundary node missing from father frame";
          return false;
        }
        L.maps.insert(L.maps.end(), m.begin(), m.end());
      }
      moff += 2 * int64_t(nd.U() + 1);
    }
  }
  return true;
}

double algorithmic_flops(int n) {
  const int nc = n + 1;
  auto dir = [&](int i, int j) { return i == 0 || j == 0 || i == nc || j == nc; };
  const auto raw = enumerate(0, 0, nc, nc, 2, [&](int i, int j, bool) { return !dir(i, j); });
  double fl = 0;
  for (const auto& lv : raw)
    for (const auto& nd : lv) {
      const double g = double(nd.gam.size()), G = double(nd.bnd.size());
      fl += g * g * g / 3.0 + g * g * G + g * G * G;
    }
  return fl;
}

}  // namespace hdd
