// Host check of the HDD tree plan, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitize.py.
//
// For a range of meshes it builds the plan and checks the structure the
// kernels rely on: 2^d nodes on depth d whose rectangles halve their
// father's (Section 2.1), gamma on the node's cut and inside the node
// (eq. gamma_def), Gamma on the node's perimeter, ids and frames of a level
// that do not overlap, and father-to-son maps that point into the son's
// [Gamma ; rhs] rows and are increasing above the block level.  Exit code 0
// when every check holds; the first failing check is printed.
#include <cstdio>
#include <cstdlib>
#include <set>

#include "plan.hpp"

using hdd::Plan;
using hdd::PlanOptions;

static int fails = 0;
#define CHECK(c, ...)                              \
  do {                                             \
    if (!(c)) {                                    \
      if (fails++ < 5) {                           \
        std::fprintf(stderr, "check failed: " #c); \
        std::fprintf(stderr, " | " __VA_ARGS__);   \
        std::fprintf(stderr, "\n");                \
      }                                            \
    }                                              \
  } while (0)

static void check_plan(int n, int leaf, int block, bool keepd) {
  PlanOptions o;
  o.n = n;
  o.leaf = leaf;
  o.block = block;
  o.keep_dirichlet = keepd;
  Plan p;
  const bool ok = hdd::build_plan(o, p);
  CHECK(ok, "n=%d leaf=%d: %s", n, leaf, p.error.c_str());
  if (!ok) return;
  const int nc = p.nc;
  CHECK(int(p.levels.size()) == p.depth_block + 1, "n=%d", n);
  for (size_t d = 0; d < p.levels.size(); ++d) {
    const auto& L = p.levels[d];
    CHECK(int(L.nodes.size()) == (1 << d), "n=%d depth %zu", n, d);
    int64_t prev_end = 0;
    size_t ids = 0;
    for (const auto& nd : L.nodes) {
      const int U = nd.U();
      CHECK(nd.ld >= U + 1, "n=%d", n);
      CHECK(nd.frame_off >= prev_end, "n=%d depth %zu: frames overlap", n, d);
      prev_end = nd.frame_off + int64_t(nd.ld) * nd.ld;
      CHECK(prev_end <= L.frame_elems, "n=%d depth %zu", n, d);
      CHECK(nd.ids_off == int64_t(ids), "n=%d", n);
      for (int k = 0; k < U; ++k) {
        const int32_t g = k < int(nd.gam.size()) ? nd.gam[k] : nd.bnd[k - nd.gam.size()];
        CHECK(L.ids[ids + k] == g, "n=%d", n);
      }
      ids += U;
      std::set<int32_t> seen;
      for (const int32_t g : nd.gam) {
        const int i = g % (nc + 1), j = g / (nc + 1);
        CHECK(i > nd.x0 && i < nd.x0 + nd.w && j > nd.y0 && j < nd.y0 + nd.h, "gamma outside the node");
        if (!nd.block || nd.w > 2 || nd.h > 2) {
          if (nd.vertical) CHECK(i == nd.x0 + nd.w / 2, "gamma not on the cut");
          else CHECK(j == nd.y0 + nd.h / 2, "gamma not on the cut");
        }
        CHECK(seen.insert(g).second, "duplicate id");
      }
      for (const int32_t g : nd.bnd) {
        const int i = g % (nc + 1), j = g / (nc + 1);
        const bool on = (i == nd.x0 || i == nd.x0 + nd.w) ? (j >= nd.y0 && j <= nd.y0 + nd.h)
                                                        : ((j == nd.y0 || j == nd.y0 + nd.h) && i >= nd.x0 &&
                                                           i <= nd.x0 + nd.w);
        CHECK(on, "Gamma off the perimeter");
        CHECK(keepd || nd.block || !p.dirichlet(i, j), "Dirichlet node kept above the blocks");
        CHECK(seen.insert(g).second, "duplicate id");
      }
      if (d + 1 < p.levels.size()) {
        const auto& C = p.levels[d + 1];
        for (int sidx = 0; sidx < 2; ++sidx) {
          const auto& son = C.nodes[2 * nd.index + sidx];
          CHECK(son.w * son.h * 2 == nd.w * nd.h, "son is not half of the father");
          const int32_t* m = L.maps.data() + nd.map_off + sidx * (U + 1);
          CHECK(nd.map_off + 2 * (U + 1) <= int64_t(L.maps.size()), "map outside the table");
          CHECK(m[U] == int(son.bnd.size()), "rhs row maps to the son's rhs row");
          int last = -1, hits = 0;
          for (int r = 0; r < U; ++r) {
            CHECK(m[r] >= -1 && m[r] < int(son.bnd.size()), "map out of range");
            if (m[r] < 0) continue;
            ++hits;
            const int32_t g = r < int(nd.gam.size()) ? nd.gam[r] : nd.bnd[r - nd.gam.size()];
            CHECK(son.bnd[m[r]] == g, "map names another node");
            if (!son.block) CHECK(m[r] > last, "map not increasing");
            last = m[r];
          }
          int kept = 0;
          for (const int32_t g : son.bnd) kept += (keepd || !p.dirichlet(g % (nc + 1), g / (nc + 1))) ? 1 : 0;
          CHECK(hits == kept, "a kept son boundary node is not in the father frame");
        }
      }
    }
    CHECK(ids == L.ids.size(), "n=%d", n);
  }
  // block template: son maps inside the son frame, local ids inside the block
  const auto& T = p.sub;
  const int s = T.s;
  for (size_t k = 0; k < T.lv.size(); ++k) {
    const auto& L = T.lv[k];
    CHECK(L.fsz == (L.U + 1) * (L.U + 2) / 2, "template frame size");
    CHECK(L.lid_off + L.n * L.U <= int(T.lids.size()), "template ids");
    for (int e = 0; e < L.n * L.U; ++e) {
      const int v = T.lids[L.lid_off + e];
      CHECK(v >= 0 && v < (s + 1) * (s + 1), "local id outside the block");
    }
    if (k + 1 < T.lv.size()) {
      const auto& C = T.lv[k + 1];
      CHECK(2 * L.n == C.n, "template level sizes");
      CHECK(L.map_off + L.n * 2 * (L.U + 1) <= int(T.maps.size()), "template maps");
      for (int e = 0; e < L.n * 2 * (L.U + 1); ++e) {
        const int v = T.maps[L.map_off + e];
        CHECK(v >= -1 && v <= C.bnd, "template map out of range");
      }
    }
  }
  CHECK(int(T.micro_xy.size()) == 2 * T.lv.back().n, "micro-blocks");
}

int main() {
  const int cases[][3] = {{3, 2, 16}, {7, 4, 16}, {15, 8, 16}, {15, 16, 16}, {31, 8, 8},
                          {63, 8, 16}, {63, 16, 16}, {127, 16, 16}, {255, 16, 16}, {255, 32, 16}};
  for (const auto& c : cases)
    for (int keepd = 0; keepd < 2; ++keepd) check_plan(c[0], c[1], c[2], keepd != 0);
  // invalid options are refused with a message
  Plan p;
  PlanOptions bad;
  bad.n = 10;
  bad.leaf = 4;
  CHECK(!hdd::build_plan(bad, p) && !p.error.empty(), "n + 1 not leaf * 2^k is refused");
  bad.n = 15;
  bad.leaf = 3;
  CHECK(!hdd::build_plan(bad, p) && !p.error.empty(), "leaf not a power of two is refused");
  std::printf("plan checks: %d failures\n", fails);
  return fails ? 1 : 0;
}
