// Checks of the host tree builder's index arithmetic, built with the host
// sanitizers (address, undefined behaviour) by tests/test_tree_host_sanitized.py:
// on seeded point sets (uniform, clustered on ellipses, a line, tiny sets,
// a pair in one key cell, deep trees) every invariant of the tree and of the
// four pair lists is verified; exit status 0 when all hold.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "tree.hpp"

using namespace hfmm;

static int failures = 0;
#define CHECK(cond, ...)                        \
  do {                                          \
    if (!(cond)) {                              \
      std::printf("FAIL %s: ", label);          \
      std::printf(__VA_ARGS__);                 \
      std::printf("\n");                        \
      ++failures;                               \
      return;                                   \
    }                                           \
  } while (0)

static bool adjacent(const Box& a, const Box& b) { return std::abs(a.ix - b.ix) <= 1 && std::abs(a.iy - b.iy) <= 1; }

// every target leaf reaches every point exactly once through the pairs
// (A, s) whose target A is the leaf or an ancestor
static bool complete(const TreeOut& t, const std::vector<TreePair>& far, const std::vector<TreePair>& near,
                     int64_t n) {
  std::vector<std::vector<int>> by_t(t.boxes.size());
  for (const auto& p : far) by_t[p.t].push_back(p.s);
  for (const auto& p : near) by_t[p.t].push_back(p.s);
  std::vector<int> cover((size_t)n);
  for (size_t b = 0; b < t.boxes.size(); ++b) {
    if (!t.boxes[b].leaf) continue;
    std::fill(cover.begin(), cover.end(), 0);
    for (int a = (int)b; a >= 0; a = t.boxes[a].parent)
      for (int s : by_t[a])
        for (int j = t.boxes[s].begin; j < t.boxes[s].end; ++j) ++cover[j];
    for (int64_t j = 0; j < n; ++j)
      if (cover[j] != 1) return false;
  }
  return true;
}

static void check(const char* label, const TreeParams& p, const std::vector<double>& xy) {
  TreeOut t;
  host_tree_build(p, xy.data(), t);
  CHECK(t.status == TREE_OK, "status %d (%s)", t.status, t.msg.c_str());
  const int64_t n = p.n;
  CHECK((int64_t)t.perm.size() == n && (int64_t)t.keys.size() == n, "sizes");
  std::vector<int> seen((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) {
    CHECK(t.perm[i] >= 0 && t.perm[i] < n && !seen[t.perm[i]]++, "perm not a permutation at %lld", (long long)i);
    if (i > 0) CHECK(t.keys[i - 1] < t.keys[i] || (t.keys[i - 1] == t.keys[i] && t.perm[i - 1] < t.perm[i]),
                     "keys not sorted at %lld", (long long)i);
  }
  const auto& B = t.boxes;
  CHECK(t.nlev >= 1 && (int)t.lev_begin.size() == t.nlev + 1 && t.lev_begin.back() == (int)B.size(), "levels");
  CHECK(B[0].begin == 0 && B[0].end == n && B[0].parent == -1, "root");
  for (int l = 0; l < t.nlev; ++l)
    for (int b = t.lev_begin[l]; b < t.lev_begin[l + 1]; ++b) {
      const Box& x = B[b];
      CHECK(x.level == l && x.begin < x.end, "box %d level / range", b);
      const int shift = 2 * (KEY_BITS - l);
      for (int j = x.begin; j < x.end && l > 0; ++j)
        CHECK((t.keys[j] >> shift) == (t.keys[x.begin] >> shift), "box %d key prefix", b);
      int kids = 0, at = x.begin;
      for (int q = 0; q < 4; ++q) {
        const int c = x.child[q];
        if (c < 0) continue;
        ++kids;
        CHECK(c > b && c < (int)B.size(), "box %d child index", b);
        const Box& y = B[c];
        CHECK(y.parent == b && y.quad == q && y.level == l + 1, "box %d child links", b);
        CHECK(y.ix == 2 * x.ix + (q & 1) && y.iy == 2 * x.iy + (q >> 1), "box %d child position", b);
        CHECK(y.begin == at, "box %d children not contiguous", b);
        at = y.end;
      }
      CHECK(x.leaf == (kids == 0), "box %d leaf flag", b);
      if (kids) CHECK(at == x.end, "box %d children do not cover it", b);
      if (l > 0) CHECK(b > t.lev_begin[l] ? B[b - 1].begin < x.begin : true, "box %d order", b);
    }
  const std::vector<TreePair>* lists[4] = {&t.fv, &t.fu, &t.iv, &t.iu};
  for (int w = 0; w < 4; ++w)
    for (size_t i = 0; i < lists[w]->size(); ++i) {
      const TreePair pr = (*lists[w])[i];
      CHECK(pr.t >= 0 && pr.t < (int)B.size() && pr.s >= 0 && pr.s < (int)B.size(), "list %d pair range", w);
      CHECK(B[pr.t].level == B[pr.s].level, "list %d pair levels", w);
      if (i > 0) {
        const TreePair q = (*lists[w])[i - 1];
        CHECK(q.t < pr.t || (q.t == pr.t && q.s < pr.s), "list %d order", w);
      }
      if (w == 0) CHECK(!adjacent(B[pr.t], B[pr.s]) && B[pr.t].level >= t.top, "fv pair admissibility");
      if (w == 1 || w == 3) CHECK(B[pr.t].leaf || B[pr.s].leaf, "near pair without a leaf");
      if (w == 2) CHECK(B[pr.t].level >= t.top, "iv level");
    }
  CHECK(complete(t, t.fv, t.fu, n), "free lists incomplete");
  CHECK(complete(t, t.iv, t.iu, n), "image lists incomplete");
}

int main() {
  std::mt19937_64 rng(17039136);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  auto uniform = [&](int n, double y0) {
    std::vector<double> xy(2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
      xy[2 * i] = U(rng);
      xy[2 * i + 1] = y0 + U(rng);
    }
    return xy;
  };
  auto ellipses = [&](int n, int m) {
    std::vector<double> xy;
    for (int e = 0; e < m; ++e) {
      const double cx = U(rng), cy = 0.6 + 0.3 * U(rng), a = 0.02 + 0.06 * U(rng), b = 0.02 + 0.06 * U(rng);
      for (int i = 0; i < n / m; ++i) {
        const double t = 2.0 * M_PI * i / (n / m);
        xy.push_back(cx + a * std::cos(t));
        xy.push_back(cy + b * std::sin(t));
      }
    }
    return xy;
  };
  TreeParams p;
  p.k = 8.0 * M_PI;
  p.leaf_size = 32;
  p.leaf_kb = 8.0;
  {
    const char* label = "uniform";
    auto xy = uniform(3000, 0.05);
    p.n = 3000;
    check(label, p, xy);
  }
  {
    const char* label = "ellipses";
    auto xy = ellipses(4000, 8);
    p.n = (int64_t)xy.size() / 2;
    check(label, p, xy);
  }
  {
    const char* label = "line";
    std::vector<double> xy;
    for (int i = 0; i < 300; ++i) {
      xy.push_back(0.3);
      xy.push_back(0.1 + 0.8 * U(rng));
    }
    p.n = 300;
    check(label, p, xy);
  }
  {
    const char* label = "tiny";
    std::vector<double> xy{0.25, 0.5};
    p.n = 1;
    check(label, p, xy);
    xy = {0.25, 0.5, 0.75, 0.6};
    p.n = 2;
    check(label, p, xy);
  }
  {
    const char* label = "one key cell";
    auto xy = uniform(200, 0.05);
    xy.push_back(xy[0] + 1e-13);
    xy.push_back(xy[1]);
    p.n = 201;
    check(label, p, xy);
  }
  {
    const char* label = "deep, no refinement";
    auto xy = uniform(500, 0.001);
    TreeParams q = p;
    q.n = 500;
    q.leaf_size = 1;
    q.leaf_kb = 0.0;
    q.interface_refine = 0;
    check(label, q, xy);
    q.max_level = 3;
    q.top_level = 2;
    check(label, q, xy);
  }
  {
    const char* label = "coincident points are refused";
    auto xy = uniform(100, 0.05);
    xy[2 * 70] = xy[2 * 3];
    xy[2 * 70 + 1] = xy[2 * 3 + 1];
    TreeOut t;
    p.n = 100;
    host_tree_build(p, xy.data(), t);
    if (t.status != TREE_DOMAIN) {
      std::printf("FAIL %s\n", label);
      ++failures;
    }
  }
  std::printf("%s\n", failures ? "FAILED" : "all tree checks passed");
  return failures ? 1 : 0;
}
