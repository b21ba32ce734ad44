// Host reference builder of the quadtree and its interaction lists (Section
// 3.1, Section 3.3): the same TreeOut as the GPU builder, by plain loops, a
// comparison sort and a depth-first dual-tree traversal. Plans use the GPU
// builder; this one is what the tests check it against, and it compiles
// without HIP (a sanitizer build of its index arithmetic runs on the CPU).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <utility>

#include "tree.hpp"

namespace hfmm {

double tree_root_side(double xmin, double xmax, double ymin, double ymax) {
  double S = std::max(xmax - xmin, ymax - ymin);
  if (!(S > 0.0)) S = std::max(1e-3, 1e-6 * std::fabs(ymin));
  return S * (1.0 + 1e-12);
}

int tree_top_level(const TreeOut& t, int top_option) {
  // Starting the multipole-to-local pairs at a finer level than 2 splits the
  // coarse levels' few pairs (of the highest orders, whose launches are
  // latency bound) into more pairs of a lower order at that level; the
  // automatic choice keeps every pair of boxes of the top level below
  // kTopPairs. No leaf may lie above it.
  constexpr int64_t kTopPairs = 4096;
  int minleaf = t.nlev;
  for (const Box& b : t.boxes)
    if (b.leaf) minleaf = std::min(minleaf, b.level);
  int top = 2;
  if (top_option >= 2) {
    top = top_option;
  } else {
    for (int l = 3; l < t.nlev; ++l) {
      const int64_t nbl = t.lev_begin[l + 1] - t.lev_begin[l];
      if (nbl * nbl > kTopPairs) break;
      top = l;
    }
  }
  return std::max(2, std::min(top, std::min(minleaf, t.nlev - 1)));
}

namespace {

uint64_t spread_bits(uint32_t v) {
  uint64_t x = v;
  x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
  x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
  x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x;
}

bool split_box(const TreeParams& p, int cnt, int iy, int level, double b, double ymin, int maxl) {
  bool split = cnt > p.leaf_size;
  if (p.leaf_kb > 0.0 && p.k * b > p.leaf_kb) {
    if (cnt > std::max(1, p.leaf_size / 4) || p.k * b > 2.0 * p.leaf_kb) split = true;
  }
  if (p.interface_refine && iy == 0 && 2.0 * ymin < b && cnt > 1) split = true;
  if (level >= maxl) split = false;
  return split;
}

bool pair_less(const TreePair& a, const TreePair& b) { return a.t < b.t || (a.t == b.t && a.s < b.s); }

// Depth-first dual-tree traversal from the root pair: a pair goes to the
// "far" list when admissible, else to the "near" list when either box is a
// leaf, else its children pairs are visited.
template <typename Adm>
void traverse(const std::vector<Box>& B, Adm admissible, std::vector<TreePair>& far, std::vector<TreePair>& near) {
  std::vector<TreePair> stack{{0, 0}};
  while (!stack.empty()) {
    const TreePair pr = stack.back();
    stack.pop_back();
    if (admissible(pr)) {
      far.push_back(pr);
    } else if (B[pr.t].leaf || B[pr.s].leaf) {
      near.push_back(pr);
    } else {
      for (int a = 0; a < 4; ++a) {
        if (B[pr.t].child[a] < 0) continue;
        for (int c = 0; c < 4; ++c)
          if (B[pr.s].child[c] >= 0) stack.push_back({B[pr.t].child[a], B[pr.s].child[c]});
      }
    }
  }
  std::sort(far.begin(), far.end(), pair_less);
  std::sort(near.begin(), near.end(), pair_less);
}

}  // namespace

void host_tree_build(const TreeParams& p, const double* xy, TreeOut& out) {
  out = TreeOut{};
  const int64_t n = p.n;
  // ---- frame and domain checks: finite, strictly above the top interface
  std::vector<double> fy((size_t)n);
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  for (int64_t i = 0; i < n; ++i) {
    const double x = xy[2 * i], y = xy[2 * i + 1] - p.y_top;
    if (!std::isfinite(x) || !std::isfinite(y)) {
      out.status = TREE_DOMAIN;
      out.msg = "non-finite point " + std::to_string(i);
      return;
    }
    if (!(y > 0.0)) {
      out.status = TREE_DOMAIN;
      out.msg = "point " + std::to_string(i) + " is not strictly above the top interface";
      return;
    }
    fy[i] = y;
    xmin = std::min(xmin, x);
    xmax = std::max(xmax, x);
    ymin = std::min(ymin, y);
    ymax = std::max(ymax, y);
  }
  const double S = tree_root_side(xmin, xmax, ymin, ymax);
  out.S = S;
  out.x0 = xmin;
  out.y0 = ymin;
  // ---- Morton keys of 2 x 30 bits, sorted with ties by input index
  std::vector<std::pair<uint64_t, int>> key((size_t)n);
  const double scale = (double)(1u << KEY_BITS) / S;
  const double kmax = (double)((1u << KEY_BITS) - 1);
  for (int64_t i = 0; i < n; ++i) {
    const double gx = (xy[2 * i] - xmin) * scale, gy = (fy[i] - ymin) * scale;
    const uint32_t ix = (uint32_t)std::min(std::max(std::floor(gx), 0.0), kmax);
    const uint32_t iy = (uint32_t)std::min(std::max(std::floor(gy), 0.0), kmax);
    key[i] = {spread_bits(ix) | (spread_bits(iy) << 1), (int)i};
  }
  std::sort(key.begin(), key.end());
  out.keys.resize((size_t)n);
  out.perm.resize((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    out.keys[i] = key[i].first;
    out.perm[i] = key[i].second;
  }
  // Coincident points share a key. Within each run of equal keys the points
  // are compared after sorting the run by (x, y), so that two equal points
  // are found even when a different point with the same key lies between
  // them in index order.
  std::vector<std::pair<std::pair<double, double>, int>> run;
  for (int64_t i = 0; i < n;) {
    int64_t e = i + 1;
    while (e < n && key[e].first == key[i].first) ++e;
    if (e - i > 1) {
      run.clear();
      for (int64_t t = i; t < e; ++t) {
        const int a = key[t].second;
        run.push_back({{xy[2 * a], fy[a]}, a});
      }
      std::sort(run.begin(), run.end());
      for (size_t t = 1; t < run.size(); ++t)
        if (run[t].first == run[t - 1].first) {
          out.status = TREE_DOMAIN;
          out.msg = "coincident points " + std::to_string(std::min(run[t - 1].second, run[t].second)) + " and " +
                    std::to_string(std::max(run[t - 1].second, run[t].second));
          return;
        }
    }
    i = e;
  }
  // ---- adaptive quadtree, breadth first
  std::vector<Box>& B = out.boxes;
  B.push_back(Box{0, 0, 0, 0, (int)n, -1, 0, {-1, -1, -1, -1}, 1});
  out.lev_begin.push_back(0);
  const int maxl = std::min(p.max_level, KEY_BITS);
  for (int l = 0;; ++l) {
    const int lb = out.lev_begin[l], le = (int)B.size();
    const double b = S / (double)(1u << l);
    out.bsize.push_back(b);
    bool any = false;
    for (int bi = lb; bi < le; ++bi) {
      if (!split_box(p, B[bi].end - B[bi].begin, B[bi].iy, l, b, ymin, maxl)) continue;
      any = true;
      B[bi].leaf = 0;
      const int shift = 2 * (KEY_BITS - l - 1);
      int s = B[bi].begin;
      for (int q = 0; q < 4; ++q) {
        // the points of quadrant q are contiguous: the run of digit q
        int e = s;
        while (e < B[bi].end && (int)((key[e].first >> shift) & 3u) == q) ++e;
        if (e > s) {
          Box c{l + 1, 2 * B[bi].ix + (q & 1), 2 * B[bi].iy + (q >> 1), s, e, bi, q, {-1, -1, -1, -1}, 1};
          B[bi].child[q] = (int)B.size();
          B.push_back(c);
        }
        s = e;
      }
    }
    if (!any) break;
    out.lev_begin.push_back(le);
  }
  out.nlev = (int)out.lev_begin.size();
  out.lev_begin.push_back((int)B.size());
  if (out.nlev > kTreeMaxLevels) {
    out.status = TREE_DEPTH;
    out.msg = "tree deeper than supported";
    return;
  }
  out.top = tree_top_level(out, p.top_level);
  // ---- interaction lists
  const int top = out.top;
  auto adjacent = [&](const TreePair& pr) {
    return std::abs(B[pr.t].ix - B[pr.s].ix) <= 1 && std::abs(B[pr.t].iy - B[pr.s].iy) <= 1;
  };
  traverse(
      B, [&](const TreePair& pr) { return !adjacent(pr) && B[pr.t].level >= top; }, out.fv, out.fu);
  traverse(
      B,
      [&](const TreePair& pr) {
        const int l = B[pr.t].level;
        return l >= top && (B[pr.t].iy + B[pr.s].iy >= 1 || 2.0 * ymin >= out.bsize[l]);
      },
      out.iv, out.iu);
}

}  // namespace hfmm
