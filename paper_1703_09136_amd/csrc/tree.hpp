// The adaptive quadtree of a plan and its interaction lists (Section 3.1:
// the hierarchical partition of the points; Section 3.3: the pairs of boxes
// that exchange multipole-to-local translations, free and heterogeneous).
//
// Two builders produce the same TreeOut bit for bit: the GPU builder
// (tree.hip: Morton keys, LSD radix sort, level-by-level splitting and
// pair-frontier list expansion as HIP kernels), which every plan uses, and
// the host reference builder (tree_host.cpp), which the tests compare it
// against and which builds without HIP for a sanitizer run of its index
// arithmetic. This header is plain C++.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace hfmm {

constexpr int KEY_BITS = 30;        // bits per coordinate of a Morton key
constexpr int kTreeMaxLevels = 32;  // the deepest tree a plan accepts (levels 0 .. 31)

// A box of the tree: level, integer position (ix, iy) on its level's grid,
// its points [begin, end) in sorted order, parent and quadrant, children by
// quadrant (-1: empty quadrant), and whether it is a leaf. Boxes are stored
// breadth first: the boxes of a level are contiguous and in Morton order.
struct Box {
  int level, ix, iy, begin, end, parent, quad;
  int child[4];
  int leaf;
};

// An ordered pair of boxes of one level (target t, source s).
struct TreePair {
  int t, s;
};

// The inputs of a tree: the points' frame (y measured from the top
// interface y_top) and the splitting rule of the plan options. A box of
// level l (side b) with cnt points splits when it holds more points than a
// leaf; under the wavelength bound (k b > leaf_kb > 0) when it holds more
// than a quarter leaf, and beyond twice the bound always; when refining at
// the interface, a bottom-row box (iy = 0) of more than one point whose own
// image pair is not admissible (2 y0 < b); never at max_level or deeper.
struct TreeParams {
  int64_t n = 0;
  double y_top = 0.0;
  double k = 1.0;         // wavenumber of the top layer
  int leaf_size = 64;
  double leaf_kb = 0.0;   // wavelength bound on k b (0: off)
  int interface_refine = 1;
  int max_level = KEY_BITS;
  int top_level = 0;      // 0: automatic
};

// status of a build
enum TreeStatus { TREE_OK = 0, TREE_DOMAIN = 1, TREE_DEPTH = 2, TREE_DEVICE = 3, TREE_MEMORY = 4 };

// The tree of a plan. Frame: x0 = min x, y0 = min (y - y_top), S the side
// of the root square. keys: the sorted Morton keys; perm[i]: the input index
// of the i-th point in key order (ties by input index). lev_begin[l]: first
// box of level l (nlev + 1 entries). top: the coarsest level of the
// expansions. fv: pairs of boxes that are not adjacent, of a level >= top,
// whose parents are adjacent (free multipole-to-local); fu: the remaining
// pairs with a leaf (free direct interaction); iv / iu the same for the
// image part, whose admissibility is the separation of the target from the
// source's mirror image. Every list is sorted by (t, s).
struct TreeOut {
  int status = TREE_OK;
  std::string msg;
  double S = 0.0, x0 = 0.0, y0 = 0.0;
  std::vector<uint64_t> keys;
  std::vector<int> perm;
  std::vector<Box> boxes;
  std::vector<int> lev_begin;
  int nlev = 0;
  std::vector<double> bsize;
  int top = 2;
  std::vector<TreePair> fv, iv, fu, iu;
};

// The root square from the frame's extent: the larger side, widened by a
// relative 1e-12 so that the largest coordinate maps inside the key range.
double tree_root_side(double xmin, double xmax, double ymin, double ymax);

// The coarsest expansion level from the level sizes and the shallowest leaf.
int tree_top_level(const TreeOut& t, int top_option);

// The host reference builder. xy: the n points (x, y) in the caller's frame.
void host_tree_build(const TreeParams& p, const double* xy, TreeOut& out);

}  // namespace hfmm
