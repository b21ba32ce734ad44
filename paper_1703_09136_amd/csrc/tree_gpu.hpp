// The GPU builder of the quadtree and its interaction lists (tree.hip).
#pragma once

#include "devbuf.hpp"
#include "tree.hpp"

namespace hfmm {

// Device arrays of a built tree: the sorted Morton keys and the
// permutation (sorted position -> input index).
struct TreeDev {
  DevBuf<uint64_t> keys;
  DevBuf<int> perm;
};

// Builds the tree of the n points at d_points (device, (x, y) pairs in the
// caller's frame) on stream s: Morton keys, an LSD radix sort, level-by-
// level splitting and the dual-tree pair lists, all as HIP kernels; out
// receives host copies of the boxes, levels, frame and lists (and of keys and
// perm when copy_keys is set; out.perm always), dev the device keys and
// permutation. Synchronises s (the level loop reads a count per level).
// out.status: TREE_OK, TREE_DOMAIN (non-finite point, point not above the
// top interface, coincident points), TREE_DEPTH, TREE_DEVICE / TREE_MEMORY
// (a HIP call failed; out.msg says which).
void gpu_tree_build(const TreeParams& p, const double* d_points, hipStream_t s, bool copy_keys, TreeOut& out,
                    TreeDev& dev);

}  // namespace hfmm
