// GPU builder of the quadtree and its interaction lists (Section 3.1: the
// adaptive hierarchical partition; Section 3.3: the box pairs of the free and
// heterogeneous multipole-to-local translations).
//
//  1. frame: a min / max reduction of the points (interface frame), which
//     also finds the first point that is not finite or not above the top
//     interface;
//  2. Morton keys (2 x 30 bits) and a stable LSD radix sort of (key, index),
//     four bits per pass: per-tile digit counts, one exclusive scan over
//     (digit, tile), and a stable scatter that ranks each tile's items with
//     wavefront ballots;
//  3. the tree level by level: per box of the level the splitting rule and
//     its quadrant runs (binary searches of the sorted keys: the boxes of a
//     level share their key prefix, so a box's quadrant digits are sorted),
//     an exclusive scan of the child counts, and the children written in
//     breadth-first order;
//  4. the pair lists by frontier expansion: the pairs of a level are
//     classified in parallel (admissible, near, or expanded into the pairs of
//     their children), each block reserving its output range with one atomic
//     addition; the lists are then radix sorted by (t, s).
#include "tree_gpu.hpp"

#include <algorithm>
#include <cmath>
#include <string>
#include <utility>

namespace hfmm {
namespace {

constexpr int TB = 256;  // threads per block
constexpr int WV = 64;   // wavefront size
constexpr int NW = TB / WV;

// ---------------------------------------------------------------- frame
struct FrameRed {
  double xmin, xmax, ymin, ymax;
  long long bad;  // first offending input index (n: none)
};

__device__ inline void frame_merge(FrameRed& a, const FrameRed& b) {
  a.xmin = a.xmin < b.xmin ? a.xmin : b.xmin;
  a.xmax = a.xmax > b.xmax ? a.xmax : b.xmax;
  a.ymin = a.ymin < b.ymin ? a.ymin : b.ymin;
  a.ymax = a.ymax > b.ymax ? a.ymax : b.ymax;
  a.bad = a.bad < b.bad ? a.bad : b.bad;
}

__device__ inline void frame_block_reduce(FrameRed r, FrameRed* out) {
  __shared__ FrameRed sr[TB];
  sr[threadIdx.x] = r;
  __syncthreads();
  for (int w = TB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) frame_merge(sr[threadIdx.x], sr[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sr[0];
}

__global__ void __launch_bounds__(TB) k_frame(const double2* __restrict__ pts, int64_t n, double y_top,
                                              FrameRed* __restrict__ part) {
  FrameRed r{1e300, -1e300, 1e300, -1e300, (long long)n};
  for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
    const double2 v = pts[i];
    const double x = v.x, y = v.y - y_top;
    if (!isfinite(x) || !isfinite(y) || !(y > 0.0)) {
      if (i < r.bad) r.bad = i;
      continue;
    }
    r.xmin = x < r.xmin ? x : r.xmin;
    r.xmax = x > r.xmax ? x : r.xmax;
    r.ymin = y < r.ymin ? y : r.ymin;
    r.ymax = y > r.ymax ? y : r.ymax;
  }
  frame_block_reduce(r, part + blockIdx.x);
}

__global__ void __launch_bounds__(TB) k_frame_final(const FrameRed* __restrict__ part, int np, int64_t n,
                                                    FrameRed* __restrict__ out) {
  FrameRed r{1e300, -1e300, 1e300, -1e300, (long long)n};
  for (int i = threadIdx.x; i < np; i += TB) frame_merge(r, part[i]);
  frame_block_reduce(r, out);
}

// ---------------------------------------------------------------- keys
__device__ inline uint64_t interleave(uint32_t v) {
  uint64_t x = v;
  x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
  x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
  x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x;
}

// grid cell of a coordinate: floor, clamped to [0, 2^30 - 1]
__device__ inline uint32_t grid_cell(double g) {
  const double kmax = (double)((1u << KEY_BITS) - 1);
  double f = floor(g);
  f = f < 0.0 ? 0.0 : f;
  f = kmax < f ? kmax : f;
  return (uint32_t)f;
}

__global__ void k_morton(const double2* __restrict__ pts, int64_t n, double y_top, double xmin, double ymin,
                         double scale, uint64_t* __restrict__ keys, int* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  const double2 v = pts[i];
  const double fy = v.y - y_top;
  const double gx = (v.x - xmin) * scale;
  const double gy = (fy - ymin) * scale;
  keys[i] = interleave(grid_cell(gx)) | (interleave(grid_cell(gy)) << 1);
  vals[i] = (int)i;
}

// adjacent equal keys (a coincident pair is only possible where they occur)
__global__ void k_count_dups(const uint64_t* __restrict__ keys, int64_t n, int* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  const bool dup = i > 0 && i < n && keys[i] == keys[i - 1];
  const unsigned long long m = __ballot(dup);
  if ((threadIdx.x & (WV - 1)) == 0 && m) atomicAdd(count, (int)__popcll(m));
}

// ---------------------------------------------------------------- exclusive scan (int)
constexpr int SC_ITEMS = 4;
constexpr int SC_TILE = TB * SC_ITEMS;

// block-wide exclusive scan of one value per thread; returns the block total
__device__ inline int block_excl_scan(int v, int& excl) {
  __shared__ int ws[NW];
  const int lane = threadIdx.x & (WV - 1), wave = threadIdx.x / WV;
  int x = v;
  for (int o = 1; o < WV; o <<= 1) {
    const int y = __shfl_up(x, o, WV);
    if (lane >= o) x += y;
  }
  if (lane == WV - 1) ws[wave] = x;
  __syncthreads();
  int pre = 0, tot = 0;
  for (int w = 0; w < NW; ++w) {
    if (w < wave) pre += ws[w];
    tot += ws[w];
  }
  __syncthreads();
  excl = pre + x - v;
  return tot;
}

__global__ void __launch_bounds__(TB) k_scan_tile(const int* __restrict__ in, int* __restrict__ out, int64_t m,
                                                  int* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
  int v[SC_ITEMS], t = 0;
#pragma unroll
  for (int j = 0; j < SC_ITEMS; ++j) {
    v[j] = base + j < m ? in[base + j] : 0;
    t += v[j];
  }
  int excl;
  const int tot = block_excl_scan(t, excl);
#pragma unroll
  for (int j = 0; j < SC_ITEMS; ++j) {
    if (base + j < m) out[base + j] = excl;
    excl += v[j];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void k_scan_add(int* __restrict__ out, int64_t m, const int* __restrict__ off) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < m) out[i] += off[i / SC_TILE];
}

// total = out[m - 1] + in[m - 1] (after an exclusive scan of in into out)
__global__ void k_scan_total(const int* __restrict__ in, const int* __restrict__ out, int64_t m, int* __restrict__ total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *total = m > 0 ? out[m - 1] + in[m - 1] : 0;
}

inline int nblocks(int64_t n, int per) { return (int)((n + per - 1) / per); }

// scratch of the scans (one pair of buffers per recursion depth)
struct ScanTmp {
  DevBuf<int> sums[4], offs[4];
};

hipError_t scan_excl(hipStream_t s, const int* in, int* out, int64_t m, ScanTmp& tmp, int depth = 0) {
  if (m <= 0) return hipSuccess;
  if (depth >= 4) return hipErrorInvalidValue;  // 1024^4 elements: beyond any tree
  const int nt = nblocks(m, SC_TILE);
  hipError_t e = tmp.sums[depth].ensure((size_t)nt);
  if (e == hipSuccess) e = tmp.offs[depth].ensure((size_t)nt);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_tile, dim3(nt), dim3(TB), 0, s, in, out, m, tmp.sums[depth].p);
  if (nt > 1) {
    e = scan_excl(s, tmp.sums[depth].p, tmp.offs[depth].p, nt, tmp, depth + 1);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3(nblocks(m, TB)), dim3(TB), 0, s, out, m, tmp.offs[depth].p);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- LSD radix sort
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = TB * RS_ITEMS;
constexpr int RS_DIGITS = 16;  // four bits per pass

__global__ void __launch_bounds__(TB) k_rs_count(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                 int* __restrict__ cnt, int ntile) {
  __shared__ int h[RS_DIGITS];
  if (threadIdx.x < RS_DIGITS) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ITEMS; ++r) {
    const int64_t i = base + r * TB + threadIdx.x;
    if (i < n) atomicAdd(&h[(int)((keys[i] >> shift) & 15u)], 1);
  }
  __syncthreads();
  if (threadIdx.x < RS_DIGITS) cnt[threadIdx.x * ntile + blockIdx.x] = h[threadIdx.x];
}

// stable scatter: an item's destination is the scanned count of its digit
// for this tile, plus the items of that digit before it in the tile (earlier
// rounds, earlier wavefronts of its round, earlier lanes of its wavefront)
__global__ void __launch_bounds__(TB) k_rs_scatter(const uint64_t* __restrict__ kin, const int* __restrict__ vin,
                                                   uint64_t* __restrict__ kout, int* __restrict__ vout, int64_t n,
                                                   int shift, const int* __restrict__ off, int ntile) {
  __shared__ int run[RS_DIGITS];
  __shared__ int wc[NW][RS_DIGITS];
  const int tid = threadIdx.x, lane = tid & (WV - 1), wave = tid / WV;
  if (tid < RS_DIGITS) run[tid] = off[tid * ntile + blockIdx.x];
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ITEMS; ++r) {
    const int64_t i = base + r * TB + tid;
    const bool valid = i < n;
    const uint64_t k = valid ? kin[i] : 0ull;
    const int d = valid ? (int)((k >> shift) & 15u) : RS_DIGITS;
    int rank = 0;
    for (int dd = 0; dd < RS_DIGITS; ++dd) {
      const unsigned long long m = __ballot(d == dd);
      if (lane == 0) wc[wave][dd] = (int)__popcll(m);
      if (d == dd) rank = (int)__popcll(m & below);
    }
    __syncthreads();
    if (valid) {
      int dst = run[d] + rank;
      for (int w = 0; w < wave; ++w) dst += wc[w][d];
      kout[dst] = k;
      if (vin) vout[dst] = vin[i];
    }
    __syncthreads();
    if (tid < RS_DIGITS) {
      int t = 0;
      for (int w = 0; w < NW; ++w) t += wc[w][tid];
      run[tid] += t;
    }
    __syncthreads();
  }
}

struct SortTmp {
  DevBuf<uint64_t> k2;
  DevBuf<int> v2, cnt, off;
  ScanTmp scan;
};

// sorts keys[0, n) on their low `bits` bits (values alongside when vals is
// given), stable; the result ends in keys (and vals)
hipError_t radix_sort(hipStream_t s, DevBuf<uint64_t>& keys, DevBuf<int>* vals, int64_t n, int bits, SortTmp& t) {
  if (n <= 1) return hipSuccess;
  const int ntile = nblocks(n, RS_TILE);
  hipError_t e = t.k2.ensure((size_t)n);
  if (e == hipSuccess && vals) e = t.v2.ensure((size_t)n);
  if (e == hipSuccess) e = t.cnt.ensure((size_t)RS_DIGITS * ntile);
  if (e == hipSuccess) e = t.off.ensure((size_t)RS_DIGITS * ntile);
  if (e != hipSuccess) return e;
  for (int shift = 0; shift < bits; shift += 4) {
    hipLaunchKernelGGL(k_rs_count, dim3(ntile), dim3(TB), 0, s, keys.p, n, shift, t.cnt.p, ntile);
    e = scan_excl(s, t.cnt.p, t.off.p, (int64_t)RS_DIGITS * ntile, t.scan);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rs_scatter, dim3(ntile), dim3(TB), 0, s, keys.p, vals ? vals->p : nullptr, t.k2.p,
                       vals ? t.v2.p : nullptr, n, shift, t.off.p, ntile);
    std::swap(keys, t.k2);
    if (vals) std::swap(*vals, t.v2);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- tree
// the splitting rule (see TreeParams); per-level parts precomputed on the host
__device__ inline bool box_splits(int cnt, int iy, int level, int leaf_size, int kb_on, int kb_all, int refine,
                                  int maxl) {
  bool split = cnt > leaf_size;
  if (kb_on) {
    const int quarter = leaf_size / 4 > 1 ? leaf_size / 4 : 1;
    if (cnt > quarter || kb_all) split = true;
  }
  if (refine && iy == 0 && cnt > 1) split = true;
  if (level >= maxl) split = false;
  return split;
}

__global__ void k_tree_split(const Box* __restrict__ B, int lb, int m, const uint64_t* __restrict__ keys, int level,
                             int leaf_size, int kb_on, int kb_all, int refine, int maxl, int* __restrict__ nchild,
                             int* __restrict__ bnd) {
  const int i = blockIdx.x * TB + threadIdx.x;
  if (i >= m) return;
  const Box b = B[lb + i];
  int nc = 0;
  if (box_splits(b.end - b.begin, b.iy, level, leaf_size, kb_on, kb_all, refine, maxl)) {
    const int shift = 2 * (KEY_BITS - level - 1);
    int e[5];
    e[0] = b.begin;
    e[4] = b.end;
    for (int q = 1; q < 4; ++q) {
      // the first point of the box whose quadrant digit is >= q
      int lo = b.begin, hi = b.end;
      while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if ((int)((keys[mid] >> shift) & 3u) < q)
          lo = mid + 1;
        else
          hi = mid;
      }
      e[q] = lo;
    }
    for (int q = 0; q < 5; ++q) bnd[5 * i + q] = e[q];
    for (int q = 0; q < 4; ++q) nc += e[q + 1] > e[q] ? 1 : 0;
  }
  nchild[i] = nc;
}

__global__ void k_tree_children(Box* __restrict__ B, int lb, int m, int le, int level, const int* __restrict__ nchild,
                                const int* __restrict__ cbase, const int* __restrict__ bnd) {
  const int i = blockIdx.x * TB + threadIdx.x;
  if (i >= m || nchild[i] == 0) return;
  Box p = B[lb + i];
  int idx = le + cbase[i];
  for (int q = 0; q < 4; ++q) {
    const int s = bnd[5 * i + q], e = bnd[5 * i + q + 1];
    if (e > s) {
      Box c;
      c.level = level + 1;
      c.ix = 2 * p.ix + (q & 1);
      c.iy = 2 * p.iy + (q >> 1);
      c.begin = s;
      c.end = e;
      c.parent = lb + i;
      c.quad = q;
      for (int a = 0; a < 4; ++a) c.child[a] = -1;
      c.leaf = 1;
      B[idx] = c;
      p.child[q] = idx;
      ++idx;
    }
  }
  p.leaf = 0;
  B[lb + i] = p;
}

// ---------------------------------------------------------------- pair lists
// class of a pair: 0 admissible (far list), 1 near list, 2 expanded into the
// pairs of the children. mode 0: free (not adjacent); mode 1: image (the
// target separated from the source's mirror image: iy_t + iy_s >= 1, or every
// pair of the level when 2 y0 >= b, img_all).
__device__ inline int pair_class(const Box& t, const Box& s, int mode, int top, int img_all) {
  bool adm;
  if (mode == 0) {
    const int dx = t.ix - s.ix, dy = t.iy - s.iy;
    adm = !(dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) && t.level >= top;
  } else {
    adm = t.level >= top && (t.iy + s.iy >= 1 || img_all);
  }
  if (adm) return 0;
  if (t.leaf || s.leaf) return 1;
  return 2;
}

__device__ inline int nkids(const Box& b) {
  int c = 0;
  for (int q = 0; q < 4; ++q) c += b.child[q] >= 0 ? 1 : 0;
  return c;
}

// counts of the level's pairs: [0] far, [1] near, [2] children pairs
__global__ void __launch_bounds__(TB) k_pairs_count(const Box* __restrict__ B, const TreePair* __restrict__ F, int m,
                                                    int mode, int top, int img_all, int* __restrict__ cnt) {
  const int i = blockIdx.x * TB + threadIdx.x;
  int c0 = 0, c1 = 0, c2 = 0;
  if (i < m) {
    const Box t = B[F[i].t], s = B[F[i].s];
    const int c = pair_class(t, s, mode, top, img_all);
    if (c == 0) c0 = 1;
    else if (c == 1) c1 = 1;
    else c2 = nkids(t) * nkids(s);
  }
  int e;
  const int t0 = block_excl_scan(c0, e);
  const int t1 = block_excl_scan(c1, e);
  const int t2 = block_excl_scan(c2, e);
  if (threadIdx.x == 0) {
    if (t0) atomicAdd(cnt + 0, t0);
    if (t1) atomicAdd(cnt + 1, t1);
    if (t2) atomicAdd(cnt + 2, t2);
  }
}

// writes the level's far / near pairs after the lists' current ends and the
// children pairs into the next frontier; pos[0..2] are the running ends
__global__ void __launch_bounds__(TB) k_pairs_emit(const Box* __restrict__ B, const TreePair* __restrict__ F, int m,
                                                   int mode, int top, int img_all, TreePair* __restrict__ far,
                                                   TreePair* __restrict__ near, TreePair* __restrict__ next,
                                                   int* __restrict__ pos) {
  __shared__ int base[3];
  const int i = blockIdx.x * TB + threadIdx.x;
  int cls = -1, c0 = 0, c1 = 0, c2 = 0;
  Box t, s;
  if (i < m) {
    t = B[F[i].t];
    s = B[F[i].s];
    cls = pair_class(t, s, mode, top, img_all);
    if (cls == 0) c0 = 1;
    else if (cls == 1) c1 = 1;
    else c2 = nkids(t) * nkids(s);
  }
  int e0, e1, e2;
  const int t0 = block_excl_scan(c0, e0);
  const int t1 = block_excl_scan(c1, e1);
  const int t2 = block_excl_scan(c2, e2);
  if (threadIdx.x == 0) {
    base[0] = t0 ? atomicAdd(pos + 0, t0) : 0;
    base[1] = t1 ? atomicAdd(pos + 1, t1) : 0;
    base[2] = t2 ? atomicAdd(pos + 2, t2) : 0;
  }
  __syncthreads();
  if (cls == 0) far[base[0] + e0] = F[i];
  if (cls == 1) near[base[1] + e1] = F[i];
  if (cls == 2) {
    int o = base[2] + e2;
    for (int a = 0; a < 4; ++a) {
      if (t.child[a] < 0) continue;
      for (int c = 0; c < 4; ++c)
        if (s.child[c] >= 0) next[o++] = TreePair{t.child[a], s.child[c]};
    }
  }
}

__global__ void k_pair_keys(const TreePair* __restrict__ P, int64_t m, int sbits, uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < m) keys[i] = ((uint64_t)(uint32_t)P[i].t << sbits) | (uint64_t)(uint32_t)P[i].s;
}

__global__ void k_pair_decode(const uint64_t* __restrict__ keys, int64_t m, int sbits, TreePair* __restrict__ P) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < m) {
    const uint64_t k = keys[i];
    P[i] = TreePair{(int)(k >> sbits), (int)(k & ((1ull << sbits) - 1ull))};
  }
}

// grows buf to hold count elements, keeping its first keep elements
template <class T>
hipError_t grow_keep(DevBuf<T>& buf, size_t count, size_t keep, hipStream_t s) {
  if (buf.p && buf.n >= count) return hipSuccess;
  DevBuf<T> nb;
  hipError_t e = nb.alloc(std::max(count, 2 * buf.n));
  if (e == hipSuccess && keep > 0) e = hipMemcpyAsync(nb.p, buf.p, keep * sizeof(T), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) {
    nb.release();
    return e;
  }
  // the copy must finish before the old buffer is freed
  e = hipStreamSynchronize(s);
  std::swap(buf, nb);
  nb.release();
  return e;
}

}  // namespace

void gpu_tree_build(const TreeParams& p, const double* d_points, hipStream_t s, bool copy_keys, TreeOut& out,
                    TreeDev& dev) {
  out = TreeOut{};
  const int64_t n = p.n;
  const double2* pts = (const double2*)d_points;
  auto failed = [&](hipError_t e, const char* what) {
    if (e == hipSuccess) return false;
    out.status = e == hipErrorOutOfMemory ? TREE_MEMORY : TREE_DEVICE;
    out.msg = std::string("tree build, ") + what + ": " + hipGetErrorString(e);
    return true;
  };
#define TREE_TRY(expr, what) \
  if (failed((expr), what)) return
  // ---- 1. frame
  const int npart = std::max(1, std::min(1024, nblocks(n, TB)));
  DevBuf<FrameRed> fr;
  TREE_TRY(fr.alloc((size_t)npart + 1), "frame");
  hipLaunchKernelGGL(k_frame, dim3(npart), dim3(TB), 0, s, pts, n, p.y_top, fr.p);
  hipLaunchKernelGGL(k_frame_final, dim3(1), dim3(TB), 0, s, fr.p, npart, n, fr.p + npart);
  FrameRed hf;
  TREE_TRY(hipMemcpyAsync(&hf, fr.p + npart, sizeof(FrameRed), hipMemcpyDeviceToHost, s), "frame");
  TREE_TRY(hipStreamSynchronize(s), "frame");
  if (hf.bad < n) {
    double2 v;
    TREE_TRY(hipMemcpy(&v, pts + hf.bad, sizeof(double2), hipMemcpyDeviceToHost), "frame");
    const double y = v.y - p.y_top;
    out.status = TREE_DOMAIN;
    out.msg = (!std::isfinite(v.x) || !std::isfinite(y))
                  ? "non-finite point " + std::to_string(hf.bad)
                  : "point " + std::to_string(hf.bad) + " is not strictly above the top interface";
    return;
  }
  const double S = tree_root_side(hf.xmin, hf.xmax, hf.ymin, hf.ymax);
  const double ymin = hf.ymin;
  out.S = S;
  out.x0 = hf.xmin;
  out.y0 = ymin;
  // ---- 2. keys and the sort
  TREE_TRY(dev.keys.alloc((size_t)n), "keys");
  TREE_TRY(dev.perm.alloc((size_t)n), "keys");
  hipLaunchKernelGGL(k_morton, dim3(nblocks(n, TB)), dim3(TB), 0, s, pts, n, p.y_top, hf.xmin, ymin,
                     (double)(1u << KEY_BITS) / S, dev.keys.p, dev.perm.p);
  SortTmp st;
  TREE_TRY(radix_sort(s, dev.keys, &dev.perm, n, 2 * KEY_BITS, st), "radix sort");
  st.k2.release();
  st.v2.release();
  DevBuf<int> cnt;
  TREE_TRY(cnt.alloc(8), "counters");
  TREE_TRY(hipMemsetAsync(cnt.p, 0, 8 * sizeof(int), s), "counters");
  hipLaunchKernelGGL(k_count_dups, dim3(nblocks(n, TB)), dim3(TB), 0, s, dev.keys.p, n, cnt.p);
  int ndup = 0;
  TREE_TRY(hipMemcpyAsync(&ndup, cnt.p, sizeof(int), hipMemcpyDeviceToHost, s), "duplicates");
  out.perm.resize((size_t)n);
  TREE_TRY(hipMemcpyAsync(out.perm.data(), dev.perm.p, sizeof(int) * n, hipMemcpyDeviceToHost, s), "perm");
  TREE_TRY(hipStreamSynchronize(s), "perm");
  if (copy_keys || ndup > 0) {
    out.keys.resize((size_t)n);
    TREE_TRY(hipMemcpy(out.keys.data(), dev.keys.p, sizeof(uint64_t) * n, hipMemcpyDeviceToHost), "keys");
  }
  if (ndup > 0) {
    // runs of equal keys: compare their points after sorting each run by
    // (x, y) (rare: the grid cell is 2^-30 of the root side)
    std::vector<double2> hp((size_t)n);
    TREE_TRY(hipMemcpy(hp.data(), pts, sizeof(double2) * n, hipMemcpyDeviceToHost), "points");
    std::vector<std::pair<std::pair<double, double>, int>> run;
    for (int64_t i = 0; i < n;) {
      int64_t e = i + 1;
      while (e < n && out.keys[e] == out.keys[i]) ++e;
      if (e - i > 1) {
        run.clear();
        for (int64_t t = i; t < e; ++t) {
          const int a = out.perm[t];
          run.push_back({{hp[a].x, hp[a].y - p.y_top}, a});
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
    if (!copy_keys) std::vector<uint64_t>().swap(out.keys);
  }
  // ---- 3. the tree, level by level
  DevBuf<Box> B;
  TREE_TRY(B.alloc((size_t)std::max<int64_t>(64, n / 8)), "boxes");
  const Box root{0, 0, 0, 0, (int)n, -1, 0, {-1, -1, -1, -1}, 1};
  TREE_TRY(hipMemcpyAsync(B.p, &root, sizeof(Box), hipMemcpyHostToDevice, s), "boxes");
  DevBuf<int> nchild, cbase, bnd;
  ScanTmp scan;
  int nboxes = 1;
  out.lev_begin.push_back(0);
  const int maxl = std::min(p.max_level, KEY_BITS);
  for (int l = 0;; ++l) {
    const int lb = out.lev_begin[l], le = nboxes, m = le - lb;
    const double b = S / (double)(1u << l);
    out.bsize.push_back(b);
    const int kb_on = p.leaf_kb > 0.0 && p.k * b > p.leaf_kb;
    const int kb_all = p.k * b > 2.0 * p.leaf_kb;
    const int refine = p.interface_refine && 2.0 * ymin < b;
    TREE_TRY(nchild.ensure((size_t)m), "tree");
    TREE_TRY(cbase.ensure((size_t)m), "tree");
    TREE_TRY(bnd.ensure((size_t)5 * m), "tree");
    hipLaunchKernelGGL(k_tree_split, dim3(nblocks(m, TB)), dim3(TB), 0, s, B.p, lb, m, dev.keys.p, l, p.leaf_size,
                       kb_on, kb_all, refine, maxl, nchild.p, bnd.p);
    TREE_TRY(scan_excl(s, nchild.p, cbase.p, m, scan), "tree scan");
    hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(64), 0, s, nchild.p, cbase.p, (int64_t)m, cnt.p);
    int total = 0;
    TREE_TRY(hipMemcpyAsync(&total, cnt.p, sizeof(int), hipMemcpyDeviceToHost, s), "tree");
    TREE_TRY(hipStreamSynchronize(s), "tree");
    if (total == 0) break;
    TREE_TRY(grow_keep(B, (size_t)le + total, (size_t)le, s), "boxes");
    hipLaunchKernelGGL(k_tree_children, dim3(nblocks(m, TB)), dim3(TB), 0, s, B.p, lb, m, le, l, nchild.p, cbase.p,
                       bnd.p);
    nboxes = le + total;
    out.lev_begin.push_back(le);
  }
  out.nlev = (int)out.lev_begin.size();
  out.lev_begin.push_back(nboxes);
  out.boxes.resize((size_t)nboxes);
  TREE_TRY(hipMemcpyAsync(out.boxes.data(), B.p, sizeof(Box) * nboxes, hipMemcpyDeviceToHost, s), "boxes");
  TREE_TRY(hipStreamSynchronize(s), "boxes");
  if (out.nlev > kTreeMaxLevels) {
    out.status = TREE_DEPTH;
    out.msg = "tree deeper than supported";
    return;
  }
  out.top = tree_top_level(out, p.top_level);
  // ---- 4. the pair lists
  int sbits = 1;
  while ((1ll << sbits) <= nboxes) ++sbits;
  for (int mode = 0; mode < 2; ++mode) {
    DevBuf<TreePair> F, Fn, far, near;
    TREE_TRY(F.alloc(1), "lists");
    const TreePair rootp{0, 0};
    TREE_TRY(hipMemcpyAsync(F.p, &rootp, sizeof(TreePair), hipMemcpyHostToDevice, s), "lists");
    int m = 1, nfar = 0, nnear = 0;
    for (int l = 0; m > 0; ++l) {
      const int img_all = 2.0 * ymin >= out.bsize[std::min(l, out.nlev - 1)];
      TREE_TRY(hipMemsetAsync(cnt.p, 0, 3 * sizeof(int), s), "lists");
      hipLaunchKernelGGL(k_pairs_count, dim3(nblocks(m, TB)), dim3(TB), 0, s, B.p, F.p, m, mode, out.top, img_all,
                         cnt.p);
      int c[3];
      TREE_TRY(hipMemcpyAsync(c, cnt.p, 3 * sizeof(int), hipMemcpyDeviceToHost, s), "lists");
      TREE_TRY(hipStreamSynchronize(s), "lists");
      TREE_TRY(grow_keep(far, (size_t)nfar + c[0] + 1, (size_t)nfar, s), "lists");
      TREE_TRY(grow_keep(near, (size_t)nnear + c[1] + 1, (size_t)nnear, s), "lists");
      TREE_TRY(Fn.ensure((size_t)c[2] + 1), "lists");
      const int pos[3] = {nfar, nnear, 0};
      TREE_TRY(hipMemcpyAsync(cnt.p, pos, 3 * sizeof(int), hipMemcpyHostToDevice, s), "lists");
      hipLaunchKernelGGL(k_pairs_emit, dim3(nblocks(m, TB)), dim3(TB), 0, s, B.p, F.p, m, mode, out.top, img_all,
                         far.p, near.p, Fn.p, cnt.p);
      nfar += c[0];
      nnear += c[1];
      m = c[2];
      std::swap(F, Fn);
    }
    // canonical order: sorted by (t, s)
    DevBuf<TreePair>* lists[2] = {&far, &near};
    std::vector<TreePair>* outs[2] = {mode == 0 ? &out.fv : &out.iv, mode == 0 ? &out.fu : &out.iu};
    const int cnts[2] = {nfar, nnear};
    for (int w = 0; w < 2; ++w) {
      const int64_t cm = cnts[w];
      outs[w]->resize((size_t)cm);
      if (cm == 0) continue;
      DevBuf<uint64_t> pk;
      TREE_TRY(pk.alloc((size_t)cm), "lists");
      hipLaunchKernelGGL(k_pair_keys, dim3(nblocks(cm, TB)), dim3(TB), 0, s, lists[w]->p, cm, sbits, pk.p);
      TREE_TRY(radix_sort(s, pk, nullptr, cm, 2 * sbits, st), "list sort");
      hipLaunchKernelGGL(k_pair_decode, dim3(nblocks(cm, TB)), dim3(TB), 0, s, pk.p, cm, sbits, lists[w]->p);
      TREE_TRY(hipMemcpyAsync(outs[w]->data(), lists[w]->p, sizeof(TreePair) * cm, hipMemcpyDeviceToHost, s),
               "lists");
      TREE_TRY(hipStreamSynchronize(s), "lists");
    }
  }
  TREE_TRY(hipGetLastError(), "tree kernels");
#undef TREE_TRY
}

}  // namespace hfmm
