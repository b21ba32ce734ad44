// C interface of the tree builders (hfmm_tree_*): the plan's quadtree and
// interaction lists for inspection and tests.
#include "../../include/hfmm.h"
#include "plan_internal.hpp"
#include "tree_gpu.hpp"

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

struct hfmm_tree_s {
  hfmm::TreeOut t;
};

extern "C" {

hfmm_status_t hfmm_tree_build(hfmm_tree_t* out, const double* wavenumbers, const double* interfaces, int64_t n,
                              const double* points, const hfmm_options_t* opts, int32_t builder,
                              hfmm_stream_t stream) {
  using namespace hfmm;
  if (!out) return report(HFMM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!wavenumbers || !interfaces || !points) return report(HFMM_ERR_INVALID_ARG, "NULL wavenumbers, interfaces or points");
  if (n < 1 || n > (int64_t)1 << 30) return report(HFMM_ERR_INVALID_ARG, "n out of range");
  if (builder != HFMM_TREE_GPU && builder != HFMM_TREE_HOST)
    return report(HFMM_ERR_INVALID_ARG, "builder must be HFMM_TREE_GPU or HFMM_TREE_HOST");
  hfmm_options_t o;
  hfmm_default_options(&o);
  if (opts) {
    if (opts->struct_size != (int32_t)sizeof(hfmm_options_t))
      return report(HFMM_ERR_INVALID_ARG, "options struct_size mismatch");
    o = *opts;
  }
  if (o.leaf_size < 1 || o.leaf_size > 4096) return report(HFMM_ERR_INVALID_ARG, "leaf_size out of range");
  if (o.max_level < 2 || o.max_level > KEY_BITS) return report(HFMM_ERR_INVALID_ARG, "max_level out of range");
  if (!(o.leaf_kb == 0.0 || (o.leaf_kb >= 0.25 && std::isfinite(o.leaf_kb))))
    return report(HFMM_ERR_INVALID_ARG, "leaf_kb must be 0 or a finite value >= 0.25");
  if (o.top_level != 0 && (o.top_level < 2 || o.top_level > KEY_BITS))
    return report(HFMM_ERR_INVALID_ARG, "top_level must be 0 or in [2, 30]");
  if (!(wavenumbers[0] > 0.0) || !std::isfinite(wavenumbers[0]) || !std::isfinite(interfaces[0]))
    return report(HFMM_ERR_INVALID_ARG, "the wavenumber must be finite and > 0, the interface finite");
  TreeParams tp;
  tp.n = n;
  tp.y_top = interfaces[0];
  tp.k = wavenumbers[0];
  tp.leaf_size = o.leaf_size;
  tp.leaf_kb = o.leaf_kb;
  tp.interface_refine = o.interface_refine;
  tp.max_level = o.max_level;
  tp.top_level = o.top_level;
  hfmm_tree_s* t = new hfmm_tree_s();
  hipStream_t s = (hipStream_t)stream;
  if (builder == HFMM_TREE_GPU) {
    Allocator al{o.alloc, o.free, o.alloc_ctx};
    AllocScope scope(&al);
    TreeDev dev;
    gpu_tree_build(tp, points, s, true, t->t, dev);
  } else {
    std::vector<double> hp((size_t)2 * n);
    hipError_t e = hipMemcpyAsync(hp.data(), points, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      delete t;
      return report(HFMM_ERR_DEVICE, std::string("copying points: ") + hipGetErrorString(e));
    }
    host_tree_build(tp, hp.data(), t->t);
  }
  if (t->t.status != TREE_OK) {
    const hfmm_status_t st = t->t.status == TREE_DOMAIN   ? HFMM_ERR_DOMAIN
                             : t->t.status == TREE_DEPTH  ? HFMM_ERR_ACCURACY
                             : t->t.status == TREE_MEMORY ? HFMM_ERR_NO_MEMORY
                                                          : HFMM_ERR_DEVICE;
    const std::string msg = t->t.msg;
    delete t;
    return report(st, msg);
  }
  *out = t;
  return HFMM_OK;
}

hfmm_status_t hfmm_tree_counts(hfmm_tree_t tree, int64_t counts[8]) {
  if (!tree || !counts) return hfmm::report(HFMM_ERR_INVALID_ARG, "NULL tree or counts");
  const hfmm::TreeOut& t = tree->t;
  counts[0] = (int64_t)t.perm.size();
  counts[1] = (int64_t)t.boxes.size();
  counts[2] = t.nlev;
  counts[3] = t.top;
  counts[4] = (int64_t)t.fv.size();
  counts[5] = (int64_t)t.iv.size();
  counts[6] = (int64_t)t.fu.size();
  counts[7] = (int64_t)t.iu.size();
  return HFMM_OK;
}

hfmm_status_t hfmm_tree_copy(hfmm_tree_t tree, double* frame, uint64_t* keys, int32_t* perm, int32_t* boxes,
                             int32_t* lev_begin, int32_t* fv, int32_t* iv, int32_t* fu, int32_t* iu) {
  if (!tree) return hfmm::report(HFMM_ERR_INVALID_ARG, "NULL tree");
  const hfmm::TreeOut& t = tree->t;
  static_assert(sizeof(hfmm::Box) == 12 * sizeof(int32_t), "a box is 12 int32");
  static_assert(sizeof(hfmm::TreePair) == 2 * sizeof(int32_t), "a pair is 2 int32");
  if (frame) {
    frame[0] = t.S;
    frame[1] = t.x0;
    frame[2] = t.y0;
  }
  if (keys && !t.keys.empty()) std::memcpy(keys, t.keys.data(), t.keys.size() * sizeof(uint64_t));
  if (perm && !t.perm.empty()) std::memcpy(perm, t.perm.data(), t.perm.size() * sizeof(int32_t));
  if (boxes && !t.boxes.empty()) std::memcpy(boxes, t.boxes.data(), t.boxes.size() * sizeof(hfmm::Box));
  if (lev_begin) std::memcpy(lev_begin, t.lev_begin.data(), t.lev_begin.size() * sizeof(int32_t));
  const std::vector<hfmm::TreePair>* lists[4] = {&t.fv, &t.iv, &t.fu, &t.iu};
  int32_t* dst[4] = {fv, iv, fu, iu};
  for (int w = 0; w < 4; ++w)
    if (dst[w] && !lists[w]->empty()) std::memcpy(dst[w], lists[w]->data(), lists[w]->size() * sizeof(hfmm::TreePair));
  return HFMM_OK;
}

void hfmm_tree_destroy(hfmm_tree_t tree) { delete tree; }

}  // extern "C"
