// Host side of the layered-media heterogeneous FMM: the C interface, the plan
// (tree, interaction lists, expansion orders, quadrature rules, tables) and the
// apply / adjoint pipelines (Algorithm 1 of the paper).
//
// Interaction structure. The free-space part follows the classical FMM on the
// adaptive quadtree (Section 3.1): same-level pairs that are not adjacent get a
// multipole-to-local translation (V list), adjacent pairs involving a leaf are
// evaluated directly. The scattered part uses the same multipoles through the
// heterogeneous M2L (Section 3.3 / Section 5), but it is paired with the mirror
// images of the source boxes: a pair of boxes at a level is "image admissible"
// when Y = y_t + y_s >= 2b (centres, interface frame, box side b), i.e. the
// mirrored source box is at least one box away from the target box. Admissible
// pairs are translated at the coarsest level (>= 2) where they become
// admissible; pairs that are still not admissible at the leaves are evaluated
// by direct Sommerfeld quadrature (Section 5, local direct interactions,
// strategy (b)). Keeping Y >= 2b also keeps the FP64 Sommerfeld quadrature of
// the heterogeneous tables well conditioned at every order the level uses.
#include "../../include/hfmm.h"
#include "blocked.hpp"
#include "devbuf.hpp"
#include "kernels.hpp"
#include "plan_internal.hpp"
#include "tree_gpu.hpp"
#include "special.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

using namespace hfmm;

namespace {

thread_local std::string g_err;

hfmm_status_t fail(hfmm_status_t s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(HFMM_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)


// 16-point Gauss-Legendre rule on [-1, 1] by Newton iteration on P_16.
void gauss_legendre16(double* x, double* w) {
  const int n = 16;
  auto legendre = [&](double z, double& pn, double& dpn) {
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    pn = p1;
    dpn = n * (z * p1 - p0) / (z * z - 1.0);
  };
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double pn, dpn;
    for (int it = 0; it < 100; ++it) {
      legendre(z, pn, dpn);
      double dz = pn / dpn;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    legendre(z, pn, dpn);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dpn * dpn);
  }
}

// |J_n(x)| and |Y_n(x)| for the order selection (host, FP64).
double host_absj(double x, int n) {
  double out = 0.0;
  bessel_j_each(x, n, [&](int m, double j) {
    if (m == n) out = std::fabs(j);
  });
  return out;
}
// log10 |Y_n(x)| by forward recurrence (may exceed the double range in value).
double host_log10_absy(double x, int n) {
  double ym1 = ::y0(x), yn = ::y1(x);
  if (n == 0) return std::log10(std::fabs(ym1));
  double lscale = 0.0;
  for (int m = 1; m < n; ++m) {
    double yp1 = (2.0 * m / x) * yn - ym1;
    ym1 = yn;
    yn = yp1;
    if (std::fabs(yn) > 1e200) {
      yn *= 1e-200;
      ym1 *= 1e-200;
      lscale += 200.0;
    }
  }
  return lscale + std::log10(std::fabs(yn));
}

// Quadrature rule of the Sommerfeld integrals for one translation (or for the
// direct near-interface pairs with N = 0): panels for the tau part and the
// evanescent t part, with the t contour dipping below the real axis over the
// branch points sqrt(k_j^2 - k1^2) and the guided-mode poles between them.
struct Rule {
  std::vector<Panel> panels;
  double dip = 0.0, send = 1.0;
  bool ok = true;
};
constexpr size_t kMaxPanels = 100000;
constexpr int kItemSources = 2048;   // at most this many sources per direct work item
// and about this many pairs, by series class: the longer series have fewer
// items per launch, so their items are smaller, which spreads each class
// launch over the GPU instead of ending it with a few long waves
constexpr int kItemPairs[kH0Classes + 1] = {8192, 8192, 8192, 4096, 2048, 2048};
// per-translation truncation bound as a fraction of the requested tolerance
#ifndef HFMM_ORDER_SAFETY
#define HFMM_ORDER_SAFETY 0.5
#endif
constexpr double kOrderSafety = HFMM_ORDER_SAFETY;
// largest expansion order: the batched M2L keeps a 16-pair operand tile of
// 2P+1 coefficients and the 4P+1 table entries in LDS
constexpr int kMaxOrder = 255;
constexpr int kScaleStride = kMaxOrder + 1;  // scale factors per level
constexpr int kUpDownNt = 8;  // row tiles per item of the blocked M2M and L2L
// Launch shaping: the CUs of the GPU (MI355X: 256), the LDS of one CU, and the
// most dynamic LDS a translation block may take (the CU's less the kernel's
// static offsets).
constexpr int64_t kNumCu = 256;
constexpr size_t kCuLds = 160 * 1024;
constexpr size_t kSplitLdsMax = kCuLds - 1024;

// cut: the t range ends where the integrand has fallen by e^-cut from its
// largest value (44 by default, below double precision)
// phase: radians of phase per 16-point panel (4 for the tables; the direct
// near-interface nodes, applied at every call, take 8: Gauss-Legendre
// integrates e^{i phi} over 8 radians to about 1e-16)
Rule build_rule(const Medium& m, double xmax, double ymin, double ymax, int N, double cut = 44.0,
                double phase = 4.0) {
  Rule r;
  const double k = m.k1;
  xmax = std::fabs(xmax);
  double rho = std::hypot(xmax, ymax);
  // tau part: the phase k (Y sin tau - X cos tau) - n tau changes by at most
  // k rho + N per unit tau (plus the slab's, below); <= 4 radians per 16-point
  // panel.
  {
    double kmin_over = 1e300;
    for (double kj : {m.k2, m.k3})
      if (kj > k) kmin_over = std::min(kmin_over, std::sqrt(kj * kj - k * k) / k);
    double eps = (kmin_over < 1e299) ? kmin_over : 1.0;  // scale of sigma near tau = 0, pi
    // the impedance sigma-hat turns from -1 at tau = 0 over k sin(tau) ~ alpha
    if (m.layers == 1) eps = std::min(1.0, m.alpha / k);
    // three layers: sigma_1 carries the slab round trip e^{-2 gamma_2 d}, whose
    // phase 2 d sqrt(k2^2 - k1^2 cos^2 tau) turns at up to
    // min(d k1^2 / sqrt(k2^2 - k1^2), 2 d k1) per unit tau
    double slab = 0.0;
    if (m.layers == 3 && m.k2 > k) slab = std::min(m.d * k * k / std::sqrt(m.k2 * m.k2 - k * k), 2.0 * m.d * k);
    double wmax = std::min(phase / (k * rho + N + 1.0 + slab), M_PI / 4.0);
    double s = 0.0;
    while (s < M_PI) {
      double dist = std::min(s, M_PI - s);
      double w = std::min(wmax, 0.5 * (dist + eps));
      double e = std::min(M_PI, s + w);
      if (M_PI - e < 1e-3 * w) e = M_PI;
      r.panels.push_back({s, e, 0, 0});
      s = e;
    }
  }
  // t part
  double tj[2];
  int nsing = 0;
  for (double kj : {m.k2, m.k3})
    if (kj > k) tj[nsing++] = std::sqrt(kj * kj - k * k);
  double tsmax = 0.0, tsmin = 1e300;
  for (int i = 0; i < nsing; ++i) {
    tsmax = std::max(tsmax, tj[i]);
    tsmin = std::min(tsmin, tj[i]);
  }
  if (nsing) {
    r.send = 1.25 * tsmax + 1.0;
    r.dip = std::min(1.0 / std::max(xmax, 1e-9), 0.15 * r.send);
  } else {
    r.send = 1.0;
    r.dip = 0.0;
  }
  // end of the t range: log|z^{-N} e^{-t Y}| = -t Y + N log((t + lambda)/k)
  auto f = [&](double t) { return -t * ymin + N * std::log((t + std::sqrt(t * t + k * k)) / k); };
  double tpk = 0.0, fmaxv = f(0.0);
  if (N > 0) {
    // maximiser: N / lambda = Y  => lambda = N / Y
    double lam = N / ymin;
    if (lam > k) {
      tpk = std::sqrt(lam * lam - k * k);
      fmaxv = f(tpk);
    }
  }
  double tend = std::max(tpk, 1.0);
  while (f(tend) > fmaxv - cut) tend *= 1.25;
  tend = std::max(tend, r.send + 1.0);
  const double rate = ymax + xmax + (double)N / k;
  const double wcap = std::max(phase / rate, 1e-6);
  auto width = [&](double s) {
    double w = wcap;
    double h = (s < r.send) ? r.dip * std::sin(M_PI * s / r.send) : 0.0;
    for (int i = 0; i < nsing; ++i) w = std::min(w, 0.5 * std::hypot(s - tj[i], h));
    // the impedance sigma-hat's pole at t = i alpha
    if (m.layers == 1) w = std::min(w, 0.5 * std::hypot(s, m.alpha));
    if (m.layers == 3 && nsing && s > tsmin - 1.0 && s < tsmax + 1.0) w = std::min(w, 0.5 * std::max(h, 1e-6));
    return std::max(w, 1e-6);
  };
  double s = 0.0;
  for (double stop : {r.send, tend}) {
    if (stop <= s) continue;
    while (s < stop) {
      double w = width(s);
      w = std::min(w, 1.5 * width(std::min(s + w, stop)));
      double e = std::min(stop, s + w);
      if (stop - e < 1e-3 * w) e = stop;
      r.panels.push_back({s, e, 1, 0});
      s = e;
      if (r.panels.size() > kMaxPanels) {
        r.ok = false;
        return r;
      }
    }
  }
  return r;
}

}  // namespace

// fn(i) for i in [0, n) on up to 16 host threads (plan-time work whose items
// are independent; each item writes only its own slot)
template <class F>
void parallel_for(int n, F fn) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nt = std::min({hw, 16, std::max(1, n / 8)});
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (int i = next.fetch_add(1); i < n; i = next.fetch_add(1)) fn(i);
    });
  for (auto& t : th) t.join();
}

struct hfmm_plan_s {
  Allocator al{};  // where the plan's device memory comes from
  Medium med{};
  double y_top = 0.0;
  int n = 0;
  double tol = 0.0;
  hfmm_options_t opt{};
  int nlev = 0;
  int top = 2;  // coarsest level of the expansions
  double S = 1.0, x0 = 0.0, y0 = 0.0;
  int P[HFMM_MAX_LEVELS] = {0};
  double bsize[HFMM_MAX_LEVELS] = {0};
  std::vector<Box> boxes;
  std::vector<int> lev_begin;   // boxes of level l: [lev_begin[l], lev_begin[l+1])
  int64_t ctot = 0;

  DevBuf<double2> pts, ctr;
  DevBuf<int> perm, level, parent, quad, child;
  DevBuf<int2> prange;
  DevBuf<int64_t> coff;
  DevBuf<int> leaves;  // leaf boxes, ascending level
  DevBuf<int> pt_box;  // leaf box of each sorted point
  int precision = HFMM_FP64;  // HFMM_FP64 or HFMM_FP32 (near field in single precision)
  int nleaves = 0;
  std::vector<int> leaf_lev;  // leaves of level l: [leaf_lev[l], leaf_lev[l + 1])
  int leaf_pmax = 0;          // largest expansion order among the leaves
  // batched translations: item groups, one launch each (M2M / L2L: per level;
  // M2L: runs of consecutive levels); Ps, Pd: the largest orders of the items
  struct Group {
    int first = 0, count = 0, Ps = 0, Pd = 0, ntw = 8;  // ntw: row tiles per wave of the items
    int max_rhs = 0;  // split gather: the most right-hand sides whose blocks fit the GPU at once
  };
  // M2L: items, (source, target) pair arrays, contribution row offsets, and the
  // per-box lists of pairs for the reduction by target (forward) / by source
  DevBuf<TransItem> m2l_items;
  DevBuf<int64_t> m2l_soff, m2l_toff;  // coefficient offsets of each pair's source / target box
  DevBuf<int64_t> m2l_pcoff, m2l_pcoffT;  // row offsets: grouped by target box / by source box
  std::vector<Group> m2l_groups;
  int64_t cstride = 0;  // contribution doubles per right-hand side
  // reductions: boxes of levels >= 2, pair counts per box (CSR) by target and
  // by source, and where each box's rows begin
  DevBuf<int> red_boxes, red_ptr, redT_ptr;
  DevBuf<int64_t> red_beg, redT_beg;
  int nred_boxes = 0;
  // M2M / L2L: (child, parent) pairs grouped by parent level and quadrant;
  // items shaped child -> parent (up) and parent -> child (down), by parent level
  DevBuf<int64_t> cp_child, cp_parent;  // coefficient offsets of each pair's child / parent box
  DevBuf<int64_t> up_doff, up_soff4;     // child -> parent: parent offsets, and their four children's (-1: none)
  std::vector<Toff4> m2m_q4, l2l_q4;      // per parent level: the four tables' offsets
  DevBuf<TransItem> up_items, down_items;
  std::vector<Group> up_groups, down_groups;
  // small up levels: the same parents as items of the split gather (a child
  // quadrant per wave, one row tile per item), used when the stages run in
  // sequence; count 0 where the standard form is kept
  std::vector<Group> up_split_groups;
  DevBuf<double> contrib;
  DevBuf<TableRef> tabs;
  DevBuf<double2> tdata;
  std::vector<int> m2m_tab, l2l_tab;  // per parent level: index of 4 consecutive tables
  DevBuf<int> p2p_ptr, p2p_items, p2p_sym;
  bool p2p_symmetric = false;  // cross items evaluate each pair once
  int64_t p2p_evals = 0;       // H0 evaluations per apply
  double p2p_flops = 0.0;      // their flops (series terms by class)
  int p2p_cls_ptr[kH0Classes + 2] = {0};  // items of series class c: [p2p_cls_ptr[c], p2p_cls_ptr[c + 1])
  DevBuf<int2> p2p_rng;
  int np2p_items = 0;
  // near-interface pairs: source boxes, target leaves and their source slots,
  // the rules' nodes (the classes' lists and nodes one after another), the
  // node sums of one group of right-hand sides (shared by the classes, which
  // run in sequence); ifl holds the classes' device pointers and sizes
  DevBuf<int> if_sbox, if_tleaf, if_tptr, if_tsrc;
  DevBuf<double2> qc, qky, qkx, if_S, if_T;
  std::vector<IfaceLists> ifl;  // one per class of pairs (one rule each)
  // tables of the horizontally separated near-interface pairs, one per class
  // that has such pairs (lists, panel edges and coefficients one after another)
  DevBuf<int> ift_tleaf, ift_tptr, ift_tsrc, ift_item_t;
  DevBuf<int2> ift_item_e;
  DevBuf<double4> ift_xpan;
  DevBuf<int2> ift_ypan;
  DevBuf<double2> ift_coef;
  std::vector<IfTable> ift;
  int ws_nrhs = 0;
  int64_t ws_gen = 0;  // bumped whenever the workspace buffers are reallocated
  DevBuf<double2> qs, us, alpha, beta;
  // HFMM_SELF_NONE: per sorted point the scattered self term G^s(x_i, x_i) and
  // its derivative in the source height, subtracted from the output and the
  // coordinate gradient
  DevBuf<double2> self_g, self_dy;
  DevBuf<double2> gq, gs;  // coordinate gradient: sorted q, per-point (d/dx, d/dy)
  hfmm_info_t info{};
  // ---- right-hand-side-blocked pipeline (applies with many right-hand sides)
  struct TgGroup {
    int first = 0, count = 0;
    int buf = 1;  // largest operator buffer of an item (elements)
  };
  bool blk_ok = false;   // the plan can run the blocked pipeline
  int blk_prec_m2l = BLK_F64, blk_prec_p2p = BLK_F64;
  DevBuf<TgItem> tg_items;
  DevBuf<TgPair> tg_pairs;
  std::vector<TgGroup> m2m_tg, l2l_tg;  // per parent level
  // M2L item lists per target level for the candidate tile shapes (row
  // tiles per item, the kernel variant's register allocation): one launch
  // per level, its LDS sized for that level's orders; the autotuner picks a
  // shape per level on the first blocked apply
  static constexpr int kTileCands = 3;
  static constexpr int kTileNt[kTileCands] = {2, 4, 8};
  std::vector<TgGroup> m2l_tgl[kTileCands];  // [candidate][level]
  std::vector<int> m2l_pick;                 // per level (-1: not tuned yet)
  bool m2l_tuned = false;
  DevBuf<BpItem> bp_items;
  DevBuf<int2> bp_rng;
  int bp_cls_ptr[kH0Classes + 2] = {0};
  DevBuf<int64_t> vmat_off;  // per leaf of level >= 2 (leaf order)
  int64_t vmat_tot = 0;
  bool vmat_ready = false;
  DevBuf<double2> vmat;
  DevBuf<double> blk_scale;  // a_l(n) at [l * kScaleStride + n]
  DevBuf<int64_t> coff16;
  int64_t ctot16 = 0;
  int blk_Rp = 0;  // pass width the blocked workspace holds
  DevBuf<double2> qb, ub, ab, bb;
  DevBuf<char> alo;   // scaled reduced-precision multipoles
  DevBuf<char> olo;   // scaled reduced-precision multipole-to-local operators
  DevBuf<float2> qlo; // FP32 strengths of the FP32 near field
  // the near field runs on a stream of its own, beside the far-field chain
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_done = nullptr;  // recorded after the last launch of every call
  // stage timing
  bool prof_on = false;
  std::vector<std::vector<hipEvent_t>> prof_pending;
  double prof_ms[HFMM_NSTAGES] = {0};
  int prof_n = 0;

  TreeView view(int nrhs) const {
    TreeView tv{};
    tv.n = n;
    tv.nboxes = (int)boxes.size();
    tv.nlev = nlev;
    tv.nrhs = nrhs;
    tv.k = med.k1;
    tv.pts = pts.p;
    tv.ctr = ctr.p;
    tv.level = level.p;
    tv.prange = prange.p;
    tv.coff = coff.p;
    tv.child = child.p;
    tv.parent = parent.p;
    tv.quad = quad.p;
    tv.ctot = ctot;
    for (int l = 0; l < HFMM_MAX_LEVELS; ++l) tv.P[l] = P[l];
    return tv;
  }
  void release_all() {
    pts.release(); ctr.release(); perm.release(); level.release(); parent.release(); quad.release();
    child.release(); prange.release(); coff.release(); leaves.release(); pt_box.release();
    m2l_items.release(); m2l_soff.release(); m2l_toff.release(); m2l_pcoff.release(); m2l_pcoffT.release();
    red_boxes.release(); red_ptr.release(); red_beg.release(); redT_ptr.release(); redT_beg.release(); cp_child.release();
    cp_parent.release(); up_doff.release(); up_soff4.release(); up_items.release(); down_items.release(); contrib.release();
    tabs.release(); tdata.release(); p2p_ptr.release();
    p2p_items.release(); p2p_sym.release(); p2p_rng.release(); if_sbox.release(); if_tleaf.release(); if_tptr.release(); if_tsrc.release(); qc.release();
    if_S.release(); if_T.release(); ift_tleaf.release(); ift_tptr.release(); ift_tsrc.release(); ift_xpan.release(); ift_ypan.release();
    ift_item_t.release(); ift_item_e.release();
    ift_coef.release();
    qky.release(); qkx.release(); qs.release(); us.release(); alpha.release(); beta.release(); gq.release(); gs.release();
    self_g.release(); self_dy.release();
    tg_items.release(); tg_pairs.release(); bp_items.release(); bp_rng.release(); vmat_off.release(); vmat.release();
    blk_scale.release(); coff16.release(); qb.release(); ub.release(); ab.release(); bb.release(); alo.release();
    qlo.release(); olo.release();
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_done) (void)hipEventDestroy(ev_done);
    ev_done = nullptr;
    if (side) (void)hipStreamDestroy(side);
    ev_fork = ev_join = nullptr;
    side = nullptr;
  }
};

namespace {

// Right-hand sides per pass through the pipeline: the M2L contribution rows
// (one per pair and right-hand side) stay within kContribBudget bytes per
// plan. Each pass repeats the coarse levels' short launches, so passes are
// made large: 2 GiB per plan (a batch of 32 plans stays within 64 GiB of the
// GPU's 288 GB; 512 MiB measured 6% slower eagerly and 21% as a graph replay
// on 32 geometries x 256 right-hand sides, 4 GiB the same as 2). HFMM_RHS_CHUNK
// in the environment caps the pass size further (diagnostics and tests).
constexpr double kContribBudget = 2048.0 * 1024 * 1024;
// device bytes of the near-interface node sums of one group of right-hand
// sides, and the classes of near-interface pairs (octaves of the least height
// sum)
constexpr size_t kIfBufBudget = (size_t)256 << 20;
constexpr int kIfClasses = 24;
// bounds on one near-interface table: panels (host and device memory of the
// panel values, 144 points each), and rule evaluations at plan time (about a
// second of the GPU)
constexpr int64_t kIfMaxPanels = (int64_t)1 << 18;
constexpr double kIfMaxGridWork = 1e12;
int rhs_chunk(hfmm_plan_t pl, int nrhs) {
  const double per_rhs = 8.0 * (double)std::max<int64_t>(pl->cstride, 1);
  int c = std::max(1, std::min(nrhs, (int)std::max(1.0, kContribBudget / per_rhs)));
  if (const char* env = std::getenv("HFMM_RHS_CHUNK")) {
    const int cap = std::atoi(env);
    if (cap >= 1) c = std::min(c, cap);
  }
  return c;
}

hfmm_status_t ensure_workspace(hfmm_plan_t pl, int nrhs) {
  if (pl->ws_nrhs >= nrhs) return HFMM_OK;
  if (pl->ws_nrhs > 0) {
    // earlier calls may still read the buffers about to be released
    HIP_TRY(hipEventSynchronize(pl->ev_done));
    HIP_TRY(hipStreamSynchronize(pl->side));
  }
  ++pl->ws_gen;
  HIP_TRY(pl->qs.alloc((size_t)pl->n * nrhs));
  HIP_TRY(pl->us.alloc((size_t)pl->n * nrhs));
  HIP_TRY(pl->alpha.alloc((size_t)std::max<int64_t>(pl->ctot, 1) * nrhs));
  HIP_TRY(pl->beta.alloc((size_t)std::max<int64_t>(pl->ctot, 1) * nrhs));
  HIP_TRY(pl->contrib.alloc((size_t)std::max<int64_t>(pl->cstride, 1) * nrhs));
  pl->ws_nrhs = nrhs;
  return HFMM_OK;
}

// HFMM_LOG=1 in the environment: plan statistics and autotuning results on stderr.
bool log_on() {
  const char* env = std::getenv("HFMM_LOG");
  return env && env[0] && env[0] != '0';
}

// The right-hand-side-blocked pipeline: used from kBlkMinRhs right-hand
// sides on (HFMM_BLOCKED=0 in the environment turns it off, =1 uses it for
// any count: diagnostics and tests). A pass holds a multiple of kBlkCols
// right-hand sides, within kBlkBudget bytes of workspace per plan
// (HFMM_BLK_RHS caps the pass width further).
constexpr int kBlkMinRhs = 48;
constexpr double kBlkBudget = 8192.0 * 1024 * 1024;
bool use_blocked(hfmm_plan_t pl, int nrhs) {
  if (pl->opt.deterministic) return true;  // the plan was refused unless blk_ok
  if (!pl->blk_ok || pl->prof_on) return false;
  const char* env = std::getenv("HFMM_BLOCKED");
  if (env && env[0] == '0') return false;
  if (env && env[0] == '1') return true;
  return nrhs >= kBlkMinRhs;
}
size_t blk_bytes_per_col(hfmm_plan_t pl) {
  size_t b = 16 * (2 * (size_t)pl->n + 2 * (size_t)std::max<int64_t>(pl->ctot, 1));
  if (pl->blk_prec_m2l == BLK_F32) b += 8 * (size_t)std::max<int64_t>(pl->ctot, 1);
  if (pl->blk_prec_m2l == BLK_BF16) b += 4 * (size_t)std::max<int64_t>(pl->ctot16, 1);
  if (pl->blk_prec_p2p == BLK_F32) b += 8 * (size_t)pl->n;
  return b;
}
int blk_pass_width(hfmm_plan_t pl, int nrhs) {
  const int want = (nrhs + kBlkCols - 1) / kBlkCols * kBlkCols;
  int cap = (int)(kBlkBudget / (double)blk_bytes_per_col(pl)) / kBlkCols * kBlkCols;
  if (const char* env = std::getenv("HFMM_BLK_RHS")) {
    const int c = std::atoi(env) / kBlkCols * kBlkCols;
    if (c >= kBlkCols) cap = std::min(cap, c);
  }
  return std::min(want, std::max(cap, kBlkCols));
}
// Blocked workspace for passes of Rp right-hand sides, and the leaves'
// expansion matrices (computed once, on stream s).
hfmm_status_t ensure_blk_workspace(hfmm_plan_t pl, int Rp, hipStream_t s) {
  if (pl->blk_Rp < Rp) {
    if (pl->blk_Rp > 0) {
      HIP_TRY(hipEventSynchronize(pl->ev_done));  // earlier calls may still read the buffers
      HIP_TRY(hipStreamSynchronize(pl->side));
    }
    ++pl->ws_gen;
    const size_t n = (size_t)pl->n, ct = (size_t)std::max<int64_t>(pl->ctot, 1), R = (size_t)Rp;
    pl->blk_Rp = 0;
    HIP_TRY(pl->qb.alloc(n * R));
    HIP_TRY(pl->ub.alloc(n * R));
    HIP_TRY(pl->ab.alloc(ct * R));
    HIP_TRY(pl->bb.alloc(ct * R));
    if (pl->blk_prec_m2l == BLK_F32) HIP_TRY(pl->alo.alloc(8 * ct * R));
    if (pl->blk_prec_m2l == BLK_BF16) HIP_TRY(pl->alo.alloc(4 * (size_t)std::max<int64_t>(pl->ctot16, 1) * R));
    if (pl->blk_prec_p2p == BLK_F32) HIP_TRY(pl->qlo.alloc(n * R));
    pl->blk_Rp = Rp;
  }
  if (!pl->m2l_tuned) {
    // M2L tile autotuner: per target level, each candidate item shape (row
    // tiles per item) runs that level's multipole-to-local launch on cleared
    // coefficients, once to warm up and once timed; the fastest is kept
    const int64_t n_ab = std::max<int64_t>(pl->ctot, 1) * Rp;
    launch_fill_zero(s, pl->ab.p, n_ab);
    if (pl->blk_prec_m2l == BLK_F32) launch_fill_zero(s, (double2*)pl->alo.p, n_ab / 2);
    if (pl->blk_prec_m2l == BLK_BF16) launch_fill_zero(s, (double2*)pl->alo.p, std::max<int64_t>(pl->ctot16, 1) * Rp / 4);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    pl->m2l_pick.assign(pl->nlev, hfmm_plan_s::kTileCands - 1);
    float total = 0.0f, most = -1.0f;
    // deterministic mode: a fixed tile shape, no timing (the choice then
    // cannot differ from run to run)
    for (int l = 0; l < (pl->opt.deterministic ? 0 : pl->nlev); ++l) {
      float best = 1e30f, ms_c[hfmm_plan_s::kTileCands] = {0, 0, 0};
      for (int c = 0; c < hfmm_plan_s::kTileCands; ++c) {
        const auto& g = pl->m2l_tgl[c][l];
        if (g.count == 0) break;
        for (int rep = 0; rep < 2; ++rep) {
          HIP_TRY(hipEventRecord(e0, s));
          launch_tgemm(s, pl->blk_prec_m2l, hfmm_plan_s::kTileNt[c], Rp, pl->tg_items.p + g.first, g.count, g.buf,
                       pl->tg_pairs.p, pl->tdata.p, pl->olo.p, pl->ab.p, pl->alo.p, pl->blk_scale.p, kScaleStride,
                       pl->bb.p, 0);
          HIP_TRY(hipEventRecord(e1, s));
          HIP_TRY(hipEventSynchronize(e1));
          HIP_TRY(hipEventElapsedTime(&ms_c[c], e0, e1));
        }
        if (ms_c[c] < best) {
          best = ms_c[c];
          pl->m2l_pick[l] = c;
        }
      }
      if (pl->m2l_tgl[0][l].count == 0) continue;
      total += best;
      if (best > most) {
        most = best;
        pl->info.m2l_tile = hfmm_plan_s::kTileNt[pl->m2l_pick[l]];
      }
      if (log_on())
        std::fprintf(stderr, "[hfmm] M2L tile autotune, level %d (order %d, %d right-hand sides, precision %d): "
                             "2 -> %.3f ms, 4 -> %.3f ms, 8 -> %.3f ms; picked %d\n",
                     l, pl->P[l], Rp, pl->blk_prec_m2l, ms_c[0], ms_c[1], ms_c[2],
                     hfmm_plan_s::kTileNt[pl->m2l_pick[l]]);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_TRY(hipGetLastError());
    pl->m2l_tuned = true;
    if (pl->opt.deterministic) pl->info.m2l_tile = hfmm_plan_s::kTileNt[hfmm_plan_s::kTileCands - 1];
    if (log_on()) std::fprintf(stderr, "[hfmm] M2L tuned: %.3f ms over all levels\n", total);
  }
  if (!pl->vmat_ready) {
    HIP_TRY(pl->vmat.alloc((size_t)std::max<int64_t>(pl->vmat_tot, 1)));
    const int lb2 = pl->leaf_lev[std::min(2, pl->nlev)];
    launch_vmat(s, pl->view(1), pl->leaves.p + lb2, pl->nleaves - lb2, pl->vmat_off.p, pl->vmat.p);
    HIP_TRY(hipGetLastError());
    pl->vmat_ready = true;
  }
  return HFMM_OK;
}

// Expansion order of a level: the smallest P with
// |J_{P+1}(k R)| |H_{P+1}(k (D - R))| <= eps, R = b/sqrt(2) the box radius and
// D = 2b the closest centre distance of a translated pair.
int choose_order(double k, double b, double eps, int& status) {
  double R = b * std::sqrt(0.5);
  double D = 2.0 * b;
  status = 0;
  for (int P = 3; P <= kMaxOrder; ++P) {
    double j = host_absj(k * R, P + 1);
    if (j == 0.0) return P;
    double ly = host_log10_absy(k * (D - R), P + 1);
    double lj = std::log10(j);
    double hl = std::max(ly, std::log10(std::max(host_absj(k * (D - R), P + 1), 1e-300)));
    if (lj + hl <= std::log10(eps)) return P;
  }
  status = 1;
  return kMaxOrder;
}

}  // namespace

namespace hfmm {
// Workspace for nrhs right-hand sides, allocated ahead of a graph capture.
hfmm_status_t plan_reserve(hfmm_plan_t pl, int nrhs, hipStream_t s) {
  AllocScope alloc_scope(&pl->al);
  if (use_blocked(pl, nrhs)) return ensure_blk_workspace(pl, blk_pass_width(pl, nrhs), s);
  return ensure_workspace(pl, rhs_chunk(pl, nrhs));
}
int64_t plan_points(hfmm_plan_t pl) { return pl->n; }
double plan_wavenumber(hfmm_plan_t pl) { return pl->med.k1; }
int64_t plan_workspace_generation(hfmm_plan_t pl) { return pl->ws_gen; }
size_t workspace_bytes(hfmm_plan_t pl, int nrhs) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t r = (size_t)nrhs;
  return 2 * al(sizeof(double2) * (size_t)pl->n * r) + 2 * al(sizeof(double2) * (size_t)std::max<int64_t>(pl->ctot, 1) * r) +
         al(sizeof(double) * (size_t)std::max<int64_t>(pl->cstride, 1) * r);
}
hfmm_status_t report(hfmm_status_t st, const std::string& msg) { return fail(st, msg); }
}  // namespace hfmm

extern "C" {

void hfmm_default_options(hfmm_options_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(hfmm_options_t);
  o->leaf_size = 64;
  o->precision = HFMM_FP64;
  o->self_term = HFMM_SELF_SCATTERED;
  o->interface_refine = 1;
  o->max_level = 24;
  o->leaf_kb = 1.5;
}

const char* hfmm_status_string(hfmm_status_t s) {
  switch (s) {
    case HFMM_OK: return "ok";
    case HFMM_ERR_INVALID_ARG: return "invalid argument";
    case HFMM_ERR_DOMAIN: return "point outside the top layer, non-finite or coincident";
    case HFMM_ERR_UNSUPPORTED: return "unsupported medium";
    case HFMM_ERR_NO_MEMORY: return "out of memory";
    case HFMM_ERR_DEVICE: return "HIP runtime error";
    case HFMM_ERR_ACCURACY: return "tolerance not attainable";
  }
  return "unknown status";
}

const char* hfmm_last_error_message(void) { return g_err.c_str(); }

void hfmm_destroy(hfmm_plan_t pl) {
  if (!pl) return;
  // the plan's work ends with ev_done on the stream of its last call (calls
  // on one plan are stream ordered); the side stream joins into that stream
  if (pl->ev_done) (void)hipEventSynchronize(pl->ev_done);
  if (pl->side) (void)hipStreamSynchronize(pl->side);
  pl->release_all();
  delete pl;
}

hfmm_status_t hfmm_plan_info(hfmm_plan_t pl, hfmm_info_t* out) {
  if (!pl || !out) return fail(HFMM_ERR_INVALID_ARG, "null plan or output");
  *out = pl->info;
  return HFMM_OK;
}

hfmm_status_t hfmm_plan(hfmm_plan_t* out, int32_t layers, const double* wavenumbers, const double* interfaces,
                        int64_t n, const double* points, double tol, const hfmm_options_t* opts,
                        hfmm_stream_t stream_) {
  auto t_start = std::chrono::steady_clock::now();
  hipStream_t stream = (hipStream_t)stream_;
  if (!out) return fail(HFMM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!wavenumbers || !points || !interfaces)
    return fail(HFMM_ERR_INVALID_ARG, "NULL wavenumbers, interfaces or points");
  if (layers != 1 && layers != 2 && layers != 3) return fail(HFMM_ERR_UNSUPPORTED, "layers must be 1, 2 or 3");
  if (n < 1 || n > (int64_t)1 << 30) return fail(HFMM_ERR_INVALID_ARG, "n out of range");
  if (!(tol >= 1e-14 && tol <= 1e-2)) return fail(HFMM_ERR_INVALID_ARG, "tol must be in [1e-14, 1e-2]");
  hfmm_options_t o;
  hfmm_default_options(&o);
  if (opts) {
    if (opts->struct_size != (int32_t)sizeof(hfmm_options_t))
      return fail(HFMM_ERR_INVALID_ARG, "options struct_size mismatch");
    o = *opts;
  }
  if (o.leaf_size < 1 || o.leaf_size > 4096) return fail(HFMM_ERR_INVALID_ARG, "leaf_size out of range");
  if (o.precision != HFMM_FP64 && o.precision != HFMM_FP32 && o.precision != HFMM_BF16)
    return fail(HFMM_ERR_UNSUPPORTED, "precision must be HFMM_FP64, HFMM_FP32 or HFMM_BF16");
  if (o.self_term != HFMM_SELF_SCATTERED && o.self_term != HFMM_SELF_NONE)
    return fail(HFMM_ERR_INVALID_ARG, "self_term must be HFMM_SELF_SCATTERED or HFMM_SELF_NONE");
  if (o.max_nrhs < 0 || o.max_nrhs > (1 << 20)) return fail(HFMM_ERR_INVALID_ARG, "max_nrhs out of range");
  if (o.deterministic != 0 && o.deterministic != 1) return fail(HFMM_ERR_INVALID_ARG, "deterministic must be 0 or 1");
  if (o.order < 0 || o.order > kMaxOrder) return fail(HFMM_ERR_INVALID_ARG, "order must be in [0, 255]");
  if ((o.alloc == nullptr) != (o.free == nullptr))
    return fail(HFMM_ERR_INVALID_ARG, "alloc and free must be given together");
  if (o.max_level < 2 || o.max_level > KEY_BITS) return fail(HFMM_ERR_INVALID_ARG, "max_level out of range");
  if (!(o.leaf_kb == 0.0 || (o.leaf_kb >= 0.25 && std::isfinite(o.leaf_kb))))
    return fail(HFMM_ERR_INVALID_ARG, "leaf_kb must be 0 or a finite value >= 0.25");
  if (o.top_level != 0 && (o.top_level < 2 || o.top_level > KEY_BITS))
    return fail(HFMM_ERR_INVALID_ARG, "top_level must be 0 or in [2, 30]");
  for (int i = 0; i < layers; ++i)
    if (!(wavenumbers[i] > 0.0) || !std::isfinite(wavenumbers[i]))
      return fail(HFMM_ERR_UNSUPPORTED, "wavenumbers must be finite and > 0");
  for (int i = 1; i < layers; ++i)
    if (wavenumbers[i] < wavenumbers[0])
      return fail(HFMM_ERR_UNSUPPORTED, "a lower layer has a smaller wavenumber than the top layer");
  for (int i = 0; i < std::max(1, layers - 1); ++i)
    if (!std::isfinite(interfaces[i])) return fail(HFMM_ERR_INVALID_ARG, "interfaces must be finite");
  if (layers == 1 && !(o.impedance > 0.0 && std::isfinite(o.impedance)))
    return fail(HFMM_ERR_INVALID_ARG, "the impedance half-space (layers = 1) needs impedance > 0");
  if (layers > 1 && o.impedance != 0.0)
    return fail(HFMM_ERR_INVALID_ARG, "impedance applies to the half-space (layers = 1) only");
  if (layers == 3 && !(interfaces[0] > interfaces[1]))
    return fail(HFMM_ERR_INVALID_ARG, "interfaces must be strictly decreasing");

  {
    hipError_t e = init_kernel_attributes();
    if (e == hipSuccess) e = init_blocked_attributes();
    if (e != hipSuccess) return fail(HFMM_ERR_DEVICE, std::string("kernel attributes: ") + hipGetErrorString(e));
  }
  hfmm_plan_t pl = new hfmm_plan_s();
  pl->al.alloc = o.alloc;
  pl->al.free = o.free;
  pl->al.ctx = o.alloc_ctx;
  AllocScope alloc_scope(&pl->al);
  auto bail = [&](hfmm_status_t s) {
    pl->release_all();
    delete pl;
    return s;
  };
  {
    hipError_t e = hipStreamCreateWithFlags(&pl->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_done, hipEventDisableTiming);
    if (e != hipSuccess) {
      fail(HFMM_ERR_DEVICE, std::string("plan stream: ") + hipGetErrorString(e));
      return bail(HFMM_ERR_DEVICE);
    }
  }
  pl->precision = o.precision;
  pl->n = (int)n;
  pl->tol = tol;
  pl->opt = o;
  pl->y_top = interfaces[0];
  pl->med.layers = layers;
  pl->med.k1 = wavenumbers[0];
  pl->med.k2 = layers == 1 ? wavenumbers[0] : wavenumbers[1];
  pl->med.k3 = layers == 3 ? wavenumbers[2] : pl->med.k2;
  pl->med.d = layers == 3 ? interfaces[0] - interfaces[1] : 1.0;
  pl->med.alpha = layers == 1 ? o.impedance : 0.0;
  const double k = pl->med.k1;
  // plan phases (seconds), printed when HFMM_LOG is set
  std::vector<std::pair<const char*, double>> phases;
  auto t_phase = t_start;
  auto phase = [&](const char* name) {
    const auto now = std::chrono::steady_clock::now();
    phases.push_back({name, std::chrono::duration<double>(now - t_phase).count()});
    t_phase = now;
  };

  // ---- the tree, its interaction lists and the point order (GPU builder)
  TreeOut tree;
  {
    TreeParams tp;
    tp.n = n;
    tp.y_top = pl->y_top;
    tp.k = k;
    tp.leaf_size = o.leaf_size;
    tp.leaf_kb = o.leaf_kb;
    tp.interface_refine = o.interface_refine;
    tp.max_level = o.max_level;
    tp.top_level = o.top_level;
    TreeDev tdev;
    gpu_tree_build(tp, points, stream, false, tree, tdev);
    if (tree.status != TREE_OK) {
      const hfmm_status_t st = tree.status == TREE_DOMAIN  ? HFMM_ERR_DOMAIN
                               : tree.status == TREE_DEPTH ? HFMM_ERR_ACCURACY
                               : tree.status == TREE_MEMORY ? HFMM_ERR_NO_MEMORY
                                                            : HFMM_ERR_DEVICE;
      fail(st, tree.msg);
      return bail(st);
    }
    std::swap(pl->perm, tdev.perm);
  }
  phase("tree");
  // ---- points on the host, interface frame
  std::vector<double> hp((size_t)2 * n);
  {
    hipError_t e = hipMemcpyAsync(hp.data(), points, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      fail(HFMM_ERR_DEVICE, std::string("copying points: ") + hipGetErrorString(e));
      return bail(HFMM_ERR_DEVICE);
    }
  }
  for (int64_t i = 0; i < n; ++i) hp[2 * i + 1] -= pl->y_top;
  const double xmin = tree.x0, ymin = tree.y0, S = tree.S;
  double ymax = ymin;
  for (int64_t i = 0; i < n; ++i) ymax = std::max(ymax, hp[2 * i + 1]);
  pl->S = S;
  pl->x0 = xmin;
  pl->y0 = ymin;
  const std::vector<int>& perm = tree.perm;
  pl->boxes = std::move(tree.boxes);
  std::vector<Box>& B = pl->boxes;
  pl->lev_begin = tree.lev_begin;
  pl->nlev = tree.nlev;
  for (int l = 0; l < pl->nlev; ++l) pl->bsize[l] = tree.bsize[l];
  const int nb = (int)B.size();
  pl->top = tree.top;
  phase("points");
  // ---- expansion orders (levels >= 2)
  const double eps = tol * kOrderSafety;
  for (int l = 2; l < pl->nlev; ++l) {
    int st = 0;
    pl->P[l] = o.order > 0 ? o.order : choose_order(k, pl->bsize[l], eps, st);
    if (st) {
      fail(HFMM_ERR_ACCURACY, "expansion order above the cap at level " + std::to_string(l));
      return bail(HFMM_ERR_ACCURACY);
    }
    // range of the free M2L table: |H_{2P}(k 2b)| must stay in FP64 range
    double ly = host_log10_absy(2.0 * k * pl->bsize[l], 2 * pl->P[l]);
    double lj = std::log10(std::max(host_absj(k * pl->bsize[l] * std::sqrt(0.5), pl->P[l]), 1e-308));
    if (ly > 280.0 || lj < -280.0) {
      fail(HFMM_ERR_ACCURACY, "expansions out of FP64 range at level " + std::to_string(l) +
                                  " (tree too deep for this wavenumber; raise leaf_size)");
      return bail(HFMM_ERR_ACCURACY);
    }
  }

  // ---- coefficient offsets
  std::vector<int64_t> coff(nb, 0);
  int64_t ctot = 0;
  for (int i = 0; i < nb; ++i) {
    coff[i] = ctot;
    if (B[i].level >= 2) ctot += 2 * pl->P[B[i].level] + 1;
  }
  pl->ctot = ctot;

  phase("orders");
  // ---- interaction lists (from the tree builder, sorted by target)
  using PairL = TreePair;
  const std::vector<PairL>& fv = tree.fv;
  const std::vector<PairL>& iv = tree.iv;
  const std::vector<PairL>& fu = tree.fu;
  const std::vector<PairL>& iu = tree.iu;
  phase("lists");
  // ---- tables
  std::vector<TableRef> tabs;
  int64_t toff = 0;
  auto new_table = [&](int half) {
    tabs.push_back(TableRef{toff, half, 0});
    toff += 2 * half + 1;
    return (int)tabs.size() - 1;
  };
  std::map<std::tuple<int, int, int>, int> free_id, image_id;
  std::vector<double> fh_dx, fh_dy;
  std::vector<int> fh_ref;
  struct ImgCombo { int level, dix, m; };
  std::vector<ImgCombo> combos;
  std::vector<int> img_ref;
  auto free_table = [&](int l, int dx, int dy) {
    auto key3 = std::make_tuple(l, dx, dy);
    auto it = free_id.find(key3);
    if (it != free_id.end()) return it->second;
    int id = new_table(2 * pl->P[l]);
    free_id[key3] = id;
    fh_dx.push_back(dx * pl->bsize[l]);
    fh_dy.push_back(dy * pl->bsize[l]);
    fh_ref.push_back(id);
    return id;
  };
  auto image_table = [&](int l, int dix, int m) {
    auto key3 = std::make_tuple(l, dix, m);
    auto it = image_id.find(key3);
    if (it != image_id.end()) return it->second;
    int id = new_table(2 * pl->P[l]);
    image_id[key3] = id;
    combos.push_back({l, dix, m});
    img_ref.push_back(id);
    return id;
  };
  // M2L pairs grouped by translation table (the batched contraction works per table)
  std::vector<std::vector<std::pair<int, int>>> pairs_of;   // (source, target) per table id
  std::vector<int> table_level, table_image;
  auto add_pair = [&](int id, int l, int img, int s, int t) {
    if ((int)pairs_of.size() <= id) {
      pairs_of.resize(id + 1);
      table_level.resize(id + 1, -1);
      table_image.resize(id + 1, 0);
    }
    pairs_of[id].push_back({s, t});
    table_level[id] = l;
    table_image[id] = img;
  };
  std::vector<int> fv_tab, iv_tab;  // table of each pair
  for (auto& pr : fv) {
    int l = B[pr.t].level;
    int id = free_table(l, B[pr.t].ix - B[pr.s].ix, B[pr.t].iy - B[pr.s].iy);
    add_pair(id, l, 0, pr.s, pr.t);
    fv_tab.push_back(id);
  }
  for (auto& pr : iv) {
    int l = B[pr.t].level;
    int id = image_table(l, B[pr.t].ix - B[pr.s].ix, B[pr.t].iy + B[pr.s].iy);
    add_pair(id, l, 1, pr.s, pr.t);
    iv_tab.push_back(id);
  }
  // batched M2L items: per level, per table, batches of up to 64 pairs (16 when
  // 2P+1 > 64), and groups of row tiles of the real-embedded operator (ntw per
  // wave). Each pair owns a contribution row of 2(2P+1) doubles, reduced per
  // box afterwards: the rows of one target box are contiguous (and, for the
  // transpose, those of one source box).
  auto add_items = [](std::vector<TransItem>& items, int table, int pbeg, int cnt, int image, int Ps, int Pd,
                      int ntw, int64_t toff) {
    const int nrt = (2 * (2 * Pd + 1) + 15) / 16;
    const int step = trans_rows_per_item(Ps, Pd, ntw);
    for (int rt = 0; rt < nrt; rt += step)
      items.push_back(TransItem{table, pbeg, cnt, image, rt, Ps, Pd, ntw, toff});
  };
  // row tiles per wave for a launch of `batches` pair batches: the most (up to
  // 8, the longest MFMA chains, and no more than the rows need) that still
  // give about four blocks per CU
  auto choose_ntw = [](int64_t batches, int Ps, int Pd) {
    const int nrt = (2 * (2 * Pd + 1) + 15) / 16;
    int ntw = 8;
    while (ntw > 1 && trans_rows_per_item(Ps, Pd, ntw / 2) >= nrt) ntw /= 2;
    for (; ntw > 1; ntw = (ntw + 1) / 2) {
      const int step = trans_rows_per_item(Ps, Pd, ntw);
      if (batches * ((nrt + step - 1) / step) >= 1024) return ntw;
    }
    return 1;
  };
  std::vector<TransItem> m2l_items;
  std::vector<int> m2l_psrc, m2l_pdst;
  std::vector<int64_t> m2l_pcoff;
  int64_t cstride = 0;
  for (int l = 0; l < pl->nlev; ++l) {
    hfmm_plan_s::Group g;
    g.first = (int)m2l_items.size();
    g.Ps = g.Pd = pl->P[l];
    const int npi = trans_pairs_per_item(pl->P[l], pl->P[l]);
    int64_t batches = 0;
    for (size_t id = 0; id < pairs_of.size(); ++id)
      if (table_level[id] == l) batches += ((int64_t)pairs_of[id].size() + npi - 1) / npi;
    const int ntw = choose_ntw(batches, pl->P[l], pl->P[l]);
    g.ntw = ntw;
    for (size_t id = 0; id < pairs_of.size(); ++id) {
      if (table_level[id] != l) continue;
      auto& v = pairs_of[id];
      for (size_t c0 = 0; c0 < v.size(); c0 += npi) {
        int cnt = (int)std::min<size_t>(npi, v.size() - c0);
        int pbeg = (int)m2l_psrc.size();
        for (int c = 0; c < cnt; ++c) {
          m2l_psrc.push_back(v[c0 + c].first);
          m2l_pdst.push_back(v[c0 + c].second);
          cstride += 2 * (2 * pl->P[l] + 1);
        }
        add_items(m2l_items, (int)id, pbeg, cnt, table_image[id], pl->P[l], pl->P[l], ntw,
                  tabs[id].off + tabs[id].half - 2 * pl->P[l]);
      }
    }
    g.count = (int)m2l_items.size() - g.first;
    if (!g.count) continue;
    // Consecutive levels share one launch where that costs little, which
    // removes the drain at the end of each launch. A launch reserves the LDS
    // of its largest order, so a level joins the launch before it when that
    // LDS is at most 1.25 times its own, or when the level alone has under
    // four blocks per CU and so cannot fill the GPU by itself. Both use the
    // same kernel instantiation (ntw up to 2, or more).
    if (!pl->m2l_groups.empty()) {
      auto& run = pl->m2l_groups.back();
      const double lds_ratio = (double)trans_lds_bytes(run.Ps, run.Pd) / (double)trans_lds_bytes(g.Ps, g.Pd);
      if ((run.ntw <= 2) == (g.ntw <= 2) && g.Ps <= run.Ps && g.Pd <= run.Pd &&
          (lds_ratio <= 1.25 || g.count < 1024)) {
        run.count += g.count;
        continue;
      }
    }
    pl->m2l_groups.push_back(g);
  }
  pl->cstride = cstride;
  // contribution rows in box order, by target (forward) and by source
  // (transpose), and the per-box counts and first rows for the reductions
  std::vector<int> red_boxes, red_ptr(1, 0), redT_ptr(1, 0);
  std::vector<int64_t> red_beg, redT_beg, m2l_pcoffT;
  {
    std::vector<std::vector<int>> as_t(nb), as_s(nb);
    for (int i = 0; i < (int)m2l_psrc.size(); ++i) {
      as_t[m2l_pdst[i]].push_back(i);
      as_s[m2l_psrc[i]].push_back(i);
    }
    m2l_pcoff.assign(m2l_psrc.size(), 0);
    m2l_pcoffT.assign(m2l_psrc.size(), 0);
    int64_t of = 0, ofT = 0;
    for (int i = pl->lev_begin[std::min(2, pl->nlev)]; i < nb; ++i) {
      const int64_t row = 2 * (2 * pl->P[B[i].level] + 1);
      red_boxes.push_back(i);
      red_beg.push_back(of);
      for (int pr : as_t[i]) { m2l_pcoff[pr] = of; of += row; }
      red_ptr.push_back(red_ptr.back() + (int)as_t[i].size());
      redT_beg.push_back(ofT);
      for (int pr : as_s[i]) { m2l_pcoffT[pr] = ofT; ofT += row; }
      redT_ptr.push_back(redT_ptr.back() + (int)as_s[i].size());
    }
    if (of != cstride || ofT != cstride) return bail(fail(HFMM_ERR_DEVICE, "internal: contribution rows"));
  }
  // M2M / L2L tables per parent level l (children at l + 1), quadrant order
  std::vector<double> fb_dx, fb_dy;
  std::vector<int> fb_sgn, fb_ref;
  pl->m2m_tab.assign(pl->nlev, -1);
  pl->l2l_tab.assign(pl->nlev, -1);
  pl->m2m_q4.assign(pl->nlev, Toff4{});
  pl->l2l_q4.assign(pl->nlev, Toff4{});
  for (int l = pl->top; l + 1 < pl->nlev; ++l) {
    double bc = pl->bsize[l + 1];
    for (int pass = 0; pass < 2; ++pass) {
      int base = (int)tabs.size();
      for (int q = 0; q < 4; ++q) {
        int id = new_table(pl->P[l] + pl->P[l + 1]);
        fb_dx.push_back(((q & 1) ? 0.5 : -0.5) * bc);
        fb_dy.push_back(((q >> 1) ? 0.5 : -0.5) * bc);
        fb_sgn.push_back(pass == 0 ? -1 : 1);
        fb_ref.push_back(id);
      }
      (pass == 0 ? pl->m2m_tab : pl->l2l_tab)[l] = base;
      Toff4 q4{};
      for (int q = 0; q < 4; ++q) q4.v[q] = tabs[base + q].off + tabs[base + q].half - (pl->P[l] + pl->P[l + 1]);
      (pass == 0 ? pl->m2m_q4 : pl->l2l_q4)[l] = q4;
    }
  }

  // (child, parent) pairs per parent level l >= 2 and quadrant q, with items
  // shaped parent -> child ("down": L2L, transposed M2M); the table of an item
  // is the quadrant, taken from the level's four M2M or L2L tables at launch.
  // Child -> parent ("up": M2M, transposed L2L) items list 16 parents each and
  // gather their four children.
  std::vector<int> cp_child, cp_parent;
  std::vector<int64_t> up_doff_h, up_soff4_h;
  std::vector<TransItem> up_items, down_items;
  pl->up_groups.assign(pl->nlev, {});
  pl->down_groups.assign(pl->nlev, {});
  pl->up_split_groups.assign(pl->nlev, {});
  for (int l = pl->top; l + 1 < pl->nlev; ++l) {
    auto& gu = pl->up_groups[l];
    auto& gd = pl->down_groups[l];
    gu.first = (int)up_items.size();
    gd.first = (int)down_items.size();
    gu.Ps = gd.Pd = pl->P[l + 1];
    gu.Pd = gd.Ps = pl->P[l];
    const int npi = trans_pairs_per_item(pl->P[l + 1], pl->P[l]);
    std::vector<int> kids[4], parents;
    for (int i = pl->lev_begin[l + 1]; i < pl->lev_begin[l + 2]; ++i) kids[B[i].quad].push_back(i);
    for (int i = pl->lev_begin[l]; i < pl->lev_begin[l + 1]; ++i)
      if (!B[i].leaf) parents.push_back(i);
    int64_t batches = 0;
    for (int q = 0; q < 4; ++q) batches += ((int64_t)kids[q].size() + npi - 1) / npi;
    const int64_t pbatches = ((int64_t)parents.size() + npi - 1) / npi;
    const int ntw_up = choose_ntw(pbatches, pl->P[l + 1], pl->P[l]);
    const int ntw_down = choose_ntw(batches, pl->P[l], pl->P[l + 1]);
    gu.ntw = ntw_up;
    gd.ntw = ntw_down;
    // The split gather where its blocks (one per parent batch and row tile)
    // all fit on the GPU at once: such small launches are bound by each
    // block's chain of quadrants, which the split form runs side by side. Its
    // LDS (four tables and source tiles) must fit a CU. Beside the near field
    // its large blocks wait for LDS, so the overlapped apply keeps the
    // standard form.
    const int nrt_up = (2 * (2 * pl->P[l] + 1) + 15) / 16;
    bool split = false;
    int split_rhs = 0;
    {
      const size_t lds_split = trans_lds_bytes_split(pl->P[l + 1], pl->P[l]);
      const int64_t per_cu = lds_split <= kSplitLdsMax ? (int64_t)(kCuLds / lds_split) : 0;
      split = per_cu > 0 && pbatches * nrt_up <= kNumCu * per_cu;
      if (split) split_rhs = (int)std::min<int64_t>(1 << 20, kNumCu * per_cu / std::max<int64_t>(pbatches * nrt_up, 1));
    }
    std::vector<std::pair<int, int>> batch_pairs;  // (pbeg, count) per parent batch
    for (size_t c0 = 0; c0 < parents.size(); c0 += npi) {
      const int cnt = (int)std::min<size_t>(npi, parents.size() - c0);
      const int pbeg = (int)up_doff_h.size();
      for (int c = 0; c < cnt; ++c) {
        const Box& par = B[parents[c0 + c]];
        up_doff_h.push_back(coff[parents[c0 + c]]);
        for (int q = 0; q < 4; ++q) up_soff4_h.push_back(par.child[q] >= 0 ? coff[par.child[q]] : -1);
      }
      add_items(up_items, 0, pbeg, cnt, 0, pl->P[l + 1], pl->P[l], ntw_up, -1);
      batch_pairs.emplace_back(pbeg, cnt);
    }
    gu.count = (int)up_items.size() - gu.first;
    if (split) {
      auto& gs = pl->up_split_groups[l];
      gs = gu;
      gs.first = (int)up_items.size();
      gs.ntw = 1;
      gs.max_rhs = split_rhs;
      for (const auto& bp : batch_pairs)
        for (int rt = 0; rt < nrt_up; ++rt)
          up_items.push_back(TransItem{0, bp.first, bp.second, 0, rt, pl->P[l + 1], pl->P[l], 1, -1});
      gs.count = (int)up_items.size() - gs.first;
    }
    for (int q = 0; q < 4; ++q) {
      const std::vector<int>& kids_q = kids[q];
      for (size_t c0 = 0; c0 < kids_q.size(); c0 += npi) {
        int cnt = (int)std::min<size_t>(npi, kids_q.size() - c0);
        int pbeg = (int)cp_child.size();
        for (int c = 0; c < cnt; ++c) {
          cp_child.push_back(kids_q[c0 + c]);
          cp_parent.push_back(B[kids_q[c0 + c]].parent);
        }
        add_items(down_items, q, pbeg, cnt, 0, pl->P[l], pl->P[l + 1], ntw_down, -1);
      }
    }
    gd.count = (int)down_items.size() - gd.first;
  }

  phase("tables (host)");
  // ---- per-level box lists
  std::vector<int> leaves;
  std::vector<int> leaf_index(nb, -1);
  pl->leaf_lev.assign(pl->nlev + 1, 0);
  for (int i = 0; i < nb; ++i)  // boxes are in level order, so are the leaves
    if (B[i].leaf) {
      leaf_index[i] = (int)leaves.size();
      leaves.push_back(i);
      pl->leaf_lev[B[i].level + 1] = (int)leaves.size();
    }
  for (int l = 1; l <= pl->nlev; ++l) pl->leaf_lev[l] = std::max(pl->leaf_lev[l], pl->leaf_lev[l - 1]);
  // the leaves' point ranges partition the sorted points
  std::vector<int> pt_box_h((size_t)n, 0);
  for (int x : leaves)
    for (int j = B[x].begin; j < B[x].end; ++j) pt_box_h[j] = x;
  pl->leaf_pmax = 0;
  for (int l = 0; l < pl->nlev; ++l)
    if (pl->leaf_lev[l + 1] > pl->leaf_lev[l]) pl->leaf_pmax = std::max(pl->leaf_pmax, pl->P[l]);

  phase("level lists");
  // ---- direct lists, grouped by target leaf, source ranges merged
  auto leaves_under = [&](int b, std::vector<int>& outv) {
    std::vector<int> st{b};
    while (!st.empty()) {
      int x = st.back();
      st.pop_back();
      if (B[x].leaf) outv.push_back(x);
      else
        for (int q = 3; q >= 0; --q)
          if (B[x].child[q] >= 0) st.push_back(B[x].child[q]);
    }
  };
  auto group = [&](const std::vector<PairL>& prs, std::vector<std::vector<int2>>& per_leaf, int64_t& npairs) {
    per_leaf.assign(leaves.size(), {});
    npairs = 0;
    std::vector<int> tl;
    for (auto& pr : prs) {
      tl.clear();
      leaves_under(pr.t, tl);
      int2 r = make_int2(B[pr.s].begin, B[pr.s].end);
      for (int t : tl) {
        per_leaf[leaf_index[t]].push_back(r);
        npairs += (int64_t)(B[t].end - B[t].begin) * (r.y - r.x);
      }
    }
    for (auto& v : per_leaf) {
      std::sort(v.begin(), v.end(), [](int2 a, int2 b) { return a.x < b.x; });
      std::vector<int2> m;
      for (auto& r : v) {
        if (!m.empty() && r.x <= m.back().y) m.back().y = std::max(m.back().y, r.y);
        else m.push_back(r);
      }
      v.swap(m);
    }
  };
  std::vector<std::vector<int2>> u_per;
  int64_t np2p = 0, nifp = 0;
  group(fu, u_per, np2p);
  // Bounding boxes of the points of every leaf, then of every merged source
  // range (a union of whole leaves, found through the leaves in point order).
  std::vector<double4> leaf_bb(leaves.size());
  for (size_t li = 0; li < leaves.size(); ++li) {
    const Box& bx = B[leaves[li]];
    double4 bb = make_double4(INFINITY, -INFINITY, INFINITY, -INFINITY);
    for (int j = bx.begin; j < bx.end; ++j) {
      const double px = hp[2 * perm[j]], py = hp[2 * perm[j] + 1];
      bb.x = std::min(bb.x, px); bb.y = std::max(bb.y, px);
      bb.z = std::min(bb.z, py); bb.w = std::max(bb.w, py);
    }
    leaf_bb[li] = bb;
  }
  std::vector<int> leaf_at(pl->n, -1);  // leaf whose points start at index j
  for (size_t li = 0; li < leaves.size(); ++li) leaf_at[B[leaves[li]].begin] = (int)li;
  auto range_bb = [&](int2 r) {
    double4 bb = make_double4(INFINITY, -INFINITY, INFINITY, -INFINITY);
    for (int j = r.x; j < r.y;) {
      const int li = leaf_at[j];
      if (li < 0) return make_double4(-INFINITY, INFINITY, -INFINITY, INFINITY);  // not leaf-aligned: widest class
      const double4& lb = leaf_bb[li];
      bb.x = std::min(bb.x, lb.x); bb.y = std::max(bb.y, lb.y);
      bb.z = std::min(bb.z, lb.z); bb.w = std::max(bb.w, lb.w);
      j = B[leaves[li]].end;
    }
    return bb;
  };
  // Near-interface pairs: per target leaf (every leaf under a pair's target
  // box) its source boxes in point order; a source box inside another box of
  // the same leaf's list adds no pairs (the pairs form a set), so it is
  // dropped. Each (leaf, source box) pair then goes to a class by the least
  // height sum Y = y_i + y_j its point bounding boxes allow, in octaves above
  // the least over all pairs: the Sommerfeld rule of a class reaches t ~ 44 /
  // Y_min with panels ~ 4 / (Y_max + X_max) wide, so the few pairs right at
  // the interface get the long rule and the rest short ones.
  struct IfPair {
    int li, sb, cls;
    double ylo, yhi, xsp, gap;  // Y range, largest |X| and least |X| of the pair
    double tw;                  // width in x of the target leaf's points
  };
  std::vector<IfPair> ifp;
  {
    std::vector<std::vector<int>> per_leaf(leaves.size());
    std::vector<int> tl;
    for (auto& pr : iu) {
      tl.clear();
      leaves_under(pr.t, tl);
      for (int t : tl) per_leaf[leaf_index[t]].push_back(pr.s);
    }
    for (size_t li = 0; li < leaves.size(); ++li) {
      std::vector<int>& v = per_leaf[li];
      if (v.empty()) continue;
      // by first point, the larger of two boxes with the same first point first
      std::sort(v.begin(), v.end(), [&](int a, int b) {
        return B[a].begin != B[b].begin ? B[a].begin < B[b].begin : B[a].end > B[b].end;
      });
      const int nt = B[leaves[li]].end - B[leaves[li]].begin;
      const double4& tb = leaf_bb[li];
      int reach = -1;
      for (int sb : v) {
        if (B[sb].end <= reach) continue;  // box ranges nest or are disjoint
        reach = B[sb].end;
        const double4 sbb = range_bb(make_int2(B[sb].begin, B[sb].end));
        if (std::isfinite(sbb.z) && std::isfinite(sbb.w))
          ifp.push_back({(int)li, sb, 0, tb.z + sbb.z, tb.w + sbb.w, std::max(tb.y - sbb.x, sbb.y - tb.x),
                         std::max(0.0, std::max(tb.x - sbb.y, sbb.x - tb.y)), tb.y - tb.x});
        else  // not a union of leaves: the extent of all points
          ifp.push_back({(int)li, sb, 0, 2.0 * ymin, 2.0 * ymax, S, 0.0, tb.y - tb.x});
        nifp += (int64_t)nt * (B[sb].end - B[sb].begin);
      }
    }
  }
  // Within a class, pairs at least X0 apart in x go to its table, the rest
  // (neighbours) to its quadrature rule: X0 is the class's widest target leaf,
  // at most its largest Y. The quadrature rule's length grows with its |X|
  // range; the table's panels only in number as X0 shrinks.
  struct IfClass {
    std::vector<int> sbox, tleaf, tptr{0}, tsrc;  // quadrature pairs
    double xsp = 0.0, ylo = INFINITY, yhi = 0.0;
    std::vector<int> ftleaf, ftptr{0}, ftsrc;      // table pairs (source box ids)
    double x0 = 0.0, fxmax = 0.0, fylo = INFINITY, fyhi = 0.0;
  };
  std::vector<IfClass> ifc;
  {
    double y0 = INFINITY;
    for (const IfPair& p : ifp) y0 = std::min(y0, p.ylo);
    y0 = std::max(y0, 1e-12);
    for (IfPair& p : ifp)
      p.cls = std::min(kIfClasses - 1, (int)std::floor(std::log2(std::max(p.ylo, y0) / y0)));
    std::stable_sort(ifp.begin(), ifp.end(), [](const IfPair& a, const IfPair& b) { return a.cls < b.cls; });
    std::vector<int> slot_of(nb, -1);
    for (size_t a = 0; a < ifp.size();) {
      size_t b = a;
      double yall = 0.0, wall = 0.0;
      for (; b < ifp.size() && ifp[b].cls == ifp[a].cls; ++b) {
        yall = std::max(yall, ifp[b].yhi);
        wall = std::max(wall, ifp[b].tw);
      }
      IfClass C;
      C.x0 = std::max(std::min(yall, wall), 1e-3 * yall);
      // HFMM_IFACE_TABLE=0 in the environment: every pair by quadrature
      // (diagnostics and tests)
      if (const char* env = std::getenv("HFMM_IFACE_TABLE"))
        if (env[0] == '0') C.x0 = INFINITY;
      for (size_t i = a; i < b; ++i) {  // leaves in order, each one's pairs together
        const IfPair& p = ifp[i];
        if (p.gap >= C.x0) {
          if (C.ftleaf.empty() || C.ftleaf.back() != leaves[p.li]) {
            if (!C.ftleaf.empty()) C.ftptr.push_back((int)C.ftsrc.size());
            C.ftleaf.push_back(leaves[p.li]);
          }
          C.ftsrc.push_back(p.sb);
          C.fxmax = std::max(C.fxmax, p.xsp);
          C.fylo = std::min(C.fylo, p.ylo);
          C.fyhi = std::max(C.fyhi, p.yhi);
          continue;
        }
        if (C.tleaf.empty() || C.tleaf.back() != leaves[p.li]) {
          if (!C.tleaf.empty()) C.tptr.push_back((int)C.tsrc.size());
          C.tleaf.push_back(leaves[p.li]);
        }
        if (slot_of[p.sb] < 0) {
          slot_of[p.sb] = (int)C.sbox.size();
          C.sbox.push_back(p.sb);
        }
        C.tsrc.push_back(slot_of[p.sb]);
        C.xsp = std::max(C.xsp, p.xsp);
        C.ylo = std::min(C.ylo, p.ylo);
        C.yhi = std::max(C.yhi, p.yhi);
      }
      if (!C.tleaf.empty()) C.tptr.push_back((int)C.tsrc.size());
      if (!C.ftleaf.empty()) C.ftptr.push_back((int)C.ftsrc.size());
      for (int sb : C.sbox) slot_of[sb] = -1;
      ifc.push_back(std::move(C));
      a = b;
    }
  }
  // H0 series class of a (target leaf, source range) pair from the largest
  // z = (k r / 2)^2 its two boxes allow
  const double qk2 = 0.25 * pl->med.k1 * pl->med.k1;
  auto series_class = [&](const double4& t, const double4& r) {
    const double dx = std::max(t.y - r.x, r.y - t.x), dy = std::max(t.w - r.z, r.w - t.z);
    const double zmax = qk2 * (dx * dx + dy * dy);
    int c = 0;
    while (c < kH0Classes && zmax > kH0ClassZmax[c]) ++c;
    return c;
  };
  // Split every leaf's merged ranges at its own points: the part before the
  // leaf, the leaf itself, and the part after it. The direct-pair relation is
  // symmetric (leaf T lists leaf S exactly when S lists T), so the pairs of T
  // with the leaves after it are evaluated once, in T's cross items, and the
  // parts before are dropped. The plan checks the symmetry leaf pair by leaf
  // pair and otherwise keeps every ordered pair in one-sided items.
  const int nl = (int)leaves.size();
  std::vector<std::vector<int2>> before(nl), self_r(nl), after(nl);
  for (int li = 0; li < nl; ++li) {
    const int tb = B[leaves[li]].begin, te = B[leaves[li]].end;
    for (const int2& rg : u_per[li]) {
      if (rg.x < std::min(rg.y, tb)) before[li].push_back(make_int2(rg.x, std::min(rg.y, tb)));
      if (std::max(rg.x, tb) < std::min(rg.y, te)) self_r[li].push_back(make_int2(std::max(rg.x, tb), std::min(rg.y, te)));
      if (std::max(rg.x, te) < rg.y) after[li].push_back(make_int2(std::max(rg.x, te), rg.y));
    }
  }
  bool symmetric = true;
  {
    std::vector<std::pair<int, int>> fwd, rev;  // (earlier leaf, later leaf)
    for (int li = 0; li < nl; ++li) {
      for (const int2& r : after[li])
        for (int j = r.x; j < r.y;) {
          const int lj = leaf_at[j];
          if (lj < 0) { symmetric = false; break; }
          fwd.emplace_back(li, lj);
          j = B[leaves[lj]].end;
        }
      for (const int2& r : before[li])
        for (int j = r.x; j < r.y;) {
          const int lj = leaf_at[j];
          if (lj < 0) { symmetric = false; break; }
          rev.emplace_back(lj, li);
          j = B[leaves[lj]].end;
        }
    }
    std::sort(fwd.begin(), fwd.end());
    std::sort(rev.begin(), rev.end());
    symmetric = symmetric && fwd == rev;
  }
  pl->p2p_symmetric = symmetric;
  // direct work items: a target leaf, one series class, at most kItemSources
  // sources; cross items (sym) when the relation is symmetric. Per class,
  // largest first.
  struct Item {
    int leaf;
    int sym;
    int cls;
    int64_t cost;
    std::vector<int2> r;
  };
  std::vector<Item> items;
  auto add_ranges = [&](int li, const std::vector<int2>& rs, int sym) {
    const size_t first = items.size();
    // about kItemPairs[c] pairs per item, so that no single wave dominates a launch
    const int nt_leaf = B[leaves[li]].end - B[leaves[li]].begin;
    std::vector<int2> by_cls[kH0Classes + 1];
    for (const int2& rg : rs) by_cls[series_class(leaf_bb[li], range_bb(rg))].push_back(rg);
    for (int c = 0; c <= kH0Classes; ++c) {
      const int cap = std::max(64, std::min(kItemSources, (kItemPairs[c] / std::max(nt_leaf, 1)) & ~63));
      Item cur{leaves[li], sym, c, 0, {}};
      int cur_n = 0;
      for (const int2& rg : by_cls[c]) {
        int a = rg.x;
        while (a < rg.y) {
          int take = std::min(rg.y - a, cap - cur_n);
          cur.r.push_back(make_int2(a, a + take));
          cur_n += take;
          a += take;
          if (cur_n == cap) {
            items.push_back(cur);
            cur = Item{leaves[li], sym, c, 0, {}};
            cur_n = 0;
          }
        }
      }
      if (cur_n > 0) items.push_back(cur);
    }
    const int nt = B[leaves[li]].end - B[leaves[li]].begin;
    for (size_t it = first; it < items.size(); ++it) {
      int64_t ns = 0;
      for (auto& r : items[it].r) ns += r.y - r.x;
      const int c = items[it].cls;
      // per pair: the two series chains plus about 24 operations of logarithm
      // and update, and 10 more for the reverse sum of a cross item
      items[it].cost = ns * nt * (2 * kH0ClassTerms[c < kH0Classes ? c : kH0Classes - 1] + 24 + (sym ? 10 : 0));
    }
  };
  for (int li = 0; li < nl; ++li) {
    if (symmetric) {
      add_ranges(li, self_r[li], 0);
      add_ranges(li, after[li], 1);
    } else {
      add_ranges(li, u_per[li], 0);
    }
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
    return a.cls != b.cls ? a.cls < b.cls : a.cost > b.cost;
  });
  for (int c = 0; c <= kH0Classes + 1; ++c) pl->p2p_cls_ptr[c] = 0;
  for (auto& it : items) ++pl->p2p_cls_ptr[it.cls + 1];
  for (int c = 1; c <= kH0Classes + 1; ++c) pl->p2p_cls_ptr[c] += pl->p2p_cls_ptr[c - 1];
  std::vector<int> p2p_ptr(1, 0), p2p_items, p2p_sym;
  std::vector<int2> p2p_rng;
  int64_t p2p_evals = 0;
  double p2p_flops = 0.0;
  for (auto& it : items) {
    p2p_items.push_back(it.leaf);
    p2p_sym.push_back(it.sym);
    p2p_rng.insert(p2p_rng.end(), it.r.begin(), it.r.end());
    p2p_ptr.push_back((int)p2p_rng.size());
    int64_t ns = 0;
    for (auto& r : it.r) ns += r.y - r.x;
    const int64_t ev = ns * (B[it.leaf].end - B[it.leaf].begin);
    p2p_evals += ev;
    // flops of one evaluation: two Horner chains of M terms (4M), the
    // table logarithm (21), distance and assembly (11), and a complex
    // multiply-add per direction (8 each)
    const int M = kH0ClassTerms[it.cls < kH0Classes ? it.cls : kH0Classes - 1];
    p2p_flops += (double)ev * (4.0 * M + 32.0 + (it.sym ? 16.0 : 8.0));
  }
  pl->p2p_evals = p2p_evals;
  pl->p2p_flops = p2p_flops;

  phase("direct lists");
  // ---- lists of the right-hand-side-blocked pipeline: per target box its
  // translation pairs (M2M: its children, L2L: its parent, M2L: its free and
  // image pairs), the direct pairs in pieces of 16 targets, the offsets of the
  // leaves' expansion matrices and the per-level scale factors of the
  // reduced-precision multipole-to-local contraction
  std::vector<TgItem> tg_items_h;
  std::vector<TgPair> tg_pairs_h;
  std::vector<int64_t> coff16_h(nb, 0);
  std::vector<BpItem> bp_items_h;
  std::vector<int2> bp_rng_h;
  std::vector<int64_t> voff_h;
  std::vector<double> scale_h;
  // reduced-precision operators of the multipole-to-local tables (made
  // after the tables): per table its Toeplitz offset, order, level, image
  // flag and the offset of its scaled operator
  std::vector<int64_t> lo_toff, lo_off;
  std::vector<int> lo_P, lo_lev, lo_img;
  int64_t lo_tot = 0;
  {
    const int mprec = o.precision == HFMM_FP64 ? BLK_F64 : (o.precision == HFMM_FP32 ? BLK_F32 : BLK_BF16);
    pl->blk_prec_m2l = mprec;
    pl->blk_prec_p2p = o.precision == HFMM_FP64 ? BLK_F64 : BLK_F32;
    int64_t c16 = 0;
    for (int i = 0; i < nb; ++i) {
      coff16_h[i] = c16;
      if (B[i].level >= 2) c16 += (2 * pl->P[B[i].level] + 1 + 15) & ~15;
    }
    pl->ctot16 = c16;
    auto toff_of = [&](int id, int Ps, int Pd) { return tabs[id].off + tabs[id].half - (Ps + Pd); };
    // the items of one target: groups of at most ntmax row tiles sharing its pairs
    auto add_target = [&](hfmm_plan_s::TgGroup& g, int prec, int t, int Ps, int Pd, int ntmax, int pbeg) {
      const int Md = 2 * Pd + 1, nrt = (2 * Md + 15) / 16;
      for (int rt = 0; rt < nrt; rt += ntmax) {
        const int nt = std::min(ntmax, nrt - rt);
        tg_items_h.push_back(TgItem{coff[t], pbeg, (int)tg_pairs_h.size(), rt, nt, Ps, Pd, B[t].level, 0});
        g.buf = std::max(g.buf, tgemm_buf_elems(prec, Ps, Pd, std::min(8 * nt, Md - 8 * rt)));
      }
    };
    // M2L: every box of levels >= top is a target (without pairs its rows are cleared)
    std::map<int, int64_t> lo_of;  // table id -> offset of its scaled operator
    auto lo_offset = [&](int id, int l, int img) -> int64_t {
      if (mprec == BLK_F64) return 0;
      auto it = lo_of.find(id);
      if (it != lo_of.end()) return it->second;
      const int Pl = pl->P[l], M = 2 * Pl + 1, Ms16 = (M + 15) & ~15;
      const int64_t o = lo_tot;
      lo_tot += mprec == BLK_F32 ? (int64_t)M * ((M + 7) & ~7) : (int64_t)(2 * M) * (2 * Ms16);
      lo_of[id] = o;
      lo_toff.push_back(toff_of(id, Pl, Pl));
      lo_P.push_back(Pl);
      lo_lev.push_back(l);
      lo_img.push_back(img);
      lo_off.push_back(o);
      return o;
    };
    std::vector<std::vector<std::pair<int, int>>> m2l_of(nb);  // (pair index, image)
    for (size_t i = 0; i < fv.size(); ++i) m2l_of[fv[i].t].push_back({(int)i, 0});
    for (size_t i = 0; i < iv.size(); ++i) m2l_of[iv[i].t].push_back({(int)i, 1});
    // the pairs of every target once; its items for each candidate tile shape
    std::vector<int> m2l_pbeg(nb, 0), m2l_pend(nb, 0);
    for (int t = pl->lev_begin[pl->top]; t < nb; ++t) {
      const int Pl = pl->P[B[t].level];
      m2l_pbeg[t] = (int)tg_pairs_h.size();
      for (auto& pr : m2l_of[t]) {
        const int src = pr.second ? iv[pr.first].s : fv[pr.first].s;
        const int id = pr.second ? iv_tab[pr.first] : fv_tab[pr.first];
        tg_pairs_h.push_back(
            TgPair{coff[src], toff_of(id, Pl, Pl), coff16_h[src], lo_offset(id, B[t].level, pr.second), pr.second, 0});
      }
      m2l_pend[t] = (int)tg_pairs_h.size();
    }
    for (int c = 0; c < hfmm_plan_s::kTileCands; ++c) {
      pl->m2l_tgl[c].assign(pl->nlev, hfmm_plan_s::TgGroup{});
      for (int l = pl->top; l < pl->nlev; ++l) {
        auto& g = pl->m2l_tgl[c][l];
        g.first = (int)tg_items_h.size();
        const int Pl = pl->P[l];
        const int Md = 2 * Pl + 1, nrt = (2 * Md + 15) / 16;
        const int ntmax = std::min(hfmm_plan_s::kTileNt[c], tgemm_max_nt(mprec, Pl));
        const int tend = l + 1 < pl->nlev ? pl->lev_begin[l + 1] : nb;
        for (int t = pl->lev_begin[l]; t < tend; ++t) {
          for (int rt = 0; rt < nrt; rt += ntmax) {
            const int nt = std::min(ntmax, nrt - rt);
            tg_items_h.push_back(TgItem{coff[t], m2l_pbeg[t], m2l_pend[t], rt, nt, Pl, Pl, l, 0});
            g.buf = std::max(g.buf, tgemm_buf_elems(mprec, Pl, Pl, std::min(8 * nt, Md - 8 * rt)));
          }
        }
        g.count = (int)tg_items_h.size() - g.first;
      }
    }
    // M2M (children to parent) and L2L (parent to child) per parent level
    pl->m2m_tg.assign(pl->nlev, hfmm_plan_s::TgGroup{});
    pl->l2l_tg.assign(pl->nlev, hfmm_plan_s::TgGroup{});
    for (int l = pl->top; l + 1 < pl->nlev; ++l) {
      auto& gu = pl->m2m_tg[l];
      gu.first = (int)tg_items_h.size();
      for (int t = pl->lev_begin[l]; t < pl->lev_begin[l + 1]; ++t) {
        if (B[t].leaf) continue;
        const int pbeg = (int)tg_pairs_h.size();
        for (int q = 0; q < 4; ++q) {
          const int c = B[t].child[q];
          if (c >= 0) tg_pairs_h.push_back(TgPair{coff[c], pl->m2m_q4[l].v[q], 0, 0, 0, 0});
        }
        add_target(gu, BLK_F64, t, pl->P[l + 1], pl->P[l], kUpDownNt, pbeg);
      }
      gu.count = (int)tg_items_h.size() - gu.first;
      auto& gd = pl->l2l_tg[l];
      gd.first = (int)tg_items_h.size();
      for (int c = pl->lev_begin[l + 1]; c < pl->lev_begin[l + 2]; ++c) {
        const int pbeg = (int)tg_pairs_h.size();
        tg_pairs_h.push_back(TgPair{coff[B[c].parent], pl->l2l_q4[l].v[B[c].quad], 0, 0, 0, 0});
        add_target(gd, BLK_F64, c, pl->P[l], pl->P[l + 1], kUpDownNt, pbeg);
      }
      gd.count = (int)tg_items_h.size() - gd.first;
    }
    // direct pairs: every leaf in pieces of 16 targets against its merged
    // direct ranges, one item per series class (the class from the leaf's
    // and the range's bounding boxes); the pieces of a leaf share the ranges
    std::vector<BpItem> by_cls[kH0Classes + 1];
    for (int li = 0; li < nl; ++li) {
      const int tb = B[leaves[li]].begin, te = B[leaves[li]].end;
      std::vector<int2> rc[kH0Classes + 1];
      for (const int2& rg : u_per[li]) rc[series_class(leaf_bb[li], range_bb(rg))].push_back(rg);
      for (int c = 0; c <= kH0Classes; ++c) {
        if (rc[c].empty()) continue;
        const int rb = (int)bp_rng_h.size();
        bp_rng_h.insert(bp_rng_h.end(), rc[c].begin(), rc[c].end());
        const int re = (int)bp_rng_h.size();
        for (int t0 = tb; t0 < te; t0 += 16) by_cls[c].push_back(BpItem{t0, std::min(16, te - t0), rb, re});
      }
    }
    pl->bp_cls_ptr[0] = 0;
    for (int c = 0; c <= kH0Classes; ++c) {
      bp_items_h.insert(bp_items_h.end(), by_cls[c].begin(), by_cls[c].end());
      pl->bp_cls_ptr[c + 1] = (int)bp_items_h.size();
    }
    // expansion matrices of the leaves of levels >= 2 (leaf order)
    int64_t vo = 0;
    for (int i = pl->leaf_lev[std::min(2, pl->nlev)]; i < nl; ++i) {
      voff_h.push_back(vo);
      const Box& bx = B[leaves[i]];
      vo += (int64_t)(2 * pl->P[bx.level] + 1) * (bx.end - bx.begin);
    }
    pl->vmat_tot = vo;
    // a_l(n): |J_n(k R_l)| (R_l the box radius) where n > k R_l, 1 below;
    // J_n(k rho) of every point of a box of level l is bounded by it there
    scale_h.assign((size_t)pl->nlev * kScaleStride, 1.0);
    for (int l = 2; l < pl->nlev; ++l) {
      const double kR = k * pl->bsize[l] * std::sqrt(0.5);
      for (int nn = 0; nn <= pl->P[l]; ++nn) {
        double a = 1.0;
        if (nn > kR) a = std::min(1.0, 2.0 * host_absj(kR, nn));
        scale_h[(size_t)l * kScaleStride + nn] = std::max(a, 1e-250);
      }
    }
    bool staged = true;  // every translation's operator fits the staging of the kernel
    for (int l = pl->top; l < pl->nlev; ++l) {
      staged = staged && tgemm_supported(mprec, pl->P[l], pl->P[l]);
      if (l + 1 < pl->nlev)
        staged = staged && tgemm_supported(BLK_F64, pl->P[l + 1], pl->P[l]) &&
                 tgemm_supported(BLK_F64, pl->P[l], pl->P[l + 1]);
    }
    pl->blk_ok = pl->leaf_pmax <= kBlkLeafPmax && staged;
  }
  if (o.deterministic && !pl->blk_ok) {
    fail(HFMM_ERR_UNSUPPORTED,
         "deterministic mode runs every apply through the right-hand-side-blocked pipeline, which this plan cannot "
         "use (a leaf expansion order above " + std::to_string(kBlkLeafPmax) + ")");
    return bail(HFMM_ERR_UNSUPPORTED);
  }

  phase("blocked lists");
  // ---- near-interface rules. Their t ranges end where e^{-t Y_min} has
  // fallen to tol / 100 (times e^-3): past it the tail of the integral, about
  // e^{-t Y} / (t Y), is below the plan's accuracy.
  const double if_cut = std::log(100.0 / pl->tol) + 3.0;
  std::vector<double2> qc, qky, qkx;
  double glx[16], glw[16];
  gauss_legendre16(glx, glw);
  // nodes of a rule as G^s(X, Y) = sum_q c_q exp(ky_q Y + kx_q X)
  auto rule_nodes = [&](const Rule& r, std::vector<double2>& nc, std::vector<double2>& nky,
                        std::vector<double2>& nkx) {
    const double inv4pi = 0.25 / M_PI;
    for (auto& pn : r.panels) {
      double hw = 0.5 * (pn.b - pn.a), mid = 0.5 * (pn.a + pn.b);
      for (int g = 0; g < 16; ++g) {
        double s = mid + hw * glx[g], w = hw * glw[g];
        if (pn.kind == 0) {
          double st = std::sin(s), ct = std::cos(s);
          double2 sig = sigma1_tau(pl->med, ct, st);
          // (i/4)(1/pi) w sigma e^{i k (Y st - X ct)}
          nc.push_back(cmul(cmk(0.0, 0.25 / M_PI * w), sig));
          nky.push_back(cmk(0.0, k * st));
          nkx.push_back(cmk(0.0, -k * ct));
        } else {
          double2 t = cmk(s, 0.0), dt = cmk(1.0, 0.0);
          if (s < r.send) {
            t = cmk(s, -r.dip * std::sin(M_PI * s / r.send));
            dt = cmk(1.0, -r.dip * M_PI / r.send * std::cos(M_PI * s / r.send));
          }
          double2 lam = csqrt2(cadd(cmul(t, t), cmk(k * k, 0.0)));
          double2 sig = sigma1_t(pl->med, t);
          double2 c = cdiv(cmul(cscale(dt, w * inv4pi), sig), lam);
          double2 il = cmul(cmk(0.0, 1.0), lam);
          nc.push_back(c); nky.push_back(cscale(t, -1.0)); nkx.push_back(il);
          nc.push_back(c); nky.push_back(cscale(t, -1.0)); nkx.push_back(cscale(il, -1.0));
        }
      }
    }
  };
  // one rule per class of near-interface pairs, over its X and Y ranges
  std::vector<int> if_node_off;
  for (const IfClass& C : ifc) {
    if (C.tleaf.empty()) {
      if_node_off.push_back((int)qc.size());
      continue;
    }
    Rule r = build_rule(pl->med, C.xsp, C.ylo, C.yhi, 0, if_cut, 8.0);
    if (!r.ok) {
      fail(HFMM_ERR_ACCURACY, "near-interface quadrature rule too long");
      return bail(HFMM_ERR_ACCURACY);
    }
    if_node_off.push_back((int)qc.size());
    rule_nodes(r, qc, qky, qkx);
    if (log_on())
      std::fprintf(stderr, "[hfmm] near-interface class: %zu leaves, %zu pairs, X <= %.3g, Y in [%.3g, %.3g]: %d nodes\n",
                   C.tleaf.size(), C.tsrc.size(), C.xsp, C.ylo, C.yhi, (int)qc.size() - if_node_off.back());
  }
  if_node_off.push_back((int)qc.size());
  // HFMM_SELF_NONE: a rule for X = 0 and Y over [2 ymin, 2 ymax] gives every
  // point's scattered self term and its height derivative
  std::vector<double2> sc_c, sc_ky, sc_kx;
  if (o.self_term == HFMM_SELF_NONE) {
    Rule r = build_rule(pl->med, 0.0, 2.0 * ymin, 2.0 * ymax, 0);
    if (!r.ok) {
      fail(HFMM_ERR_ACCURACY, "self-term quadrature rule too long");
      return bail(HFMM_ERR_ACCURACY);
    }
    rule_nodes(r, sc_c, sc_ky, sc_kx);
  }

  // ---- heterogeneous table rules
  std::vector<double> cX, cY, cdip, csend;
  std::vector<int> cpbeg(1, 0);
  std::vector<Panel> cpanels;
  // the rules are independent: built on a few host threads, joined in order
  std::vector<Rule> crules(combos.size());
  parallel_for((int)combos.size(), [&](int i) {
    const auto& cb = combos[i];
    const double b = pl->bsize[cb.level];
    crules[i] = build_rule(pl->med, cb.dix * b, 2.0 * ymin + (cb.m + 1) * b, 2.0 * ymin + (cb.m + 1) * b,
                           2 * pl->P[cb.level]);
  });
  for (size_t i = 0; i < combos.size(); ++i) {
    const auto& cb = combos[i];
    double b = pl->bsize[cb.level];
    double X = cb.dix * b;
    double Y = 2.0 * ymin + (cb.m + 1) * b;
    int N = 2 * pl->P[cb.level];
    if (2 * N + 1 > 256 * 8) {
      fail(HFMM_ERR_ACCURACY, "heterogeneous table order too large");
      return bail(HFMM_ERR_ACCURACY);
    }
    const Rule& r = crules[i];
    if (!r.ok) {
      fail(HFMM_ERR_ACCURACY, "heterogeneous table quadrature rule too long");
      return bail(HFMM_ERR_ACCURACY);
    }
    cX.push_back(X);
    cY.push_back(Y);
    cdip.push_back(r.dip);
    csend.push_back(r.send);
    cpanels.insert(cpanels.end(), r.panels.begin(), r.panels.end());
    cpbeg.push_back((int)cpanels.size());
  }

  phase("rules");
  // ---- upload and generate tables
  std::vector<double2> hpts((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    const int j = perm[i];
    hpts[i] = cmk(hp[2 * j], hp[2 * j + 1]);
  }
  std::vector<double2> hctr(nb);
  std::vector<int> hlev(nb), hpar(nb), hquad(nb), hchild(4 * nb);
  std::vector<int2> hpr(nb);
  for (int i = 0; i < nb; ++i) {
    double b = pl->bsize[B[i].level];
    hctr[i] = cmk(xmin + (B[i].ix + 0.5) * b, ymin + (B[i].iy + 0.5) * b);
    hlev[i] = B[i].level;
    hpar[i] = B[i].parent;
    hquad[i] = B[i].quad;
    for (int q = 0; q < 4; ++q) hchild[4 * i + q] = B[i].child[q];
    hpr[i] = make_int2(B[i].begin, B[i].end);
  }
  // pair lists as coefficient offsets of their boxes
  auto offsets_of = [&](const std::vector<int>& boxes_of_pairs) {
    std::vector<int64_t> o(boxes_of_pairs.size());
    for (size_t i = 0; i < o.size(); ++i) o[i] = coff[boxes_of_pairs[i]];
    return o;
  };
  const std::vector<int64_t> m2l_soff = offsets_of(m2l_psrc), m2l_toff = offsets_of(m2l_pdst);
  const std::vector<int64_t> cp_child_off = offsets_of(cp_child), cp_parent_off = offsets_of(cp_parent);
  std::vector<int> if_sbox, if_tleaf, if_tptr, if_tsrc;
  for (const IfClass& C : ifc) {
    if_sbox.insert(if_sbox.end(), C.sbox.begin(), C.sbox.end());
    if_tleaf.insert(if_tleaf.end(), C.tleaf.begin(), C.tleaf.end());
    if_tptr.insert(if_tptr.end(), C.tptr.begin(), C.tptr.end());
    if_tsrc.insert(if_tsrc.end(), C.tsrc.begin(), C.tsrc.end());
  }
  hipError_t e = hipSuccess;
#define UP(buf, vec)                                  \
  if (e == hipSuccess) e = pl->buf.upload(vec, stream);
  UP(pts, hpts) UP(ctr, hctr) UP(level, hlev) UP(parent, hpar) UP(quad, hquad)
  UP(child, hchild) UP(prange, hpr) UP(coff, coff) UP(leaves, leaves) UP(pt_box, pt_box_h)
  UP(m2l_items, m2l_items) UP(m2l_soff, m2l_soff) UP(m2l_toff, m2l_toff) UP(m2l_pcoff, m2l_pcoff) UP(m2l_pcoffT, m2l_pcoffT)
  UP(red_boxes, red_boxes) UP(red_ptr, red_ptr) UP(red_beg, red_beg) UP(redT_ptr, redT_ptr)
  UP(redT_beg, redT_beg) UP(cp_child, cp_child_off) UP(cp_parent, cp_parent_off) UP(up_doff, up_doff_h) UP(up_soff4, up_soff4_h) UP(up_items, up_items)
  UP(down_items, down_items) UP(tabs, tabs) UP(p2p_ptr, p2p_ptr)
  UP(p2p_items, p2p_items) UP(p2p_sym, p2p_sym) UP(p2p_rng, p2p_rng) UP(if_sbox, if_sbox) UP(if_tleaf, if_tleaf) UP(if_tptr, if_tptr) UP(if_tsrc, if_tsrc) UP(qc, qc)
  UP(qky, qky) UP(qkx, qkx)
  UP(tg_items, tg_items_h) UP(tg_pairs, tg_pairs_h) UP(bp_items, bp_items_h) UP(bp_rng, bp_rng_h)
  UP(vmat_off, voff_h) UP(blk_scale, scale_h) UP(coff16, coff16_h)
  // node sums of the near-interface stages, for groups of up to kIfRhs
  // right-hand sides (fewer where the group would pass kIfBufBudget)
  {
    size_t s_max = 0, t_max = 0;
    for (size_t c = 0; c < ifc.size(); ++c) {
      const size_t nqp = (size_t)(if_node_off[c + 1] - if_node_off[c] + 63) / 64 * 64;
      s_max = std::max(s_max, nqp * ifc[c].sbox.size());
      t_max = std::max(t_max, nqp * ifc[c].tleaf.size());
    }
    int rif = kIfRhs;
    while (rif > 1 && sizeof(double2) * (s_max + t_max) * (size_t)rif > kIfBufBudget) rif /= 2;
    if (e == hipSuccess) e = pl->if_S.alloc(s_max * rif);
    if (e == hipSuccess) e = pl->if_T.alloc(t_max * rif);
    pl->ifl.assign(ifc.size(), IfaceLists{});
    for (IfaceLists& L : pl->ifl) L.rif = rif;
  }
  DevBuf<double> d_fhdx, d_fhdy, d_fbdx, d_fbdy, d_cX, d_cY, d_cdip, d_csend, d_glx, d_glw;
  DevBuf<int> d_fhref, d_fbsgn, d_fbref, d_cpbeg, d_imgref;
  DevBuf<Panel> d_cpanels;
  std::vector<double> vglx(glx, glx + 16), vglw(glw, glw + 16);
  std::vector<TableRef> fh_refs, fb_refs, img_refs;
  for (int id : fh_ref) fh_refs.push_back(tabs[id]);
  for (int id : fb_ref) fb_refs.push_back(tabs[id]);
  for (int id : img_ref) img_refs.push_back(tabs[id]);
  DevBuf<TableRef> d_fhr, d_fbr, d_imr;
  // the image tables: blocks per table so that the launch has about 2048
  // blocks (at most 32 per table); their partial tables one after another
  const int img_split = combos.empty() ? 1 : (int)std::min<size_t>(32, std::max<size_t>(1, 2048 / combos.size()));
  std::vector<int64_t> img_soff;
  int64_t img_plen = 0;
  for (const TableRef& r : img_refs) {
    img_soff.push_back(img_plen);
    img_plen += 2 * r.half + 1;
  }
  DevBuf<int64_t> d_imsoff;
  DevBuf<double2> d_impart;
  if (img_split > 1) {
    if (e == hipSuccess) e = d_imsoff.upload(img_soff, stream);
    if (e == hipSuccess) e = d_impart.alloc((size_t)img_split * (size_t)std::max<int64_t>(img_plen, 1));
  }
  if (e == hipSuccess) e = d_fhdx.upload(fh_dx, stream);
  if (e == hipSuccess) e = d_fhdy.upload(fh_dy, stream);
  if (e == hipSuccess) e = d_fhr.upload(fh_refs, stream);
  if (e == hipSuccess) e = d_fbdx.upload(fb_dx, stream);
  if (e == hipSuccess) e = d_fbdy.upload(fb_dy, stream);
  if (e == hipSuccess) e = d_fbsgn.upload(fb_sgn, stream);
  if (e == hipSuccess) e = d_fbr.upload(fb_refs, stream);
  if (e == hipSuccess) e = d_cX.upload(cX, stream);
  if (e == hipSuccess) e = d_cY.upload(cY, stream);
  if (e == hipSuccess) e = d_cdip.upload(cdip, stream);
  if (e == hipSuccess) e = d_csend.upload(csend, stream);
  if (e == hipSuccess) e = d_cpbeg.upload(cpbeg, stream);
  if (e == hipSuccess) e = d_cpanels.upload(cpanels, stream);
  if (e == hipSuccess) e = d_imr.upload(img_refs, stream);
  if (e == hipSuccess) e = d_glx.upload(vglx, stream);
  if (e == hipSuccess) e = d_glw.upload(vglw, stream);
  if (e == hipSuccess) e = pl->tdata.alloc((size_t)std::max<int64_t>(toff, 1));
  DevBuf<double2> d_scc, d_scky;
  if (o.self_term == HFMM_SELF_NONE) {
    if (e == hipSuccess) e = d_scc.upload(sc_c, stream);
    if (e == hipSuccess) e = d_scky.upload(sc_ky, stream);
    if (e == hipSuccess) e = pl->self_g.alloc((size_t)n);
    if (e == hipSuccess) e = pl->self_dy.alloc((size_t)n);
    if (e == hipSuccess)
      launch_self_term(stream, (int)n, pl->pts.p, (int)sc_c.size(), d_scc.p, d_scky.p, pl->self_g.p, pl->self_dy.p);
  }
  if (e == hipSuccess) {
    launch_table_hankel(stream, (int)fh_ref.size(), d_fhdx.p, d_fhdy.p, d_fhr.p, k, pl->tdata.p);
    launch_table_bessel(stream, (int)fb_ref.size(), d_fbdx.p, d_fbdy.p, d_fbsgn.p, d_fbr.p, k, pl->tdata.p);
    launch_table_image(stream, pl->med, (int)combos.size(), d_cX.p, d_cY.p, d_cdip.p, d_csend.p, d_cpbeg.p,
                       d_cpanels.p, d_imr.p, d_glx.p, d_glw.p, pl->tdata.p, img_split, d_imsoff.p, d_impart.p,
                       img_plen);
    e = hipGetLastError();
  }
  DevBuf<int64_t> d_lotoff, d_looff;
  DevBuf<int> d_loP, d_lolev, d_loimg;
  if (e == hipSuccess && !lo_off.empty()) {
    e = pl->olo.alloc((size_t)lo_tot * (pl->blk_prec_m2l == BLK_F32 ? 8 : 2));
    if (e == hipSuccess) e = d_lotoff.upload(lo_toff, stream);
    if (e == hipSuccess) e = d_looff.upload(lo_off, stream);
    if (e == hipSuccess) e = d_loP.upload(lo_P, stream);
    if (e == hipSuccess) e = d_lolev.upload(lo_lev, stream);
    if (e == hipSuccess) e = d_loimg.upload(lo_img, stream);
    if (e == hipSuccess) {
      launch_lo_tables(stream, pl->blk_prec_m2l, (int)lo_off.size(), d_lotoff.p, d_loP.p, d_lolev.p, d_loimg.p,
                       d_looff.p, pl->blk_scale.p, kScaleStride, pl->tdata.p, pl->olo.p);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  d_fhdx.release(); d_fhdy.release(); d_fbdx.release(); d_fbdy.release(); d_cX.release(); d_cY.release();
  d_cdip.release(); d_csend.release(); d_glx.release(); d_glw.release(); d_fhref.release(); d_fbsgn.release();
  d_fbref.release(); d_cpbeg.release(); d_imgref.release(); d_cpanels.release(); d_fhr.release();
  d_fbr.release(); d_imr.release(); d_scc.release(); d_scky.release();
  d_lotoff.release(); d_looff.release(); d_loP.release(); d_lolev.release(); d_loimg.release();
  d_imsoff.release(); d_impart.release();
  if (e != hipSuccess) {
    fail(e == hipErrorOutOfMemory ? HFMM_ERR_NO_MEMORY : HFMM_ERR_DEVICE,
         std::string("plan upload/tables: ") + hipGetErrorString(e));
    return bail(e == hipErrorOutOfMemory ? HFMM_ERR_NO_MEMORY : HFMM_ERR_DEVICE);
  }
  pl->nleaves = (int)leaves.size();
  pl->np2p_items = (int)p2p_items.size();
  pl->nred_boxes = (int)red_boxes.size();
  {
    size_t o_sb = 0, o_tl = 0, o_tp = 0, o_ts = 0;
    for (size_t c = 0; c < ifc.size(); ++c) {
      IfaceLists& L = pl->ifl[c];
      L.nsb = (int)ifc[c].sbox.size();
      L.ntl = (int)ifc[c].tleaf.size();
      L.nq = if_node_off[c + 1] - if_node_off[c];
      L.nqp = (L.nq + 63) / 64 * 64;
      L.sbox = pl->if_sbox.p + o_sb;
      L.tleaf = pl->if_tleaf.p + o_tl;
      L.tptr = pl->if_tptr.p + o_tp;
      L.tsrc = pl->if_tsrc.p + o_ts;
      L.qc = pl->qc.p + if_node_off[c];
      L.qky = pl->qky.p + if_node_off[c];
      L.qkx = pl->qkx.p + if_node_off[c];
      L.S = pl->if_S.p;
      L.T = pl->if_T.p;
      o_sb += ifc[c].sbox.size();
      o_tl += ifc[c].tleaf.size();
      o_tp += ifc[c].tptr.size();
      o_ts += ifc[c].tsrc.size();
    }
  }

  // ---- tables of the horizontally separated near-interface pairs. Panel
  // sizes for a relative error tol / 100 with kIfTP Chebyshev points: the
  // Bernstein ellipse of a panel [a, a + w] of |X| stays clear of the
  // singularities at X = +-iY when w <= 2 a / (A - 1), A = (rho + 1 / rho) / 2,
  // rho^P = 100 / tol; the wave part e^{i k X} (k up to the largest wavenumber
  // of the medium, or of the impedance surface wave) needs half widths with
  // (k h / 2)^P / P! <= tol / 100. Y panels likewise, X >= X0 away.
  int64_t if_table_pairs = 0;
  {
    const double tol_eff = 0.01 * pl->tol;
    const double rho = std::pow(1.0 / tol_eff, 1.0 / kIfTP);
    const double A = 0.5 * (rho + 1.0 / rho);
    double kmax = std::max(pl->med.k1, std::max(pl->med.k2, pl->med.k3));
    if (pl->med.layers == 1) kmax = std::hypot(pl->med.k1, pl->med.alpha);
    double fact = 1.0;
    for (int i = 2; i <= kIfTP; ++i) fact *= i;
    const double wosc = 4.0 * std::pow(fact * tol_eff, 1.0 / kIfTP) / kmax;
    double cosm[kIfTP][kIfTP];  // cos(pi a (m + 1/2) / P)
    for (int a = 0; a < kIfTP; ++a)
      for (int m = 0; m < kIfTP; ++m) cosm[a][m] = std::cos(M_PI * a * (m + 0.5) / kIfTP);
    std::vector<int> tl_all, tp_all, ts_all, it_all;
    std::vector<int2> ie_all;
    std::vector<double4> xe_all;
    std::vector<int2> yp_all;
    std::vector<double2> cf_all;
    std::vector<size_t> offs;  // per table: tleaf, tptr, tsrc, xpan, coef, item offsets
    for (const IfClass& C : ifc) {
      if (C.ftleaf.empty()) continue;
      IfTable T{};
      const double g = 1.0 + 2.0 / (A - 1.0);
      std::vector<double> xe{C.x0};
      int p1 = 0;
      while (xe.size() < 2 || xe.back() < C.fxmax) {
        const double a = xe.back();
        if (p1 == (int)xe.size() - 1 && 2.0 * a / (A - 1.0) < wosc) {
          xe.push_back(a * g);
          ++p1;
        } else {
          xe.push_back(xe[p1] + (double)((int)xe.size() - p1) * wosc);
        }
        if (xe.size() > 200000) {
          fail(HFMM_ERR_ACCURACY, "near-interface table too long");
          return bail(HFMM_ERR_ACCURACY);
        }
      }
      T.npx = (int)xe.size() - 1;
      T.x0 = C.x0;
      T.p1 = p1;
      T.a1 = xe[p1];
      T.wmax = wosc;
      T.inv_x0 = 1.0 / C.x0;
      T.inv_wmax = 1.0 / wosc;
      T.inv_lg2 = (float)(1.0 / std::log2(g));
      // Y panels per panel of |X|: the singularities in Y sit |X| off the
      // real axis, so the farther panels take wider ones
      const double yr = std::max(C.fyhi - C.fylo, 1e-12 * std::max(1.0, C.fylo));
      T.ylo = C.fylo;
      std::vector<double4> xp(T.npx);
      std::vector<int2> yp(T.npx);
      int64_t npan = 0;
      for (int px = 0; px < T.npx; ++px) {
        const double wy_max = std::min(2.0 * xe[px] / (A - 1.0), wosc);
        const int npy = std::max(1, (int)std::ceil(yr / wy_max));
        xp[px] = make_double4(xe[px], 1.0 / (xe[px + 1] - xe[px]), yr / npy, npy / yr);
        yp[px] = make_int2(npy, (int)npan);
        npan += npy;
      }
      if (npan > kIfMaxPanels) {
        fail(HFMM_ERR_ACCURACY, "near-interface table of " + std::to_string(npan) +
                                    " panels: too large (raise leaf_size or keep interface_refine on)");
        return bail(HFMM_ERR_ACCURACY);
      }
      // values at the panels' Chebyshev points from one rule over the whole range
      const int64_t npts = npan * kIfTP * kIfTP;
      std::vector<double2> gxy((size_t)npts);
      for (int px = 0; px < T.npx; ++px)
        for (int py = 0; py < yp[px].x; ++py)
          for (int m = 0; m < kIfTP; ++m)
            for (int nn = 0; nn < kIfTP; ++nn) {
              const double u = std::cos(M_PI * (m + 0.5) / kIfTP), v = std::cos(M_PI * (nn + 0.5) / kIfTP);
              const double X = 0.5 * (xe[px] + xe[px + 1]) + 0.5 * (xe[px + 1] - xe[px]) * u;
              const double wy = xp[px].z;
              const double Y = T.ylo + (py + 0.5) * wy + 0.5 * wy * v;
              gxy[(((size_t)(yp[px].y + py)) * kIfTP + m) * kIfTP + nn] = cmk(X, Y);
            }
      Rule r = build_rule(pl->med, xe.back(), C.fylo, C.fylo + yr, 0, if_cut);
      if (!r.ok) {
        fail(HFMM_ERR_ACCURACY, "near-interface table rule too long");
        return bail(HFMM_ERR_ACCURACY);
      }
      std::vector<double2> rc, rky, rkx;
      rule_nodes(r, rc, rky, rkx);
      if ((double)npts * (double)rc.size() > kIfMaxGridWork) {
        fail(HFMM_ERR_ACCURACY, "near-interface table: " + std::to_string(npts) + " points x " +
                                    std::to_string(rc.size()) +
                                    " rule nodes is too costly to tabulate (raise leaf_size or keep interface_refine on)");
        return bail(HFMM_ERR_ACCURACY);
      }
      DevBuf<double2> d_xy, d_c, d_ky, d_kx, d_out;
      hipError_t eg = d_xy.upload(gxy, stream);
      if (eg == hipSuccess) eg = d_c.upload(rc, stream);
      if (eg == hipSuccess) eg = d_ky.upload(rky, stream);
      if (eg == hipSuccess) eg = d_kx.upload(rkx, stream);
      if (eg == hipSuccess) eg = d_out.alloc((size_t)3 * npts);
      std::vector<double2> vals((size_t)3 * npts);
      if (eg == hipSuccess) {
        launch_if_grid(stream, (int)npts, d_xy.p, (int)rc.size(), d_c.p, d_ky.p, d_kx.p, d_out.p);
        eg = hipMemcpyAsync(vals.data(), d_out.p, sizeof(double2) * vals.size(), hipMemcpyDeviceToHost, stream);
      }
      if (eg == hipSuccess) eg = hipStreamSynchronize(stream);
      if (eg != hipSuccess) {
        fail(eg == hipErrorOutOfMemory ? HFMM_ERR_NO_MEMORY : HFMM_ERR_DEVICE,
             std::string("near-interface table: ") + hipGetErrorString(eg));
        return bail(eg == hipErrorOutOfMemory ? HFMM_ERR_NO_MEMORY : HFMM_ERR_DEVICE);
      }
      // coefficients c_ab = (2/P)^2 sum_mn f_mn cos(pi a (m+1/2)/P) cos(pi b (n+1/2)/P),
      // halved for a = 0 and for b = 0
      const size_t cf0 = cf_all.size();
      cf_all.resize(cf0 + (size_t)npan * 3 * kIfTri);
      std::vector<double2> tmp((size_t)kIfTP * kIfTP);
      for (int64_t pn = 0; pn < npan; ++pn)
        for (int f = 0; f < 3; ++f) {
          const double2* fv = vals.data() + (size_t)f * npts + (size_t)pn * kIfTP * kIfTP;
          for (int a = 0; a < kIfTP; ++a)
            for (int nn = 0; nn < kIfTP; ++nn) {
              double2 acc = cmk(0, 0);
              for (int m = 0; m < kIfTP; ++m) acc = cadd(acc, cscale(fv[m * kIfTP + nn], cosm[a][m]));
              tmp[a * kIfTP + nn] = acc;
            }
          double2* out = cf_all.data() + cf0 + ((size_t)pn * 3 + f) * kIfTri;
          int k = 0;  // rows a = 0, 1, ... of b < P - a, packed
          for (int a = 0; a < kIfTP; ++a)
            for (int b = 0; b < kIfTP - a; ++b) {
              double2 acc = cmk(0, 0);
              for (int nn = 0; nn < kIfTP; ++nn) acc = cadd(acc, cscale(tmp[a * kIfTP + nn], cosm[b][nn]));
              const double sc = (2.0 / kIfTP) * (2.0 / kIfTP) * (a == 0 ? 0.5 : 1.0) * (b == 0 ? 0.5 : 1.0);
              out[k++] = cscale(acc, sc);
            }
        }
      if (log_on())
        std::fprintf(stderr,
                     "[hfmm] near-interface table: %zu leaves, %zu pairs, |X| in [%.3g, %.3g], Y in [%.3g, %.3g]: "
                     "%d x %d panels (%lld in all) from a rule of %zu nodes\n",
                     C.ftleaf.size(), C.ftsrc.size(), C.x0, xe.back(), C.fylo, C.fylo + yr, T.npx, yp[0].x,
                     (long long)npan, rc.size());
      offs.insert(offs.end(), {tl_all.size(), tp_all.size(), ts_all.size(), xe_all.size(), cf0, it_all.size()});
      // work items for launches with atomic additions: four source boxes of
      // one leaf (one per wave of the block)
      for (int t = 0; t < (int)C.ftleaf.size(); ++t)
        for (int e = C.ftptr[t]; e < C.ftptr[t + 1]; e += 4) {
          it_all.push_back(t);
          ie_all.push_back(make_int2(e, std::min(e + 4, C.ftptr[t + 1])));
        }
      T.nitem = (int)(it_all.size() - offs.back());
      tl_all.insert(tl_all.end(), C.ftleaf.begin(), C.ftleaf.end());
      tp_all.insert(tp_all.end(), C.ftptr.begin(), C.ftptr.end());
      ts_all.insert(ts_all.end(), C.ftsrc.begin(), C.ftsrc.end());
      xe_all.insert(xe_all.end(), xp.begin(), xp.end());
      yp_all.insert(yp_all.end(), yp.begin(), yp.end());
      T.ntl = (int)C.ftleaf.size();
      pl->ift.push_back(T);
      if_table_pairs += (int64_t)C.ftsrc.size();
    }
    hipError_t et = pl->ift_tleaf.upload(tl_all, stream);
    if (et == hipSuccess) et = pl->ift_tptr.upload(tp_all, stream);
    if (et == hipSuccess) et = pl->ift_tsrc.upload(ts_all, stream);
    if (et == hipSuccess) et = pl->ift_xpan.upload(xe_all, stream);
    if (et == hipSuccess) et = pl->ift_ypan.upload(yp_all, stream);
    if (et == hipSuccess) et = pl->ift_coef.upload(cf_all, stream);
    if (et == hipSuccess) et = pl->ift_item_t.upload(it_all, stream);
    if (et == hipSuccess) et = pl->ift_item_e.upload(ie_all, stream);
    if (et != hipSuccess) {
      fail(et == hipErrorOutOfMemory ? HFMM_ERR_NO_MEMORY : HFMM_ERR_DEVICE,
           std::string("near-interface tables: ") + hipGetErrorString(et));
      return bail(et == hipErrorOutOfMemory ? HFMM_ERR_NO_MEMORY : HFMM_ERR_DEVICE);
    }
    for (size_t c = 0; c < pl->ift.size(); ++c) {
      IfTable& T = pl->ift[c];
      T.tleaf = pl->ift_tleaf.p + offs[6 * c];
      T.tptr = pl->ift_tptr.p + offs[6 * c + 1];
      T.tsrc = pl->ift_tsrc.p + offs[6 * c + 2];
      T.xpan = pl->ift_xpan.p + offs[6 * c + 3];
      T.ypan = pl->ift_ypan.p + offs[6 * c + 3];
      T.coef = pl->ift_coef.p + offs[6 * c + 4];
      T.item_t = pl->ift_item_t.p + offs[6 * c + 5];
      T.item_e = pl->ift_item_e.p + offs[6 * c + 5];
    }
  }

  phase("upload and tables");
  // ---- statistics
  hfmm_info_t& inf = pl->info;
  inf.levels = pl->nlev;
  for (int l = 0; l < pl->nlev && l < 32; ++l) inf.order[l] = pl->P[l];
  inf.boxes = nb;
  inf.leaves = (int64_t)leaves.size();
  inf.m2l_pairs = (int64_t)fv.size();
  inf.image_pairs = (int64_t)iv.size();
  inf.p2p_pairs = np2p;
  inf.interface_pairs = nifp;
  inf.interface_nodes = (int32_t)qc.size();
  inf.interface_leaf_pairs = (int64_t)if_tsrc.size() + if_table_pairs;
  inf.image_tables = (int64_t)combos.size();
  double fm2l = 0.0;
  for (auto& pr : fv) { double m = 2.0 * pl->P[B[pr.t].level] + 1; fm2l += 8.0 * m * m; }
  for (auto& pr : iv) { double m = 2.0 * pl->P[B[pr.t].level] + 1; fm2l += 8.0 * m * m; }
  inf.flops_m2l = fm2l;
  double fud = 0.0;
  for (int i = 0; i < nb; ++i) {
    int l = B[i].level;
    if (l < 2) continue;
    double m = 2.0 * pl->P[l] + 1;
    if (B[i].leaf) fud += 2.0 * (B[i].end - B[i].begin) * m * 8.0;  // P2M + L2P MACs
    if (l > pl->top) fud += 2.0 * 8.0 * m * (2.0 * pl->P[l - 1] + 1);  // M2M + L2L
  }
  inf.flops_updown = fud;
  inf.flops_p2p = pl->p2p_flops;
  inf.p2p_evals = pl->p2p_evals;
  inf.top_level = pl->top;
  if (o.max_nrhs > 0) {
    const int chunk = rhs_chunk(pl, o.max_nrhs);
    hfmm_status_t st = ensure_workspace(pl, chunk);
    if (st == HFMM_OK && (pl->gq.ensure((size_t)n * chunk) != hipSuccess || pl->gs.ensure((size_t)n) != hipSuccess))
      st = fail(HFMM_ERR_NO_MEMORY, "coordinate-gradient workspace");
    if (st != HFMM_OK) return bail(st);
  }
  inf.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  phase("statistics");
  if (log_on()) {
    std::string line = "[hfmm] plan " + std::to_string(n) + " points, " + std::to_string(nb) + " boxes:";
    char buf[64];
    for (auto& ph : phases) {
      std::snprintf(buf, sizeof(buf), " %s %.1f ms,", ph.first, 1e3 * ph.second);
      line += buf;
    }
    std::fprintf(stderr, "%s total %.1f ms\n", line.c_str(), 1e3 * inf.plan_seconds);
  }
  *out = pl;
  return HFMM_OK;
}

}  // extern "C"

namespace {

// u_sorted = A q_sorted for the plan's point order (complex-linear).
// Records an event on the stream at each stage boundary while profiling is on.
struct Marker {
  std::vector<hipEvent_t>* ev = nullptr;
  hipStream_t s = nullptr;
  void operator()() {
    if (!ev) return;
    hipEvent_t e;
    if (hipEventCreate(&e) == hipSuccess) {
      (void)hipEventRecord(e, s);
      ev->push_back(e);
    }
  }
};

// P2M (or L2P^T) over all leaves of levels >= 2, one launch (leaves are in
// level order, coarse first).
void launch_p2m_all(hfmm_plan_t pl, const TreeView& tv, hipStream_t s, const double2* qs, double2* alpha,
                    int conj_w, double2 pref) {
  const int b0 = pl->leaf_lev[std::min(2, pl->nlev)], b1 = pl->leaf_lev[pl->nlev];
  launch_p2m(s, tv, pl->leaves.p + b0, b1 - b0, pl->leaf_pmax, qs, alpha, conj_w, pref);
}

// L2P (or P2M^T) over all leaves, one launch: stores u, or adds atomically
// (accumulate = 2) while the near field adds into it.
void launch_l2p_all(hfmm_plan_t pl, const TreeView& tv, hipStream_t s, const double2* beta, double2* us, int conj_w,
                    double2 pref, int accumulate) {
  launch_l2p(s, tv, pl->leaves.p, pl->nleaves, pl->pt_box.p, pl->leaf_pmax, beta, us, conj_w, pref, accumulate);
}

// One level of child -> parent (up) or parent -> child (down) translations;
// in_sequence: nothing runs beside this launch (the split gather may be used).
void launch_level(hfmm_plan_t pl, const TreeView& tv, hipStream_t s, bool up, int l, bool m2m_tables,
                  const double2* src, double2* dst, int rev, bool in_sequence) {
  // the split form while the launch (one block per item and right-hand side)
  // still fits the GPU at once
  const bool split = up && in_sequence && pl->up_split_groups[l].count > 0 && tv.nrhs <= pl->up_split_groups[l].max_rhs;
  const hfmm_plan_s::Group& g = split ? pl->up_split_groups[l] : up ? pl->up_groups[l] : pl->down_groups[l];
  if (!g.count) return;
  const Toff4& q4 = m2m_tables ? pl->m2m_q4[l] : pl->l2l_q4[l];
  const TransItem* items = (up ? pl->up_items.p : pl->down_items.p) + g.first;
  const int64_t* soff = up ? pl->up_soff4.p : pl->cp_parent.p;
  const int64_t* doff = up ? pl->up_doff.p : pl->cp_child.p;
  // a child has one parent, and up items gather a parent's children: no two
  // pairs of a launch write the same box
  launch_trans(s, tv, items, g.count, g.Ps, g.Pd, soff, doff, nullptr, q4, pl->tdata.p, src, dst, nullptr, 0, rev,
               up ? (split ? 2 : 1) : 0, g.ntw);
}

// All M2L items (forward: source -> target; transpose: target -> source) into
// the per-pair contribution rows, then the per-box reduction into dst.
void launch_m2l_all(hfmm_plan_t pl, const TreeView& tv, hipStream_t s, const double2* src, double2* dst, double* contrib,
                    int rev) {
  const int64_t* soff = rev ? pl->m2l_toff.p : pl->m2l_soff.p;
  const int64_t* doff = rev ? pl->m2l_soff.p : pl->m2l_toff.p;
  for (const auto& g : pl->m2l_groups)
    launch_trans(s, tv, pl->m2l_items.p + g.first, g.count, g.Ps, g.Pd, soff, doff,
                 rev ? pl->m2l_pcoffT.p : pl->m2l_pcoff.p, Toff4{}, pl->tdata.p, src, nullptr, contrib,
                 pl->cstride, rev, 0, g.ntw);
  launch_reduce_contrib(s, tv, pl->red_boxes.p, pl->nred_boxes, rev ? pl->redT_ptr.p : pl->red_ptr.p,
                        rev ? pl->redT_beg.p : pl->red_beg.p, contrib, pl->cstride, dst);
}

// The direct parts (free-space pairs and near-interface pairs) add into us
// atomically.
void launch_near(hfmm_plan_t pl, const TreeView& tv, hipStream_t s, const double2* qs, double2* us, Marker* mark) {
  launch_p2p(s, tv, pl->p2p_items.p, pl->p2p_cls_ptr, pl->p2p_ptr.p, pl->p2p_rng.p, pl->p2p_sym.p, qs, us,
             pl->precision == HFMM_FP32);
  if (mark) (*mark)();
  launch_iface(s, tv, pl->ifl.data(), (int)pl->ifl.size(), tv.nrhs, qs, us, 1, tv.n, 1);
  launch_iface_table(s, tv, pl->ift.data(), (int)pl->ift.size(), tv.nrhs, qs, us, 1, tv.n, 1);
  if (mark) (*mark)();
}

// Fork: us is cleared and the near field starts on the plan's side stream
// while the far-field chain runs on s; every writer of us then adds
// atomically. join() makes s wait for the side stream. The fork comes first,
// before P2M: P2M's one-wave blocks fit beside the near field's four-wave
// blocks, which measured faster than P2M alone followed by the fork.
hipError_t fork_near(hfmm_plan_t pl, const TreeView& tv, hipStream_t s, const double2* qs, double2* us) {
  launch_fill_zero(s, us, (int64_t)tv.nrhs * pl->n);
  hipError_t e = hipEventRecord(pl->ev_fork, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(pl->side, pl->ev_fork, 0);
  if (e != hipSuccess) return e;
  launch_near(pl, tv, pl->side, qs, us, nullptr);
  return hipEventRecord(pl->ev_join, pl->side);
}
hipError_t join_near(hfmm_plan_t pl, hipStream_t s) { return hipStreamWaitEvent(s, pl->ev_join, 0); }

// Whether s is being captured into a graph (or its state is unknown). A
// capture keeps every stage on s: the fork onto the side stream is not used
// there (a batch capture, which already forks per plan, crashed in the
// runtime with it).
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone;
}

// With stage timing on (mark.ev set) the stages run one after another on s.
hipError_t forward_pipeline(hfmm_plan_t pl, int nrhs, hipStream_t s, const Workspace& w, Marker& mark) {
  const double2* qs = w.qs;
  double2* us = w.us;
  TreeView tv = pl->view(nrhs);
  const bool overlap = mark.ev == nullptr && !capturing(s);
  if (overlap) {
    const hipError_t e = fork_near(pl, tv, s, qs, us);
    if (e != hipSuccess) return e;
  }
  // P2M stores the leaves' multipoles, M2M each parent's (every box of levels
  // >= 2 is one or the other)
  launch_p2m_all(pl, tv, s, qs, w.alpha, 0, cmk(1.0, 0.0));
  mark();
  for (int l = pl->nlev - 2; l >= pl->top; --l)
    launch_level(pl, tv, s, true, l, true, w.alpha, w.alpha, 0, !overlap);
  mark();
  launch_m2l_all(pl, tv, s, w.alpha, w.beta, w.contrib, 0);
  mark();
  for (int l = pl->top; l + 1 < pl->nlev; ++l)
    launch_level(pl, tv, s, false, l, false, w.beta, w.beta, 0, !overlap);
  mark();
  launch_l2p_all(pl, tv, s, w.beta, us, 0, cmk(0.0, 0.25), overlap ? 2 : 0);
  mark();
  if (overlap) return join_near(pl, s);
  launch_near(pl, tv, s, qs, us, &mark);
  return hipSuccess;
}

// w_sorted = A^T v_sorted through the transposes of the stages, in reverse order.
hipError_t transpose_pipeline(hfmm_plan_t pl, int nrhs, hipStream_t s, const double2* vs, double2* ws) {
  TreeView tv = pl->view(nrhs);
  // the direct parts are symmetric: the same near field, beside the far field
  // (in sequence under stage timing or graph capture)
  const bool overlap = !pl->prof_on && !capturing(s);
  // L2P^T: beta'_p = (i/4) sum_i v_i J_p e^{i p theta_i} at the leaves, then
  // the parents' sums (stored, as in the forward pass)
  if (overlap) {
    const hipError_t e = fork_near(pl, tv, s, vs, ws);
    if (e != hipSuccess) return e;
  }
  launch_p2m_all(pl, tv, s, vs, pl->beta.p, 1, cmk(0.0, 0.25));
  // L2L^T, finest parents first: beta'(parent) = sum over its children of T^T beta'(child)
  for (int l = pl->nlev - 2; l >= pl->top; --l)
    launch_level(pl, tv, s, true, l, false, pl->beta.p, pl->beta.p, 1, !overlap);
  // M2L^T, reduced by source box
  launch_m2l_all(pl, tv, s, pl->beta.p, pl->alpha.p, pl->contrib.p, 1);
  // M2M^T, coarse to fine: alpha'(child) += T^T alpha'(parent)
  for (int l = pl->top; l + 1 < pl->nlev; ++l)
    launch_level(pl, tv, s, false, l, true, pl->alpha.p, pl->alpha.p, 1, !overlap);
  // P2M^T: w_j = sum_p alpha'_p J_p e^{-i p theta_j}
  launch_l2p_all(pl, tv, s, pl->alpha.p, ws, 1, cmk(1.0, 0.0), overlap ? 2 : 0);
  if (overlap) return join_near(pl, s);
  launch_near(pl, tv, s, vs, ws, nullptr);
  return hipSuccess;
}

// u = A q in passes of `chunk` right-hand sides through the workspace w
// (profile: stage events, for single-pass applies).
hfmm_status_t apply_passes(hfmm_plan_t pl, const double* q, double* u, int nrhs, int chunk, hipStream_t s,
                           const Workspace& w, bool profile) {
  Marker mark;
  mark.s = s;
  if (profile && chunk >= nrhs) {
    pl->prof_pending.emplace_back();
    mark.ev = &pl->prof_pending.back();
  }
  for (int r0 = 0; r0 < nrhs; r0 += chunk) {
    const int nc = std::min(chunk, nrhs - r0);
    const double2* qc = (const double2*)q + (int64_t)r0 * pl->n;
    double2* uc = (double2*)u + (int64_t)r0 * pl->n;
    mark();
    launch_gather(s, pl->n, nc, pl->perm.p, qc, w.qs, 0);
    mark();
    HIP_TRY(forward_pipeline(pl, nc, s, w, mark));
    launch_scatter(s, pl->n, nc, pl->perm.p, w.us, uc, 0, pl->self_g.p, w.qs);
    mark();
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(pl->ev_done, s));
  return HFMM_OK;
}

}  // namespace

// u = A q through the blocked pipeline: passes of Rp right-hand sides, every
// array blocked by right-hand side, the stages in sequence on s; with conj,
// u = conj(A conj(q)) = A^H q (A is symmetric: reciprocity of the layered
// Green's function, Section 2). No stage adds atomically: every output
// element is summed in a fixed order.
hfmm_status_t blocked_passes(hfmm_plan_t pl, const double* q, double* u, int nrhs, hipStream_t s, int conj) {
  const int Rp = blk_pass_width(pl, nrhs);
  hfmm_status_t st = ensure_blk_workspace(pl, Rp, s);
  if (st != HFMM_OK) return st;
  const TreeView tv = pl->view(Rp);
  const int lb2 = pl->leaf_lev[std::min(2, pl->nlev)], nl2 = pl->nleaves - lb2;
  const int64_t n = pl->n;
  auto tg = [&](const hfmm_plan_s::TgGroup& g, int prec, int ntm, const double2* src, const void* src_lo,
                double2* dst, int add) {
    launch_tgemm(s, prec, ntm, Rp, pl->tg_items.p + g.first, g.count, g.buf, pl->tg_pairs.p, pl->tdata.p,
                 pl->olo.p, src, src_lo, pl->blk_scale.p, kScaleStride, dst, add);
  };
  for (int r0 = 0; r0 < nrhs; r0 += Rp) {
    const int nc = std::min(Rp, nrhs - r0);
    const double2* qc = (const double2*)q + (int64_t)r0 * n;
    double2* uc = (double2*)u + (int64_t)r0 * n;
    launch_gather_blk(s, pl->n, nc, Rp, pl->perm.p, qc, pl->qb.p, conj);
    if (pl->blk_prec_p2p == BLK_F32) launch_to_f32(s, n * Rp, pl->qb.p, pl->qlo.p);
    launch_fill_zero(s, pl->ub.p, n * Rp);
    for (int l = 2; l < pl->nlev; ++l) {
      const int l0 = pl->leaf_lev[l], l1 = pl->leaf_lev[l + 1];
      launch_p2m_blk2(s, tv, Rp, pl->leaves.p + l0, l1 - l0, pl->P[l], pl->vmat_off.p + (l0 - lb2), pl->vmat.p,
                      pl->qb.p, pl->ab.p);
    }
    for (int l = pl->nlev - 2; l >= pl->top; --l) tg(pl->m2m_tg[l], BLK_F64, kUpDownNt, pl->ab.p, nullptr, pl->ab.p, 0);
    if (pl->blk_prec_m2l != BLK_F64)
      launch_scale_blk(s, pl->blk_prec_m2l, tv, Rp, pl->lev_begin[pl->top], (int)pl->boxes.size(), pl->blk_scale.p,
                       kScaleStride, pl->coff16.p, pl->ab.p, pl->alo.p);
    for (int l = pl->top; l < pl->nlev; ++l) {
      const int c = pl->m2l_pick[l];
      tg(pl->m2l_tgl[c][l], pl->blk_prec_m2l, hfmm_plan_s::kTileNt[c], pl->ab.p, pl->alo.p, pl->bb.p, 0);
    }
    for (int l = pl->top; l + 1 < pl->nlev; ++l) tg(pl->l2l_tg[l], BLK_F64, kUpDownNt, pl->bb.p, nullptr, pl->bb.p, 1);
    launch_l2p_blk2(s, tv, Rp, pl->leaves.p + lb2, nl2, pl->vmat_off.p, pl->vmat.p, pl->bb.p, pl->ub.p);
    launch_p2p_blk(s, tv, pl->blk_prec_p2p, Rp, pl->bp_items.p, pl->bp_cls_ptr, pl->bp_rng.p, pl->qb.p, pl->qlo.p,
                   pl->ub.p);
    launch_iface(s, tv, pl->ifl.data(), (int)pl->ifl.size(), nc, pl->qb.p, pl->ub.p, Rp, 1, 0);
    launch_iface_table(s, tv, pl->ift.data(), (int)pl->ift.size(), nc, pl->qb.p, pl->ub.p, Rp, 1, 0);
    launch_scatter_blk(s, pl->n, nc, Rp, pl->perm.p, pl->ub.p, uc, pl->self_g.p, pl->qb.p, conj);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(pl->ev_done, s));
  return HFMM_OK;
}

namespace hfmm {
hfmm_status_t apply_in_buffer(hfmm_plan_t pl, const double* q, double* u, int nrhs, hipStream_t s, void* base,
                              size_t bytes) {
  if (!pl || !q || !u) return fail(HFMM_ERR_INVALID_ARG, "NULL plan, q or u");
  if (nrhs < 1) return fail(HFMM_ERR_INVALID_ARG, "nrhs must be >= 1");
  if (!base) return fail(HFMM_ERR_INVALID_ARG, "NULL workspace");
  if (pl->opt.deterministic)
    return fail(HFMM_ERR_UNSUPPORTED, "deterministic plans run the blocked pipeline, whose workspace the plan owns");
  if (workspace_bytes(pl, 1) > bytes)
    return fail(HFMM_ERR_NO_MEMORY, "the plan needs " + std::to_string(workspace_bytes(pl, 1)) +
                                        " bytes of workspace per right-hand side; " + std::to_string(bytes) +
                                        " are available");
  // as many right-hand sides per pass as the buffer holds (the parts grow
  // linearly with the count, up to their 256-byte alignment)
  int chunk = (int)std::min<size_t>((size_t)std::min(nrhs, rhs_chunk(pl, nrhs)), bytes / workspace_bytes(pl, 1));
  chunk = std::max(chunk, 1);
  while (chunk > 1 && workspace_bytes(pl, chunk) > bytes) --chunk;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t r = (size_t)chunk;
  char* p = (char*)base;
  Workspace w{};
  w.qs = (double2*)p; p += al(sizeof(double2) * (size_t)pl->n * r);
  w.us = (double2*)p; p += al(sizeof(double2) * (size_t)pl->n * r);
  w.alpha = (double2*)p; p += al(sizeof(double2) * (size_t)std::max<int64_t>(pl->ctot, 1) * r);
  w.beta = (double2*)p; p += al(sizeof(double2) * (size_t)std::max<int64_t>(pl->ctot, 1) * r);
  w.contrib = (double*)p;
  return apply_passes(pl, q, u, nrhs, chunk, s, w, false);
}
}  // namespace hfmm

extern "C" {

hfmm_status_t hfmm_apply(hfmm_plan_t pl, const double* q, double* u, int32_t nrhs, hfmm_stream_t stream_) {
  if (!pl || !q || !u) return fail(HFMM_ERR_INVALID_ARG, "NULL plan, q or u");
  if (nrhs < 1) return fail(HFMM_ERR_INVALID_ARG, "nrhs must be >= 1");
  hipStream_t s = (hipStream_t)stream_;
  AllocScope alloc_scope(&pl->al);
  if (use_blocked(pl, nrhs)) return blocked_passes(pl, q, u, nrhs, s, 0);
  const int chunk = rhs_chunk(pl, nrhs);
  hfmm_status_t st = ensure_workspace(pl, chunk);
  if (st != HFMM_OK) return st;
  const Workspace w{pl->qs.p, pl->us.p, pl->alpha.p, pl->beta.p, pl->contrib.p};
  return apply_passes(pl, q, u, nrhs, chunk, s, w, pl->prof_on);
}

hfmm_status_t hfmm_profile_enable(hfmm_plan_t pl, int32_t enable) {
  if (!pl) return fail(HFMM_ERR_INVALID_ARG, "NULL plan");
  pl->prof_on = enable != 0;
  return HFMM_OK;
}

hfmm_status_t hfmm_profile_read(hfmm_plan_t pl, double* stage_ms, int32_t* napplies) {
  if (!pl || !stage_ms || !napplies) return fail(HFMM_ERR_INVALID_ARG, "NULL argument");
  HIP_TRY(hipDeviceSynchronize());
  for (auto& ev : pl->prof_pending) {
    if (ev.size() == HFMM_NSTAGES + 1) {
      for (int i = 0; i < HFMM_NSTAGES; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) pl->prof_ms[i] += ms;
      }
      ++pl->prof_n;
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  pl->prof_pending.clear();
  for (int i = 0; i < HFMM_NSTAGES; ++i) {
    stage_ms[i] = pl->prof_ms[i];
    pl->prof_ms[i] = 0.0;
  }
  *napplies = pl->prof_n;
  pl->prof_n = 0;
  return HFMM_OK;
}

const char* hfmm_stage_name(int32_t stage) {
  static const char* names[HFMM_NSTAGES] = {"gather", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p", "interface", "scatter"};
  return (stage >= 0 && stage < HFMM_NSTAGES) ? names[stage] : "unknown";
}

hfmm_status_t hfmm_apply_adjoint(hfmm_plan_t pl, const double* v, double* w, int32_t nrhs, const double* q,
                                 double* grad_xy, hfmm_stream_t stream_) {
  if (!pl || !v || !w) return fail(HFMM_ERR_INVALID_ARG, "NULL plan, v or w");
  if (nrhs < 1) return fail(HFMM_ERR_INVALID_ARG, "nrhs must be >= 1");
  if (grad_xy && !q) return fail(HFMM_ERR_INVALID_ARG, "grad_xy requested without q");
  hipStream_t s = (hipStream_t)stream_;
  AllocScope alloc_scope(&pl->al);
  if (pl->opt.deterministic) {
    if (grad_xy) return fail(HFMM_ERR_UNSUPPORTED, "deterministic mode has no coordinate gradients");
    return blocked_passes(pl, v, w, nrhs, s, 1);
  }
  const int chunk = rhs_chunk(pl, nrhs);
  hfmm_status_t st = ensure_workspace(pl, chunk);
  if (st != HFMM_OK) return st;
  if (grad_xy) {
    if ((pl->gq.p && pl->gq.n < (size_t)pl->n * chunk) || (pl->gs.p && pl->gs.n < (size_t)pl->n)) {
      HIP_TRY(hipEventSynchronize(pl->ev_done));  // earlier calls may still read them
      HIP_TRY(hipStreamSynchronize(pl->side));
    }
    HIP_TRY(pl->gq.ensure((size_t)pl->n * chunk));
    HIP_TRY(pl->gs.ensure((size_t)pl->n));
  }
  for (int r0 = 0; r0 < nrhs; r0 += chunk) {
    const int nc = std::min(chunk, nrhs - r0);
    const int64_t off = (int64_t)r0 * pl->n;
    // A^H v = conj(A^T conj(v))
    launch_gather(s, pl->n, nc, pl->perm.p, (const double2*)v + off, pl->qs.p, 1);
    HIP_TRY(transpose_pipeline(pl, nc, s, pl->qs.p, pl->us.p));
    launch_scatter(s, pl->n, nc, pl->perm.p, pl->us.p, (double2*)w + off, 1, pl->self_g.p, pl->qs.p);
    if (grad_xy) {
      // g_j = Re(q_j sum_i conj(v_i) dA_ij/dx_j): the transposed pipeline has
      // left the adjoint multipole coefficients in alpha and conj(v) in qs;
      // later chunks add to the first one's sums
      TreeView tv = pl->view(nc);
      launch_gather(s, pl->n, nc, pl->perm.p, (const double2*)q + off, pl->gq.p, 0);
      launch_l2p_grad(s, tv, pl->leaves.p, pl->nleaves, pl->leaf_pmax, pl->alpha.p, pl->gq.p, pl->gs.p, r0 > 0);
      launch_p2p_grad(s, tv, pl->p2p_items.p, pl->p2p_cls_ptr, pl->p2p_ptr.p, pl->p2p_rng.p, pl->p2p_sym.p, pl->qs.p,
                      pl->gq.p, pl->gs.p);
      launch_iface_grad(s, tv, pl->ifl.data(), (int)pl->ifl.size(), nc, pl->qs.p, pl->gq.p, pl->gs.p);
      launch_iface_table_grad(s, tv, pl->ift.data(), (int)pl->ift.size(), nc, pl->qs.p, pl->gq.p, pl->gs.p);
      // HFMM_SELF_NONE: the pair (j, j) of the scattered part is not in A
      if (pl->self_dy.p) launch_self_grad(s, pl->n, nc, pl->self_dy.p, pl->qs.p, pl->gq.p, pl->gs.p);
    }
  }
  if (grad_xy) launch_scatter_grad(s, pl->n, pl->perm.p, pl->gs.p, (double2*)grad_xy);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(pl->ev_done, s));
  return HFMM_OK;
}

}  // extern "C"
