// Launchers of the HIP kernels (definitions in kernels.hip).
#pragma once

#include "common.hpp"

namespace hfmm {

void launch_gather(hipStream_t s, int n, int nrhs, const int* perm, const double2* src, double2* dst, int conj_in);
// scatter to user order; with diag, dst = src - diag * qsrc (sorted order)
void launch_scatter(hipStream_t s, int n, int nrhs, const int* perm, const double2* src, double2* dst, int conj_out,
                    const double2* diag = nullptr, const double2* qsrc = nullptr);
// the scattered self term and its source-height derivative per sorted point
// from a rule for X = 0 (nodes c_q, ky_q)
void launch_self_term(hipStream_t s, int n, const double2* pts, int nq, const double2* qc, const double2* qky,
                      double2* g, double2* dy);
// gs[j].y -= sum_r Re(q_rj vs_rj dy_j)
void launch_self_grad(hipStream_t s, int n, int nrhs, const double2* dy, const double2* vs, const double2* qs,
                      double2* gs);
// Kernel attributes that must be set before launches (and before any graph
// capture): the dynamic LDS limit of the translation kernels.
hipError_t init_kernel_attributes();

// P2M and L2P over a list of leaves; each block reads its leaf's order, Pmax
// bounds the orders of the list (sizes the LDS). L2P stores into us
// (accumulate = 0), adds with a read-modify-write (1) or adds atomically (2).
// With pt_box (the leaf box of every sorted point, all points in leaves) and
// one right-hand side, L2P runs a lane per point over the sorted order.
void launch_p2m(hipStream_t s, const TreeView& tv, const int* leaves, int nl, int Pmax, const double2* qs,
                double2* alpha, int conj_w, double2 pref);
void launch_l2p(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const int* pt_box, int Pmax,
                const double2* beta, double2* us, int conj_w, double2 pref, int accumulate);
// Batched translation contraction (M2L, M2M, L2L and transposes) for items
// sharing (Ps, Pd). With contrib != NULL each pair writes its own contribution
// row at pcoff[pair] (plane stride cstride per right-hand side); otherwise the
// result is added into dst of the pair's target box, which no other pair of
// the launch targets. Without gather4 a pair is (source, target): soff / doff
// hold the coefficient offsets of its boxes, and the table of an item is at
// item.toff in tdata or (toff < 0) at q4.v[item.table]. With gather4 (child
// to parent) a "pair" is a parent: doff its offset, soff[4 pair + q] that of
// its child in quadrant q (-1: none), translated with the table at q4.v[q].
// gather4 = 1: the quadrants in turn, items of up to 4 ntw row tiles;
// gather4 = 2: the split form, items of one row tile each, a quadrant per
// wave (LDS: trans_lds_bytes_split).
// ntw: the row tiles per wave of the items (their largest value).
void launch_trans(hipStream_t s, const TreeView& tv, const TransItem* items, int nitems, int Ps, int Pd,
                  const int64_t* soff, const int64_t* doff, const int64_t* pcoff, const Toff4& q4,
                  const double2* tdata, const double2* src, double2* dst, double* contrib, int64_t cstride, int rev,
                  int gather4, int ntw);
// dst(box) = sum of its contribution rows: ptr[w + 1] - ptr[w] rows from
// row offset beg[w] for boxes[w].
void launch_reduce_contrib(hipStream_t s, const TreeView& tv, const int* boxes, int nb, const int* ptr,
                           const int64_t* beg, const double* contrib, int64_t cstride, double2* dst);
size_t trans_lds_bytes(int Ps, int Pd);
size_t trans_lds_bytes_split(int Ps, int Pd);
void launch_fill_zero(hipStream_t s, double2* p, int64_t n);
// Free-space direct pairs. Items are sorted by H0 series class: items
// [cls_ptr[c], cls_ptr[c + 1]) use kH0ClassTerms[c] terms, class kH0Classes
// the longest series with the large-argument form for x > 6. cls_ptr is a
// host array of kH0Classes + 2 entries. sym[i] marks a cross item whose pairs
// are evaluated once and added to both points; the output is accumulated
// atomically. fp32: pair arithmetic and per-item sums in single precision.
void launch_p2p(hipStream_t s, const TreeView& tv, const int* items, const int* cls_ptr, const int* ptr,
                const int2* rng, const int* sym, const double2* qs, double2* us, int fp32);
// Near-interface pairs (Section 5: direct quadrature of the Sommerfeld
// integral for image pairs that are not admissible) in three stages, see
// kernels.hip. The device lists of a plan and its node-sum buffers:
constexpr int kIfRhs = 8;  // right-hand sides per group, at most
struct IfaceLists {
  int nsb = 0;        // source boxes (any level)
  int ntl = 0;        // target leaves
  int nq = 0;         // rule nodes
  int nqp = 0;        // nq rounded up to a multiple of 64
  int rif = 1;        // right-hand sides per group (<= kIfRhs): the buffers' width
  const int* sbox = nullptr;   // [nsb] box ids
  const int* tleaf = nullptr;  // [ntl] leaf box ids, distinct
  const int* tptr = nullptr;   // [ntl + 1] CSR into tsrc
  const int* tsrc = nullptr;   // source slots (indices into sbox), point ranges disjoint per leaf
  const double2* qc = nullptr;
  const double2* qky = nullptr;
  const double2* qkx = nullptr;
  double2* S = nullptr;        // [nsb][rif][nqp] source sums
  double2* T = nullptr;        // [ntl][rif][nqp] translated sums
  // one class of pairs: its own rule (qc, qky, qkx: nq nodes) and lists
};
// us += (near-interface part of A) qs for nrhs right-hand sides, element r of
// point j at j * ps + r * rs for both; atomic: add atomically (other writers
// of us run at the same time), else read-add-write (one writer per point).
// The classes L[0..ncls) run in sequence (they share the node-sum buffers).
void launch_iface(hipStream_t s, const TreeView& tv, const IfaceLists* L, int ncls, int nrhs, const double2* qs,
                  double2* us, int64_t ps, int64_t rs, int atomic);
// Horizontally separated near-interface pairs by tables of G^s(|X|, Y) (see
// kernels.hip): per class a Chebyshev series (the terms T_a T_b with a + b <
// kIfTP) on each panel: panels of |X| from x0 on, each split in Y over the
// class's range from ylo. The panels of |X| (xpan) are geometric (ratio 2^{1 /
// inv_lg2}) from x0 for p < p1, then wmax wide from a1.
constexpr int kIfTP = 12;
constexpr int kIfTri = kIfTP * (kIfTP + 1) / 2;  // coefficients with a + b < kIfTP
struct IfTable {
  int ntl = 0;                 // target leaves
  const int* tleaf = nullptr;  // [ntl] leaf box ids
  const int* tptr = nullptr;   // [ntl + 1] CSR into tsrc
  const int* tsrc = nullptr;   // source box ids
  // work items for launches with atomic additions: leaf index (into tleaf)
  // and a range of its entries in tsrc
  int nitem = 0;
  const int* item_t = nullptr;
  const int2* item_e = nullptr;
  double x0 = 0.0, a1 = 0.0, wmax = 1.0, ylo = 0.0;
  double inv_x0 = 0.0, inv_wmax = 1.0;
  float inv_lg2 = 0.0f;  // 1 / log2 of the geometric ratio
  int p1 = 0, npx = 0;
  // per panel of |X|: left edge, 1 / width, and the width and its inverse of
  // its Y panels; their count and the first one's index
  const double4* xpan = nullptr;
  const int2* ypan = nullptr;
  const double2* coef = nullptr;  // [panel][3][kIfTri]: G, dG/d|X|, dG/dY, rows a = 0.. packed
};
// G, dG/d|X|, dG/dY of the rule (nq nodes) at npts points (|X|, Y): out holds
// three planes of npts values (plan time)
void launch_if_grid(hipStream_t s, int npts, const double2* xy, int nq, const double2* qc, const double2* qky,
                    const double2* qkx, double2* out);
// us += table pairs of every class; layout and atomic as launch_iface
void launch_iface_table(hipStream_t s, const TreeView& tv, const IfTable* tabs, int ntab, int nrhs, const double2* qs,
                        double2* us, int64_t ps, int64_t rs, int atomic);
void launch_table_hankel(hipStream_t s, int ntab, const double* dx, const double* dy, const TableRef* refs, double k,
                         double2* tdata);
void launch_table_bessel(hipStream_t s, int ntab, const double* dx, const double* dy, const int* sgn,
                         const TableRef* refs, double k, double2* tdata);
// nsplit blocks per table, each over its share of the rule's panels; with
// nsplit > 1 they store nsplit partial tables (table c at soff[c] in each, plen
// entries per partial table) that a second launch adds in order into tdata.
void launch_table_image(hipStream_t s, const Medium& med, int ncombo, const double* X, const double* Y,
                        const double* dip, const double* send, const int* pbeg, const Panel* panels,
                        const TableRef* refs, const double* glx, const double* glw, double2* tdata, int nsplit,
                        const int64_t* soff, double2* part, int64_t plen);

// Source-coordinate gradient (see kernels.hip): far field from the adjoint
// multipole coefficients (stores gs), then the direct and near-interface
// parts (add into gs), then gs to the caller's order as [n][2] doubles.
void launch_l2p_grad(hipStream_t s, const TreeView& tv, const int* leaves, int nl, int Pmax, const double2* alpha,
                     const double2* qs, double2* gs, int add);
// Near-field gradient over the direct items, one launch per series class
// (cls_ptr: host array of kH0Classes + 2 entries, as for launch_p2p).
void launch_p2p_grad(hipStream_t s, const TreeView& tv, const int* items, const int* cls_ptr, const int* ptr,
                     const int2* rng, const int* sym, const double2* vs, const double2* qs, double2* gs);
// Near-interface part of the gradient: vs (adjoint, sources) and qs
// (strengths at the owning points) as [nrhs][n]; adds into gs.
void launch_iface_grad(hipStream_t s, const TreeView& tv, const IfaceLists* L, int ncls, int nrhs,
                       const double2* vs, const double2* qs, double2* gs);
void launch_iface_table_grad(hipStream_t s, const TreeView& tv, const IfTable* tabs, int ntab, int nrhs,
                             const double2* vs, const double2* qs, double2* gs);
void launch_scatter_grad(hipStream_t s, int n, const int* perm, const double2* gs, double2* grad);

}  // namespace hfmm
