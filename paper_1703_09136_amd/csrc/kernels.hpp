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
void launch_iface(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const int* ptr, const int2* rng,
                  int nq, const double2* qc, const double2* qky, const double2* qkx, const double2* qs, double2* us);
void launch_table_hankel(hipStream_t s, int ntab, const double* dx, const double* dy, const TableRef* refs, double k,
                         double2* tdata);
void launch_table_bessel(hipStream_t s, int ntab, const double* dx, const double* dy, const int* sgn,
                         const TableRef* refs, double k, double2* tdata);
void launch_table_image(hipStream_t s, const Medium& med, int ncombo, const double* X, const double* Y,
                        const double* dip, const double* send, const int* pbeg, const Panel* panels,
                        const TableRef* refs, const double* glx, const double* glw, double2* tdata);

// Source-coordinate gradient (see kernels.hip): far field from the adjoint
// multipole coefficients (stores gs), then the direct and near-interface
// parts (add into gs), then gs to the caller's order as [n][2] doubles.
void launch_l2p_grad(hipStream_t s, const TreeView& tv, const int* leaves, int nl, int Pmax, const double2* alpha,
                     const double2* qs, double2* gs, int add);
// Near-field gradient over the direct items, one launch per series class
// (cls_ptr: host array of kH0Classes + 2 entries, as for launch_p2p).
void launch_p2p_grad(hipStream_t s, const TreeView& tv, const int* items, const int* cls_ptr, const int* ptr,
                     const int2* rng, const int* sym, const double2* vs, const double2* qs, double2* gs);
void launch_iface_grad(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const int* ptr, const int2* rng,
                       int nq, const double2* qc, const double2* qky, const double2* qkx, const double2* vs,
                       const double2* qs, double2* gs);
void launch_scatter_grad(hipStream_t s, int n, const int* perm, const double2* gs, double2* grad);

}  // namespace hfmm
