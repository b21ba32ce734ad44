// Kernels of the right-hand-side-blocked pipeline (blocked.hip).
//
// With many right-hand sides an apply keeps every per-point and per-box
// array "blocked": row-major with the right-hand sides as the fastest index,
// X[row * Rp + r] (Rp = the pass width, a multiple of 64; columns past the
// pass's right-hand sides are zero). Each stage is then a dense contraction
// whose N dimension is the right-hand sides: the translation operators
// (M2M, M2L, L2L), the expansion matrices of P2M and L2P, and the direct
// H0 tiles of P2P are applied to 64 right-hand sides per block on the matrix
// cores, each operator entry evaluated or loaded once for all of them.
#pragma once

#include "common.hpp"

namespace hfmm {

// Arithmetic of the multipole-to-local contraction and the direct pairs.
enum BlkPrec { BLK_F64 = 0, BLK_F32 = 1, BLK_BF16 = 2 };

// A target of a translation pass: its coefficient offset ct (row of the
// blocked coefficient array), its pairs [pbeg, pend), the real row tiles
// [rt0, rt0 + nt) of the interleaved real embedding it covers (row 2p + 0/1
// holds the real / imaginary part of target order p), and the orders.
struct TgItem {
  int64_t ct;
  int32_t pbeg, pend;
  int32_t rt0, nt;
  int32_t Ps, Pd;
  int32_t lev;   // level of the sources (scale factors of the reduced-precision forms)
  int32_t pad;
};
// A source of a target: coefficient offset, offset of its Toeplitz table
// t[-(Ps + Pd)] in the table data, and whether it is an image pair (the
// operator then acts on the reflected coefficients (-1)^m alpha_{-m}).
struct TgPair {
  int64_t cs;
  int64_t toff;
  int64_t cs16;  // BF16 rows: the source's offset in the 16-aligned order count
  int64_t tlo;   // FP32 / BF16: offset of the table's scaled operator
  int32_t image;
  int32_t pad;
};

// Direct work item of the blocked near field: up to 16 consecutive target
// points [t0, t0 + nt) against source ranges [rbeg, rend) of the range array.
struct BpItem {
  int32_t t0, nt;
  int32_t rbeg, rend;
};

constexpr int kBlkCols = 64;  // right-hand sides per block (four 16-column tiles)
constexpr int kTgMaxNt = 8;   // row tiles per translation item
// most expansion order of a leaf for the blocked P2M stage (two planes of
// (2P + 1) x 34 doubles in LDS, all row tiles of a leaf in one wave)
constexpr int kBlkLeafPmax = 40;

// gather: qb[j * Rp + r] = q[(r0 + r) * n + perm[j]] (conj: conjugated) for r < nc, 0 past nc
void launch_gather_blk(hipStream_t s, int n, int nc, int Rp, const int* perm, const double2* q, double2* qb,
                       int conj);
// scatter: u[(r0 + r) * n + perm[j]] = ub[j * Rp + r] (- diag[j] qb[j * Rp + r]), conjugated with conj
void launch_scatter_blk(hipStream_t s, int n, int nc, int Rp, const int* perm, const double2* ub, double2* u,
                        const double2* diag, const double2* qb, int conj);
// The expansion matrices V[m][j] = J_m(k rho_j) e^{-i m theta_j} of the
// leaves (geometry only: computed once per plan), per leaf [2P + 1][npts] at
// voff[leaf]; P2M over leaves stores alpha rows = V q, L2P adds
// u rows += (i/4) conj(V)^T beta.
void launch_vmat(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const int64_t* voff, double2* V);
// P2M for leaves of one level (order P): leaves and voff point at that
// level's first leaf
void launch_p2m_blk2(hipStream_t s, const TreeView& tv, int Rp, const int* leaves, int nl, int P,
                     const int64_t* voff, const double2* V, const double2* qb, double2* ab);
void launch_l2p_blk2(hipStream_t s, const TreeView& tv, int Rp, const int* leaves, int nl, const int64_t* voff,
                     const double2* V, const double2* bb, double2* ub);
// translations: dst rows of every item = (add ? dst : 0) + sum over its pairs
// of the operator applied to the source rows. F64: Toeplitz tables from
// tdata. F32 / BF16: the pair's scaled operator a(|m|) a(|p|) T (from
// launch_lo_tables, at pair.tlo in olo) applied to the scaled source rows
// src_lo (launch_scale_blk), accumulated in FP32 per pair and in FP64 across
// pairs, and the rows divided by a(|p|) of the target level before they are
// stored or added in FP64. buf_elems: the largest operator buffer of an item
// of the launch (tgemm_buf_elems).
// ntm: the most row tiles of an item of the launch (2, 4 or 8: the register
// allocation of the kernel variant)
void launch_tgemm(hipStream_t s, int prec, int ntm, int Rp, const TgItem* items, int nitems, int buf_elems,
                  const TgPair* pairs, const double2* tdata, const void* olo, const double2* src, const void* src_lo,
                  const double* scale, int sstride, double2* dst, int add);
// operator buffer of an item with `rows` complex rows (bytes), and the LDS of
// a launch (two operator buffers and two source chunks)
int tgemm_buf_elems(int prec, int Ps, int Pd, int rows);
size_t tgemm_lds_bytes(int prec, int buf_bytes);
// most row tiles per item whose reduced-precision operator rows fit the
// staging registers and the LDS; whether a pair of orders can be staged at all
int tgemm_max_nt(int prec, int Ps);
bool tgemm_supported(int prec, int Ps, int Pd);
// The scaled operators of multipole-to-local tables for the reduced
// precisions (one block per table): table t at toff[t] in tdata (t[-2P]),
// order P_of[t], level lev_of[t], image flag img_of[t]; written at off[t] in
// out (FP32: rows [2P + 1][Ms8] float2; BF16: embedded rows [2(2P + 1)][2 Ms16]).
void launch_lo_tables(hipStream_t s, int prec, int ntab, const int64_t* toff, const int* P_of, const int* lev_of,
                      const int* img_of, const int64_t* off, const double* scale, int sstride, const double2* tdata,
                      void* out);
// src_lo rows = src rows / a_l(|m|) in FP32 (float2) or BF16, for the boxes
// [b0, b1) (level by box); bf16 rows are laid out per box as [Rp][Ms16]
// (orders fastest, 16-aligned, zero padded) at offset coff16[b] * Rp.
void launch_scale_blk(hipStream_t s, int prec, const TreeView& tv, int Rp, int b0, int b1, const double* scale,
                      int sstride, const int64_t* coff16, const double2* src, void* src_lo);
// direct pairs: ub rows += (i/4) sum_j H0(k |x_i - x_j|) qb rows (i != j),
// items of one series class per launch (host array cls_ptr, as launch_p2p)
void launch_p2p_blk(hipStream_t s, const TreeView& tv, int prec, int Rp, const BpItem* items, const int* cls_ptr,
                    const int2* rng, const double2* qb, const void* qb_lo, double2* ub);
// rows of qb in FP32 for the FP32 near field
void launch_to_f32(hipStream_t s, int64_t count, const double2* src, float2* dst);
hipError_t init_blocked_attributes();

}  // namespace hfmm
