// Launchers of the HIP kernels (definitions in kernels.hip).
#pragma once

#include "common.hpp"

namespace hfmm {

void launch_gather(hipStream_t s, int n, int nrhs, const int* perm, const double2* src, double2* dst, int conj_in);
void launch_scatter(hipStream_t s, int n, int nrhs, const int* perm, const double2* src, double2* dst, int conj_out);
void launch_p2m(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const double2* qs, double2* alpha,
                int conj_w, double2 pref);
void launch_l2p(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const double2* beta, double2* us,
                int conj_w, double2 pref, int accumulate);
void launch_m2l(hipStream_t s, const TreeView& tv, const int* targets, int nt, const int* ptr, const M2LEntry* ent,
                const TableRef* tabs, const double2* tdata, const double2* src, double2* dst, int rev);
void launch_m2l_mfma(hipStream_t s, const TreeView& tv, const M2LItem* items, const int* item_level_first,
                     int nlev, const int* psrc, const int* pdst, const TableRef* tabs, const double2* tdata,
                     const double2* src, double2* dst, int rev);
void launch_fill_zero(hipStream_t s, double2* p, int64_t n);
void launch_m2m(hipStream_t s, const TreeView& tv, const int* boxes, int nb, const TableRef* tabs4,
                const double2* tdata, const double2* src, double2* dst, int rev);
void launch_l2l(hipStream_t s, const TreeView& tv, const int* boxes, int nb, const TableRef* tabs4,
                const double2* tdata, const double2* src, double2* dst, int rev, int accumulate);
void launch_p2p(hipStream_t s, const TreeView& tv, const int* items, int nitems, const int* ptr, const int2* rng,
                const int* atomic, const double2* qs, double2* us);
void launch_iface(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const int* ptr, const int2* rng,
                  int nq, const double2* qc, const double2* qky, const double2* qkx, const double2* qs, double2* us);
void launch_table_hankel(hipStream_t s, int ntab, const double* dx, const double* dy, const TableRef* refs, double k,
                         double2* tdata);
void launch_table_bessel(hipStream_t s, int ntab, const double* dx, const double* dy, const int* sgn,
                         const TableRef* refs, double k, double2* tdata);
void launch_table_image(hipStream_t s, const Medium& med, int ncombo, const double* X, const double* Y,
                        const double* dip, const double* send, const int* pbeg, const Panel* panels,
                        const TableRef* refs, const double* glx, const double* glw, double2* tdata);

}  // namespace hfmm
