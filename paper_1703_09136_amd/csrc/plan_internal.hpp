// Library-internal calls between the plan (hfmm.hip) and the other host
// sources (batches, the allocation-free apply).
#pragma once

#include "../../include/hfmm.h"
#include "common.hpp"

#include <string>

namespace hfmm {

// Device buffers of one pass of an apply: strengths and results in point
// order (nrhs planes of n), multipole and local coefficients (nrhs planes of
// ctot) and the multipole-to-local contribution rows (nrhs planes of
// cstride doubles).
struct Workspace {
  double2* qs;
  double2* us;
  double2* alpha;
  double2* beta;
  double* contrib;
};

// workspace for applies with nrhs right-hand sides on stream s, ahead of a
// graph capture (allocations, and the blocked pipeline's expansion matrices)
hfmm_status_t plan_reserve(hfmm_plan_t pl, int nrhs, hipStream_t s);
int64_t plan_points(hfmm_plan_t pl);
double plan_wavenumber(hfmm_plan_t pl);  // k1, the top layer's
int64_t plan_workspace_generation(hfmm_plan_t pl);
// sets hfmm_last_error_message and returns st
hfmm_status_t report(hfmm_status_t st, const std::string& msg);
// bytes of a Workspace for nrhs right-hand sides carved from one buffer
// (every part aligned to 256 bytes)
size_t workspace_bytes(hfmm_plan_t pl, int nrhs);
// u = A q with the workspace carved from the device buffer [base, base + bytes):
// as many right-hand sides per pass as fit; HFMM_ERR_NO_MEMORY if not even
// one does. Allocates nothing.
hfmm_status_t apply_in_buffer(hfmm_plan_t pl, const double* q, double* u, int nrhs, hipStream_t s, void* base,
                              size_t bytes);

}  // namespace hfmm
