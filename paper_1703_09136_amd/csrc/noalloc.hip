// hfmm_apply_noalloc: u = A q with the apply's workspace in a fixed device
// array of the library instead of memory allocated on demand, for callers
// that cannot allocate (code under HIP graph capture, serving loops, hosts
// that forbid allocation during a call).
//
// The workspace (strengths and results in point order, multipole and local
// coefficients, multipole-to-local contribution rows) lives in `scratch`, a
// file-scope device array of kScratchBytes that every GPU the library runs on
// holds until the process ends. Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, looked up once per device with that
// device current, and only that address is used.
//
// Every call on one GPU shares that GPU's array: calls that overlap on one
// GPU (from several host threads, or on streams that are not ordered with
// each other) race on it. Nothing in it has to start at zero: every stage
// stores its buffer before it is read (the results are cleared by a fill
// kernel of the apply itself).
#include "plan_internal.hpp"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

namespace {

constexpr size_t kScratchBytes = HFMM_NOALLOC_BYTES;  // per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// The device address of this device's scratch array (looked up once).
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

hfmm_status_t hfmm_apply_noalloc(hfmm_plan_t plan, const double* q, double* u, int32_t nrhs,
                                 hfmm_stream_t stream) {
  if (!plan || !q || !u) return hfmm::report(HFMM_ERR_INVALID_ARG, "NULL plan, q or u");
  if (nrhs < 1) return hfmm::report(HFMM_ERR_INVALID_ARG, "nrhs must be >= 1");
  const size_t need = hfmm::workspace_bytes(plan, 1);
  if (need > kScratchBytes)
    return hfmm::report(HFMM_ERR_NO_MEMORY, "hfmm_apply_noalloc: the plan needs " + std::to_string(need) +
                                                " bytes of workspace for one right-hand side; the fixed workspace "
                                                "holds " + std::to_string(kScratchBytes) + " (use hfmm_apply)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return hfmm::report(HFMM_ERR_DEVICE, std::string("hfmm_apply_noalloc: current device: ") + hipGetErrorString(e));
  void* base = nullptr;
  e = scratch_address(dev, &base);
  if (e != hipSuccess)
    return hfmm::report(HFMM_ERR_DEVICE, std::string("hfmm_apply_noalloc: scratch address: ") + hipGetErrorString(e));
  return hfmm::apply_in_buffer(plan, q, u, nrhs, (hipStream_t)stream, base, kScratchBytes);
}

}  // extern "C"
