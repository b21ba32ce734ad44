// Boundary integral equation solve around the matvec (Section 1: the dense
// Nystrom system whose matrix applications the H-FMM provides): restarted
// GMRES for
//
//   (A W + D) phi = f,   W = diag(w),  D = diag(d),
//   d_i = (i/4) w_i [1 + (2i/pi)(ln(k1 w_i / 4) + gamma_E - 1)],
//
// the trapezoidal Nystrom form of the single-layer equation S phi = f on
// closed curves in the top layer (nodes x_i equispaced in a periodic
// parameter, weights w_i = |x'(t_i)| dt): A holds the domain Green's function
// between distinct nodes and its smooth scattered self term (Section 2.4),
// and d_i adds the free part's logarithmic singularity integrated over the
// node's own panel of length w_i by the small-argument form of H0^(1)
// (H0(z) ~ 1 + (2i/pi)(ln(z/2) + gamma_E)). The matrix applications run
// through the plan; the vector work of GMRES (weights, diagonal, inner
// products, updates) runs in the kernels below, the small Hessenberg least-
// squares problem on the host.
#include "../../include/hfmm.h"
#include "common.hpp"
#include "devbuf.hpp"
#include "plan_internal.hpp"

#include <cmath>
#include <complex>
#include <string>
#include <vector>

namespace hfmm {
namespace {

constexpr int BT = 256;
constexpr int kDotBlocks = 512;

__global__ void k_bie_weight(int n, const double* __restrict__ w, const double2* __restrict__ x,
                             double2* __restrict__ q) {
  const int i = blockIdx.x * BT + threadIdx.x;
  if (i < n) q[i] = cscale(x[i], w[i]);
}

// y += d x with d_i from the weights and the plan's k1
__global__ void k_bie_diag(int n, double k1, const double* __restrict__ w, const double2* __restrict__ x,
                           double2* __restrict__ y) {
  const int i = blockIdx.x * BT + threadIdx.x;
  if (i >= n) return;
  const double euler = 0.57721566490153286061;
  const double l = log(k1 * w[i] / 4.0) + euler - 1.0;
  // (i/4) w (1 + (2i/pi) l) = (w/4) (-(2/pi) l + i)
  const double2 d = cmk(-0.25 * w[i] * (2.0 / M_PI) * l, 0.25 * w[i]);
  y[i] = cadd(y[i], cmul(d, x[i]));
}

// partial sums of sum_i conj(a_i) b_i, one per block
__global__ void k_bie_dot(int n, const double2* __restrict__ a, const double2* __restrict__ b,
                          double2* __restrict__ part) {
  __shared__ double2 s[BT];
  double2 acc = cmk(0.0, 0.0);
  for (int i = blockIdx.x * BT + threadIdx.x; i < n; i += gridDim.x * BT) acc = cadd(acc, cmul(cconj(a[i]), b[i]));
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int h = BT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] = cadd(s[threadIdx.x], s[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// y = a x + b y
__global__ void k_bie_axpby(int n, double2 a, const double2* __restrict__ x, double2 b, double2* __restrict__ y) {
  const int i = blockIdx.x * BT + threadIdx.x;
  if (i < n) y[i] = cadd(cmul(a, x[i]), cmul(b, y[i]));
}

inline int nb(int n) { return (n + BT - 1) / BT; }

}  // namespace
}  // namespace hfmm

extern "C" {

hfmm_status_t hfmm_bie_solve(hfmm_plan_t plan, const double* w, const double* f, double* phi, double tol,
                             int32_t restart, int32_t max_iter, int32_t* iterations, double* residual,
                             hfmm_stream_t stream) {
  using namespace hfmm;
  using cd = std::complex<double>;
  if (!plan || !w || !f || !phi) return report(HFMM_ERR_INVALID_ARG, "NULL plan, w, f or phi");
  if (!(tol > 0.0 && tol < 1.0)) return report(HFMM_ERR_INVALID_ARG, "tol must be in (0, 1)");
  if (restart < 1 || restart > 1000 || max_iter < 1) return report(HFMM_ERR_INVALID_ARG, "restart in [1, 1000], max_iter >= 1");
  hipStream_t s = (hipStream_t)stream;
  const int n = (int)plan_points(plan);
  const double k1 = plan_wavenumber(plan);
  const int m = restart;
  DevBuf<double2> V, z, q, part;
  hipError_t e = V.alloc((size_t)n * (m + 1));
  if (e == hipSuccess) e = z.alloc((size_t)n);
  if (e == hipSuccess) e = q.alloc((size_t)n);
  if (e == hipSuccess) e = part.alloc(kDotBlocks);
  if (e != hipSuccess) return report(e == hipErrorOutOfMemory ? HFMM_ERR_NO_MEMORY : HFMM_ERR_DEVICE, "bie workspace");
  std::vector<double2> hpart(kDotBlocks);
  auto dot = [&](const double2* a, const double2* b, cd& out) -> hipError_t {
    hipLaunchKernelGGL(k_bie_dot, dim3(kDotBlocks), dim3(BT), 0, s, n, a, b, part.p);
    hipError_t err = hipMemcpyAsync(hpart.data(), part.p, sizeof(double2) * kDotBlocks, hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    cd acc = 0.0;
    for (const double2& v : hpart) acc += cd(v.x, v.y);
    out = acc;
    return err;
  };
  // y = (A W + D) x
  auto op = [&](const double2* x, double2* y) -> hfmm_status_t {
    hipLaunchKernelGGL(k_bie_weight, dim3(nb(n)), dim3(BT), 0, s, n, w, x, q.p);
    const hfmm_status_t st = hfmm_apply(plan, (const double*)q.p, (double*)y, 1, stream);
    if (st != HFMM_OK) return st;
    hipLaunchKernelGGL(k_bie_diag, dim3(nb(n)), dim3(BT), 0, s, n, k1, w, x, y);
    return HFMM_OK;
  };
  auto axpby = [&](cd a, const double2* x, cd b, double2* y) {
    hipLaunchKernelGGL(k_bie_axpby, dim3(nb(n)), dim3(BT), 0, s, n, cmk(a.real(), a.imag()), x,
                       cmk(b.real(), b.imag()), y);
  };
  const double2* F = (const double2*)f;
  double2* X = (double2*)phi;
  cd ff;
  if ((e = dot(F, F, ff)) != hipSuccess) return report(HFMM_ERR_DEVICE, "bie dot");
  const double fnorm = std::sqrt(ff.real());
  int it = 0;
  double rel = 1.0;
  std::vector<cd> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
  while (true) {
    // r = f - (A W + D) x into V[0]
    hfmm_status_t st = op(X, V.p);
    if (st != HFMM_OK) return st;
    axpby(1.0, F, -1.0, V.p);
    cd rr;
    if ((e = dot(V.p, V.p, rr)) != hipSuccess) return report(HFMM_ERR_DEVICE, "bie dot");
    double beta = std::sqrt(rr.real());
    rel = fnorm > 0.0 ? beta / fnorm : beta;
    if (rel <= tol || it >= max_iter || beta == 0.0) break;
    axpby(0.0, V.p, 1.0 / beta, V.p);
    std::fill(g.begin(), g.end(), cd(0.0));
    g[0] = beta;
    int j = 0;
    for (; j < m && it < max_iter; ++j, ++it) {
      double2* vj1 = V.p + (size_t)(j + 1) * n;
      if ((st = op(V.p + (size_t)j * n, vj1)) != HFMM_OK) return st;
      // modified Gram-Schmidt
      for (int i = 0; i <= j; ++i) {
        cd h;
        if ((e = dot(V.p + (size_t)i * n, vj1, h)) != hipSuccess) return report(HFMM_ERR_DEVICE, "bie dot");
        H[(size_t)i * m + j] = h;
        axpby(-h, V.p + (size_t)i * n, 1.0, vj1);
      }
      cd hh;
      if ((e = dot(vj1, vj1, hh)) != hipSuccess) return report(HFMM_ERR_DEVICE, "bie dot");
      const double hn = std::sqrt(hh.real());
      H[(size_t)(j + 1) * m + j] = hn;
      if (hn > 0.0) axpby(0.0, vj1, 1.0 / hn, vj1);
      // apply the previous rotations, then a new one to zero H[j+1][j]
      for (int i = 0; i < j; ++i) {
        const cd a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = std::conj(cs[i]) * a + std::conj(sn[i]) * b;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
      }
      const cd a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
      const double r = std::sqrt(std::norm(a) + std::norm(b));
      cs[j] = r > 0.0 ? a / r : cd(1.0);
      sn[j] = r > 0.0 ? b / r : cd(0.0);
      H[(size_t)j * m + j] = r;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = std::conj(cs[j]) * g[j];
      rel = fnorm > 0.0 ? std::abs(g[j + 1]) / fnorm : std::abs(g[j + 1]);
      if (rel <= tol) {
        ++j;
        ++it;
        break;
      }
    }
    // x += V y, H y = g (upper triangular, j columns)
    std::vector<cd> y(j);
    for (int i = j - 1; i >= 0; --i) {
      cd t = g[i];
      for (int c = i + 1; c < j; ++c) t -= H[(size_t)i * m + c] * y[c];
      y[i] = t / H[(size_t)i * m + i];
    }
    for (int i = 0; i < j; ++i) axpby(y[i], V.p + (size_t)i * n, 1.0, X);
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return report(HFMM_ERR_DEVICE, "bie");
  if (iterations) *iterations = it;
  if (residual) *residual = rel;
  return HFMM_OK;
}

}  // extern "C"
