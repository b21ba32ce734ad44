// FP64 Bessel and Hankel functions for the HIP kernels.
//
// Methods (all standard, written from the mathematics):
//  * J_n(x), n = 0..nmax: Miller's backward recurrence J_{n-1} = (2n/x) J_n -
//    J_{n+1} from a start index well above max(nmax, x), normalised by the
//    identity J_0 + 2 sum_k J_{2k} = 1 (Abramowitz & Stegun 9.1.27, 9.1.46).
//    Values are rescaled by exact powers of two to stay in range; a first pass
//    finds the normalisation, a second pass emits the values.
//  * H_0^(1)(x) = J_0 + i Y_0: ascending series (A&S 9.1.12, 9.1.13) for
//    x < 8, the library j0/y0 above.
//  * Y_n by the forward recurrence from Y_0, Y_1 (stable upward).
#pragma once

#include "common.hpp"

namespace hfmm {

__host__ __device__ inline int miller_start(double x, int nmax) {
  double m = fmax((double)nmax, x);
  return (int)(m + 20.0 + 12.0 * cbrt(m + 1.0));
}

constexpr double kRescaleHi = 0x1p+700;   // rescale when |J| exceeds this
constexpr double kRescaleBy = 0x1p-700;

// Pass 1: normalisation of the backward sequence. Returns 1/S in the final
// scale and the number of rescalings performed.
__host__ __device__ inline void miller_norm(double x, int nstart, double& inv_s, int& nres) {
  double jp1 = 0.0, j = 0x1p-900, s = 0.0;
  nres = 0;
  for (int n = nstart; n >= 1; --n) {
    if ((n & 1) == 0) s += 2.0 * j;
    double jm1 = (2.0 * n / x) * j - jp1;
    jp1 = j;
    j = jm1;
    if (fabs(j) > kRescaleHi) {
      j *= kRescaleBy; jp1 *= kRescaleBy; s *= kRescaleBy;
      ++nres;
    }
  }
  s += j;  // J_0
  inv_s = 1.0 / s;
}

// Pass 2: calls f(n, J_n) for n = nmax down to 0 with normalised values.
template <class F>
__host__ __device__ inline void miller_emit(double x, int nstart, int nmax, double inv_s, int nres, F f) {
  double jp1 = 0.0, j = 0x1p-900;
  int done = 0;
  // scale factor from the current scale to the final one: kRescaleBy^(nres - done)
  auto scale_now = [&]() {
    double sc = inv_s;
    for (int r = done; r < nres; ++r) sc *= kRescaleBy;
    return sc;
  };
  double sc = scale_now();
  if (nstart <= nmax) f(nstart, j * sc);
  for (int n = nstart; n >= 1; --n) {
    double jm1 = (2.0 * n / x) * j - jp1;
    jp1 = j;
    j = jm1;
    if (fabs(j) > kRescaleHi) {
      j *= kRescaleBy; jp1 *= kRescaleBy;
      ++done;
      sc = scale_now();
    }
    if (n - 1 <= nmax) f(n - 1, j * sc);
  }
}

// J_n(x) for n = 0..nmax into out[0..nmax]. x >= 0.
template <class F>
__host__ __device__ inline void bessel_j_each(double x, int nmax, F f) {
  if (x == 0.0) {
    for (int n = nmax; n >= 0; --n) f(n, n == 0 ? 1.0 : 0.0);
    return;
  }
  int ns = miller_start(x, nmax);
  double inv_s;
  int nres;
  miller_norm(x, ns, inv_s, nres);
  miller_emit(x, ns, nmax, inv_s, nres, f);
}

// H_0^(1)(x) = J_0(x) + i Y_0(x), x > 0.
__device__ inline double2 hankel0(double x) {
  if (x < 8.0) {
    const double q = 0.25 * x * x;
    double t = 1.0, j0s = 1.0, ys = 0.0, hm = 0.0;
    for (int m = 1; m < 40; ++m) {
      t *= -q / ((double)m * (double)m);
      hm += 1.0 / (double)m;
      j0s += t;
      ys -= hm * t;
      if (fabs(t) * hm < 1e-18) break;
    }
    const double two_pi = 0.63661977236758134308;   // 2/pi
    const double euler = 0.57721566490153286061;
    double y0v = two_pi * ((log(0.5 * x) + euler) * j0s + ys);
    return cmk(j0s, y0v);
  }
  return cmk(::j0(x), ::y0(x));
}

}  // namespace hfmm
