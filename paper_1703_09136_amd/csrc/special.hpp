// FP64 Bessel and Hankel functions for the HIP kernels.
//
// Methods (all standard, written from the mathematics):
//  * J_n(x), n = 0..nmax: Miller's backward recurrence J_{n-1} = (2n/x) J_n -
//    J_{n+1} from a start index well above max(nmax, x), normalised by the
//    identity J_0 + 2 sum_k J_{2k} = 1 (Abramowitz & Stegun 9.1.27, 9.1.46).
//    Values are rescaled by exact powers of two to stay in range; a first pass
//    finds the normalisation, a second pass emits the values.
//  * H_0^(1)(x) = J_0 + i Y_0: ascending series (A&S 9.1.12, 9.1.13) in
//    Horner form for x <= 6; beyond, the modulus-phase form of Hankel's
//    asymptotic representation with its smooth factor interpolated by
//    Chebyshev polynomials in 1/x (coefficients from 34-digit values).
//  * Y_n by the forward recurrence from Y_0, Y_1 (stable upward).
#pragma once

#include "common.hpp"
#include "h0_cheb.hpp"
#include "h1_cheb.hpp"
#include "log_table.hpp"

namespace hfmm {

// Start indices of the backward recurrence are multiples of 4 (the passes
// below take four steps at a time).
__host__ __device__ inline int miller_round(int n) { return (n + 3) & ~3; }

__host__ __device__ inline int miller_start(double x, int nmax) {
  double m = fmax((double)nmax, x);
  return miller_round((int)(m + 20.0 + 12.0 * cbrt(m + 1.0)));
}

// Start index for the expansions at a leaf, orders 0..nmax at arguments up to
// x, when nmax is well above x (nmax >= 2x + 2; otherwise the general start
// above). For m >= nmax > x the ratio J_{m+1}(x) / J_m(x) is at most
// x / (2(m + 1) - x): the continued fraction of the ratio, every later ratio
// being below one. A backward walk started at N computes
// J_n - (J_{N+1} / Y_{N+1}) Y_n up to normalisation, a relative error of
// (J_{N+1} Y_n) / (Y_{N+1} J_n); at large order J_m Y_m ~ -1 / (pi m), so at
// n = nmax (the worst order) it is about (J_{N+1} / J_nmax)^2 (N + 1) / nmax.
// The start is two past the index where the bound of J_{N+1} / J_nmax falls
// below 1e-10, so that this error stays under 1e-19.
__host__ __device__ inline int miller_start_expansion(double x, int nmax) {
  if (!((double)nmax >= 2.0 * x + 2.0)) return miller_start(x, nmax);
  double r = 1.0;  // bound of J_m / J_nmax
  int m = nmax;
  while (r > 1e-10) {
    r *= x / (2.0 * (double)(m + 1) - x);
    ++m;
  }
  return miller_round(m + 1);
}

constexpr double kRescaleHi = 0x1p+700;   // rescale when |J| exceeds this
constexpr double kRescaleBy = 0x1p-700;
// Arguments below kTinyX are raised to it: then J_n(x) = J_n(kTinyX) to
// 1.3e-19 absolutely for n != 1, and J_1(x) = (x / kTinyX) J_1(kTinyX) to a
// relative 1e-19 (the ascending series' second terms), which callers apply.
// It bounds the growth of the backward sequence, at most 2 n / x per step:
// below 2^41 for the starts used here (n < 1100), so four steps between
// rescaling checks stay far from overflow.
constexpr double kTinyX = 1e-9;

// Pass 1: normalisation of the backward sequence, S = J_0 + 2 sum J_{2k}
// unnormalised, four steps at a time (nstart a multiple of 4, x >= kTinyX).
// Returns 1/S in the final scale and the number of rescalings performed. The
// recurrence is j_{n-1} = fma(n (2/x), j_n, -j_{n+1}), rescaled whenever a new
// index is a multiple of 4 and |j| exceeds kRescaleHi; the walk below uses
// this same arithmetic so that both passes rescale at the same indices.
__host__ __device__ inline void miller_norm(double x, int nstart, double& inv_s, int& nres) {
  const double tx = 2.0 / x;
  double jp1 = 0.0, j = 0x1p-900, s = 0.0;
  nres = 0;
  double dn = (double)nstart;
  for (int n = nstart; n >= 4; n -= 4) {  // j = j_n, jp1 = j_{n+1}, n even
    const double a = fma(dn * tx, j, -jp1);          // j_{n-1}
    const double b = fma((dn - 1.0) * tx, a, -j);    // j_{n-2}
    const double c = fma((dn - 2.0) * tx, b, -a);    // j_{n-3}
    const double d = fma((dn - 3.0) * tx, c, -b);    // j_{n-4}
    s += 2.0 * (j + b);
    jp1 = c;
    j = d;
    dn -= 4.0;
    if (fabs(j) > kRescaleHi) {
      j *= kRescaleBy; jp1 *= kRescaleBy; s *= kRescaleBy;
      ++nres;
    }
  }
  s += j;  // J_0
  inv_s = 1.0 / s;
}

// Pass 2 as an explicit walk: value() is the normalised J_n at the current
// index n (starting at nstart); step() moves to n - 1.
struct MillerWalk {
  double tx, j, jp1, inv_s, dn;
  int n, left;  // rescalings still ahead
  __host__ __device__ MillerWalk(double x, int nstart, double inv_s_, int nres)
      : tx(2.0 / x), j(0x1p-900), jp1(0.0), inv_s(inv_s_), dn((double)nstart), n(nstart), left(nres) {}
  // J_n = j kRescaleBy^left / S, the power applied exactly by ldexp
  __host__ __device__ double value() const { return ldexp(j * inv_s, -700 * left); }
  __host__ __device__ void step() {
    const double jm1 = fma(dn * tx, j, -jp1);
    jp1 = j;
    j = jm1;
    --n;
    dn -= 1.0;
    if ((n & 3) == 0 && fabs(j) > kRescaleHi) {
      j *= kRescaleBy; jp1 *= kRescaleBy;
      --left;
    }
  }
};
static_assert(kRescaleBy == 0x1p-700, "MillerWalk::value applies the rescale factor as 2^-700");

// Pass 2: calls f(n, J_n) for n = nmax down to 0 with normalised values.
template <class F>
__host__ __device__ inline void miller_emit(double x, int nstart, int nmax, double inv_s, int nres, F f) {
  MillerWalk w(x, nstart, inv_s, nres);
  if (nstart <= nmax) f(nstart, w.value());
  while (w.n >= 1) {
    w.step();
    if (w.n <= nmax) f(w.n, w.value());
  }
}

// J_n(x) for n = 0..nmax into out[0..nmax]. x >= 0.
template <class F>
__host__ __device__ inline void bessel_j_each(double x, int nmax, F f) {
  if (x == 0.0) {
    for (int n = nmax; n >= 0; --n) f(n, n == 0 ? 1.0 : 0.0);
    return;
  }
  const double xr = fmax(x, kTinyX), s1 = x < kTinyX ? x / kTinyX : 1.0;
  int ns = miller_start(xr, nmax);
  double inv_s;
  int nres;
  miller_norm(xr, ns, inv_s, nres);
  miller_emit(xr, ns, nmax, inv_s, nres, [&](int n, double v) { f(n, n == 1 ? s1 * v : v); });
}

// Coefficients of the ascending series in z = x^2/4 (A&S 9.1.12, 9.1.13):
//   J_0 = sum_m c_m z^m,  c_m = (-1)^m / (m!)^2,
//   Y_0 = (2/pi) [ (ln(x/2) + gamma) J_0 + sum_{m>=1} d_m z^m ],  d_m = -H_m c_m,
// with H_m the harmonic numbers; generated at compile time.
constexpr int kSeriesTerms = 28;
struct H0Series {
  double c[kSeriesTerms];
  double d[kSeriesTerms];
  constexpr H0Series() : c(), d() {
    double cm = 1.0, hm = 0.0;
    c[0] = 1.0;
    d[0] = 0.0;
    for (int m = 1; m < kSeriesTerms; ++m) {
      cm = cm * (-1.0 / ((double)m * (double)m));
      hm += 1.0 / (double)m;
      c[m] = cm;
      d[m] = -hm * cm;
    }
  }
};
constexpr H0Series kH0{};

// H_0^(1)(x) by the ascending series in Horner form, for 0 < x <= 6. The
// number of terms follows the range: the tail term z^M / (M!)^2 stays below
// 1e-18 (M = 13 for x <= 2, 21 for x <= 6).
template <int M>
__host__ __device__ inline double2 hankel0_series(double x) {
  const double z = 0.25 * x * x;
  double j = kH0.c[M - 1], s = kH0.d[M - 1];
#pragma unroll
  for (int m = M - 2; m >= 0; --m) {
    j = fma(j, z, kH0.c[m]);
    s = fma(s, z, kH0.d[m]);
  }
  const double two_over_pi = 0.63661977236758134308;
  const double euler = 0.57721566490153286061;
  return cmk(j, two_over_pi * ((0.5 * log(z) + euler) * j + s));
}

// H_0^(1)(x) for x >= 6 from its modulus-phase form
// sqrt(2/(pi x)) F(1/x) e^{i(x - pi/4)}, with F interpolated by Chebyshev
// polynomials in w = 1/x on [0, 1/6] (coefficients in h0_cheb.hpp) and summed
// by Clenshaw's recurrence.
__host__ __device__ inline double2 hankel0_large(double x) {
  const double t = 2.0 * kH0ChebX0 / x - 1.0;
  const double t2 = 2.0 * t;
  double br1 = 0.0, br2 = 0.0, bi1 = 0.0, bi2 = 0.0;
#pragma unroll
  for (int k = kH0ChebN - 1; k >= 1; --k) {
    double br = fma(t2, br1, kH0ChebRe[k] - br2);
    double bi = fma(t2, bi1, kH0ChebIm[k] - bi2);
    br2 = br1; br1 = br;
    bi2 = bi1; bi1 = bi;
  }
  double fr = fma(t, br1, kH0ChebRe[0] - br2);
  double fi = fma(t, bi1, kH0ChebIm[0] - bi2);
  double s, c;
  sincos(x - 0.78539816339744830962, &s, &c);
  double a = sqrt(0.63661977236758134308 / x);
  return cmk(a * (fr * c - fi * s), a * (fr * s + fi * c));
}

// H_0^(1)(x) = J_0(x) + i Y_0(x), x > 0: the ascending series up to x = 6,
// the Chebyshev modulus-phase form beyond.
__host__ __device__ inline double2 hankel0(double x) {
  if (x <= 2.0) return hankel0_series<13>(x);
  if (x <= 6.0) return hankel0_series<21>(x);
  return hankel0_large(x);
}

// Out-of-line large-argument form for the pair loops (keeps its coefficients
// out of the registers of the caller).
__device__ __noinline__ double2 hankel0_large_call(double x);

// Four values of H_0^(1) at once from z_u = x_u^2/4 by the ascending series
// with M terms, the four Horner chains interleaved. M is chosen by the caller
// from a bound on z: the first dropped term max(|c_M|, |d_M|) z^M stays below
// 2^-56 for z <= h0_series_zmax(M) (from the closed forms of c_M and d_M).
// With LARGE, entries with z > 9 (x > 6) take the large-argument form.
// ln(z) for a positive normal z in about 30 operations, for the pair loops:
// z = 2^e m with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s) =
// 2 sum_k s^(2k+1)/(2k+1) with s = (m - 1)/(m + 1), |s| <= 0.1716, where
// eleven terms leave a relative remainder below 2^-56; e ln 2 is added in two
// parts (Cody and Waite's reduction; ln2_hi has 11 trailing zero bits, so
// e * ln2_hi is exact). The quotient s comes from the hardware reciprocal,
// two Newton steps and a residual correction.
__device__ inline double log_pos(double z) {
  int e;
  double m = frexp(z, &e);  // m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double num = m - 1.0, den = m + 1.0;
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  r = fma(r, fma(-den, r, 1.0), r);
  double sq = num * r;
  sq = fma(r, fma(-sq, den, num), sq);
  const double s2 = sq * sq;
  // sum_{k=0..10} s2^k / (2k + 1) by Horner
  double p = 1.0 / 21.0;
  p = fma(p, s2, 1.0 / 19.0);
  p = fma(p, s2, 1.0 / 17.0);
  p = fma(p, s2, 1.0 / 15.0);
  p = fma(p, s2, 1.0 / 13.0);
  p = fma(p, s2, 1.0 / 11.0);
  p = fma(p, s2, 1.0 / 9.0);
  p = fma(p, s2, 1.0 / 7.0);
  p = fma(p, s2, 1.0 / 5.0);
  p = fma(p, s2, 1.0 / 3.0);
  const double ln_m = 2.0 * fma(sq * s2, p, sq);
  const double ln2_hi = 0x1.62e42fefa3800p-1;
  const double ln2_lo = 0x1.ef35793c76730p-45;
  const double de = (double)e;
  return fma(de, ln2_hi, fma(de, ln2_lo, ln_m));
}

// a * b + c with c a wave-uniform constant, as one VOP3 instruction taking c
// from scalar registers. Left to itself the compiler keeps such constants in
// vector registers and copies one into the accumulator before every
// two-address v_fmac_f64, which doubles the cost of a Horner step.
__device__ inline double fma_uniform(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

// The same in FP32 (near field of the mixed-precision plans): one VOP3 FMA
// with the coefficient in a scalar register, and ln z by the reduction above
// with five atanh terms (relative remainder below 2^-26).
__device__ inline float fma_uniform(float a, float b, float c) {
  float r;
  asm("v_fma_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

__device__ inline float log_pos(float z) {
  int e;
  float m = frexpf(z, &e);  // m in [1/2, 1)
  if (m < 0.70710678f) {
    m *= 2.0f;
    e -= 1;
  }
  const float num = m - 1.0f, den = m + 1.0f;
  float r = __builtin_amdgcn_rcpf(den);
  r = fmaf(r, fmaf(-den, r, 1.0f), r);
  float sq = num * r;
  sq = fmaf(r, fmaf(-sq, den, num), sq);
  const float s2 = sq * sq;
  float p = 1.0f / 9.0f;
  p = fmaf(p, s2, 1.0f / 7.0f);
  p = fmaf(p, s2, 1.0f / 5.0f);
  p = fmaf(p, s2, 1.0f / 3.0f);
  const float ln_m = 2.0f * fmaf(sq * s2, p, sq);
  const float ln2_hi = 0x1.62e4p-1f;  // 8 trailing zero bits
  const float ln2_lo = 0x1.7f7d1cp-20f;
  const float de = (float)e;
  return fmaf(de, ln2_hi, fmaf(de, ln2_lo, ln_m));
}

// ln z for z > 0 (normal) from the mantissa bins of log_table.hpp, tab[i] =
// {a_i, -ln a_i} (staged in LDS by the caller): with z = 2^e m, m in [1, 2)
// in bin i, ln z = e ln 2 - ln a_i + ln(1 + r), r = m a_i - 1 (one fused
// multiply-add, |r| <= 2^-7), and ln(1 + r) = r - r^2/2 + ... + r^7/7 (the
// first dropped term is below 2^-59). ln 2 is split so that e ln2_hi is exact.
__device__ inline double log_tab(double z, const double2* tab) {
  int e;
  const double m = 2.0 * frexp(z, &e);  // [1, 2), z = 2^(e - 1) m
  const int i = (__double2hiint(m) >> (20 - kLogTabBits)) & ((1 << kLogTabBits) - 1);
  const double2 t = tab[i];
  const double r = fma(m, t.x, -1.0);
  double w = fma(r, 1.0 / 7.0, -1.0 / 6.0);
  w = fma_uniform(w, r, 1.0 / 5.0);
  w = fma_uniform(w, r, -0.25);
  w = fma_uniform(w, r, 1.0 / 3.0);
  w = fma_uniform(w, r, -0.5);
  const double p = fma(w, r * r, r);
  const double ln2_hi = 0x1.62e42fefa3800p-1;
  const double ln2_lo = 0x1.ef35793c76730p-45;
  const double de = (double)(e - 1);
  return fma(de, ln2_hi, fma(de, ln2_lo, t.y) + p);
}

// NV values (four by default) of H_0^(1) at once from z_u = x_u^2/4, in the
// precision T, by the ascending series with M terms and the NV Horner chains
// interleaved. M is chosen by the caller from a bound on z: the first dropped
// term max(|c_M|, |d_M|) z^M stays below the precision's half-ulp for
// z <= the class bound (from the closed forms of c_M and d_M). With LARGE,
// entries with z > 9 (x > 6) take the FP64 large-argument form. In FP64 the
// logarithm takes the bin table ltab (LDS).
template <typename T, int M, bool LARGE, int NV = 4>
__device__ inline void hankel0_x4(const T z[NV], T hr[NV], T hi[NV], const double2* ltab) {
  T j[NV], s[NV];
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    j[u] = (T)kH0.c[M - 1];
    s[u] = (T)kH0.d[M - 1];
  }
#pragma unroll
  for (int m = M - 2; m >= 0; --m) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      j[u] = fma_uniform(j[u], z[u], (T)kH0.c[m]);
      s[u] = fma_uniform(s[u], z[u], (T)kH0.d[m]);
    }
  }
  const T two_over_pi = (T)0.63661977236758134308;
  const T euler = (T)0.57721566490153286061;
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    if (!LARGE || z[u] <= (T)9.0) {
      hr[u] = j[u];
      T lz;
      if constexpr (sizeof(T) == 8)
        lz = log_tab(z[u], ltab);
      else
        lz = log_pos(z[u]);
      hi[u] = two_over_pi * (((T)0.5 * lz + euler) * j[u] + s[u]);
    } else {
      const double2 h = hankel0_large_call(2.0 * sqrt((double)z[u]));
      hr[u] = (T)h.x;
      hi[u] = (T)h.y;
    }
  }
}

// H_1^(1)(x) = J_1 + i Y_1 for x > 0 (coordinate gradients of the direct
// part: d/dr H_0^(1)(k r) = -k H_1^(1)(k r)). For x <= 6 the ascending series
// (A&S 9.1.10, 9.1.11) in z = x^2/4:
//   J_1 = (x/2) sum_m a_m z^m,  a_m = (-1)^m / (m! (m+1)!),
//   Y_1 = (2/pi)(ln(x/2) + gamma) J_1 - 2/(pi x) - (x/(2 pi)) sum_m b_m z^m,
//   b_m = (H_m + H_{m+1}) a_m (harmonic numbers),
// 21 terms (first dropped term below 2^-56 at z = 9); beyond, the
// modulus-phase form sqrt(2/(pi x)) F(1/x) e^{i(x - 3 pi/4)} with F from
// h1_cheb.hpp.
struct H1Series {
  double a[kSeriesTerms];
  double b[kSeriesTerms];
  constexpr H1Series() : a(), b() {
    double am = 1.0, hm = 0.0;  // a_0 = 1, H_0 = 0
    for (int m = 0; m < kSeriesTerms; ++m) {
      if (m > 0) {
        am = am * (-1.0 / ((double)m * (double)(m + 1)));
        hm += 1.0 / (double)m;
      }
      a[m] = am;
      b[m] = (2.0 * hm + 1.0 / (double)(m + 1)) * am;  // (H_m + H_{m+1}) a_m
    }
  }
};
constexpr H1Series kH1{};

__host__ __device__ inline double2 hankel1_large(double x) {
  const double t = 2.0 * kH1ChebX0 / x - 1.0;
  const double t2 = 2.0 * t;
  double br1 = 0.0, br2 = 0.0, bi1 = 0.0, bi2 = 0.0;
#pragma unroll
  for (int k = kH1ChebN - 1; k >= 1; --k) {
    double br = fma(t2, br1, kH1ChebRe[k] - br2);
    double bi = fma(t2, bi1, kH1ChebIm[k] - bi2);
    br2 = br1; br1 = br;
    bi2 = bi1; bi1 = bi;
  }
  double fr = fma(t, br1, kH1ChebRe[0] - br2);
  double fi = fma(t, bi1, kH1ChebIm[0] - bi2);
  double s, c;
  sincos(x - 2.35619449019234492885, &s, &c);
  double a = sqrt(0.63661977236758134308 / x);
  return cmk(a * (fr * c - fi * s), a * (fr * s + fi * c));
}

__host__ __device__ inline double2 hankel1_series(double x) {
  const double z = 0.25 * x * x;
  double sa = kH1.a[20], sb = kH1.b[20];
#pragma unroll
  for (int m = 19; m >= 0; --m) {
    sa = fma(sa, z, kH1.a[m]);
    sb = fma(sb, z, kH1.b[m]);
  }
  const double j1 = 0.5 * x * sa;
  const double two_over_pi = 0.63661977236758134308;
  const double euler = 0.57721566490153286061;
  const double y1 = two_over_pi * ((0.5 * log(z) + euler) * j1 - 1.0 / x) - (0.5 / 3.14159265358979323846) * x * sb;
  return cmk(j1, y1);
}

__host__ __device__ inline double2 hankel1(double x) { return x <= 6.0 ? hankel1_series(x) : hankel1_large(x); }

// Series classes of the pair loops: the largest z each covers and the terms
// it takes in FP64 (remainder below 2^-56) and in FP32 (below 2^-26).
constexpr int kH0Classes = 5;
constexpr double kH0ClassZmax[kH0Classes] = {0.0976, 0.3797, 1.0021, 2.8639, 9.0};
constexpr int kH0ClassTerms[kH0Classes] = {8, 10, 12, 15, 20};
constexpr int kH0ClassTermsF32[kH0Classes] = {5, 6, 8, 10, 14};

}  // namespace hfmm
