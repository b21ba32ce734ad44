// Shared plain-data structures and complex helpers for the host planner and the
// HIP kernels of the layered-media heterogeneous FMM.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HFMM_MAX_LEVELS 32

namespace hfmm {

// ---------------------------------------------------------------- complex helpers
// Complex numbers are double2 (x = real, y = imaginary).
__host__ __device__ inline double2 cmk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return cmk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cscale(double2 a, double s) { return cmk(a.x * s, a.y * s); }
__host__ __device__ inline double2 cconj(double2 a) { return cmk(a.x, -a.y); }
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, den = b.x + b.y * r;
    return cmk((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  }
  double r = b.x / b.y, den = b.x * r + b.y;
  return cmk((a.x * r + a.y) / den, (a.y * r - a.x) / den);
}
// w^n for n >= 0 by repeated squaring (|w| = 1 here: the error grows with the
// number of squarings, about log2 n roundings).
__host__ __device__ inline double2 cpowi(double2 w, int n) {
  double2 r = cmk(1.0, 0.0);
  while (n > 0) {
    if (n & 1) r = cmul(r, w);
    w = cmul(w, w);
    n >>= 1;
  }
  return r;
}
__host__ __device__ inline double cabs2(double2 a) { return hypot(a.x, a.y); }
__host__ __device__ inline double2 cexp2(double2 a) {
  double e = exp(a.x);
  double s, c;
  sincos(a.y, &s, &c);
  return cmk(e * c, e * s);
}
__host__ __device__ inline double2 clog2(double2 a) { return cmk(log(cabs2(a)), atan2(a.y, a.x)); }
// Integer literals mean double precision.
__host__ __device__ inline double2 cmk(int r, int i) { return make_double2(r, i); }
// The same for single precision (float2), used by the FP32 near field.
__host__ __device__ inline float2 cmk(float r, float i) { return make_float2(r, i); }
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// complex type of a real type
template <typename T> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };
template <typename T> using cplx_t = typename cplx_of<T>::type;
template <typename T> __host__ __device__ inline cplx_t<T> to_cplx(double2 v) { return cmk((T)v.x, (T)v.y); }

// Principal square root (Re >= 0); the sign of a zero imaginary part is kept.
__host__ __device__ inline double2 csqrt2(double2 a) {
  double r = cabs2(a);
  if (r == 0.0) return cmk(0.0, 0.0);
  double t = sqrt(0.5 * (r + fabs(a.x)));
  if (a.x >= 0.0) return cmk(t, a.y / (2.0 * t));
  return cmk(fabs(a.y) / (2.0 * t), copysign(t, a.y));
}
// Physical branch of sqrt(w) with w = lambda^2 - k^2: Re >= 0, and for a real
// negative w the outgoing value -i sqrt(-w). Off the real axis the contours used
// here keep Im(w) < 0, where the principal root is that branch's continuation.
__host__ __device__ inline double2 gamma_branch(double2 w) {
  if (w.y == 0.0) {
    if (w.x >= 0.0) return cmk(sqrt(w.x), 0.0);
    return cmk(0.0, -sqrt(-w.x));
  }
  return csqrt2(w);
}

// ---------------------------------------------------------------- medium
struct Medium {
  int layers;     // 2 or 3; 1: the impedance half-space
  double k1, k2, k3;  // k3 == k2 for two layers, k2 == k3 == k1 for the half-space
  double d;       // slab thickness (three layers)
  double alpha;   // impedance of the half-space's boundary (layers == 1)
};

// sigma_1 from the physical gammas of the three layers (two layers: r12).
// Closed form of the interface system: a slab of thickness d between the
// half-spaces, sigma_1 = (r12 + r23 E)/(1 + r12 r23 E), E = exp(-2 g2 d).
// The impedance half-space (Section 2.2, Eq. multisommer): sigma-hat =
// (g1 + i alpha)/(g1 - i alpha); with alpha > 0 its pole g1 = i alpha lies
// off the physical sheet's contours (there Im g1 <= 0).
__host__ __device__ inline double2 sigma1_from(const Medium& m, double2 g1, double2 g2, double2 g3) {
  if (m.layers == 1) return cdiv(cmk(g1.x, g1.y + m.alpha), cmk(g1.x, g1.y - m.alpha));
  double2 r12 = cdiv(csub(g1, g2), cadd(g1, g2));
  if (m.layers == 2) return r12;
  double2 r23 = cdiv(csub(g2, g3), cadd(g2, g3));
  double2 e = cexp2(cscale(g2, -2.0 * m.d));
  double2 num = cadd(r12, cmul(r23, e));
  double2 den = cadd(cmk(1.0, 0.0), cmul(cmul(r12, r23), e));
  return cdiv(num, den);
}

// sigma_1 on the evanescent parametrisation: lambda^2 = t^2 + k1^2, gamma_1 = t.
__host__ __device__ inline double2 sigma1_t(const Medium& m, double2 t) {
  double2 t2 = cmul(t, t);
  double2 w2 = cmk(t2.x + (m.k1 * m.k1 - m.k2 * m.k2), t2.y);
  double2 w3 = cmk(t2.x + (m.k1 * m.k1 - m.k3 * m.k3), t2.y);
  return sigma1_from(m, t, gamma_branch(w2), gamma_branch(w3));
}

// sigma_1 on the propagating parametrisation lambda = -k1 cos(tau), tau in [0, pi].
// All lower layers have k_j >= k1, so gamma_j = -i sqrt(k_j^2 - lambda^2).
__host__ __device__ inline double2 sigma1_tau(const Medium& m, double ct, double st) {
  double l2 = m.k1 * m.k1 * ct * ct;
  double2 g1 = cmk(0.0, -m.k1 * st);
  double2 g2 = cmk(0.0, -sqrt(fmax(m.k2 * m.k2 - l2, 0.0)));
  double2 g3 = cmk(0.0, -sqrt(fmax(m.k3 * m.k3 - l2, 0.0)));
  return sigma1_from(m, g1, g2, g3);
}

// ---------------------------------------------------------------- plan views
// Table descriptor: a Toeplitz vector T[n], n in [-half, half], stored at
// data[off + half + n].
struct TableRef {
  int64_t off;
  int32_t half;
  int32_t pad;
};

// A contour panel for the Sommerfeld quadratures: kind 0 = tau in [a, b]
// (propagating part), kind 1 = s in [a, b] on the evanescent contour
// t(s) = s - i*dip*sin(pi s / send) for s < send, t = s beyond.
struct Panel {
  double a, b;
  int32_t kind;
  int32_t pad;
};

// Pairs per translation item: one 16-column MFMA tile; the four waves of the
// block split its row tiles. (Larger items, 32 or 64 pairs sharing the staged
// table, measured slower: their source tiles cut the blocks per CU.)
__host__ __device__ inline int trans_pairs_per_item(int Ps, int Pd) {
  (void)Ps;
  (void)Pd;
  return 16;
}

// A work item of the batched translation contraction: one translation table
// and up to 64 (source, target) box pairs that use it, pairs
// [pbeg, pbeg + npairs) of the pair arrays; source order Ps, target order Pd;
// rt_base is the first row tile of the real-embedded operator and ntw the
// number of row tiles per wave (1..8); image marks heterogeneous M2L tables
// (reflected source coefficients).
struct TransItem {
  int32_t table;  // M2M / L2L: quadrant, an index into the launch's four tables
  int32_t pbeg;
  int32_t npairs;
  int32_t image;
  int32_t rt_base;
  int32_t Ps, Pd;
  int32_t ntw;
  int64_t toff;  // M2L: offset of t[-(Ps + Pd)] in the table data (-1: by quadrant)
};
// The four tables of an M2M or L2L launch (offsets of t[-(Ps + Pd)]), passed
// by value.
struct Toff4 {
  int64_t v[4];
};

// Row tiles one item covers: ntw per wave, the four waves interleaved over
// the rows.
__host__ __device__ inline int trans_rows_per_item(int Ps, int Pd, int ntw) {
  (void)Ps;
  (void)Pd;
  return 4 * ntw;
}


struct TreeView {
  int32_t n;
  int32_t nboxes;
  int32_t nlev;
  int32_t nrhs;
  double k;
  const double2* pts;      // sorted points, interface frame
  const double2* ctr;      // box centres
  const int32_t* level;    // box level
  const int2* prange;      // box point range [begin, end)
  const int64_t* coff;     // box coefficient offset (per right-hand side plane)
  const int32_t* child;    // 4 per box, -1 if absent; quadrant q = 2*ybit + xbit
  const int32_t* parent;
  const int32_t* quad;     // quadrant of a box within its parent
  int64_t ctot;            // coefficients per right-hand side plane
  int32_t P[HFMM_MAX_LEVELS];
};

}  // namespace hfmm
