// Fields below the top interface of top-layer sources (hfmm_transmit): the
// middle- and bottom-layer fields of Section 2.3 (u_2 = u_2^t + u_2^b with the
// densities sigma_2^+ and sigma_2^-, u_3 with sigma_3; two layers: the lower
// half-space's field) summed over a source set.
//
// Solving the interface system of Section 2.3 by elimination (continuity of u
// and du/dy at y = 0 and y = -d, the paper's unknowns and right-hand side)
// gives, with g_j = sqrt(lambda^2 - k_j^2), E = e^{-g2 d} and
// R = (g2 - g3) / (g2 + g3):
//   sigma_2^+ / g2 = 2 / ((g1 + g2) + E^2 R (g1 - g2)),
//   sigma_2^- = E R sigma_2^+,   sigma_3 / g3 = 2 E g2 (sigma_2^+ / g2) / (g2 + g3).
// So in the interface frame (top interface y = 0), for a source at (x0, y0),
//   layer 2: u = (1/4pi) int (sigma_2^+/g2) [e^{g2 y} + R e^{-g2 (y + 2d)}] e^{-g1 y0} e^{i lambda (x - x0)} d lambda,
//   layer 3: u = (1/4pi) int (sigma_3/g3) e^{g3 (y + d)} e^{-g1 y0} e^{i lambda (x - x0)} d lambda.
// The integrand factors into a source part and a target part, so one
// quadrature rule for the whole point sets turns the sum over the sources
// into node sums: with x' = x - xc (xc the centre of the sets' x range),
//   S_q^+ = sum_s q_s e^{-g1 y_s} e^{-i lambda_q x'_s},   S_q^- = same with e^{+i lambda_q x'_s},
//   u_t = sum_q T_q(y_t) (S_q^+ e^{i lambda_q x'_t} + S_q^- e^{-i lambda_q x'_t}),
// O((ns + nt) Q). The integrand is even in lambda, so the line folds onto a
// half contour from 0 to infinity (the two plane waves of each node are the
// two halves); it dips below the real axis over the branch points k_j and the
// slab's guided-mode poles (the outgoing, limiting-absorption side), by at
// most 3 / (x range) so that |e^{+-i lambda x'}| stays below e^{3/2} (a pair's
// product below e^3: about one digit of the terms' rounding, for panels about
// a quarter fewer than with a dip of 1 / (x range)).
#include "../../include/hfmm.h"
#include "common.hpp"
#include "devbuf.hpp"
#include "plan_internal.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

namespace hfmm {
namespace {

using cd = std::complex<double>;

constexpr int XL_THREADS = 256;
constexpr int XL_RB = 4;              // right-hand sides per source-sum block
constexpr size_t kXlMaxPanels = 200000;

// Per quadrature node: lambda, the source decay g1, and the target factors
// (layer 2: a e^{g2 y} + b e^{-g2 (y + 2d)}; layer 3: c e^{g3 (y + d)}), the
// weight (1/4pi) w dlambda/ds folded into a, b and c.
struct XlNode {
  double2 lam, g1, g2, g3, a, b, c;
};

// Source node sums of one chunk of sources: block (node tile, source chunk,
// right-hand-side group), a thread per node; part[chunk][r][q] holds (S+, S-)
// as two double2.
template <int RB>
__global__ void __launch_bounds__(XL_THREADS) k_xl_src(int nq, const XlNode* __restrict__ nodes, int64_t ns,
                                                       const double2* __restrict__ src, double xc, double yif,
                                                       const double2* __restrict__ q, int nrhs, int64_t chunk,
                                                       double2* __restrict__ part) {
  __shared__ double s_x[XL_THREADS], s_y[XL_THREADS];
  __shared__ double2 s_q[RB][XL_THREADS];
  const int iq = blockIdx.x * XL_THREADS + threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.y * chunk, j1 = min(ns, j0 + chunk);
  const int r0 = blockIdx.z * RB, nr = min(RB, nrhs - r0);
  double2 lam = cmk(0.0, 0.0), g1 = cmk(0.0, 0.0);
  if (iq < nq) {
    lam = nodes[iq].lam;
    g1 = nodes[iq].g1;
  }
  double2 sp[RB], sm[RB];
  for (int r = 0; r < RB; ++r) sp[r] = sm[r] = cmk(0.0, 0.0);
  for (int64_t b0 = j0; b0 < j1; b0 += XL_THREADS) {
    const int cnt = (int)min((int64_t)XL_THREADS, j1 - b0);
    __syncthreads();
    if (threadIdx.x < cnt) {
      const double2 p = src[b0 + threadIdx.x];
      s_x[threadIdx.x] = p.x - xc;
      s_y[threadIdx.x] = p.y - yif;
      for (int r = 0; r < RB; ++r)
        s_q[r][threadIdx.x] = r < nr ? q[(int64_t)(r0 + r) * ns + b0 + threadIdx.x] : cmk(0.0, 0.0);
    }
    __syncthreads();
    if (iq < nq && lam.y == 0.0 && g1.y == 0.0) {
      // a node on the real axis past every branch point: g1 and lambda real
      for (int j = 0; j < cnt; ++j) {
        const double m0 = exp(-g1.x * s_y[j]);
        double sb, cb;
        sincos(lam.x * s_x[j], &sb, &cb);
        const double2 ep = cmk(m0 * cb, -m0 * sb), em = cmk(m0 * cb, m0 * sb);
        for (int r = 0; r < RB; ++r) {
          const double2 qq = s_q[r][j];
          sp[r] = cadd(sp[r], cmul(qq, ep));
          sm[r] = cadd(sm[r], cmul(qq, em));
        }
      }
    } else if (iq < nq) {
      for (int j = 0; j < cnt; ++j) {
        const double x = s_x[j], y = s_y[j];
        // -g1 y -+ i lambda x: magnitudes e^{-g1.x y} e^{+- lambda.y x}, phases -g1.y y -+ lambda.x x
        const double m0 = exp(-g1.x * y), mx = exp(lam.y * x);
        double sa, ca, sb, cb;
        sincos(-g1.y * y, &sa, &ca);
        sincos(lam.x * x, &sb, &cb);
        const double mp = m0 * mx, mm = m0 / mx;
        const double2 ep = cmk(mp * (ca * cb + sa * sb), mp * (sa * cb - ca * sb));  // angle a - b
        const double2 em = cmk(mm * (ca * cb - sa * sb), mm * (sa * cb + ca * sb));  // angle a + b
        for (int r = 0; r < RB; ++r) {
          const double2 qq = s_q[r][j];
          sp[r] = cadd(sp[r], cmul(qq, ep));
          sm[r] = cadd(sm[r], cmul(qq, em));
        }
      }
    }
  }
  if (iq >= nq) return;
  for (int r = 0; r < nr; ++r) {
    double2* o = part + (((int64_t)blockIdx.y * nrhs + r0 + r) * nq + iq) * 2;
    o[0] = sp[r];
    o[1] = sm[r];
  }
}

// S[r][q] = sum over the chunks in order
__global__ void k_xl_sum(int64_t len, int nchunk, const double2* __restrict__ part, double2* __restrict__ S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double2 v = part[i];
  for (int c = 1; c < nchunk; ++c) v = cadd(v, part[(int64_t)c * len + i]);
  S[i] = v;
}

// u[r][t] = sum_q T_q(y_t) (S+ e^{i lambda x'} + S- e^{-i lambda x'}); a thread
// per target, the nodes staged through LDS.
template <int RB>
__global__ void __launch_bounds__(XL_THREADS) k_xl_eval(int nq, const XlNode* __restrict__ nodes,
                                                        const double2* __restrict__ S, int nrhs, int64_t nt,
                                                        const double2* __restrict__ tgt, double xc, double yif,
                                                        double d, int layers, double2* __restrict__ u) {
  __shared__ XlNode s_n[XL_THREADS / 4];
  __shared__ double2 s_s[RB][XL_THREADS / 4][2];
  constexpr int NB = XL_THREADS / 4;
  const int64_t it = (int64_t)blockIdx.x * XL_THREADS + threadIdx.x;
  const bool valid = it < nt;
  const int r0 = blockIdx.y * RB, nr = min(RB, nrhs - r0);
  double x = 0.0, y = -1.0;
  if (valid) {
    const double2 p = tgt[it];
    x = p.x - xc;
    y = p.y - yif;
  }
  const bool low = layers == 3 && y < -d;
  double2 acc[RB];
  for (int r = 0; r < RB; ++r) acc[r] = cmk(0.0, 0.0);
  for (int q0 = 0; q0 < nq; q0 += NB) {
    const int cnt = min(NB, nq - q0);
    __syncthreads();
    if (threadIdx.x < cnt) s_n[threadIdx.x] = nodes[q0 + threadIdx.x];
    for (int e = threadIdx.x; e < RB * cnt * 2; e += XL_THREADS) {
      const int r = e / (cnt * 2), rem = e - r * cnt * 2, j = rem >> 1, h = rem & 1;
      s_s[r][j][h] = r < nr ? S[((int64_t)(r0 + r) * nq + q0 + j) * 2 + h] : cmk(0.0, 0.0);
    }
    __syncthreads();
    if (!valid) continue;
    for (int j = 0; j < cnt; ++j) {
      const XlNode nd = s_n[j];
      if (nd.lam.y == 0.0 && nd.g2.y == 0.0 && nd.g3.y == 0.0) {
        // a node on the real axis past every branch point: real exponentials
        double2 T;
        if (low) {
          T = cscale(nd.c, exp(nd.g3.x * (y + d)));
        } else {
          T = cscale(nd.a, exp(nd.g2.x * y));
          if (layers == 3) T = cadd(T, cscale(nd.b, exp(-nd.g2.x * (y + 2.0 * d))));
        }
        double sn, cs;
        sincos(nd.lam.x * x, &sn, &cs);
        const double2 wp = cmk(cs, sn), wm = cmk(cs, -sn);
        for (int r = 0; r < RB; ++r) {
          const double2 v = cadd(cmul(s_s[r][j][0], wp), cmul(s_s[r][j][1], wm));
          acc[r] = cadd(acc[r], cmul(T, v));
        }
        continue;
      }
      double2 T;
      if (low) {
        T = cmul(nd.c, cexp2(cscale(nd.g3, y + d)));
      } else {
        T = cmul(nd.a, cexp2(cscale(nd.g2, y)));
        // the lower interface's reflection (three layers: y + 2d >= d > 0)
        if (layers == 3) T = cadd(T, cmul(nd.b, cexp2(cscale(nd.g2, -(y + 2.0 * d)))));
      }
      // e^{+- i lambda x} = e^{-+ lambda.y x} (cos(lambda.x x), +- sin(lambda.x x))
      const double mx = exp(-nd.lam.y * x);
      double sn, cs;
      sincos(nd.lam.x * x, &sn, &cs);
      const double2 wp = cmk(mx * cs, mx * sn), wm = cmk(cs / mx, -sn / mx);
      for (int r = 0; r < RB; ++r) {
        const double2 v = cadd(cmul(s_s[r][j][0], wp), cmul(s_s[r][j][1], wm));
        acc[r] = cadd(acc[r], cmul(T, v));
      }
    }
  }
  if (!valid) return;
  for (int r = 0; r < nr; ++r) u[(int64_t)(r0 + r) * nt + it] = acc[r];
}

// The transposed direction (hfmm_transmit with the sources below and the
// targets in the top layer): the domain Green's function is symmetric,
// G(x_t, x_s) = G(x_s, x_t), so the lower-layer factor T_q moves to the
// source sums and e^{-g1 y} to the targets:
//   S_q^+- = sum_s q_s T_q(y_s) e^{-+ i lambda_q x'_s},
//   u_t = sum_q e^{-g1 y_t} (S_q^+ e^{i lambda_q x'_t} + S_q^- e^{-i lambda_q x'_t}).
__device__ inline double2 xl_lower(const XlNode& nd, double y, double d, int layers) {
  if (layers == 3 && y < -d) return cmul(nd.c, cexp2(cscale(nd.g3, y + d)));
  double2 T = cmul(nd.a, cexp2(cscale(nd.g2, y)));
  if (layers == 3) T = cadd(T, cmul(nd.b, cexp2(cscale(nd.g2, -(y + 2.0 * d)))));
  return T;
}

template <int RB>
__global__ void __launch_bounds__(XL_THREADS) k_xu_src(int nq, const XlNode* __restrict__ nodes, int64_t ns,
                                                       const double2* __restrict__ src, double xc, double yif,
                                                       double d, int layers, const double2* __restrict__ q, int nrhs,
                                                       int64_t chunk, double2* __restrict__ part) {
  __shared__ double s_x[XL_THREADS], s_y[XL_THREADS];
  __shared__ double2 s_q[RB][XL_THREADS];
  const int iq = blockIdx.x * XL_THREADS + threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.y * chunk, j1 = min(ns, j0 + chunk);
  const int r0 = blockIdx.z * RB, nr = min(RB, nrhs - r0);
  XlNode nd{};
  if (iq < nq) nd = nodes[iq];
  double2 sp[RB], sm[RB];
  for (int r = 0; r < RB; ++r) sp[r] = sm[r] = cmk(0.0, 0.0);
  for (int64_t b0 = j0; b0 < j1; b0 += XL_THREADS) {
    const int cnt = (int)min((int64_t)XL_THREADS, j1 - b0);
    __syncthreads();
    if (threadIdx.x < cnt) {
      const double2 p = src[b0 + threadIdx.x];
      s_x[threadIdx.x] = p.x - xc;
      s_y[threadIdx.x] = p.y - yif;
      for (int r = 0; r < RB; ++r)
        s_q[r][threadIdx.x] = r < nr ? q[(int64_t)(r0 + r) * ns + b0 + threadIdx.x] : cmk(0.0, 0.0);
    }
    __syncthreads();
    if (iq >= nq) continue;
    for (int j = 0; j < cnt; ++j) {
      const double x = s_x[j];
      const double2 T = xl_lower(nd, s_y[j], d, layers);
      // e^{-+ i lambda x} = e^{+- lambda.y x} (cos(lambda.x x), -+ sin(lambda.x x))
      const double mx = exp(nd.lam.y * x);
      double sn, cs;
      sincos(nd.lam.x * x, &sn, &cs);
      const double2 ep = cmul(T, cmk(mx * cs, -mx * sn)), em = cmul(T, cmk(cs / mx, sn / mx));
      for (int r = 0; r < RB; ++r) {
        const double2 qq = s_q[r][j];
        sp[r] = cadd(sp[r], cmul(qq, ep));
        sm[r] = cadd(sm[r], cmul(qq, em));
      }
    }
  }
  if (iq >= nq) return;
  for (int r = 0; r < nr; ++r) {
    double2* o = part + (((int64_t)blockIdx.y * nrhs + r0 + r) * nq + iq) * 2;
    o[0] = sp[r];
    o[1] = sm[r];
  }
}

template <int RB>
__global__ void __launch_bounds__(XL_THREADS) k_xu_eval(int nq, const XlNode* __restrict__ nodes,
                                                        const double2* __restrict__ S, int nrhs, int64_t nt,
                                                        const double2* __restrict__ tgt, double xc, double yif,
                                                        double2* __restrict__ u) {
  constexpr int NB = XL_THREADS / 4;
  __shared__ double2 s_lam[NB], s_g1[NB];
  __shared__ double2 s_s[RB][NB][2];
  const int64_t it = (int64_t)blockIdx.x * XL_THREADS + threadIdx.x;
  const bool valid = it < nt;
  const int r0 = blockIdx.y * RB, nr = min(RB, nrhs - r0);
  double x = 0.0, y = 1.0;
  if (valid) {
    const double2 p = tgt[it];
    x = p.x - xc;
    y = p.y - yif;
  }
  double2 acc[RB];
  for (int r = 0; r < RB; ++r) acc[r] = cmk(0.0, 0.0);
  for (int q0 = 0; q0 < nq; q0 += NB) {
    const int cnt = min(NB, nq - q0);
    __syncthreads();
    if (threadIdx.x < cnt) {
      s_lam[threadIdx.x] = nodes[q0 + threadIdx.x].lam;
      s_g1[threadIdx.x] = nodes[q0 + threadIdx.x].g1;
    }
    for (int e = threadIdx.x; e < RB * cnt * 2; e += XL_THREADS) {
      const int r = e / (cnt * 2), rem = e - r * cnt * 2, j = rem >> 1, h = rem & 1;
      s_s[r][j][h] = r < nr ? S[((int64_t)(r0 + r) * nq + q0 + j) * 2 + h] : cmk(0.0, 0.0);
    }
    __syncthreads();
    if (!valid) continue;
    for (int j = 0; j < cnt; ++j) {
      const double2 lam = s_lam[j];
      const double2 T = cexp2(cscale(s_g1[j], -y));
      const double mx = exp(-lam.y * x);
      double sn, cs;
      sincos(lam.x * x, &sn, &cs);
      const double2 wp = cmul(T, cmk(mx * cs, mx * sn)), wm = cmul(T, cmk(cs / mx, -sn / mx));
      for (int r = 0; r < RB; ++r) acc[r] = cadd(acc[r], cadd(cmul(s_s[r][j][0], wp), cmul(s_s[r][j][1], wm)));
    }
  }
  if (!valid) return;
  for (int r = 0; r < nr; ++r) u[(int64_t)(r0 + r) * nt + it] = acc[r];
}

// Sources and targets in the middle layer (hfmm_middle_scattered): the
// middle layer's scattered field. With R1 = (g2 - g1)/(g2 + g1), R3 = (g2 -
// g3)/(g2 + g3), E = e^{-g2 d} and D = 1 - R1 R3 E^2 (the waves of a layer-2
// source reflected at the top and at the lower interface, and their repeated
// round trips), a unit source at y0 leaves
//   u = (1/(g2 D)) [R1 e^{g2 y} (e^{g2 y0} + R3 E e^{-g2 (y0 + d)})
//                   + R3 e^{-g2 (y + d)} (e^{-g2 (y0 + d)} + R1 E e^{g2 y0})]
// under (1/4pi) int ... e^{i lambda (x - x0)} d lambda, every factor at most 1
// in modulus for -d < y, y0 < 0. Per node two source sums (the factors
// e^{g2 y_s} and e^{-g2 (y_s + d)}, each with both plane waves) and per target
// u_t = sum_q sum_+- w_+-(x_t) [e^{g2 y} (c1 S1 + c2E S3) + e^{-g2 (y + d)} (c3 S3 + c2E S1)].
struct XmNode {
  double2 lam, g2, c1, c2e, c3;
};

// part[chunk][r][q][4]: S1+, S1-, S3+, S3-
template <int RB>
__global__ void __launch_bounds__(XL_THREADS) k_ml_src(int nq, const XmNode* __restrict__ nodes, int64_t ns,
                                                       const double2* __restrict__ src, double xc, double yif,
                                                       double d, const double2* __restrict__ q, int nrhs,
                                                       int64_t chunk, double2* __restrict__ part) {
  __shared__ double s_x[XL_THREADS], s_y[XL_THREADS];
  __shared__ double2 s_q[RB][XL_THREADS];
  const int iq = blockIdx.x * XL_THREADS + threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.y * chunk, j1 = min(ns, j0 + chunk);
  const int r0 = blockIdx.z * RB, nr = min(RB, nrhs - r0);
  double2 lam = cmk(0.0, 0.0), g2 = cmk(0.0, 0.0);
  if (iq < nq) {
    lam = nodes[iq].lam;
    g2 = nodes[iq].g2;
  }
  double2 acc[RB][4];
  for (int r = 0; r < RB; ++r)
    for (int h = 0; h < 4; ++h) acc[r][h] = cmk(0.0, 0.0);
  for (int64_t b0 = j0; b0 < j1; b0 += XL_THREADS) {
    const int cnt = (int)min((int64_t)XL_THREADS, j1 - b0);
    __syncthreads();
    if (threadIdx.x < cnt) {
      const double2 p = src[b0 + threadIdx.x];
      s_x[threadIdx.x] = p.x - xc;
      s_y[threadIdx.x] = p.y - yif;
      for (int r = 0; r < RB; ++r)
        s_q[r][threadIdx.x] = r < nr ? q[(int64_t)(r0 + r) * ns + b0 + threadIdx.x] : cmk(0.0, 0.0);
    }
    __syncthreads();
    if (iq >= nq) continue;
    if (lam.y == 0.0 && g2.y == 0.0) {
      // a node on the real axis past every branch point: real factors
      for (int j = 0; j < cnt; ++j) {
        const double x = s_x[j], y = s_y[j];
        const double f1 = exp(g2.x * y), f3 = exp(-g2.x * (y + d));
        double sn, cs;
        sincos(lam.x * x, &sn, &cs);
        const double2 t[4] = {cmk(f1 * cs, -f1 * sn), cmk(f1 * cs, f1 * sn), cmk(f3 * cs, -f3 * sn),
                              cmk(f3 * cs, f3 * sn)};
        for (int r = 0; r < RB; ++r) {
          const double2 qq = s_q[r][j];
          for (int h = 0; h < 4; ++h) acc[r][h] = cadd(acc[r][h], cmul(qq, t[h]));
        }
      }
      continue;
    }
    for (int j = 0; j < cnt; ++j) {
      const double x = s_x[j], y = s_y[j];
      const double2 f1 = cexp2(cscale(g2, y)), f3 = cexp2(cscale(g2, -(y + d)));
      // e^{-+ i lambda x} = e^{+- lambda.y x} (cos(lambda.x x), -+ sin(lambda.x x))
      const double mx = exp(lam.y * x);
      double sn, cs;
      sincos(lam.x * x, &sn, &cs);
      const double2 pp = cmk(mx * cs, -mx * sn), pm = cmk(cs / mx, sn / mx);
      const double2 t[4] = {cmul(f1, pp), cmul(f1, pm), cmul(f3, pp), cmul(f3, pm)};
      for (int r = 0; r < RB; ++r) {
        const double2 qq = s_q[r][j];
        for (int h = 0; h < 4; ++h) acc[r][h] = cadd(acc[r][h], cmul(qq, t[h]));
      }
    }
  }
  if (iq >= nq) return;
  for (int r = 0; r < nr; ++r) {
    double2* o = part + (((int64_t)blockIdx.y * nrhs + r0 + r) * nq + iq) * 4;
    for (int h = 0; h < 4; ++h) o[h] = acc[r][h];
  }
}

template <int RB>
__global__ void __launch_bounds__(XL_THREADS) k_ml_eval(int nq, const XmNode* __restrict__ nodes,
                                                        const double2* __restrict__ S, int nrhs, int64_t nt,
                                                        const double2* __restrict__ tgt, double xc, double yif,
                                                        double d, double2* __restrict__ u) {
  constexpr int NB = XL_THREADS / 4;
  __shared__ XmNode s_n[NB];
  __shared__ double2 s_s[RB][NB][4];
  const int64_t it = (int64_t)blockIdx.x * XL_THREADS + threadIdx.x;
  const bool valid = it < nt;
  const int r0 = blockIdx.y * RB, nr = min(RB, nrhs - r0);
  double x = 0.0, y = -0.5 * d;
  if (valid) {
    const double2 p = tgt[it];
    x = p.x - xc;
    y = p.y - yif;
  }
  double2 acc[RB];
  for (int r = 0; r < RB; ++r) acc[r] = cmk(0.0, 0.0);
  for (int q0 = 0; q0 < nq; q0 += NB) {
    const int cnt = min(NB, nq - q0);
    __syncthreads();
    if (threadIdx.x < cnt) s_n[threadIdx.x] = nodes[q0 + threadIdx.x];
    for (int e = threadIdx.x; e < RB * cnt * 4; e += XL_THREADS) {
      const int r = e / (cnt * 4), rem = e - r * cnt * 4, j = rem >> 2, h = rem & 3;
      s_s[r][j][h] = r < nr ? S[((int64_t)(r0 + r) * nq + q0 + j) * 4 + h] : cmk(0.0, 0.0);
    }
    __syncthreads();
    if (!valid) continue;
    for (int j = 0; j < cnt; ++j) {
      const XmNode nd = s_n[j];
      const bool rl = nd.lam.y == 0.0 && nd.g2.y == 0.0;  // real axis past the branch points
      const double2 ta = rl ? cmk(exp(nd.g2.x * y), 0.0) : cexp2(cscale(nd.g2, y));
      const double2 tb = rl ? cmk(exp(-nd.g2.x * (y + d)), 0.0) : cexp2(cscale(nd.g2, -(y + d)));
      const double mx = rl ? 1.0 : exp(-nd.lam.y * x);
      double sn, cs;
      sincos(nd.lam.x * x, &sn, &cs);
      const double2 wp = cmk(mx * cs, mx * sn), wm = cmk(cs / mx, -sn / mx);
      for (int r = 0; r < RB; ++r) {
        const double2 s1p = s_s[r][j][0], s1m = s_s[r][j][1], s3p = s_s[r][j][2], s3m = s_s[r][j][3];
        const double2 xp = cadd(cmul(ta, cadd(cmul(nd.c1, s1p), cmul(nd.c2e, s3p))),
                                cmul(tb, cadd(cmul(nd.c3, s3p), cmul(nd.c2e, s1p))));
        const double2 xm = cadd(cmul(ta, cadd(cmul(nd.c1, s1m), cmul(nd.c2e, s3m))),
                                cmul(tb, cadd(cmul(nd.c3, s3m), cmul(nd.c2e, s1m))));
        acc[r] = cadd(acc[r], cadd(cmul(wp, xp), cmul(wm, xm)));
      }
    }
  }
  if (!valid) return;
  for (int r = 0; r < nr; ++r) u[(int64_t)(r0 + r) * nt + it] = acc[r];
}

// sqrt(lambda^2 - k^2) with Re >= 0 (the principal root; on the half contour
// below the real axis this is the outgoing branch)
cd gam(cd lam, double k) { return std::sqrt(lam * lam - k * k); }

// Panels of the half contour s in [0, send]: lambda(s) = s - i h(s), h = dip
// sin(pi s / L) on [0, L]. Widths: 8 radians of the phase of e^{i lambda x}
// and of the e^{-g y} factors away from the branch points, half the distance
// to each branch point k_j (measured from the dipped contour), half the dip
// over the range of the guided-mode poles; 16 Gauss-Legendre nodes per panel.
struct XlRule {
  std::vector<double> a, b;  // panel ends
  double dip = 0.0, L = 1.0;
  bool ok = true;
};
XlRule xl_rule(const double k[3], int layers, double xspan, double ysum_min, double yrate, double tol) {
  XlRule r;
  const double kmax = std::max({k[0], k[1], layers == 3 ? k[2] : k[1]});
  const double kmin = std::min({k[0], k[1], layers == 3 ? k[2] : k[1]});
  r.L = 1.25 * kmax + 1.0;
  r.dip = std::min(3.0 / std::max(xspan, 1e-9), 0.15 * r.L);
  // beyond L every factor decays at least like e^{-lambda ysum_min}
  const double send = r.L + (std::log(1.0 / tol) + 10.0) / ysum_min;
  // at most 8 radians of phase per 16-node panel (Gauss-Legendre integrates
  // e^{i phi} over 8 radians to about 1e-16)
  const double wcap = std::max(8.0 / (xspan + yrate), 1e-6);
  const double ks[3] = {k[0], k[1], layers == 3 ? k[2] : k[1]};
  auto h_of = [&](double s) { return s < r.L ? r.dip * std::sin(M_PI * s / r.L) : 0.0; };
  auto width = [&](double s) {
    double w = wcap;
    const double h = h_of(s);
    for (double kj : ks) w = std::min(w, 0.5 * std::hypot(s - kj, h));
    if (s > kmin - 1.0 && s < kmax + 1.0) w = std::min(w, 0.5 * std::max(h, 1e-6));
    return std::max(w, 1e-6);
  };
  double s = 0.0;
  for (double stop : {r.L, send}) {
    while (s < stop) {
      double w = width(s);
      w = std::min(w, 1.5 * width(std::min(s + w, stop)));
      double e = std::min(stop, s + w);
      if (stop - e < 1e-3 * w) e = stop;
      r.a.push_back(s);
      r.b.push_back(e);
      s = e;
      if (r.a.size() > kXlMaxPanels) {
        r.ok = false;
        return r;
      }
    }
  }
  return r;
}

// 16-point Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_16)
void gauss16(double* x, double* w) {
  const int n = 16;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int m = 2; m <= n; ++m) {
        const double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace
}  // namespace hfmm

namespace hfmm {
namespace {
// up = false: sources in the top layer, targets below it; up = true: the
// reverse (the transposed node sums).
hfmm_status_t transmit_impl(bool up, int32_t layers, const double* wavenumbers, const double* interfaces, int64_t ns,
                            const double* src, const double* q, int32_t nrhs, int64_t nt, const double* tgt,
                            double* u, double tol, hfmm_stream_t stream) {
  if (!wavenumbers || !interfaces || !src || !q || !tgt || !u)
    return report(HFMM_ERR_INVALID_ARG, "NULL wavenumbers, interfaces, src, q, tgt or u");
  if (layers != 2 && layers != 3)
    return report(HFMM_ERR_UNSUPPORTED, "hfmm_transmit: layers must be 2 or 3 (the impedance half-space has no field below)");
  if (ns < 1 || nt < 1 || ns > ((int64_t)1 << 31) || nt > ((int64_t)1 << 31) || nrhs < 1 || nrhs > 65536)
    return report(HFMM_ERR_INVALID_ARG, "ns, nt or nrhs out of range");
  if (!(tol >= 1e-14 && tol <= 1e-2)) return report(HFMM_ERR_INVALID_ARG, "tol must be in [1e-14, 1e-2]");
  double k[3] = {wavenumbers[0], wavenumbers[1], layers == 3 ? wavenumbers[2] : wavenumbers[1]};
  for (int j = 0; j < layers; ++j)
    if (!(k[j] > 0.0) || !std::isfinite(k[j])) return report(HFMM_ERR_UNSUPPORTED, "wavenumbers must be finite and > 0");
  const double yif = interfaces[0];
  const double d = layers == 3 ? interfaces[0] - interfaces[1] : 1.0;
  if (!std::isfinite(yif) || !(d > 0.0) || !std::isfinite(d))
    return report(HFMM_ERR_INVALID_ARG, "interfaces must be finite and strictly decreasing");
  hipStream_t s = (hipStream_t)stream;
  // the point sets' extents (host copies)
  std::vector<double> hs((size_t)2 * ns), ht((size_t)2 * nt);
  hipError_t e = hipMemcpyAsync(hs.data(), src, sizeof(double) * 2 * ns, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(ht.data(), tgt, sizeof(double) * 2 * nt, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return report(HFMM_ERR_DEVICE, std::string("copying points: ") + hipGetErrorString(e));
  // hs_*: heights of the top-layer set, ht_*: depths of the set below
  double xmin = 1e300, xmax = -1e300, hs_min = 1e300, hs_max = 0.0, ht_min = 1e300, ht_max = 0.0;
  const std::vector<double>& hi = up ? ht : hs;
  const std::vector<double>& lo = up ? hs : ht;
  const char* hi_name = up ? "a target" : "a source";
  const char* lo_name = up ? "a source" : "a target";
  for (int64_t i = 0; i < (up ? nt : ns); ++i) {
    const double x = hi[2 * i], y = hi[2 * i + 1] - yif;
    if (!std::isfinite(x) || !std::isfinite(y)) return report(HFMM_ERR_DOMAIN, "a coordinate is not finite");
    if (!(y > 0.0)) return report(HFMM_ERR_DOMAIN, std::string(hi_name) + " is not above the top interface");
    xmin = std::min(xmin, x);
    xmax = std::max(xmax, x);
    hs_min = std::min(hs_min, y);
    hs_max = std::max(hs_max, y);
  }
  for (int64_t i = 0; i < (up ? ns : nt); ++i) {
    const double x = lo[2 * i], y = lo[2 * i + 1] - yif;
    if (!std::isfinite(x) || !std::isfinite(y)) return report(HFMM_ERR_DOMAIN, "a coordinate is not finite");
    if (!(y < 0.0)) return report(HFMM_ERR_DOMAIN, std::string(lo_name) + " is not below the top interface");
    xmin = std::min(xmin, x);
    xmax = std::max(xmax, x);
    ht_min = std::min(ht_min, -y);
    ht_max = std::max(ht_max, -y);
  }
  const double xc = 0.5 * (xmin + xmax), xspan = xmax - xmin;
  // the slowest decay at large lambda: the nearest point above over the nearest below
  const double ysum_min = hs_min + ht_min;
  // phase rates of the y factors: the heights, and the slab's round trips
  XlRule rule = xl_rule(k, layers, xspan, ysum_min, hs_max + ht_max + (layers == 3 ? 2.0 * d : 0.0), tol);
  if (!rule.ok)
    return report(HFMM_ERR_ACCURACY, "hfmm_transmit: quadrature rule too long (points too close to the interface for their x range)");
  double gx[16], gw[16];
  gauss16(gx, gw);
  std::vector<XlNode> nodes;
  nodes.reserve(rule.a.size() * 16);
  const double inv4pi = 0.25 / M_PI;
  for (size_t p = 0; p < rule.a.size(); ++p) {
    const double hw = 0.5 * (rule.b[p] - rule.a[p]), mid = 0.5 * (rule.a[p] + rule.b[p]);
    for (int g = 0; g < 16; ++g) {
      const double sv = mid + hw * gx[g];
      cd lam(sv, 0.0), dl(1.0, 0.0);
      if (sv < rule.L) {
        lam = cd(sv, -rule.dip * std::sin(M_PI * sv / rule.L));
        dl = cd(1.0, -rule.dip * M_PI / rule.L * std::cos(M_PI * sv / rule.L));
      }
      const cd w = inv4pi * hw * gw[g] * dl;
      const cd g1 = gam(lam, k[0]), g2 = gam(lam, k[1]), g3 = gam(lam, k[2]);
      cd a, b, c;
      if (layers == 2) {
        a = w * 2.0 / (g1 + g2);
        b = 0.0;
        c = 0.0;
      } else {
        const cd E = std::exp(-g2 * d), R = (g2 - g3) / (g2 + g3);
        const cd P = 2.0 / ((g1 + g2) + E * E * R * (g1 - g2));  // sigma_2^+ / g2
        a = w * P;
        b = w * P * R;
        c = w * 2.0 * E * g2 * P / (g2 + g3);
      }
      auto d2 = [](cd v) { return make_double2(v.real(), v.imag()); };
      nodes.push_back(XlNode{d2(lam), d2(g1), d2(g2), d2(g3), d2(a), d2(b), d2(c)});
    }
  }
  const int nq = (int)nodes.size();
  if (const char* env = std::getenv("HFMM_LOG"))
    if (env[0] == '1')
      std::fprintf(stderr, "[hfmm] transmit: %zu panels, %d nodes (x range %.4g, nearest source + target %.4g)\n",
                   rule.a.size(), nq, xspan, ysum_min);
  // source chunks: about 2048 blocks for the node sums
  const int ntile = (nq + XL_THREADS - 1) / XL_THREADS;
  const int64_t maxchunk = (ns + XL_THREADS - 1) / XL_THREADS;
  const int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(maxchunk, 2048 / std::max(ntile, 1)));
  const int64_t chunk = ((ns + nchunk - 1) / nchunk + XL_THREADS - 1) / XL_THREADS * XL_THREADS;
  const int rb = nrhs == 1 ? 1 : XL_RB;  // right-hand sides per block
  const int nrg = (nrhs + rb - 1) / rb;
  DevBuf<XlNode> d_nodes;
  DevBuf<double2> d_part, d_S;
  const int64_t slen = (int64_t)nrhs * nq * 2;
  e = d_nodes.upload(nodes, s);
  if (e == hipSuccess) e = d_part.alloc((size_t)nchunk * slen);
  if (e == hipSuccess) e = d_S.alloc((size_t)slen);
  if (e == hipSuccess) {
    if (up) {
      if (rb == 1)
        hipLaunchKernelGGL(k_xu_src<1>, dim3(ntile, nchunk, nrg), dim3(XL_THREADS), 0, s, nq, d_nodes.p, ns,
                           (const double2*)src, xc, yif, d, (int)layers, (const double2*)q, (int)nrhs, chunk,
                           d_part.p);
      else
        hipLaunchKernelGGL(k_xu_src<XL_RB>, dim3(ntile, nchunk, nrg), dim3(XL_THREADS), 0, s, nq, d_nodes.p, ns,
                           (const double2*)src, xc, yif, d, (int)layers, (const double2*)q, (int)nrhs, chunk,
                           d_part.p);
      hipLaunchKernelGGL(k_xl_sum, dim3((unsigned)((slen + 255) / 256)), dim3(256), 0, s, slen, nchunk, d_part.p,
                         d_S.p);
      const dim3 ge((unsigned)((nt + XL_THREADS - 1) / XL_THREADS), nrg);
      if (rb == 1)
        hipLaunchKernelGGL(k_xu_eval<1>, ge, dim3(XL_THREADS), 0, s, nq, d_nodes.p, d_S.p, (int)nrhs, nt,
                           (const double2*)tgt, xc, yif, (double2*)u);
      else
        hipLaunchKernelGGL(k_xu_eval<XL_RB>, ge, dim3(XL_THREADS), 0, s, nq, d_nodes.p, d_S.p, (int)nrhs, nt,
                           (const double2*)tgt, xc, yif, (double2*)u);
    } else {
      if (rb == 1)
        hipLaunchKernelGGL(k_xl_src<1>, dim3(ntile, nchunk, nrg), dim3(XL_THREADS), 0, s, nq, d_nodes.p, ns,
                           (const double2*)src, xc, yif, (const double2*)q, (int)nrhs, chunk, d_part.p);
      else
        hipLaunchKernelGGL(k_xl_src<XL_RB>, dim3(ntile, nchunk, nrg), dim3(XL_THREADS), 0, s, nq, d_nodes.p, ns,
                           (const double2*)src, xc, yif, (const double2*)q, (int)nrhs, chunk, d_part.p);
      hipLaunchKernelGGL(k_xl_sum, dim3((unsigned)((slen + 255) / 256)), dim3(256), 0, s, slen, nchunk, d_part.p,
                         d_S.p);
      const dim3 ge((unsigned)((nt + XL_THREADS - 1) / XL_THREADS), nrg);
      if (rb == 1)
        hipLaunchKernelGGL(k_xl_eval<1>, ge, dim3(XL_THREADS), 0, s, nq, d_nodes.p, d_S.p, (int)nrhs, nt,
                           (const double2*)tgt, xc, yif, d, (int)layers, (double2*)u);
      else
        hipLaunchKernelGGL(k_xl_eval<XL_RB>, ge, dim3(XL_THREADS), 0, s, nq, d_nodes.p, d_S.p, (int)nrhs, nt,
                           (const double2*)tgt, xc, yif, d, (int)layers, (double2*)u);
    }
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  else (void)hipStreamSynchronize(s);  // nothing of this call is left in flight before its buffers go
  d_nodes.release();
  d_part.release();
  d_S.release();
  if (e != hipSuccess)
    return report(e == hipErrorOutOfMemory ? HFMM_ERR_NO_MEMORY : HFMM_ERR_DEVICE,
                  std::string("hfmm_transmit: ") + hipGetErrorString(e));
  return HFMM_OK;
}
}  // namespace
}  // namespace hfmm

extern "C" hfmm_status_t hfmm_transmit(int32_t layers, const double* wavenumbers, const double* interfaces,
                                       int64_t ns, const double* src, const double* q, int32_t nrhs, int64_t nt,
                                       const double* tgt, double* u, double tol, hfmm_stream_t stream) {
  return hfmm::transmit_impl(false, layers, wavenumbers, interfaces, ns, src, q, nrhs, nt, tgt, u, tol, stream);
}

extern "C" hfmm_status_t hfmm_transmit_up(int32_t layers, const double* wavenumbers, const double* interfaces,
                                          int64_t ns, const double* src, const double* q, int32_t nrhs, int64_t nt,
                                          const double* tgt, double* u, double tol, hfmm_stream_t stream) {
  return hfmm::transmit_impl(true, layers, wavenumbers, interfaces, ns, src, q, nrhs, nt, tgt, u, tol, stream);
}

extern "C" hfmm_status_t hfmm_middle_scattered(const double* wavenumbers, const double* interfaces, int64_t ns,
                                               const double* src, const double* q, int32_t nrhs, int64_t nt,
                                               const double* tgt, double* u, double tol, hfmm_stream_t stream) {
  using namespace hfmm;
  if (!wavenumbers || !interfaces || !src || !q || !tgt || !u)
    return report(HFMM_ERR_INVALID_ARG, "NULL wavenumbers, interfaces, src, q, tgt or u");
  if (ns < 1 || nt < 1 || ns > ((int64_t)1 << 31) || nt > ((int64_t)1 << 31) || nrhs < 1 || nrhs > 65536)
    return report(HFMM_ERR_INVALID_ARG, "ns, nt or nrhs out of range");
  if (!(tol >= 1e-14 && tol <= 1e-2)) return report(HFMM_ERR_INVALID_ARG, "tol must be in [1e-14, 1e-2]");
  const double k[3] = {wavenumbers[0], wavenumbers[1], wavenumbers[2]};
  for (int j = 0; j < 3; ++j)
    if (!(k[j] > 0.0) || !std::isfinite(k[j])) return report(HFMM_ERR_UNSUPPORTED, "wavenumbers must be finite and > 0");
  const double yif = interfaces[0], d = interfaces[0] - interfaces[1];
  if (!std::isfinite(yif) || !(d > 0.0) || !std::isfinite(d))
    return report(HFMM_ERR_INVALID_ARG, "interfaces must be finite and strictly decreasing");
  hipStream_t s = (hipStream_t)stream;
  std::vector<double> hs((size_t)2 * ns), ht((size_t)2 * nt);
  hipError_t e = hipMemcpyAsync(hs.data(), src, sizeof(double) * 2 * ns, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(ht.data(), tgt, sizeof(double) * 2 * nt, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return report(HFMM_ERR_DEVICE, std::string("copying points: ") + hipGetErrorString(e));
  // the nearest approach of any point to either interface
  double xmin = 1e300, xmax = -1e300, hmin = 1e300;
  for (int set = 0; set < 2; ++set) {
    const std::vector<double>& h = set ? ht : hs;
    const int64_t n = set ? nt : ns;
    for (int64_t i = 0; i < n; ++i) {
      const double x = h[2 * i], y = h[2 * i + 1] - yif;
      if (!std::isfinite(x) || !std::isfinite(y)) return report(HFMM_ERR_DOMAIN, "a coordinate is not finite");
      if (!(y < 0.0 && y > -d)) return report(HFMM_ERR_DOMAIN, "a point is not strictly inside the middle layer");
      xmin = std::min(xmin, x);
      xmax = std::max(xmax, x);
      hmin = std::min(hmin, std::min(-y, y + d));
    }
  }
  const double xc = 0.5 * (xmin + xmax), xspan = xmax - xmin;
  // slowest decay: a pair both at the nearest approach of one interface; phase
  // rates up to the longest path (2d plus the layer's height)
  XlRule rule = xl_rule(k, 3, xspan, 2.0 * hmin, 3.0 * d, tol);
  if (!rule.ok)
    return report(HFMM_ERR_ACCURACY, "hfmm_middle_scattered: quadrature rule too long (points too close to an interface for their x range)");
  double gx[16], gw[16];
  gauss16(gx, gw);
  std::vector<XmNode> nodes;
  nodes.reserve(rule.a.size() * 16);
  const double inv4pi = 0.25 / M_PI;
  auto d2 = [](cd v) { return make_double2(v.real(), v.imag()); };
  for (size_t p = 0; p < rule.a.size(); ++p) {
    const double hw = 0.5 * (rule.b[p] - rule.a[p]), mid = 0.5 * (rule.a[p] + rule.b[p]);
    for (int g = 0; g < 16; ++g) {
      const double sv = mid + hw * gx[g];
      cd lam(sv, 0.0), dl(1.0, 0.0);
      if (sv < rule.L) {
        lam = cd(sv, -rule.dip * std::sin(M_PI * sv / rule.L));
        dl = cd(1.0, -rule.dip * M_PI / rule.L * std::cos(M_PI * sv / rule.L));
      }
      const cd w = inv4pi * hw * gw[g] * dl;
      const cd g1 = gam(lam, k[0]), g2 = gam(lam, k[1]), g3 = gam(lam, k[2]);
      const cd E = std::exp(-g2 * d), R1 = (g2 - g1) / (g2 + g1), R3 = (g2 - g3) / (g2 + g3);
      const cd base = w / (g2 * (1.0 - R1 * R3 * E * E));
      nodes.push_back(XmNode{d2(lam), d2(g2), d2(base * R1), d2(base * R1 * R3 * E), d2(base * R3)});
    }
  }
  const int nq = (int)nodes.size();
  if (const char* env = std::getenv("HFMM_LOG"))
    if (env[0] == '1')
      std::fprintf(stderr, "[hfmm] middle layer: %zu panels, %d nodes (x range %.4g, nearest approach %.4g)\n",
                   rule.a.size(), nq, xspan, hmin);
  const int ntile = (nq + XL_THREADS - 1) / XL_THREADS;
  const int64_t maxchunk = (ns + XL_THREADS - 1) / XL_THREADS;
  const int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(maxchunk, 2048 / std::max(ntile, 1)));
  const int64_t chunk = ((ns + nchunk - 1) / nchunk + XL_THREADS - 1) / XL_THREADS * XL_THREADS;
  const int rb = nrhs == 1 ? 1 : XL_RB;
  const int nrg = (nrhs + rb - 1) / rb;
  DevBuf<XmNode> d_nodes;
  DevBuf<double2> d_part, d_S;
  const int64_t slen = (int64_t)nrhs * nq * 4;
  e = d_nodes.upload(nodes, s);
  if (e == hipSuccess) e = d_part.alloc((size_t)nchunk * slen);
  if (e == hipSuccess) e = d_S.alloc((size_t)slen);
  if (e == hipSuccess) {
    const dim3 gs(ntile, nchunk, nrg);
    if (rb == 1)
      hipLaunchKernelGGL(k_ml_src<1>, gs, dim3(XL_THREADS), 0, s, nq, d_nodes.p, ns, (const double2*)src, xc, yif, d,
                         (const double2*)q, (int)nrhs, chunk, d_part.p);
    else
      hipLaunchKernelGGL(k_ml_src<XL_RB>, gs, dim3(XL_THREADS), 0, s, nq, d_nodes.p, ns, (const double2*)src, xc, yif,
                         d, (const double2*)q, (int)nrhs, chunk, d_part.p);
    hipLaunchKernelGGL(k_xl_sum, dim3((unsigned)((slen + 255) / 256)), dim3(256), 0, s, slen, nchunk, d_part.p,
                       d_S.p);
    const dim3 ge((unsigned)((nt + XL_THREADS - 1) / XL_THREADS), nrg);
    if (rb == 1)
      hipLaunchKernelGGL(k_ml_eval<1>, ge, dim3(XL_THREADS), 0, s, nq, d_nodes.p, d_S.p, (int)nrhs, nt,
                         (const double2*)tgt, xc, yif, d, (double2*)u);
    else
      hipLaunchKernelGGL(k_ml_eval<XL_RB>, ge, dim3(XL_THREADS), 0, s, nq, d_nodes.p, d_S.p, (int)nrhs, nt,
                         (const double2*)tgt, xc, yif, d, (double2*)u);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  else (void)hipStreamSynchronize(s);
  d_nodes.release();
  d_part.release();
  d_S.release();
  if (e != hipSuccess)
    return report(e == hipErrorOutOfMemory ? HFMM_ERR_NO_MEMORY : HFMM_ERR_DEVICE,
                  std::string("hfmm_middle_scattered: ") + hipGetErrorString(e));
  return HFMM_OK;
}
