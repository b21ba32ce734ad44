// HIP kernels of the layered-media heterogeneous FMM (gfx950, FP64).
//
// Stages (Algorithm 1 of the paper): P2M at leaves (Eq. multi_coeff), M2M and
// L2L by the free-space Graf translations, M2L with the free-space operator
// (Section 3.3) and with the heterogeneous operator of the scattered field
// (Eq. m2l / m2loperator, sigma_1 of Section 5), L2P, and the local direct
// interactions of image pairs that are not admissible: the Sommerfeld
// integral evaluated by quadrature (Section 5, strategy (b) for the local
// direct interactions). The free-space direct pairs are in p2p.hip.
//
// Every translation operator is a Toeplitz matrix in (m - p); it is stored as
// the vector T[n], n = m - p, and applied as dst[p] += sum_m T[m - p] src[m].
// For the scattered field the source coefficients are the image coefficients
// abar_m = (-1)^m alpha_{-m} (the image of a complex source set; equal to the
// complex conjugate of alpha_m only for real strengths).
#include "kernels.hpp"
#include "special.hpp"

namespace hfmm {

constexpr int WAVE = 64;

__device__ inline double2 shfl_xor_c(double2 v, int mask) {
  return cmk(__shfl_xor(v.x, mask, WAVE), __shfl_xor(v.y, mask, WAVE));
}
__device__ inline double2 wave_sum(double2 v) {
  for (int m = 1; m < WAVE; m <<= 1) v = cadd(v, shfl_xor_c(v, m));
  return v;
}

// ------------------------------------------------------------------ gather / scatter
__global__ void k_gather(int n, int nrhs, const int* __restrict__ perm, const double2* __restrict__ src,
                         double2* __restrict__ dst, int conj_in) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t tot = (int64_t)n * nrhs;
  if (idx >= tot) return;
  int r = (int)(idx / n), i = (int)(idx % n);
  double2 v = src[(int64_t)r * n + perm[i]];
  dst[idx] = conj_in ? cconj(v) : v;
}

// With diag (the self term dropped by HFMM_SELF_NONE): src - diag * qsrc.
__global__ void k_scatter(int n, int nrhs, const int* __restrict__ perm, const double2* __restrict__ src,
                          double2* __restrict__ dst, int conj_out, const double2* __restrict__ diag,
                          const double2* __restrict__ qsrc) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t tot = (int64_t)n * nrhs;
  if (idx >= tot) return;
  int r = (int)(idx / n), i = (int)(idx % n);
  double2 v = src[idx];
  if (diag) v = csub(v, cmul(diag[i], qsrc[idx]));
  dst[(int64_t)r * n + perm[i]] = conj_out ? cconj(v) : v;
}

// Scattered self term of every sorted point from a rule for X = 0:
// G^s(x_i, x_i) = sum_q c_q exp(ky_q Y), Y = 2 y_i (interface frame), and its
// derivative in the source height, sum_q c_q ky_q exp(ky_q Y). The rule's
// nodes are staged through LDS.
constexpr int SELF_THREADS = 256;
__global__ void __launch_bounds__(SELF_THREADS) k_self_term(int n, const double2* __restrict__ pts, int nq,
                                                            const double2* __restrict__ qc,
                                                            const double2* __restrict__ qky,
                                                            double2* __restrict__ g, double2* __restrict__ dy) {
  __shared__ double2 s_c[SELF_THREADS], s_ky[SELF_THREADS];
  const int i = blockIdx.x * SELF_THREADS + threadIdx.x;
  const double Y = i < n ? 2.0 * pts[i].y : 0.0;
  double2 a = cmk(0.0, 0.0), ad = cmk(0.0, 0.0);
  for (int q0 = 0; q0 < nq; q0 += SELF_THREADS) {
    __syncthreads();
    if (q0 + threadIdx.x < nq) {
      s_c[threadIdx.x] = qc[q0 + threadIdx.x];
      s_ky[threadIdx.x] = qky[q0 + threadIdx.x];
    }
    __syncthreads();
    const int m = min(SELF_THREADS, nq - q0);
    for (int t = 0; t < m; ++t) {
      const double2 e = cmul(s_c[t], cexp2(cscale(s_ky[t], Y)));
      a = cadd(a, e);
      ad = cadd(ad, cmul(e, s_ky[t]));
    }
  }
  if (i < n) {
    g[i] = a;
    dy[i] = ad;
  }
}

// HFMM_SELF_NONE: remove the self pair's term from the coordinate gradient,
// gs[j].y -= sum_r Re(q_rj vs_rj dG^s/dY(0, 2 y_j)) (its x derivative is 0).
__global__ void k_self_grad(int n, int nrhs, const double2* __restrict__ dy, const double2* __restrict__ vs,
                            const double2* __restrict__ qs, double2* __restrict__ gs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double sy = 0.0;
  for (int r = 0; r < nrhs; ++r) {
    const int64_t idx = (int64_t)r * n + j;
    sy += cmul(cmul(qs[idx], vs[idx]), dy[j]).x;
  }
  gs[j].y -= sy;
}

// The far-field kernels (P2M first) form a chain of short, latency-bound
// launches that share the GPU with the near field (a stream of its own): their
// waves take the highest issue priority within a SIMD (s_setprio), so that
// the near field's long arithmetic runs fill the cycles they leave.
__device__ inline void far_field_priority() { __builtin_amdgcn_s_setprio(3); }

// ------------------------------------------------------------------ P2M
// alpha_p = sum_j q_j J_p(k rho_j) e^{-i p theta_j}, p in [-P, P] (Eq. multi_coeff).
// One wave per leaf and group of up to RB right-hand sides (grid y; one
// launch for all levels, the order read per leaf), a lane per point. Each lane
// walks the backward Bessel recurrence once and parks V_{n,j} = J_n(k rho_j)
// w_j^n (w = e^{-i theta}) for a chunk of P2M_CH orders in LDS; the chunk is
// then reduced over the points for every right-hand side, giving
// alpha_n = sum q V and, through J_{-n} = (-1)^n J_n,
// alpha_{-n} = (-1)^n sum q conj(V). Both come from the four real sums
// A = sum q.x v.x, B = sum q.y v.y, C = sum q.x v.y, D = sum q.y v.x:
// sum q V = (A - B, C + D), sum q conj(V) = (A + B, D - C). The coefficients
// accumulate in LDS and are stored once. With conj_w the phase is
// e^{+i p theta} and the result is scaled by pref: the transpose of L2P.
constexpr int P2M_CH = 8;   // orders per reduction chunk
constexpr int P2M_RB = 4;   // right-hand sides per pass (several right-hand sides)
constexpr int P2M_VS = WAVE + 1;  // padded row of the V tile
constexpr int P2M_PARTS = WAVE / P2M_CH;  // lanes that share one order in the reduction

template <int RB>
__global__ void __launch_bounds__(WAVE) k_p2m(TreeView tv, const int* __restrict__ leaves, int nleaves,
                                              const double2* __restrict__ qs, double2* __restrict__ alpha,
                                              int conj_w, double2 pref) {
  extern __shared__ double2 lds_c[];
  double2* s_V = lds_c;                     // [P2M_CH][P2M_VS]
  double2* s_q = s_V + P2M_CH * P2M_VS;     // [RB][WAVE]
  double2* s_a = s_q + RB * WAVE;           // [RB][2P + 1]
  const int li = blockIdx.x;
  if (li >= nleaves) return;
  far_field_priority();
  const int b = leaves[li];
  const int lane = threadIdx.x;
  const int P = tv.P[tv.level[b]];
  const int M = 2 * P + 1;
  const int2 pr = tv.prange[b];
  const double2 c = tv.ctr[b];
  const int64_t cb = tv.coff[b];
  // a bound on k*rho for the whole box gives one recurrence length per wave
  double rmax = 0.0;
  for (int j = pr.x + lane; j < pr.y; j += WAVE) {
    double2 p = tv.pts[j];
    rmax = fmax(rmax, hypot(p.x - c.x, p.y - c.y));
  }
  for (int m = 1; m < WAVE; m <<= 1) rmax = fmax(rmax, __shfl_xor(rmax, m, WAVE));
  const int nstart = miller_start_expansion(tv.k * rmax, P);
  // reduction role of this lane: order slot t of the chunk, point block part
  const int t_red = lane & (P2M_CH - 1), part = lane / P2M_CH;
  const int r0 = blockIdx.y * RB;  // right-hand sides r0 .. r0 + nr - 1
  const int nr = min(RB, tv.nrhs - r0);
  for (int e = lane; e < nr * M; e += WAVE) s_a[e] = cmk(0.0, 0.0);
  for (int j0 = pr.x; j0 < pr.y; j0 += WAVE) {
    const int j = j0 + lane;
    const bool valid = j < pr.y;
    double dx = 0, dy = 0;
    if (valid) {
      double2 p = tv.pts[j];
      dx = p.x - c.x;
      dy = p.y - c.y;
    }
#pragma unroll
    for (int rr = 0; rr < RB; ++rr)
      if (rr < nr) s_q[rr * WAVE + lane] = valid ? qs[(int64_t)(r0 + rr) * tv.n + j] : cmk(0.0, 0.0);
    const double rho = hypot(dx, dy);
    const double x = fmax(tv.k * rho, kTinyX), s1 = tv.k * rho < kTinyX ? tv.k * rho / kTinyX : 1.0;
    const double2 w = rho > 0 ? cmk(dx / rho, (conj_w ? dy : -dy) / rho) : cmk(1.0, 0.0);
    double2 wn = cpowi(w, P);
    double inv_s;
    int nres;
    miller_norm(x, nstart, inv_s, nres);
    MillerWalk mw(x, nstart, inv_s, nres);
    while (mw.n > P) mw.step();
    for (int nh = P; nh >= 0; nh -= P2M_CH) {
#pragma unroll
      for (int t = 0; t < P2M_CH; ++t) {
        if (nh - t >= 0) {
          const double jv = nh - t == 1 ? s1 * mw.value() : mw.value();
          s_V[t * P2M_VS + lane] = cscale(wn, valid ? jv : 0.0);
          wn = cmul(wn, cconj(w));
          if (mw.n > 0) mw.step();
        }
      }
      __syncthreads();
      const int n = nh - t_red;
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        if (rr >= nr) break;
        double A = 0.0, B = 0.0, C = 0.0, D = 0.0;
        if (n >= 0) {
          const double2* V = s_V + t_red * P2M_VS + part * (WAVE / P2M_PARTS);
          const double2* Q = s_q + rr * WAVE + part * (WAVE / P2M_PARTS);
#pragma unroll
          for (int i = 0; i < WAVE / P2M_PARTS; ++i) {
            const double2 v = V[i], q = Q[i];
            A = fma(q.x, v.x, A);
            B = fma(q.y, v.y, B);
            C = fma(q.x, v.y, C);
            D = fma(q.y, v.x, D);
          }
        }
#pragma unroll
        for (int m = P2M_CH; m < WAVE; m <<= 1) {
          A += __shfl_xor(A, m, WAVE);
          B += __shfl_xor(B, m, WAVE);
          C += __shfl_xor(C, m, WAVE);
          D += __shfl_xor(D, m, WAVE);
        }
        if (part == 0 && n >= 0) {
          double2* a = s_a + rr * M + P;
          a[n] = cadd(a[n], cmul(pref, cmk(A - B, C + D)));
          if (n > 0) {
            const double2 sm = cmk(A + B, D - C);
            a[-n] = cadd(a[-n], cmul(pref, (n & 1) ? cscale(sm, -1.0) : sm));
          }
        }
      }
      __syncthreads();
    }
  }
  for (int e = lane; e < nr * M; e += WAVE) {
    const int rr = e / M;
    alpha[(int64_t)(r0 + rr) * tv.ctot + cb + (e - rr * M)] = s_a[e];
  }
}

size_t p2m_lds_bytes(int Pmax, int rb) {
  return sizeof(double2) * (size_t)(P2M_CH * P2M_VS + rb * WAVE + rb * (2 * Pmax + 1));
}

// ------------------------------------------------------------------ L2P
// u_i (+)= pref * sum_p beta_p J_p(k r_i) e^{i p theta_i} (local expansion,
// Section 3.2). One wave per leaf and group of up to RB right-hand sides
// (grid y), a lane per point; one recurrence walk serves the whole group.
// With w = e^{i theta}, a_n = beta_n and b_n = (-1)^n beta_{-n}, the orders
// +n and -n together give J_n (a_n w^n + b_n conj(w^n)); with
// s = a + b, d = a - b and (J_n w^n) = (c, e) this is
// (s.x c - d.y e, d.x e + s.y c), four multiply-adds per order. The group's
// s_n and d_n (b_0 = 0) are staged in LDS. With conj_w the phase is
// e^{-i p theta_i}: the transpose of P2M, used by the adjoint.
constexpr int L2P_RB = 4;

template <int RB>
__global__ void __launch_bounds__(WAVE) k_l2p(TreeView tv, const int* __restrict__ leaves, int nleaves,
                                              const double2* __restrict__ beta, double2* __restrict__ us,
                                              int conj_w, double2 pref, int accumulate) {
  extern __shared__ double2 lds_c[];  // [RB][P + 1][s, d]
  const int li = blockIdx.x;
  if (li >= nleaves) return;
  far_field_priority();
  const int b = leaves[li];
  const int lane = threadIdx.x;
  const int lev = tv.level[b];
  const bool has_local = lev >= 2;
  const int P = tv.P[lev];
  const int2 pr = tv.prange[b];
  const double2 c = tv.ctr[b];
  const int64_t cb = tv.coff[b];
  const int r0 = blockIdx.y * RB;  // right-hand sides r0 .. r0 + nr - 1
  const int nr = min(RB, tv.nrhs - r0);
  int nstart = 0;
  if (has_local) {
    double rmax = 0.0;
    for (int j = pr.x + lane; j < pr.y; j += WAVE) {
      double2 p = tv.pts[j];
      rmax = fmax(rmax, hypot(p.x - c.x, p.y - c.y));
    }
    for (int m = 1; m < WAVE; m <<= 1) rmax = fmax(rmax, __shfl_xor(rmax, m, WAVE));
    nstart = miller_start_expansion(tv.k * rmax, P);
    for (int e = lane; e < nr * (P + 1); e += WAVE) {
      const int rr = e / (P + 1), n = e - rr * (P + 1);
      const double2* bt = beta + (int64_t)(r0 + rr) * tv.ctot + cb + P;
      const double2 an = bt[n];
      double2 bn = n > 0 ? bt[-n] : cmk(0.0, 0.0);
      if (n & 1) bn = cscale(bn, -1.0);
      lds_c[2 * e] = cadd(an, bn);
      lds_c[2 * e + 1] = csub(an, bn);
    }
    __syncthreads();
  }
  for (int j = pr.x + lane; j < pr.y; j += WAVE) {
    double2 acc[RB];
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) acc[rr] = cmk(0.0, 0.0);
    if (has_local) {
      const double2 p = tv.pts[j];
      const double dx = p.x - c.x, dy = p.y - c.y;
      const double rho = hypot(dx, dy);
      const double x = fmax(tv.k * rho, kTinyX), s1 = tv.k * rho < kTinyX ? tv.k * rho / kTinyX : 1.0;
      const double2 w = rho > 0 ? cmk(dx / rho, (conj_w ? -dy : dy) / rho) : cmk(1.0, 0.0);
      double2 wn = cpowi(w, P);
      double inv_s;
      int nres;
      miller_norm(x, nstart, inv_s, nres);
      MillerWalk mw(x, nstart, inv_s, nres);
      while (mw.n > P) mw.step();
      for (int n = P; n >= 0; --n) {
        const double2 jw = cscale(wn, n == 1 ? s1 * mw.value() : mw.value());
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
          if (rr < nr) {
            const double2 sn = lds_c[2 * (rr * (P + 1) + n)], dn = lds_c[2 * (rr * (P + 1) + n) + 1];
            acc[rr].x = fma(sn.x, jw.x, fma(-dn.y, jw.y, acc[rr].x));
            acc[rr].y = fma(dn.x, jw.y, fma(sn.y, jw.x, acc[rr].y));
          }
        }
        wn = cmul(wn, cconj(w));
        if (n > 0) mw.step();
      }
    }
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      if (rr < nr) {
        const int64_t idx = (int64_t)(r0 + rr) * tv.n + j;
        const double2 v = cmul(pref, acc[rr]);
        if (accumulate == 2) {
          unsafeAtomicAdd(&us[idx].x, v.x);
          unsafeAtomicAdd(&us[idx].y, v.y);
        } else {
          us[idx] = accumulate ? cadd(us[idx], v) : v;
        }
      }
    }
  }
}

size_t l2p_lds_bytes(int Pmax, int rb) { return sizeof(double2) * (size_t)(rb * 2 * (Pmax + 1)); }

// The same sum for one right-hand side with a lane per point of the sorted
// order: a wave takes 64 consecutive points, which lie in a few leaves (runs
// of equal box[j]; leaves average about 35 points, so a wave per leaf leaves
// about half its lanes idle). The runs' s_n and d_n are staged in LDS,
// L2P_RUNS runs at a time, and each lane walks the recurrence for its own
// argument and order.
constexpr int L2P_RUNS = 4;
__global__ void __launch_bounds__(WAVE) k_l2p_flat(TreeView tv, const int* __restrict__ pt_box, int Pmax,
                                                   const double2* __restrict__ beta, double2* __restrict__ us,
                                                   int conj_w, double2 pref, int accumulate) {
  extern __shared__ double2 lds_c[];  // [L2P_RUNS][Pmax + 1][s, d]
  far_field_priority();
  const int lane = threadIdx.x;
  const int j = blockIdx.x * WAVE + lane;
  const bool valid = j < tv.n;
  const int b = valid ? pt_box[j] : -1;
  const int b_prev = __shfl_up(b, 1, WAVE);
  const uint64_t runs = __ballot(valid && (lane == 0 || b != b_prev));
  const int nruns = __popcll(runs);
  // this lane's run: the run heads at or below it, less one
  const int my_run = valid ? __popcll(runs & (~0ull >> (63 - lane))) - 1 : -1;
  const int lev = valid ? tv.level[b] : 0;
  const bool has_local = valid && lev >= 2;
  const int P = has_local ? tv.P[lev] : 0;
  double2 acc = cmk(0.0, 0.0);
  uint64_t heads = runs;
  for (int g0 = 0; g0 < nruns; g0 += L2P_RUNS) {
    // stage the coefficients of runs g0 .. g0 + L2P_RUNS - 1 (the wave's
    // lanes together, one run after another)
    for (int r = 0; r < L2P_RUNS && g0 + r < nruns; ++r) {
      const int head = __ffsll((long long)heads) - 1;
      heads &= heads - 1;
      const int br = __shfl(b, head, WAVE);
      const int lr = tv.level[br];
      if (lr < 2) continue;
      const int Pr = tv.P[lr];
      const double2* bt = beta + tv.coff[br] + Pr;
      for (int n = lane; n <= Pr; n += WAVE) {
        const double2 an = bt[n];
        double2 bn = n > 0 ? bt[-n] : cmk(0.0, 0.0);
        if (n & 1) bn = cscale(bn, -1.0);
        lds_c[2 * (r * (Pmax + 1) + n)] = cadd(an, bn);
        lds_c[2 * (r * (Pmax + 1) + n) + 1] = csub(an, bn);
      }
    }
    __syncthreads();
    if (has_local && my_run >= g0 && my_run < g0 + L2P_RUNS) {
      const double2* sd = lds_c + 2 * (my_run - g0) * (Pmax + 1);
      const double2 p = tv.pts[j], c = tv.ctr[b];
      const double dx = p.x - c.x, dy = p.y - c.y;
      const double rho = hypot(dx, dy);
      const double x = fmax(tv.k * rho, kTinyX), s1 = tv.k * rho < kTinyX ? tv.k * rho / kTinyX : 1.0;
      const double2 w = rho > 0 ? cmk(dx / rho, (conj_w ? -dy : dy) / rho) : cmk(1.0, 0.0);
      double2 wn = cpowi(w, P);
      const int nstart = miller_start_expansion(tv.k * rho, P);
      double inv_s;
      int nres;
      miller_norm(x, nstart, inv_s, nres);
      MillerWalk mw(x, nstart, inv_s, nres);
      while (mw.n > P) mw.step();
      for (int n = P; n >= 0; --n) {
        const double2 jw = cscale(wn, n == 1 ? s1 * mw.value() : mw.value());
        const double2 sn = sd[2 * n], dn = sd[2 * n + 1];
        acc.x = fma(sn.x, jw.x, fma(-dn.y, jw.y, acc.x));
        acc.y = fma(dn.x, jw.y, fma(sn.y, jw.x, acc.y));
        wn = cmul(wn, cconj(w));
        if (n > 0) mw.step();
      }
    }
    __syncthreads();
  }
  if (!valid) return;
  const double2 v = cmul(pref, acc);
  if (accumulate == 2) {
    unsafeAtomicAdd(&us[j].x, v.x);
    unsafeAtomicAdd(&us[j].y, v.y);
  } else {
    us[j] = accumulate ? cadd(us[j], v) : v;
  }
}

// ------------------------------------------------------------------ batched translations on MFMA
// For one table t (t[n], n = m - p, m in [-Ps, Ps] source orders, p in
// [-Pd, Pd] target orders) and a batch of (source, target) box pairs using it:
//   out_c[p] = sum_m t[m - p] S_c[m]        (REV: t[p - m], the transpose)
// computed as a real GEMM through the 2x2 embedding of complex numbers,
//   [Re out; Im out] = [[Tr, -Ti], [Ti, Tr]] [Re S; Im S],
// with 16x16x4 FP64 MFMA tiles: rows = 2 Md in tiles of 16, k = 2 Ms in steps
// of 4, columns = 16 pairs per wave. Operator tiles are expanded from the
// Toeplitz vector in LDS on the fly. Image pairs use the reflected source
// coefficients abar_m = (-1)^m alpha_{-m}; in the transpose the reflection
// moves to the output. Three output modes:
//  * contribution rows (M2L): each pair writes its own row, reduced per box
//    afterwards;
//  * exclusive (parent to child): every target box of the launch receives
//    exactly one pair and the result is added with a read-modify-write;
//  * four-quadrant gather (child to parent): the 16 columns are parents and
//    the contraction runs over the four child quadrants in turn, each with its
//    table, so that k spans the stacked children; a missing child is a zero
//    column. Each parent receives its whole sum at once and is stored;
//  * split four-quadrant gather (child to parent, launches too small to fill
//    the GPU): an item is one row tile, and wave q contracts child quadrant q
//    with its own table and source tile, all four staged at once; the four
//    partial tiles are added through LDS and stored. Each SIMD's MFMA chain
//    is a quarter of the in-turn form's, and the four rounds of loads are one.
// This one kernel runs M2L (free and heterogeneous), M2M, L2L and their
// transposes.
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int TR_THREADS = 256;

enum { OUT_GATHER4 = 0, OUT_CONTRIB = 1, OUT_EXCLUSIVE = 2, OUT_GATHER4_SPLIT = 3 };

// LDS layout of an item: the table as three zero-padded vectors Tr, Ti, -Ti of
// trans_table_stride(nt) doubles each (value n at index kTabPad + n), then the
// source coefficients, one row of Ms4 = Ms rounded up to 4 per pair (zeros
// past Ms), so that the real and the imaginary halves of the contraction
// index k each fill whole 4-deep MFMA steps.
constexpr int kTabPad = 4;
__host__ __device__ inline int trans_table_stride(int nt) { return (nt + 2 * kTabPad + 1) & ~1; }
__host__ __device__ inline int round4(int m) { return (m + 3) & ~3; }

// The contraction of one wave: NT row tiles of 16 rows of the real-embedded
// operator against one 16-column tile of pairs, added into acc. Row r of the
// operator is (rim, p) = (r >= Md, r mod Md), column k = (kim, m) with the
// halves padded to Ms4; its entry is Tr, Ti or -Ti at table index 2Pd - p + m
// (forward) or p + 2Ps - m (transpose). Each lane holds one address per row
// tile and half, so every operand element is one LDS read and the k-loop has
// no branches.
template <bool REV, int NT>
__device__ inline void trans_contract(d4* acc, const double* lds_d, int ntp, const double2* s_s, int Ps, int Pd,
                                      int rt_lo, int rt_stride) {
  const int Ms4 = round4(2 * Ps + 1), Md = 2 * Pd + 1;
  const int lane = threadIdx.x & 63, lrow = lane & 15, lk = lane >> 4;
  int a_re[NT], a_im[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int row = (rt_lo + j * rt_stride) * 16 + lrow;
    const bool ok = row < 2 * Md;  // rows past the operator compute garbage that is never stored
    const bool rim = ok && row >= Md;
    const int p = ok ? (rim ? row - Md : row) : 0;
    const int tb = kTabPad + (REV ? p + 2 * Ps : 2 * Pd - p) + (REV ? -lk : lk);
    a_re[j] = (rim ? ntp : 0) + tb;      // Tr (rim == kim) or Ti
    a_im[j] = (rim ? 0 : 2 * ntp) + tb;  // Tr or -Ti
  }
  const double* Bcol = (const double*)(s_s + lrow * Ms4) + 2 * lk;
  const int nks = Ms4 / 4;
  // real half of k, then the imaginary half
#pragma unroll 2
  for (int ks = 0; ks < nks; ++ks) {
    const int kk = REV ? -4 * ks : 4 * ks;
    const double b = Bcol[8 * ks];
    double a[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) a[j] = lds_d[a_re[j] + kk];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j], b, acc[j], 0, 0, 0);
  }
#pragma unroll 2
  for (int ks = 0; ks < nks; ++ks) {
    const int kk = REV ? -4 * ks : 4 * ks;
    const double b = Bcol[8 * ks + 1];
    double a[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) a[j] = lds_d[a_im[j] + kk];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j], b, acc[j], 0, 0, 0);
  }
}

// Output slot of operator row `row` for this lane's column: D[row][col] of a
// 16x16x4 FP64 tile sits in lane col + 16 (row % 4), register row / 4. False
// past the operator's rows; idx is the double within the target's
// coefficients (real and imaginary parts interleaved) or, for a contribution
// row, within the row (real parts, then imaginary parts); neg is the sign of
// the output reflection.
template <bool CONTRIB>
__device__ inline bool trans_slot(int row, int Md, int Pd, bool reflect_out, int& idx, bool& neg) {
  if (row >= 2 * Md) return false;
  const bool rim = row >= Md;
  const int p = rim ? row - Md : row;
  int po = p;
  neg = false;
  if (reflect_out) {
    po = Md - 1 - p;
    neg = ((p + Pd) & 1) != 0;
  }
  idx = CONTRIB ? (rim ? Md : 0) + po : 2 * po + (rim ? 1 : 0);
  return true;
}

// Store (contribution rows, gathered parents) or add (exclusive targets: old
// holds their values read before the contraction when PREFETCH, else they are
// read here).
template <int MODE, bool PREFETCH, int NT>
__device__ inline void trans_store(const d4* acc, const double* old, double* outd, int rt_lo, int rt_stride, int Md,
                                   int Pd, bool reflect_out) {
  const int lk = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int idx;
      bool neg;
      const int row = (rt_lo + j * rt_stride) * 16 + 4 * i + lk;
      if (!trans_slot<MODE == OUT_CONTRIB>(row, Md, Pd, reflect_out, idx, neg)) continue;
      const double v = neg ? -acc[j][i] : acc[j][i];
      if (MODE != OUT_EXCLUSIVE)
        outd[idx] = v;
      else
        outd[idx] = (PREFETCH ? old[4 * j + i] : outd[idx]) + v;
    }
  }
}

// NTMAX bounds the row tiles per wave of the launch: the register allocation
// is that of the largest instantiated case, so launches with few row tiles use
// a variant with NTMAX = 2 and more waves fit a SIMD.
template <bool REV, int MODE, int NTMAX>
__global__ void __launch_bounds__(TR_THREADS) k_trans_mfma(TreeView tv, const TransItem* __restrict__ items,
                                                          const int64_t* __restrict__ soff,
                                                          const int64_t* __restrict__ doff,
                                                          const int64_t* __restrict__ pcoff, Toff4 q4,
                                                          const double2* __restrict__ tdata,
                                                          const double2* __restrict__ src, double2* __restrict__ dst,
                                                          double* __restrict__ contrib, int64_t cstride) {
  extern __shared__ double lds_d[];
  __shared__ int64_t s_off[64];
  far_field_priority();
  constexpr bool G4 = MODE == OUT_GATHER4;
  constexpr bool GS = MODE == OUT_GATHER4_SPLIT;  // quadrant per wave
  constexpr bool CONTRIB = MODE == OUT_CONTRIB;
  const int r = blockIdx.y;  // right-hand side
  const TransItem it = items[blockIdx.x];
  const int Ps = it.Ps, Pd = it.Pd;
  const int Ms = 2 * Ps + 1, Ms4 = round4(Ms), Md = 2 * Pd + 1;
  const int nt = 2 * (Ps + Pd) + 1;  // table length
  const int ntp = trans_table_stride(nt);
  const int nrt = (2 * Md + 15) / 16;
  const int npi = trans_pairs_per_item(Ps, Pd);
  // split gather: the four quadrants' tables, then their source tiles
  double2* s_s = (double2*)(lds_d + (GS ? 4 : 1) * 3 * ntp);  // 16-byte aligned: ntp is even
  const int tid = threadIdx.x, wave = tid >> 6;
  // wave -> row tiles: the four waves split up to 4 it.ntw row tiles of the
  // item's column tile with stride 4 (split gather: all take tile rt_base)
  const int rt_lo = it.rt_base + (GS ? 0 : wave), rt_stride = 4;
  const int rt_cnt = rt_lo < nrt ? (GS ? 1 : min((nrt - rt_lo + 3) / 4, it.ntw)) : 0;
  // this lane's column (pair) and output; exclusive targets are read now, so
  // that the read overlaps the contraction
  const int lane = tid & 63, lk = lane >> 4;
  const int col = lane & 15;
  const bool col_ok = col < it.npairs;
  const int pair = it.pbeg + (col_ok ? col : 0);
  const bool reflect_out = REV && it.image;
  double* outd = CONTRIB ? contrib + (int64_t)r * cstride + pcoff[pair]
                         : (double*)(dst + (int64_t)r * tv.ctot + doff[pair]);
  constexpr bool PREFETCH = MODE == OUT_EXCLUSIVE && NTMAX <= 2;
  double old[PREFETCH ? 4 * NTMAX : 1];
  if (PREFETCH) {
#pragma unroll
    for (int j = 0; j < (PREFETCH ? NTMAX : 1); ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int idx;
        bool neg;
        const int row = (rt_lo + j * rt_stride) * 16 + 4 * i + lk;
        old[4 * j + i] =
            (j < rt_cnt && col_ok && trans_slot<false>(row, Md, Pd, reflect_out, idx, neg)) ? outd[idx] : 0.0;
      }
  }
  d4 acc[NTMAX];
#pragma unroll
  for (int j = 0; j < NTMAX; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
  const bool reflect_in = it.image && !REV;
  const double2* Sr = src + (int64_t)r * tv.ctot;
  const int tot = (GS ? 4 : 1) * npi * Ms4;
#pragma unroll 1
  for (int ph = 0; ph < (G4 ? 4 : 1); ++ph) {
    if (ph > 0) __syncthreads();  // the previous quadrant's operands are no longer read
    // Every global load of the prologue is issued in one of two rounds: the
    // pairs' coefficient offsets and the table first, then all source rows.
    if (GS) {  // s_off[q npi + c]: quadrant q of parent c
      if (tid < 4 * npi) {
        const int q = tid / npi, c = tid - q * npi;
        s_off[tid] = c < it.npairs ? soff[4 * (it.pbeg + c) + q] : -1;
      }
    } else if (tid < npi) {
      s_off[tid] = tid < it.npairs ? soff[G4 ? 4 * (it.pbeg + tid) + ph : it.pbeg + tid] : -1;
    }
    for (int i = tid; i < (GS ? 4 : 1) * ntp; i += TR_THREADS) {
      const int q = GS ? i / ntp : 0, j = i - q * ntp;
      // T[0] = t[-(Ps + Pd)]
      const double2* T = tdata + (it.toff >= 0 ? it.toff : q4.v[GS ? q : G4 ? ph : (it.table & 3)]);
      const int n = j - kTabPad;
      const double2 v = (n >= 0 && n < nt) ? T[n] : cmk(0.0, 0.0);
      double* L = lds_d + 3 * ntp * q;
      L[j] = v.x;
      L[ntp + j] = v.y;
      L[2 * ntp + j] = -v.y;
    }
    __syncthreads();
    // source coefficients, flattened (pair, order) so consecutive lanes read
    // consecutive coefficients of a row; four loads in flight per lane
    for (int e0 = tid; e0 < tot; e0 += 4 * TR_THREADS) {
      double2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * TR_THREADS;
        v[u] = cmk(0.0, 0.0);
        if (e < tot) {
          const int c = e / Ms4, m = e - c * Ms4;
          const int64_t off = s_off[c];
          if (off >= 0 && m < Ms) {
            if (reflect_in) {
              v[u] = Sr[off + Ms - 1 - m];
              if ((m + Ps) & 1) v[u] = cscale(v[u], -1.0);
            } else {
              v[u] = Sr[off + m];
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u * TR_THREADS < tot) s_s[e0 + u * TR_THREADS] = v[u];
    }
    __syncthreads();
    if (GS) {
      if (rt_cnt > 0)
        trans_contract<REV, 1>(acc, lds_d + 3 * ntp * wave, ntp, s_s + npi * Ms4 * wave, Ps, Pd, rt_lo, rt_stride);
    } else if (rt_cnt > 0) {
      if (NTMAX <= 2) {
        if (rt_cnt == 1)
          trans_contract<REV, 1>(acc, lds_d, ntp, s_s, Ps, Pd, rt_lo, rt_stride);
        else
          trans_contract<REV, (NTMAX < 2 ? NTMAX : 2)>(acc, lds_d, ntp, s_s, Ps, Pd, rt_lo, rt_stride);
      } else {
#define HFMM_CONTRACT(N) \
  case N: trans_contract<REV, N>(acc, lds_d, ntp, s_s, Ps, Pd, rt_lo, rt_stride); break;
        switch (rt_cnt) {
          HFMM_CONTRACT(1) HFMM_CONTRACT(2) HFMM_CONTRACT(3) HFMM_CONTRACT(4) HFMM_CONTRACT(5) HFMM_CONTRACT(6)
          HFMM_CONTRACT(7)
          default: trans_contract<REV, NTMAX>(acc, lds_d, ntp, s_s, Ps, Pd, rt_lo, rt_stride);
        }
#undef HFMM_CONTRACT
      }
    }
  }
  if (GS) {  // add the four quadrants' tiles (every wave has the same rt_cnt)
    if (rt_cnt <= 0) return;
    __syncthreads();  // the source tiles are no longer read
    double* red = (double*)s_s;  // [wave][4][64]
#pragma unroll
    for (int i = 0; i < 4; ++i) red[(wave * 4 + i) * 64 + lane] = acc[0][i];
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      acc[0][i] = (red[i * 64 + lane] + red[(4 + i) * 64 + lane]) + (red[(8 + i) * 64 + lane] + red[(12 + i) * 64 + lane]);
  }
  if (rt_cnt <= 0 || !col_ok) return;
  if (NTMAX <= 2) {
    if (rt_cnt == 1)
      trans_store<MODE, PREFETCH, 1>(acc, old, outd, rt_lo, rt_stride, Md, Pd, reflect_out);
    else
      trans_store<MODE, PREFETCH, (NTMAX < 2 ? NTMAX : 2)>(acc, old, outd, rt_lo, rt_stride, Md, Pd, reflect_out);
  } else {
#define HFMM_STORE(N) \
  case N: trans_store<MODE, PREFETCH, N>(acc, old, outd, rt_lo, rt_stride, Md, Pd, reflect_out); break;
    switch (rt_cnt) {
      HFMM_STORE(1) HFMM_STORE(2) HFMM_STORE(3) HFMM_STORE(4) HFMM_STORE(5) HFMM_STORE(6) HFMM_STORE(7)
      default: trans_store<MODE, PREFETCH, NTMAX>(acc, old, outd, rt_lo, rt_stride, Md, Pd, reflect_out);
    }
#undef HFMM_STORE
  }
}
// beta_b = sum of the contribution rows of box b, plain store. The box's
// ptr[wi + 1] - ptr[wi] rows lie one after another from beg[wi] (each 2M
// doubles: the real parts, then the imaginary parts). One block per box and
// right-hand side (grid y), a thread per double of the row; four partial sums
// keep several loads in flight.
constexpr int RED_THREADS = 128;
__global__ void __launch_bounds__(RED_THREADS) k_reduce_contrib(TreeView tv, const int* __restrict__ boxes, int nb,
                                                                const int* __restrict__ ptr,
                                                                const int64_t* __restrict__ beg,
                                                                const double* __restrict__ contrib, int64_t cstride,
                                                                double2* __restrict__ dst) {
  const int wi = blockIdx.x;
  if (wi >= nb) return;
  far_field_priority();
  const int b = boxes[wi];
  const int M = 2 * tv.P[tv.level[b]] + 1, W = 2 * M;
  const int cnt = ptr[wi + 1] - ptr[wi];
  const int r = blockIdx.y;
  const double* rows = contrib + (int64_t)r * cstride + beg[wi];
  double* out = (double*)(dst + (int64_t)r * tv.ctot + tv.coff[b]);
  for (int t = threadIdx.x; t < W; t += RED_THREADS) {
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    int e = 0;
    for (; e + 4 <= cnt; e += 4) {
      v0 += rows[(int64_t)e * W + t];
      v1 += rows[(int64_t)(e + 1) * W + t];
      v2 += rows[(int64_t)(e + 2) * W + t];
      v3 += rows[(int64_t)(e + 3) * W + t];
    }
    for (; e < cnt; ++e) v0 += rows[(int64_t)e * W + t];
    out[t < M ? 2 * t : 2 * (t - M) + 1] = (v0 + v1) + (v2 + v3);
  }
}

__global__ void k_fill_zero(double2* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = cmk(0.0, 0.0);
}

// ------------------------------------------------------------------ source-coordinate gradient
// The gradient of L = Re sum_i conj(v_i) (A q)_i with respect to the source
// coordinates x_j, targets held fixed: g_j = Re(q_j sum_i vs_i dA_ij/dx_j)
// with vs = conj(v). The transposed pipeline has left alpha', the adjoint
// multipole coefficients of every box, so at a leaf the far field seen by a
// source is w_j = sum_p alpha'_p f_p(x_j), f_p = J_p(k rho) e^{-i p theta}.
// The ladder relations of the cylindrical waves (from J_p' and
// (p/x) J_p = (J_{p-1} + J_{p+1})/2) give
//   d f_p/dx = (k/2)(f_{p-1} - f_{p+1}),  d f_p/dy = -(ik/2)(f_{p-1} + f_{p+1}),
// so dw/dx = sum_m (k/2)(a_{m+1} - a_{m-1}) f_m and
//    dw/dy = -(ik/2) sum_m (a_{m+1} + a_{m-1}) f_m,  m in [-P-1, P+1].
// gs[j] = (sum_r Re(q_rj dw_r/dx), sum_r Re(q_rj dw_r/dy)), stored (first
// writer, or added with add); leaves without a local expansion store zero.
__global__ void __launch_bounds__(WAVE) k_l2p_grad(TreeView tv, const int* __restrict__ leaves, int nleaves, int rb,
                                                   const double2* __restrict__ alpha, const double2* __restrict__ qs,
                                                   double2* __restrict__ gs, int add) {
  extern __shared__ double2 lds_c[];  // [rb][2P + 5]: a_m at P + 2 + m, zero for |m| > P
  const int li = blockIdx.x;
  if (li >= nleaves) return;
  const int b = leaves[li];
  const int lane = threadIdx.x;
  const int lev = tv.level[b];
  const bool has_local = lev >= 2;
  const int P = tv.P[lev], Pg = P + 1, S = 2 * P + 5;
  const int2 pr = tv.prange[b];
  const double2 c = tv.ctr[b];
  const int64_t cb = tv.coff[b];
  const double hk = 0.5 * tv.k;
  int nstart = 0;
  if (has_local) {
    double rmax = 0.0;
    for (int j = pr.x + lane; j < pr.y; j += WAVE) {
      double2 p = tv.pts[j];
      rmax = fmax(rmax, hypot(p.x - c.x, p.y - c.y));
    }
    for (int m = 1; m < WAVE; m <<= 1) rmax = fmax(rmax, __shfl_xor(rmax, m, WAVE));
    nstart = miller_start_expansion(tv.k * rmax, Pg);
  }
  for (int r0 = 0; r0 < tv.nrhs; r0 += rb) {
    const int nr = min(rb, tv.nrhs - r0);
    if (has_local) {
      for (int e = lane; e < nr * S; e += WAVE) {
        const int rr = e / S, m = e - rr * S - (P + 2);
        lds_c[e] = (m >= -P && m <= P) ? alpha[(int64_t)(r0 + rr) * tv.ctot + cb + P + m] : cmk(0.0, 0.0);
      }
      __syncthreads();
    }
    for (int j = pr.x + lane; j < pr.y; j += WAVE) {
      double sx = 0.0, sy = 0.0;
      if (has_local) {
        double2 gx[L2P_RB], gy[L2P_RB];
#pragma unroll
        for (int rr = 0; rr < L2P_RB; ++rr) gx[rr] = gy[rr] = cmk(0.0, 0.0);
        const double2 p = tv.pts[j];
        const double dx = p.x - c.x, dy = p.y - c.y;
        const double rho = hypot(dx, dy);
        const double x = fmax(tv.k * rho, kTinyX), s1 = tv.k * rho < kTinyX ? tv.k * rho / kTinyX : 1.0;
        const double2 w = rho > 0 ? cmk(dx / rho, -dy / rho) : cmk(1, 0);  // e^{-i theta}
        double2 wn = cpowi(w, Pg);
        double inv_s;
        int nres;
        miller_norm(x, nstart, inv_s, nres);
        MillerWalk mw(x, nstart, inv_s, nres);
        while (mw.n > Pg) mw.step();
        for (int n = Pg; n >= 0; --n) {
          const double jn = n == 1 ? s1 * mw.value() : mw.value();
          const double2 wc = cconj(wn);
#pragma unroll
          for (int rr = 0; rr < L2P_RB; ++rr) {
            if (rr < nr) {
              const double2* a = lds_c + rr * S + P + 2;
              // ladder coefficients at +n and -n
              const double2 dxp = cscale(csub(a[n + 1], a[n - 1]), hk);
              const double2 syp = cadd(a[n + 1], a[n - 1]);
              const double2 dyp = cmk(hk * syp.y, -hk * syp.x);  // -(ik/2) syp
              double2 tx = cmul(dxp, wn), ty = cmul(dyp, wn);
              if (n > 0) {
                const double2 dxm = cscale(csub(a[-n + 1], a[-n - 1]), hk);
                const double2 sym = cadd(a[-n + 1], a[-n - 1]);
                const double2 dym = cmk(hk * sym.y, -hk * sym.x);
                const double2 ux = cmul(dxm, wc), uy = cmul(dym, wc);
                tx = (n & 1) ? csub(tx, ux) : cadd(tx, ux);
                ty = (n & 1) ? csub(ty, uy) : cadd(ty, uy);
              }
              gx[rr] = cadd(gx[rr], cscale(tx, jn));
              gy[rr] = cadd(gy[rr], cscale(ty, jn));
            }
          }
          wn = cmul(wn, cconj(w));
          if (n > 0) mw.step();
        }
#pragma unroll
        for (int rr = 0; rr < L2P_RB; ++rr) {
          if (rr < nr) {
            const double2 q = qs[(int64_t)(r0 + rr) * tv.n + j];
            sx += cmul(q, gx[rr]).x;
            sy += cmul(q, gy[rr]).x;
          }
        }
      }
      if (r0 == 0 && !add)
        gs[j] = cmk(sx, sy);
      else
        gs[j] = cadd(gs[j], cmk(sx, sy));
    }
    if (has_local) __syncthreads();
  }
}

size_t l2p_grad_lds_bytes(int Pmax, int rb) { return sizeof(double2) * (size_t)(rb * (2 * Pmax + 5)); }

// Gradient of the free-space direct part, on the direct work items. With
// g(r) = d/dr (i/4) H_0^(1)(k r) / r = -(i/4) k H_1^(1)(k r) / r, a pair (i, j)
// adds Re(g sum_r vs_ri q_rj) (x_j - x_i) to the source j (summed in LDS per
// staged chunk and flushed atomically) and, in a cross item, where the pair
// stands for both orders, Re(g sum_r vs_rj q_ri) (x_i - x_j) to i.
constexpr int GRAD_CS = 64;

// H1^(1)(x) / x from z = x^2/4 within a series class: the series of M terms
// (the class's H0 term count; the H1 coefficients fall faster, and at each
// class's largest argument the truncation stays below 2e-18 relative) with
// the logarithm from the LDS table. J1/x = (1/2) sum a_m z^m and
// Y1/x = (2/pi)((ln z / 2 + gamma) J1/x - 1/(4z)) - (1/(2 pi)) sum b_m z^m need
// no square root; LARGE: the large-argument form above x = 6 (z > 9).
template <int M, bool LARGE>
__device__ inline double2 hankel1_over_x_class(double z, double inv_z, const double2* ltab) {
  if (LARGE && z > 9.0) {
    const double x = 2.0 * sqrt(z);
    const double2 h = hankel1_large(x);
    const double ix = 1.0 / x;
    return cmk(h.x * ix, h.y * ix);
  }
  double sa = kH1.a[M - 1], sb = kH1.b[M - 1];
#pragma unroll
  for (int m = M - 2; m >= 0; --m) {
    sa = fma(sa, z, kH1.a[m]);
    sb = fma(sb, z, kH1.b[m]);
  }
  const double jx = 0.5 * sa;
  const double two_over_pi = 0.63661977236758134308;
  const double euler = 0.57721566490153286061;
  const double yx =
      two_over_pi * ((0.5 * log_tab(z, ltab) + euler) * jx - 0.25 * inv_z) - (0.5 / 3.14159265358979323846) * sb;
  return cmk(jx, yx);
}

// ONE: a single right-hand side, whose v_i and q_i stay in registers and
// whose sources' q_j and v_j are staged in LDS with their positions (the
// general form reads them from memory for every pair and right-hand side).
// One launch per series class, as for the near field itself.
template <bool ONE, int CLS>
__global__ void __launch_bounds__(WAVE) k_p2p_grad(TreeView tv, const int* __restrict__ leaves, int nitems,
                                                   const int* __restrict__ ptr, const int2* __restrict__ rng,
                                                   const int* __restrict__ sym, const double2* __restrict__ vs,
                                                   const double2* __restrict__ qs, double2* __restrict__ gs) {
  constexpr int M = kH0ClassTerms[CLS < kH0Classes ? CLS : kH0Classes - 1];
  constexpr bool LARGE = CLS >= kH0Classes;
  __shared__ double2 s_x[GRAD_CS];
  __shared__ double2 s_g[GRAD_CS];
  __shared__ double2 s_qj[ONE ? GRAD_CS : 1];
  __shared__ double2 s_vj[ONE ? GRAD_CS : 1];
  __shared__ double2 s_ln[1 << kLogTabBits];
  for (int l = threadIdx.x; l < (1 << kLogTabBits); l += WAVE) s_ln[l] = cmk(kLogTab[l][0], kLogTab[l][1]);
  __syncthreads();
  const int li = blockIdx.x;
  if (li >= nitems) return;
  const int b = leaves[li];
  const bool both = sym[li] != 0;
  const int lane = threadIdx.x;
  const int2 pr = tv.prange[b];
  const int nrhs = tv.nrhs;
  const double qk2 = 0.25 * tv.k * tv.k, kk4 = 0.25 * tv.k * tv.k;
  // targets in chunks of 32 with two lanes each, the remainder in a chunk of
  // the next power of two with more lanes per target; the g lanes of a
  // target take every g-th source of a staged chunk
  for (int c0 = pr.x, csz = 0; c0 < pr.y; c0 += csz) {
    const int rem = pr.y - c0;
    csz = 32;
    if (rem < 32) {
      csz = 1;
      while (csz < rem) csz *= 2;
    }
    const int g = WAVE / csz;
    const int ti = lane / g, sub = lane % g;
    const int i = c0 + ti;
    const bool valid = ti < min(csz, rem);
    const double2 xi = valid ? tv.pts[i] : cmk(0, 0);
    const double2 vi = (ONE && valid) ? vs[i] : cmk(0, 0), qi = (ONE && valid) ? qs[i] : cmk(0, 0);
    double gix = 0.0, giy = 0.0;
    for (int e = ptr[li]; e < ptr[li + 1]; ++e) {
      const int2 sr = rng[e];
      for (int j0 = sr.x; j0 < sr.y; j0 += GRAD_CS) {
        const int cnt = min(GRAD_CS, sr.y - j0);
        __syncthreads();
        if (lane < cnt) {
          s_x[lane] = tv.pts[j0 + lane];
          s_g[lane] = cmk(0.0, 0.0);
          if (ONE) {
            s_qj[lane] = qs[j0 + lane];
            s_vj[lane] = both ? vs[j0 + lane] : cmk(0.0, 0.0);
          }
        }
        __syncthreads();
        const int K = (cnt - sub + g - 1) / g;  // this lane's sources: sub + g k, k < K
        if (valid && K > 0) {
          // targets start at different sources, so the LDS adds seldom
          // collide; four pairs at a time give the series chains room to overlap
          const int r0 = ti % K;
          for (int t0 = 0; t0 < K; t0 += 4) {
            int jl[4];
            bool use[4];
            double dx[4], dy[4], z[4], inv_z[4];
            double2 hx[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int k = t0 + u;
              int kr = k + r0;
              if (kr >= K) kr -= K;
              jl[u] = sub + g * (k < K ? kr : 0);
              use[u] = k < K && j0 + jl[u] != i;
              const double2 xj = s_x[jl[u]];
              dx[u] = xj.x - xi.x;
              dy[u] = xj.y - xi.y;
              z[u] = use[u] ? qk2 * (dx[u] * dx[u] + dy[u] * dy[u]) : 1.0;
              inv_z[u] = 1.0 / z[u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) hx[u] = hankel1_over_x_class<M, LARGE>(z[u], inv_z[u], s_ln);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if (!use[u]) continue;
              // -(i/4) k H1(k r) / r = -(i/4) k^2 H1(x) / x
              const double2 gg = cmk(kk4 * hx[u].y, -kk4 * hx[u].x);
              double2 cij = cmk(0.0, 0.0), cji = cmk(0.0, 0.0);
              if (ONE) {
                cij = cmul(vi, s_qj[jl[u]]);
                if (both) cji = cmul(s_vj[jl[u]], qi);
              } else {
                const int j = j0 + jl[u];
                for (int rr = 0; rr < nrhs; ++rr) {
                  const int64_t o = (int64_t)rr * tv.n;
                  cij = cadd(cij, cmul(vs[o + i], qs[o + j]));
                  if (both) cji = cadd(cji, cmul(vs[o + j], qs[o + i]));
                }
              }
              const double sj = cmul(gg, cij).x;
              atomicAdd(&s_g[jl[u]].x, sj * dx[u]);
              atomicAdd(&s_g[jl[u]].y, sj * dy[u]);
              if (both) {
                const double si = cmul(gg, cji).x;
                gix -= si * dx[u];
                giy -= si * dy[u];
              }
            }
          }
        }
        __syncthreads();
        if (lane < cnt) {
          unsafeAtomicAdd(&gs[j0 + lane].x, s_g[lane].x);
          unsafeAtomicAdd(&gs[j0 + lane].y, s_g[lane].y);
        }
      }
    }
    // the target's sums over its g lanes (neighbouring lanes)
    for (int m = 1; m < g; m <<= 1) {
      gix += __shfl_xor(gix, m, WAVE);
      giy += __shfl_xor(giy, m, WAVE);
    }
    if (valid && both && sub == 0) {
      unsafeAtomicAdd(&gs[i].x, gix);
      unsafeAtomicAdd(&gs[i].y, giy);
    }
  }
}

// ------------------------------------------------------------------ near-interface direct
// u_i += sum_j q_j G^s(x_i, x_j) for image pairs that are not admissible, with
// G^s = sum_q c_q exp(ky_q (y_i + y_j) + kx_q (x_i - x_j)) the Sommerfeld
// integral under one fixed rule (the propagating tau part and the evanescent t
// part on a contour below the real-axis singularities). Every node term
// factors through box centres, kx (x_i - x_j) = kx (x_i - x_t) + kx (x_t -
// x_s) + kx (x_s - x_j), so the pairs go in three stages:
//   k_if_src    S_q(s) = sum_{j in s} q_j exp(ky_q y_j - kx_q (x_j - x_s)),
//               once per source box;
//   k_if_trans  T_q(t) = c_q sum_s S_q(s) exp(kx_q (x_t - x_s)) over the source
//               boxes of target leaf t;
//   k_if_eval   u_i += sum_q T_q(t) exp(ky_q y_i + kx_q (x_i - x_t)) for the
//               points of t.
// Every factor stays bounded: Re(ky) <= 0 above the interface, and the x
// offsets are at most the rule's x separation. The right-hand sides go in
// groups of up to kIfRhs (one exponential serves the whole group); element r
// of point j sits at j * ps + r * rs.

// S for the source boxes: grid (nsb, nqp / 64), four waves split the points
// of a box, lane = node
__global__ void __launch_bounds__(256) k_if_src(TreeView tv, const int* __restrict__ sbox, int nq, int nqp, int rif,
                                                const double2* __restrict__ qky, const double2* __restrict__ qkx,
                                                const double2* __restrict__ qs, int64_t ps, int64_t rs, int nr,
                                                double2* __restrict__ S) {
  __shared__ double2 s_red[3][kIfRhs][WAVE];
  const int slot = blockIdx.x, lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int q = blockIdx.y * WAVE + lane;
  const int b = sbox[slot];
  const int2 pr = tv.prange[b];
  const double xs = tv.ctr[b].x;
  double2 ky = cmk(0, 0), kx = cmk(0, 0);
  if (q < nq) {
    ky = qky[q];
    kx = qkx[q];
  }
  double2 acc[kIfRhs];
#pragma unroll
  for (int r = 0; r < kIfRhs; ++r) acc[r] = cmk(0, 0);
  for (int j = pr.x + w; j < pr.y; j += 4) {
    const double2 xj = tv.pts[j];
    const double2 e = cexp2(cadd(cscale(ky, xj.y), cscale(kx, xs - xj.x)));
    const double2* qj = qs + (int64_t)j * ps;
#pragma unroll
    for (int r = 0; r < kIfRhs; ++r)
      if (r < nr) acc[r] = cadd(acc[r], cmul(qj[r * rs], e));
  }
  if (w > 0)
#pragma unroll
    for (int r = 0; r < kIfRhs; ++r)
      if (r < nr) s_red[w - 1][r][lane] = acc[r];
  __syncthreads();
  if (w == 0)
#pragma unroll
    for (int r = 0; r < kIfRhs; ++r)
      if (r < nr) {
        double2 v = cadd(cadd(acc[r], s_red[0][r][lane]), cadd(s_red[1][r][lane], s_red[2][r][lane]));
        S[((int64_t)slot * rif + r) * nqp + q] = q < nq ? v : cmk(0, 0);
      }
}

// T for the target leaves: grid (ntl, nqp / 64), lane = node
__global__ void __launch_bounds__(WAVE) k_if_trans(TreeView tv, const int* __restrict__ tleaf,
                                                   const int* __restrict__ tptr, const int* __restrict__ tsrc,
                                                   const int* __restrict__ sbox, int nq, int nqp, int rif,
                                                   const double2* __restrict__ qc, const double2* __restrict__ qkx,
                                                   const double2* __restrict__ S, int nr, double2* __restrict__ T) {
  const int t = blockIdx.x, lane = threadIdx.x;
  const int q = blockIdx.y * WAVE + lane;
  const double xt = tv.ctr[tleaf[t]].x;
  double2 kx = cmk(0, 0), c = cmk(0, 0);
  if (q < nq) {
    kx = qkx[q];
    c = qc[q];
  }
  double2 acc[kIfRhs];
#pragma unroll
  for (int r = 0; r < kIfRhs; ++r) acc[r] = cmk(0, 0);
  for (int e = tptr[t]; e < tptr[t + 1]; ++e) {
    const int sl = tsrc[e];
    const double2 f = cexp2(cscale(kx, xt - tv.ctr[sbox[sl]].x));
    const double2* Ss = S + (int64_t)sl * rif * nqp + q;
#pragma unroll
    for (int r = 0; r < kIfRhs; ++r)
      if (r < nr) acc[r] = cadd(acc[r], cmul(Ss[(int64_t)r * nqp], f));
  }
#pragma unroll
  for (int r = 0; r < kIfRhs; ++r)
    if (r < nr) T[((int64_t)t * rif + r) * nqp + q] = cmul(c, acc[r]);
}

// Evaluation at the points of the target leaves: a block per (leaf, range
// of nodes), four waves taking every fourth 64-node chunk of the range. A
// chunk of nt <= 64 target points occupies the lanes of a wave floor(64 / nt)
// times over (lane groups), the groups taking every G-th node; the groups'
// and waves' sums meet in LDS in a fixed order. With one range per leaf
// (gridDim.y = 1) and atomic = 0 each point has one writer. GRAD: the
// coordinate gradient of the adjoint (T from the adjoint vector, see
// launch_iface_grad) instead of u.
template <bool GRAD>
__global__ void __launch_bounds__(4 * WAVE) k_if_eval(TreeView tv, const int* __restrict__ tleaf, int nq, int nqp,
                                                      int rif, const double2* __restrict__ qky,
                                                      const double2* __restrict__ qkx, const double2* __restrict__ T,
                                                      int nr, const double2* __restrict__ qg, double2* __restrict__ us,
                                                      int64_t ps, int64_t rs, int atomic) {
  __shared__ double2 s_red[4][kIfRhs][WAVE];
  const int t = blockIdx.x, lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int b = tleaf[t];
  const int2 pr = tv.prange[b];
  const double xt = tv.ctr[b].x;
  const double2* Tt = T + (int64_t)t * rif * nqp;
  const int nch = nqp / WAVE;
  const int cb = (int)((int64_t)blockIdx.y * nch / gridDim.y), ce = (int)((int64_t)(blockIdx.y + 1) * nch / gridDim.y);
  for (int c0 = pr.x; c0 < pr.y; c0 += WAVE) {
    const int nt = min(WAVE, pr.y - c0), G = WAVE / nt;
    const int g = lane / nt, il = lane - g * nt;
    const bool act = g < G;
    const int i = c0 + il;
    const double2 xi = act ? tv.pts[i] : cmk(xt, 0.0);
    double2 acc[kIfRhs], accy[kIfRhs];
#pragma unroll
    for (int r = 0; r < kIfRhs; ++r) acc[r] = accy[r] = cmk(0, 0);
    if (act)
      for (int ch = cb + w; ch < ce; ch += 4) {
        const int q1 = min(nq, (ch + 1) * WAVE);
        for (int q = ch * WAVE + g; q < q1; q += G) {
          const double2 ky = qky[q], kx = qkx[q];
          const double2 e = cexp2(cadd(cscale(ky, xi.y), cscale(kx, xi.x - xt)));
#pragma unroll
          for (int r = 0; r < kIfRhs; ++r)
            if (r < nr) {
              const double2 v = cmul(Tt[(int64_t)r * nqp + q], e);
              if (GRAD) {
                acc[r] = cadd(acc[r], cmul(kx, v));
                accy[r] = cadd(accy[r], cmul(ky, v));
              } else {
                acc[r] = cadd(acc[r], v);
              }
            }
        }
      }
    // groups and waves in a fixed order (GRAD: sum_r Re(q_ri (d/dx, d/dy)) first)
    __syncthreads();
    if (GRAD) {
      double sx = 0.0, sy = 0.0;
      if (act)
#pragma unroll
        for (int r = 0; r < kIfRhs; ++r)
          if (r < nr) {
            const double2 q = qg[(int64_t)i * ps + r * rs];
            sx += cmul(q, acc[r]).x;
            sy += cmul(q, accy[r]).x;
          }
      s_red[w][0][lane] = cmk(sx, sy);
    } else {
#pragma unroll
      for (int r = 0; r < kIfRhs; ++r)
        if (r < nr) s_red[w][r][lane] = acc[r];
    }
    __syncthreads();
    if (w == 0 && lane < nt) {
      const int nrr = GRAD ? 1 : nr;
      for (int r = 0; r < nrr; ++r) {
        double2 a = cmk(0, 0);
        for (int ww = 0; ww < 4; ++ww)
          for (int gg = 0; gg < G; ++gg) a = cadd(a, s_red[ww][r][gg * nt + lane]);
        double2* ui = GRAD ? us + i : us + (int64_t)i * ps + r * rs;
        if (atomic) {  // other writers of us may run at the same time
          unsafeAtomicAdd(&ui->x, a.x);
          unsafeAtomicAdd(&ui->y, a.y);
        } else {
          *ui = cadd(*ui, a);
        }
      }
    }
  }
}

// Horizontally separated near-interface pairs by interpolation: G^s depends
// only on (|X|, Y), X = x_i - x_j, Y = y_i + y_j, and is analytic away from
// X = +-iY, so on pairs with |X| >= X0 >= Y it is a tensor Chebyshev series
// of kIfTP x kIfTP terms per panel (panels graded geometrically from X0 and
// at most a fraction of the shortest wavelength wide). The panel values come
// from the Sommerfeld rule once per plan (k_if_grid); the series coefficients
// from the host.

// G, dG/d|X| and dG/dY at npts points (|X|, Y) from one rule: three planes of
// npts values
__global__ void __launch_bounds__(WAVE) k_if_grid(int npts, const double2* __restrict__ xy, int nq,
                                                  const double2* __restrict__ qc, const double2* __restrict__ qky,
                                                  const double2* __restrict__ qkx, double2* __restrict__ out) {
  __shared__ double2 s_c[WAVE], s_ky[WAVE], s_kx[WAVE];
  const int lane = threadIdx.x;
  const int i = blockIdx.x * WAVE + lane;
  const double2 p = i < npts ? xy[i] : cmk(0.0, 0.0);
  double2 g = cmk(0, 0), gx = cmk(0, 0), gy = cmk(0, 0);
  for (int q0 = 0; q0 < nq; q0 += WAVE) {
    __syncthreads();
    const bool qv = q0 + lane < nq;
    s_c[lane] = qv ? qc[q0 + lane] : cmk(0, 0);
    s_ky[lane] = qv ? qky[q0 + lane] : cmk(0, 0);
    s_kx[lane] = qv ? qkx[q0 + lane] : cmk(0, 0);
    __syncthreads();
    const int qn = min(WAVE, nq - q0);
    for (int qq = 0; qq < qn; ++qq) {
      const double2 v = cmul(s_c[qq], cexp2(cadd(cscale(s_ky[qq], p.y), cscale(s_kx[qq], p.x))));
      g = cadd(g, v);
      gx = cadd(gx, cmul(s_kx[qq], v));
      gy = cadd(gy, cmul(s_ky[qq], v));
    }
  }
  if (i < npts) {
    out[i] = g;
    out[(int64_t)npts + i] = gx;
    out[2 * (int64_t)npts + i] = gy;
  }
}

// the series of one panel at local coordinates (u, v): sum_{a + b < P} c_ab
// T_a(u) T_b(v), the coefficients packed row by row (kIfTri of them). Only the
// terms with a + b < P enter: the coefficients of a function analytic in a
// polyellipse fall off like rho_x^-a rho_y^-b, so the dropped ones are each
// below the truncation level the panels are sized for (tol / 100).
template <typename P>
__device__ inline double2 cheb2(P c, const double* tu, const double* tv) {
  double2 acc = cmk(0, 0);
  int k = 0;
#pragma unroll
  for (int a = 0; a < kIfTP; ++a) {
    double2 row = cmk(0, 0);
#pragma unroll
    for (int b = 0; b < kIfTP - a; ++b, ++k) {
      const double2 cab = c[k];
      row.x = fma(cab.x, tv[b], row.x);
      row.y = fma(cab.y, tv[b], row.y);
    }
    acc.x = fma(row.x, tu[a], acc.x);
    acc.y = fma(row.y, tu[a], acc.y);
  }
  return acc;
}

// LDS written by some lanes of a wave and read by others: order the two
// within the wave (no block barrier: the waves of a block run different
// loops here)
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Table pairs of the target leaves: a block per work item (a leaf and up to
// four of its source boxes), or per leaf without items; wave w takes every
// fourth source box. A chunk of nt <= 64 target points occupies the lanes
// floor(64 / nt) times over (lane groups), the groups taking every G-th
// source point, so that every lane works on small leaves too; the groups'
// and waves' sums meet in LDS in a fixed order. GRAD: the coordinate
// gradient (sources vs, owner strengths qg; X = owner - source, d/dx =
// sign(X) dG/d|X|, d/dy = dG/dY).
template <bool GRAD>
__global__ void __launch_bounds__(4 * WAVE) k_if_table(TreeView tv, IfTable tb,
                                                       const double2* __restrict__ coef, int nr,
                                                       const double2* __restrict__ qs,
                                                       const double2* __restrict__ qg, double2* __restrict__ us,
                                                       int64_t ps, int64_t rs, int atomic) {
  __shared__ double2 s_red[4][kIfRhs][WAVE];
  __shared__ double2 s_cf[4][2 * kIfTri];  // per wave: the panel in use (one or two series)
  constexpr int NF = GRAD ? 2 : 1;
  int staged = -1;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int t = tb.item_t ? tb.item_t[blockIdx.x] : blockIdx.x;
  const int b = tb.tleaf[t];
  const int2 pr = tv.prange[b];
  const int e0 = tb.item_t ? tb.item_e[blockIdx.x].x : tb.tptr[t];
  const int e1 = tb.item_t ? tb.item_e[blockIdx.x].y : tb.tptr[t + 1];
  for (int c0 = pr.x; c0 < pr.y; c0 += WAVE) {
    const int nt = min(WAVE, pr.y - c0), G = WAVE / nt;
    const int g = lane / nt, il = lane - g * nt;
    const bool act = g < G;
    const int i = c0 + il;
    const double2 xi = tv.pts[act ? i : c0];
    double2 acc[kIfRhs], accy[kIfRhs];
#pragma unroll
    for (int r = 0; r < kIfRhs; ++r) acc[r] = accy[r] = cmk(0, 0);
    for (int e = e0 + w; e < e1; e += 4) {
      const int2 sr = tv.prange[tb.tsrc[e]];
      // every lane runs every step (the LDS staging below needs the whole
      // wave); lanes past the box's end add nothing
      for (int jj = sr.x; jj < sr.y; jj += G) {
        const int j = jj + g;
        const bool ok = act && j < sr.y;
        const double2 xj = tv.pts[ok ? j : sr.x];
        const double X = xi.x - xj.x, ax = fabs(X), Y = xi.y + xj.y;
        // panel of |X| (the index in single precision: a point a rounding off
        // the panel edge evaluates the neighbour's series a hair outside
        // [-1, 1], where it is just as accurate)
        const int pg = (int)floorf(__log2f(fmaxf((float)(ax * tb.inv_x0), 1.0f)) * tb.inv_lg2);
        const int pu = tb.p1 + (int)floorf((float)((ax - tb.a1) * tb.inv_wmax));
        const int px = min(max(ax < tb.a1 ? pg : pu, 0), tb.npx - 1);
        const double4 xw = tb.xpan[px];  // left edge, 1 / width; Y panel width, 1 / width
        const int2 yw = tb.ypan[px];     // Y panels: count, first
        const int py = min(max((int)floorf((float)((Y - tb.ylo) * xw.w)), 0), yw.x - 1);
        const double u = (2.0 * (ax - xw.x)) * xw.y - 1.0;
        const double v = (2.0 * (Y - tb.ylo - py * xw.z)) * xw.w - 1.0;
        double tu[kIfTP], tvv[kIfTP];
        tu[0] = 1.0;
        tu[1] = u;
        tvv[0] = 1.0;
        tvv[1] = v;
#pragma unroll
        for (int a = 2; a < kIfTP; ++a) {
          tu[a] = 2.0 * u * tu[a - 1] - tu[a - 2];
          tvv[a] = 2.0 * v * tvv[a - 1] - tvv[a - 2];
        }
        // a panel shared by the whole wave (the usual case: a leaf is
        // narrower than a panel) is staged in LDS and read as broadcasts;
        // lanes in different panels read their own from memory
        const int pp = yw.y + py;
        const int p0 = __builtin_amdgcn_readfirstlane(pp);
        const bool uni = __all(pp == p0);
        const double2* cs;
        if (uni) {
          if (p0 != staged) {
            const double2* src = coef + ((int64_t)p0 * 3 + (GRAD ? 1 : 0)) * kIfTri;
            wave_lds_sync();
            for (int l = lane; l < NF * kIfTri; l += WAVE) s_cf[w][l] = src[l];
            wave_lds_sync();
            staged = p0;
          }
          cs = &s_cf[w][0];
        } else {
          cs = coef + ((int64_t)pp * 3 + (GRAD ? 1 : 0)) * kIfTri;
        }
        if (!ok) continue;
        const double2* qj = qs + (int64_t)j * ps;
        if (GRAD) {
          double2 gx = cheb2(cs, tu, tvv);
          const double2 gy = cheb2(cs + kIfTri, tu, tvv);
          if (X < 0.0) gx = cscale(gx, -1.0);
#pragma unroll
          for (int r = 0; r < kIfRhs; ++r)
            if (r < nr) {
              const double2 q = qj[r * rs];
              acc[r] = cadd(acc[r], cmul(gx, q));
              accy[r] = cadd(accy[r], cmul(gy, q));
            }
        } else {
          const double2 gv = cheb2(cs, tu, tvv);
#pragma unroll
          for (int r = 0; r < kIfRhs; ++r)
            if (r < nr) acc[r] = cadd(acc[r], cmul(gv, qj[r * rs]));
        }
      }
    }
    // groups and waves in a fixed order (GRAD: sum_r Re(q_ri (d/dx, d/dy)) first)
    __syncthreads();
    if (GRAD) {
      double sx = 0.0, sy = 0.0;
      if (act)
#pragma unroll
        for (int r = 0; r < kIfRhs; ++r)
          if (r < nr) {
            const double2 q = qg[(int64_t)i * ps + r * rs];
            sx += cmul(q, acc[r]).x;
            sy += cmul(q, accy[r]).x;
          }
      s_red[w][0][lane] = cmk(sx, sy);
    } else {
#pragma unroll
      for (int r = 0; r < kIfRhs; ++r)
        if (r < nr) s_red[w][r][lane] = acc[r];
    }
    __syncthreads();
    if (w == 0 && lane < nt) {
      const int nrr = GRAD ? 1 : nr;
      for (int r = 0; r < nrr; ++r) {
        double2 a = cmk(0, 0);
        for (int ww = 0; ww < 4; ++ww)
          for (int gg = 0; gg < G; ++gg) a = cadd(a, s_red[ww][r][gg * nt + lane]);
        double2* ui = GRAD ? us + i : us + (int64_t)i * ps + r * rs;
        if (atomic) {
          unsafeAtomicAdd(&ui->x, a.x);
          unsafeAtomicAdd(&ui->y, a.y);
        } else {
          *ui = cadd(*ui, a);
        }
      }
    }
  }
}

__global__ void k_scatter_grad(int n, const int* __restrict__ perm, const double2* __restrict__ gs,
                               double2* __restrict__ grad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  grad[perm[i]] = gs[i];
}

// ------------------------------------------------------------------ tables
// Free-space M2L: T[n] = H_n(k rho) e^{i n theta}, n in [-half, half]
// (Section 3.3); (rho, theta) polar form of (target centre - source centre).
__global__ void k_table_hankel(int ntab, const double* __restrict__ dx, const double* __restrict__ dy,
                               const TableRef* __restrict__ refs, double k, double2* __restrict__ tdata) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntab) return;
  TableRef tr = refs[t];
  double2* T = tdata + tr.off + tr.half;
  int N = tr.half;
  double rho = hypot(dx[t], dy[t]);
  double th = atan2(dy[t], dx[t]);
  double x = k * rho;
  // J_n into the real part
  bessel_j_each(x, N, [&](int n, double jn) { T[n] = cmk(jn, 0.0); });
  // Y_n by forward recurrence into the imaginary part
  double ym1 = ::y0(x), yn = ::y1(x);
  T[0].y = ym1;
  if (N >= 1) T[1].y = yn;
  for (int n = 1; n < N; ++n) {
    double yp1 = (2.0 * n / x) * yn - ym1;
    ym1 = yn;
    yn = yp1;
    T[n + 1].y = yn;
  }
  for (int n = N; n >= 0; --n) {
    double s, c;
    sincos((double)n * th, &s, &c);
    double2 h = T[n];
    double2 pos = cmul(h, cmk(c, s));
    double2 neg = cmul(h, cmk(c, -s));  // H_{-n} e^{-in th} = (-1)^n H_n e^{-in th}
    T[n] = pos;
    if (n > 0) T[-n] = (n & 1) ? cscale(neg, -1.0) : neg;
  }
}

// Bessel translation tables: T[n] = sgn^n J_n(k d) e^{i n phi}, n in
// [-half, half]. L2L uses sgn = +1 with (d, phi) the polar form of
// (child - parent); M2M uses sgn = -1 (J_{p-m} indexed by m - p).
__global__ void k_table_bessel(int ntab, const double* __restrict__ dx, const double* __restrict__ dy,
                               const int* __restrict__ sgn, const TableRef* __restrict__ refs, double k,
                               double2* __restrict__ tdata) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntab) return;
  TableRef tr = refs[t];
  double2* T = tdata + tr.off + tr.half;
  int N = tr.half;
  double d = hypot(dx[t], dy[t]);
  double ph = atan2(dy[t], dx[t]);
  bool alt = sgn[t] < 0;
  bessel_j_each(k * d, N, [&](int n, double jn) {
    double s, c;
    sincos((double)n * ph, &s, &c);
    double v = (alt && (n & 1)) ? -jn : jn;
    T[n] = cmk(v * c, v * s);
    if (n > 0) {
      double vm = (n & 1) ? -jn : jn;   // J_{-n} = (-1)^n J_n
      if (alt && (n & 1)) vm = -vm;
      T[-n] = cmk(vm * c, -vm * s);
    }
  });
}

// Heterogeneous M2L tables (Eq. m2loperator with sigma_1, Section 5):
//   A_n(X, Y) = (i^n/pi) int_0^pi e^{i k (Y sin tau - X cos tau)} e^{-i n tau}
//                 sigma_1(-k cos tau) d tau
//             + ((-i)^n/(i pi)) int_0^inf e^{-t Y}/lambda [e^{i lambda X} z^n
//                 + e^{-i lambda X} (-1)^n z^{-n}] sigma_1(lambda) dt,
// lambda = sqrt(t^2 + k^2), z = (lambda - t)/k (so that (-lambda - t)/k = -1/z).
// The t contour dips below the real axis over the branch points and guided-mode
// poles of sigma_1. nsplit blocks per (X, Y) (grid y), each over its share of
// the rule's panels: the block's threads split into G groups of 8 consecutive
// orders and H = 256 / G phases of the quadrature nodes (thread (g, h) sums
// the nodes h, h + H, ... for its orders), and the H partial sums of each
// group are added through LDS. With nsplit > 1 the blocks store partial
// tables, which k_table_image_sum adds in block order.
struct ImageTableArgs {
  Medium med;
  int ncombo;
  const double* X;
  const double* Y;
  const double* dip;    // dip depth of the t contour
  const double* send;   // end of the dip
  const int* pbeg;      // panel range of each combo
  const Panel* panels;
  const TableRef* refs;
  const double* glx;    // 16-point Gauss-Legendre nodes/weights on [-1, 1]
  const double* glw;
  double2* tdata;
  int nsplit;           // blocks per table
  const int64_t* soff;  // nsplit > 1: each table's offset in a partial table
  double2* part;        // nsplit partial tables of plen entries each
  int64_t plen;
};

constexpr int TB_THREADS = 256;
constexpr int TB_NB = 8;

__global__ void __launch_bounds__(TB_THREADS) k_table_image(ImageTableArgs a) {
  __shared__ double2 s_l0a[TB_THREADS], s_lsa[TB_THREADS], s_l0b[TB_THREADS], s_lsb[TB_THREADS];
  __shared__ int s_kind[TB_THREADS];
  __shared__ double2 s_red[TB_THREADS * TB_NB];
  int cb = blockIdx.x;
  if (cb >= a.ncombo) return;
  int tid = threadIdx.x;
  const double k = a.med.k1;
  const double X = a.X[cb], Y = a.Y[cb];
  const double dip = a.dip[cb], send = a.send[cb];
  TableRef tr = a.refs[cb];
  const int N = tr.half;
  // order groups (at most 128: N <= 2 kMaxOrder) and node phases
  const int G = (2 * N + TB_NB) / TB_NB;
  const int H = TB_THREADS / G;
  const int grp = tid % G, ph = tid / G;
  const bool active = ph < H;
  const int n0 = -N + TB_NB * grp;
  // class "i":  i^n * sum exp(l0 + n ls)   (tau nodes; t nodes' minus branch)
  // class "mi": (-i)^n * sum exp(l0 + n ls) (t nodes' plus branch)
  double2 acc_i[TB_NB], acc_mi[TB_NB];
  for (int j = 0; j < TB_NB; ++j) { acc_i[j] = cmk(0, 0); acc_mi[j] = cmk(0, 0); }
  const int pa = a.pbeg[cb], pz = a.pbeg[cb + 1];
  const int pper = (pz - pa + a.nsplit - 1) / a.nsplit;
  const int p0 = min(pz, pa + (int)blockIdx.y * pper), p1 = min(pz, p0 + pper);
  const int nnode = (p1 - p0) * 16;
  const double inv_pi = 0.31830988618379067154;
  for (int q0 = 0; q0 < nnode; q0 += TB_THREADS) {
    int q = q0 + tid;
    int kind = -1;
    double2 l0a = cmk(0, 0), lsa = cmk(0, 0), l0b = cmk(0, 0), lsb = cmk(0, 0);
    if (q < nnode) {
      Panel pn = a.panels[p0 + q / 16];
      int g = q % 16;
      double hw = 0.5 * (pn.b - pn.a), mid = 0.5 * (pn.a + pn.b);
      double s = mid + hw * a.glx[g];
      double w = hw * a.glw[g];
      if (pn.kind == 0) {
        double st, ct;
        sincos(s, &st, &ct);
        double2 sig = sigma1_tau(a.med, ct, st);
        // W = (w/pi) e^{i k (Y st - X ct)} sigma  -> log
        double2 lw = clog2(cscale(sig, w * inv_pi));
        l0a = cmk(lw.x, lw.y + k * (Y * st - X * ct));
        lsa = cmk(0.0, -s);
        kind = 0;
      } else {
        double2 t = cmk(s, 0.0), dt = cmk(1.0, 0.0);
        if (s < send) {
          double sn, cs;
          sincos(M_PI * s / send, &sn, &cs);
          t = cmk(s, -dip * sn);
          dt = cmk(1.0, -dip * M_PI / send * cs);
        }
        double2 lam = csqrt2(cadd(cmul(t, t), cmk(k * k, 0.0)));
        double2 z = cscale(csub(lam, t), 1.0 / k);
        double2 sig = sigma1_t(a.med, t);
        // C = w dt e^{-tY} sigma / (lambda i pi)
        double2 cc = cdiv(cmul(cscale(dt, w * inv_pi), sig), cmul(lam, cmk(0.0, 1.0)));
        double2 lc = clog2(cc);
        double2 lz = clog2(z);
        double2 ilx = cmul(cmk(0.0, X), lam);   // i lambda X
        double2 base = cadd(lc, cscale(t, -Y));
        l0a = cadd(base, ilx);                  // plus branch: e^{i lambda X} z^n, class (-i)^n
        lsa = lz;
        l0b = csub(base, ilx);                  // minus branch: e^{-i lambda X} z^{-n}, class i^n
        lsb = cscale(lz, -1.0);
        kind = 1;
      }
    }
    __syncthreads();
    s_kind[tid] = kind;
    s_l0a[tid] = l0a; s_lsa[tid] = lsa; s_l0b[tid] = l0b; s_lsb[tid] = lsb;
    __syncthreads();
    if (active) {
      int qn = min(TB_THREADS, nnode - q0);
      for (int qq = ph; qq < qn; qq += H) {
        int kd = s_kind[qq];
        double2 la = s_l0a[qq], sa = s_lsa[qq];
        double2 v = cexp2(cadd(la, cscale(sa, (double)n0)));
        double2 st = cexp2(sa);
        if (kd == 0) {
          for (int j = 0; j < TB_NB; ++j) { acc_i[j] = cadd(acc_i[j], v); v = cmul(v, st); }
        } else {
          for (int j = 0; j < TB_NB; ++j) { acc_mi[j] = cadd(acc_mi[j], v); v = cmul(v, st); }
          double2 lb = s_l0b[qq], sb = s_lsb[qq];
          double2 vb = cexp2(cadd(lb, cscale(sb, (double)n0)));
          double2 stb = cexp2(sb);
          for (int j = 0; j < TB_NB; ++j) {
            // (-1)^n (-i)^n = i^n
            acc_i[j] = cadd(acc_i[j], vb);
            vb = cmul(vb, stb);
          }
        }
      }
    }
  }
  // sum the node phases of each order group (phase order fixed)
  for (int cls = 0; cls < 2; ++cls) {
    __syncthreads();
    if (active)
      for (int j = 0; j < TB_NB; ++j) s_red[tid * TB_NB + j] = cls == 0 ? acc_i[j] : acc_mi[j];
    __syncthreads();
    if (ph == 0) {
      for (int j = 0; j < TB_NB; ++j) {
        double2 v = s_red[grp * TB_NB + j];
        for (int h = 1; h < H; ++h) v = cadd(v, s_red[(h * G + grp) * TB_NB + j]);
        if (cls == 0)
          acc_i[j] = v;
        else
          acc_mi[j] = v;
      }
    }
  }
  if (ph != 0) return;
  double2* T = a.nsplit > 1 ? a.part + (int64_t)blockIdx.y * a.plen + a.soff[cb] + tr.half : a.tdata + tr.off + tr.half;
  for (int j = 0; j < TB_NB; ++j) {
    int n = n0 + j;
    if (n < -N || n > N) continue;
    int r = ((n % 4) + 4) % 4;  // i^n
    double2 ip = r == 0 ? cmk(1, 0) : r == 1 ? cmk(0, 1) : r == 2 ? cmk(-1, 0) : cmk(0, -1);
    double2 im = cconj(ip);     // (-i)^n
    T[n] = cadd(cmul(ip, acc_i[j]), cmul(im, acc_mi[j]));
  }
}

// ------------------------------------------------------------------ launchers
static inline int blocks(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

void launch_gather(hipStream_t s, int n, int nrhs, const int* perm, const double2* src, double2* dst, int cj) {
  int64_t tot = (int64_t)n * nrhs;
  hipLaunchKernelGGL(k_gather, dim3(blocks(tot, 256)), dim3(256), 0, s, n, nrhs, perm, src, dst, cj);
}
void launch_scatter(hipStream_t s, int n, int nrhs, const int* perm, const double2* src, double2* dst, int cj,
                    const double2* diag, const double2* qsrc) {
  int64_t tot = (int64_t)n * nrhs;
  hipLaunchKernelGGL(k_scatter, dim3(blocks(tot, 256)), dim3(256), 0, s, n, nrhs, perm, src, dst, cj, diag, qsrc);
}
void launch_self_term(hipStream_t s, int n, const double2* pts, int nq, const double2* qc, const double2* qky,
                      double2* g, double2* dy) {
  hipLaunchKernelGGL(k_self_term, dim3(blocks(n, SELF_THREADS)), dim3(SELF_THREADS), 0, s, n, pts, nq, qc, qky, g, dy);
}
void launch_self_grad(hipStream_t s, int n, int nrhs, const double2* dy, const double2* vs, const double2* qs,
                      double2* gs) {
  hipLaunchKernelGGL(k_self_grad, dim3(blocks(n, 256)), dim3(256), 0, s, n, nrhs, dy, vs, qs, gs);
}
void launch_p2m(hipStream_t s, const TreeView& tv, const int* leaves, int nl, int Pmax, const double2* qs,
                double2* alpha, int conj_w, double2 pref) {
  if (nl <= 0) return;
  // at most 37 KiB (Pmax = 255): within the default dynamic LDS limit
  if (tv.nrhs == 1)
    hipLaunchKernelGGL(k_p2m<1>, dim3(nl, 1), dim3(WAVE), p2m_lds_bytes(Pmax, 1), s, tv, leaves, nl, qs, alpha,
                       conj_w, pref);
  else
    hipLaunchKernelGGL(k_p2m<P2M_RB>, dim3(nl, (tv.nrhs + P2M_RB - 1) / P2M_RB), dim3(WAVE),
                       p2m_lds_bytes(Pmax, P2M_RB), s, tv, leaves, nl, qs, alpha, conj_w, pref);
}
void launch_l2p(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const int* pt_box, int Pmax,
                const double2* beta, double2* us, int conj_w, double2 pref, int accumulate) {
  if (nl <= 0) return;
  if (tv.nrhs == 1 && pt_box)
    hipLaunchKernelGGL(k_l2p_flat, dim3((tv.n + WAVE - 1) / WAVE), dim3(WAVE),
                       sizeof(double2) * (size_t)(L2P_RUNS * 2 * (Pmax + 1)), s, tv, pt_box, Pmax, beta, us, conj_w,
                       pref, accumulate);
  else if (tv.nrhs == 1)
    hipLaunchKernelGGL(k_l2p<1>, dim3(nl, 1), dim3(WAVE), l2p_lds_bytes(Pmax, 1), s, tv, leaves, nl, beta, us,
                       conj_w, pref, accumulate);
  else
    hipLaunchKernelGGL(k_l2p<L2P_RB>, dim3(nl, (tv.nrhs + L2P_RB - 1) / L2P_RB), dim3(WAVE),
                       l2p_lds_bytes(Pmax, L2P_RB), s, tv, leaves, nl, beta, us, conj_w, pref, accumulate);
}
// LDS bytes of a translation item: the padded table (real, imaginary and
// negated imaginary parts) and the padded source-coefficient tile.
size_t trans_lds_bytes(int Ps, int Pd) {
  const int ntp = trans_table_stride(2 * (Ps + Pd) + 1);
  const int npi = trans_pairs_per_item(Ps, Pd);
  return sizeof(double) * (size_t)(3 * ntp) + sizeof(double2) * (size_t)npi * round4(2 * Ps + 1);
}
// The split gather stages four tables and four source tiles; the source area
// also holds the four waves' partial tiles (4 x 4 x 64 doubles) at the end.
size_t trans_lds_bytes_split(int Ps, int Pd) {
  const int ntp = trans_table_stride(2 * (Ps + Pd) + 1);
  const int npi = trans_pairs_per_item(Ps, Pd);
  const size_t src = sizeof(double2) * (size_t)(4 * npi) * round4(2 * Ps + 1);
  const size_t red = sizeof(double) * (size_t)(16 * 64);
  return sizeof(double) * (size_t)(12 * ntp) + (src > red ? src : red);
}

// Dynamic LDS limit of the translation kernels: the CU's 160 KiB less each
// kernel's static LDS. Called when a plan is built (before any launch or
// graph capture); returns the first HIP error.
template <bool REV, int MODE, int NTMAX>
static hipError_t trans_lds_limit_one() {
  const void* f = (const void*)k_trans_mfma<REV, MODE, NTMAX>;
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, f);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - (int)fa.sharedSizeBytes);
}

template <bool REV, int MODE>
static hipError_t trans_lds_limit() {
  const hipError_t e = trans_lds_limit_one<REV, MODE, 2>();
  return e != hipSuccess ? e : trans_lds_limit_one<REV, MODE, 8>();
}

hipError_t init_kernel_attributes() {
  const hipError_t es[8] = {trans_lds_limit<false, OUT_GATHER4>(),          trans_lds_limit<false, OUT_CONTRIB>(),
                            trans_lds_limit<false, OUT_EXCLUSIVE>(),        trans_lds_limit<true, OUT_GATHER4>(),
                            trans_lds_limit<true, OUT_CONTRIB>(),           trans_lds_limit<true, OUT_EXCLUSIVE>(),
                            trans_lds_limit_one<false, OUT_GATHER4_SPLIT, 1>(), trans_lds_limit_one<true, OUT_GATHER4_SPLIT, 1>()};
  for (hipError_t e : es)
    if (e != hipSuccess) return e;
  return hipSuccess;
}

template <bool REV, int MODE>
static void trans_one(hipStream_t s, const TreeView& tv, const TransItem* items, int nitems, size_t lds, int ntw,
                      const int64_t* soff, const int64_t* doff, const int64_t* pcoff, const Toff4& q4,
                      const double2* tdata, const double2* src, double2* dst, double* contrib, int64_t cstride) {
  if (MODE == OUT_GATHER4_SPLIT)
    hipLaunchKernelGGL((k_trans_mfma<REV, OUT_GATHER4_SPLIT, 1>), dim3(nitems, tv.nrhs), dim3(TR_THREADS), lds, s, tv,
                       items, soff, doff, pcoff, q4, tdata, src, dst, contrib, cstride);
  else if (ntw <= 2)
    hipLaunchKernelGGL((k_trans_mfma<REV, MODE, 2>), dim3(nitems, tv.nrhs), dim3(TR_THREADS), lds, s, tv, items,
                       soff, doff, pcoff, q4, tdata, src, dst, contrib, cstride);
  else
    hipLaunchKernelGGL((k_trans_mfma<REV, MODE, 8>), dim3(nitems, tv.nrhs), dim3(TR_THREADS), lds, s, tv, items,
                       soff, doff, pcoff, q4, tdata, src, dst, contrib, cstride);
}

void launch_trans(hipStream_t s, const TreeView& tv, const TransItem* items, int nitems, int Ps, int Pd,
                  const int64_t* soff, const int64_t* doff, const int64_t* pcoff, const Toff4& q4,
                  const double2* tdata, const double2* src, double2* dst, double* contrib, int64_t cstride, int rev,
                  int gather4, int ntw) {
  if (nitems <= 0) return;
  const size_t lds = gather4 == 2 ? trans_lds_bytes_split(Ps, Pd) : trans_lds_bytes(Ps, Pd);
#define HFMM_TRANS(R, M) \
  trans_one<R, M>(s, tv, items, nitems, lds, ntw, soff, doff, pcoff, q4, tdata, src, dst, contrib, cstride)
  if (contrib) {
    if (rev) HFMM_TRANS(true, OUT_CONTRIB); else HFMM_TRANS(false, OUT_CONTRIB);
  } else if (gather4 == 2) {
    if (rev) HFMM_TRANS(true, OUT_GATHER4_SPLIT); else HFMM_TRANS(false, OUT_GATHER4_SPLIT);
  } else if (gather4) {
    if (rev) HFMM_TRANS(true, OUT_GATHER4); else HFMM_TRANS(false, OUT_GATHER4);
  } else {
    if (rev) HFMM_TRANS(true, OUT_EXCLUSIVE); else HFMM_TRANS(false, OUT_EXCLUSIVE);
  }
#undef HFMM_TRANS
}

void launch_reduce_contrib(hipStream_t s, const TreeView& tv, const int* boxes, int nb, const int* ptr,
                           const int64_t* beg, const double* contrib, int64_t cstride, double2* dst) {
  if (nb)
    hipLaunchKernelGGL(k_reduce_contrib, dim3(nb, tv.nrhs), dim3(RED_THREADS), 0, s, tv, boxes, nb, ptr, beg, contrib,
                       cstride, dst);
}

void launch_fill_zero(hipStream_t s, double2* p, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_fill_zero, dim3(blocks(n, 256)), dim3(256), 0, s, p, n);
}
// node ranges per leaf for the evaluation: enough blocks to fill the GPU
static int if_qsplit(const IfaceLists& L, int atomic) {
  if (!atomic) return 1;
  const int nch = L.nqp / WAVE;
  return max(1, min(nch / 4, (2048 + L.ntl - 1) / max(L.ntl, 1)));
}
void launch_iface(hipStream_t s, const TreeView& tv, const IfaceLists* Ls, int ncls, int nrhs, const double2* qs,
                  double2* us, int64_t ps, int64_t rs, int atomic) {
  for (int c = 0; c < ncls; ++c) {
    const IfaceLists& L = Ls[c];
    if (!L.ntl || !L.nq) continue;
    for (int r0 = 0; r0 < nrhs; r0 += L.rif) {
      const int nr = min(L.rif, nrhs - r0);
      hipLaunchKernelGGL(k_if_src, dim3(L.nsb, L.nqp / WAVE), dim3(4 * WAVE), 0, s, tv, L.sbox, L.nq, L.nqp, L.rif,
                         L.qky, L.qkx, qs + r0 * rs, ps, rs, nr, L.S);
      hipLaunchKernelGGL(k_if_trans, dim3(L.ntl, L.nqp / WAVE), dim3(WAVE), 0, s, tv, L.tleaf, L.tptr, L.tsrc,
                         L.sbox, L.nq, L.nqp, L.rif, L.qc, L.qkx, L.S, nr, L.T);
      hipLaunchKernelGGL(k_if_eval<false>, dim3(L.ntl, if_qsplit(L, atomic)), dim3(4 * WAVE), 0, s, tv, L.tleaf,
                         L.nq, L.nqp, L.rif, L.qky, L.qkx, L.T, nr, nullptr, us + r0 * rs, ps, rs, atomic);
    }
  }
}
void launch_if_grid(hipStream_t s, int npts, const double2* xy, int nq, const double2* qc, const double2* qky,
                    const double2* qkx, double2* out) {
  if (npts > 0) hipLaunchKernelGGL(k_if_grid, dim3(blocks(npts, WAVE)), dim3(WAVE), 0, s, npts, xy, nq, qc, qky, qkx, out);
}
void launch_iface_table(hipStream_t s, const TreeView& tv, const IfTable* tabs, int ntab, int nrhs, const double2* qs,
                        double2* us, int64_t ps, int64_t rs, int atomic) {
  for (int c = 0; c < ntab; ++c) {
    if (!tabs[c].ntl) continue;
    // with atomic additions a block per work item, else a block per leaf
    IfTable tb = tabs[c];
    if (!atomic) tb.item_t = nullptr;
    const int nblk = atomic ? tb.nitem : tb.ntl;
    for (int r0 = 0; r0 < nrhs; r0 += kIfRhs)
      hipLaunchKernelGGL(k_if_table<false>, dim3(nblk), dim3(4 * WAVE), 0, s, tv, tb, tb.coef, min(kIfRhs, nrhs - r0),
                         qs + r0 * rs, nullptr, us + r0 * rs, ps, rs, atomic);
  }
}
void launch_table_hankel(hipStream_t s, int ntab, const double* dx, const double* dy, const TableRef* refs, double k,
                         double2* tdata) {
  if (ntab) hipLaunchKernelGGL(k_table_hankel, dim3(blocks(ntab, 64)), dim3(64), 0, s, ntab, dx, dy, refs, k, tdata);
}
void launch_table_bessel(hipStream_t s, int ntab, const double* dx, const double* dy, const int* sgn,
                         const TableRef* refs, double k, double2* tdata) {
  if (ntab) hipLaunchKernelGGL(k_table_bessel, dim3(blocks(ntab, 64)), dim3(64), 0, s, ntab, dx, dy, sgn, refs, k, tdata);
}
// tdata[off + i] = sum over the partial tables in order (one block per table)
__global__ void k_table_image_sum(int ncombo, const TableRef* __restrict__ refs, const int64_t* __restrict__ soff,
                                  int nsplit, int64_t plen, const double2* __restrict__ part,
                                  double2* __restrict__ tdata) {
  const int cb = blockIdx.x;
  if (cb >= ncombo) return;
  const TableRef tr = refs[cb];
  const int len = 2 * tr.half + 1;
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    double2 v = part[soff[cb] + i];
    for (int sp = 1; sp < nsplit; ++sp) v = cadd(v, part[(int64_t)sp * plen + soff[cb] + i]);
    tdata[tr.off + i] = v;
  }
}

void launch_table_image(hipStream_t s, const Medium& med, int ncombo, const double* X, const double* Y,
                        const double* dip, const double* send, const int* pbeg, const Panel* panels,
                        const TableRef* refs, const double* glx, const double* glw, double2* tdata, int nsplit,
                        const int64_t* soff, double2* part, int64_t plen) {
  if (!ncombo) return;
  if (nsplit < 1 || !part) nsplit = 1;
  ImageTableArgs a{med, ncombo, X, Y, dip, send, pbeg, panels, refs, glx, glw, tdata, nsplit, soff, part, plen};
  hipLaunchKernelGGL(k_table_image, dim3(ncombo, nsplit), dim3(TB_THREADS), 0, s, a);
  if (nsplit > 1)
    hipLaunchKernelGGL(k_table_image_sum, dim3(ncombo), dim3(TB_THREADS), 0, s, ncombo, refs, soff, nsplit, plen,
                       part, tdata);
}


void launch_l2p_grad(hipStream_t s, const TreeView& tv, const int* leaves, int nl, int Pmax, const double2* alpha,
                     const double2* qs, double2* gs, int add) {
  if (nl <= 0) return;
  const int rb = min(L2P_RB, tv.nrhs);
  hipLaunchKernelGGL(k_l2p_grad, dim3(nl), dim3(WAVE), l2p_grad_lds_bytes(Pmax, rb), s, tv, leaves, nl, rb, alpha,
                     qs, gs, add);
}
template <int CLS>
static void p2p_grad_class(hipStream_t s, const TreeView& tv, const int* items, int nl, const int* ptr,
                           const int2* rng, const int* sym, const double2* vs, const double2* qs, double2* gs) {
  if (nl <= 0) return;
  if (tv.nrhs == 1)
    hipLaunchKernelGGL((k_p2p_grad<true, CLS>), dim3(nl), dim3(WAVE), 0, s, tv, items, nl, ptr, rng, sym, vs, qs, gs);
  else
    hipLaunchKernelGGL((k_p2p_grad<false, CLS>), dim3(nl), dim3(WAVE), 0, s, tv, items, nl, ptr, rng, sym, vs, qs, gs);
}

void launch_p2p_grad(hipStream_t s, const TreeView& tv, const int* items, const int* cls_ptr, const int* ptr,
                     const int2* rng, const int* sym, const double2* vs, const double2* qs, double2* gs) {
#define HFMM_P2P_GRAD(C)                                                                                          \
  p2p_grad_class<C>(s, tv, items + cls_ptr[C], cls_ptr[C + 1] - cls_ptr[C], ptr + cls_ptr[C], rng, sym + cls_ptr[C], \
                    vs, qs, gs)
  HFMM_P2P_GRAD(0); HFMM_P2P_GRAD(1); HFMM_P2P_GRAD(2); HFMM_P2P_GRAD(3); HFMM_P2P_GRAD(4); HFMM_P2P_GRAD(5);
#undef HFMM_P2P_GRAD
  static_assert(kH0Classes == 5, "one launch per class and one for the large-argument class");
}
void launch_iface_grad(hipStream_t s, const TreeView& tv, const IfaceLists* Ls, int ncls, int nrhs,
                       const double2* vs, const double2* qs, double2* gs) {
  const int64_t rs = tv.n;
  for (int c = 0; c < ncls; ++c) {
    const IfaceLists& L = Ls[c];
    if (!L.ntl || !L.nq) continue;
    for (int r0 = 0; r0 < nrhs; r0 += L.rif) {
      const int nr = min(L.rif, nrhs - r0);
      hipLaunchKernelGGL(k_if_src, dim3(L.nsb, L.nqp / WAVE), dim3(4 * WAVE), 0, s, tv, L.sbox, L.nq, L.nqp, L.rif,
                         L.qky, L.qkx, vs + r0 * rs, (int64_t)1, rs, nr, L.S);
      hipLaunchKernelGGL(k_if_trans, dim3(L.ntl, L.nqp / WAVE), dim3(WAVE), 0, s, tv, L.tleaf, L.tptr, L.tsrc,
                         L.sbox, L.nq, L.nqp, L.rif, L.qc, L.qkx, L.S, nr, L.T);
      hipLaunchKernelGGL(k_if_eval<true>, dim3(L.ntl, if_qsplit(L, 1)), dim3(4 * WAVE), 0, s, tv, L.tleaf, L.nq,
                         L.nqp, L.rif, L.qky, L.qkx, L.T, nr, qs + r0 * rs, gs, (int64_t)1, rs, 1);
    }
  }
}
void launch_iface_table_grad(hipStream_t s, const TreeView& tv, const IfTable* tabs, int ntab, int nrhs,
                             const double2* vs, const double2* qs, double2* gs) {
  const int64_t rs = tv.n;
  for (int c = 0; c < ntab; ++c) {
    if (!tabs[c].ntl) continue;
    for (int r0 = 0; r0 < nrhs; r0 += kIfRhs)
      hipLaunchKernelGGL(k_if_table<true>, dim3(tabs[c].nitem), dim3(4 * WAVE), 0, s, tv, tabs[c], tabs[c].coef,
                         min(kIfRhs, nrhs - r0), vs + r0 * rs, qs + r0 * rs, gs, (int64_t)1, rs, 1);
  }
}
void launch_scatter_grad(hipStream_t s, int n, const int* perm, const double2* gs, double2* grad) {
  hipLaunchKernelGGL(k_scatter_grad, dim3(blocks(n, 256)), dim3(256), 0, s, n, perm, gs, grad);
}

}  // namespace hfmm
