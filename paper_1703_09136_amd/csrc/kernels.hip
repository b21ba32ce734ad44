// HIP kernels of the layered-media heterogeneous FMM (gfx950, FP64).
//
// Stages (Algorithm 1 of the paper): P2M at leaves (Eq. multi_coeff), M2M and
// L2L by the free-space Graf translations, M2L with the free-space operator
// (Section 3.3) and with the heterogeneous operator of the scattered field
// (Eq. m2l / m2loperator, sigma_1 of Section 5), L2P, and the local direct
// interactions: free-space H0 pairs and, for image pairs that are not
// admissible, the Sommerfeld integral evaluated by quadrature (Section 5,
// strategy (b) for the local direct interactions).
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

__device__ __noinline__ double2 hankel0_large_call(double x) { return hankel0_large(x); }

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

__global__ void k_scatter(int n, int nrhs, const int* __restrict__ perm, const double2* __restrict__ src,
                          double2* __restrict__ dst, int conj_out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t tot = (int64_t)n * nrhs;
  if (idx >= tot) return;
  int r = (int)(idx / n), i = (int)(idx % n);
  double2 v = src[idx];
  dst[(int64_t)r * n + perm[i]] = conj_out ? cconj(v) : v;
}

// ------------------------------------------------------------------ P2M
// alpha_p = sum_j q_j J_p(k rho_j) e^{-i p theta_j}, p in [-P, P] (Eq. multi_coeff).
// One wave per leaf; lanes own points; every order is reduced across the wave.
// With conj_w the phase is e^{+i p theta_j} and the result is scaled by pref:
// this is the transpose of L2P, used by the adjoint.
__global__ void __launch_bounds__(WAVE) k_p2m(TreeView tv, const int* __restrict__ leaves, int nleaves,
                                              const double2* __restrict__ qs, double2* __restrict__ alpha,
                                              int conj_w, double2 pref) {
  int li = blockIdx.x;
  if (li >= nleaves) return;
  int b = leaves[li];
  int lane = threadIdx.x;
  int P = tv.P[tv.level[b]];
  int2 pr = tv.prange[b];
  double2 c = tv.ctr[b];
  for (int r = 0; r < tv.nrhs; ++r)
    for (int o = lane; o < 2 * P + 1; o += WAVE) alpha[r * tv.ctot + tv.coff[b] + o] = cmk(0, 0);
  // a bound on k*rho for the whole box gives one recurrence length per wave
  double rmax = 0.0;
  for (int j = pr.x + lane; j < pr.y; j += WAVE) {
    double2 p = tv.pts[j];
    rmax = fmax(rmax, hypot(p.x - c.x, p.y - c.y));
  }
  for (int m = 1; m < WAVE; m <<= 1) rmax = fmax(rmax, __shfl_xor(rmax, m, WAVE));
  int nstart = miller_start(tv.k * rmax, P);
  for (int j0 = pr.x; j0 < pr.y; j0 += WAVE) {
    int j = j0 + lane;
    bool valid = j < pr.y;
    double dx = 0, dy = 0;
    if (valid) { double2 p = tv.pts[j]; dx = p.x - c.x; dy = p.y - c.y; }
    double rho = hypot(dx, dy);
    double x = fmax(tv.k * rho, 1e-100);
    double2 w = rho > 0 ? cmk(dx / rho, (conj_w ? dy : -dy) / rho) : cmk(1, 0);
    double th = atan2(w.y, w.x);
    double s, co;
    sincos((double)P * th, &s, &co);
    double2 wn = cmk(co, s);  // w^P
    double inv_s;
    int nres;
    miller_norm(x, nstart, inv_s, nres);
    miller_emit(x, nstart, P, inv_s, nres, [&](int n, double jn) {
      if (!valid) jn = 0.0;
      double2 wpos = cscale(wn, jn);
      double2 wneg = cscale(cconj(wn), (n & 1) ? -jn : jn);
      for (int r = 0; r < tv.nrhs; ++r) {
        double2 q = valid ? qs[(int64_t)r * tv.n + j] : cmk(0, 0);
        double2 cp = wave_sum(cmul(q, wpos));
        double2 cm = n > 0 ? wave_sum(cmul(q, wneg)) : cmk(0, 0);
        if (lane == 0) {
          double2* a = alpha + r * tv.ctot + tv.coff[b] + P;
          a[n] = cadd(a[n], cmul(pref, cp));
          if (n > 0) a[-n] = cadd(a[-n], cmul(pref, cm));
        }
      }
      wn = cmul(wn, cconj(w));
    });
  }
}

// ------------------------------------------------------------------ L2P
// u_i (+)= pref * sum_p beta_p J_p(k r_i) e^{i p theta_i} (local expansion,
// Section 3.2). One wave per leaf, a lane per point. With conj_w the phase is
// e^{-i p theta_i} (transpose of P2M, used by the adjoint). Leaves above level 2
// have no local expansion and write zeros. accumulate = 0 stores.
__global__ void __launch_bounds__(WAVE) k_l2p(TreeView tv, const int* __restrict__ leaves, int nleaves,
                                              const double2* __restrict__ beta, double2* __restrict__ us,
                                              int conj_w, double2 pref, int accumulate) {
  int li = blockIdx.x;
  if (li >= nleaves) return;
  int b = leaves[li];
  int lane = threadIdx.x;
  int lev = tv.level[b];
  int P = tv.P[lev];
  int2 pr = tv.prange[b];
  double2 c = tv.ctr[b];
  bool has_local = lev >= 2;
  for (int j = pr.x + lane; j < pr.y; j += WAVE) {
    double2 p = tv.pts[j];
    double dx = p.x - c.x, dy = p.y - c.y;
    double rho = hypot(dx, dy);
    double x = fmax(tv.k * rho, 1e-100);
    double2 w = rho > 0 ? cmk(dx / rho, (conj_w ? -dy : dy) / rho) : cmk(1, 0);
    for (int r = 0; r < tv.nrhs; ++r) {
      double2 acc = cmk(0, 0);
      if (has_local) {
        const double2* bt = beta + r * tv.ctot + tv.coff[b] + P;
        double th = atan2(w.y, w.x);
        double s, co;
        sincos((double)P * th, &s, &co);
        double2 wn = cmk(co, s);
        bessel_j_each(x, P, [&](int n, double jn) {
          double2 t = cmul(bt[n], wn);
          if (n > 0) {
            double2 tm = cmul(bt[-n], cconj(wn));
            t = cadd(t, (n & 1) ? cscale(tm, -1.0) : tm);
          }
          acc = cadd(acc, cscale(t, jn));
          wn = cmul(wn, cconj(w));
        });
      }
      int64_t idx = (int64_t)r * tv.n + j;
      double2 v = cmul(pref, acc);
      us[idx] = accumulate ? cadd(us[idx], v) : v;
    }
  }
}

// ------------------------------------------------------------------ Toeplitz contraction
// acc(p) = sum_{m=-Ps}^{Ps} T[m - p] s(m), s(m) = src[m] or, for image sources,
// (-1)^m src[-m]; rev reads T[p - m] instead (the transposed operator).
__device__ inline double2 toeplitz_dot(const double2* __restrict__ T, const double2* __restrict__ S, int Ps,
                                       int p, int image, int rev) {
  double2 acc = cmk(0, 0);
  if (!image) {
    if (!rev)
      for (int m = -Ps; m <= Ps; ++m) acc = cadd(acc, cmul(T[m - p], S[m]));
    else
      for (int m = -Ps; m <= Ps; ++m) acc = cadd(acc, cmul(T[p - m], S[m]));
  } else {
    // s(m) = (-1)^m S[-m]  =>  sum_m' T[-m' - p] (-1)^m' S[m']
    if (!rev)
      for (int m = -Ps; m <= Ps; ++m) {
        double2 v = cmul(T[-m - p], S[m]);
        acc = (m & 1) ? csub(acc, v) : cadd(acc, v);
      }
    else {
      // transpose of the reflected operator: the sign moves to the output,
      // out(p) = (-1)^p sum_m T[-p - m] S[m]
      for (int m = -Ps; m <= Ps; ++m) acc = cadd(acc, cmul(T[-p - m], S[m]));
      if (p & 1) acc = cscale(acc, -1.0);
    }
  }
  return acc;
}

// M2L: beta_t = sum over the list of t of T_e * s_e (free: alpha of the source
// box; image: reflected alpha). One wave per target box; the list of a box
// holds all its free and heterogeneous entries, so beta_t is written once.
__global__ void __launch_bounds__(WAVE) k_m2l(TreeView tv, const int* __restrict__ targets, int ntargets,
                                              const int* __restrict__ ptr, const M2LEntry* __restrict__ ent,
                                              const TableRef* __restrict__ tabs, const double2* __restrict__ tdata,
                                              const double2* __restrict__ src, double2* __restrict__ dst,
                                              int rev) {
  int wi = blockIdx.x;
  if (wi >= ntargets) return;
  int t = targets[wi];
  int lane = threadIdx.x;
  int P = tv.P[tv.level[t]];
  int nout = 2 * P + 1;
  int e0 = ptr[wi], e1 = ptr[wi + 1];
  for (int r = 0; r < tv.nrhs; ++r) {
    for (int o0 = 0; o0 < nout; o0 += WAVE) {
      int o = o0 + lane;
      double2 acc = cmk(0, 0);
      if (o < nout) {
        int p = o - P;
        for (int e = e0; e < e1; ++e) {
          M2LEntry en = ent[e];
          TableRef tr = tabs[en.table];
          const double2* T = tdata + tr.off + tr.half;
          const double2* S = src + r * tv.ctot + tv.coff[en.src] + P;
          acc = cadd(acc, toeplitz_dot(T, S, P, p, en.image, rev));
        }
        dst[r * tv.ctot + tv.coff[t] + o] = acc;
      }
    }
  }
}

// ------------------------------------------------------------------ batched M2L on MFMA
// For one table t (t[n], n = m - p in [-2P, 2P]) and a batch of (source,
// target) pairs using it:
//   out_c[p] += sum_m t[m - p] S_c[m]        (REV: t[p - m], the transpose)
// computed as a real GEMM through the 2x2 embedding of complex numbers,
//   [Re out; Im out] = [[Tr, -Ti], [Ti, Tr]] [Re S; Im S],
// with 16x16x4 FP64 MFMA tiles: rows = 2M (M = 2P + 1) in tiles of 16, k = 2M
// in steps of 4, columns = 16 pairs per wave. Operator tiles are expanded from
// the Toeplitz vector in LDS on the fly. Image pairs use the reflected source
// coefficients abar_m = (-1)^m alpha_{-m}; in the transpose the reflection
// moves to the output. Results are added atomically into the target boxes.
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int M2L_THREADS = 256;

template <bool REV>
__global__ void __launch_bounds__(M2L_THREADS) k_m2l_mfma(TreeView tv, const M2LItem* __restrict__ items,
                                                         const int* __restrict__ psrc, const int* __restrict__ pdst,
                                                         const TableRef* __restrict__ tabs,
                                                         const double2* __restrict__ tdata,
                                                         const double2* __restrict__ src, double2* __restrict__ dst,
                                                         int r) {
  extern __shared__ double2 lds[];
  const M2LItem it = items[blockIdx.x];
  const int P = tv.P[it.level];
  const int M = 2 * P + 1;
  const int M2 = 2 * M;
  const int nrt = (M2 + 15) / 16;
  const int nks = (M2 + 3) / 4;
  const int npi = (M <= 64) ? 64 : 16;
  double2* s_t = lds;
  double2* s_s = lds + (4 * P + 1);
  const int tid = threadIdx.x;
  const TableRef tr = tabs[it.table];
  const double2* T = tdata + tr.off + tr.half - 2 * P;  // T[0] = t[-2P]
  for (int i = tid; i < 4 * P + 1; i += M2L_THREADS) s_t[i] = T[i];
  const bool reflect_in = it.image && !REV;
  for (int idx = tid; idx < npi * M; idx += M2L_THREADS) {
    int c = idx / M, m = idx - c * M;
    double2 v = cmk(0, 0);
    if (c < it.npairs) {
      const double2* S = src + (int64_t)r * tv.ctot + tv.coff[psrc[it.pbeg + c]];
      if (reflect_in) {
        v = S[M - 1 - m];
        if ((m + P) & 1) v = cscale(v, -1.0);
      } else {
        v = S[m];
      }
    }
    s_s[idx] = v;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  int ntile, rt_lo, rt_stride, rt_cnt;
  const int rt_end = min(nrt, it.rt_base + 32);
  if (npi == 64) {
    ntile = wave;
    rt_lo = it.rt_base;
    rt_stride = 1;
    rt_cnt = min(rt_end - rt_lo, 8);
  } else {
    ntile = 0;
    rt_lo = it.rt_base + wave;
    rt_stride = 4;
    rt_cnt = rt_lo < rt_end ? min((rt_end - rt_lo + 3) / 4, 8) : 0;
  }
  if (ntile * 16 >= it.npairs || rt_cnt <= 0) return;
  const int lrow = lane & 15, lk = lane >> 4;
  const double2* Scol = s_s + (ntile * 16 + lrow) * M;
  d4 acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
  for (int ks = 0; ks < nks; ++ks) {
    const int k = 4 * ks + lk;
    double b = 0.0;
    int mk = -1;
    bool kim = false;
    if (k < M) {
      b = Scol[k].x;
      mk = k;
    } else if (k < M2) {
      b = Scol[k - M].y;
      mk = k - M;
      kim = true;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < rt_cnt) {
        const int row = (rt_lo + j * rt_stride) * 16 + lrow;
        double a = 0.0;
        if (mk >= 0 && row < M2) {
          const bool rim = row >= M;
          const int p = rim ? row - M : row;
          const int tix = REV ? (p - mk + 2 * P) : (mk - p + 2 * P);
          const double2 t = s_t[tix];
          a = (rim == kim) ? t.x : (rim ? t.y : -t.y);
        }
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
      }
    }
  }
  const int col = ntile * 16 + lrow;
  if (col >= it.npairs) return;
  double2* out = dst + (int64_t)r * tv.ctot + tv.coff[pdst[it.pbeg + col]];
  const bool reflect_out = REV && it.image;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (j >= rt_cnt) continue;
    const int rt = rt_lo + j * rt_stride;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // D[row][col] of a 16x16x4 FP64 tile sits in lane col + 16 (row % 4), register row / 4
      const int row = rt * 16 + 4 * i + lk;
      if (row >= M2) continue;
      const bool rim = row >= M;
      const int p = rim ? row - M : row;
      double v = acc[j][i];
      int po = p;
      if (reflect_out) {
        po = M - 1 - p;
        if ((p + P) & 1) v = -v;
      }
      unsafeAtomicAdd(rim ? &out[po].y : &out[po].x, v);
    }
  }
}

__global__ void k_fill_zero(double2* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = cmk(0.0, 0.0);
}

// M2M: alpha_parent = sum over children of T_q * alpha_child (q = quadrant of
// the child). One wave per parent box of the level.
__global__ void __launch_bounds__(WAVE) k_m2m(TreeView tv, const int* __restrict__ boxes, int nb,
                                              const TableRef* __restrict__ tabs4, const double2* __restrict__ tdata,
                                              const double2* __restrict__ src, double2* __restrict__ dst, int rev) {
  int wi = blockIdx.x;
  if (wi >= nb) return;
  int b = boxes[wi];
  int lane = threadIdx.x;
  int lev = tv.level[b];
  int P = tv.P[lev], Pc = tv.P[lev + 1];
  int nout = 2 * P + 1;
  for (int r = 0; r < tv.nrhs; ++r)
    for (int o0 = 0; o0 < nout; o0 += WAVE) {
      int o = o0 + lane;
      if (o >= nout) continue;
      int p = o - P;
      double2 acc = cmk(0, 0);
      for (int qd = 0; qd < 4; ++qd) {
        int ch = tv.child[4 * b + qd];
        if (ch < 0) continue;
        TableRef tr = tabs4[qd];
        const double2* T = tdata + tr.off + tr.half;
        const double2* S = src + r * tv.ctot + tv.coff[ch] + Pc;
        acc = cadd(acc, toeplitz_dot(T, S, Pc, p, 0, rev));
      }
      dst[r * tv.ctot + tv.coff[b] + o] = acc;
    }
}

// L2L: beta_child += T_q * beta_parent. One wave per child box of the level.
// The same kernel applies the transpose of M2M in the adjoint (rev = 1,
// accumulate = 0 writes instead of adding).
__global__ void __launch_bounds__(WAVE) k_l2l(TreeView tv, const int* __restrict__ boxes, int nb,
                                              const TableRef* __restrict__ tabs4, const double2* __restrict__ tdata,
                                              const double2* __restrict__ src, double2* __restrict__ dst, int rev,
                                              int accumulate) {
  int wi = blockIdx.x;
  if (wi >= nb) return;
  int b = boxes[wi];
  int par = tv.parent[b];
  int lane = threadIdx.x;
  int lev = tv.level[b];
  int P = tv.P[lev], Pp = tv.P[lev - 1];
  int nout = 2 * P + 1;
  TableRef tr = tabs4[tv.quad[b]];
  const double2* T = tdata + tr.off + tr.half;
  for (int r = 0; r < tv.nrhs; ++r)
    for (int o0 = 0; o0 < nout; o0 += WAVE) {
      int o = o0 + lane;
      if (o >= nout) continue;
      int p = o - P;
      const double2* S = src + r * tv.ctot + tv.coff[par] + Pp;
      double2 acc = toeplitz_dot(T, S, Pp, p, 0, rev);
      double2* d = dst + r * tv.ctot + tv.coff[b] + o;
      *d = accumulate ? cadd(*d, acc) : acc;
    }
}

// ------------------------------------------------------------------ P2P (free space)
// u_i += (i/4) sum_{j in U(i), j != i} q_j H0^(1)(k |x_i - x_j|). One wave per
// target leaf; when the leaf holds fewer than 64 points several lanes share a
// target and split its sources, then combine by shuffles.
// Sources are staged through LDS 64 at a time; RB right-hand sides share each
// H0 evaluation (right-hand sides r0 .. r0+RB-1 in this launch).
template <int RB>
__global__ void __launch_bounds__(WAVE) k_p2p(TreeView tv, const int* __restrict__ leaves, int nleaves,
                                              const int* __restrict__ ptr, const int2* __restrict__ rng,
                                              const int* __restrict__ atomic, const double2* __restrict__ qs,
                                              double2* __restrict__ us, int r0) {
  __shared__ double2 s_x[WAVE];
  __shared__ double2 s_q[RB][WAVE];
  int li = blockIdx.x;
  if (li >= nleaves) return;
  int b = leaves[li];
  int lane = threadIdx.x;
  int2 pr = tv.prange[b];
  int e0 = ptr[li], e1 = ptr[li + 1];
  const double qk2 = 0.25 * tv.k * tv.k;
  // targets in chunks of 32 (two lanes per target), the remainder in a chunk of
  // the next power of two with more lanes per target
  for (int c0 = pr.x, csz = 0; c0 < pr.y; c0 += csz) {
    int rem = pr.y - c0;
    csz = 32;
    if (rem < 32) {
      csz = 1;
      while (csz < rem) csz *= 2;
    }
    int nt = min(csz, rem);
    int g = WAVE / csz;  // lanes per target
    int ti = lane / g, sub = lane % g;
    int i = c0 + ti;
    bool valid = ti < nt;
    double2 xi = valid ? tv.pts[i] : cmk(0, 0);
    double2 acc[RB];
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) acc[rr] = cmk(0, 0);
    for (int e = e0; e < e1; ++e) {
      int2 sr = rng[e];
      for (int j0 = sr.x; j0 < sr.y; j0 += WAVE) {
        int cnt = min(WAVE, sr.y - j0);
        __syncthreads();
        if (lane < cnt) {
          s_x[lane] = tv.pts[j0 + lane];
#pragma unroll
          for (int rr = 0; rr < RB; ++rr)
            s_q[rr][lane] = (r0 + rr < tv.nrhs) ? qs[(int64_t)(r0 + rr) * tv.n + j0 + lane] : cmk(0, 0);
        }
        __syncthreads();
        if (valid) {
          // four sources per step: z = (k r / 2)^2; dropped terms (the target
          // itself, past the chunk) get a harmless z = 1 and weight 0
          for (int jj = sub; jj < cnt; jj += 4 * g) {
            double z[4];
            bool use[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              int jl = jj + u * g;
              use[u] = jl < cnt && (j0 + jl) != i;
              double2 xj = s_x[use[u] ? jl : 0];
              double dx = xi.x - xj.x, dy = xi.y - xj.y;
              z[u] = use[u] ? qk2 * (dx * dx + dy * dy) : 1.0;
            }
            double2 h[4];
            hankel0_x4(z, h);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if (!use[u]) continue;
              int jl = jj + u * g;
#pragma unroll
              for (int rr = 0; rr < RB; ++rr) acc[rr] = cadd(acc[rr], cmul(h[u], s_q[rr][jl]));
            }
          }
        }
      }
    }
#pragma unroll
    for (int rr = 0; rr < RB; ++rr)
      for (int m = 1; m < g; m <<= 1) acc[rr] = cadd(acc[rr], shfl_xor_c(acc[rr], m));
    if (valid && sub == 0)
#pragma unroll
      for (int rr = 0; rr < RB; ++rr)
        if (r0 + rr < tv.nrhs) {
          int64_t idx = (int64_t)(r0 + rr) * tv.n + i;
          double2 v = cmk(-0.25 * acc[rr].y, 0.25 * acc[rr].x);  // (i/4) acc
          if (atomic[li]) {
            unsafeAtomicAdd(&us[idx].x, v.x);
            unsafeAtomicAdd(&us[idx].y, v.y);
          } else {
            us[idx] = cadd(us[idx], v);
          }
        }
  }
}

// ------------------------------------------------------------------ near-interface direct
// u_i += sum_j q_j G^s(x_i, x_j) for image pairs that are not admissible, with
// G^s = sum_q c_q exp(ky_q (y_i + y_j) + kx_q (x_i - x_j)) the Sommerfeld
// integral under a fixed rule (the propagating tau part and the evanescent t
// part on a contour below the real-axis singularities). The sum over sources
// moves inside the rule: per node S_q = sum_j q_j exp(ky_q y_j - kx_q x_j).
__global__ void __launch_bounds__(WAVE) k_iface(TreeView tv, const int* __restrict__ leaves, int nleaves,
                                                const int* __restrict__ ptr, const int2* __restrict__ rng,
                                                int nq, const double2* __restrict__ qc, const double2* __restrict__ qky,
                                                const double2* __restrict__ qkx, const double2* __restrict__ qs,
                                                double2* __restrict__ us) {
  __shared__ double2 s_c[WAVE], s_ky[WAVE], s_kx[WAVE];
  int li = blockIdx.x;
  if (li >= nleaves) return;
  int b = leaves[li];
  int lane = threadIdx.x;
  int2 pr = tv.prange[b];
  double xref = tv.ctr[b].x;
  for (int r = 0; r < tv.nrhs; ++r) {
    for (int c0 = pr.x; c0 < pr.y; c0 += WAVE) {
      int i = c0 + lane;
      bool valid = i < pr.y;
      double2 xi = valid ? tv.pts[i] : cmk(0, 0);
      double2 acc = cmk(0, 0);
      for (int e = ptr[li]; e < ptr[li + 1]; ++e) {
        int2 sr = rng[e];
        for (int q0 = 0; q0 < nq; q0 += WAVE) {
          int q = q0 + lane;
          double2 sq = cmk(0, 0), ky = cmk(0, 0), kx = cmk(0, 0), cq = cmk(0, 0);
          if (q < nq) {
            ky = qky[q]; kx = qkx[q]; cq = qc[q];
            for (int j = sr.x; j < sr.y; ++j) {
              double2 xj = tv.pts[j];
              double2 ex = cadd(cscale(ky, xj.y), cscale(kx, -(xj.x - xref)));
              sq = cadd(sq, cmul(qs[(int64_t)r * tv.n + j], cexp2(ex)));
            }
          }
          __syncthreads();
          s_c[lane] = cmul(cq, sq);
          s_ky[lane] = ky;
          s_kx[lane] = kx;
          __syncthreads();
          int qn = min(WAVE, nq - q0);
          if (valid)
            for (int qq = 0; qq < qn; ++qq) {
              double2 ex = cadd(cscale(s_ky[qq], xi.y), cscale(s_kx[qq], xi.x - xref));
              acc = cadd(acc, cmul(s_c[qq], cexp2(ex)));
            }
        }
      }
      if (valid) {
        int64_t idx = (int64_t)r * tv.n + i;
        us[idx] = cadd(us[idx], acc);
      }
    }
  }
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
// poles of sigma_1. One block per (X, Y); a thread owns 8 consecutive orders.
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
};

constexpr int TB_THREADS = 256;
constexpr int TB_NB = 8;

__global__ void __launch_bounds__(TB_THREADS) k_table_image(ImageTableArgs a) {
  __shared__ double2 s_l0a[TB_THREADS], s_lsa[TB_THREADS], s_l0b[TB_THREADS], s_lsb[TB_THREADS];
  __shared__ int s_kind[TB_THREADS];
  int cb = blockIdx.x;
  if (cb >= a.ncombo) return;
  int tid = threadIdx.x;
  const double k = a.med.k1;
  const double X = a.X[cb], Y = a.Y[cb];
  const double dip = a.dip[cb], send = a.send[cb];
  TableRef tr = a.refs[cb];
  const int N = tr.half;
  const int n0 = -N + TB_NB * tid;
  // class "i":  i^n * sum exp(l0 + n ls)   (tau nodes; t nodes' minus branch)
  // class "mi": (-i)^n * sum exp(l0 + n ls) (t nodes' plus branch)
  double2 acc_i[TB_NB], acc_mi[TB_NB];
  for (int j = 0; j < TB_NB; ++j) { acc_i[j] = cmk(0, 0); acc_mi[j] = cmk(0, 0); }
  const int p0 = a.pbeg[cb], p1 = a.pbeg[cb + 1];
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
    if (n0 <= N) {
      int qn = min(TB_THREADS, nnode - q0);
      for (int qq = 0; qq < qn; ++qq) {
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
  double2* T = a.tdata + tr.off + tr.half;
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
void launch_scatter(hipStream_t s, int n, int nrhs, const int* perm, const double2* src, double2* dst, int cj) {
  int64_t tot = (int64_t)n * nrhs;
  hipLaunchKernelGGL(k_scatter, dim3(blocks(tot, 256)), dim3(256), 0, s, n, nrhs, perm, src, dst, cj);
}
void launch_p2m(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const double2* qs, double2* alpha,
                int conj_w, double2 pref) {
  if (nl) hipLaunchKernelGGL(k_p2m, dim3(nl), dim3(WAVE), 0, s, tv, leaves, nl, qs, alpha, conj_w, pref);
}
void launch_l2p(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const double2* beta, double2* us,
                int conj_w, double2 pref, int accumulate) {
  if (nl) hipLaunchKernelGGL(k_l2p, dim3(nl), dim3(WAVE), 0, s, tv, leaves, nl, beta, us, conj_w, pref, accumulate);
}
void launch_m2l(hipStream_t s, const TreeView& tv, const int* targets, int nt, const int* ptr, const M2LEntry* ent,
                const TableRef* tabs, const double2* tdata, const double2* src, double2* dst, int rev) {
  if (nt) hipLaunchKernelGGL(k_m2l, dim3(nt), dim3(WAVE), 0, s, tv, targets, nt, ptr, ent, tabs, tdata, src, dst, rev);
}
// LDS bytes of an M2L item at order P.
static size_t m2l_lds_bytes(int P) {
  int M = 2 * P + 1;
  int npi = (M <= 64) ? 64 : 16;
  return sizeof(double2) * (size_t)(4 * P + 1 + npi * M);
}

void launch_m2l_mfma(hipStream_t s, const TreeView& tv, const M2LItem* items, const int* item_level_first,
                     int nlev, const int* psrc, const int* pdst, const TableRef* tabs, const double2* tdata,
                     const double2* src, double2* dst, int rev) {
  static bool attr_done = false;
  if (!attr_done) {
    (void)hipFuncSetAttribute((const void*)k_m2l_mfma<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipFuncSetAttribute((const void*)k_m2l_mfma<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr_done = true;
  }
  // items are grouped by level (item_level_first[l] .. item_level_first[l+1]);
  // one launch per level with that level's LDS size
  for (int l = 0; l < nlev; ++l) {
    int i0 = item_level_first[l], i1 = item_level_first[l + 1];
    if (i1 <= i0) continue;
    size_t lds = m2l_lds_bytes(tv.P[l]);
    for (int r = 0; r < tv.nrhs; ++r) {
      if (rev)
        hipLaunchKernelGGL(k_m2l_mfma<true>, dim3(i1 - i0), dim3(M2L_THREADS), lds, s, tv, items + i0, psrc, pdst,
                           tabs, tdata, src, dst, r);
      else
        hipLaunchKernelGGL(k_m2l_mfma<false>, dim3(i1 - i0), dim3(M2L_THREADS), lds, s, tv, items + i0, psrc, pdst,
                           tabs, tdata, src, dst, r);
    }
  }
}

void launch_fill_zero(hipStream_t s, double2* p, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_fill_zero, dim3(blocks(n, 256)), dim3(256), 0, s, p, n);
}

void launch_m2m(hipStream_t s, const TreeView& tv, const int* boxes, int nb, const TableRef* tabs4,
                const double2* tdata, const double2* src, double2* dst, int rev) {
  if (nb) hipLaunchKernelGGL(k_m2m, dim3(nb), dim3(WAVE), 0, s, tv, boxes, nb, tabs4, tdata, src, dst, rev);
}
void launch_l2l(hipStream_t s, const TreeView& tv, const int* boxes, int nb, const TableRef* tabs4,
                const double2* tdata, const double2* src, double2* dst, int rev, int accumulate) {
  if (nb) hipLaunchKernelGGL(k_l2l, dim3(nb), dim3(WAVE), 0, s, tv, boxes, nb, tabs4, tdata, src, dst, rev, accumulate);
}
void launch_p2p(hipStream_t s, const TreeView& tv, const int* items, int nl, const int* ptr, const int2* rng,
                const int* atomic, const double2* qs, double2* us) {
  if (!nl) return;
  if (tv.nrhs == 1) {
    hipLaunchKernelGGL(k_p2p<1>, dim3(nl), dim3(WAVE), 0, s, tv, items, nl, ptr, rng, atomic, qs, us, 0);
    return;
  }
  for (int r0 = 0; r0 < tv.nrhs; r0 += 4)
    hipLaunchKernelGGL(k_p2p<4>, dim3(nl), dim3(WAVE), 0, s, tv, items, nl, ptr, rng, atomic, qs, us, r0);
}
void launch_iface(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const int* ptr, const int2* rng,
                  int nq, const double2* qc, const double2* qky, const double2* qkx, const double2* qs, double2* us) {
  if (nl && nq) hipLaunchKernelGGL(k_iface, dim3(nl), dim3(WAVE), 0, s, tv, leaves, nl, ptr, rng, nq, qc, qky, qkx, qs, us);
}
void launch_table_hankel(hipStream_t s, int ntab, const double* dx, const double* dy, const TableRef* refs, double k,
                         double2* tdata) {
  if (ntab) hipLaunchKernelGGL(k_table_hankel, dim3(blocks(ntab, 64)), dim3(64), 0, s, ntab, dx, dy, refs, k, tdata);
}
void launch_table_bessel(hipStream_t s, int ntab, const double* dx, const double* dy, const int* sgn,
                         const TableRef* refs, double k, double2* tdata) {
  if (ntab) hipLaunchKernelGGL(k_table_bessel, dim3(blocks(ntab, 64)), dim3(64), 0, s, ntab, dx, dy, sgn, refs, k, tdata);
}
void launch_table_image(hipStream_t s, const Medium& med, int ncombo, const double* X, const double* Y,
                        const double* dip, const double* send, const int* pbeg, const Panel* panels,
                        const TableRef* refs, const double* glx, const double* glw, double2* tdata) {
  if (!ncombo) return;
  ImageTableArgs a{med, ncombo, X, Y, dip, send, pbeg, panels, refs, glx, glw, tdata};
  hipLaunchKernelGGL(k_table_image, dim3(ncombo), dim3(TB_THREADS), 0, s, a);
}

}  // namespace hfmm
