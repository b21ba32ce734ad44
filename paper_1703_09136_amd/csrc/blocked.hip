// Kernels of the right-hand-side-blocked pipeline (see blocked.hpp): with
// many right-hand sides every stage of Algorithm 1 is a contraction whose N
// dimension is the right-hand sides, run on the matrix cores.
//
// Complex products go through the interleaved real embedding: real row 2p
// (2p + 1) of an operator holds the real (imaginary) part of output p, real
// column 2m (2m + 1) multiplies the real (imaginary) part of input m, so
//   A[2p][2m] = Re T, A[2p][2m+1] = -Im T, A[2p+1][2m] = Im T, A[2p+1][2m+1] = Re T,
// and a blocked complex row X[m][r] read as doubles is the real column pair
// (2m, 2m + 1) of the B operand. Each lane of an MFMA then reads one operand
// element per step whose kind (Re T, Im T or -Im T) depends only on the lane,
// so the operator is staged as planes and read without branches.
//
// MFMA lane layouts (gfx950): for 16x16x4 (FP64, FP32) a lane supplies
// A[lane % 16][lane / 16] and B[lane / 16][lane % 16]; for 16x16x32 BF16
// A[lane % 16][8 (lane / 16) + t] and B[8 (lane / 16) + t][lane % 16], t < 8.
// The result D[row][lane % 16] sits in register i with row = 4 i + lane / 16
// (FP64) or row = 4 (lane / 16) + i (FP32 and BF16 accumulation).
#include "blocked.hpp"
#include "kernels.hpp"
#include "special.hpp"

namespace hfmm {

constexpr int WAVE = 64;
constexpr int BLK_THREADS = 256;
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __noinline__ double2 hankel0_large_call(double x) { return hankel0_large(x); }


// ------------------------------------------------------------------ layout changes
__global__ void k_gather_blk(int n, int nc, int Rp, const int* __restrict__ perm, const double2* __restrict__ q,
                             double2* __restrict__ qb) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * Rp) return;
  const int j = (int)(idx / Rp), r = (int)(idx % Rp);
  qb[idx] = r < nc ? q[(int64_t)r * n + perm[j]] : cmk(0.0, 0.0);
}

__global__ void k_scatter_blk(int n, int nc, int Rp, const int* __restrict__ perm, const double2* __restrict__ ub,
                              double2* __restrict__ u, const double2* __restrict__ diag,
                              const double2* __restrict__ qb) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * Rp) return;
  const int j = (int)(idx / Rp), r = (int)(idx % Rp);
  if (r >= nc) return;
  double2 v = ub[idx];
  if (diag) v = csub(v, cmul(diag[j], qb[idx]));
  u[(int64_t)r * n + perm[j]] = v;
}

__global__ void k_to_f32(int64_t count, const double2* __restrict__ src, float2* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}

// ------------------------------------------------------------------ expansion matrices
// V[m][j] = J_m(k rho_j) e^{-i m theta_j} (m in [-P, P], rho, theta the polar
// form of x_j - centre) for the points of every leaf, stored per leaf as
// [2P + 1][npts] at voff[leaf]. P2M is alpha = V q; L2P uses conj(V)^T.
// One thread per point walks the Miller recurrence once.
__global__ void k_vmat(TreeView tv, const int* __restrict__ leaves, int nl, const int64_t* __restrict__ voff,
                       double2* __restrict__ V) {
  const int li = blockIdx.x;
  if (li >= nl) return;
  const int b = leaves[li];
  const int P = tv.P[tv.level[b]];
  const int2 pr = tv.prange[b];
  const int np = pr.y - pr.x;
  const double2 c = tv.ctr[b];
  double2* Vl = V + voff[li];
  for (int jl = threadIdx.x; jl < np; jl += blockDim.x) {
    const double2 p = tv.pts[pr.x + jl];
    const double dx = p.x - c.x, dy = p.y - c.y;
    const double rho = hypot(dx, dy);
    const double x = fmax(tv.k * rho, kTinyX), s1 = tv.k * rho < kTinyX ? tv.k * rho / kTinyX : 1.0;
    const double2 w = rho > 0 ? cmk(dx / rho, -dy / rho) : cmk(1.0, 0.0);  // e^{-i theta}
    double2 wn = cpowi(w, P);
    const int nstart = miller_start_expansion(tv.k * rho, P);
    double inv_s;
    int nres;
    miller_norm(x, nstart, inv_s, nres);
    MillerWalk mw(x, nstart, inv_s, nres);
    while (mw.n > P) mw.step();
    for (int m = P; m >= 0; --m) {
      const double jm = m == 1 ? s1 * mw.value() : mw.value();
      const double2 v = cscale(wn, jm);
      Vl[(int64_t)(P + m) * np + jl] = v;
      // J_{-m} = (-1)^m J_m and e^{i m theta} = conj(w^m)
      if (m > 0) Vl[(int64_t)(P - m) * np + jl] = cscale(cconj(wn), (m & 1) ? -jm : jm);
      wn = cmul(wn, cconj(w));
      if (m > 0) mw.step();
    }
  }
}

// alpha[c_b + m][r] = sum_j V[m][j] q[j][r] for one leaf, 64 right-hand sides
// per block (grid y), a 16-column tile per wave, all row tiles of the leaf's
// 2(2P + 1) real rows per wave (at most kBlkLeafPmax). The V chunk (32
// points) is staged in LDS as planes (Re V, Im V, -Im V).
constexpr int P2M_PC = 32;
constexpr int BLK_MAX_RT = (2 * (2 * kBlkLeafPmax + 1) + 15) / 16;

__global__ void __launch_bounds__(BLK_THREADS) k_p2m_blk(TreeView tv, int Rp, const int* __restrict__ leaves,
                                                         int nl, const int64_t* __restrict__ voff,
                                                         const double2* __restrict__ V, const double2* __restrict__ qb,
                                                         double2* __restrict__ ab) {
  extern __shared__ double lds[];
  const int li = blockIdx.x;
  if (li >= nl) return;
  const int b = leaves[li];
  const int P = tv.P[tv.level[b]];
  const int Md = 2 * P + 1;
  const int2 pr = tv.prange[b];
  const int np = pr.y - pr.x;
  const double2* Vl = V + voff[li];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = blockIdx.y * kBlkCols + wave * 16 + (lane & 15);
  const int nrt = (2 * Md + 15) / 16;
  const int kl = lane >> 4;
  // lane's operand plane and row offset per row tile: row R = 16 rt + lane % 16
  const int rp = lane & 1, kp = kl & 1;
  const int plane = (rp == kp) ? 0 : (rp ? 1 : 2);
  d4 acc[BLK_MAX_RT];
#pragma unroll
  for (int j = 0; j < BLK_MAX_RT; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
  double* Lr = lds;                     // [Md][P2M_PC] real parts
  double* Li = Lr + Md * P2M_PC;        // imaginary parts
  double* Ln = Li + Md * P2M_PC;        // negated imaginary parts
  const double* Lp = plane == 0 ? Lr : plane == 1 ? Li : Ln;
  for (int j0 = 0; j0 < np; j0 += P2M_PC) {
    const int nj = min(P2M_PC, np - j0);
    __syncthreads();
    for (int e = tid; e < Md * P2M_PC; e += BLK_THREADS) {
      const int m = e / P2M_PC, jj = e - m * P2M_PC;
      const double2 v = jj < nj ? Vl[(int64_t)m * np + j0 + jj] : cmk(0.0, 0.0);
      Lr[e] = v.x;
      Li[e] = v.y;
      Ln[e] = -v.y;
    }
    __syncthreads();
    // k = 2 jj + part over the chunk's points, four per step
    const int nks = (2 * nj + 3) / 4;
    for (int ks = 0; ks < nks; ++ks) {
      const int jj = 2 * ks + (kl >> 1);
      const double bq = jj < nj ? ((const double*)(qb + (int64_t)(pr.x + j0 + jj) * Rp + col))[kp] : 0.0;
#pragma unroll
      for (int j = 0; j < BLK_MAX_RT; ++j) {
        if (j < nrt) {
          const int R = 16 * j + (lane & 15);
          const int m = R < 2 * Md ? R >> 1 : 0;
          const double a = Lp[m * P2M_PC + jj];
          acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bq, acc[j], 0, 0, 0);
        }
      }
    }
  }
  const int64_t cb = tv.coff[b];
#pragma unroll
  for (int j = 0; j < BLK_MAX_RT; ++j) {
    if (j >= nrt) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int R = 16 * j + 4 * i + kl;
      if (R < 2 * Md) ((double*)(ab + (cb + (R >> 1)) * Rp + col))[R & 1] = acc[j][i];
    }
  }
}

// u[j][r] += (i/4) sum_m conj(V[m][j]) beta[c_b + m][r] for the points of one
// leaf: rows are the leaf's points (2 np real rows, 64 points per group of
// eight row tiles), k the 2(2P + 1) real orders. The embedding of conj(V):
// [2j][2m] = Re V, [2j][2m+1] = Im V, [2j+1][2m] = -Im V, [2j+1][2m+1] = Re V;
// V is staged in LDS sixteen orders at a time as planes (Re V, Im V, -Im V).
constexpr int L2P_MC = 16;
__global__ void __launch_bounds__(BLK_THREADS) k_l2p_blk(TreeView tv, int Rp, const int* __restrict__ leaves,
                                                         int nl, const int64_t* __restrict__ voff,
                                                         const double2* __restrict__ V, const double2* __restrict__ bb,
                                                         double2* __restrict__ ub) {
  __shared__ double s_v[3][L2P_MC][64];
  const int li = blockIdx.x;
  if (li >= nl) return;
  const int b = leaves[li];
  const int P = tv.P[tv.level[b]];
  const int Md = 2 * P + 1;
  const int2 pr = tv.prange[b];
  const int np = pr.y - pr.x;
  const double2* Vl = V + voff[li];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = blockIdx.y * kBlkCols + wave * 16 + (lane & 15);
  const int kl = lane >> 4;
  const int rp = lane & 1, kp = kl & 1;
  const int plane = (rp == kp) ? 0 : (rp ? 2 : 1);
  const int64_t cb = tv.coff[b];
  for (int g0 = 0; g0 < np; g0 += 64) {  // groups of 64 points: 8 row tiles
    const int ng = min(64, np - g0);
    const int nrt = (2 * ng + 15) / 16;
    d4 acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
    for (int m0 = 0; m0 < Md; m0 += L2P_MC) {
      __syncthreads();
      for (int e = tid; e < L2P_MC * 64; e += BLK_THREADS) {
        const int mi = e >> 6, jp = e & 63;
        const double2 v = (m0 + mi < Md && jp < ng) ? Vl[(int64_t)(m0 + mi) * np + g0 + jp] : cmk(0.0, 0.0);
        s_v[0][mi][jp] = v.x;
        s_v[1][mi][jp] = v.y;
        s_v[2][mi][jp] = -v.y;
      }
      __syncthreads();
      const int nks = (2 * min(L2P_MC, Md - m0) + 3) / 4;
      for (int ks = 0; ks < nks; ++ks) {
        const int mi = 2 * ks + (kl >> 1);
        const int m = m0 + mi;
        const double bq = m < Md ? ((const double*)(bb + (cb + m) * Rp + col))[kp] : 0.0;
        const double* Lp = &s_v[plane][mi][0];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (j < nrt) {
            const int R = 16 * j + (lane & 15);
            const double a = Lp[R < 2 * ng ? (R >> 1) : 0];
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bq, acc[j], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j >= nrt) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // (i/4) z: the real row takes -Im z / 4, the imaginary row Re z / 4;
        // the partner row (R ^ 1) sits in the lane 16 apart (kl ^ 1)
        const int R = 16 * j + 4 * i + kl;
        const double other = __shfl_xor(acc[j][i], 16, WAVE);
        if (R < 2 * ng) {
          double* o = (double*)(ub + (int64_t)(pr.x + g0 + (R >> 1)) * Rp + col) + (R & 1);
          *o += (R & 1) ? 0.25 * other : -0.25 * other;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ translations
// Toeplitz planes of one table in LDS: Re T, Im T, -Im T, -Re T, each of
// stride ntp with value n at index kTabPadB + n and zeros around.
constexpr int kTabPadB = 4;
__host__ __device__ inline int tg_table_stride(int nt) { return (nt + 2 * kTabPadB + 1) & ~1; }

// Per-lane plane of the FP64 operator element: free pairs read
// {Re, -Im, Im, Re}[(rp, kp)], image pairs the same with the sign (-1)^m'
// (constant per lane, m' = 2 ks + kl / 2 shifted by Ps).
__device__ inline int tg_plane(int rp, int kp, bool neg) {
  // planes: 0 Re, 1 Im, 2 -Im, 3 -Re
  int pl = (rp == kp) ? 0 : (rp ? 1 : 2);
  if (neg) pl = pl == 0 ? 3 : (pl == 1 ? 2 : 1);
  return pl;
}

template <int PREC>
struct TgTraits;
template <>
struct TgTraits<BLK_F64> {
  using acc_t = d4;
};
template <>
struct TgTraits<BLK_F32> {
  using acc_t = f4;
};
template <>
struct TgTraits<BLK_BF16> {
  using acc_t = f4;
};

// dst rows of item t = (add ? dst : 0) + sum_pairs Op_pair src_pair. Block:
// one item, 64 right-hand sides (grid y), wave w the columns 16 w .. 16 w + 15,
// all nt row tiles of the item. FP64: A from the Toeplitz planes of each pair's
// table (staged per pair), B from the blocked FP64 source rows. FP32 / BF16:
// the pair's operator scaled by a_s(|m|) a_t(|p|) is built in LDS for the
// item's rows (FP32 planes, or BF16 real-embedded rows), B from the scaled
// low-precision source rows; the FP32 accumulators are divided by a_t(|p|) in
// FP64 at the end. Items are spread over the XCDs in contiguous runs: the
// grid has a multiple of 8 blocks and block b (dispatched to XCD b mod 8)
// takes item (b mod 8) * ceil(n / 8) + b / 8, so neighbouring targets, which
// share source boxes, share an L2.
template <int PREC>
__global__ void __launch_bounds__(BLK_THREADS) k_tgemm(int Rp, const TgItem* __restrict__ items, int nitems,
                                                       const TgPair* __restrict__ pairs,
                                                       const double2* __restrict__ tdata,
                                                       const double2* __restrict__ src, const void* __restrict__ src_lo,
                                                       const double* __restrict__ scale, int sstride,
                                                       double2* __restrict__ dst, int add, int lds_rows) {
  extern __shared__ double lds[];
  using acc_t = typename TgTraits<PREC>::acc_t;
  const int per_xcd = (nitems + 7) / 8;
  const int it_id = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (it_id >= nitems) return;
  const TgItem it = items[it_id];
  const int Ps = it.Ps, Pd = it.Pd;
  const int Ms = 2 * Ps + 1, Md = 2 * Pd + 1;
  const int nt_tab = 2 * (Ps + Pd) + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kl = lane >> 4;
  const int col = blockIdx.y * kBlkCols + wave * 16 + (lane & 15);
  const int rp = lane & 1, kp = kl & 1;
  acc_t acc[kTgMaxNt];
#pragma unroll
  for (int j = 0; j < kTgMaxNt; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[j][i] = 0;
  // reduced precision: each pair's contraction accumulates in FP32 on the
  // matrix cores and is added to these FP64 sums (one FP32 chain per pair,
  // not one over all the pairs of a target)
  constexpr int NT64 = PREC == BLK_F64 ? 1 : kTgMaxNt;
  double acc64[NT64][4];
#pragma unroll
  for (int j = 0; j < NT64; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc64[j][i] = 0.0;
  // lane's output order index per row tile (rows past 2 Md use index 0)
  int pidx[kTgMaxNt];
#pragma unroll
  for (int j = 0; j < kTgMaxNt; ++j) {
    const int R = 16 * (it.rt0 + j) + (lane & 15);
    pidx[j] = (j < it.nt && R < 2 * Md) ? (R >> 1) : 0;
  }
  const int p_lo = 8 * it.rt0;  // first complex row of the item
  const int nrow = min(8 * it.nt, Md - p_lo);
  for (int e = it.pbeg; e < it.pend; ++e) {
    const TgPair pa = pairs[e];
    __syncthreads();  // the previous pair's operator is no longer read
    if constexpr (PREC == BLK_F64) {
      const int ntp = tg_table_stride(nt_tab);
      const double2* T = tdata + pa.toff;
      for (int i = tid; i < ntp; i += BLK_THREADS) {
        const int n = i - kTabPadB;
        const double2 v = (n >= 0 && n < nt_tab) ? T[n] : cmk(0.0, 0.0);
        lds[i] = v.x;
        lds[ntp + i] = v.y;
        lds[2 * ntp + i] = -v.y;
        lds[3 * ntp + i] = -v.x;
      }
      __syncthreads();
      // free: index 2 Pd - p + m; image: 2 Ps + 2 Pd - p - m', sign (-1)^(m' + Ps)
      const bool img = pa.image != 0;
      const bool neg = img && (((kl >> 1) + Ps) & 1);
      const double* Lp = lds + tg_plane(rp, kp, neg) * ntp + kTabPadB;
      int base[kTgMaxNt];
#pragma unroll
      for (int j = 0; j < kTgMaxNt; ++j)
        base[j] = img ? 2 * Ps + 2 * Pd - pidx[j] - (kl >> 1) : 2 * Pd - pidx[j] + (kl >> 1);
      const int step = img ? -2 : 2;
      const int nks = (2 * Ms + 3) / 4;
      const double* S = (const double*)(src + pa.cs * Rp + col) + kp;
      const int64_t rs = 2 * (int64_t)Rp;  // doubles per source row
      double b0 = (kl >> 1) < Ms ? S[(int64_t)(kl >> 1) * rs] : 0.0;
      for (int ks = 0; ks < nks; ++ks) {
        const int mn = 2 * (ks + 1) + (kl >> 1);
        const double b1 = mn < Ms ? S[(int64_t)mn * rs] : 0.0;
#pragma unroll
        for (int j = 0; j < kTgMaxNt; ++j) {
          if (j < it.nt) {
            const double a = Lp[base[j] + step * ks];
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, acc[j], 0, 0, 0);
          }
        }
        b0 = b1;
      }
    } else {
      // scaled operator rows p_lo .. p_lo + nrow - 1 for this pair
      const double2* T = tdata + pa.toff;
      const double* sa = scale + it.lev * sstride;  // same level for source and target
      const bool img = pa.image != 0;
      if constexpr (PREC == BLK_F32) {
        const int Ms2 = Ms + 1;  // even: k-steps of two orders
        float* Or = (float*)lds;
        float* Oi = Or + lds_rows * Ms2;
        float* On = Oi + lds_rows * Ms2;
        for (int e2 = tid; e2 < nrow * Ms2; e2 += BLK_THREADS) {
          const int pl = e2 / Ms2, m = e2 - pl * Ms2;
          const int p = p_lo + pl;
          double2 v = cmk(0.0, 0.0);
          if (m < Ms) {
            const int pp = p - Pd, mm = m - Ps;
            const int idx = img ? -mm - pp + Ps + Pd : mm - pp + Ps + Pd;
            v = T[idx];
            const double s = sa[mm < 0 ? -mm : mm] * sa[pp < 0 ? -pp : pp] * ((img && ((mm & 1) != 0)) ? -1.0 : 1.0);
            v = cscale(v, s);
          }
          Or[e2] = (float)v.x;
          Oi[e2] = (float)v.y;
          On[e2] = -(float)v.y;
        }
        __syncthreads();
        const int pl_sel = (rp == kp) ? 0 : (rp ? 1 : 2);
        const float* Lp = (pl_sel == 0 ? Or : pl_sel == 1 ? Oi : On);
        int rowoff[kTgMaxNt];
#pragma unroll
        for (int j = 0; j < kTgMaxNt; ++j) rowoff[j] = (pidx[j] - p_lo >= 0 ? pidx[j] - p_lo : 0) * Ms2 + (kl >> 1);
        const int nks = Ms2 / 2;
        const float* S = (const float*)src_lo + (pa.cs * Rp + col) * 2 + kp;
        const int64_t rs = 2 * (int64_t)Rp;
        float b0 = (kl >> 1) < Ms ? S[(int64_t)(kl >> 1) * rs] : 0.0f;
        for (int ks = 0; ks < nks; ++ks) {
          const int mn = 2 * (ks + 1) + (kl >> 1);
          const float b1 = mn < Ms ? S[(int64_t)mn * rs] : 0.0f;
#pragma unroll
          for (int j = 0; j < kTgMaxNt; ++j) {
            if (j < it.nt) {
              const float a = Lp[rowoff[j] + 2 * ks];
              acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b0, acc[j], 0, 0, 0);
            }
          }
          b0 = b1;
        }
      } else {
        // BF16: rows 2p + rp of the real embedding, k = 2m + kp, Ms16 orders
        const int Ms16 = (Ms + 15) & ~15;
        const int K = 2 * Ms16;
        __bf16* A = (__bf16*)lds;  // [2 nrow][K]
        for (int e2 = tid; e2 < nrow * Ms16; e2 += BLK_THREADS) {
          const int pl = e2 / Ms16, m = e2 - pl * Ms16;
          const int p = p_lo + pl;
          double2 v = cmk(0.0, 0.0);
          if (m < Ms) {
            const int pp = p - Pd, mm = m - Ps;
            const int idx = img ? -mm - pp + Ps + Pd : mm - pp + Ps + Pd;
            v = T[idx];
            const double s = sa[mm < 0 ? -mm : mm] * sa[pp < 0 ? -pp : pp] * ((img && ((mm & 1) != 0)) ? -1.0 : 1.0);
            v = cscale(v, s);
          }
          __bf16* r0 = A + (int64_t)(2 * pl) * K + 2 * m;
          __bf16* r1 = r0 + K;
          r0[0] = (__bf16)(float)v.x;
          r0[1] = (__bf16)(float)(-v.y);
          r1[0] = (__bf16)(float)v.y;
          r1[1] = (__bf16)(float)v.x;
        }
        __syncthreads();
        int rowoff[kTgMaxNt];
#pragma unroll
        for (int j = 0; j < kTgMaxNt; ++j) {
          const int R = 16 * (it.rt0 + j) + (lane & 15);
          const int rl = R - 2 * p_lo;
          rowoff[j] = (j < it.nt && rl >= 0 && rl < 2 * nrow ? rl : 0) * K + 8 * kl;
        }
        const int nks = Ms16 / 16;
        // B: four consecutive orders of one right-hand side (16 bytes); the
        // source's BF16 rows are laid out [Rp][Ms16] from cs16 * Rp
        const __bf16* Src = (const __bf16*)src_lo + 2 * (pa.cs16 * Rp + (int64_t)col * Ms16);
        for (int ks = 0; ks < nks; ++ks) {
          const bf8 bv = *(const bf8*)(Src + 2 * (16 * ks + 4 * kl));
#pragma unroll
          for (int j = 0; j < kTgMaxNt; ++j) {
            if (j < it.nt) {
              const bf8 av = *(const bf8*)(A + rowoff[j] + 32 * ks);
              acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[j], 0, 0, 0);
            }
          }
        }
      }
      if constexpr (PREC != BLK_F64) {
#pragma unroll
        for (int j = 0; j < NT64; ++j)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            acc64[j][i] += (double)acc[j][i];
            acc[j][i] = 0;
          }
      }
    }
  }
  // store / add: FP64 rows R = 4 i + kl, FP32 rows R = 4 kl + i within a tile
  const double* st = PREC == BLK_F64 ? nullptr : scale + it.lev * sstride;
#pragma unroll
  for (int j = 0; j < kTgMaxNt; ++j) {
    if (j >= it.nt) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int R = 16 * (it.rt0 + j) + (PREC == BLK_F64 ? 4 * i + kl : 4 * kl + i);
      if (R >= 2 * Md) continue;
      double v;
      if constexpr (PREC == BLK_F64) v = acc[j][i];
      else v = acc64[j < NT64 ? j : 0][i];
      if (PREC != BLK_F64) {
        const int pp = (R >> 1) - Pd;
        v /= st[pp < 0 ? -pp : pp];
      }
      double* o = (double*)(dst + (it.ct + (R >> 1)) * Rp + col) + (R & 1);
      *o = add ? *o + v : v;
    }
  }
}

// src_lo = src / a_l(|m|) for the boxes [b0, b1): FP32 in the blocked layout,
// or BF16 per box as [Rp][Ms16] (orders fastest, zero padded) at coff16[b] * Rp.
template <int PREC>
__global__ void k_scale_blk(TreeView tv, int Rp, int b0, const double* __restrict__ scale, int sstride,
                            const int64_t* __restrict__ coff16, const double2* __restrict__ src,
                            void* __restrict__ src_lo) {
  const int b = b0 + blockIdx.x;
  const int lev = tv.level[b];
  if (lev < 2) return;
  const int P = tv.P[lev], Ms = 2 * P + 1;
  const double* sa = scale + lev * sstride;
  const int64_t cb = tv.coff[b];
  if (PREC == BLK_F32) {
    float2* d = (float2*)src_lo;
    for (int e = threadIdx.x; e < Ms * Rp; e += blockDim.x) {
      const int m = e / Rp, r = e - m * Rp;
      const int mm = m - P;
      const double inv = 1.0 / sa[mm < 0 ? -mm : mm];
      const double2 v = src[(cb + m) * Rp + r];
      d[(cb + m) * Rp + r] = make_float2((float)(v.x * inv), (float)(v.y * inv));
    }
  } else {
    const int Ms16 = (Ms + 15) & ~15;
    __bf16* d = (__bf16*)src_lo + 2 * coff16[b] * Rp;
    for (int e = threadIdx.x; e < Ms16 * Rp; e += blockDim.x) {
      const int r = e / Ms16, m = e - r * Ms16;
      double2 v = cmk(0.0, 0.0);
      if (m < Ms) {
        const int mm = m - P;
        v = cscale(src[(cb + m) * Rp + r], 1.0 / sa[mm < 0 ? -mm : mm]);
      }
      d[2 * (int64_t)e] = (__bf16)(float)v.x;
      d[2 * (int64_t)e + 1] = (__bf16)(float)v.y;
    }
  }
}

// ------------------------------------------------------------------ direct pairs
// ub[i][r] += (i/4) sum_j H0^(1)(k |x_i - x_j|) qb[j][r] (i != j) for up to 16
// targets of an item against its source ranges. A block takes every right-
// hand side of the pass (wave w: column tiles w, w + 4, ... of 16), so each
// H0 tile is evaluated once: 16 targets x 64 sources per chunk, four
// evaluations per thread, staged in LDS as planes (Re G, Im G, -Im G) and
// applied on the matrix cores (FP64, or FP32 with the FP32 series and
// strengths).
constexpr int BP_SC = 64;  // sources per chunk
constexpr int BP_MAX_CTW = 4;  // column tiles per wave (256 right-hand sides per block)

template <int PREC, int CLS>
__global__ void __launch_bounds__(BLK_THREADS) k_p2p_blk(TreeView tv, int Rp, const BpItem* __restrict__ items,
                                                         int nitems, const int2* __restrict__ rng,
                                                         const double2* __restrict__ qb, const void* __restrict__ qb_lo,
                                                         double2* __restrict__ ub) {
  using T = typename std::conditional<PREC == BLK_F64, double, float>::type;
  using acc_t = typename std::conditional<PREC == BLK_F64, d4, f4>::type;
  constexpr int CL = CLS < kH0Classes ? CLS : kH0Classes - 1;
  constexpr int M = PREC == BLK_F64 ? kH0ClassTerms[CL] : kH0ClassTermsF32[CL];
  constexpr bool LARGE = CLS >= kH0Classes;
  __shared__ T s_g[3][16][BP_SC];
  __shared__ double2 s_ln[1 << kLogTabBits];
  __shared__ double2 s_xs[BP_SC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (PREC == BLK_F64)
    for (int l = tid; l < (1 << kLogTabBits); l += BLK_THREADS) s_ln[l] = cmk(kLogTab[l][0], kLogTab[l][1]);
  const int per_xcd = (nitems + 7) / 8;
  const int it_id = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (it_id >= nitems) return;
  const BpItem it = items[it_id];
  const int kl = lane >> 4, rp = lane & 1, kp = kl & 1;
  const int plane = (rp == kp) ? 0 : (rp ? 1 : 2);
  const int c0 = blockIdx.y * (4 * 16 * BP_MAX_CTW);  // first column of this block
  const int ncol = min(Rp - c0, 4 * 16 * BP_MAX_CTW);
  const int ctw = (ncol / 16 + 3) / 4;  // column tiles per wave
  acc_t acc[2][BP_MAX_CTW];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < BP_MAX_CTW; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[a][c][i] = 0;
  // evaluation role: target tt, sources ss + 16 u
  const int tt = tid >> 4, ss = tid & 15;
  const bool tvalid = tt < it.nt;
  const double2 xt = tvalid ? tv.pts[it.t0 + tt] : cmk(0.0, 0.0);
  const T qk2 = (T)(0.25 * tv.k * tv.k);
  for (int e = it.rbeg; e < it.rend; ++e) {
    const int2 sr = rng[e];
    for (int j0 = sr.x; j0 < sr.y; j0 += BP_SC) {
      const int cnt = min(BP_SC, sr.y - j0);
      __syncthreads();
      if (tid < BP_SC) s_xs[tid] = tid < cnt ? tv.pts[j0 + tid] : cmk(0.0, 0.0);
      __syncthreads();
      T z[4], hr[4], hi[4];
      bool use[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int sl = ss + 16 * u;
        use[u] = tvalid && sl < cnt && (j0 + sl) != (it.t0 + tt);
        const double2 xs = s_xs[sl];
        const T dx = (T)(xt.x - xs.x), dy = (T)(xt.y - xs.y);
        z[u] = use[u] ? qk2 * (dx * dx + dy * dy) : (T)1.0;
      }
      hankel0_x4<T, M, LARGE>(z, hr, hi, s_ln);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int sl = ss + 16 * u;
        const T gr = use[u] ? hr[u] : (T)0, gi = use[u] ? hi[u] : (T)0;
        s_g[0][tt][sl] = gr;
        s_g[1][tt][sl] = gi;
        s_g[2][tt][sl] = -gi;
      }
      __syncthreads();
      const T* G = &s_g[plane][0][0];
      const int nks = (2 * cnt + 3) / 4;
      for (int ks = 0; ks < nks; ++ks) {
        const int sl = 2 * ks + (kl >> 1);
        T bq[BP_MAX_CTW];
#pragma unroll
        for (int c = 0; c < BP_MAX_CTW; ++c) {
          const int cc = c0 + 16 * (wave + 4 * c) + (lane & 15);
          bq[c] = 0;
          if (c < ctw && sl < cnt) {
            if (PREC == BLK_F64)
              bq[c] = ((const double*)(qb + (int64_t)(j0 + sl) * Rp + cc))[kp];
            else
              bq[c] = ((const float*)((const float2*)qb_lo + (int64_t)(j0 + sl) * Rp + cc))[kp];
          }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int R = 16 * a + (lane & 15);
          const T av = G[(R >> 1) * BP_SC + (sl < BP_SC ? sl : 0)];
#pragma unroll
          for (int c = 0; c < BP_MAX_CTW; ++c) {
            if (c < ctw) {
              if constexpr (PREC == BLK_F64)
                acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bq[c], acc[a][c], 0, 0, 0);
              else
                acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bq[c], acc[a][c], 0, 0, 0);
            }
          }
        }
      }
    }
  }
  // ub += (i/4) acc: the real row takes -Im / 4, the imaginary row Re / 4;
  // the partner row of R sits in the lane 16 apart (FP64) or in the
  // neighbouring register (FP32)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < BP_MAX_CTW; ++c) {
      if (c >= ctw) continue;
      const int cc = c0 + 16 * (wave + 4 * c) + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int R;
        double mine = (double)acc[a][c][i], other;
        if (PREC == BLK_F64) {
          R = 16 * a + 4 * i + kl;
          other = __shfl_xor(mine, 16, WAVE);
        } else {
          R = 16 * a + 4 * kl + i;
          other = (double)acc[a][c][i ^ 1];
        }
        const int t = R >> 1;
        if (t < it.nt) {
          double* o = (double*)(ub + (int64_t)(it.t0 + t) * Rp + cc) + (R & 1);
          *o += (R & 1) ? 0.25 * other : -0.25 * other;
        }
      }
    }
}

// ------------------------------------------------------------------ launchers
static inline int nblk(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

void launch_gather_blk(hipStream_t s, int n, int nc, int Rp, const int* perm, const double2* q, double2* qb) {
  hipLaunchKernelGGL(k_gather_blk, dim3(nblk((int64_t)n * Rp, 256)), dim3(256), 0, s, n, nc, Rp, perm, q, qb);
}
void launch_scatter_blk(hipStream_t s, int n, int nc, int Rp, const int* perm, const double2* ub, double2* u,
                        const double2* diag, const double2* qb) {
  hipLaunchKernelGGL(k_scatter_blk, dim3(nblk((int64_t)n * Rp, 256)), dim3(256), 0, s, n, nc, Rp, perm, ub, u, diag,
                     qb);
}
void launch_to_f32(hipStream_t s, int64_t count, const double2* src, float2* dst) {
  if (count > 0) hipLaunchKernelGGL(k_to_f32, dim3(nblk(count, 256)), dim3(256), 0, s, count, src, dst);
}
void launch_vmat(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const int64_t* voff, double2* V) {
  if (nl > 0) hipLaunchKernelGGL(k_vmat, dim3(nl), dim3(64), 0, s, tv, leaves, nl, voff, V);
}
static size_t p2m_blk_lds(int Pmax) { return sizeof(double) * 3 * (size_t)(2 * Pmax + 1) * P2M_PC; }
void launch_p2m_blk2(hipStream_t s, const TreeView& tv, int Rp, const int* leaves, int nl, int Pmax,
                     const int64_t* voff, const double2* V, const double2* qb, double2* ab) {
  if (nl > 0)
    hipLaunchKernelGGL(k_p2m_blk, dim3(nl, Rp / kBlkCols), dim3(BLK_THREADS), p2m_blk_lds(Pmax), s, tv, Rp, leaves, nl,
                       voff, V, qb, ab);
}
void launch_l2p_blk2(hipStream_t s, const TreeView& tv, int Rp, const int* leaves, int nl, const int64_t* voff,
                     const double2* V, const double2* bb, double2* ub) {
  if (nl > 0)
    hipLaunchKernelGGL(k_l2p_blk, dim3(nl, Rp / kBlkCols), dim3(BLK_THREADS), 0, s, tv, Rp, leaves, nl, voff, V, bb,
                       ub);
}
// LDS of a translation launch: the four Toeplitz planes (FP64), or the scaled
// operator rows of an item of at most `rows` complex rows (FP32 planes,
// BF16 real-embedded rows).
size_t tgemm_lds_bytes(int prec, int Pmax_s, int Pmax_d, int rows) {
  const int Ms = 2 * Pmax_s + 1;
  if (prec == BLK_F64) return sizeof(double) * 4 * (size_t)tg_table_stride(2 * (Pmax_s + Pmax_d) + 1);
  if (prec == BLK_F32) return sizeof(float) * 3 * (size_t)rows * (size_t)(Ms + 1);
  const int Ms16 = (Ms + 15) & ~15;
  return sizeof(__bf16) * 2 * (size_t)rows * (size_t)(2 * Ms16);
}
// Most row tiles of an item so that its operator rows fit the LDS budget.
int tgemm_max_nt(int prec, int Ps) {
  if (prec == BLK_F64) return kTgMaxNt;
  const size_t budget = 96 * 1024;
  for (int nt = kTgMaxNt; nt > 1; --nt)
    if (tgemm_lds_bytes(prec, Ps, Ps, 8 * nt) <= budget) return nt;
  return 1;
}
void launch_tgemm(hipStream_t s, int prec, int Rp, const TgItem* items, int nitems, int Pmax_s, int Pmax_d, int rows,
                  const TgPair* pairs, const double2* tdata, const double2* src, const void* src_lo,
                  const double* scale, int sstride, double2* dst, int add) {
  if (nitems <= 0) return;
  const size_t lds = tgemm_lds_bytes(prec, Pmax_s, Pmax_d, rows);
  // a multiple of 8 blocks: block b takes item (b mod 8) * ceil(n / 8) + b / 8
  const dim3 grid((nitems + 7) / 8 * 8, Rp / kBlkCols);
  if (prec == BLK_F64)
    hipLaunchKernelGGL(k_tgemm<BLK_F64>, grid, dim3(BLK_THREADS), lds, s, Rp, items, nitems, pairs, tdata, src, src_lo,
                       scale, sstride, dst, add, rows);
  else if (prec == BLK_F32)
    hipLaunchKernelGGL(k_tgemm<BLK_F32>, grid, dim3(BLK_THREADS), lds, s, Rp, items, nitems, pairs, tdata, src, src_lo,
                       scale, sstride, dst, add, rows);
  else
    hipLaunchKernelGGL(k_tgemm<BLK_BF16>, grid, dim3(BLK_THREADS), lds, s, Rp, items, nitems, pairs, tdata, src,
                       src_lo, scale, sstride, dst, add, rows);
}
void launch_scale_blk(hipStream_t s, int prec, const TreeView& tv, int Rp, int b0, int b1, const double* scale,
                      int sstride, const int64_t* coff16, const double2* src, void* src_lo) {
  if (b1 <= b0) return;
  if (prec == BLK_F32)
    hipLaunchKernelGGL(k_scale_blk<BLK_F32>, dim3(b1 - b0), dim3(256), 0, s, tv, Rp, b0, scale, sstride, coff16, src,
                       src_lo);
  else
    hipLaunchKernelGGL(k_scale_blk<BLK_BF16>, dim3(b1 - b0), dim3(256), 0, s, tv, Rp, b0, scale, sstride, coff16, src,
                       src_lo);
}
template <int PREC, int CLS>
static void p2p_blk_class(hipStream_t s, const TreeView& tv, int Rp, const BpItem* items, int ni, const int2* rng,
                          const double2* qb, const void* qb_lo, double2* ub) {
  if (ni <= 0) return;
  const int ngrp = (Rp + 4 * 16 * BP_MAX_CTW - 1) / (4 * 16 * BP_MAX_CTW);
  hipLaunchKernelGGL((k_p2p_blk<PREC, CLS>), dim3((ni + 7) / 8 * 8, ngrp), dim3(BLK_THREADS), 0, s, tv, Rp, items, ni,
                     rng, qb, qb_lo, ub);
}
void launch_p2p_blk(hipStream_t s, const TreeView& tv, int prec, int Rp, const BpItem* items, const int* cls_ptr,
                    const int2* rng, const double2* qb, const void* qb_lo, double2* ub) {
#define HFMM_BP(C)                                                                                                    \
  if (prec == BLK_F64)                                                                                                \
    p2p_blk_class<BLK_F64, C>(s, tv, Rp, items + cls_ptr[C], cls_ptr[C + 1] - cls_ptr[C], rng, qb, qb_lo, ub);      \
  else                                                                                                                \
    p2p_blk_class<BLK_F32, C>(s, tv, Rp, items + cls_ptr[C], cls_ptr[C + 1] - cls_ptr[C], rng, qb, qb_lo, ub)
  HFMM_BP(0); HFMM_BP(1); HFMM_BP(2); HFMM_BP(3); HFMM_BP(4); HFMM_BP(5);
#undef HFMM_BP
  static_assert(kH0Classes == 5, "one launch per class and one for the large-argument class");
}

hipError_t init_blocked_attributes() {
  const void* fs[] = {(const void*)k_tgemm<BLK_F64>, (const void*)k_tgemm<BLK_F32>, (const void*)k_tgemm<BLK_BF16>,
                      (const void*)k_p2m_blk};
  for (const void* f : fs) {
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, f);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - (int)fa.sharedSizeBytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace hfmm
