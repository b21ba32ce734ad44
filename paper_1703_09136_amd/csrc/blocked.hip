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
// Both layout changes go through 32 x 32 tiles in LDS (points j by
// right-hand sides r): the user-order side is read or written along the
// points (neighbouring sorted points mostly neighbour in input order too),
// the blocked side along the right-hand sides; a block takes two tiles of
// consecutive points.
constexpr int LT = 32;  // tile side
__global__ void __launch_bounds__(256) k_gather_blk(int n, int nc, int Rp, const int* __restrict__ perm,
                                                    const double2* __restrict__ q, double2* __restrict__ qb,
                                                    int conj) {
  __shared__ double2 t[2][LT][LT + 1];
  const int tx = threadIdx.x & (LT - 1), ty = threadIdx.x / LT;  // 32 x 8
  const int w = ty >> 2, sub = ty & 3;                           // the thread's tile, its row phase
  const int j0 = (blockIdx.x * 2 + w) * LT, r0 = blockIdx.y * LT;
  // read: lane tx along the points, rows r of the tile by 2
  const int j = j0 + tx;
  const int pj = j < n ? perm[j] : 0;
  for (int rr = sub; rr < LT; rr += 4) {
    const int r = r0 + rr;
    double2 v = (j < n && r < nc) ? q[(int64_t)r * n + pj] : cmk(0.0, 0.0);
    if (conj) v.y = -v.y;
    t[w][rr][tx] = v;
  }
  __syncthreads();
  // write: lane tx along the right-hand sides
  for (int jj = sub; jj < LT; jj += 4) {
    const int jw = j0 + jj, r = r0 + tx;
    if (jw < n && r < Rp) qb[(int64_t)jw * Rp + r] = t[w][tx][jj];
  }
}

__global__ void __launch_bounds__(256) k_scatter_blk(int n, int nc, int Rp, const int* __restrict__ perm,
                                                     const double2* __restrict__ ub, double2* __restrict__ u,
                                                     const double2* __restrict__ diag,
                                                     const double2* __restrict__ qb, int conj) {
  __shared__ double2 t[2][LT][LT + 1];
  const int tx = threadIdx.x & (LT - 1), ty = threadIdx.x / LT;
  const int w = ty >> 2, sub = ty & 3;
  const int j0 = (blockIdx.x * 2 + w) * LT, r0 = blockIdx.y * LT;
  // read along the right-hand sides
  for (int jj = sub; jj < LT; jj += 4) {
    const int j = j0 + jj, r = r0 + tx;
    double2 v = cmk(0.0, 0.0);
    if (j < n && r < nc) {
      const int64_t idx = (int64_t)j * Rp + r;
      v = ub[idx];
      if (diag) v = csub(v, cmul(diag[j], qb[idx]));
      if (conj) v.y = -v.y;
    }
    t[w][jj][tx] = v;
  }
  __syncthreads();
  // write along the points
  const int j = j0 + tx;
  if (j >= n) return;
  const int pj = perm[j];
  for (int rr = sub; rr < LT; rr += 4) {
    const int r = r0 + rr;
    if (r < nc) u[(int64_t)r * n + pj] = t[w][tx][rr];
  }
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

// alpha[c_b + m][r] = sum_j V[m][j] q[j][r] for the leaves of one level, 64
// right-hand sides per block (grid y), a 16-column tile per wave and all NRT
// row tiles of the level's 2(2P + 1) real rows per wave. V goes through LDS
// in chunks of 32 points as the planes Re V and Im V (rows padded so that
// one wave's operand reads fall in distinct banks; the embedding's -Im V is a
// sign per lane); the chunk's strengths are loaded into registers before the
// chunk is staged, so their latency hides behind the staging.
constexpr int P2M_PC = 32;  // points per chunk
constexpr int P2M_PS = 34;  // LDS row stride (doubles)

template <int NRT>
__global__ void __launch_bounds__(BLK_THREADS) k_p2m_blk(TreeView tv, int Rp, const int* __restrict__ leaves,
                                                         int nl, const int64_t* __restrict__ voff,
                                                         const double2* __restrict__ V, const double2* __restrict__ qb,
                                                         double2* __restrict__ ab) {
  constexpr int MR = 8 * NRT;  // orders the planes hold
  constexpr int PL = MR * P2M_PS + ((NRT & 1) ? 0 : 16);  // plane stride: the second plane 32 banks over
  __shared__ double s_v[2 * PL];
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
  const int kl = lane >> 4, rp = lane & 1, kp = kl & 1;
  // A = [[Re, -Im], [Im, Re]] V: the lane's plane and sign
  const double* Lp = s_v + (rp == kp ? 0 : PL) + (kl >> 1);
  const double sg = (rp == 0 && kp == 1) ? -1.0 : 1.0;
  int mrow[NRT];
#pragma unroll
  for (int j = 0; j < NRT; ++j) {
    const int R = 16 * j + (lane & 15);
    mrow[j] = (R < 2 * Md ? R >> 1 : 0) * P2M_PS;
  }
  d4 acc[NRT];
#pragma unroll
  for (int j = 0; j < NRT; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
  for (int j0 = 0; j0 < np; j0 += P2M_PC) {
    const int nj = min(P2M_PC, np - j0);
    double bq[P2M_PC / 2];
#pragma unroll
    for (int ks = 0; ks < P2M_PC / 2; ++ks) {
      const int jj = 2 * ks + (kl >> 1);
      const double v = ((const double*)(qb + (int64_t)(pr.x + j0 + (jj < nj ? jj : 0)) * Rp + col))[kp];
      bq[ks] = jj < nj ? v : 0.0;
    }
    __syncthreads();  // the previous chunk's operand reads are done
    for (int e = tid; e < Md * P2M_PC; e += BLK_THREADS) {
      const int m = e / P2M_PC, jj = e - m * P2M_PC;
      const double2 v = jj < nj ? Vl[(int64_t)m * np + j0 + jj] : cmk(0.0, 0.0);
      s_v[m * P2M_PS + jj] = v.x;
      s_v[PL + m * P2M_PS + jj] = v.y;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < P2M_PC / 2; ++ks) {
#pragma unroll
      for (int j = 0; j < NRT; ++j)
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(sg * Lp[mrow[j] + 2 * ks], bq[ks], acc[j], 0, 0, 0);
    }
  }
  const int64_t cb = tv.coff[b];
#pragma unroll
  for (int j = 0; j < NRT; ++j) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int R = 16 * j + 4 * i + kl;
      if (R < 2 * Md) ((double*)(ab + (cb + (R >> 1)) * Rp + col))[R & 1] = acc[j][i];
    }
  }
}

// u[j][r] += (i/4) sum_m conj(V[m][j]) beta[c_b + m][r] for the points of one
// leaf: rows are the leaf's points (2 np real rows; groups of up to 64 points,
// NRT row tiles for the group's rows), k the 2(2P + 1) real orders. The
// embedding of conj(V): [2j][2m] = Re V, [2j][2m+1] = Im V, [2j+1][2m] =
// -Im V, [2j+1][2m+1] = Re V; V is staged in LDS sixteen orders at a time as
// the planes Re V and Im V (padded rows: one wave's reads in distinct banks),
// the chunk's local coefficients loaded into registers before the staging.
constexpr int L2P_MC = 16;  // orders per chunk
constexpr int L2P_RS = 72;  // LDS row stride (doubles)
constexpr int L2P_PL = L2P_MC * L2P_RS + 16;  // plane stride: the second plane 32 banks over

template <int NRT>
__device__ inline void l2p_group(int Md, int np, int g0, int ng, int64_t cb, int pr0, int Rp, int col,
                                 const double2* __restrict__ Vl, const double2* __restrict__ bb,
                                 double2* __restrict__ ub, double* s_v) {
  const int tid = threadIdx.x, lane = tid & 63, kl = lane >> 4, rp = lane & 1, kp = kl & 1;
  const double* Lp = s_v + (rp == kp ? 0 : L2P_PL) + (kl >> 1) * L2P_RS;
  const double sg = (rp == 1 && kp == 0) ? -1.0 : 1.0;
  int prow[NRT];
#pragma unroll
  for (int j = 0; j < NRT; ++j) {
    const int R = 16 * j + (lane & 15);
    prow[j] = R < 2 * ng ? R >> 1 : 0;
  }
  d4 acc[NRT];
#pragma unroll
  for (int j = 0; j < NRT; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
  for (int m0 = 0; m0 < Md; m0 += L2P_MC) {
    double bq[L2P_MC / 2];
#pragma unroll
    for (int ks = 0; ks < L2P_MC / 2; ++ks) {
      const int m = m0 + 2 * ks + (kl >> 1);
      const double v = ((const double*)(bb + (cb + (m < Md ? m : 0)) * Rp + col))[kp];
      bq[ks] = m < Md ? v : 0.0;
    }
    __syncthreads();  // the previous chunk's operand reads are done
    for (int e = tid; e < L2P_MC * 64; e += BLK_THREADS) {
      const int mi = e >> 6, jp = e & 63;
      const double2 v = (m0 + mi < Md && jp < ng) ? Vl[(int64_t)(m0 + mi) * np + g0 + jp] : cmk(0.0, 0.0);
      s_v[mi * L2P_RS + jp] = v.x;
      s_v[L2P_PL + mi * L2P_RS + jp] = v.y;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < L2P_MC / 2; ++ks) {
#pragma unroll
      for (int j = 0; j < NRT; ++j)
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(sg * Lp[2 * ks * L2P_RS + prow[j]], bq[ks], acc[j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < NRT; ++j) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // (i/4) z: the real row takes -Im z / 4, the imaginary row Re z / 4;
      // the partner row (R ^ 1) sits in the lane 16 apart (kl ^ 1)
      const int R = 16 * j + 4 * i + kl;
      const double other = __shfl_xor(acc[j][i], 16, WAVE);
      if (R < 2 * ng) {
        double* o = (double*)(ub + (int64_t)(pr0 + g0 + (R >> 1)) * Rp + col) + (R & 1);
        *o += (R & 1) ? 0.25 * other : -0.25 * other;
      }
    }
  }
}

__global__ void __launch_bounds__(BLK_THREADS) k_l2p_blk(TreeView tv, int Rp, const int* __restrict__ leaves,
                                                         int nl, const int64_t* __restrict__ voff,
                                                         const double2* __restrict__ V, const double2* __restrict__ bb,
                                                         double2* __restrict__ ub) {
  __shared__ double s_v[2 * L2P_PL];
  const int li = blockIdx.x;
  if (li >= nl) return;
  const int b = leaves[li];
  const int P = tv.P[tv.level[b]];
  const int Md = 2 * P + 1;
  const int2 pr = tv.prange[b];
  const int np = pr.y - pr.x;
  const double2* Vl = V + voff[li];
  const int wave = threadIdx.x >> 6;
  const int col = blockIdx.y * kBlkCols + wave * 16 + (threadIdx.x & 15);
  const int64_t cb = tv.coff[b];
  for (int g0 = 0; g0 < np; g0 += 64) {  // groups of 64 points, the last one by its row tiles
    const int ng = min(64, np - g0);
    switch ((2 * ng + 15) / 16) {
      case 1: l2p_group<1>(Md, np, g0, ng, cb, pr.x, Rp, col, Vl, bb, ub, s_v); break;
      case 2: l2p_group<2>(Md, np, g0, ng, cb, pr.x, Rp, col, Vl, bb, ub, s_v); break;
      case 3: l2p_group<3>(Md, np, g0, ng, cb, pr.x, Rp, col, Vl, bb, ub, s_v); break;
      case 4: l2p_group<4>(Md, np, g0, ng, cb, pr.x, Rp, col, Vl, bb, ub, s_v); break;
      case 5: l2p_group<5>(Md, np, g0, ng, cb, pr.x, Rp, col, Vl, bb, ub, s_v); break;
      case 6: l2p_group<6>(Md, np, g0, ng, cb, pr.x, Rp, col, Vl, bb, ub, s_v); break;
      case 7: l2p_group<7>(Md, np, g0, ng, cb, pr.x, Rp, col, Vl, bb, ub, s_v); break;
      default: l2p_group<8>(Md, np, g0, ng, cb, pr.x, Rp, col, Vl, bb, ub, s_v); break;
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

// The scaled reduced-precision operators of the multipole-to-local tables,
// made once per plan: O[p][m] = a(|m|) a(|p|) T_pm for orders p, m in
// [-P, P] of the table's level, T_pm = t[m - p] (free) or (-1)^m t[-m - p]
// (image: the operator acting on unreflected multipoles). FP32: complex
// rows [2P + 1][Ms8] (orders padded with zeros to a multiple of 8) at off[t]
// (float2 units). BF16: the interleaved real
// embedding, rows 2p and 2p + 1 of K = 2 Ms16 values (zero past the orders),
// at off[t] (bf16 units). One block per table.
__global__ void k_lo_tables(int prec, int ntab, const int64_t* __restrict__ toff, const int* __restrict__ P_of,
                            const int* __restrict__ lev_of, const int* __restrict__ img_of,
                            const int64_t* __restrict__ off, const double* __restrict__ scale, int sstride,
                            const double2* __restrict__ tdata, void* __restrict__ out) {
  const int t = blockIdx.x;
  if (t >= ntab) return;
  const int P = P_of[t], M = 2 * P + 1;
  const bool img = img_of[t] != 0;
  const double* sa = scale + lev_of[t] * sstride;
  const double2* T = tdata + toff[t];  // t[-2P]
  const int Ms8 = (M + 7) & ~7, Ms16 = (M + 15) & ~15, K = 2 * Ms16;
  const int cols = prec == BLK_F32 ? Ms8 : Ms16;
  for (int e = threadIdx.x; e < M * cols; e += blockDim.x) {
    const int p = e / cols, m = e - p * cols;
    double2 v = cmk(0.0, 0.0);
    if (m < M) {
      const int pp = p - P, mm = m - P;
      const int idx = img ? -mm - pp + 2 * P : mm - pp + 2 * P;
      const double sg = (img && (mm & 1)) ? -1.0 : 1.0;
      v = cscale(T[idx], sg * sa[mm < 0 ? -mm : mm] * sa[pp < 0 ? -pp : pp]);
    }
    if (prec == BLK_F32) {
      ((float2*)out)[off[t] + (int64_t)p * Ms8 + m] = make_float2((float)v.x, (float)v.y);
    } else {
      __bf16* r0 = (__bf16*)out + off[t] + (int64_t)(2 * p) * K + 2 * m;
      __bf16* r1 = r0 + K;
      r0[0] = (__bf16)(float)v.x;
      r0[1] = (__bf16)(float)(-v.y);
      r1[0] = (__bf16)(float)v.y;
      r1[1] = (__bf16)(float)v.x;
    }
  }
}

template <int PREC>
struct TgTraits;
template <>
struct TgTraits<BLK_F64> {
  using acc_t = d4;
  using b_t = double;
};
template <>
struct TgTraits<BLK_F32> {
  using acc_t = f4;
  using b_t = float;
};
template <>
struct TgTraits<BLK_BF16> {
  using acc_t = f4;
  using b_t = bf8;
};

// Source rows of a pair arrive in LDS in chunks of TG_CH orders (16 for
// BF16) by asynchronous global-to-LDS copies (global_load_lds_dwordx4: lane
// i's 16 bytes go to the wave's LDS address + 16 i), double-buffered: the
// copy of chunk s + 1 is issued right after the barrier that makes chunk s
// visible and runs while chunk s is contracted, so the MFMA loop reads only
// LDS. The reduced-precision operators (row-padded plan tables) are copied
// the same way, one pair ahead; the FP64 Toeplitz planes are loaded into
// registers one pair ahead and stored after the pair's last chunk.
typedef __attribute__((address_space(3))) void lds_void_t;
__device__ inline void copy16_to_lds(const void* g, void* l) {
  __builtin_amdgcn_global_load_lds(g, (lds_void_t*)l, 16, 0, 0);
}
// orders per source chunk: 16 KiB per chunk in every precision
template <int PREC>
struct TgChunk {
  static constexpr int CH = PREC == BLK_F64 ? 16 : (PREC == BLK_F32 ? 32 : 64);
  static constexpr int BYTES = CH * 64 * (PREC == BLK_F64 ? 16 : (PREC == BLK_F32 ? 8 : 4));
};
constexpr int TG_PF64 = 2;  // Toeplitz values per thread (ntp <= 512)

// dst rows of item t = (add ? dst : 0) + sum_pairs Op_pair src_pair. Block:
// one item, 64 right-hand sides (grid y), wave w the columns 16 w .. 16 w + 15,
// all nt row tiles of the item (at most NTM). FP64: A from the Toeplitz
// planes (Re, Im, -Im, -Re), B the blocked FP64 source rows. FP32 / BF16: A
// from the plan's scaled operators (FP32 complex rows of Ms8 orders; BF16
// embedded rows of 2 Ms16 values), B the scaled low-precision source rows;
// each pair accumulates in FP32 on the matrix cores and is added to FP64
// sums, divided by a_t(|p|) at the end. Items are spread over the XCDs in
// contiguous runs: the grid has a multiple of 8 blocks and block b
// (dispatched to XCD b mod 8) takes item (b mod 8) * ceil(n / 8) + b / 8, so
// neighbouring targets, which share source boxes, share an L2.
template <int PREC, int NTM>
__global__ void __launch_bounds__(BLK_THREADS) k_tgemm(int Rp, const TgItem* __restrict__ items, int nitems,
                                                       const TgPair* __restrict__ pairs,
                                                       const double2* __restrict__ tdata, const void* __restrict__ olo,
                                                       const double2* __restrict__ src, const void* __restrict__ src_lo,
                                                       const double* __restrict__ scale, int sstride,
                                                       double2* __restrict__ dst, int add, int abuf) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds8[];
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
  const int col0 = blockIdx.y * kBlkCols;     // the block's first right-hand side
  const int cl = wave * 16 + (lane & 15);     // this lane's column within the block
  const int col = col0 + cl;
  const int rp = lane & 1, kp = kl & 1;
  acc_t acc[NTM];
#pragma unroll
  for (int j = 0; j < NTM; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[j][i] = 0;
  constexpr int NT64 = PREC == BLK_F64 ? 1 : NTM;
  double acc64[NT64][4];
#pragma unroll
  for (int j = 0; j < NT64; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc64[j][i] = 0.0;
  // every one of the NTM tiles is contracted (no per-tile branches in the
  // MFMA loops): rows past the item's tiles or past 2 Md read order 0's
  // operator and are not stored
  int pidx[NTM];
#pragma unroll
  for (int j = 0; j < NTM; ++j) {
    const int R = 16 * (it.rt0 + j) + (lane & 15);
    pidx[j] = (j < it.nt && R < 2 * Md) ? (R >> 1) : 0;
  }
  const int p_lo = 8 * it.rt0;
  const int nrow = min(8 * it.nt, Md - p_lo);
  const int ntp = tg_table_stride(nt_tab);
  const int Ms8 = (Ms + 7) & ~7, Ms16 = (Ms + 15) & ~15, K16 = 2 * Ms16;
  constexpr int CH = TgChunk<PREC>::CH;  // orders per chunk
  const int nch = (Ms + CH - 1) / CH;
  const int npair = it.pend - it.pbeg;
  const int nstage = npair * nch;
  // LDS: two operator buffers of abuf bytes, then two source chunks
  constexpr int BBUF = TgChunk<PREC>::BYTES;
  unsigned char* const Ab0 = lds8;
  unsigned char* const Bb0 = lds8 + 2 * abuf;
  // ---- FP64 operator: Toeplitz planes through registers
  double2 r64[TG_PF64];
  auto fetchA64 = [&](int e) {
    const double2* T = tdata + pairs[e].toff;
#pragma unroll
    for (int u = 0; u < TG_PF64; ++u) {
      const int i = tid + u * BLK_THREADS, n = i - kTabPadB;
      r64[u] = (i < ntp && n >= 0 && n < nt_tab) ? T[n] : cmk(0.0, 0.0);
    }
  };
  auto storeA64 = [&](int buf) {
    double* L = (double*)(Ab0 + buf * abuf);
#pragma unroll
    for (int u = 0; u < TG_PF64; ++u) {
      const int i = tid + u * BLK_THREADS;
      if (i < ntp) {
        L[i] = r64[u].x;
        L[ntp + i] = r64[u].y;
        L[2 * ntp + i] = -r64[u].y;
        L[3 * ntp + i] = -r64[u].x;
      }
    }
  };
  // ---- asynchronous copies: operator rows (reduced precision) of pair e
  auto copyA = [&](int e, int buf) {
    const TgPair pa = pairs[e];
    const unsigned char* g;
    int bytes;
    if (PREC == BLK_F32) {
      g = (const unsigned char*)((const float2*)olo + pa.tlo + (int64_t)p_lo * Ms8);
      bytes = nrow * Ms8 * 8;
    } else {
      g = (const unsigned char*)((const __bf16*)olo + pa.tlo + (int64_t)(2 * p_lo) * K16);
      bytes = 2 * nrow * K16 * 2;
    }
    unsigned char* L = Ab0 + buf * abuf;
    for (int o = wave * 1024; o < bytes; o += 4096)
      if (o + 16 * lane < bytes) copy16_to_lds(g + o + 16 * lane, L + o);
  };
  // source chunk c of pair e (rows of orders c CH .. c CH + CH - 1; zeros past Ms)
  auto copyB = [&](int e, int c, int buf) {
    const TgPair pa = pairs[e];
    unsigned char* L = Bb0 + buf * BBUF;
    if constexpr (PREC == BLK_F64) {
      // CH rows of 64 complex doubles (1 KiB each), CH / 4 per wave
#pragma unroll
      for (int rr = 0; rr < CH / 4; ++rr) {
        const int r = wave * (CH / 4) + rr, m = c * CH + r;
        if (m < Ms)
          copy16_to_lds(src + (pa.cs + m) * Rp + col0 + lane, L + r * 1024);
        else
          ((double2*)(L + r * 1024))[lane] = cmk(0.0, 0.0);
      }
    } else if constexpr (PREC == BLK_F32) {
      // CH rows of 64 complex floats (512 bytes), two per copy, CH / 8 copies per wave
#pragma unroll
      for (int rr = 0; rr < CH / 8; ++rr) {
        const int blk = wave * (CH / 8) + rr;
        const int r = 2 * blk + (lane >> 5), m = c * CH + r;
        const float2* S = (const float2*)src_lo + (pa.cs + m) * Rp + col0 + 2 * (lane & 31);
        if (m < Ms)
          copy16_to_lds(S, L + blk * 1024);
        else
          ((float4*)(L + blk * 1024))[lane] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    } else {
      // 64 columns x CH orders of 4-byte complex bf16 (CH * 4 bytes per
      // column, 1024 / (CH * 4) columns per copy), 16 columns per wave
      constexpr int LPC = CH * 4 / 16;  // lanes per column
#pragma unroll
      for (int rr = 0; rr < 16 * LPC / 64; ++rr) {
        const int cc = wave * 16 + rr * (64 / LPC) + lane / LPC;
        const __bf16* S =
            (const __bf16*)src_lo + 2 * (pa.cs16 * Rp + (int64_t)(col0 + cc) * Ms16 + c * CH + 4 * (lane % LPC));
        if (c * CH + 4 * (lane % LPC) < Ms16)
          copy16_to_lds(S, L + (wave * 16 + rr * (64 / LPC)) * CH * 4);
        else
          ((float4*)(L + (wave * 16 + rr * (64 / LPC)) * CH * 4))[lane] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  };
  // stage st = chunk c of pair e: the operator of pair e goes to buffer e & 1
  // with its first chunk (issued while the previous pair's last chunk is
  // contracted; that buffer was last read by the pair before)
  auto issue = [&](int st) {
    const int pi = st / nch, c = st - pi * nch;
    if (PREC != BLK_F64 && c == 0) copyA(it.pbeg + pi, pi & 1);
    copyB(it.pbeg + pi, c, st & 1);
  };
  if (nstage > 0) {
    if (PREC == BLK_F64) {
      fetchA64(it.pbeg);
      storeA64(0);
    }
    issue(0);
  }
  for (int st = 0; st < nstage; ++st) {
    const int pi = st / nch, c = st - pi * nch;
    const int e = it.pbeg + pi;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of chunk st (and older) have landed
    __syncthreads();                // every wave's; and chunk st - 1 is no longer read
    if (PREC == BLK_F64 && c == 0 && e + 1 < it.pend) fetchA64(e + 1);
    if (st + 1 < nstage) issue(st + 1);
    const TgPair pa = pairs[e];
    const bool img = pa.image != 0;
    const unsigned char* Bb = Bb0 + (st & 1) * BBUF;
    const unsigned char* Ab = Ab0 + (pi & 1) * abuf;
    if constexpr (PREC == BLK_F64) {
      const bool neg = img && (((kl >> 1) + Ps) & 1);
      const double* Lp = (const double*)Ab + tg_plane(rp, kp, neg) * ntp + kTabPadB;
      const int step = img ? -2 : 2;
      int base[NTM];
#pragma unroll
      for (int j = 0; j < NTM; ++j)
        base[j] = (img ? 2 * Ps + 2 * Pd - pidx[j] - (kl >> 1) : 2 * Pd - pidx[j] + (kl >> 1)) + step * (c * CH / 2);
      const double* Bl = (const double*)Bb + 2 * cl + kp;
      const int kend = min(CH / 2, (Ms - c * CH + 1) / 2);  // k-steps holding orders below Ms
#pragma unroll
      for (int ks = 0; ks < CH / 2; ++ks) {
        if (ks < kend) {
          const double b = Bl[(2 * ks + (kl >> 1)) * 128];
#pragma unroll
          for (int j = 0; j < NTM; ++j)
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(Lp[base[j] + step * ks], b, acc[j], 0, 0, 0);
        }
      }
      if (c == nch - 1 && e + 1 < it.pend) storeA64((pi + 1) & 1);
    } else if constexpr (PREC == BLK_F32) {
      // A: row (p - p_lo), order m = c CH + 2 ks + kl / 2; the lane takes the
      // real part (rp == kp) or the imaginary part, negated for rp = 0, kp = 1
      const float* Af = (const float*)Ab + (rp == kp ? 0 : 1);
      const float sg = (rp == 0 && kp == 1) ? -1.0f : 1.0f;
      int aoff[NTM];
#pragma unroll
      for (int j = 0; j < NTM; ++j) aoff[j] = 2 * ((pidx[j] - p_lo > 0 ? pidx[j] - p_lo : 0) * Ms8 + c * CH + (kl >> 1));
      const float* Bl = (const float*)Bb + 2 * cl + kp;
      const int kend = min(CH / 2, (Ms - c * CH + 1) / 2);
#pragma unroll
      for (int ks = 0; ks < CH / 2; ++ks) {
        if (ks < kend) {
          const float b = Bl[(2 * ks + (kl >> 1)) * 128];
#pragma unroll
          for (int j = 0; j < NTM; ++j)
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(sg * Af[aoff[j] + 4 * ks], b, acc[j], 0, 0, 0);
        }
      }
    } else {
      // A: embedded row R - 2 p_lo, k = 2 (c CH + 16 ks) + 8 kl; B: column cl,
      // orders c CH + 16 ks + 4 kl .. + 3 (k-steps of 16 orders below Ms16)
      int ro[NTM];
#pragma unroll
      for (int j = 0; j < NTM; ++j) {
        const int R = 16 * (it.rt0 + j) + (lane & 15);
        const int rl = R - 2 * p_lo;
        ro[j] = (rl >= 0 && rl < 2 * nrow ? rl : 0) * K16 + 2 * c * CH + 8 * kl;
      }
      const int kend = min(CH / 16, (Ms16 - c * CH) / 16);
#pragma unroll
      for (int ks = 0; ks < CH / 16; ++ks) {
        if (ks < kend) {
          const bf8 b = *(const bf8*)(Bb + (cl * CH + 16 * ks + 4 * kl) * 4);
#pragma unroll
          for (int j = 0; j < NTM; ++j)
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*(const bf8*)(Ab + 2 * (ro[j] + 32 * ks)), b, acc[j], 0, 0,
                                                             0);
        }
      }
    }
    if constexpr (PREC != BLK_F64) {
      if (c == nch - 1) {
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
  for (int j = 0; j < NTM; ++j) {
    if (j >= it.nt) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int R = 16 * (it.rt0 + j) + (PREC == BLK_F64 ? 4 * i + kl : 4 * kl + i);
      if (R >= 2 * Md) continue;
      double v;
      if constexpr (PREC == BLK_F64) {
        v = acc[j][i];
      } else {
        const int pp = (R >> 1) - Pd;
        v = acc64[j][i] / st[pp < 0 ? -pp : pp];
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
// targets of an item against its source ranges, 64 right-hand sides per
// block (wave w: the 16 columns 16 w ..; grid y: the pass's 64-column groups).
// The sources go in chunks of 32: every thread evaluates two H0 values of
// the 16 x 32 tile (Horner chains interleaved), stored in LDS as the planes
// Re G and Im G (rows padded so that the MFMA operand reads of one wave fall
// in distinct banks); the tile is applied on the matrix cores as the real
// embedding [[Re, -Im], [Im, Re]] (FP64, or FP32 with the FP32 series and
// strengths). The strengths of the next chunk are loaded into registers
// before the current chunk's contraction, so their latency hides behind it.
constexpr int BP_SC = 32;                 // sources per chunk
constexpr int BP_GS = 34;                 // LDS row stride of a G plane (elements)
constexpr int BP_GP = 16 * BP_GS + 16;    // LDS plane stride (elements)

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
  constexpr int NKS = BP_SC / 2;  // k-steps per chunk (two sources each)
  __shared__ T s_g[2 * BP_GP];
  __shared__ double2 s_ln[1 << kLogTabBits];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (PREC == BLK_F64)
    for (int l = tid; l < (1 << kLogTabBits); l += BLK_THREADS) s_ln[l] = cmk(kLogTab[l][0], kLogTab[l][1]);
  __syncthreads();
  const int per_xcd = (nitems + 7) / 8;
  const int it_id = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (it_id >= nitems) return;
  const BpItem it = items[it_id];
  const int kl = lane >> 4, rp = lane & 1, kp = kl & 1;
  // A operand: row R = 16 a + (lane & 15) (target R / 2, part rp), k = 4 ks + kl
  // (source 2 ks + kl / 2, part kp): Re G if rp == kp, else +-Im G
  const T* Gp = s_g + (rp == kp ? 0 : BP_GP) + (kl >> 1);
  const T sg = (rp == 0 && kp == 1) ? (T)-1 : (T)1;
  const int col = blockIdx.y * kBlkCols + wave * 16 + (lane & 15);  // this lane's right-hand side
  acc_t acc[2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[a][i] = 0;
  // evaluation role: target tt, sources ss and ss + 16 of the chunk
  const int tt = tid >> 4, ss = tid & 15;
  const bool tvalid = tt < it.nt;
  const double2 xt = tvalid ? tv.pts[it.t0 + tt] : cmk(0.0, 0.0);
  const T qk2 = (T)(0.25 * tv.k * tv.k);
  // the chunk sequence: (range e, first source j0)
  auto advance = [&](int& e, int& j0) {
    j0 += BP_SC;
    if (j0 >= rng[e].y) {
      ++e;
      if (e < it.rend) j0 = rng[e].x;
    }
  };
  // branch-free: sources past the chunk read the item's first target and are zeroed
  auto load_b = [&](int e, int j0, T (&b)[NKS]) {
    const int cnt = e < it.rend ? rng[e].y - j0 : 0;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int sl = 2 * ks + (kl >> 1);
      const int js = sl < cnt ? j0 + sl : it.t0;
      T v;
      if constexpr (PREC == BLK_F64)
        v = ((const double*)(qb + (int64_t)js * Rp + col))[kp];
      else
        v = ((const float*)((const float2*)qb_lo + (int64_t)js * Rp + col))[kp];
      b[ks] = sl < cnt ? v : (T)0;
    }
  };
  int e = it.rbeg, j0 = e < it.rend ? rng[e].x : 0;
  T bq[NKS];
  load_b(e, j0, bq);
  while (e < it.rend) {
    const int cnt = min(BP_SC, rng[e].y - j0);
    T z[2], hr[2], hi[2];
    bool use[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int sl = ss + 16 * u;
      use[u] = tvalid && sl < cnt && (j0 + sl) != (it.t0 + tt);
      const double2 xs = tv.pts[sl < cnt ? j0 + sl : it.t0];
      const T dx = (T)(xt.x - xs.x), dy = (T)(xt.y - xs.y);
      z[u] = use[u] ? qk2 * (dx * dx + dy * dy) : (T)1.0;
    }
    hankel0_x4<T, M, LARGE, 2>(z, hr, hi, s_ln);
    __syncthreads();  // the previous chunk's operand reads are done
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int sl = ss + 16 * u;
      s_g[tt * BP_GS + sl] = use[u] ? hr[u] : (T)0;
      s_g[BP_GP + tt * BP_GS + sl] = use[u] ? hi[u] : (T)0;
    }
    __syncthreads();
    int en = e, jn = j0;
    advance(en, jn);
    T bn[NKS];
    load_b(en, jn, bn);
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const T av = sg * Gp[(8 * a + ((lane & 15) >> 1)) * BP_GS + 2 * ks];
        if constexpr (PREC == BLK_F64)
          acc[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bq[ks], acc[a], 0, 0, 0);
        else
          acc[a] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bq[ks], acc[a], 0, 0, 0);
      }
    }
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) bq[ks] = bn[ks];
    e = en;
    j0 = jn;
  }
  // ub += (i/4) acc: the real row takes -Im / 4, the imaginary row Re / 4;
  // the partner row of R sits in the lane 16 apart (FP64) or in the
  // neighbouring register (FP32)
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int R;
      double mine = (double)acc[a][i], other;
      if (PREC == BLK_F64) {
        R = 16 * a + 4 * i + kl;
        other = __shfl_xor(mine, 16, WAVE);
      } else {
        R = 16 * a + 4 * kl + i;
        other = (double)acc[a][i ^ 1];
      }
      const int t = R >> 1;
      if (t < it.nt) {
        double* o = (double*)(ub + (int64_t)(it.t0 + t) * Rp + col) + (R & 1);
        *o += (R & 1) ? 0.25 * other : -0.25 * other;
      }
    }
  }
}

// ------------------------------------------------------------------ launchers
static inline int nblk(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

void launch_gather_blk(hipStream_t s, int n, int nc, int Rp, const int* perm, const double2* q, double2* qb,
                       int conj) {
  hipLaunchKernelGGL(k_gather_blk, dim3(nblk(n, 2 * LT), Rp / LT), dim3(256), 0, s, n, nc, Rp, perm, q, qb, conj);
}
void launch_scatter_blk(hipStream_t s, int n, int nc, int Rp, const int* perm, const double2* ub, double2* u,
                        const double2* diag, const double2* qb, int conj) {
  hipLaunchKernelGGL(k_scatter_blk, dim3(nblk(n, 2 * LT), (nc + LT - 1) / LT), dim3(256), 0, s, n, nc, Rp, perm, ub,
                     u, diag, qb, conj);
}
void launch_to_f32(hipStream_t s, int64_t count, const double2* src, float2* dst) {
  if (count > 0) hipLaunchKernelGGL(k_to_f32, dim3(nblk(count, 256)), dim3(256), 0, s, count, src, dst);
}
void launch_vmat(hipStream_t s, const TreeView& tv, const int* leaves, int nl, const int64_t* voff, double2* V) {
  if (nl > 0) hipLaunchKernelGGL(k_vmat, dim3(nl), dim3(64), 0, s, tv, leaves, nl, voff, V);
}
template <int NRT>
static void p2m_one(hipStream_t s, const TreeView& tv, int Rp, const int* leaves, int nl, const int64_t* voff,
                    const double2* V, const double2* qb, double2* ab) {
  hipLaunchKernelGGL((k_p2m_blk<NRT>), dim3(nl, Rp / kBlkCols), dim3(BLK_THREADS), 0, s, tv, Rp, leaves, nl, voff, V,
                     qb, ab);
}
void launch_p2m_blk2(hipStream_t s, const TreeView& tv, int Rp, const int* leaves, int nl, int P,
                     const int64_t* voff, const double2* V, const double2* qb, double2* ab) {
  if (nl <= 0) return;
  switch ((2 * (2 * P + 1) + 15) / 16) {
#define HFMM_P2M(N) \
  case N: p2m_one<N>(s, tv, Rp, leaves, nl, voff, V, qb, ab); break;
    HFMM_P2M(1) HFMM_P2M(2) HFMM_P2M(3) HFMM_P2M(4) HFMM_P2M(5) HFMM_P2M(6) HFMM_P2M(7) HFMM_P2M(8) HFMM_P2M(9)
    HFMM_P2M(10) HFMM_P2M(11)
#undef HFMM_P2M
    default: break;
  }
}
void launch_l2p_blk2(hipStream_t s, const TreeView& tv, int Rp, const int* leaves, int nl, const int64_t* voff,
                     const double2* V, const double2* bb, double2* ub) {
  if (nl > 0)
    hipLaunchKernelGGL(k_l2p_blk, dim3(nl, Rp / kBlkCols), dim3(BLK_THREADS), 0, s, tv, Rp, leaves, nl, voff, V, bb,
                       ub);
}
// Bytes of one operator buffer for an item with `rows` complex rows (two
// are used): the four Toeplitz planes (FP64), its FP32 rows of Ms8 complex
// floats, or its BF16 embedded rows (2 rows x 2 Ms16 values); and the LDS of
// a launch: two operator buffers and two source chunks.
int tgemm_buf_elems(int prec, int Ps, int Pd, int rows) {
  const int Ms = 2 * Ps + 1;
  if (prec == BLK_F64) return 8 * 4 * tg_table_stride(2 * (Ps + Pd) + 1);
  if (prec == BLK_F32) return 8 * rows * ((Ms + 7) & ~7);
  return 2 * 2 * rows * 2 * ((Ms + 15) & ~15);
}
size_t tgemm_lds_bytes(int prec, int buf_bytes) {
  const int bbuf = prec == BLK_F64 ? TgChunk<BLK_F64>::BYTES
                                   : (prec == BLK_F32 ? TgChunk<BLK_F32>::BYTES : TgChunk<BLK_BF16>::BYTES);
  return 2 * (size_t)((buf_bytes + 1023) & ~1023) + 2 * (size_t)bbuf;
}
int tgemm_max_nt(int prec, int Ps) {
  if (prec == BLK_F64) return kTgMaxNt;
  for (int nt = kTgMaxNt; nt > 1; --nt)
    if (tgemm_lds_bytes(prec, tgemm_buf_elems(prec, Ps, Ps, 8 * nt)) <= 96 * 1024) return nt;
  return 1;
}
// FP64 Toeplitz staging holds ntp <= 512 (P up to 125 for M2L); the
// reduced-precision operator rows of one row tile must fit the LDS budget
bool tgemm_supported(int prec, int Ps, int Pd) {
  if (prec == BLK_F64) return tg_table_stride(2 * (Ps + Pd) + 1) <= TG_PF64 * BLK_THREADS;
  return tgemm_lds_bytes(prec, tgemm_buf_elems(prec, Ps, Pd, 8)) <= 96 * 1024;
}
template <int PREC, int NTM>
static void tgemm_one(hipStream_t s, dim3 grid, size_t lds, int Rp, const TgItem* items, int nitems, int be,
                      const TgPair* pairs, const double2* tdata, const void* olo, const double2* src,
                      const void* src_lo, const double* scale, int sstride, double2* dst, int add) {
  hipLaunchKernelGGL((k_tgemm<PREC, NTM>), grid, dim3(BLK_THREADS), lds, s, Rp, items, nitems, pairs, tdata, olo, src,
                     src_lo, scale, sstride, dst, add, (be + 1023) & ~1023);
}
template <int PREC>
static void tgemm_prec(int ntm, hipStream_t s, dim3 grid, size_t lds, int Rp, const TgItem* items, int nitems, int be,
                       const TgPair* pairs, const double2* tdata, const void* olo, const double2* src,
                       const void* src_lo, const double* scale, int sstride, double2* dst, int add) {
  if (ntm <= 2)
    tgemm_one<PREC, 2>(s, grid, lds, Rp, items, nitems, be, pairs, tdata, olo, src, src_lo, scale, sstride, dst, add);
  else if (ntm <= 4)
    tgemm_one<PREC, 4>(s, grid, lds, Rp, items, nitems, be, pairs, tdata, olo, src, src_lo, scale, sstride, dst, add);
  else
    tgemm_one<PREC, 8>(s, grid, lds, Rp, items, nitems, be, pairs, tdata, olo, src, src_lo, scale, sstride, dst, add);
}
void launch_tgemm(hipStream_t s, int prec, int ntm, int Rp, const TgItem* items, int nitems, int buf_elems,
                  const TgPair* pairs, const double2* tdata, const void* olo, const double2* src, const void* src_lo,
                  const double* scale, int sstride, double2* dst, int add) {
  if (nitems <= 0) return;
  const size_t lds = tgemm_lds_bytes(prec, buf_elems);
  // a multiple of 8 blocks: block b takes item (b mod 8) * ceil(n / 8) + b / 8
  const dim3 grid((nitems + 7) / 8 * 8, Rp / kBlkCols);
  if (prec == BLK_F64)
    tgemm_prec<BLK_F64>(ntm, s, grid, lds, Rp, items, nitems, buf_elems, pairs, tdata, olo, src, src_lo, scale, sstride,
                        dst, add);
  else if (prec == BLK_F32)
    tgemm_prec<BLK_F32>(ntm, s, grid, lds, Rp, items, nitems, buf_elems, pairs, tdata, olo, src, src_lo, scale, sstride,
                        dst, add);
  else
    tgemm_prec<BLK_BF16>(ntm, s, grid, lds, Rp, items, nitems, buf_elems, pairs, tdata, olo, src, src_lo, scale,
                         sstride, dst, add);
}
void launch_lo_tables(hipStream_t s, int prec, int ntab, const int64_t* toff, const int* P_of, const int* lev_of,
                      const int* img_of, const int64_t* off, const double* scale, int sstride, const double2* tdata,
                      void* out) {
  if (ntab > 0)
    hipLaunchKernelGGL(k_lo_tables, dim3(ntab), dim3(256), 0, s, prec, ntab, toff, P_of, lev_of, img_of, off, scale,
                       sstride, tdata, out);
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
  hipLaunchKernelGGL((k_p2p_blk<PREC, CLS>), dim3((ni + 7) / 8 * 8, Rp / kBlkCols), dim3(BLK_THREADS), 0, s, tv, Rp, items, ni,
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
  const void* fs[] = {(const void*)k_tgemm<BLK_F64, 2>,  (const void*)k_tgemm<BLK_F64, 4>,
                      (const void*)k_tgemm<BLK_F64, 8>,  (const void*)k_tgemm<BLK_F32, 2>,
                      (const void*)k_tgemm<BLK_F32, 4>,  (const void*)k_tgemm<BLK_F32, 8>,
                      (const void*)k_tgemm<BLK_BF16, 2>, (const void*)k_tgemm<BLK_BF16, 4>,
                      (const void*)k_tgemm<BLK_BF16, 8>};
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
