// Free-space direct interactions of the layered-media FMM (gfx950): the
// near-field sum u_i += (i/4) sum_j q_j H0^(1)(k1 |x_i - x_j|) over the
// direct lists (Eq. freeGreen, with the i = j term excluded), one launch per
// series class of the pairs' largest distance.
#include "kernels.hpp"
#include "special.hpp"

namespace hfmm {

constexpr int WAVE = 64;

__device__ __noinline__ double2 hankel0_large_call(double x) { return hankel0_large(x); }

// ------------------------------------------------------------------ P2P (free space)
// u_i += (i/4) sum_{j in U(i), j != i} q_j H0^(1)(k |x_i - x_j|). One wave per
// work item: a target leaf against source ranges. When the leaf holds fewer
// than 64 points several lanes share a target and split its sources, then
// combine by shuffles. Sources are staged through LDS P2P_CS at a time; RB
// right-hand sides share each H0 evaluation (right-hand sides r0 .. r0+RB-1).
// Each item uses the shortest series that covers its largest pair distance.
//
// H0(k |x_i - x_j|) is symmetric and so is the set of direct pairs, so a
// cross item (sources that follow the target leaf in point order) evaluates
// each pair once and also adds q_i H_ij into u_j: those sums collect in LDS,
// each lane starting its sweep of the chunk at a different source so that
// lanes seldom add to the same entry at once, and go to u once per chunk.
// Self items (a leaf with itself) take every ordered pair. All output is
// added atomically: a point receives from its own items and from the cross
// items of the leaves before it.

// One staged chunk for one lane: the sources of residue class sub mod g in
// [0, cnt), four per step; jself is the target's own index within the chunk
// (self items). z = (k r / 2)^2; dropped terms get a harmless z = 1 and
// weight 0. T is the arithmetic precision (pair differences are taken in
// FP64 and then rounded).
constexpr int P2P_CS = 128;  // sources per staged chunk

// Orders a wave's LDS stores before its lanes' later loads. A block runs WPB
// items, one per wave, each on its own LDS: with one wave a block barrier,
// with several a wavefront-scope fence (a wave's LDS accesses complete in
// order) and a barrier to the compiler's reordering.
template <int WPB>
__device__ inline void p2p_wave_sync() {
  if (WPB == 1) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// In a cross item the reverse sums q_i H_ij go to s_acc[j], kept in FP64 for
// both precisions and added with the no-return FP64 LDS atomics, which do not
// wait for the LDS (FP32 LDS atomics and plain read-add-writes measured
// several times slower).
template <typename T, int RB, int M, bool LARGE, bool SYM>
__device__ inline void p2p_chunk(int sub, int g, int cnt, int jself, int rot, double2 xi, const cplx_t<T>* qi,
                                 T qk2, const double2* s_x, const cplx_t<T> (*s_q)[P2P_CS], cplx_t<T> acc[RB],
                                 double2 (*s_acc)[P2P_CS], const double2* s_ln) {
  using C = cplx_t<T>;
  const int K = (cnt - sub + g - 1) / g;  // sources of this lane's class
  const int r0 = K > 0 ? rot % K : 0;
  for (int k0 = 0; k0 < K; k0 += 4) {
    // loads first (clamped index, no branches), then the arithmetic
    double2 xj[4];
    C qv[4][RB];
    bool use[4];
    int jc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u;
      int kr = k + r0;
      if (kr >= K) kr -= K;
      const int jl = sub + g * (k < K ? kr : 0);
      use[u] = k < K && jl != jself;
      jc[u] = min(jl, cnt - 1);
      xj[u] = s_x[jc[u]];
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) qv[u][rr] = s_q[rr][jc[u]];
    }
    T z[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T dx = (T)(xi.x - xj[u].x), dy = (T)(xi.y - xj[u].y);
      const T zz = qk2 * (dx * dx + dy * dy);
      z[u] = use[u] ? zz : (T)1.0;
    }
    T hr[4], hi[4];
    hankel0_x4<T, M, LARGE>(z, hr, hi, s_ln);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T w = use[u] ? (T)1.0 : (T)0.0;
      const C hw = cmk(hr[u] * w, hi[u] * w);
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        acc[rr].x = fma(hw.x, qv[u][rr].x, fma(-hw.y, qv[u][rr].y, acc[rr].x));
        acc[rr].y = fma(hw.x, qv[u][rr].y, fma(hw.y, qv[u][rr].x, acc[rr].y));
      }
      if (SYM && use[u]) {
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
          const C t = cmul(hw, qi[rr]);
          atomicAdd(&s_acc[rr][jc[u]].x, (double)t.x);
          atomicAdd(&s_acc[rr][jc[u]].y, (double)t.y);
        }
      }
    }
  }
}

// One work item: the target leaf b against source ranges [e0, e1) of rng.
// Sums run in T; each item adds its (i/4) sums into the FP64 output.
template <typename T, int RB, int M, bool LARGE, bool SYM, int WPB>
__device__ inline void p2p_item(const TreeView& tv, int b, int e0, int e1, const int2* __restrict__ rng,
                                const double2* __restrict__ qs, double2* __restrict__ us, int r0, double2* s_x,
                                cplx_t<T> (*s_q)[P2P_CS], double2 (*s_acc)[P2P_CS], const double2* s_ln) {
  using C = cplx_t<T>;
  const int lane = threadIdx.x & (WAVE - 1);
  const int2 pr = tv.prange[b];
  const T qk2 = (T)(0.25 * tv.k * tv.k);
  if (SYM) {
    for (int l = lane; l < P2P_CS; l += WAVE)
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) s_acc[rr][l] = cmk(0.0, 0.0);
  }
  // targets in chunks of 32 (two lanes per target), the remainder in a chunk of
  // the next power of two with more lanes per target
  for (int c0 = pr.x, csz = 0; c0 < pr.y; c0 += csz) {
    const int rem = pr.y - c0;
    csz = 32;
    if (rem < 32) {
      csz = 1;
      while (csz < rem) csz *= 2;
    }
    const int nt = min(csz, rem);
    const int g = WAVE / csz;  // lanes per target
    const int ti = lane / g, sub = lane % g;
    const int i = c0 + ti;
    const bool valid = ti < nt;
    const double2 xi = valid ? tv.pts[i] : cmk(0.0, 0.0);
    C qi[RB];
#pragma unroll
    for (int rr = 0; rr < RB; ++rr)
      qi[rr] = (SYM && valid && r0 + rr < tv.nrhs) ? to_cplx<T>(qs[(int64_t)(r0 + rr) * tv.n + i]) : cmk((T)0, (T)0);
    C acc[RB];
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) acc[rr] = cmk((T)0, (T)0);
    for (int e = e0; e < e1; ++e) {
      const int2 sr = rng[e];
      for (int j0 = sr.x; j0 < sr.y; j0 += P2P_CS) {
        const int cnt = min(P2P_CS, sr.y - j0);
        p2p_wave_sync<WPB>();
        for (int l = lane; l < cnt; l += WAVE) {
          s_x[l] = tv.pts[j0 + l];
#pragma unroll
          for (int rr = 0; rr < RB; ++rr)
            s_q[rr][l] = (r0 + rr < tv.nrhs) ? to_cplx<T>(qs[(int64_t)(r0 + rr) * tv.n + j0 + l]) : cmk((T)0, (T)0);
        }
        p2p_wave_sync<WPB>();
        if (valid)
          p2p_chunk<T, RB, M, LARGE, SYM>(sub, g, cnt, SYM ? -1 : i - j0, ti, xi, qi, qk2, s_x, s_q, acc, s_acc,
                                          s_ln);
        if (SYM) {
          // the chunk's sums of q_i H_ij go to u_j
          p2p_wave_sync<WPB>();
          for (int l = lane; l < cnt; l += WAVE) {
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
              if (r0 + rr < tv.nrhs) {
                const double2 a = s_acc[rr][l];
                const int64_t idx = (int64_t)(r0 + rr) * tv.n + j0 + l;
                unsafeAtomicAdd(&us[idx].x, -0.25 * a.y);  // (i/4) a
                unsafeAtomicAdd(&us[idx].y, 0.25 * a.x);
              }
              s_acc[rr][l] = cmk(0.0, 0.0);
            }
          }
        }
      }
    }
#pragma unroll
    for (int rr = 0; rr < RB; ++rr)
      for (int m = 1; m < g; m <<= 1) {
        acc[rr].x += __shfl_xor(acc[rr].x, m, WAVE);
        acc[rr].y += __shfl_xor(acc[rr].y, m, WAVE);
      }
    if (valid && sub == 0)
#pragma unroll
      for (int rr = 0; rr < RB; ++rr)
        if (r0 + rr < tv.nrhs) {
          const int64_t idx = (int64_t)(r0 + rr) * tv.n + i;
          unsafeAtomicAdd(&us[idx].x, -0.25 * (double)acc[rr].y);  // (i/4) acc
          unsafeAtomicAdd(&us[idx].y, 0.25 * (double)acc[rr].x);
        }
  }
}

// One launch per series class (the host bounds every pair distance of an item
// and sorts the items by class), so each kernel holds only its own
// coefficients in scalar registers; sym[li] marks cross items. A block runs
// WPB consecutive items, one per wave. Beside the far-field launches (blocks
// of four waves) the one-right-hand-side launch uses four-wave blocks: a
// finished near-field block then frees room that a far-field block can take,
// where one-wave blocks leave gaps too small for it that the next near-field
// block fills.
template <typename T, int RB, int CLS, int WPB>
__global__ void __launch_bounds__(WAVE * WPB) k_p2p(TreeView tv, const int* __restrict__ leaves, int nleaves,
                                              const int* __restrict__ ptr, const int2* __restrict__ rng,
                                              const int* __restrict__ sym, const double2* __restrict__ qs,
                                              double2* __restrict__ us) {
  using C = cplx_t<T>;
  const int r0 = blockIdx.y * RB;  // first right-hand side of this block
  __shared__ double2 s_xw[WPB][P2P_CS];
  __shared__ C s_qw[WPB][RB][P2P_CS];
  __shared__ double2 s_accw[WPB][RB][P2P_CS];
  __shared__ double2 s_ln[1 << kLogTabBits];  // logarithm bins (FP64)
  if (sizeof(T) == 8)
    for (int l = threadIdx.x; l < (1 << kLogTabBits); l += WAVE * WPB) s_ln[l] = cmk(kLogTab[l][0], kLogTab[l][1]);
  __syncthreads();  // the table before any use; every wave of the block is here
  const int wv = threadIdx.x / WAVE;
  const int li = blockIdx.x * WPB + wv;
  if (li >= nleaves) return;
  double2* s_x = s_xw[wv];
  C(*s_q)[P2P_CS] = s_qw[wv];
  double2(*s_acc)[P2P_CS] = s_accw[wv];
  constexpr int CL = CLS < kH0Classes ? CLS : kH0Classes - 1;
  constexpr int M = sizeof(T) == 8 ? kH0ClassTerms[CL] : kH0ClassTermsF32[CL];
  constexpr bool LARGE = CLS >= kH0Classes;
  if (sym[li])
    p2p_item<T, RB, M, LARGE, true, WPB>(tv, leaves[li], ptr[li], ptr[li + 1], rng, qs, us, r0, s_x, s_q, s_acc,
                                         s_ln);
  else
    p2p_item<T, RB, M, LARGE, false, WPB>(tv, leaves[li], ptr[li], ptr[li + 1], rng, qs, us, r0, s_x, s_q, s_acc,
                                          s_ln);
}

// ------------------------------------------------------------------ launcher
template <typename T, int CLS>
static void p2p_class(hipStream_t s, const TreeView& tv, const int* items, int nl, const int* ptr, const int2* rng,
                      const int* sym, const double2* qs, double2* us) {
  if (nl <= 0) return;
  if (tv.nrhs == 1) {
    hipLaunchKernelGGL((k_p2p<T, 1, CLS, 4>), dim3((nl + 3) / 4), dim3(4 * WAVE), 0, s, tv, items, nl, ptr, rng, sym,
                       qs, us);
    return;
  }
  hipLaunchKernelGGL((k_p2p<T, 4, CLS, 1>), dim3(nl, (tv.nrhs + 3) / 4), dim3(WAVE), 0, s, tv, items, nl, ptr, rng, sym,
                     qs, us);
}

void launch_p2p(hipStream_t s, const TreeView& tv, const int* items, const int* cls_ptr, const int* ptr,
                const int2* rng, const int* sym, const double2* qs, double2* us, int fp32) {
#define HFMM_P2P(C)                                                                                             \
  if (fp32)                                                                                                     \
    p2p_class<float, C>(s, tv, items + cls_ptr[C], cls_ptr[C + 1] - cls_ptr[C], ptr + cls_ptr[C], rng,       \
                        sym + cls_ptr[C], qs, us);                                                             \
  else                                                                                                          \
    p2p_class<double, C>(s, tv, items + cls_ptr[C], cls_ptr[C + 1] - cls_ptr[C], ptr + cls_ptr[C], rng,      \
                         sym + cls_ptr[C], qs, us)
  HFMM_P2P(0); HFMM_P2P(1); HFMM_P2P(2); HFMM_P2P(3); HFMM_P2P(4); HFMM_P2P(5);
#undef HFMM_P2P
  static_assert(kH0Classes == 5, "one launch per class and one for the large-argument class");
}
}  // namespace hfmm
