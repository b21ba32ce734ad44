/*
 * hfmm.h - C interface of the MI355X heterogeneous FMM for the 2-D Helmholtz
 * equation in two- and three-layer media.
 *
 * The library applies the matrix A with entries A_ij = u_{x_j}(x_i), the
 * domain Green's function of the layered medium evaluated at target x_i for a
 * unit source at x_j (the discretised potential of Section 2.4 of Cho, Huang,
 * Chen and Cai, "A heterogeneous FMM for 2-D layered media Helmholtz equation
 * I"). Sources and targets are the same N points, all in the top layer
 * (Section 2.3). The Green's function is the free-space part
 * (i/4) H0^(1)(k1 |x - x0|) (Eq. freeGreen) plus the top-layer scattered field
 * given by the Sommerfeld integral with the reflection function sigma_1
 * (Eq. multitop); sigma_1 is the solution of the interface system of
 * Section 2.3 (two layers: the same system with k3 = k2).
 *
 * Self term: the singular free term i = j is left out; the smooth scattered
 * self term G^s(x_i, x_i) is included (HFMM_SELF_NONE drops it).
 *
 * Conventions shared by every call:
 *  - All arrays named "device" live in GPU memory of the current device; the
 *    caller owns them. The plan copies what it needs and keeps no caller
 *    pointer after a call returns.
 *  - Work is enqueued on the given stream and is asynchronous unless stated.
 *  - Complex values are interleaved (re, im) doubles; a complex array with
 *    "nrhs" right-hand sides is laid out [nrhs][n].
 *  - Points are interleaved (x, y) doubles, [n][2], in the caller's frame:
 *    interfaces are horizontal lines y = interfaces[i].
 *  - Errors are reported by status code only. Argument and domain checks run
 *    on the host before any launch. hfmm_last_error_message() returns a
 *    thread-local description of the last failure.
 *  - A plan's workspaces (expansions, contribution rows, near-interface node
 *    sums, the near field's side stream) belong to the plan: calls on one plan
 *    from several host threads, or on streams not ordered with each other,
 *    race. Different plans are independent.
 */
#ifndef HFMM_H
#define HFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hfmm_plan_s *hfmm_plan_t;
typedef void *hfmm_stream_t; /* a hipStream_t; NULL is the null stream */

typedef enum {
  HFMM_OK = 0,
  HFMM_ERR_INVALID_ARG = 1, /* NULL pointer, bad size, bad option value */
  HFMM_ERR_DOMAIN = 2,      /* point on/below the top interface, non-finite
                               value, coincident points */
  HFMM_ERR_UNSUPPORTED = 3, /* layers not 2 or 3, k <= 0, a lower layer with
                               a smaller wavenumber than the top layer */
  HFMM_ERR_NO_MEMORY = 4,
  HFMM_ERR_DEVICE = 5,      /* a HIP runtime error */
  HFMM_ERR_ACCURACY = 6     /* the tolerance cannot be met (expansion order
                               above its cap, or out of FP64 range), or a
                               Sommerfeld rule or near-interface table would
                               be too long for the point set */
} hfmm_status_t;

/* Self term of the matrix. HFMM_SELF_SCATTERED (default): A_ii is the
 * smooth scattered self term G^s(x_i, x_i) (the image of x_i lies 2 y_i away);
 * HFMM_SELF_NONE: A_ii = 0 (both the free and the scattered i = i term are
 * left out). The free term i = i is singular and is never included. */
enum { HFMM_SELF_SCATTERED = 0, HFMM_SELF_NONE = 1 };
/* Arithmetic of the hot stages.
 * HFMM_FP64: everything in double precision.
 * HFMM_FP32 (mixed): the multipole-to-local translations (free and
 *   heterogeneous) run as complex single-precision contractions on the FP32
 *   matrix cores on per-level scaled coefficients, and the free-space direct
 *   pairs (H0 series, logarithm, per-item sums) run in single precision with
 *   pair differences rounded from FP64. Tables are generated in FP64 and
 *   rounded once; P2M, M2M, L2L, L2P, the Bessel recurrences and the
 *   accumulation of u stay FP64.
 * HFMM_BF16 (mixed): as HFMM_FP32, with the multipole-to-local operands
 *   (tables and scaled coefficients) rounded to bfloat16 and multiplied on the
 *   BF16 matrix cores with FP32 accumulation.
 * The reduced-precision results carry about 1e-7 (FP32) or 1e-3 (BF16)
 * relative error on top of the tolerance. */
enum { HFMM_FP64 = 0, HFMM_FP32 = 1, HFMM_BF16 = 2 };

/* Caller-supplied device allocator (e.g. a framework's caching allocator):
 * alloc returns device memory of at least `bytes` bytes on the current device
 * (NULL on failure), free releases a pointer alloc returned. Both receive
 * alloc_ctx. The library releases its buffers only after the work that uses
 * them has completed. */
typedef void *(*hfmm_alloc_fn)(size_t bytes, void *ctx);
typedef void (*hfmm_free_fn)(void *ptr, void *ctx);

typedef struct {
  int32_t struct_size;      /* sizeof(hfmm_options_t) */
  int32_t leaf_size;        /* max points per leaf box; default 64 */
  int32_t precision;        /* HFMM_FP64 (default), HFMM_FP32 or HFMM_BF16 */
  int32_t self_term;        /* HFMM_SELF_SCATTERED (default) or HFMM_SELF_NONE */
  int32_t interface_refine; /* 1 (default): refine boxes touching the bottom
                               row until every image pair is admissible;
                               0: leave such pairs to direct Sommerfeld
                               quadrature */
  int32_t max_level;        /* deepest tree level; default 24 */
  double leaf_kb;           /* wavelength bound on leaves, which keeps the
                               direct pairs at small k1 r: a box is split
                               while k1 times its side exceeds leaf_kb and it
                               holds more than leaf_size / 4 points, or
                               exceeds 2 leaf_kb (default 1.5; 0 turns the
                               bound off). Must be 0 or >= 0.25. */
  int32_t top_level;        /* coarsest level of the expansions: multipole-
                               to-local pairs of coarser levels are split into
                               their children's pairs at this level, and the
                               passes up and down stop there. 2 is the
                               classical choice (every level that can hold a
                               separated pair); 0 (default) takes the
                               deepest level whose
                               boxes form at most 4096 ordered pairs and
                               which no leaf lies above. Must be 0 or >= 2;
                               it is lowered to the shallowest leaf level. */
  int32_t max_nrhs;         /* 0 (default): workspace grows on demand; > 0:
                               the workspace for this many right-hand sides is
                               reserved when the plan is built, so that applies
                               with up to max_nrhs right-hand sides allocate
                               nothing */
  int32_t deterministic;    /* 0 (default); 1: bitwise reproducible results
                               from run to run. hfmm_apply and
                               hfmm_apply_adjoint then run the right-hand-
                               side-blocked pipeline for any count (stages in
                               sequence on the caller's stream, no atomic
                               additions, every output element summed in a
                               fixed order, a fixed M2L tile shape): slower
                               for few right-hand sides, each pass being 64
                               columns wide. hfmm_plan fails with
                               HFMM_ERR_UNSUPPORTED where that pipeline
                               cannot run (a leaf expansion order above
                               40); coordinate
                               gradients and hfmm_apply_noalloc return
                               HFMM_ERR_UNSUPPORTED */
  int32_t order;            /* 0 (default): expansion order per level from
                               tol; > 0: this order at every level (the
                               paper's fixed-p experiments), at most 255 */
  double impedance;         /* layers == 1 only: alpha > 0 of the impedance
                               half-space (Section 2.2): one medium of
                               wavenumber wavenumbers[0] above y =
                               interfaces[0], with du/dn - i alpha u = 0 on
                               that line (n the outward normal, -y), whose
                               reflection function is (g + i alpha)/(g - i
                               alpha), g = sqrt(lambda^2 - k^2). Must be 0
                               (default) with two or three layers. */
  hfmm_alloc_fn alloc;      /* NULL (default): hipMalloc / hipFree */
  hfmm_free_fn free;        /* must be set together with alloc */
  void *alloc_ctx;
} hfmm_options_t;

typedef struct {
  int32_t levels;           /* number of tree levels (root = level 0) */
  int32_t order[32];        /* expansion order P_l per level (0 if unused) */
  int64_t boxes, leaves;
  int64_t m2l_pairs;        /* free-space multipole-to-local pairs */
  int64_t image_pairs;      /* heterogeneous (image) multipole-to-local pairs */
  int64_t p2p_pairs;        /* free-space direct point pairs */
  int64_t interface_pairs;  /* direct Sommerfeld point pairs */
  int64_t image_tables;     /* heterogeneous translation tables generated */
  double flops_m2l;         /* algorithmic flops of one apply, per RHS */
  double flops_updown;      /* P2M + M2M + L2L + L2P */
  double flops_p2p;         /* free-space direct part as evaluated: per H0
                               value 4M (series of M terms, by item class)
                               + 32 (logarithm, distance, assembly) + 8 per
                               complex multiply-add */
  double plan_seconds;
  int64_t p2p_evals;        /* H0 evaluations per apply and right-hand side:
                               each cross-leaf pair once, same-leaf pairs
                               in both orders */
  int32_t top_level;        /* coarsest level of the expansions in use */
  int32_t m2l_tile;         /* row tiles per multipole-to-local work item of
                               the many-right-hand-side contraction, chosen by
                               timing the candidates 2, 4, 8 on the plan's own
                               launch at its first such apply (0: not yet) */
  int32_t interface_nodes;  /* nodes of the near-interface quadrature rule
                               (0 without direct Sommerfeld pairs) */
  int64_t interface_leaf_pairs; /* (target leaf, source box) pairs of the
                               direct Sommerfeld part */
} hfmm_info_t;

/* Default options. */
void hfmm_default_options(hfmm_options_t *opts);

/*
 * Build a plan: tree, interaction lists, expansion orders and translation
 * tables (Algorithm 1, step 1; tables by FP64 quadrature of the Sommerfeld
 * form of the multipole-to-local operator, Section 3.3 Eq. m2loperator with
 * sigma_1 as in Section 5).
 *   layers       2 or 3; 1: the impedance half-space of Section 2.2 (its
 *                alpha in opts->impedance).
 *   wavenumbers  host [layers], top layer first, > 0; every lower layer must
 *                have k_j >= k_1.
 *   interfaces   host [max(layers-1, 1)], strictly decreasing heights (the
 *                half-space: its boundary).
 *   n            number of points, >= 1.
 *   points       device [n][2] doubles; every y strictly above interfaces[0].
 *   tol          requested relative accuracy, in [1e-14, 1e-2].
 *   opts         NULL for defaults.
 * On success *out owns the plan; release it with hfmm_destroy. The call
 * synchronises the stream (the tree is built on the GPU level by level, and
 * the lists and tables are planned on the host).
 */
hfmm_status_t hfmm_plan(hfmm_plan_t *out, int32_t layers, const double *wavenumbers,
                        const double *interfaces, int64_t n, const double *points, double tol,
                        const hfmm_options_t *opts, hfmm_stream_t stream);

/*
 * u = A q (Algorithm 1, steps 2-5).
 *   q  device complex [nrhs][n], user point order.
 *   u  device complex [nrhs][n], written (not accumulated).
 * q and u must not overlap. nrhs >= 1.
 */
hfmm_status_t hfmm_apply(hfmm_plan_t plan, const double *q, double *u, int32_t nrhs,
                         hfmm_stream_t stream);

/*
 * w = A^H v, the conjugate transpose, and optionally the gradient of
 * Re <v, A q> with respect to the source coordinates (the vector-Jacobian
 * product of u = A q for a real loss with dL/du = v in PyTorch's convention).
 * The stages run transposed in reverse order; A^H v = conj(A^T conj(v)).
 *   v        device complex [nrhs][n], user point order.
 *   w        device complex [nrhs][n], written.
 *   q        device complex [nrhs][n] or NULL (needed only for grad_xy).
 *   grad_xy  device [n][2] doubles or NULL: grad_xy[j] =
 *            sum_r Re( q_rj sum_i conj(v_ri) dA_ij/d(x_j, y_j) ), targets held
 *            fixed; the free i = j term stays excluded. Far field by the
 *            ladder relations of the cylindrical waves applied to the adjoint
 *            multipole coefficients, direct pairs by H_1^(1), near-interface
 *            pairs by the same Sommerfeld rule as the apply.
 * Errors: HFMM_ERR_INVALID_ARG for NULL plan, v or w, nrhs < 1, or grad_xy
 * without q; HFMM_ERR_NO_MEMORY / HFMM_ERR_DEVICE from the workspace or the
 * launches. Buffers must not overlap.
 */
hfmm_status_t hfmm_apply_adjoint(hfmm_plan_t plan, const double *v, double *w, int32_t nrhs,
                                 const double *q, double *grad_xy, hfmm_stream_t stream);

/*
 * Batches of independent geometries (same medium, tolerance and options):
 * one plan per geometry, applied together so that small geometries share
 * the GPU with large ones.
 *   hfmm_plan_batch  builds nplans plans from n[g] points at the device
 *                    pointers points[g] (host arrays of nplans entries); the
 *                    batch owns the plans. Synchronises like hfmm_plan.
 *   hfmm_apply_batch u[g] = A_g q[g] for every g, q and u host arrays of
 *                    device pointers ([nrhs][n[g]] complex each), stream
 *                    ordered on stream: the plans run on up to four internal
 *                    streams (default priority) forked from and joined back
 *                    to stream.
 *   hfmm_batch_graph with enable != 0, hfmm_apply_batch captures its launches
 *                    into a HIP graph on the first call for a set of
 *                    (q, u, nrhs, stream) and replays the graph on later calls
 *                    with the same set (stage profiling is switched off).
 *   hfmm_batch_plan  the g-th plan (owned by the batch), e.g. for its info
 *                    or adjoint.
 * Errors: HFMM_ERR_INVALID_ARG for NULL arrays, entries or nrhs < 1; the
 * plan errors of hfmm_plan / hfmm_apply; HFMM_ERR_DEVICE for stream, event or
 * graph failures.
 */
typedef struct hfmm_batch_s *hfmm_batch_t;
hfmm_status_t hfmm_plan_batch(hfmm_batch_t *out, int32_t nplans, int32_t layers, const double *wavenumbers,
                              const double *interfaces, const int64_t *n, const double *const *points,
                              double tol, const hfmm_options_t *opts, hfmm_stream_t stream);
hfmm_status_t hfmm_apply_batch(hfmm_batch_t batch, const double *const *q, double *const *u, int32_t nrhs,
                               hfmm_stream_t stream);
hfmm_status_t hfmm_batch_graph(hfmm_batch_t batch, int32_t enable);
hfmm_status_t hfmm_batch_plan(hfmm_batch_t batch, int32_t g, hfmm_plan_t *out);
void hfmm_batch_destroy(hfmm_batch_t batch);

/*
 * u = A q like hfmm_apply, for callers that cannot allocate device memory
 * during the call (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation): the apply's workspace comes from a fixed device
 * array of HFMM_NOALLOC_BYTES that the library holds on every GPU it runs on
 * until the process ends, and the call makes no allocation of its own.
 *   q, u, nrhs, stream  as for hfmm_apply.
 * Right-hand sides go through in passes of as many as fit the array.
 * Errors: HFMM_ERR_INVALID_ARG as hfmm_apply; HFMM_ERR_NO_MEMORY when one
 * right-hand side of this plan needs more than HFMM_NOALLOC_BYTES (about
 * 32 n + 32 ctot + 8 cstride bytes: points, expansion coefficients and
 * multipole-to-local rows; roughly n <= 1.5e5 points at tolerance 1e-8);
 * HFMM_ERR_DEVICE if the array's address cannot be found.
 * All calls on one GPU share its array: calls that overlap on one GPU (other
 * host threads, or streams not ordered with each other) race.
 */
#define HFMM_NOALLOC_BYTES ((size_t)64 << 20)
hfmm_status_t hfmm_apply_noalloc(hfmm_plan_t plan, const double *q, double *u, int32_t nrhs,
                                 hfmm_stream_t stream);

/*
 * The quadtree and interaction lists of a point set as hfmm_plan builds them
 * (Section 3.1: the adaptive partition of the points; Section 3.3: the box
 * pairs of the free and heterogeneous multipole-to-local translations), for
 * inspection and tests.
 *   wavenumbers[0], interfaces[0]: the top layer's wavenumber and the top
 *       interface (the wavelength bound and the interface frame);
 *   points: device pointer, n x 2 doubles (x, y), as for hfmm_plan;
 *   opts: NULL or options; leaf_size, leaf_kb, interface_refine, max_level
 *       and top_level are read;
 *   builder: HFMM_TREE_GPU, the HIP kernels every plan runs (Morton keys, a
 *       radix sort, level-by-level splitting, pair-frontier lists), or
 *       HFMM_TREE_HOST, the host reference builder (comparison sort and a
 *       depth-first dual-tree traversal) that the GPU builder is checked
 *       against. Both give the same tree bit for bit.
 * Synchronises the stream. Errors as for hfmm_plan: HFMM_ERR_DOMAIN (a point
 * not finite, not strictly above the top interface, or two coincident
 * points), HFMM_ERR_ACCURACY (a tree deeper than 32 levels),
 * HFMM_ERR_INVALID_ARG, HFMM_ERR_DEVICE, HFMM_ERR_NO_MEMORY.
 */
typedef struct hfmm_tree_s *hfmm_tree_t;
enum { HFMM_TREE_GPU = 0, HFMM_TREE_HOST = 1 };
hfmm_status_t hfmm_tree_build(hfmm_tree_t *out, const double *wavenumbers, const double *interfaces, int64_t n,
                              const double *points, const hfmm_options_t *opts, int32_t builder,
                              hfmm_stream_t stream);
/* counts[0..7] = n, boxes, levels, top level, and the lengths of the lists
 * fv (free M2L pairs), iv (image M2L pairs), fu (free direct pairs), iu
 * (near-interface direct pairs). */
hfmm_status_t hfmm_tree_counts(hfmm_tree_t tree, int64_t counts[8]);
/* Copies into host buffers sized from hfmm_tree_counts (a NULL buffer is
 * skipped): frame[0..2] = root side S, x0 = min x, y0 = min (y - interface);
 * keys[n], the sorted Morton keys (2 x 30 bits, x in the even bits); perm[n],
 * the input index of each sorted point (ties by input index);
 * boxes[12 * boxes]: per box level, ix, iy, begin, end (its sorted points),
 * parent (-1 at the root), quadrant, child[4] (-1: none) and leaf (0 / 1), in
 * breadth-first order (the boxes of a level contiguous, in Morton order);
 * lev_begin[levels + 1], the first box of each level; each list as (t, s)
 * pairs of box indices, sorted by t, then s. */
hfmm_status_t hfmm_tree_copy(hfmm_tree_t tree, double *frame, uint64_t *keys, int32_t *perm, int32_t *boxes,
                             int32_t *lev_begin, int32_t *fv, int32_t *iv, int32_t *fu, int32_t *iu);
/* NULL is a no-op. */
void hfmm_tree_destroy(hfmm_tree_t tree);

/*
 * A boundary integral equation solved around the matvec (Section 1: the
 * dense Nystrom system whose applications the method provides): restarted
 * GMRES(restart) for (A W + D) phi = f with W = diag(w) and
 *   D_ii = (i/4) w_i [1 + (2i/pi)(ln(k1 w_i / 4) + gamma_E - 1)],
 * the trapezoidal Nystrom form of the single-layer equation S phi = f on
 * closed curves in the top layer: the plan's points are the nodes, equispaced
 * in a periodic parameter of each curve, w_i = |x'(t_i)| dt their weights; A
 * is the plan's matrix (the domain Green's function between distinct nodes
 * and the smooth scattered self term), and D adds the free part's logarithmic
 * singularity integrated over each node's own panel by the small-argument
 * form of H0^(1) (a first-order local correction, no high-order end-point
 * corrections). E.g. a sound-soft obstacle lit by u_inc: f = -u_inc at the
 * nodes; the scattered field is then sum_j G(x, x_j) w_j phi_j.
 *   w      device [n] doubles, user point order.
 *   f      device complex [n].
 *   phi    device complex [n]: the initial guess on entry, the solution on
 *          return.
 *   tol    relative residual ||f - (A W + D) phi|| / ||f|| to reach, (0, 1).
 *   restart, max_iter  Krylov dimension (1..1000) and most matvecs.
 *   iterations, residual  NULL or host outputs: matvecs used and the final
 *          relative residual (recomputed with a true product).
 * The plan's applies run on the stream; the call synchronises it after every
 * inner product. Returns HFMM_OK also when max_iter ends the iteration: check
 * *residual. Errors: HFMM_ERR_INVALID_ARG, HFMM_ERR_NO_MEMORY (the Krylov basis
 * of restart + 1 vectors), and those of hfmm_apply.
 */
hfmm_status_t hfmm_bie_solve(hfmm_plan_t plan, const double *w, const double *f, double *phi, double tol,
                             int32_t restart, int32_t max_iter, int32_t *iterations, double *residual,
                             hfmm_stream_t stream);

/*
 * The field below the top interface of top-layer sources: the middle- and
 * bottom-layer fields of Section 2.3 (u_2 = u_2^t + u_2^b with the densities
 * sigma_2^+ and sigma_2^-, u_3 with sigma_3, from the interface system; two
 * layers: the field of the lower half-space),
 *   u_rt = sum_s q_rs G(x_t, x_s),  x_s in layer 1, x_t in layer 2 or 3
 * (a target at or above the lower interface is in layer 2). The spectral
 * integral factors into a source and a target part, so one quadrature rule
 * for the whole point sets (a contour below the branch points and the slab's
 * guided-mode poles, built on the host from the sets' extents) gives the sum
 * in O((ns + nt) Q) for Q nodes; Q grows with the x range times the largest
 * wavenumber and with 1 / (the nearest source's height + the nearest
 * target's depth).
 *   layers, wavenumbers, interfaces  as hfmm_plan; layers 2 or 3.
 *   ns, src   device [ns][2] doubles, every y strictly above interfaces[0].
 *   q         device complex [nrhs][ns].
 *   nt, tgt   device [nt][2] doubles, every y strictly below interfaces[0].
 *   u         device complex [nrhs][nt], written.
 *   tol       relative accuracy of the quadrature, in [1e-14, 1e-2].
 * Allocates its node tables and sums with hipMalloc and synchronises the
 * stream (the points' extents are read on the host). Errors:
 * HFMM_ERR_INVALID_ARG (NULL pointers, sizes, tol), HFMM_ERR_UNSUPPORTED
 * (layers not 2 or 3, k not finite and > 0), HFMM_ERR_DOMAIN (a source not
 * above or a target not below the top interface, a non-finite coordinate),
 * HFMM_ERR_ACCURACY (the rule would pass 200000 panels), HFMM_ERR_NO_MEMORY,
 * HFMM_ERR_DEVICE.
 */
hfmm_status_t hfmm_transmit(int32_t layers, const double *wavenumbers, const double *interfaces, int64_t ns,
                            const double *src, const double *q, int32_t nrhs, int64_t nt, const double *tgt,
                            double *u, double tol, hfmm_stream_t stream);

/*
 * The reverse pairs: sources below the top interface (layer 2 or 3), targets
 * in the top layer, u_rt = sum_s q_rs G(x_t, x_s). The domain Green's function
 * is symmetric (the interface conditions of Section 2.3 make the operator
 * self-adjoint), G(x_t, x_s) = G(x_s, x_t), so this is the transpose of
 * hfmm_transmit's sum: the same rule, the lower-layer factors in the source
 * sums and e^{-g1 y} at the targets. Arguments as hfmm_transmit with the
 * roles of the sets exchanged: every source y strictly below, every target y
 * strictly above interfaces[0].
 */
hfmm_status_t hfmm_transmit_up(int32_t layers, const double *wavenumbers, const double *interfaces, int64_t ns,
                               const double *src, const double *q, int32_t nrhs, int64_t nt, const double *tgt,
                               double *u, double tol, hfmm_stream_t stream);

/*
 * Sources and targets in the middle layer of three layers: the middle layer's
 * scattered field (the paper leaves sources below the top layer to a
 * follow-up; this takes the interface conditions of Section 2.3 with the free
 * field of a layer-2 source as the incident field):
 *   u_rt = sum_s q_rs G^s_22(x_t, x_s),
 * G^s_22 the waves of a layer-2 source reflected at the top and at the lower
 * interface with all their round trips (four spectral terms: two mirror
 * images and two shifted by e^{-2 g2 d}); the smooth pair of a point with
 * itself is included. The full middle-layer matvec adds the free part
 * (i/4) H0(k2 |x_t - x_s|), i.e. hfmm_apply of a plan whose layers all have
 * the wavenumber k2 (no reflection) over the same points. As hfmm_transmit:
 * one quadrature rule for the whole point sets, O((ns + nt) Q).
 *   wavenumbers   host [3]; interfaces host [2], strictly decreasing.
 *   ns, src   device [ns][2] doubles; nt, tgt device [nt][2] doubles; every
 *             point strictly between the interfaces.
 *   q         device complex [nrhs][ns]; u device complex [nrhs][nt], written.
 *   tol       relative accuracy of the quadrature, in [1e-14, 1e-2].
 * Allocates with hipMalloc and synchronises the stream. Errors as
 * hfmm_transmit (HFMM_ERR_DOMAIN: a point not strictly inside the middle
 * layer).
 */
hfmm_status_t hfmm_middle_scattered(const double *wavenumbers, const double *interfaces, int64_t ns,
                                    const double *src, const double *q, int32_t nrhs, int64_t nt,
                                    const double *tgt, double *u, double tol, hfmm_stream_t stream);

/* Plan statistics (host struct, filled synchronously). */
hfmm_status_t hfmm_plan_info(hfmm_plan_t plan, hfmm_info_t *out);

/*
 * Stage timing (diagnostics). While enabled, every hfmm_apply records HIP
 * events on its stream between its stages, and the stages of hfmm_apply and
 * hfmm_apply_adjoint run one after another on that stream (the near field is
 * not run beside the far field, as during graph capture; results agree with
 * the overlapped form up to the order of rounding). hfmm_profile_read synchronises the
 * device, writes the accumulated milliseconds per stage and the number of
 * applies into stage_ms[0..HFMM_NSTAGES-1] and *napplies, and clears the
 * accumulators. Stages: see hfmm_stage_name.
 */
enum { HFMM_NSTAGES = 9 };
hfmm_status_t hfmm_profile_enable(hfmm_plan_t plan, int32_t enable);
hfmm_status_t hfmm_profile_read(hfmm_plan_t plan, double *stage_ms, int32_t *napplies);
const char *hfmm_stage_name(int32_t stage);

/* Release a plan and its device memory (synchronises the device). NULL is a no-op. */
void hfmm_destroy(hfmm_plan_t plan);

const char *hfmm_status_string(hfmm_status_t status);
const char *hfmm_last_error_message(void);

#ifdef __cplusplus
}
#endif
#endif /* HFMM_H */
