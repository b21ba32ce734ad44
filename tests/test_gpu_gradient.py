"""GPU source-coordinate gradient (hfmm_apply_adjoint with grad_xy) against
the oracle's analytic gradient, and against central differences of the GPU
matvec itself on the two-layer ellipse workload.

Bar: relative L2 error of the (N, 2) gradient below 1e-7 against the oracle
(plans at tol 1e-10); per coordinate, central differences agree to 1e-6
relative (h = 1e-6, FP64, the plan rebuilt for each moved point with the
same tree); an FP32-near-field plan's gradient equals the FP64 plan's to
1e-12 (both run the FP64 gradient kernels).
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _grad_case(hf, w, tol, seed, **opts):
    import torch
    dev = torch.device("cuda:0")
    rng = workloads.rng_for(1703, 9136, seed)
    v = workloads.complex_normal(rng, (1, w.n))
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    plan = hf.Plan(w.k, w.interfaces, pts, tol=tol, **opts)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    vv = torch.tensor(v, dtype=torch.complex128, device=dev)
    wv, g = plan.apply_adjoint(vv, q=q, grad_xy=True)
    media = oracle.Media(w.k, w.interfaces)
    ref = oracle.source_gradient(media, w.xy, w.q, v)
    # the adjoint itself: w = A^H v = conj(A^T conj v) and A is symmetric
    wref = np.conj(oracle.direct_apply(media, w.xy, np.conj(v)))
    return plan, g.cpu().numpy(), ref, wv.cpu().numpy(), wref


def test_gradient_two_layer_n1024(gpu_lib):
    w = workloads.two_layer_uniform()
    plan, g, ref, wv, wref = _grad_case(gpu_lib, w, 1e-10, 81, leaf_size=32)
    e = rel(g, ref)
    print("two-layer N=1024 gradient E =", e, "adjoint E =", rel(wv, wref))
    assert e < 1e-7
    assert rel(wv, wref) < 1e-9


def test_gradient_with_near_interface_pairs(gpu_lib):
    """No interface refinement and no wavelength bound: the near-interface
    quadrature pairs take part."""
    w = workloads.two_layer_uniform(n=1024, seed=12)
    plan, g, ref, _, _ = _grad_case(gpu_lib, w, 1e-10, 82, leaf_size=32, interface_refine=0, leaf_kb=0.0)
    assert plan.info()["interface_pairs"] > 0
    e = rel(g, ref)
    print("near-interface gradient E =", e)
    assert e < 1e-7


def test_gradient_three_layer(gpu_lib):
    import math
    k3 = (2 * math.pi * 20, 2 * math.pi * 30, 2 * math.pi * 25)
    rng = workloads.rng_for(1703, 9136, 83)
    n = 1500
    xy = workloads.random_points_above(rng, n, k3, (0.5, 0.0), height=(0.01, 0.8))
    q = workloads.complex_normal(rng, (1, n))
    w = workloads.Workload("three-layer reduced", k3, (0.5, 0.0), xy, q, leaf=32, tol=1e-10)
    plan, g, ref, _, _ = _grad_case(gpu_lib, w, 1e-10, 84, leaf_size=32)
    e = rel(g, ref)
    print("three-layer gradient E =", e)
    assert e < 1e-7


def test_autograd_points_and_strengths(gpu_lib):
    """torch autograd through hfmm_apply_autograd: grad_q = A^H grad_u and the
    point gradient equal the direct calls."""
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_uniform(n=600, seed=85)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev, requires_grad=True)
    plan = gpu_lib.Plan(w.k, w.interfaces, pts.detach(), tol=1e-10, leaf_size=32)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev, requires_grad=True)
    u = gpu_lib.hfmm_apply_autograd(q, plan, pts)
    target = torch.zeros_like(u)
    loss = (u - target).abs().pow(2).sum()
    loss.backward()
    v = 2.0 * u.detach()
    wref, gref = plan.apply_adjoint(v, q=q.detach(), grad_xy=True)
    assert torch.allclose(q.grad, wref, rtol=0, atol=1e-12 * float(wref.abs().max()))
    assert torch.allclose(pts.grad, gref, rtol=0, atol=1e-12 * float(gref.abs().max()))


def _fd_case(gpu_lib, precision):
    """L = ||A q - u_obs||^2 on 2^18 points on 64 ellipses (two layers): the
    plan's gradient in 64 seeded source coordinates against central
    differences of the FP64 matvec. Each moved point gets a plan of its own;
    a coordinate counts only when that plan has the same tree and lists as
    the unmoved one (the FMM error then varies smoothly with the point).
    Targets stay at the unmoved points: row j of a moved plan (whose target
    moved too) is left out of the difference and its share, with the target
    held fixed, is added from the oracle's d/dY G^s (zero in x). The loss
    difference is summed as Re((r+ - r-) conj(r+ + r-)), which avoids the
    cancellation of two large sums of squares.

    Neighbouring points on an ellipse lie about 7.7e-5 apart, where the
    logarithm in H0 makes the O(h^2) term of a central difference with
    h = 1e-6 about (h / r)^2 / 3 = 6e-5 of that pair's share; the differences
    at h and 2h are therefore combined by Richardson extrapolation,
    (4 D(h) - D(2h)) / 3, which removes that term. Returns the relative
    differences of D(h) and of the extrapolated value."""
    import torch
    import oracle as _o
    dev = torch.device("cuda:0")
    w = workloads.two_layer_ellipses_grad()
    media = _o.Media(w.k, w.interfaces)
    xy = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q0 = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    xi = torch.tensor(w.extra["xi"], dtype=torch.complex128, device=dev)
    plan = gpu_lib.Plan(w.k, w.interfaces, xy, tol=w.tol, leaf_size=w.leaf)
    base_info = plan.info()
    u_obs = plan.apply(q0 + 0.1 * xi)
    u = plan.apply(q0)
    v = 2.0 * (u - u_obs)
    gplan = plan if precision == gpu_lib.HFMM_FP64 else gpu_lib.Plan(w.k, w.interfaces, xy, tol=w.tol,
                                                                        leaf_size=w.leaf, precision=precision)
    _, g = gplan.apply_adjoint(v, q=q0, grad_xy=True)
    g = g.cpu().numpy()
    keys = ("levels", "boxes", "leaves", "m2l_pairs", "image_pairs", "p2p_pairs", "interface_pairs")
    h = w.extra["h"]
    errs, errs_h = [], []
    for j, ax in zip(w.extra["fd_index"], w.extra["fd_axis"]):
        mask = torch.ones(w.n, dtype=torch.bool, device=dev)
        mask[j] = False
        same = True
        fds = []
        for step in (h, 2 * h):
            um = []
            for s in (1.0, -1.0):
                xm = xy.clone()
                xm[j, ax] += s * step
                pm = gpu_lib.Plan(w.k, w.interfaces, xm, tol=w.tol, leaf_size=w.leaf)
                inf = pm.info()
                same = same and all(inf[k] == base_info[k] for k in keys)
                um.append(pm.apply(q0))
                pm.close()
            d = (um[0] - um[1])[:, mask]
            sm = (um[0] + um[1] - 2 * u_obs)[:, mask]
            fds.append(float((d * sm.conj()).real.sum()) / (2 * step))
        if not same:
            continue
        corr = 0.0
        if ax == 1:
            yf = media.to_frame(np.array([w.xy[j, 1]]))[0]
            dA = _o.scattered_pairs(media, 0.0, 2 * yf, d_dY=True)[0]
            rj = complex((u - u_obs)[0, j].item())
            corr = 2.0 * (np.conj(rj) * complex(q0[0, j].item()) * dA).real
        fd_h = fds[0] + corr
        fd = (4.0 * fds[0] - fds[1]) / 3.0 + corr
        scale = max(abs(g[j, ax]), 1e-30)
        errs.append(abs(fd - g[j, ax]) / scale)
        errs_h.append(abs(fd_h - g[j, ax]) / scale)
    if gplan is not plan:
        gplan.close()
    plan.close()
    return np.array(errs), np.array(errs_h)


def test_gradient_central_differences_n2e18(gpu_lib):
    errs, errs_h = _fd_case(gpu_lib, gpu_lib.HFMM_FP64)
    print("central differences (FP64): %d coordinates; h alone: worst %.3e, median %.3e; "
          "extrapolated: worst %.3e, median %.3e"
          % (errs.size, errs_h.max(), np.median(errs_h), errs.max(), np.median(errs)))
    assert errs.size >= 48
    assert errs.max() < 1e-6


def test_gradient_sums_over_right_hand_sides(gpu_lib):
    """The gradient of Re sum_r <v_r, A q_r> is the sum of the per-pair terms
    over r: two right-hand sides at once (the general near-field form) equal
    the two single ones added (the one-right-hand-side form)."""
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_uniform(n=1024, seed=86, nrhs=2)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    plan = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    v = torch.tensor(workloads.complex_normal(workloads.rng_for(1703, 9136, 87), (2, w.n)),
                     dtype=torch.complex128, device=dev)
    _, g2 = plan.apply_adjoint(v, q=q, grad_xy=True)
    _, ga = plan.apply_adjoint(v[0:1].contiguous(), q=q[0:1].contiguous(), grad_xy=True)
    _, gb = plan.apply_adjoint(v[1:2].contiguous(), q=q[1:2].contiguous(), grad_xy=True)
    g2 = g2.cpu().numpy()
    gs = (ga + gb).cpu().numpy()
    print("two right-hand sides vs the sum of single ones:", rel(g2, gs))
    assert rel(g2, gs) < 1e-12
    plan.close()


def test_fp32_plan_gradient_is_the_fp64_one(gpu_lib):
    """A plan with the FP32 near field computes its coordinate gradient with
    the FP64 kernels (the direct-pair gradient has one form, and the
    single-right-hand-side expansions stay FP64), so its gradient equals the
    FP64 plan's up to the order of rounding and the central-difference check
    above covers both precisions; its adjoint matvec carries the FP32 near
    field (1e-6 of the FP64 one)."""
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_uniform(n=4096, seed=88)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    v = torch.tensor(workloads.complex_normal(workloads.rng_for(1703, 9136, 89), (1, w.n)),
                     dtype=torch.complex128, device=dev)
    p64 = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-8, leaf_size=32)
    p32 = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-8, leaf_size=32, precision=gpu_lib.HFMM_FP32)
    w64, g64 = p64.apply_adjoint(v, q=q, grad_xy=True)
    w32, g32 = p32.apply_adjoint(v, q=q, grad_xy=True)
    eg = rel(g32.cpu().numpy(), g64.cpu().numpy())
    ew = rel(w32.cpu().numpy(), w64.cpu().numpy())
    print("FP32 plan vs FP64 plan: gradient %.2e, adjoint %.2e" % (eg, ew))
    assert eg < 1e-12
    assert ew < 1e-6
    p64.close()
    p32.close()
