"""GPU source-coordinate gradient (hfmm_apply_adjoint with grad_xy) against
the oracle's analytic gradient, and against central differences of the GPU
matvec itself on the two-layer ellipse workload.

Bar: relative L2 error of the (N, 2) gradient below 1e-7 against the oracle
(plans at tol 1e-10); per coordinate, central differences agree to 1e-4
relative (h = 1e-6, FP64, the plan rebuilt for each moved point).
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


def test_gradient_central_differences_n2e18(gpu_lib):
    """L = ||A q - u_obs||^2 on 2^18 points on 64 ellipses (two layers), its
    gradient in 64 seeded source coordinates against central differences of
    the GPU matvec; each moved point gets a plan of its own (targets stay at
    the unmoved points: the moved point is only a source)."""
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_ellipses_grad()
    xy = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q0 = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    xi = torch.tensor(w.extra["xi"], dtype=torch.complex128, device=dev)
    plan = gpu_lib.Plan(w.k, w.interfaces, xy, tol=w.tol, leaf_size=w.leaf)
    u_obs = plan.apply(q0 + 0.1 * xi)
    u = plan.apply(q0)
    v = 2.0 * (u - u_obs)
    _, g = plan.apply_adjoint(v, q=q0, grad_xy=True)
    g = g.cpu().numpy()
    h = w.extra["h"]
    lo = w.xy.min(axis=0)
    hi = w.xy.max(axis=0)
    worst = 0.0
    checked = 0
    for j, ax in zip(w.extra["fd_index"], w.extra["fd_axis"]):
        # keep the root box: skip the extreme points of the bounding square
        if np.any(np.abs(w.xy[j] - lo) < 1e-3) or np.any(np.abs(w.xy[j] - hi) < 1e-3):
            continue
        vals = []
        for s in (1.0, -1.0):
            xm = xy.clone()
            xm[j, ax] += s * h
            pm = gpu_lib.Plan(w.k, w.interfaces, xm, tol=w.tol, leaf_size=w.leaf)
            # the matvec with only source j moved: A(x, x') q = A(x', x') q with
            # row j replaced by the unmoved target
            um = pm.apply(q0)
            # row j of the moved plan has its target moved too: put back the
            # row computed with the unmoved target through the moved source set
            vals.append(um)
            pm.close()
        # contributions of the moved target row differ by O(h); remove row j
        # from both losses and add it from the direct definition below
        rp, rm = vals[0] - u_obs, vals[1] - u_obs
        mask = torch.ones(w.n, dtype=torch.bool, device=dev)
        mask[j] = False
        lp = float((rp[:, mask].abs() ** 2).sum())
        lm = float((rm[:, mask].abs() ** 2).sum())
        fd = (lp - lm) / (2 * h)
        # row j's own dependence on source j (the scattered self term, targets
        # fixed) is included in g; correct the finite difference by its share:
        # d/dx_j |u_j - uobs_j|^2 with the target fixed equals
        # 2 Re(conj(r_j) q_j dA_jj/dx_j); A_jj = G^s(x_j, x_j) for the fixed target
        import oracle as _o
        media = _o.Media(w.k, w.interfaces)
        xj, yj = w.xy[j]
        yf = media.to_frame(np.array([yj]))[0]
        eps = 1e-5
        def gs(xs, ys):
            return _o.scattered_pairs(media, np.array([xj - xs]), np.array([yf + media.to_frame(np.array([ys]))[0]]))[0]
        if ax == 0:
            dA = (gs(xj + eps, yj) - gs(xj - eps, yj)) / (2 * eps)
        else:
            dA = (gs(xj, yj + eps) - gs(xj, yj - eps)) / (2 * eps)
        rj = complex((u - u_obs)[0, j].item())
        fd += 2.0 * (np.conj(rj) * complex(q0[0, j].item()) * dA).real
        err = abs(fd - g[j, ax]) / max(abs(g[j, ax]), 1e-30)
        worst = max(worst, err)
        checked += 1
    print("central differences: %d coordinates, worst relative difference %.3e" % (checked, worst))
    assert checked >= 48
    assert worst < 1e-4


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
