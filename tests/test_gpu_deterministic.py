"""Deterministic mode: every apply and adjoint apply runs the right-hand-side-
blocked pipeline (no atomic additions, a fixed summation order, a fixed M2L
tile shape), so repeated calls agree bit for bit.

Bars: two calls equal bitwise (one and three right-hand sides, forward and
adjoint); deterministic vs default plan 1e-12 (the same FP64 approximation
summed in another order); vs the oracle at the plan tolerance; the adjoint
against the oracle's conjugate transpose; coordinate gradients and the
allocation-free entry point refused with HFMM_ERR_UNSUPPORTED; a plan with
near-interface quadrature pairs repeats bitwise and matches the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_deterministic_repeats_bitwise_and_matches(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_uniform(n=1024, seed=51, nrhs=3)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    det = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32, deterministic=1)
    ref = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32)
    for nr in (1, 3):
        a = det.apply(q[:nr]).cpu().numpy()
        b = det.apply(q[:nr]).cpu().numpy()
        assert np.array_equal(a, b), "forward applies differ between calls"
        e = rel(a, ref.apply(q[:nr]).cpu().numpy())
        print("nrhs %d: deterministic vs default %.2e" % (nr, e))
        assert e < 1e-12
    eo = rel(det.apply(q[:1]).cpu().numpy(), oracle.direct_apply(oracle.Media(w.k, w.interfaces), w.xy, w.q[:1]))
    print("deterministic vs oracle %.2e" % eo)
    assert eo < 1e-10
    # adjoint: repeats bitwise, equals the default plan's and the oracle's A^H v
    v = q[:2].conj() * 0.5 + q[1:3]
    wa = det.apply_adjoint(v).cpu().numpy()
    wb = det.apply_adjoint(v).cpu().numpy()
    assert np.array_equal(wa, wb), "adjoint applies differ between calls"
    assert rel(wa, ref.apply_adjoint(v).cpu().numpy()) < 1e-12
    # the oracle's A is symmetric (reciprocity, pinned in its own tests):
    # A^H v = conj(A conj(v))
    wd = np.conj(oracle.direct_apply(oracle.Media(w.k, w.interfaces), w.xy, np.conj(v[:1].cpu().numpy())))
    ea = rel(wa[:1], wd)
    print("deterministic adjoint vs oracle A^H %.2e" % ea)
    assert ea < 1e-10
    with pytest.raises(gpu_lib.HFMMError, match="UNSUPPORTED|gradient"):
        det.apply_adjoint(v[:1], q=q[:1], grad_xy=True)
    with pytest.raises(gpu_lib.HFMMError, match="UNSUPPORTED|deterministic"):
        det.apply_noalloc(q[:1], out=torch.empty_like(q[:1]))
    det.close()
    ref.close()


def test_deterministic_with_near_interface_pairs(gpu_lib):
    """Without interface refinement and wavelength bound the bottom boxes keep
    near-interface quadrature pairs; the blocked pipeline evaluates them too
    (one writer per point), so the deterministic plan repeats bitwise and
    matches the oracle and the default plan."""
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_uniform(n=1024, seed=12, nrhs=3)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    kw = dict(tol=1e-10, leaf_size=32, interface_refine=0, leaf_kb=0.0)
    ref = gpu_lib.Plan(w.k, w.interfaces, pts, **kw)
    assert ref.info()["interface_pairs"] > 0
    det = gpu_lib.Plan(w.k, w.interfaces, pts, deterministic=1, **kw)
    a = det.apply(q).cpu().numpy()
    assert np.array_equal(a, det.apply(q).cpu().numpy()), "forward applies differ between calls"
    e = rel(a, ref.apply(q).cpu().numpy())
    eo = rel(a[:1], oracle.direct_apply(oracle.Media(w.k, w.interfaces), w.xy, w.q[:1]))
    print("near-interface pairs %d: deterministic vs default %.2e, vs oracle %.2e"
          % (ref.info()["interface_pairs"], e, eo))
    assert e < 1e-12
    assert eo < 1e-10
    det.close()
    ref.close()
