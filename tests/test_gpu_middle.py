"""Sources and targets in the middle layer (hfmm_middle_scattered): the middle
layer's scattered field, the interface conditions of Section 2.3 with a
layer-2 source's free field as the incident field (the oracle's ``middle``
module, pinned by matched interfaces, reciprocity and continuity).

Bars: the scattered part against the oracle on points through the slab,
1e-10 at tol 1e-12; the full matvec, a plan with the slab's wavenumber in
every layer (free part only) plus the scattered part, against the oracle's
middle-layer matvec at 1e-8 (plan tol 1e-10); one wavenumber everywhere
leaves no scattered field (1e-13 of the free field); five right-hand sides
against single columns (1e-14); points outside the slab are HFMM_ERR_DOMAIN.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
KM = (2 * math.pi * 8, 2 * math.pi * 12, 2 * math.pi * 10)
IF3 = (0.5, 0.0)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def slab_points(seed, n, nrhs=1):
    rng = workloads.rng_for(1703, 9136, seed)
    xy = np.c_[rng.uniform(0.0, 1.0, n), IF3[0] - rng.uniform(0.02, 0.48, n)]
    return xy, workloads.complex_normal(rng, (nrhs, n))


def scat(hf, k, xy, q, tgt=None, tol=1e-12):
    import torch
    dev = torch.device("cuda:0")
    p = torch.tensor(xy, device=dev)
    t = p if tgt is None else torch.tensor(tgt, device=dev)
    return hf.middle_scattered(k, IF3, p, torch.tensor(q, device=dev), t, tol=tol).cpu().numpy()


def test_scattered_part_against_the_oracle(gpu_lib):
    xy, q = slab_points(301, 40)
    u = scat(gpu_lib, KM, xy, q[0])
    ref = oracle.middle_apply(oracle.Media(KM, IF3), xy, q[0], scattered_only=True)
    e = rel(u, ref)
    print("middle-layer scattered part vs oracle: %.2e" % e)
    assert e < 1e-10


def test_full_matvec_with_a_free_space_plan(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    xy, q = slab_points(302, 250)
    pts = torch.tensor(xy, device=dev)
    qt = torch.tensor(q, device=dev)
    # every layer k2: sigma_1 = 0, the plan's matvec is the free part
    plan = gpu_lib.Plan((KM[1], KM[1]), (float(xy[:, 1].min()) - 1.0,), pts, tol=1e-10, leaf_size=32)
    u = plan.apply(qt).cpu().numpy()[0] + scat(gpu_lib, KM, xy, q[0], tol=1e-10)
    plan.close()
    tid = np.arange(3, 250, 41)
    ref = oracle.middle_apply(oracle.Media(KM, IF3), xy, q[0], targets=tid)
    e = rel(u[tid], ref)
    print("middle-layer matvec vs oracle (%d targets): %.2e" % (tid.size, e))
    assert e < 1e-8


def test_homogeneous_medium_has_no_scattered_field(gpu_lib):
    xy, q = slab_points(303, 200)
    k = (40.0, 40.0, 40.0)
    u = scat(gpu_lib, k, xy, q[0])
    r = np.hypot(xy[:, None, 0] - xy[None, :, 0], xy[:, None, 1] - xy[None, :, 1])
    np.fill_diagonal(r, 1.0)
    from scipy.special import hankel1
    h = 0.25j * hankel1(0, 40.0 * r)
    np.fill_diagonal(h, 0.0)
    free = h @ q[0]
    print("homogeneous: |u| / |free| = %.2e" % (np.linalg.norm(u) / np.linalg.norm(free)))
    assert np.linalg.norm(u) < 1e-13 * np.linalg.norm(free)


def test_several_right_hand_sides_and_separate_targets(gpu_lib):
    xy, q = slab_points(304, 500, nrhs=5)
    tgt, _ = slab_points(305, 300)
    u = scat(gpu_lib, KM, xy, q, tgt=tgt, tol=1e-10)
    cols = np.stack([scat(gpu_lib, KM, xy, q[r], tgt=tgt, tol=1e-10) for r in range(5)])
    assert u.shape == (5, 300)
    assert rel(u, cols) < 1e-14


def test_points_outside_the_slab_are_refused(gpu_lib):
    xy, q = slab_points(306, 20)
    for y in (IF3[0] + 0.01, IF3[1] - 0.01, IF3[0]):
        bad = xy.copy()
        bad[4, 1] = y
        with pytest.raises(gpu_lib.HFMMError) as ei:
            scat(gpu_lib, KM, bad, q[0])
        assert ei.value.status == 2  # HFMM_ERR_DOMAIN
