"""Fields below the top interface of top-layer sources (hfmm_transmit): the
middle- and bottom-layer fields of Section 2.3 for a source set in the top
layer and targets in the layers below.

Bars: one wavenumber everywhere gives the free field (i/4) H0(k r) (scipy's
Hankel function) to 1e-10; three layers (targets in the middle and the bottom
layer) and two layers against the oracle's sum of the middle- and
bottom-layer densities to 1e-10 at tol 1e-12, and the reverse pairs (sources
below, targets in the top layer) against the same fields read by
reciprocity; the pairs between the middle and the bottom layer (both
directions, by the mirrored medium) against the oracle's middle-layer source
to 1e-10; five right-hand sides (two
groups of the node sums) against single columns to 1e-14; points on the
wrong side of the interface are HFMM_ERR_DOMAIN, the impedance half-space
HFMM_ERR_UNSUPPORTED.
"""
import math

import numpy as np
import pytest
from scipy.special import hankel1

import oracle
import workloads

pytestmark = pytest.mark.gpu
K3 = (2 * math.pi * 10, 2 * math.pi * 15, 2 * math.pi * 12.5)
IF3 = (0.5, 0.0)
K2 = (8 * math.pi, 12 * math.pi)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sets(seed, ifs, ns, nt, depth):
    rng = workloads.rng_for(1703, 9136, seed)
    src = np.c_[rng.uniform(0.0, 1.0, ns), ifs[0] + rng.uniform(0.01, 0.3, ns)]
    tgt = np.c_[rng.uniform(0.0, 1.0, nt), ifs[0] - rng.uniform(0.01, depth, nt)]
    q = workloads.complex_normal(rng, (5, ns))
    return src, tgt, q


def run(hf, k, ifs, src, q, tgt, tol):
    import torch
    dev = torch.device("cuda:0")
    return hf.transmit(k, ifs, torch.tensor(src, device=dev), torch.tensor(q, device=dev),
                       torch.tensor(tgt, device=dev), tol=tol).cpu().numpy()


@pytest.mark.parametrize("ks,ifs", [((31.0, 31.0, 31.0), IF3), ((31.0, 31.0), (0.0,))])
def test_homogeneous_medium_gives_the_free_field(gpu_lib, ks, ifs):
    src, tgt, q = sets(201, ifs, 400, 300, 0.9)
    u = run(gpu_lib, ks, ifs, src, q[0], tgt, 1e-12)
    r = np.hypot(tgt[:, None, 0] - src[None, :, 0], tgt[:, None, 1] - src[None, :, 1])
    ref = (0.25j * hankel1(0, ks[0] * r)) @ q[0]
    e = rel(u, ref)
    print("homogeneous %d layers: %.2e" % (len(ks), e))
    assert e < 1e-10


@pytest.mark.parametrize("k,ifs", [(K3, IF3), (K2, (0.0,))])
def test_against_the_oracle(gpu_lib, k, ifs):
    """Three layers: targets down to 0.9 below the top interface (the lower
    interface is at depth 0.5), so both layer formulas are used."""
    src, tgt, q = sets(202, ifs, 60, 30, 0.9)
    u = run(gpu_lib, k, ifs, src, q[0], tgt, 1e-12)
    ref = oracle.cross_layer_apply(oracle.Media(k, ifs), src, q[0], tgt)
    e = rel(u, ref)
    print("%d layers vs oracle: %.2e" % (len(k), e))
    assert e < 1e-10


def test_several_right_hand_sides(gpu_lib):
    src, tgt, q = sets(203, IF3, 700, 500, 0.9)
    u = run(gpu_lib, K3, IF3, src, q, tgt, 1e-10)
    cols = np.stack([run(gpu_lib, K3, IF3, src, q[r], tgt, 1e-10) for r in range(5)])
    assert u.shape == (5, 500)
    assert rel(u, cols) < 1e-14


def test_domain_and_medium_errors(gpu_lib):
    src, tgt, q = sets(204, IF3, 20, 10, 0.9)
    bad_src = src.copy()
    bad_src[3, 1] = IF3[0] - 0.01
    with pytest.raises(gpu_lib.HFMMError) as ei:
        run(gpu_lib, K3, IF3, bad_src, q[0], tgt, 1e-8)
    assert ei.value.status == 2  # HFMM_ERR_DOMAIN
    bad_tgt = tgt.copy()
    bad_tgt[0, 1] = IF3[0]
    with pytest.raises(gpu_lib.HFMMError) as ei:
        run(gpu_lib, K3, IF3, src, q[0], bad_tgt, 1e-8)
    assert ei.value.status == 2  # HFMM_ERR_DOMAIN
    with pytest.raises(gpu_lib.HFMMError) as ei:
        run(gpu_lib, (10.0,), (0.0,), src - [0, 0.5], q[0], tgt - [0, 0.5], 1e-8)
    assert ei.value.status == 3  # HFMM_ERR_UNSUPPORTED


@pytest.mark.parametrize("k,ifs", [(K3, IF3), (K2, (0.0,))])
def test_reverse_pairs_against_the_oracle(gpu_lib, k, ifs):
    """Sources below the interface, targets in the top layer
    (hfmm_transmit_up) against the oracle's transmitted fields read by
    reciprocity, G(x_t, x_s) = G(x_s, x_t) (pinned between two independent
    oracle paths in tests/test_oracle.py)."""
    top, below, q = sets(205, ifs, 16, 40, 0.9)
    rng = workloads.rng_for(1703, 9136, 206)
    qb = workloads.complex_normal(rng, (1, below.shape[0]))[0]
    u = run_up(gpu_lib, k, ifs, below, qb, top, 1e-12)
    # M[j, i] = G(below_i; top_j): the oracle's field of each top point at the points below
    M = oracle.cross_layer_apply(oracle.Media(k, ifs), top, np.eye(top.shape[0]), below)
    ref = M @ qb
    e = rel(u, ref)
    print("%d layers, reverse pairs vs oracle: %.2e" % (len(k), e))
    assert e < 1e-10


def test_reverse_pairs_domain_errors(gpu_lib):
    top, below, q = sets(207, IF3, 10, 20, 0.9)
    with pytest.raises(gpu_lib.HFMMError) as ei:
        run_up(gpu_lib, K3, IF3, top, q[0][:10], top, 1e-8)  # sources above the interface
    assert ei.value.status == 2  # HFMM_ERR_DOMAIN


def run_up(hf, k, ifs, src, q, tgt, tol):
    import torch
    dev = torch.device("cuda:0")
    return hf.transmit(k, ifs, torch.tensor(src, device=dev), torch.tensor(q, device=dev),
                       torch.tensor(tgt, device=dev), tol=tol, up=True).cpu().numpy()


def test_middle_to_bottom_pairs_by_the_mirrored_medium(gpu_lib):
    """Sources in the middle layer, targets in the bottom layer: mirrored in y
    (y -> -y) the medium is (k3, k2, k1) with the old lower interface on top,
    the targets lie in its top layer and the sources below it, so
    hfmm_transmit_up of the mirrored medium gives them; against the oracle's
    middle-layer source seen in the bottom layer (oracle.middle)."""
    from oracle.middle import middle_source_field
    rng = workloads.rng_for(1703, 9136, 208)
    src = np.c_[rng.uniform(0.0, 1.0, 12), rng.uniform(0.03, 0.47, 12)]     # middle layer
    tgt = np.c_[rng.uniform(0.0, 1.0, 9), -rng.uniform(0.02, 0.4, 9)]       # bottom layer
    q = workloads.complex_normal(rng, (1, 12))[0]
    flip = np.array([1.0, -1.0])
    u = run_up(gpu_lib, (K3[2], K3[1], K3[0]), (-IF3[1], -IF3[0]), src * flip, q, tgt * flip, 1e-12)
    m = oracle.Media(K3, IF3)
    ref = np.zeros(tgt.shape[0], complex)
    for j in range(src.shape[0]):
        ref += q[j] * middle_source_field(m, 3, tgt[:, 0], tgt[:, 1] - IF3[0], src[j, 0], src[j, 1] - IF3[0])
    e = rel(u, ref)
    print("middle -> bottom by the mirrored medium vs oracle: %.2e" % e)
    assert e < 1e-10


def test_bottom_to_middle_pairs_by_the_mirrored_medium(gpu_lib):
    """Sources in the bottom layer, targets in the middle layer: mirrored in y
    the sources lie in the top layer of (k3, k2, k1) and the targets below
    its interface, so hfmm_transmit of the mirrored medium gives them. The
    oracle's value by the symmetry of the Green's function: the field at each
    bottom-layer source of a unit source at the middle-layer target
    (oracle.middle, the middle-layer source seen in the bottom layer)."""
    from oracle.middle import middle_source_field
    rng = workloads.rng_for(1703, 9136, 209)
    src = np.c_[rng.uniform(0.0, 1.0, 11), -rng.uniform(0.02, 0.4, 11)]     # bottom layer
    tgt = np.c_[rng.uniform(0.0, 1.0, 8), rng.uniform(0.03, 0.47, 8)]       # middle layer
    q = workloads.complex_normal(rng, (1, 11))[0]
    flip = np.array([1.0, -1.0])
    u = run(gpu_lib, (K3[2], K3[1], K3[0]), (-IF3[1], -IF3[0]), src * flip, q, tgt * flip, 1e-12)
    m = oracle.Media(K3, IF3)
    ref = np.array([np.dot(q, middle_source_field(m, 3, src[:, 0], src[:, 1] - IF3[0], t[0], t[1] - IF3[0]))
                    for t in tgt])
    e = rel(u, ref)
    print("bottom -> middle by the mirrored medium vs oracle: %.2e" % e)
    assert e < 1e-10
