"""The boundary integral equation solve around the matvec (hfmm_bie_solve):
GMRES for the trapezoidal Nystrom single-layer system (A W + D) phi = f of a
sound-soft obstacle in the top layer, f = -u_inc at the nodes.

* Homogeneous medium (two layers of one wavenumber: sigma_1 = 0), a circle lit
  by a point source: the scattered field converges to the closed-form series
  u_sc = -(i/4) sum_n J_n(kR)/H_n(kR) H_n(k r_s) H_n(k r) e^{i n (theta -
  theta_s)} (addition theorem; kR kept away from the interior Dirichlet
  eigenvalues, the zeros of J_n), at first order in the node spacing (the
  local correction of the logarithmic self term is first order), and the
  total field inside the circle tends to zero.
* Three-layer medium (the benchmark's wavenumbers scaled down), an ellipse:
  the GPU solution equals the dense solve of the same discrete system built
  from the oracle's matrix, to the solver and plan tolerances.
"""
import math

import numpy as np
import pytest
from scipy.special import hankel1, jv

import oracle

pytestmark = pytest.mark.gpu


def ellipse_nodes(cx, cy, a, b, n):
    t = 2 * math.pi * np.arange(n) / n
    xy = np.stack([cx + a * np.cos(t), cy + b * np.sin(t)], 1)
    speed = np.hypot(a * np.sin(t), b * np.cos(t))
    return xy, speed * (2 * math.pi / n)


def diag_term(k, w):
    # the local panel correction of the solver's documentation
    l = np.log(k * w / 4.0) + np.euler_gamma - 1.0
    return 0.25j * w * (1.0 + 2j / math.pi * l)


def test_bie_circle_against_series(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    k = 8 * math.pi
    R, c = 0.18, np.array([0.5, 1.0])
    src = c + np.array([0.45, 0.1])
    rs, ths = np.hypot(*(src - c)), math.atan2(*(src - c)[::-1])
    probes = c + np.array([[0.3, 0.0], [-0.25, 0.2], [0.0, -0.35]])
    inside = c + np.array([[0.05, 0.02], [-0.03, -0.06]])

    def series(x):
        r, th = np.hypot(*(x - c)), math.atan2(*(x - c)[::-1])
        nn = np.arange(-60, 61)
        return -0.25j * np.sum(jv(nn, k * R) / hankel1(nn, k * R) * hankel1(nn, k * rs) * hankel1(nn, k * r)
                               * np.exp(1j * nn * (th - ths)))

    exact = np.array([series(x) for x in probes])
    errs = []
    for n in (256, 512, 1024):
        xy, w = ellipse_nodes(c[0], c[1], R, R, n)
        f = -0.25j * hankel1(0, k * np.hypot(*(xy - src).T))
        plan = gpu_lib.Plan((k, k), (0.0,), torch.tensor(xy, device=dev), tol=1e-12, leaf_size=32)
        phi, its, res = plan.bie_solve(torch.tensor(w, device=dev), torch.tensor(f, device=dev), tol=1e-12)
        plan.close()
        phi = phi.cpu().numpy()
        assert res <= 1e-12, res

        def field(x):
            return np.sum(0.25j * hankel1(0, k * np.hypot(*(xy - x).T)) * w * phi)

        num = np.array([field(x) for x in probes])
        e = float(np.max(np.abs(num - exact)) / np.max(np.abs(exact)))
        tot_in = max(abs(field(x) + 0.25j * hankel1(0, k * np.hypot(*(x - src)))) for x in inside)
        print("n %d: %d matvecs, residual %.1e, scattered field error %.2e, total field inside %.2e"
              % (n, its, res, e, tot_in))
        errs.append(e)
    assert errs[1] < 0.7 * errs[0] and errs[2] < 0.7 * errs[1]
    assert errs[2] < 2e-3


def test_bie_three_layer_equals_dense_solve(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    k3 = (2 * math.pi * 10, 2 * math.pi * 15, 2 * math.pi * 12.5)
    ifs = (0.5, 0.0)
    xy, w = ellipse_nodes(0.4, 0.8, 0.2, 0.12, 400)
    src = np.array([0.9, 0.7])
    media = oracle.Media(k3, ifs)
    # u_inc = the domain Green's function of a unit source: the oracle's
    # matvec of a unit strength at src, evaluated at the nodes
    allp = np.vstack([xy, src[None]])
    e = np.zeros(len(allp), complex)
    e[-1] = 1.0
    f = -oracle.direct_apply(media, allp, e, targets=np.arange(len(xy)))
    A = oracle.dense_matrix(media, xy)
    M = A * w[None, :] + np.diag(diag_term(k3[0], w))
    phi_dense = np.linalg.solve(M, f)
    plan = gpu_lib.Plan(k3, ifs, torch.tensor(xy, device=dev), tol=1e-12, leaf_size=32)
    phi, its, res = plan.bie_solve(torch.tensor(w, device=dev), torch.tensor(f, device=dev), tol=1e-12,
                                   restart=100)
    plan.close()
    d = float(np.linalg.norm(phi.cpu().numpy() - phi_dense) / np.linalg.norm(phi_dense))
    print("three-layer ellipse, 400 nodes: %d matvecs, residual %.1e, vs dense solve %.2e" % (its, res, d))
    assert res <= 1e-12
    assert d < 1e-8
