"""Pins of the oracle's impedance half-space (Section 2.2): the scattered
field from the Sommerfeld integral with sigma-hat = (gamma + i alpha)/(gamma -
i alpha) (Eq. multisommer) against

* the complex line-image representation of the same field (Eq. Sfield: a
  point image plus the line image 2 i alpha e^{i alpha s} below it), evaluated
  independently with scipy's Hankel function on the ray s = t e^{i pi/4},
  where the line integral decays exponentially (the integrand is analytic in
  the sector between the ray and the positive axis and decays on the arc);
* the limits alpha -> 0 (Neumann: + the mirror image) and alpha -> infinity
  (Dirichlet: - the mirror image);
* the boundary condition du/dn - i alpha u = 0 at y = 0 (n = -y), with the
  exact y-derivatives of both parts;
and a planted sign error in sigma-hat, which these pins must catch.
"""
import numpy as np
import pytest
from scipy.special import hankel1

import oracle
import oracle.media as media_mod

_GX, _GW = np.polynomial.legendre.leggauss(24)


def line_image_gs(k, alpha, X, Y, phi=np.pi / 4):
    """(i/4) [H0(k |x - x0_im|) + int_0^inf H0(k |x - (x0_im - s y)|) 2 i alpha e^{i alpha s} ds]."""
    e = np.exp(1j * phi)
    decay = (alpha + k) * np.sin(phi)
    t_end = 80.0 / decay
    width = min(0.5 / (alpha + k), 0.25 * np.hypot(X, Y), t_end)
    edges = np.linspace(0.0, t_end, int(np.ceil(t_end / width)) + 1)
    a, b = edges[:-1, None], edges[1:, None]
    t = (0.5 * (b - a) * _GX + 0.5 * (a + b)).ravel()
    w = (0.5 * (b - a) * _GW).ravel()
    s = t * e
    R = np.sqrt(X * X + (Y + s) ** 2)
    f = hankel1(0, k * R) * 2j * alpha * np.exp(1j * alpha * s) * e
    return 0.25j * (hankel1(0, k * np.hypot(X, Y)) + np.sum(w * f))


CASES = [(0.1, 1.0), (1.0, 1.0), (8 * np.pi, 3.0), (5.0, 0.2)]
POINTS = [(0.0, 0.5), (0.3, 1.2), (-1.7, 0.4), (2.5, 3.0)]


@pytest.mark.parametrize("k,alpha", CASES)
def test_sommerfeld_matches_line_images(k, alpha):
    m = oracle.Media((k,), (0.0,), impedance=alpha)
    for X, Y in POINTS:
        ref = line_image_gs(k, alpha, X, Y)
        got = oracle.scattered_pairs(m, [X], [Y])[0]
        e = abs(got - ref) / abs(ref)
        print("k %.3g alpha %.3g X %.2f Y %.2f: %.2e" % (k, alpha, X, Y, e))
        assert e < 1e-10


@pytest.mark.parametrize("alpha,sign", [(1e-9, 1.0), (1e9, -1.0)])
def test_neumann_and_dirichlet_limits(alpha, sign):
    k = 3.0
    m = oracle.Media((k,), (0.0,), impedance=alpha)
    for X, Y in POINTS:
        ref = sign * 0.25j * hankel1(0, k * np.hypot(X, Y))
        got = oracle.scattered_pairs(m, [X], [Y])[0]
        assert abs(got - ref) / abs(ref) < 1e-7


@pytest.mark.parametrize("k,alpha", CASES)
def test_impedance_boundary_condition(k, alpha):
    """du/dy + i alpha u = 0 at y = 0 for u = g(., x0) + G^s(., x0)."""
    m = oracle.Media((k,), (0.0,), impedance=alpha)
    for X, y0 in [(0.2, 0.5), (-0.7, 1.1), (1.3, 0.3)]:
        r = np.hypot(X, y0)
        u = 0.25j * hankel1(0, k * r) + oracle.scattered_pairs(m, [X], [y0])[0]
        # d/dy of (i/4) H0(k r) at y = 0: -(i/4) k H1(k r) (y - y0) / r
        du = -0.25j * k * hankel1(1, k * r) * (-y0) / r + oracle.scattered_pairs(m, [X], [y0], d_dY=True)[0]
        res = abs(du + 1j * alpha * u) / (abs(du) + alpha * abs(u))
        assert res < 1e-10, res


def test_planted_sign_error_is_caught(monkeypatch):
    """sigma-hat with the sign of alpha flipped (the boundary condition of the
    opposite normal) fails the line-image pin."""
    k, alpha, (X, Y) = 1.0, 1.0, POINTS[1]
    m = oracle.Media((k,), (0.0,), impedance=alpha)
    good = oracle.scattered_pairs(m, [X], [Y])[0]

    def wrong(lam, media):
        g = media_mod.gamma(np.asarray(lam, dtype=complex), media.k1)
        return (g - 1j * media.alpha) / (g + 1j * media.alpha)

    import oracle.sommerfeld as som
    monkeypatch.setattr(som, "sigma1", wrong)
    bad = oracle.scattered_pairs(m, [X], [Y])[0]
    ref = line_image_gs(k, alpha, X, Y)
    assert abs(good - ref) / abs(ref) < 1e-10
    assert abs(bad - ref) / abs(ref) > 1e-3
