"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a library
special function (scipy / mpmath Hankel functions), a closed form, a physical
invariant (interface continuity, the Helmholtz equation, reciprocity), a
degenerate medium, a limit (vanishing absorption) or brute force at 30 digits.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.special import hankel1

import oracle
from oracle import Media
from oracle.media import gamma, sigma_coefficients, sigma1

K3 = (2 * math.pi * 8, 2 * math.pi * 12, 2 * math.pi * 10)   # scaled-down config-3 medium
IF3 = (0.5, 0.0)
K2 = (8 * math.pi, 12 * math.pi)


def rng(seed):
    return np.random.default_rng(seed)


def path_points(r, n, kmax):
    """Random lambda on and below the real axis, as seen on the contour."""
    return r.uniform(0, 2 * kmax, n) - 1j * r.uniform(0, 2.0, n)


# ---------------------------------------------------------------- branches

def test_gamma_branch_outgoing_and_decaying():
    k = 7.0
    lam = np.array([0.0, 3.0, 6.999, 7.001, 20.0])
    g = gamma(lam, k)
    assert np.allclose(g[:3], -1j * np.sqrt(k * k - lam[:3] ** 2), rtol=0, atol=1e-12)
    assert np.allclose(g[3:], np.sqrt(lam[3:] ** 2 - k * k), rtol=0, atol=1e-12)
    lamc = path_points(rng(0), 200, k)
    gc = gamma(lamc, k)
    assert np.all(gc.real >= -1e-15)
    assert np.allclose(gc * gc, lamc * lamc - k * k, rtol=1e-13, atol=1e-10)


# ---------------------------------------------------------------- sigma

def fresnel(ga, gb):
    return (ga - gb) / (ga + gb)


def test_sigma_three_layer_matches_slab_closed_form():
    """The interface system against the slab reflection formula (derived by hand)."""
    m = Media(K3, IF3)
    lam = path_points(rng(1), 300, max(K3))
    g1, g2, g3 = (gamma(lam, k) for k in K3)
    e = np.exp(-2 * g2 * 0.5)
    r12, r23 = fresnel(g1, g2), fresnel(g2, g3)
    closed = (r12 + r23 * e) / (1 + r12 * r23 * e)
    assert np.max(np.abs(sigma1(lam, m) - closed)) < 1e-13


def test_sigma_two_layer_is_fresnel_and_independent_of_d():
    m = Media(K2, (0.0,))
    lam = path_points(rng(2), 300, max(K2))
    s = sigma1(lam, m)
    assert np.max(np.abs(s - fresnel(gamma(lam, K2[0]), gamma(lam, K2[1])))) < 1e-13
    # the same medium written as three layers with k3 = k2 at two depths
    for d in (0.3, 2.0):
        m3 = Media((K2[0], K2[1], K2[1]), (0.0, -d))
        assert np.max(np.abs(sigma1(lam, m3) - s)) < 1e-13


def test_sigma_degenerate_media():
    lam = path_points(rng(3), 200, max(K3))
    g = {k: gamma(lam, k) for k in K3}
    # a vanishing slab: the top layer sees the bottom medium directly
    thin = Media(K3, (0.0, -1e-12))
    assert np.max(np.abs(sigma1(lam, thin) - fresnel(g[K3[0]], g[K3[2]]))) < 1e-9
    # slab with the top wavenumber: the reflection of a shifted interface
    shifted = Media((K3[0], K3[0], K3[2]), (0.0, -0.5))
    ref = fresnel(g[K3[0]], g[K3[2]]) * np.exp(-2 * g[K3[0]] * 0.5)
    assert np.max(np.abs(sigma1(lam, shifted) - ref)) < 1e-13
    # one homogeneous medium: nothing is reflected
    same = Media((K3[0],) * 3, IF3)
    assert np.max(np.abs(sigma1(lam, same))) < 1e-14


def test_sigma_even_in_lambda():
    m = Media(K3, IF3)
    lam = path_points(rng(4), 100, max(K3))
    assert np.max(np.abs(sigma1(lam, m) - sigma1(-lam, m))) < 1e-13


# ---------------------------------------------------------------- Sommerfeld machinery

@pytest.mark.parametrize("k,ifs", [(K2, (0.0,)), (K3, IF3),
                                   ((2 * math.pi * 80, 2 * math.pi * 120, 2 * math.pi * 100), IF3)])
def test_reflection_one_is_mirror_image_hankel(k, ifs):
    """sigma = +-1 turns the Sommerfeld integral into (i/4) H0(k |x - x_image|)."""
    m = Media(k, ifs)
    r = rng(5)
    X = r.uniform(-1.2, 1.2, 12)
    Y = r.uniform(0.02, 2.0, 12)
    ref = 0.25j * hankel1(0, m.k1 * np.hypot(X, Y))
    for sgn in (1.0, -1.0):
        g = oracle.scattered_pairs(m, X, Y, sigma=sgn)
        assert np.max(np.abs(g - sgn * ref) / np.abs(ref)) < 1e-12


@pytest.mark.parametrize("n", [-6, -3, -1, 0, 1, 2, 5, 8])
def test_order_n_entry_with_reflection_one_is_hankel_n(n):
    """The order-n spectral form (higher-order Sommerfeld) reproduces H_n e^{in theta}."""
    m = Media(K3, IF3)
    for X, Y in ((0.3, 0.5), (-0.4, 0.6), (0.0, 0.3), (0.9, 1.1)):
        a = oracle.m2l_entry(n, X, Y, m, sigma=1.0)
        ref = hankel1(n, m.k1 * math.hypot(X, Y)) * np.exp(1j * n * math.atan2(Y, X))
        assert abs(a - ref) / abs(ref) < 1e-11, (n, X, Y)


def test_global_rule_equals_pairwise_rules():
    """The reordered one-rule matvec agrees with pair-by-pair integration."""
    m = Media(K3, IF3)
    r = rng(6)
    xs = r.uniform(0, 1, 9)
    ys = r.uniform(0.03, 0.8, 9)
    xt = r.uniform(0, 1, 7)
    yt = r.uniform(0.03, 0.8, 7)
    q = r.standard_normal(9) + 1j * r.standard_normal(9)
    u = oracle.scattered_matvec(m, xt, yt, xs, ys, q, workers=1)
    X = xt[:, None] - xs[None, :]
    Y = yt[:, None] + ys[None, :]
    g = oracle.scattered_pairs(m, X.ravel(), Y.ravel()).reshape(X.shape)
    ref = g @ q
    assert np.max(np.abs(u - ref)) / np.max(np.abs(ref)) < 1e-12


def test_result_independent_of_contour_depth_and_resolution():
    m = Media((2 * math.pi * 80, 2 * math.pi * 120, 2 * math.pi * 100), IF3)
    r = rng(7)
    X = r.uniform(-1, 1, 6)
    Y = r.uniform(0.02, 1.0, 6)
    base = oracle.scattered_pairs(m, X, Y)
    fine = oracle.scattered_pairs(m, X, Y, refine=2.0)
    assert np.max(np.abs(base - fine) / np.abs(base)) < 1e-12
    for x, y, b in zip(X, Y, base):
        lam, w = oracle.contour_rule(m, abs(x), y, y, delta=0.5 * min(1.0 / max(abs(x), 1e-9), 50.0))
        g1 = gamma(lam, m.k1)
        v = np.sum(w * np.exp(-g1 * y) / g1 * np.cos(lam * x) * sigma1(lam, m)) / (2 * math.pi)
        assert abs(v - b) / abs(b) < 5e-11


def _lossy(media_k, eps):
    return tuple(k * (1 + 1j * eps) for k in media_k)


def _real_axis_value(k, ifs, X, Y):
    m = Media(k, ifs)
    lam, w = oracle.contour_rule(m, abs(X), Y, Y, delta=0.0)
    g1 = gamma(lam, m.k1)
    return np.sum(w * np.exp(-g1 * Y) / g1 * np.cos(lam * X) * sigma1(lam, m)) / (2 * math.pi)


def test_limiting_absorption_side():
    """Lossless values are the limit of slightly lossy media integrated on the real axis.

    The slab medium has guided-mode poles on the real axis; the contour passing
    below them (Re lambda > 0) must agree with the vanishing-loss limit, while a
    contour passing above them must not.
    """
    m = Media(K3, IF3)
    for X, Y in ((0.2, 0.08), (-0.5, 0.15)):
        lossless = oracle.scattered_pairs(m, X, Y)[0]
        v1, v2, v3 = (_real_axis_value(_lossy(K3, e), IF3, X, Y) for e in (1e-3, 5e-4, 2.5e-4))
        limit = (8 * v3 - 6 * v2 + v1) / 3   # Richardson: the error is O(eps^3)
        assert abs(limit - lossless) / abs(lossless) < 2e-5
        lam, w = oracle.contour_rule(m, abs(X), Y, Y, delta=-1.0)
        g1 = gamma(lam, m.k1)
        wrong = np.sum(w * np.exp(-g1 * Y) / g1 * np.cos(lam * X) * sigma1(lam, m)) / (2 * math.pi)
        assert abs(wrong - lossless) / abs(lossless) > 1e-2


# ---------------------------------------------------------------- physics

@pytest.mark.parametrize("k,ifs", [(K2, (0.0,)), (K3, IF3)])
def test_interface_conditions(k, ifs):
    """u and du/dy are continuous across every interface (one-sided FD)."""
    m = Media(k, ifs)
    x0, y0 = 0.1, 0.3
    interfaces = [0.0] + ([-m.d] if m.layers == 3 else [])
    layer_pairs = [(1, 2)] + ([(2, 3)] if m.layers == 3 else [])
    for yi, (la, lb) in zip(interfaces, layer_pairs):
        for x in (0.1, 0.45, -0.3):
            ua = oracle.layer_field(m, la, x, yi, x0, y0)[0]
            ub = oracle.layer_field(m, lb, x, yi, x0, y0)[0]
            scale = abs(ua)
            assert abs(ua - ub) < 1e-11 * max(scale, 1e-3)

            def deriv(layer, sign, h):
                f0 = oracle.layer_field(m, layer, x, yi, x0, y0)[0]
                f1 = oracle.layer_field(m, layer, x, yi + sign * h, x0, y0)[0]
                f2 = oracle.layer_field(m, layer, x, yi + 2 * sign * h, x0, y0)[0]
                return sign * (-3 * f0 + 4 * f1 - f2) / (2 * h)

            h = 2e-3 / m.k1
            da = (4 * deriv(la, +1, h / 2) - deriv(la, +1, h)) / 3
            db = (4 * deriv(lb, -1, h / 2) - deriv(lb, -1, h)) / 3
            assert abs(da - db) < 1e-6 * m.k1 * max(scale, 1e-3), (x, yi, da, db)


def test_scattered_field_solves_helmholtz():
    m = Media(K3, IF3)
    k = m.k1
    h = 0.02 / k
    for X, Y in ((0.1, 0.4), (-0.3, 0.25)):
        offs = [(-2, 0), (-1, 0), (0, 0), (1, 0), (2, 0), (0, -2), (0, -1), (0, 1), (0, 2)]
        vals = {o: oracle.scattered_pairs(m, X + o[0] * h, Y + o[1] * h)[0] for o in offs}
        c = [-1 / 12, 4 / 3, -5 / 2, 4 / 3, -1 / 12]
        lap = sum(ci * vals[(i - 2, 0)] for i, ci in enumerate(c)) / h ** 2
        lap += sum(ci * vals[(0, i - 2)] for i, ci in enumerate(c)) / h ** 2
        resid = lap + k * k * vals[(0, 0)]
        assert abs(resid) < 1e-6 * k * k * abs(vals[(0, 0)])


def test_reciprocity_and_free_exclusion():
    m = Media(K3, IF3)
    r = rng(8)
    xy = np.stack([r.uniform(0, 1, 12), r.uniform(0.55, 1.2, 12)], axis=1)
    a = oracle.dense_matrix(m, xy)
    assert np.max(np.abs(a - a.T)) < 1e-13 * np.max(np.abs(a))
    # the diagonal holds only the scattered self term
    yf = m.to_frame(xy[:, 1])
    gs = oracle.scattered_pairs(m, np.zeros(12), 2 * yf)
    assert np.max(np.abs(np.diag(a) - gs)) < 1e-13 * np.max(np.abs(gs))
    # off the diagonal: free part + scattered part
    i, j = 3, 7
    free = 0.25j * hankel1(0, m.k1 * math.hypot(*(xy[i] - xy[j])))
    sc = oracle.scattered_pairs(m, xy[i, 0] - xy[j, 0], yf[i] + yf[j])[0]
    assert abs(a[i, j] - free - sc) < 1e-13 * abs(a[i, j])


def test_homogeneous_medium_is_free_space():
    m = Media((K3[0],) * 3, IF3)
    r = rng(9)
    xy = np.stack([r.uniform(0, 1, 10), r.uniform(0.6, 1.2, 10)], axis=1)
    q = r.standard_normal(10) + 1j * r.standard_normal(10)
    u = oracle.direct_apply(m, xy, q)
    d = np.hypot(xy[:, None, 0] - xy[None, :, 0], xy[:, None, 1] - xy[None, :, 1])
    np.fill_diagonal(d, 1.0)
    h = 0.25j * hankel1(0, m.k1 * d)
    np.fill_diagonal(h, 0.0)
    assert np.max(np.abs(u - h @ q)) < 1e-13 * np.max(np.abs(u))


# ---------------------------------------------------------------- brute force

def _mp_scattered(k, ifs, X, Y):
    """G^s by mpmath quadrature at 30 digits on a polygonal contour.

    sigma_1 comes from the interface system solved in mpmath; the contour runs
    0 -> c1 - i*dip -> c2 - i*dip -> L -> infinity, folded with cos(lambda X).
    """
    mpmath.mp.dps = 30
    k1, k2, k3 = (mpmath.mpf(v) for v in k)
    d = mpmath.mpf(ifs[0] - ifs[1])

    def gam(lam, kk):
        w = lam * lam - kk * kk
        return mpmath.sqrt(w)  # the contour keeps Im(w) < 0 off the axis

    def sig(lam):
        g1, g2, g3 = gam(lam, k1), gam(lam, k2), gam(lam, k3)
        e = mpmath.exp(-g2 * d)
        a = mpmath.matrix([[1 / g1, -1 / g2, -e / g2, 0], [0, e / g2, 1 / g2, -1 / g3],
                           [1, 1, -e, 0], [0, e, -1, -1]])
        b = mpmath.matrix([-1 / g1, 0, 1, 0])
        return mpmath.lu_solve(a, b)[0]

    def f(lam):
        g1 = gam(lam, k1)
        return mpmath.exp(-g1 * Y) / g1 * mpmath.cos(lam * X) * sig(lam)

    dip = mpmath.mpf("0.7")
    c1, c2 = k1 * mpmath.mpf("0.5"), max(k1, k2, k3) * mpmath.mpf("1.3")
    pts = [mpmath.mpf(0), mpmath.mpc(c1, -dip), mpmath.mpc(c2, -dip), c2 + 1]
    total = mpmath.mpc(0)
    for a, b in zip(pts[:-1], pts[1:]):
        total += mpmath.quad(f, [a, b])
    total += mpmath.quad(f, [c2 + 1, c2 + 1 + 60 / Y, mpmath.inf])
    return complex(total / (2 * mpmath.pi))


@pytest.mark.slow
def test_bruteforce_mpmath_tiny():
    k = (2 * math.pi * 2, 2 * math.pi * 3, 2 * math.pi * 2.5)
    ifs = (0.5, 0.0)
    m = Media(k, ifs)
    xy = np.array([[0.1, 0.8], [0.35, 0.62], [0.2, 1.1]])
    a = oracle.dense_matrix(m, xy)
    yf = xy[:, 1] - 0.5
    for i in range(3):
        for j in range(i, 3):
            ref = _mp_scattered(k, ifs, xy[i, 0] - xy[j, 0], yf[i] + yf[j])
            if i != j:
                r = math.hypot(*(xy[i] - xy[j]))
                ref += complex(0.25j * mpmath.hankel1(0, k[0] * r))
            assert abs(a[i, j] - ref) < 1e-12 * abs(ref), (i, j)


# ---------------------------------------------------------------- planted mistakes

def test_planted_mistake_in_sigma_breaks_continuity():
    """A wrong sigma (the slab term dropped) must fail the interface check."""
    m = Media(K3, IF3)
    x, x0, y0 = 0.2, 0.1, 0.3
    true_u1 = oracle.layer_field(m, 1, x, 0.0, x0, y0)[0]
    wrong_sigma = lambda lam: fresnel(gamma(lam, K3[0]), gamma(lam, K3[1]))  # noqa: E731
    free = 0.25j * hankel1(0, m.k1 * math.hypot(x - x0, y0))
    wrong_u1 = free + oracle.scattered_pairs(m, x - x0, y0, sigma=wrong_sigma)[0]
    u2 = oracle.layer_field(m, 2, x, 0.0, x0, y0)[0]
    assert abs(true_u1 - u2) < 1e-11 * abs(u2)
    assert abs(wrong_u1 - u2) > 1e-4 * abs(u2)


# ---------------------------------------------------------------- gradient
def _loss_moved_source(media, xy, q, v, j, axis, h):
    """Re <v, A(targets fixed, source j moved by h along axis) q>."""
    xs = xy[:, 0].copy()
    ys = media.to_frame(xy[:, 1]).copy()
    xt, yt = xs.copy(), ys.copy()
    if axis == 0:
        xs[j] += h
    else:
        ys[j] += h
    u = oracle.free_matvec(media.k1, xt, yt, xs, ys, q, target_ids=np.arange(xs.size), workers=1)
    u = u + oracle.scattered_matvec(media, xt, yt, xs, ys, q, workers=1)
    return float(np.real(np.vdot(v, u)))


@pytest.mark.parametrize("k,ifs", [((8 * np.pi, 12 * np.pi), (0.0,)),
                                   ((2 * np.pi * 8, 2 * np.pi * 12, 2 * np.pi * 10), (0.5, 0.0))])
def test_source_gradient_matches_central_differences(k, ifs):
    """The analytic source gradient against central differences of the matvec
    itself (targets fixed), free and scattered parts together."""
    media = Media(k, ifs)
    rng = np.random.default_rng([1703, 9136, 71])
    n = 24
    xy = np.column_stack([rng.uniform(0, 0.6, n), ifs[0] + rng.uniform(0.02, 0.4, n)])
    q = rng.normal(size=n) + 1j * rng.normal(size=n)
    v = rng.normal(size=n) + 1j * rng.normal(size=n)
    g = oracle.source_gradient(media, xy, q, v)
    h = 1e-6
    for j, axis in [(0, 0), (3, 1), (7, 0), (11, 1), (19, 0), (23, 1)]:
        fd = (_loss_moved_source(media, xy, q, v, j, axis, h) -
              _loss_moved_source(media, xy, q, v, j, axis, -h)) / (2 * h)
        assert abs(fd - g[j, axis]) <= 2e-6 * max(1.0, abs(fd)), (j, axis, fd, g[j, axis])


def test_planted_sign_error_in_scattered_gradient_is_caught():
    """A sign error in the scattered part of the gradient must show against
    central differences."""
    from oracle import gradient as og
    media = Media((8 * np.pi, 12 * np.pi), (0.0,))
    rng = np.random.default_rng([1703, 9136, 72])
    n = 16
    xy = np.column_stack([rng.uniform(0, 0.5, n), rng.uniform(0.02, 0.3, n)])
    q = rng.normal(size=n) + 1j * rng.normal(size=n)
    v = rng.normal(size=n) + 1j * rng.normal(size=n)
    y = media.to_frame(xy[:, 1])
    bad = og.free_source_gradient(media.k1, xy[:, 0], y, q, v) - og.scattered_source_gradient(media, xy[:, 0], y, q, v)
    good = oracle.source_gradient(media, xy, q, v)
    j, h = 5, 1e-6
    fd = (_loss_moved_source(media, xy, q, v, j, 1, h) - _loss_moved_source(media, xy, q, v, j, 1, -h)) / (2 * h)
    assert abs(fd - good[j, 1]) <= 2e-6 * max(1.0, abs(fd))
    assert abs(fd - bad[j, 1]) > 1e-3 * max(1.0, abs(fd))


# ---------------------------------------------------------------- self term dropped

def test_self_term_none_is_zero_diagonal_with_same_off_diagonal():
    """direct_apply(self_term=False) applies A with A_ii = 0: the same matrix
    as the default one off the diagonal, and nothing on it."""
    m = Media(K3, IF3)
    r = rng(21)
    n = 10
    xy = np.stack([r.uniform(0, 1, n), r.uniform(0.55, 1.2, n)], axis=1)
    eye = np.eye(n, dtype=complex)
    full = oracle.direct_apply(m, xy, eye, workers=1).T
    none = oracle.direct_apply(m, xy, eye, self_term=False, workers=1).T
    scale = np.max(np.abs(full))
    off = ~np.eye(n, dtype=bool)
    assert np.max(np.abs(none[off] - full[off])) < 1e-15 * scale
    assert np.max(np.abs(np.diag(none))) < 1e-12 * np.max(np.abs(np.diag(full)))
    # and several right-hand sides at once, targets a subset
    q = r.standard_normal((3, n)) + 1j * r.standard_normal((3, n))
    tid = np.array([1, 4, 8])
    u = oracle.direct_apply(m, xy, q, targets=tid, self_term=False, workers=1)
    ref = q @ none.T
    assert np.max(np.abs(u - ref[:, tid])) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("X,Y", [(0.0, 0.3), (0.2, 0.15), (-0.4, 0.9)])
def test_height_derivative_of_scattered_pair(X, Y):
    """d/dY G^s: with sigma = 1 the closed form of the mirror-image Hankel
    function, -(i/4) k H1(k rho) Y / rho; with the layered sigma central
    differences of G^s itself."""
    m = Media(K3, IF3)
    k = m.k1
    rho = math.hypot(X, Y)
    d1 = oracle.scattered_pairs(m, X, Y, sigma=1.0, d_dY=True)[0]
    ref = -0.25j * k * hankel1(1, k * rho) * Y / rho
    assert abs(d1 - ref) < 1e-11 * abs(ref)
    h = 1e-5
    d = oracle.scattered_pairs(m, X, Y, d_dY=True)[0]
    fd = (oracle.scattered_pairs(m, X, Y + h)[0] - oracle.scattered_pairs(m, X, Y - h)[0]) / (2 * h)
    assert abs(d - fd) < 1e-6 * abs(d)


def _loss_moved_source_no_self(media, xy, q, v, j, axis, h):
    """_loss_moved_source for A with A_jj = 0: the pair (target j, moved
    source j) removed from the sum."""
    full = _loss_moved_source(media, xy, q, v, j, axis, h)
    yf = media.to_frame(xy[:, 1])
    X = -h if axis == 0 else 0.0
    Y = 2 * yf[j] + (h if axis == 1 else 0.0)
    gs = oracle.scattered_pairs(media, X, Y)[0]
    return full - float(np.real(np.conj(v[j]) * gs * q[j]))


def test_source_gradient_without_self_term_matches_central_differences():
    media = Media(K2, (0.0,))
    rng_ = np.random.default_rng([1703, 9136, 73])
    n = 14
    xy = np.column_stack([rng_.uniform(0, 0.5, n), rng_.uniform(0.02, 0.3, n)])
    q = rng_.normal(size=n) + 1j * rng_.normal(size=n)
    v = rng_.normal(size=n) + 1j * rng_.normal(size=n)
    g_none = oracle.source_gradient(media, xy, q, v, self_term=False)
    g_full = oracle.source_gradient(media, xy, q, v)
    h = 1e-6
    for j, axis in [(2, 1), (5, 0), (9, 1), (13, 1)]:
        fd = (_loss_moved_source_no_self(media, xy, q, v, j, axis, h) -
              _loss_moved_source_no_self(media, xy, q, v, j, axis, -h)) / (2 * h)
        assert abs(fd - g_none[j, axis]) <= 2e-6 * max(1.0, abs(fd)), (j, axis, fd, g_none[j, axis])
        if axis == 1:  # the self pair matters in y only, and there it must
            assert abs(fd - g_full[j, axis]) > 1e-4 * max(1.0, abs(fd))


# ---------------------------------------------------------------- fields below the top interface
@pytest.mark.parametrize("ks,ifs", [((31.0, 31.0, 31.0), (0.5, 0.0)), ((31.0, 31.0), (0.0,))])
def test_cross_layer_homogeneous_is_the_free_field(ks, ifs):
    """One wavenumber everywhere: the field below the interface of a top-layer
    source is (i/4) H0(k r) (scipy's Hankel function)."""
    m = Media(ks, ifs)
    rng = np.random.default_rng(5)
    src = np.c_[rng.uniform(0, 1, 4), ifs[0] + rng.uniform(0.02, 0.3, 4)]
    tgt = np.c_[rng.uniform(0, 1, 5), ifs[0] - rng.uniform(0.02, 0.9, 5)]
    q = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    u = oracle.cross_layer_apply(m, src, q, tgt)
    r = np.hypot(tgt[:, None, 0] - src[None, :, 0], tgt[:, None, 1] - src[None, :, 1])
    ref = (0.25j * hankel1(0, ks[0] * r)) @ q
    assert np.max(np.abs(u - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("k,ifs", [(K2, (0.0,)), (K3, IF3)])
def test_cross_layer_meets_the_top_layer_field(k, ifs):
    """Just below the top interface the cross-layer sum equals the top-layer
    field just above it: the free part (i/4) H0(k1 r) plus the scattered part
    of Eq. multitop (sigma_1), a path that shares no density with the
    transmitted one (sigma_2^+). Across the lower interface the layer switch
    is continuous."""
    m = Media(k, ifs)
    x0, y0 = 0.15, ifs[0] + 0.2
    q = np.array([1.0 + 0.5j])
    for x in (0.1, 0.6):
        below = oracle.cross_layer_apply(m, [[x0, y0]], q, [[x, ifs[0] - 1e-13]])[0]
        r = math.hypot(x - x0, y0 - ifs[0])
        above = q[0] * (0.25j * hankel1(0, m.k1 * r) + oracle.scattered_pairs(m, x - x0, y0 - ifs[0])[0])
        assert abs(below - above) < 1e-10 * abs(above), (x, below, above)
        if m.layers == 3:
            lo = ifs[1]
            a = oracle.cross_layer_apply(m, [[x0, y0]], q, [[x, lo + 1e-13]])[0]
            b = oracle.cross_layer_apply(m, [[x0, y0]], q, [[x, lo - 1e-13]])[0]
            assert abs(a - b) < 1e-10 * abs(a)


def test_cross_layer_rejects_points_on_the_wrong_side():
    m = Media(K3, IF3)
    with pytest.raises(ValueError):
        oracle.cross_layer_apply(m, [[0.1, 0.4]], [1.0], [[0.2, 0.3]])
    with pytest.raises(ValueError):
        oracle.cross_layer_apply(m, [[0.1, 0.6]], [1.0], [[0.2, 0.7]])


# ---------------------------------------------------------------- sources in the middle layer
from oracle.middle import middle_apply, middle_coefficients, middle_source_field  # noqa: E402

KM = (2 * math.pi * 8, 2 * math.pi * 12, 2 * math.pi * 10)   # slab fastest: guided modes


def test_middle_homogeneous_has_no_scattered_field():
    m = Media((40.0, 40.0, 40.0), IF3)
    c = middle_coefficients(np.array([1.0, 30.0 - 2j, 60.0]), m, -0.2)
    assert np.max(np.abs(c[..., 1:3])) < 1e-14
    x0, y0 = 0.1, -0.2
    for layer, y in ((1, 0.15), (3, -0.8)):
        u = middle_source_field(m, layer, 0.4, y, x0, y0)[0]
        ref = 0.25j * hankel1(0, 40.0 * math.hypot(0.4 - x0, y - y0))
        assert abs(u - ref) < 1e-12 * abs(ref)


@pytest.mark.parametrize("kk,which", [((KM[0], KM[1], KM[1]), "top"), ((KM[1], KM[1], KM[2]), "bottom")])
def test_middle_matched_interface_reduces_to_one_reflection(kk, which):
    """A matched interface reflects nothing: the middle layer's scattered field
    is the one-interface reflection of the other, which is the top-layer
    oracle's two-layer field after a mirror (x, y) -> (x, -y) (about the
    reflecting interface)."""
    m = Media(kk, IF3)
    d = m.d
    for X, y, y0 in ((0.3, -0.1, -0.25), (-0.05, -0.4, -0.1)):
        g = middle_source_field(m, 2, X, y, 0.0, y0, scattered_only=True)[0]
        if which == "top":
            ref = oracle.scattered_pairs(Media((kk[1], kk[0]), (0.0,)), X, -(y + y0))[0]
        else:
            ref = oracle.scattered_pairs(Media((kk[1], kk[2]), (0.0,)), X, (y + d) + (y0 + d))[0]
        assert abs(g - ref) < 1e-11 * abs(ref), (which, X, y, y0, g, ref)


def test_middle_reciprocity():
    m = Media(KM, IF3)
    a = middle_source_field(m, 2, 0.35, -0.1, 0.05, -0.3, scattered_only=True)[0]
    b = middle_source_field(m, 2, 0.05, -0.3, 0.35, -0.1, scattered_only=True)[0]
    assert abs(a - b) < 1e-11 * abs(a)


def test_middle_interface_conditions():
    """u and du/dy continuous across both interfaces for a middle-layer source
    (one-sided differences, as for the top-layer source)."""
    m = Media(KM, IF3)
    x0, y0 = 0.1, -0.22
    for yi, (la, lb) in ((0.0, (1, 2)), (-m.d, (2, 3))):
        for x in (0.15, 0.5):
            ua = middle_source_field(m, la, x, yi, x0, y0)[0]
            ub = middle_source_field(m, lb, x, yi, x0, y0)[0]
            assert abs(ua - ub) < 1e-10 * abs(ua), (yi, x, ua, ub)

            def deriv(layer, sign, h):
                f0 = middle_source_field(m, layer, x, yi, x0, y0)[0]
                f1 = middle_source_field(m, layer, x, yi + sign * h, x0, y0)[0]
                f2 = middle_source_field(m, layer, x, yi + 2 * sign * h, x0, y0)[0]
                return sign * (-3 * f0 + 4 * f1 - f2) / (2 * h)

            h = 2e-3 / KM[1]
            da = (4 * deriv(la, +1, h / 2) - deriv(la, +1, h)) / 3
            db = (4 * deriv(lb, -1, h / 2) - deriv(lb, -1, h)) / 3
            assert abs(da - db) < 1e-6 * KM[1] * abs(ua), (yi, x, da, db)


def test_middle_apply_is_the_pairwise_sum():
    m = Media(KM, IF3)
    rng = np.random.default_rng(9)
    xy = np.c_[rng.uniform(0, 1, 5), IF3[0] - rng.uniform(0.05, 0.45, 5)]
    q = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    u = middle_apply(m, xy, q)
    y = xy[:, 1] - IF3[0]
    for i in (0, 3):
        ref = 0.0
        for j in range(5):
            g = middle_source_field(m, 2, xy[i, 0], y[i], xy[j, 0], y[j], scattered_only=True)[0]
            if j != i:
                g += 0.25j * hankel1(0, KM[1] * math.hypot(xy[i, 0] - xy[j, 0], y[i] - y[j]))
            ref += q[j] * g
        assert abs(u[i] - ref) < 1e-13 * abs(ref)


def test_cross_layer_reciprocity_between_independent_paths():
    """G(x, x0) = G(x0, x) across the top interface, the two values coming
    from different interface systems: a middle-layer source seen in the top
    layer (``middle``) and a top-layer source seen in the middle layer
    (``layer_field``)."""
    m = Media(KM, IF3)
    for (xt, yt), (xm, ym) in (((0.3, 0.12), (0.05, -0.2)), ((-0.1, 0.05), (0.4, -0.41))):
        a = middle_source_field(m, 1, xt, yt, xm, ym)[0]
        b = oracle.layer_field(m, 2, xm, ym, xt, yt)[0]
        assert abs(a - b) < 1e-10 * abs(a), (a, b)


def test_middle_to_bottom_equals_the_mirrored_medium():
    """A middle-layer source seen in the bottom layer (``middle``) equals, after
    the mirror y -> -y and the symmetry of G, a top-layer source of the
    mirrored medium (k3, k2, k1) seen in its middle layer (``layer_field``)."""
    m = Media(KM, IF3)
    mf = Media((KM[2], KM[1], KM[0]), (-IF3[1], -IF3[0]))
    for (xs, ys), (xt, yt) in (((0.1, 0.3), (0.4, -0.2)), ((0.7, 0.06), (0.2, -0.05))):
        a = middle_source_field(m, 3, xt, yt - IF3[0], xs, ys - IF3[0])[0]
        b = oracle.layer_field(mf, 2, xs, -ys - mf.y_top, xt, -yt - mf.y_top)[0]
        assert abs(a - b) < 1e-10 * abs(a), (a, b)
