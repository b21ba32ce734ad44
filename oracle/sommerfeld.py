"""Sommerfeld integrals of the layered-media Green's function on a deformed contour.

Test infrastructure only (see the package docstring).

Paper passages followed:
* Section 2.1, Eq. spectralfree: g = (1/4pi) int e^{-gamma|y-y0|}/gamma
  e^{i lambda (x-x0)} d lambda (the normalisation used throughout).
* Section 2.3, Eq. multitop: the top-layer scattered field
  u1^s = (1/4pi) int e^{-g1 y}/g1 e^{i lambda x} e^{-g1 y0} e^{-i lambda x0}
  sigma_1(lambda) d lambda, and the middle/bottom layer fields of the same
  section (used only to check the interface conditions).
* Section 3.2, Eq. higherordersommer with sigma_1 inserted (Section 5, the
  three-layer M2L operator): the order-n entry
  A_n(X, Y) = ((-i)^n/(i pi)) int e^{-g1 Y}/g1 e^{i lambda X} z^n sigma_1 d lambda,
  z = (lambda - g1)/k1.

The integrals run over the whole real lambda axis. gamma and sigma are even in
lambda, so the line is folded onto the half contour Gamma+ from 0 to infinity:
lambda(s) = s - i h(s), with the dip h(s) = delta sin(pi s / L) on [0, L] and
h = 0 beyond. L exceeds every branch point and guided-mode pole, so the
contour passes below all real-axis singularities with Re(lambda) > 0, which is
the limiting-absorption (outgoing) choice; its mirror image -Gamma+ passes
above those with Re(lambda) < 0.

Each panel of the contour carries a 16-point Gauss-Legendre rule; the panel
width follows the local scale of the integrand: the oscillation of
e^{i lambda X}, the phase/decay rate of e^{-gamma_1 Y}, and the distance to the
nearest singularity.
"""
from __future__ import annotations

import math
import os

import numpy as np

from .media import Media, gamma, sigma1, sigma_coefficients

_GL_X, _GL_W = np.polynomial.legendre.leggauss(16)


def _singularities(media: Media):
    ks = [complex(k).real for k in media.k]
    return sorted(set(ks))


def contour_rule(media: Media, x_span: float, y_min: float, y_max: float, *,
                 refine: float = 1.0, delta: float | None = None, s_end: float | None = None,
                 extra_rate: float = 0.0):
    """Nodes and weights of a rule for int over Gamma+ of f(lambda) d lambda.

    ``x_span`` bounds |X| (the horizontal distances the rule must resolve),
    ``y_min``/``y_max`` bound the decay lengths Y > 0 of e^{-gamma_1 Y}.
    ``extra_rate`` adds a growth rate (per unit lambda) to the resolution
    requirement, used for the z^n factor of the order-n entries.
    Returns (lam, w): complex arrays; sum(w * f(lam)) approximates the integral.
    """
    if not (y_min > 0 and y_max >= y_min):
        raise ValueError("need 0 < y_min <= y_max")
    ks = _singularities(media)
    k1 = abs(complex(media.k1).real)
    kmax = max(ks)
    big_l = 1.5 * kmax + 1.0
    x_span = max(float(x_span), 1e-12)
    if delta is None:
        delta = min(1.0 / x_span, 0.2 * k1)
    if s_end is None:
        s_end = big_l + 42.0 / y_min
    kc = [complex(k) for k in media.k]
    loss = min(abs(k.imag) for k in kc)

    def lam_of(s):
        s = np.asarray(s, dtype=float)
        inside = s < big_l
        h = np.where(inside, delta * np.sin(np.pi * s / big_l), 0.0)
        dh = np.where(inside, delta * np.pi / big_l * np.cos(np.pi * s / big_l), 0.0)
        return s - 1j * h, 1.0 - 1j * dh

    c_phase = 3.0 / refine
    c_sing = 0.5 / refine
    w_cap = max(kmax / 32.0, 1.0) / refine

    def width(s):
        lam, _ = lam_of(s)
        lam = complex(lam)
        g1 = complex(gamma(lam, k1))
        w = w_cap
        w = min(w, c_phase / x_span)
        rate = abs(lam / g1) * y_max if abs(g1) > 0 else 1e300
        w = min(w, c_phase / (rate + extra_rate + 1e-300))
        w = min(w, 8.0 / refine / y_max)
        for kj in kc:
            w = min(w, c_sing * abs(lam - kj))
        if ks[0] - 1.0 <= s <= kmax + 1.0 and s < big_l:
            # guided-mode poles may sit anywhere near the real axis in this
            # range: at most the dip depth plus the loss offset away
            off = abs(delta * math.sin(math.pi * s / big_l)) + loss
            w = min(w, c_sing * max(off, 1e-9))
        return max(w, 1e-9)

    # the contour has a kink where the dip ends (s = L): a panel edge goes there
    breaks = sorted(b for b in (big_l, s_end) if 0.0 < b <= s_end)
    edges = [0.0]
    s = 0.0
    for stop in breaks:
        while s < stop:
            w = width(s)
            # keep the width consistent over the panel: also check its far end
            w = min(w, width(min(s + w, stop)) * 1.5)
            s = min(s + w, stop)
            if stop - s < 1e-3 * w:
                s = stop
            edges.append(s)
    edges = np.asarray(edges)
    a = edges[:-1, None]
    b = edges[1:, None]
    s_nodes = (0.5 * (b - a) * _GL_X[None, :] + 0.5 * (a + b)).ravel()
    s_w = (0.5 * (b - a) * _GL_W[None, :]).ravel()
    lam, dlam = lam_of(s_nodes)
    return lam, s_w * dlam


def _sigma_or(media, lam, sigma):
    if sigma is None:
        return sigma1(lam, media)
    if callable(sigma):
        return np.asarray(sigma(lam), dtype=complex) * np.ones_like(lam)
    return complex(sigma) * np.ones_like(lam)


def scattered_pairs(media: Media, X, Y, *, sigma=None, refine: float = 1.0, d_dY: bool = False):
    """G^s(X, Y) pair by pair, each with its own contour rule.

    X = x - x0, Y = y + y0 > 0 in the interface frame. ``sigma`` overrides
    sigma_1 (a constant or a callable of lambda) for the identity checks.
    G^s = (1/2pi) int_{Gamma+} e^{-g1 Y}/g1 cos(lambda X) sigma_1 d lambda.
    With ``d_dY`` the derivative in Y (the integrand times -g1), which is the
    derivative in either height y or y0.
    """
    X = np.atleast_1d(np.asarray(X, dtype=float))
    Y = np.atleast_1d(np.asarray(Y, dtype=float))
    out = np.empty(X.shape, dtype=complex)
    k1 = media.k1
    for i in range(X.size):
        lam, w = contour_rule(media, abs(X.flat[i]), Y.flat[i], Y.flat[i], refine=refine)
        g1 = gamma(lam, k1)
        sig = _sigma_or(media, lam, sigma)
        f = np.exp(-g1 * Y.flat[i]) / g1 * np.cos(lam * X.flat[i]) * sig
        if d_dY:
            f = -g1 * f
        out.flat[i] = np.sum(w * f) / (2.0 * np.pi)
    return out


# --------------------------------------------------------------------------
# Matvec with one rule for all pairs: the sum over sources is moved inside the
# integral, u_i = sum_q w_q F_q(x_i) S_q. This is exactly the pairwise sum of
# the same quadrature, reordered.
# --------------------------------------------------------------------------

_SHARED = {}


def _scatter_chunk(bounds):
    d = _SHARED
    lo, hi = bounds
    lam = d["lam"][lo:hi][None, :]
    g = d["g1"][lo:hi][None, :]
    coef = d["coef"][lo:hi]
    xs, ys, q = d["xs"], d["ys"], d["q"]
    xt, yt = d["xt"], d["yt"]
    u = np.zeros((q.shape[0], xt.size), dtype=complex)
    step = max(1, 4_000_000 // max(1, (hi - lo)))
    sm = np.zeros((q.shape[0], hi - lo), dtype=complex)
    sp = np.zeros((q.shape[0], hi - lo), dtype=complex)
    for j0 in range(0, xs.size, step):
        j1 = min(xs.size, j0 + step)
        base = np.exp(-g * ys[j0:j1, None])
        ph = np.exp(1j * lam * xs[j0:j1, None])
        sm += q[:, j0:j1] @ (base / ph)
        sp += q[:, j0:j1] @ (base * ph)
    sm *= coef[None, :]
    sp *= coef[None, :]
    for i0 in range(0, xt.size, step):
        i1 = min(xt.size, i0 + step)
        base = np.exp(-g * yt[i0:i1, None])
        ph = np.exp(1j * lam * xt[i0:i1, None])
        u[:, i0:i1] += sm @ (base * ph).T + sp @ (base / ph).T
    return u


def _workers():
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def scattered_matvec(media: Media, xt, yt, xs, ys, q, *, sigma=None, refine: float = 1.0,
                     workers: int | None = None):
    """u^s_i = sum_j G^s(x_i - x_j, y_i + y_j) q_j (interface frame).

    q has shape (nrhs, Ns) or (Ns,). Targets and sources may differ.
    """
    xt = np.asarray(xt, float)
    yt = np.asarray(yt, float)
    xs = np.asarray(xs, float)
    ys = np.asarray(ys, float)
    q = np.asarray(q, complex)
    squeeze = q.ndim == 1
    q = np.atleast_2d(q)
    if np.any(yt <= 0) or np.any(ys <= 0):
        raise ValueError("points must lie strictly above the top interface")
    x_mid = 0.5 * (min(xt.min(), xs.min()) + max(xt.max(), xs.max()))
    span = max(xt.max(), xs.max()) - min(xt.min(), xs.min())
    y_min = yt.min() + ys.min()
    y_max = yt.max() + ys.max()
    lam, w = contour_rule(media, span, y_min, y_max, refine=refine)
    g1 = gamma(lam, media.k1)
    sig = _sigma_or(media, lam, sigma)
    coef = w * sig / g1 / (4.0 * np.pi)
    _SHARED.update(lam=lam, g1=g1, coef=coef, xs=xs - x_mid, ys=ys, q=q, xt=xt - x_mid, yt=yt)
    nq = lam.size
    workers = workers or _workers()
    work = xs.size * nq + xt.size * nq
    if workers > 1 and work > 5e7:
        import multiprocessing as mp
        nchunk = workers * 4
        edges = np.linspace(0, nq, nchunk + 1).astype(int)
        tasks = [(int(edges[i]), int(edges[i + 1])) for i in range(nchunk) if edges[i + 1] > edges[i]]
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_scatter_chunk, tasks)
        u = sum(parts)
    else:
        u = np.zeros((q.shape[0], xt.size), dtype=complex)
        for lo in range(0, nq, 512):
            u += _scatter_chunk((lo, min(nq, lo + 512)))
    _SHARED.clear()
    return u[0] if squeeze else u


def layer_field(media: Media, layer: int, x, y, x0: float, y0: float, *, refine: float = 1.0):
    """Total field of a unit source at (x0, y0), y0 > 0, at points of a layer.

    Layer 1 (y >= 0): (i/4) H0(k1 r) + G^s. Layer 2 (-d <= y <= 0) and layer 3
    (y <= -d) use the densities sigma_2^+, sigma_2^-, sigma_3 of the interface
    system. Used only to check the interface conditions.
    """
    from scipy.special import hankel1

    x = np.atleast_1d(np.asarray(x, float))
    y = np.atleast_1d(np.asarray(y, float))
    k1, k2, k3, d = media.three_layer_view()
    out = np.empty(x.shape, dtype=complex)
    for i in range(x.size):
        xi, yi = x.flat[i], y.flat[i]
        X = xi - x0
        if layer == 1:
            r = math.hypot(X, yi - y0)
            out.flat[i] = 0.25j * hankel1(0, k1 * r) + scattered_pairs(media, X, yi + y0, refine=refine)[0]
            continue
        y_lo = y0
        y_hi = y0 + abs(yi) + d
        lam, w = contour_rule(media, abs(X), y_lo, y_hi, refine=refine)
        sc = sigma_coefficients(lam, media)
        g1 = gamma(lam, k1)
        src = np.exp(-g1 * y0)
        if layer == 2:
            g2 = gamma(lam, k2)
            dens = (np.exp(g2 * yi) * sc[..., 1] + np.exp(-g2 * (yi + d)) * sc[..., 2]) / g2
        elif layer == 3:
            g3 = gamma(lam, k3)
            dens = np.exp(g3 * (yi + d)) / g3 * sc[..., 3]
        else:
            raise ValueError("layer must be 1, 2 or 3")
        out.flat[i] = np.sum(w * dens * src * np.cos(lam * X)) / (2.0 * np.pi)
    return out


def m2l_entry(n: int, X: float, Y: float, media: Media, *, sigma=None, refine: float = 1.0):
    """A_n(X, Y): the order-n heterogeneous translation entry (n = m - p).

    The whole-line integral is folded: int_Gamma f = int_{Gamma+} [f(lam) + f(-lam)].
    Only well conditioned when |n| is modest compared with k1 * Y; used to pin
    the table generator at such entries.
    """
    k1 = media.k1
    n = int(n)
    rate = abs(n) / max(k1, 1e-300)
    s_peak = abs(n) / Y
    s_end = 1.5 * max(_singularities(media)) + 1.0 + s_peak + (42.0 + 2.0 * abs(n)) / Y
    lam, w = contour_rule(media, abs(X), Y, Y, refine=refine, s_end=s_end, extra_rate=rate)
    g1 = gamma(lam, k1)
    sig = _sigma_or(media, lam, sigma)
    base = np.exp(-g1 * Y) / g1 * sig
    zp = (lam - g1) / k1
    zm = (-lam - g1) / k1
    f = base * (np.exp(1j * lam * X) * zp ** n + np.exp(-1j * lam * X) * zm ** n)
    return ((-1j) ** n / (1j * np.pi)) * np.sum(w * f)
