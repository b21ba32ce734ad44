"""Sources in the middle layer of the three-layer medium (TEST INFRASTRUCTURE).

Test infrastructure only (see the package docstring).

The paper treats sources in the top layer and leaves the middle layer to a
follow-up (Section 2.3, closing paragraph). This module writes the middle
layer's fields from the same spectral representation as Section 2.3, with the
free field of a layer-2 source as the incident field:

* incident in layer 2: e^{-g2 |y - y0|}/g2 (the density of Eq. spectralfree
  with k2), times (1/4pi) e^{i lambda (x - x0)} under the integral;
* layer 1 (y > 0): a1 e^{-g1 y}; layer 2: a2 e^{g2 y} + b2 e^{-g2 (y + d)}
  (the waves leaving the top and the bottom interface); layer 3 (y < -d):
  a3 e^{g3 (y + d)};
* continuity of u and du/dy at y = 0 and y = -d (the interface conditions of
  Section 2.3): four equations in (a1, a2, b2, a3), solved numerically at
  every node with numpy.

The interface frame is the paper's: the top interface at y = 0, the lower at
y = -d. Integrals run on the half contour of ``sommerfeld.contour_rule``
(folded with cos(lambda X), as there).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import hankel1

from .media import Media, gamma
from .sommerfeld import contour_rule


def middle_coefficients(lam, media: Media, y0: float):
    """(a1, a2, b2, a3) at each lambda for a unit source at height y0 in the
    middle layer (-d < y0 < 0, interface frame). Returns an array (..., 4)."""
    k1, k2, k3, d = media.three_layer_view()
    lam = np.asarray(lam, dtype=complex)
    g1, g2, g3 = gamma(lam, k1), gamma(lam, k2), gamma(lam, k3)
    e = np.exp(-g2 * d)
    up = np.exp(g2 * y0)            # the incident wave at y = 0 (times 1/g2)
    dn = np.exp(-g2 * (y0 + d))     # the incident wave at y = -d (times 1/g2)
    m = np.zeros(lam.shape + (4, 4), dtype=complex)
    rhs = np.zeros(lam.shape + (4, 1), dtype=complex)
    # y = 0: u1 = u2,  du1/dy = du2/dy
    m[..., 0, 0] = 1.0
    m[..., 0, 1] = -1.0
    m[..., 0, 2] = -e
    rhs[..., 0, 0] = up / g2
    m[..., 1, 0] = -g1
    m[..., 1, 1] = -g2
    m[..., 1, 2] = g2 * e
    rhs[..., 1, 0] = -up
    # y = -d: u2 = u3,  du2/dy = du3/dy
    m[..., 2, 1] = e
    m[..., 2, 2] = 1.0
    m[..., 2, 3] = -1.0
    rhs[..., 2, 0] = -dn / g2
    m[..., 3, 1] = g2 * e
    m[..., 3, 2] = -g2
    m[..., 3, 3] = -g3
    rhs[..., 3, 0] = -dn
    return np.linalg.solve(m, rhs)[..., 0]


def middle_source_field(media: Media, layer: int, x, y, x0: float, y0: float, *, refine: float = 1.0,
                        scattered_only: bool = False):
    """Field of a unit source at (x0, y0) in the middle layer at points of a
    layer (interface frame): layer 2 the free part (i/4) H0(k2 r) (omitted with
    ``scattered_only``) plus a2 e^{g2 y} + b2 e^{-g2 (y + d)}; layers 1 and 3
    the transmitted fields."""
    k1, k2, k3, d = media.three_layer_view()
    if media.layers != 3:
        raise ValueError("the middle layer needs three layers")
    if not -d < y0 < 0:
        raise ValueError("the source must lie strictly inside the middle layer")
    x = np.atleast_1d(np.asarray(x, float))
    y = np.atleast_1d(np.asarray(y, float))
    out = np.empty(x.shape, dtype=complex)
    for i in range(x.size):
        xi, yi = x.flat[i], y.flat[i]
        X = xi - x0
        if layer == 2:
            ylo = min(-(yi + y0), yi + y0 + 2 * d)
        elif layer == 1:
            ylo = yi - y0
        else:
            ylo = y0 - yi
        lam, w = contour_rule(media, abs(X), ylo, max(ylo, 2 * d + abs(yi)), refine=refine)
        c = middle_coefficients(lam, media, y0)
        if layer == 2:
            dens = c[..., 1] * np.exp(gamma(lam, k2) * yi) + c[..., 2] * np.exp(-gamma(lam, k2) * (yi + d))
        elif layer == 1:
            dens = c[..., 0] * np.exp(-gamma(lam, k1) * yi)
        elif layer == 3:
            dens = c[..., 3] * np.exp(gamma(lam, k3) * (yi + d))
        else:
            raise ValueError("layer must be 1, 2 or 3")
        v = np.sum(w * dens * np.cos(lam * X)) / (2.0 * math.pi)
        if layer == 2 and not scattered_only:
            v += 0.25j * hankel1(0, k2 * math.hypot(X, yi - y0))
        out.flat[i] = v
    return out


def middle_apply(media: Media, xy, q, targets=None, *, scattered_only=False, refine=1.0):
    """(A q)_i for points in the middle layer (caller's frame): the free part
    (i/4) H0(k2 |x_i - x_j|) with the i = j term dropped, plus the scattered
    part of the middle layer with its smooth self term kept (the same readings
    as the top-layer matvec); ``scattered_only`` leaves the free part out.
    xy: (N, 2) strictly between the interfaces; q: (N,) or (nrhs, N)."""
    xy = np.asarray(xy, float)
    q = np.asarray(q, complex)
    squeeze = q.ndim == 1
    q = np.atleast_2d(q)
    n = xy.shape[0]
    tid = np.arange(n) if targets is None else np.asarray(targets, np.int64)
    x = xy[:, 0]
    y = media.to_frame(xy[:, 1])
    k1, k2, k3, d = media.three_layer_view()
    if media.layers != 3 or np.any(y >= 0) or np.any(y <= -d):
        raise ValueError("points must lie strictly inside the middle layer of a three-layer medium")
    u = np.zeros((q.shape[0], tid.size), dtype=complex)
    for j in range(n):
        f = middle_source_field(media, 2, x[tid], y[tid], x[j], y[j], refine=refine, scattered_only=True)
        if not scattered_only:
            r = np.hypot(x[tid] - x[j], y[tid] - y[j])
            free = np.where(tid == j, 0.0, 0.25j * hankel1(0, k2 * np.where(tid == j, 1.0, r)))
            f = f + free
        u += q[:, j:j + 1] * f[None, :]
    return u[0] if squeeze else u


__all__ = ["middle_coefficients", "middle_source_field", "middle_apply"]
