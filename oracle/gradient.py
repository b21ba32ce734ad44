"""Source-coordinate gradient of Re <v, A q> (test infrastructure only).

g_j = sum_r Re( q_rj sum_i conj(v_ri) dA_ij/d(x_j, y_j) ), targets held fixed,
written out from the definition of A (Section 2.4) term by term:

* free part, Eq. freeGreen: d/dx_j (i/4) H0^(1)(k1 r_ij) = -(i/4) k1 H1^(1)(k1 r) (x_j - x_i)/r
  (H0' = -H1), the i = j term excluded by index as in the matvec;
* scattered part, Eq. multitop in its full-line form
  G^s = (1/4pi) int e^{-g1 (y + y0)} / g1 e^{i lambda (x - x0)} sigma_1 d lambda:
  the source coordinates enter only through e^{-g1 y0 - i lambda x0}, so
  d/dx0 multiplies the integrand by -i lambda and d/dy0 by -g1. It uses the
  same single contour rule as ``sommerfeld.scattered_matvec`` with the sums over
  targets moved inside the integral.
"""
from __future__ import annotations

import numpy as np
from scipy.special import hankel1

from .media import Media, gamma
from .sommerfeld import _sigma_or, contour_rule


def free_source_gradient(k1, x, y, q, v):
    """(N, 2) gradient of the free part; x, y in any common frame."""
    q = np.atleast_2d(np.asarray(q, complex))
    v = np.atleast_2d(np.asarray(v, complex))
    n = x.size
    g = np.zeros((n, 2))
    step = max(1, 2_000_000 // n)
    for i0 in range(0, n, step):
        i1 = min(n, i0 + step)
        dx = x[None, :] - x[i0:i1, None]          # x_j - x_i, rows i
        dy = y[None, :] - y[i0:i1, None]
        r = np.hypot(dx, dy)
        same = np.arange(i0, i1)[:, None] == np.arange(n)[None, :]
        r = np.where(same, 1.0, r)
        d = -0.25j * k1 * hankel1(1, k1 * r) / r   # d/dr of (i/4) H0 divided by r
        d = np.where(same, 0.0, d)
        for rr in range(q.shape[0]):
            sx = np.conj(v[rr, i0:i1]) @ (d * dx)
            sy = np.conj(v[rr, i0:i1]) @ (d * dy)
            g[:, 0] += np.real(q[rr] * sx)
            g[:, 1] += np.real(q[rr] * sy)
    return g


def scattered_source_gradient(media: Media, x, y, q, v, *, refine: float = 1.0):
    """(N, 2) gradient of the scattered part; x, y in the interface frame."""
    q = np.atleast_2d(np.asarray(q, complex))
    v = np.atleast_2d(np.asarray(v, complex))
    x_mid = 0.5 * (x.min() + x.max())
    xc = x - x_mid
    span = x.max() - x.min()
    lam, w = contour_rule(media, span, 2.0 * y.min(), 2.0 * y.max(), refine=refine)
    g1 = gamma(lam, media.k1)
    coef = w * _sigma_or(media, lam, None) / g1 / (4.0 * np.pi)
    g = np.zeros((x.size, 2))
    step = max(1, 4_000_000 // max(1, lam.size))
    for rr in range(q.shape[0]):
        # target sums: t_plus = sum_i conj(v_i) e^{-g1 y_i + i lam x_i}, t_minus with -i lam
        tp = np.zeros(lam.size, complex)
        tm = np.zeros(lam.size, complex)
        for i0 in range(0, x.size, step):
            i1 = min(x.size, i0 + step)
            base = np.exp(-g1[None, :] * y[i0:i1, None])
            ph = np.exp(1j * lam[None, :] * xc[i0:i1, None])
            cv = np.conj(v[rr, i0:i1])
            tp += cv @ (base * ph)
            tm += cv @ (base / ph)
        for j0 in range(0, x.size, step):
            j1 = min(x.size, j0 + step)
            base = np.exp(-g1[None, :] * y[j0:j1, None])
            ph = np.exp(1j * lam[None, :] * xc[j0:j1, None])
            # source factors e^{-g1 y_j -/+ i lam x_j} pair with t_plus / t_minus
            e_m = base / ph * (coef * tp)[None, :]
            e_p = base * ph * (coef * tm)[None, :]
            sx = (e_m * (-1j * lam)[None, :] + e_p * (1j * lam)[None, :]).sum(axis=1)
            sy = ((e_m + e_p) * (-g1)[None, :]).sum(axis=1)
            g[j0:j1, 0] += np.real(q[rr, j0:j1] * sx)
            g[j0:j1, 1] += np.real(q[rr, j0:j1] * sy)
    return g


def source_gradient(media: Media, xy, q, v, *, refine: float = 1.0, self_term: bool = True):
    """g_j = sum_r Re( q_rj sum_i conj(v_ri) dA_ij/d(x_j, y_j) ) for all j.

    xy: (N, 2) in the caller's frame (all points above the top interface);
    q, v: (N,) or (nrhs, N). Returns (N, 2); y derivatives are frame-free.
    With ``self_term=False`` A has no scattered self term (A_jj = 0): the
    pair (j, j) is removed, whose derivative in the source point, the target
    held at x_j, is d/dY G^s(0, 2 y_j) in y and zero in x (G^s is even in X).
    """
    xy = np.asarray(xy, float)
    x = xy[:, 0]
    y = media.to_frame(xy[:, 1])
    g = free_source_gradient(media.k1, x, y, q, v) + scattered_source_gradient(media, x, y, q, v, refine=refine)
    if not self_term:
        from .sommerfeld import scattered_pairs
        qq = np.atleast_2d(np.asarray(q, complex))
        vv = np.atleast_2d(np.asarray(v, complex))
        dgs = scattered_pairs(media, np.zeros(x.size), 2.0 * y, refine=refine, d_dY=True)
        g[:, 1] -= np.real((qq * np.conj(vv)).sum(axis=0) * dgs)
    return g


__all__ = ["source_gradient", "free_source_gradient", "scattered_source_gradient"]
