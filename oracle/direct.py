"""Direct sums of the domain Green's function (the definition of the matvec).

Test infrastructure only (see the package docstring).

Paper passages followed:
* Section 2.4: phi(x) = int u_{x0}(x) rho(x0) dx0, discretised as A v with
  A_ij = u_{x_j}(x_i).
* Section 2.1, Eq. freeGreen: g = (i/4) H0^(1)(k1 |x - x0|).
* Section 2.3, Eq. multitop: the scattered part (see ``sommerfeld``); the
  middle- and bottom-layer fields of the same section for targets below the
  top interface (``cross_layer_apply``).

Self term (the paper is silent): the free term is dropped for i = j by index,
the scattered self term G^s(x_i, x_i) is kept.
"""
from __future__ import annotations

import numpy as np
from scipy.special import hankel1

from .media import Media
from .sommerfeld import _SHARED, _workers, scattered_matvec, scattered_pairs

_FREE = {}


def _free_block(bounds):
    d = _FREE
    i0, i1 = bounds
    xt, yt, tid = d["xt"][i0:i1], d["yt"][i0:i1], d["tid"][i0:i1]
    xs, ys, q, k = d["xs"], d["ys"], d["q"], d["k"]
    u = np.zeros((q.shape[0], i1 - i0), dtype=complex)
    step = max(1, 2_000_000 // max(1, i1 - i0))
    for j0 in range(0, xs.size, step):
        j1 = min(xs.size, j0 + step)
        r = np.hypot(xt[:, None] - xs[None, j0:j1], yt[:, None] - ys[None, j0:j1])
        same = tid[:, None] == np.arange(j0, j1)[None, :]
        r = np.where(same, 1.0, r)
        h = hankel1(0, k * r)
        h = np.where(same, 0.0, h)
        u += q[:, j0:j1] @ h.T
    return 0.25j * u


def free_matvec(k1, xt, yt, xs, ys, q, target_ids=None, workers=None):
    """u_i = (i/4) sum_{j != id_i} H0^(1)(k1 |x_i - x_j|) q_j.

    ``target_ids[i]`` is the source index that coincides with target i (its
    term is dropped), or -1. q is (nrhs, Ns) or (Ns,).
    """
    xt = np.asarray(xt, float)
    yt = np.asarray(yt, float)
    q = np.asarray(q, complex)
    squeeze = q.ndim == 1
    q = np.atleast_2d(q)
    if target_ids is None:
        target_ids = -np.ones(xt.size, dtype=np.int64)
    _FREE.update(xt=xt, yt=yt, tid=np.asarray(target_ids, np.int64), xs=np.asarray(xs, float),
                 ys=np.asarray(ys, float), q=q, k=k1)
    workers = workers or _workers()
    nt = xt.size
    if workers > 1 and nt * len(xs) > 2e7:
        import multiprocessing as mp
        nchunk = min(nt, workers * 4)
        edges = np.linspace(0, nt, nchunk + 1).astype(int)
        tasks = [(int(edges[i]), int(edges[i + 1])) for i in range(nchunk) if edges[i + 1] > edges[i]]
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_free_block, tasks)
        u = np.concatenate(parts, axis=1)
    else:
        u = _free_block((0, nt))
    _FREE.clear()
    return u[0] if squeeze else u


def direct_apply(media: Media, xy, q, targets=None, *, self_term=True, refine=1.0, workers=None):
    """(A q)_i for i in ``targets`` (all points if None); caller's frame.

    xy: (N, 2) points, all strictly above the top interface; q: (N,) or
    (nrhs, N). Returns (len(targets),) or (nrhs, len(targets)).
    """
    xy = np.asarray(xy, float)
    q = np.asarray(q, complex)
    n = xy.shape[0]
    tid = np.arange(n) if targets is None else np.asarray(targets, np.int64)
    x = xy[:, 0]
    y = media.to_frame(xy[:, 1])
    if np.any(y <= 0):
        raise ValueError("points must lie strictly above the top interface")
    uf = free_matvec(media.k1, x[tid], y[tid], x, y, q, target_ids=tid, workers=workers)
    us = scattered_matvec(media, x[tid], y[tid], x, y, q, refine=refine, workers=workers)
    if not self_term:
        gs_self = scattered_pairs(media, np.zeros(tid.size), 2.0 * y[tid], refine=refine)
        qq = np.atleast_2d(q)[:, tid]
        us = us - (gs_self[None, :] * qq).reshape(us.shape)
    return uf + us


def cross_layer_apply(media: Media, xy_src, q, xy_tgt, *, refine=1.0):
    """u_t = sum_s q_s u_{x_s}(x_t) for sources in the top layer and targets
    below it (caller's frame): the middle- and bottom-layer fields of a
    top-layer source (Section 2.3, u_2 = u_2^t + u_2^b and u_3, with the
    densities sigma_2^+, sigma_2^-, sigma_3 of the interface system), summed
    over the sources one at a time (``sommerfeld.layer_field``). A target at
    or above the lower interface (three layers) is in the middle layer; with
    two layers every target is in the lower half-space.

    xy_src: (Ns, 2), strictly above the top interface; xy_tgt: (Nt, 2),
    strictly below it; q: (Ns,) or (nrhs, Ns). Returns (Nt,) or (nrhs, Nt).
    """
    from .sommerfeld import layer_field

    xs = np.asarray(xy_src, float)
    xt = np.asarray(xy_tgt, float)
    q = np.asarray(q, complex)
    squeeze = q.ndim == 1
    q = np.atleast_2d(q)
    ys = media.to_frame(xs[:, 1])
    yt = media.to_frame(xt[:, 1])
    if np.any(ys <= 0) or np.any(yt >= 0):
        raise ValueError("sources strictly above and targets strictly below the top interface")
    layer = np.full(yt.size, 2)
    if media.layers == 3:
        layer[yt < -media.d] = 3
    u = np.zeros((q.shape[0], yt.size), dtype=complex)
    for j in range(xs.shape[0]):
        for lay in (2, 3):
            idx = np.nonzero(layer == lay)[0]
            if idx.size:
                f = layer_field(media, lay, xt[idx, 0], yt[idx], xs[j, 0], ys[j], refine=refine)
                u[:, idx] += q[:, j:j + 1] * f[None, :]
    return u[0] if squeeze else u


def dense_matrix(media: Media, xy, *, refine=1.0):
    """The dense N x N matrix A (small N only): column j = A applied to e_j."""
    xy = np.asarray(xy, float)
    n = xy.shape[0]
    eye = np.eye(n, dtype=complex)
    return direct_apply(media, xy, eye, refine=refine, workers=1).T


__all__ = ["free_matvec", "direct_apply", "cross_layer_apply", "dense_matrix", "_SHARED"]
