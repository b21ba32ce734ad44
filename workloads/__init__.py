"""Seeded synthetic workloads for the layered-media Helmholtz matvec.

This module only draws inputs: point sets, strengths and the description of the
layered medium. It holds none of the method's arithmetic, so that both the CPU
oracle and the GPU library can be fed from it without sharing any code.

Random numbers come from NumPy's PCG64 seeded with a SeedSequence built from a
list of integers. The draw order is fixed: geometry first, then strengths (the
real block, then the imaginary block).

Coordinates are given in the frame of the workload description (the "config
frame"); the interfaces are horizontal lines y = const listed top to bottom, and
the wavenumbers are listed top layer first.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass
class Workload:
    name: str
    k: tuple                 # wavenumbers, top layer first
    interfaces: tuple        # interface heights, top first (strictly decreasing)
    xy: np.ndarray           # (N, 2) float64 points; sources = targets
    q: np.ndarray            # (nrhs, N) complex128 strengths
    leaf: int                # maximum points per leaf box
    tol: float               # requested relative accuracy
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.xy.shape[0])


def rng_for(*seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))


def complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im


def uniform_box(rng, n, x0, x1, y0, y1) -> np.ndarray:
    x = rng.uniform(x0, x1, n)
    y = rng.uniform(y0, y1, n)
    return np.stack([x, y], axis=1)


def ellipse_points(rng, n_total, n_ellipses, cy_range, min_bottom,
                   axis_range=(0.02, 0.08), cx_range=(0.0, 1.0), max_top=None) -> np.ndarray:
    """Points on random ellipses, equispaced in the parameter.

    Per ellipse, in this order: semi-axes a, b ~ U(axis_range), orientation
    phi ~ U(0, pi), centre x ~ U(cx_range), centre y ~ U(cy_range), the last
    redrawn until the lowest point of the ellipse is at least ``min_bottom``
    (and, with ``max_top``, its highest point at most ``max_top``).
    ``n_total`` points are split evenly, the remainder going to the first
    ellipses.
    """
    base, rem = divmod(n_total, n_ellipses)
    out = []
    for e in range(n_ellipses):
        a = rng.uniform(*axis_range)
        b = rng.uniform(*axis_range)
        phi = rng.uniform(0.0, math.pi)
        cx = rng.uniform(*cx_range)
        half_height = math.sqrt((a * math.sin(phi)) ** 2 + (b * math.cos(phi)) ** 2)
        while True:
            cy = rng.uniform(*cy_range)
            if cy - half_height >= min_bottom and (max_top is None or cy + half_height <= max_top):
                break
        m = base + (1 if e < rem else 0)
        t = TWO_PI * np.arange(m) / m
        ex = a * np.cos(t)
        ey = b * np.sin(t)
        c, s = math.cos(phi), math.sin(phi)
        out.append(np.stack([cx + c * ex - s * ey, cy + s * ex + c * ey], axis=1))
    return np.concatenate(out, axis=0)


# ---------------------------------------------------------------------------
# The five workloads (full size) and reduced versions of the same recipes.
# ---------------------------------------------------------------------------

def two_layer_uniform(n=1024, seed=1, nrhs=1):
    """Two layers, interface y=0, k1=8pi over k2=12pi; N uniform in [0,1]x[0.05,1.05]."""
    rng = rng_for(1703, 9136, seed)
    xy = uniform_box(rng, n, 0.0, 1.0, 0.05, 1.05)
    q = complex_normal(rng, (nrhs, n))
    return Workload("two-layer k=(8pi,12pi) uniform N=%d" % n, (8 * math.pi, 12 * math.pi),
                    (0.0,), xy, q, leaf=32, tol=1e-10)


def two_layer_hf(n=1 << 17, seed=2, nrhs=1):
    """Two layers, interface y=0, k=2pi*(64, 96); N uniform in [0,1]x[0.01,1.01]."""
    rng = rng_for(1703, 9136, seed)
    xy = uniform_box(rng, n, 0.0, 1.0, 0.01, 1.01)
    q = complex_normal(rng, (nrhs, n))
    return Workload("two-layer k=2pi*(64,96) uniform N=%d" % n, (TWO_PI * 64, TWO_PI * 96),
                    (0.0,), xy, q, leaf=64, tol=1e-8)


THREE_LAYER_K = (TWO_PI * 80, TWO_PI * 120, TWO_PI * 100)
THREE_LAYER_IF = (0.5, 0.0)


def three_layer_ellipses(n=1_000_000, seed=3, nrhs=1, n_ellipses=64):
    """Three layers (interfaces y=0.5, y=0; k=2pi*(80,120,100) top to bottom).

    The points lie in the top layer: 64 ellipses with centres y ~ U(0.5, 1.0),
    every ellipse at least 0.01 above the top interface.
    """
    rng = rng_for(1703, 9136, seed)
    xy = ellipse_points(rng, n, n_ellipses, (0.5, 1.0), 0.51)
    q = complex_normal(rng, (nrhs, n))
    return Workload("three-layer k=2pi*(80,120,100) 64 ellipses N=%d" % n, THREE_LAYER_K,
                    THREE_LAYER_IF, xy, q, leaf=64, tol=1e-8)


def middle_layer_ellipses(n=1_000_000, seed=5, nrhs=1, n_ellipses=64):
    """The three-layer medium above with the points in the middle layer: 64
    ellipses with centres y ~ U(0, 0.5) (uniform in the slab), every ellipse
    at least 0.01 inside both interfaces."""
    rng = rng_for(1703, 9136, seed)
    xy = ellipse_points(rng, n, n_ellipses, (0.0, 0.5), 0.01, max_top=0.49)
    q = complex_normal(rng, (nrhs, n))
    return Workload("middle layer k=2pi*(80,120,100) 64 ellipses N=%d" % n, THREE_LAYER_K,
                    THREE_LAYER_IF, xy, q, leaf=64, tol=1e-8)


def batched_geometry(g, nrhs=256, lo=12.0, hi=18.0, size_scale=1.0):
    """Geometry g of the batched workload: three layers as above, N_g =
    round(2**U(12,18)) points on 64 ellipses placed as in the N = 10^6
    workload, nrhs complex N(0,1) right-hand sides."""
    rng = rng_for(1703, 9136, 4, g)
    n = int(round(2.0 ** rng.uniform(lo, hi) * size_scale))
    n = max(n, 64)
    xy = ellipse_points(rng, n, 64, (0.5, 1.0), 0.51)
    q = complex_normal(rng, (nrhs, n))
    return Workload("batched geometry %d N=%d" % (g, n), THREE_LAYER_K, THREE_LAYER_IF,
                    xy, q, leaf=64, tol=1e-8)


def batched_geometries(n_geom=32, nrhs=256, lo=12.0, hi=18.0, size_scale=1.0):
    """32 three-layer ellipse geometries, N_g = round(2**U(12,18)), nrhs each."""
    return [batched_geometry(g, nrhs, lo, hi, size_scale) for g in range(n_geom)]


# the smallest, a median and the largest geometry of the batched workload
BATCHED_SMALLEST, BATCHED_MEDIAN, BATCHED_LARGEST = 11, 23, 8


def two_layer_ellipses_grad(n=1 << 18, seed=5, n_fd=64):
    """Two layers k=2pi*(64,96); 64 ellipses with centres y~U(0,1), 0.01 clearance.

    Returns the workload with q0, the perturbation xi (u_obs = A(q0 + 0.1 xi))
    and the finite-difference sample: ``n_fd`` (source index, axis) pairs.
    """
    rng = rng_for(1703, 9136, seed)
    xy = ellipse_points(rng, n, 64, (0.0, 1.0), 0.01)
    q0 = complex_normal(rng, (1, n))
    xi = complex_normal(rng, (1, n))
    fd_index = rng.integers(0, n, n_fd)
    fd_axis = rng.integers(0, 2, n_fd)
    w = Workload("two-layer k=2pi*(64,96) 64 ellipses N=%d" % n, (TWO_PI * 64, TWO_PI * 96),
                 (0.0,), xy, q0, leaf=64, tol=1e-8)
    w.extra.update(xi=xi, fd_index=fd_index, fd_axis=fd_axis, h=1e-6)
    return w


def random_points_above(rng, n, k, interfaces, box=(0.0, 1.0), height=(0.02, 1.0)):
    """Small generic helper for tests: n points uniform above the top interface."""
    y_top = interfaces[0]
    return uniform_box(rng, n, box[0], box[1], y_top + height[0], y_top + height[1])
