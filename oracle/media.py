"""Layered medium: the branch of gamma_j and the interface system for sigma.

Test infrastructure only (see the package docstring).

Paper passages followed:
* Section 2.1, Eq. evanprop: gamma = sqrt(lambda^2 - k^2), evanescent for
  |lambda| > k, propagating for |lambda| < k (outgoing: gamma = -i sqrt(k^2 -
  lambda^2)).
* Section 2.3: the three-layer representation (u1^s, u2^t, u2^b, u3) and the
  4x4 linear system for (sigma_1, sigma_2^+, sigma_2^-, sigma_3) obtained from
  [u] = [du/dn] = 0 at y = 0 and y = -d.
* Section 2.2: the impedance half-space (one medium above y = 0 with
  du/dn - i alpha u = 0 there), whose scattered field has the Sommerfeld form
  of Eq. multisommer with sigma-hat = (gamma + i alpha)/(gamma - i alpha).

Reading: the source factor in the middle and bottom layer fields is
exp(-gamma_1 y0) (the source sits in layer 1); with that reading the system
does not depend on y0, and it is the system printed in the paper.
"""
from __future__ import annotations

import numpy as np


class Media:
    """A two- or three-layer medium, wavenumbers top layer first; or, with
    ``impedance`` = alpha > 0, the impedance half-space: one wavenumber and
    one boundary height, the boundary condition du/dn - i alpha u = 0 (n the
    outward normal of the half-space, -y).

    ``interfaces`` are heights in the caller's frame, top first. The oracle
    works in the interface frame, where the top interface is y = 0; use
    ``to_frame`` to shift coordinates.
    """

    def __init__(self, k, interfaces, impedance=None):
        k = tuple(complex(v) if np.iscomplexobj(v) else float(v) for v in k)
        interfaces = tuple(float(v) for v in interfaces)
        self.alpha = None
        if impedance is not None:
            if len(k) != 1 or len(interfaces) != 1:
                raise ValueError("the impedance half-space has one wavenumber and one boundary")
            if not float(impedance) > 0.0:
                raise ValueError("the impedance alpha must be > 0")
            self.alpha = float(impedance)
        elif len(k) not in (2, 3) or len(interfaces) != len(k) - 1:
            raise ValueError("need 2 or 3 layers and layers-1 interfaces")
        self.k = k
        self.interfaces = interfaces
        self.y_top = interfaces[0]
        if len(k) == 3:
            self.d = interfaces[0] - interfaces[1]
            if not self.d > 0:
                raise ValueError("interfaces must be strictly decreasing")
        else:
            self.d = None

    @property
    def layers(self) -> int:
        return len(self.k)

    @property
    def k1(self):
        return self.k[0]

    def three_layer_view(self):
        """(k1, k2, k3, d): two layers are the three-layer system with k3 = k2."""
        if self.alpha is not None:
            raise ValueError("the impedance half-space has no interface system")
        if self.layers == 3:
            return self.k[0], self.k[1], self.k[2], self.d
        return self.k[0], self.k[1], self.k[1], 1.0

    def to_frame(self, y):
        return np.asarray(y, dtype=float) - self.y_top


def gamma(lam, k):
    """sqrt(lambda^2 - k^2) on the physical sheet.

    Re(gamma) >= 0. Where lambda^2 - k^2 is a negative real number (real
    |lambda| < k) the outgoing value -i sqrt(k^2 - lambda^2) is taken; off the
    real axis the principal root is the continuation of that choice from the
    limiting-absorption side (Im(lambda^2 - k^2) < 0).
    """
    lam = np.asarray(lam, dtype=complex)
    w = lam * lam - k * k
    g = np.sqrt(w)
    on_cut = (w.imag == 0.0) & (w.real < 0.0)
    if np.any(on_cut):
        g = np.where(on_cut, -1j * np.sqrt(np.abs(w.real)), g)
    return g


def sigma_coefficients(lam, media: Media):
    """Solve the interface system of Section 2.3 at each lambda.

    Returns an array (..., 4): sigma_1, sigma_2^+, sigma_2^-, sigma_3.
    Unknown order and equations as printed: continuity of u and of du/dy at
    y = 0 and y = -d, the spectral densities being
      u1^s ~ e^{-g1 y}/g1 sigma_1,  u2^t ~ e^{g2 y}/g2 sigma_2^+,
      u2^b ~ e^{-g2 (y+d)}/g2 sigma_2^-,  u3 ~ e^{g3 (y+d)}/g3 sigma_3,
    all times e^{-g1 y0} e^{i lambda (x - x0)}, and the incident density
    e^{-g1 |y - y0|}/g1.
    """
    k1, k2, k3, d = media.three_layer_view()
    lam = np.asarray(lam, dtype=complex)
    g1 = gamma(lam, k1)
    g2 = gamma(lam, k2)
    g3 = gamma(lam, k3)
    e = np.exp(-g2 * d)
    m = np.zeros(lam.shape + (4, 4), dtype=complex)
    m[..., 0, 0] = 1.0 / g1
    m[..., 0, 1] = -1.0 / g2
    m[..., 0, 2] = -e / g2
    m[..., 1, 1] = e / g2
    m[..., 1, 2] = 1.0 / g2
    m[..., 1, 3] = -1.0 / g3
    m[..., 2, 0] = 1.0
    m[..., 2, 1] = 1.0
    m[..., 2, 2] = -e
    m[..., 3, 1] = e
    m[..., 3, 2] = -1.0
    m[..., 3, 3] = -1.0
    rhs = np.zeros(lam.shape + (4, 1), dtype=complex)
    rhs[..., 0, 0] = -1.0 / g1
    rhs[..., 2, 0] = 1.0
    return np.linalg.solve(m, rhs)[..., 0]


def sigma1(lam, media: Media):
    """The reflection function sigma_1(lambda) of the top layer; for the
    impedance half-space sigma-hat = (gamma + i alpha)/(gamma - i alpha)
    (Section 2.2, after Eq. spectraldomain)."""
    if media.alpha is not None:
        g = gamma(np.asarray(lam, dtype=complex), media.k1)
        return (g + 1j * media.alpha) / (g - 1j * media.alpha)
    return sigma_coefficients(lam, media)[..., 0]
