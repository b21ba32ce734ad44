"""The series classes of the direct pairs (the near-field kernels and their
gradient): at the largest argument of each class, x = 2 sqrt(zmax), the
class's term count truncates the small-argument series of H0^(1) (forward)
and H1^(1) (gradient) below the stated bounds, against mpmath's Bessel
functions. The class table is read from the kernel header.
"""
import os
import re

import pytest

mpmath = pytest.importorskip("mpmath")

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_1703_09136_amd", "csrc", "special.hpp")


def _table(name):
    text = open(HDR).read()
    m = re.search(r"%s\[kH0Classes\] = \{([^}]*)\}" % name, text)
    assert m, name
    return [float(v) for v in m.group(1).split(",")]


def _h0_series(x, terms):
    mp = mpmath
    z = x * x / 4
    a, h = mp.mpf(1), mp.mpf(0)
    j0 = y = mp.mpf(0)
    for m in range(terms):
        if m > 0:
            a = a * (-1) / (m * m)
            h += mp.mpf(1) / m
        j0 += a * z ** m
        y -= h * a * z ** m
    y0 = 2 / mp.pi * ((mp.log(x / 2) + mp.euler) * j0 + y)
    return j0, y0


def _h1_series(x, terms):
    mp = mpmath
    z = x * x / 4
    a, h = mp.mpf(1), mp.mpf(0)
    sa = sb = mp.mpf(0)
    for m in range(terms):
        if m > 0:
            a = a * (-1) / (m * (m + 1))
            h += mp.mpf(1) / m
        sa += a * z ** m
        sb += (2 * h + mp.mpf(1) / (m + 1)) * a * z ** m
    j1 = x / 2 * sa
    y1 = 2 / mp.pi * ((mp.log(z) / 2 + mp.euler) * j1 - 1 / x) - x / (2 * mp.pi) * sb
    return j1, y1


def test_class_tables_cover_the_series_range():
    zmax = _table("kH0ClassZmax")
    terms = _table("kH0ClassTerms")
    assert len(zmax) == len(terms) == 5
    assert zmax == sorted(zmax) and terms == sorted(terms)
    assert abs(zmax[-1] - 9.0) < 1e-12          # the last class ends at x = 6 (large-argument form above)


@pytest.mark.parametrize("c", range(5))
def test_h0_and_h1_truncation_per_class(c):
    mp = mpmath
    mp.mp.dps = 40
    zmax = _table("kH0ClassZmax")[c]
    m = int(_table("kH0ClassTerms")[c])
    x = 2 * mp.sqrt(zmax)
    j0, y0 = _h0_series(x, m)
    e0 = abs(mp.mpc(j0 - mp.besselj(0, x), y0 - mp.bessely(0, x))) / abs(mp.mpc(mp.besselj(0, x), mp.bessely(0, x)))
    j1, y1 = _h1_series(x, m)
    e1 = abs(mp.mpc(j1 - mp.besselj(1, x), y1 - mp.bessely(1, x))) / abs(mp.mpc(mp.besselj(1, x), mp.bessely(1, x)))
    print("class %d x=%.3f terms %d: H0 %.2e, H1 %.2e" % (c, float(x), m, float(e0), float(e1)))
    assert e0 < 2.0 ** -52
    assert e1 < 2e-18
    # the table is tight: one term fewer leaves an H0 remainder above 2^-56
    j0s, y0s = _h0_series(x, m - 1)
    es = abs(mp.mpc(j0s - mp.besselj(0, x), y0s - mp.bessely(0, x))) / abs(mp.mpc(mp.besselj(0, x), mp.bessely(0, x)))
    assert es > 2.0 ** -56
