"""CPU oracle for the layered-media Helmholtz matvec (TEST INFRASTRUCTURE).

This package is a plain, slow, FP64 implementation of what the GPU library
computes, written from the paper's definitions (Cho, Huang, Chen, Cai, "A
heterogeneous FMM for 2-D layered media Helmholtz equation I: two and three
layers cases"). It exists only to check the GPU path: only the test suite, the
package smoke test and the CPU-baseline leg of the benchmark may import it.
The product path never imports, links or runs anything here, and nothing here
imports the product package.

What it computes (Section 2 of the paper):

* u_i = sum_j A_ij q_j with A_ij = u_{x_j}(x_i), the domain Green's function
  (Section 2.4, the discretised potential).
* u_{x0}(x) = g(x, x0) + u^s(x): the free-space part g = (i/4) H0^(1)(k1|x-x0|)
  (Section 2.1, Eq. freeGreen) and the scattered part of the top layer given
  by the Sommerfeld integral with the reflection function sigma_1
  (Section 2.3, Eq. multitop), sigma_1 being fixed by the interface system of
  Section 2.3.

Readings taken where the paper is silent:

* two layers with a transmission interface are the three-layer system with
  k3 = k2 (the result does not depend on d);
* the self term: the singular free term i = j is dropped (by index), the smooth
  scattered self term G^s(x_i, x_i) is kept;
* lossless media are integrated on the limiting-absorption side: the contour
  passes below the real-axis singularities with Re(lambda) > 0 (above those
  with Re(lambda) < 0).

Modules: ``media`` (branches, sigma), ``sommerfeld`` (contour rules and the
Sommerfeld integrals), ``direct`` (the dense direct sums), ``gradient`` (the
source-coordinate gradient of Re <v, A q>, targets held fixed), ``middle``
(sources in the middle layer: the interface system with a layer-2 source,
which the paper leaves to a follow-up).
"""
from .media import Media, gamma, sigma_coefficients, sigma1  # noqa: F401
from .sommerfeld import (contour_rule, scattered_pairs, scattered_matvec,  # noqa: F401
                         layer_field, m2l_entry)
from .direct import free_matvec, direct_apply, cross_layer_apply, dense_matrix  # noqa: F401
from .gradient import source_gradient  # noqa: F401
from .middle import middle_coefficients, middle_source_field, middle_apply  # noqa: F401
