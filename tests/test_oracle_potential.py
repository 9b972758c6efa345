"""Pins of the oracle's pair functions (Sec. 2.1, eq. lj_cutoff).

What pins them, independently of the oracle's own formulas:
  * exact rational arithmetic: c2, c0 are re-derived here by solving the two
    linear conditions V(rc) = V'(rc) = 0 with Fractions, and V, g are evaluated
    exactly at rational r^2 (chain rule through r^2, a different form from the
    oracle's);
  * central differences of the oracle's own V for g = -V'/r, V'' and dV/dsigma;
  * the explicit force expression printed in Sec. 3.2 (sign and factors);
  * the untruncated limit rc -> infinity (well depth -eps at r = 2^(1/6) sigma);
  * the scaling law V(r; eps, sigma, rc) = eps V(r/sigma; 1, 1, rc/sigma).
"""

from fractions import Fraction as Fr

import numpy as np
import pytest


def exact_coeffs(rc2: Fr, sig2: Fr = Fr(1)):
    """Solve V(rc) = 0 and dV/d(r^2)(rc) = 0 for (c2, c0), exactly.

    In terms of s = r^2: V/4eps = sig^12 s^-6 - sig^6 s^-3 + c2 s/sig^2 + c0.
    Row 1: (rc2/sig2) c2 + c0 = -(sig^12 rc2^-6 - sig^6 rc2^-3)
    Row 2: (1/sig2) c2       = 6 sig^12 rc2^-7 - 3 sig^6 rc2^-4
    """
    s6, s12 = sig2 ** 3, sig2 ** 6
    a11, a12, b1 = rc2 / sig2, Fr(1), -(s12 / rc2 ** 6 - s6 / rc2 ** 3)
    a21, a22, b2 = 1 / sig2, Fr(0), 6 * s12 / rc2 ** 7 - 3 * s6 / rc2 ** 4
    det = a11 * a22 - a12 * a21
    c2 = (b1 * a22 - a12 * b2) / det
    c0 = (a11 * b2 - a21 * b1) / det
    return c2, c0


def exact_V_g(r2: Fr, eps=Fr(1), sig2=Fr(1), rc2=Fr(25, 4)):
    c2, c0 = exact_coeffs(rc2, sig2)
    s6, s12 = sig2 ** 3, sig2 ** 6
    V = 4 * eps * (s12 / r2 ** 6 - s6 / r2 ** 3 + c2 * r2 / sig2 + c0)
    dV_ds = 4 * eps * (-6 * s12 / r2 ** 7 + 3 * s6 / r2 ** 4 + c2 / sig2)
    g = -2 * dV_ds  # -V'(r)/r = -2 dV/d(r^2)
    return V, g


def test_coefficients_exact(ref):
    c2, c0 = ref.lj_coeffs(1.0, 2.5)
    e2, e0 = exact_coeffs(Fr(25, 4))
    assert c2 == pytest.approx(float(e2), rel=1e-15)
    assert c0 == pytest.approx(float(e0), rel=1e-15)


@pytest.mark.parametrize("r2", [Fr(1), Fr(2), Fr(9, 4), Fr(4), Fr(6), Fr(81, 16), Fr(6)])
def test_pair_exact_rational(ref, r2):
    V, g = ref.pair(float(r2))
    eV, eg = exact_V_g(r2)
    assert V == pytest.approx(float(eV), rel=1e-14, abs=1e-16)
    assert g == pytest.approx(float(eg), rel=1e-14, abs=1e-16)


def test_pair_exact_rational_other_params(ref):
    eps, sig = 1.5, 1.25
    for r2 in [Fr(2), Fr(3), Fr(5)]:
        V, g = ref.pair(float(r2), eps, sig, 2.5)
        eV, eg = exact_V_g(r2, Fr(3, 2), Fr(25, 16))
        assert V == pytest.approx(float(eV), rel=1e-13)
        assert g == pytest.approx(float(eg), rel=1e-13)


def test_truncation_conditions(ref):
    # V(rc) = V'(rc) = 0 (Sec. 2.1)
    V, g = ref.pair(2.5 * 2.5)
    assert abs(V) < 1e-15 and abs(g) < 1e-15
    V, g = ref.pair(3.0 * 3.0, 0.7, 1.1, 3.0)
    assert abs(V) < 1e-15 and abs(g) < 1e-15


@pytest.mark.parametrize("r", [0.95, 1.1, 1.3, 1.7, 2.2, 2.45])
def test_g_is_minus_dVdr_over_r(ref, r):
    h = 1e-5
    Vp, _ = ref.pair((r + h) ** 2)
    Vm, _ = ref.pair((r - h) ** 2)
    _, g = ref.pair(r * r)
    dV = (Vp - Vm) / (2 * h)
    assert g == pytest.approx(-dV / r, rel=1e-7, abs=1e-9)


@pytest.mark.parametrize("r", [0.95, 1.2, 1.6, 2.3])
def test_second_derivative_and_sigma_derivative(ref, r):
    h = 1e-5
    # V'' from central differences of V' = -g r
    _, gp = ref.pair((r + h) ** 2)
    _, gm = ref.pair((r - h) ** 2)
    d2_fd = (-gp * (r + h) + gm * (r - h)) / (2 * h)
    d2V, dVs, dgs = ref.pair_derivs(r * r)
    assert d2V == pytest.approx(d2_fd, rel=1e-6, abs=1e-8)
    # dV/dsigma and dg/dsigma by central differences in sigma (c2, c0 follow sigma)
    Vp, gp = ref.pair(r * r, 1.0, 1.0 + h, 2.5)
    Vm, gm = ref.pair(r * r, 1.0, 1.0 - h, 2.5)
    assert dVs == pytest.approx((Vp - Vm) / (2 * h), rel=1e-6, abs=1e-8)
    assert dgs == pytest.approx((gp - gm) / (2 * h), rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("r", [0.9, 1.05, 1.5, 2.4])
def test_explicit_force_expression_of_the_paper(ref, r):
    # Sec. 3.2: with sigma = eps = 1, fdt = [(24 r^6 - 48)/r^14 + 8 c2] dt and
    # p[i] += fdt * (q[j] - q[i]).  Our convention F_i = -g (q_j - q_i), so the
    # bracket must equal -g.  (r^6, r^14 are powers of the distance.)
    c2, _ = ref.lj_coeffs(1.0, 2.5)
    bracket = (24 * r ** 6 - 48) / r ** 14 + 8 * c2
    _, g = ref.pair(r * r)
    assert -g == pytest.approx(bracket, rel=1e-13, abs=1e-15)


def test_untruncated_limit(ref):
    # rc -> infinity recovers 4 eps [(s/r)^12 - (s/r)^6]: minimum -eps at 2^(1/6) sigma
    rmin = 2.0 ** (1.0 / 6.0)
    V, g = ref.pair(rmin * rmin, 1.0, 1.0, 1.0e4)
    assert V == pytest.approx(-1.0, abs=1e-12)
    assert abs(g) < 1e-12
    V, _ = ref.pair(1.0, 1.0, 1.0, 1.0e4)  # V(sigma) = 0
    assert abs(V) < 1e-12


def test_scaling_law(ref):
    eps, sig, rc = 2.0, 1.3, 3.1
    for r in [1.2, 1.7, 2.9]:
        V, g = ref.pair(r * r, eps, sig, rc)
        V1, g1 = ref.pair((r / sig) ** 2, 1.0, 1.0, rc / sig)
        assert V == pytest.approx(eps * V1, rel=1e-12)
        # g = -V'/r scales as eps / sigma^2
        assert g == pytest.approx(eps * g1 / sig ** 2, rel=1e-12)


def test_derived_table(ref):
    # Values of the truncated potential at rc = 2.5 (eps = sigma = 1) that follow
    # from the closed form; reproduced here by exact rational evaluation.
    for r2 in [Fr(2), Fr(4), Fr(6)]:
        V, g = ref.pair(float(r2))
        eV, eg = exact_V_g(r2)
        assert np.isclose(V, float(eV), rtol=1e-14)
        assert np.isclose(g, float(eg), rtol=1e-14)
