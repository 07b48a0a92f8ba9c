"""Pins of the oracle's quadrature (no GPU).

* 6-point Dunavant rule: exact for every monomial of degree <= 4 in the
  barycentric coordinates (closed form a! b! c! 2|T| / (a+b+c+2)!), and its
  nodes solve the moment equations (re-derived here by Newton's method).
* Gauss-Legendre on [0,1]: exact to degree 7 for 4 points.
* Singular rules: weight sum |K|^2, polynomial exactness, and convergence to
  the closed-form Laplace potential of a flat triangle integrated by a
  high-order outer rule (coincident, common edge, common vertex).
"""
from math import factorial

import numpy as np
import pytest

from oracle import quadrature as Q
from oracle.operators import pair_kernel_integral
from tests._laplace_analytic import triangle_potential, triangle_rule


def test_dunavant_degree4_exact():
    bary, w = Q.dunavant6()
    assert abs(w.sum() - 1.0) < 1e-15
    for a in range(5):
        for b in range(5 - a):
            for c in range(5 - a - b):
                exact = 2.0 * factorial(a) * factorial(b) * factorial(c) / \
                    factorial(a + b + c + 2)
                q = np.sum(w * bary[:, 0] ** a * bary[:, 1] ** b *
                           bary[:, 2] ** c)
                assert abs(q - exact) < 1e-15, (a, b, c)
    # degree 5 is not integrated exactly (the rule is of degree 4 only)
    q5 = np.sum(w * bary[:, 0] ** 5)
    assert abs(q5 - 2.0 * factorial(5) / factorial(7)) > 1e-6


def test_dunavant_nodes_solve_moment_equations():
    # unknowns (a1, w1, a2, w2); orbits (1-2a, a, a): moments of x^2, x^3, x^4
    # of lambda_0 plus the weight sum must match the exact integrals.
    def F(u):
        a1, w1, a2, w2 = u
        out = [3.0 * (w1 + w2) - 1.0]
        for p in (2, 3, 4):
            exact = 2.0 * factorial(p) / factorial(p + 2)
            s = sum(w * ((1 - 2 * a) ** p + 2 * a ** p)
                    for a, w in ((a1, w1), (a2, w2)))
            out.append(s - exact)
        return np.array(out)

    u = np.array([0.44, 0.22, 0.09, 0.11])
    for _ in range(50):
        J = np.zeros((4, 4))
        f0 = F(u)
        for i in range(4):
            du = np.zeros(4)
            du[i] = 1e-7
            J[:, i] = (F(u + du) - f0) / 1e-7
        u = u - np.linalg.solve(J, f0)
    assert abs(u[0] - Q._DUN_A1) < 1e-13
    assert abs(u[2] - Q._DUN_A2) < 1e-13
    # weights here are per point with sum over 3 points of each orbit = 1
    assert abs(u[1] - Q._DUN_W1) < 1e-13
    assert abs(u[3] - Q._DUN_W2) < 1e-13


def test_gauss01_degree7():
    t, w = Q.gauss01(4)
    for p in range(8):
        assert abs(np.sum(w * t ** p) - 1.0 / (p + 1)) < 1e-15
    assert abs(np.sum(w * t ** 8) - 1.0 / 9) > 1e-8


def _IK(a, b):
    # int_K x1^a x2^b over K = {0 <= x2 <= x1 <= 1}
    return 1.0 / ((b + 1) * (a + b + 2))


@pytest.mark.parametrize("rule", [Q.rule_coincident, Q.rule_edge,
                                  Q.rule_vertex])
def test_singular_rule_weights_and_polynomials(rule):
    r = rule(4)
    assert abs(r[:, 4].sum() - 0.25) < 1e-15
    assert np.all(r[:, 1] <= r[:, 0] + 1e-15) and np.all(r[:, 3] <= r[:, 2] + 1e-15)
    assert r[:, :4].min() >= 0.0 and r[:, :4].max() <= 1.0
    for a in range(3):
        for b in range(3 - a):
            for c in range(3):
                for d in range(3 - c):
                    q = np.sum(r[:, 0] ** a * r[:, 1] ** b * r[:, 2] ** c *
                               r[:, 3] ** d * r[:, 4])
                    assert abs(q - _IK(a, b) * _IK(c, d)) < 1e-15


def test_region_counts():
    assert Q.rule_coincident(4).shape[0] == 6 * 256
    assert Q.rule_edge(4).shape[0] == 4 * 256
    assert Q.rule_vertex(4).shape[0] == 2 * 256


_A = np.array([0.0, 0.0, 0.0])
_B = np.array([1.0, 0.0, 0.0])
_C = np.array([0.3, 0.8, 0.0])
_TAU = np.array([_A, _B, _C])


def _reference(tau, sig):
    p, w = triangle_rule(tau, 60)
    return sum(wi * triangle_potential(sig, pi) for pi, wi in zip(p, w))


CASES = {
    # which, sigma, px, py
    "coincident": (0, _TAU, [0, 1, 2], [0, 1, 2]),
    "edge": (1, np.array([_B, _A, [0.6, -0.5, 0.4]]), [0, 1, 2], [1, 0, 2]),
    "edge_coplanar": (1, np.array([_B, _A, [0.5, -0.7, 0.0]]), [0, 1, 2],
                      [1, 0, 2]),
    "vertex": (2, np.array([_A, [-0.5, 0.2, 0.6], [-0.7, -0.4, 0.1]]),
               [0, 1, 2], [0, 1, 2]),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_singular_rules_match_closed_form_laplace(oracle_lib, case):
    which, sig, px, py = CASES[case]
    ref = _reference(_TAU, sig)
    i4 = pair_kernel_integral(_TAU, sig, which, px, py, 0.0, 1, n_ss=4).real
    i8 = pair_kernel_integral(_TAU, sig, which, px, py, 0.0, 1, n_ss=8).real
    i12 = pair_kernel_integral(_TAU, sig, which, px, py, 0.0, 1, n_ss=12).real
    assert abs(i4 - ref) / ref < 2e-5
    assert abs(i8 - ref) / ref < 5e-7     # reference outer-rule accuracy
    assert abs(i12 - i8) / ref < 1e-8     # self-convergence
    assert abs(i12 - ref) < abs(i4 - ref) + 1e-12


def test_singular_rules_kernel_one_gives_area_product(oracle_lib):
    for case, (which, sig, px, py) in CASES.items():
        v = pair_kernel_integral(_TAU, sig, which, px, py, 0.0, 0, n_ss=4)
        at = 0.5 * np.linalg.norm(np.cross(_TAU[1] - _TAU[0], _TAU[2] - _TAU[0]))
        asg = 0.5 * np.linalg.norm(np.cross(sig[1] - sig[0], sig[2] - sig[0]))
        assert abs(v - at * asg) < 1e-14, case


def test_helmholtz_singular_self_convergence(oracle_lib):
    # exp(ikr)/r = 1/r + smooth: the rules converge for k != 0 too.  Errors
    # are scaled by the Laplace integral (the size of |integrand|).
    for case, (which, sig, px, py) in CASES.items():
        k = 3.0 + 0.5j
        scale = pair_kernel_integral(_TAU, sig, which, px, py, 0.0, 1, 4).real
        i4 = pair_kernel_integral(_TAU, sig, which, px, py, k, 1, n_ss=4)
        i8 = pair_kernel_integral(_TAU, sig, which, px, py, k, 1, n_ss=8)
        i16 = pair_kernel_integral(_TAU, sig, which, px, py, k, 1, n_ss=16)
        assert abs(i8 - i16) < abs(i4 - i16)
        assert abs(i4 - i16) / scale < 3e-4, case
        assert abs(i8 - i16) / scale < 5e-9, case
