"""Pins of the oracle's lattice, Hermite tensors and equilibria against what
the paper and the mathematics fix (Eqs. 1, 7-9, 26-30, 47-48, 56-64; App. B).
"""
import itertools
import json
import os

import numpy as np
import pytest
import sympy as sp

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "equilibrium_central_moments.json")
CS2 = 1.0 / 3.0
RNG = np.random.default_rng(12345)


def _states(n=12):
    out = []
    for _ in range(n):
        rho = RNG.uniform(0.05, 3.0)
        p = RNG.uniform(0.002, 1.5)
        u = RNG.uniform(-0.2, 0.2, size=3)
        out.append((rho, p, u))
    out.append((1.0, 1.0 / 3.0, np.zeros(3)))
    return out


def test_velocity_set_is_the_27_points_of_the_unit_cube():
    c, w = O.lattice()
    assert c[0].tolist() == [0, 0, 0]
    assert len({tuple(v) for v in c}) == 27
    assert set(map(tuple, c)) == set(itertools.product((-1, 0, 1), repeat=3))
    # opposite pairs (2k-1, 2k) in the order printed in Eq. (1)
    for k in range(1, 14):
        assert (c[2 * k - 1] == -c[2 * k]).all()


def test_weights_are_tensor_products_of_d1q3():
    c, w = O.lattice()
    w1 = {0: 2.0 / 3.0, 1: 1.0 / 6.0, -1: 1.0 / 6.0}
    for i in range(27):
        assert w[i] == pytest.approx(w1[c[i, 0]] * w1[c[i, 1]] * w1[c[i, 2]], rel=1e-15)


def test_lattice_isotropy_to_sixth_order():
    c, w = O.lattice()
    cx, cy, cz = c[:, 0], c[:, 1], c[:, 2]
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert (w * cx * cx).sum() == pytest.approx(CS2, abs=1e-15)
    assert (w * cx * cy).sum() == pytest.approx(0.0, abs=1e-16)
    assert (w * cx ** 4).sum() == pytest.approx(CS2, abs=1e-15)
    assert (w * cx ** 2 * cy ** 2).sum() == pytest.approx(CS2 ** 2, abs=1e-15)
    assert (w * cx ** 2 * cy ** 2 * cz ** 2).sum() == pytest.approx(CS2 ** 3, abs=1e-15)
    for a, b, cc in itertools.product(range(4), repeat=3):
        if (a % 2) or (b % 2) or (cc % 2):
            assert abs((w * cx ** a * cy ** b * cz ** cc).sum()) < 1e-16


def test_hermite_orthogonality():
    """sum_i w_i H_a H_b = delta_ab * prod over axes of (1, cs2, 2 cs2^2)."""
    c, w = O.lattice()
    idx = list(itertools.product(range(3), repeat=3))
    norm1 = {0: 1.0, 1: CS2, 2: 2.0 * CS2 ** 2}
    for A in idx:
        HA = np.array([O.hermite(i, *A) for i in range(27)])
        for B in idx:
            HB = np.array([O.hermite(i, *B) for i in range(27)])
            g = (w * HA * HB).sum()
            exp = norm1[A[0]] * norm1[A[1]] * norm1[A[2]] if A == B else 0.0
            assert g == pytest.approx(exp, abs=1e-15)


def test_isotropic_operator_closed_form():
    """E_i of Eq. (29) reduces to (w_i - delta_i0)/c_s^2."""
    c, w = O.lattice()
    E = O.isotropic_E()
    delta = np.zeros(27)
    delta[0] = 1.0
    np.testing.assert_allclose(E, (w - delta) / CS2, rtol=0, atol=1e-14)


def test_sixth_order_equilibrium_is_product_of_d1q3_equilibria():
    """g^{eq,6} (Eq. 27) equals rho * prod_axes w(c)[1 + c u/cs2 + (c^2-cs2)u^2/(2cs2^2)],
    the tensor product of the complete one-dimensional Hermite equilibria."""
    c, w = O.lattice()
    for rho, _, u in _states():
        p = rho * CS2                       # removes the (p - rho cs2) part of Eq. 28
        fe = O.feq(O.MODEL_B, rho, p, u)
        prod = np.full(27, rho)
        for a in range(3):
            ca = c[:, a].astype(float)
            wa = np.where(ca == 0, 2.0 / 3.0, 1.0 / 6.0)
            prod *= wa * (1 + ca * u[a] / CS2 + (ca * ca - CS2) * u[a] ** 2 / (2 * CS2 ** 2))
        np.testing.assert_allclose(fe, prod, rtol=1e-13, atol=1e-16)


def test_model_a_equals_standard_cg_equilibrium():
    """Eq. (31): Model A is the standard colour-gradient equilibrium Eqs. (7)-(8)."""
    for rho, p, u in _states():
        np.testing.assert_allclose(O.feq(O.MODEL_A, rho, p, u), O.feq_standard_cg(rho, p, u),
                                   rtol=1e-12, atol=1e-15)


def test_li_original_equals_general_form_with_second_order_g():
    """Eq. (48): the original equilibrium of Eq. (47) is g^{eq,2} + (p - rho cs2)(E + Phi3).
    Model C replaces g^{eq,2} by g^{eq,6}; the difference is g^{eq,6} - g^{eq,2},
    which Model B minus Model A isolates."""
    for rho, p, u in _states():
        li = O.feq_li_original(rho, p, u)
        g6_minus_g2 = O.feq(O.MODEL_B, rho, p, u) - O.feq(O.MODEL_A, rho, p, u)
        np.testing.assert_allclose(O.feq(O.MODEL_C, rho, p, u) - g6_minus_g2, li,
                                   rtol=1e-12, atol=1e-15)


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.mark.parametrize("model,key", [(O.MODEL_A, "model_A"), (O.MODEL_B, "model_B"),
                                       (O.MODEL_C, "model_C"), (O.MODEL_D, "model_D")])
def test_equilibrium_central_moments_match_printed_tables(model, key):
    """Brute-force central moments (Eq. 30) of the phase-space equilibria equal
    the printed tables of Eqs. (32)-(38), (40)-(46), (49)-(55), (57)-(63)."""
    table = _golden()[key]
    syms = sp.symbols("rho p ux uy uz cs2")
    exprs = {}
    for a, b, cc in itertools.product(range(3), repeat=3):
        name = "k%d%d%d" % (a, b, cc)
        exprs[(a, b, cc)] = sp.lambdify(syms, sp.sympify(table.get(name, "0")))
    for rho, p, u in _states():
        k = O.central_moments(O.feq(model, rho, p, u), u)
        for (a, b, cc), fn in exprs.items():
            exp = fn(rho, p, u[0], u[1], u[2], CS2)
            got = k[a + 3 * b + 9 * cc]
            assert got == pytest.approx(exp, rel=1e-11, abs=1e-14), (key, a, b, cc)


def test_model_d_central_moments_are_velocity_independent():
    rho, p = 0.9, 0.12
    k0 = O.central_moments(O.feq(O.MODEL_D, rho, p, np.zeros(3)), np.zeros(3))
    for _, _, u in _states():
        np.testing.assert_allclose(O.central_moments(O.feq(O.MODEL_D, rho, p, u), u), k0,
                                   rtol=0, atol=1e-14)


def test_model_d_third_order_raw_moments():
    """Eq. (64): third-order raw moments of the generalized equilibrium."""
    table = _golden()["model_D_third_raw"]
    syms = sp.symbols("rho p ux uy uz cs2")
    for rho, p, u in _states():
        m = O.raw_moments(O.feq(O.MODEL_D, rho, p, u))
        for name, ex in table.items():
            if not name.startswith("m"):
                continue
            a, b, cc = int(name[1]), int(name[2]), int(name[3])
            exp = float(sp.sympify(ex).subs(dict(zip(syms, (rho, p, u[0], u[1], u[2], CS2)))))
            assert m[a + 3 * b + 9 * cc] == pytest.approx(exp, rel=1e-11, abs=1e-15)
        # diagonal triple: sum f c_x^3 = sum f c_x = rho u_x (= rho cs2 * 3 u_x)
        assert m[1] == pytest.approx(rho * u[0], rel=1e-12, abs=1e-15)


def test_equilibria_conserve_mass_and_momentum_and_give_pressure():
    for model in range(4):
        for rho, p, u in _states():
            m = O.raw_moments(O.feq(model, rho, p, u))
            assert m[0] == pytest.approx(rho, rel=1e-13)
            assert m[1] == pytest.approx(rho * u[0], rel=1e-12, abs=1e-15)
            assert m[3] == pytest.approx(rho * u[1], rel=1e-12, abs=1e-15)
            assert m[9] == pytest.approx(rho * u[2], rel=1e-12, abs=1e-15)
            # second order: p delta + rho u u
            assert m[2] == pytest.approx(p + rho * u[0] ** 2, rel=1e-12)
            assert m[4] == pytest.approx(rho * u[0] * u[1], rel=1e-11, abs=1e-15)


def test_sound_speed_relation_table_iii():
    """Eq. (13) with xi = 9/19 reproduces the rest fractions of Table III:
    density ratio rho_r0/rho_b0 = (1 - alpha_b)/(1 - alpha_r)."""
    cases = {"A": (0.1, 0.8, 0.9), "B": (0.8, 0.1, 0.2), "C": (0.008, 8.0, 0.9992)}
    for rr, rb, ab in cases.values():
        ar = 1.0 - (1.0 - ab) * rb / rr
        assert rr / rb == pytest.approx(O.sound_speed2(ab) / O.sound_speed2(ar), rel=1e-12)
        # equal pure-phase pressures
        assert rr * O.sound_speed2(ar) == pytest.approx(rb * O.sound_speed2(ab), rel=1e-12)
    # alpha = 8/27 gives the lattice sound speed c_s^2 = 1/3 (Sec. IV.D)
    assert O.sound_speed2(8.0 / 27.0) == pytest.approx(1.0 / 3.0, rel=1e-15)


def test_symbolic_model_d_from_paper_formula():
    """Exact rational check: Eq. (56) assembled symbolically from App. B has the
    velocity-independent central moments of Eqs. (57)-(63).  This pins the
    reading of the printed formula that the oracle implements; the oracle's
    numeric values are pinned to the same table above."""
    rho, p, ux, uy, uz = sp.symbols("rho p u_x u_y u_z")
    cs2 = sp.Rational(1, 3)
    c, w = O.lattice()
    u = (ux, uy, uz)

    def h(order, ci):
        return [1, ci, ci * ci - cs2][order]

    def H(i, a, b, cc):
        return h(a, int(c[i, 0])) * h(b, int(c[i, 1])) * h(cc, int(c[i, 2]))

    wr = [sp.Rational(8, 27) if (abs(c[i]).sum() == 0) else
          sp.Rational(2, 27) if abs(c[i]).sum() == 1 else
          sp.Rational(1, 54) if abs(c[i]).sum() == 2 else sp.Rational(1, 216) for i in range(27)]
    feq = []
    for i in range(27):
        g6 = 1
        for (a, b, cc) in itertools.product(range(3), repeat=3):
            if (a, b, cc) == (0, 0, 0):
                continue
            coef = sp.Integer(1) / (sp.factorial(a) * sp.factorial(b) * sp.factorial(cc)
                                    * cs2 ** (a + b + cc))
            g6 += coef * ux ** a * uy ** b * uz ** cc * H(i, a, b, cc)
        E = ((H(i, 2, 0, 0) + H(i, 0, 2, 0) + H(i, 0, 0, 2)) / (2 * cs2 ** 2)
             - (H(i, 2, 2, 0) + H(i, 0, 2, 2) + H(i, 2, 0, 2)) / (4 * cs2 ** 3)
             + H(i, 2, 2, 2) / (8 * cs2 ** 4))
        phi = ((ux * (H(i, 1, 2, 0) + H(i, 1, 0, 2)) + uy * (H(i, 2, 1, 0) + H(i, 0, 1, 2))
                + uz * (H(i, 2, 0, 1) + H(i, 0, 2, 1))) / (2 * cs2 ** 3)
               + ((ux ** 2 + uy ** 2) * H(i, 2, 2, 0) + (uy ** 2 + uz ** 2) * H(i, 0, 2, 2)
                  + (ux ** 2 + uz ** 2) * H(i, 2, 0, 2)
                  + 2 * (uy * uz * H(i, 2, 1, 1) + ux * uz * H(i, 1, 2, 1) + ux * uy * H(i, 1, 1, 2)))
               / (4 * cs2 ** 4)
               + (ux * (uy ** 2 + uz ** 2 - cs2) * H(i, 1, 2, 2)
                  + uy * (ux ** 2 + uz ** 2 - cs2) * H(i, 2, 1, 2)
                  + uz * (ux ** 2 + uy ** 2 - cs2) * H(i, 2, 2, 1)) / (4 * cs2 ** 5)
               + (ux ** 2 * uy ** 2 + uy ** 2 * uz ** 2 + ux ** 2 * uz ** 2
                  - cs2 * (ux ** 2 + uy ** 2 + uz ** 2)) * H(i, 2, 2, 2) / (8 * cs2 ** 6))
        feq.append(rho * wr[i] * g6 + (p - rho * cs2) * wr[i] * (E + phi))
    expected = {(0, 0, 0): rho, (2, 0, 0): p, (0, 2, 0): p, (0, 0, 2): p,
                (2, 2, 0): p * cs2, (2, 0, 2): p * cs2, (0, 2, 2): p * cs2, (2, 2, 2): p * cs2 ** 2}
    for (a, b, cc) in itertools.product(range(3), repeat=3):
        k = sum(feq[i] * (int(c[i, 0]) - ux) ** a * (int(c[i, 1]) - uy) ** b
                * (int(c[i, 2]) - uz) ** cc for i in range(27))
        assert sp.expand(k - expected.get((a, b, cc), 0)) == 0, (a, b, cc)
