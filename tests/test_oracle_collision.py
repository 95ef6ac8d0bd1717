"""Pins of the oracle's moment transforms, collision and recolouring
(Sec. II.B Eqs. 23-25; Sec. III.E Eqs. 66-67; Sec. II.A Eqs. 6, 18-19)."""
import itertools

import numpy as np
import pytest

import oracle as O

CS2 = 1.0 / 3.0
RNG = np.random.default_rng(2024)


def mi(a, b, c):
    return a + 3 * b + 9 * c


def _random_population(rho=1.0, amp=0.02, u=None):
    u = np.zeros(3) if u is None else np.asarray(u)
    p = rho * CS2 * RNG.uniform(0.3, 1.2)
    return O.feq(O.MODEL_D, rho, p, u) + RNG.uniform(-amp, amp, 27) * rho, p


def test_raw_moment_matrix_inverse():
    M = O.moment_matrix()
    Mi = O.inverse_moment_matrix()
    np.testing.assert_allclose(M @ Mi, np.eye(27), atol=1e-14)
    np.testing.assert_allclose(Mi @ M, np.eye(27), atol=1e-14)


def test_round_trip_central_moments():
    for _ in range(20):
        f, _ = _random_population(RNG.uniform(0.1, 2.0))
        u = RNG.uniform(-0.15, 0.15, 3)
        k = O.central_moments(f, u)
        np.testing.assert_allclose(O.cm_to_f(k, u), f, rtol=0, atol=2e-14 * np.abs(f).max())


def test_central_moments_of_raw_shift_agree():
    """k_abc by definition (Eq. 24) equals the binomial expansion of raw moments."""
    from math import comb
    for _ in range(10):
        f, _ = _random_population()
        u = RNG.uniform(-0.2, 0.2, 3)
        m = O.raw_moments(f)
        k = O.central_moments(f, u)
        for a, b, c in itertools.product(range(3), repeat=3):
            s = 0.0
            for a2, b2, c2 in itertools.product(range(a + 1), range(b + 1), range(c + 1)):
                s += (comb(a, a2) * comb(b, b2) * comb(c, c2) * (-u[0]) ** (a - a2)
                      * (-u[1]) ** (b - b2) * (-u[2]) ** (c - c2) * m[mi(a2, b2, c2)])
            assert k[mi(a, b, c)] == pytest.approx(s, abs=1e-14)


@pytest.mark.parametrize("model", [O.MODEL_A, O.MODEL_B, O.MODEL_C, O.MODEL_D])
def test_equal_rates_reduce_to_bgk(model):
    """All rates equal, no force, no Q: the CM-MRT of Eq. (25) is the BGK
    operator of Eq. (6) with the same equilibrium."""
    for omega in (0.6, 1.0, 1.7):
        f, p = _random_population(RNG.uniform(0.5, 1.5), u=RNG.uniform(-0.1, 0.1, 3))
        rho = f.sum()
        c, _ = O.lattice()
        u = (f[:, None] * c).sum(0) / rho
        fs = O.collide(model, 1, f, rho, u, p, np.zeros(3), np.zeros(3), [omega] * 11)
        fe = O.feq(model, rho, p, u)
        np.testing.assert_allclose(fs, f - omega * (f - fe), rtol=0, atol=1e-14)


def test_equilibrium_is_a_fixed_point_of_collision():
    for model in range(4):
        rho, p, u = 1.2, 0.25, np.array([0.05, -0.03, 0.02])
        fe = O.feq(model, rho, p, u)
        omega = [1.0, 1.3, 0.8, 1.1, 1.2, 1.0, 0.9, 1.0, 1.4, 1.0, 1.0]
        fs = O.collide(model, 1, fe, rho, u, p, np.zeros(3), np.zeros(3), omega)
        np.testing.assert_allclose(fs, fe, rtol=0, atol=1e-14)


def test_unit_rates_model_d_compact_collision():
    """Eqs. (66)-(67): with omega_0 = omega_2..omega_10 = 1 and Model D, the
    post-collision central moments are fixed by F, p, Q and the six
    second-order pre-collision moments."""
    c, _ = O.lattice()
    for _ in range(10):
        f, p = _random_population(RNG.uniform(0.5, 1.5), amp=0.03,
                                  u=RNG.uniform(-0.1, 0.1, 3))
        rho = f.sum()
        F = RNG.uniform(-1e-3, 1e-3, 3)
        Q = RNG.uniform(-1e-3, 1e-3, 3)
        w1 = RNG.uniform(0.5, 1.9)
        u = ((f[:, None] * c).sum(0) + F / 2) / rho       # Eq. (11)
        omega = [1.0] * 11
        omega[1] = w1
        fs = O.collide(O.MODEL_D, 1, f, rho, u, p, F, Q, omega)
        k = O.central_moments(f, u)
        ks = O.central_moments(fs, u)
        tol = dict(abs=2e-14)
        assert ks[mi(0, 0, 0)] == pytest.approx(rho, **tol)
        for a, (i, j, l) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
            assert ks[mi(i, j, l)] == pytest.approx(F[a] / 2, **tol)
        for idx in ((1, 1, 0), (0, 1, 1), (1, 0, 1)):
            assert ks[mi(*idx)] == pytest.approx((1 - w1) * k[mi(*idx)], **tol)
        kxx, kyy, kzz = k[mi(2, 0, 0)], k[mi(0, 2, 0)], k[mi(0, 0, 2)]
        sxx, syy, szz = ks[mi(2, 0, 0)], ks[mi(0, 2, 0)], ks[mi(0, 0, 2)]
        assert sxx - syy == pytest.approx((1 - w1) * (kxx - kyy) + (1 - w1 / 2) * (Q[0] - Q[1]), **tol)
        assert sxx - szz == pytest.approx((1 - w1) * (kxx - kzz) + (1 - w1 / 2) * (Q[0] - Q[2]), **tol)
        assert sxx + syy + szz == pytest.approx(3 * p + Q.sum() / 2, **tol)
        for a, pair in enumerate((((1, 2, 0), (1, 0, 2)), ((2, 1, 0), (0, 1, 2)),
                                  ((2, 0, 1), (0, 2, 1)))):
            for idx in pair:
                assert ks[mi(*idx)] == pytest.approx(CS2 * F[a] / 2, **tol)
        assert ks[mi(1, 1, 1)] == pytest.approx(0.0, **tol)
        for idx in ((2, 2, 0), (2, 0, 2), (0, 2, 2)):
            assert ks[mi(*idx)] == pytest.approx(p * CS2, **tol)
        for idx in ((2, 1, 1), (1, 2, 1), (1, 1, 2)):
            assert ks[mi(*idx)] == pytest.approx(0.0, **tol)
        for a, idx in enumerate(((1, 2, 2), (2, 1, 2), (2, 2, 1))):
            assert ks[mi(*idx)] == pytest.approx(CS2 * CS2 * F[a] / 2, **tol)
        assert ks[mi(2, 2, 2)] == pytest.approx(p * CS2 * CS2, **tol)


def test_general_rates_relax_each_combination():
    """Eq. (25) with distinct rates: every relaxed combination obeys its own
    printed relation after the combinations are solved back."""
    c, _ = O.lattice()
    f, p = _random_population(1.1, amp=0.03, u=[0.04, 0.02, -0.05])
    rho = f.sum()
    F = np.array([2e-3, -1e-3, 5e-4])
    Q = np.array([1e-3, 4e-4, -7e-4])
    om = [0.7, 1.3, 0.9, 1.1, 1.6, 0.8, 1.2, 0.6, 1.4, 1.5, 0.5]
    u = ((f[:, None] * c).sum(0) + F / 2) / rho
    for model in range(4):
        fs = O.collide(model, 1, f, rho, u, p, F, Q, om)
        k, ks = O.central_moments(f, u), O.central_moments(fs, u)
        ke = O.central_moments(O.feq(model, rho, p, u), u)
        t = dict(abs=2e-14)
        K = lambda arr, s: arr[mi(*s)]
        assert K(ks, (1, 0, 0)) == pytest.approx((1 - om[0]) * K(k, (1, 0, 0)) + (1 - om[0] / 2) * F[0], **t)
        T = lambda arr: K(arr, (2, 0, 0)) + K(arr, (0, 2, 0)) + K(arr, (0, 0, 2))
        assert T(ks) == pytest.approx((1 - om[2]) * T(k) + om[2] * T(ke) + (1 - om[2] / 2) * Q.sum(), **t)
        S = lambda arr: K(arr, (1, 2, 0)) + K(arr, (1, 0, 2))
        D = lambda arr: K(arr, (1, 2, 0)) - K(arr, (1, 0, 2))
        assert S(ks) == pytest.approx((1 - om[3]) * S(k) + om[3] * S(ke) + 2 * (1 - om[3] / 2) * F[0] * CS2, **t)
        assert D(ks) == pytest.approx((1 - om[4]) * D(k) + om[4] * D(ke), **t)
        assert K(ks, (1, 1, 1)) == pytest.approx((1 - om[5]) * K(k, (1, 1, 1)) + om[5] * K(ke, (1, 1, 1)), **t)
        X = lambda arr: K(arr, (2, 2, 0)) - 2 * K(arr, (2, 0, 2)) + K(arr, (0, 2, 2))
        Z = lambda arr: K(arr, (2, 2, 0)) + K(arr, (2, 0, 2)) + K(arr, (0, 2, 2))
        assert X(ks) == pytest.approx((1 - om[6]) * X(k) + om[6] * X(ke), **t)
        assert Z(ks) == pytest.approx((1 - om[7]) * Z(k) + om[7] * Z(ke), **t)
        assert K(ks, (2, 1, 1)) == pytest.approx((1 - om[8]) * K(k, (2, 1, 1)) + om[8] * K(ke, (2, 1, 1)), **t)
        assert K(ks, (1, 2, 2)) == pytest.approx((1 - om[9]) * K(k, (1, 2, 2)) + om[9] * K(ke, (1, 2, 2))
                                                 + (1 - om[9] / 2) * F[0] * CS2 ** 2, **t)
        assert K(ks, (2, 2, 2)) == pytest.approx((1 - om[10]) * K(k, (2, 2, 2)) + om[10] * K(ke, (2, 2, 2)), **t)


def test_recolouring_conserves_colour_mass_and_shifts_red_momentum_by_R():
    """Eqs. (18)-(19): sum_i f^{k*}_i = rho_k; f^r* + f^b* = f*; the red
    momentum changes by exactly R (isotropy sum_i w_i c_i c_i = c_s^2 I)."""
    c, _ = O.lattice()
    for _ in range(10):
        fs, p = _random_population(1.0, amp=0.01)
        rho = fs.sum()
        frac = RNG.uniform(0.0, 1.0)
        rr, rb = frac * rho, (1 - frac) * rho
        n = RNG.normal(size=3)
        n /= np.linalg.norm(n)
        beta = 0.7
        fr, fb = O.recolour(fs, rr, rb, p, n, beta)
        assert fr.sum() == pytest.approx(rr, abs=1e-15)
        assert fb.sum() == pytest.approx(rb, abs=1e-15)
        np.testing.assert_allclose(fr + fb, fs, atol=1e-16)
        R = beta * rr * rb / rho ** 2 * p * n
        jr = (fr[:, None] * c).sum(0)
        np.testing.assert_allclose(jr, rr / rho * (fs[:, None] * c).sum(0) + R, atol=1e-16)


def test_pure_phase_recolouring_is_identity():
    fs, p = _random_population(1.0)
    fr, fb = O.recolour(fs, fs.sum(), 0.0, p, [1.0, 0.0, 0.0], 0.7)
    np.testing.assert_allclose(fr, fs, atol=0)
    np.testing.assert_allclose(fb, 0.0, atol=0)


def test_splitmix64_counter_noise_is_uniform_and_bounded():
    vals = np.array([O.noise(7, 0, n, i, 1.0) for n in range(400) for i in range(27)])
    assert np.all(np.abs(vals) <= 1.0)
    assert abs(vals.mean()) < 0.03
    assert vals.std() == pytest.approx(1 / np.sqrt(3), rel=0.03)
    assert len(np.unique(vals)) > 0.99 * len(vals)
