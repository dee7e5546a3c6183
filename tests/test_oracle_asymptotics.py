"""Pins for the oracle's asymptotic functions at r = a.

Open channels use the Coulomb functions F_l(eta, rho), G_l(eta, rho) (the paper's
asymptotic form for a charged target, section "Overview"); closed channels use the
exponentially decaying Whittaker function (Glossary, "Closed")."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special

import oracle


def _mp_coulomb(l, eta, rho):
    mp.mp.dps = 30
    F = mp.coulombf(l, eta, rho)
    G = mp.coulombg(l, eta, rho)
    Fp = mp.diff(lambda x: mp.coulombf(l, eta, x), rho)
    Gp = mp.diff(lambda x: mp.coulombg(l, eta, x), rho)
    return np.array([float(F), float(Fp), float(G), float(Gp)])


def test_wronskian_sample():
    rng = np.random.default_rng(11)
    for _ in range(300):
        eps = 10 ** rng.uniform(-6.5, 1.0)
        z = rng.choice([0.0, 1.0, 2.0, 5.0, 10.0])
        a = rng.uniform(5, 20)
        l = int(rng.integers(0, 16))
        k = math.sqrt(eps)
        F, Fp, G, Gp = oracle.coulomb(-z / k, k * a, l)
        assert abs(Fp * G - F * Gp - 1.0) < 1e-13


@pytest.mark.parametrize("l", [0, 1, 2, 5, 9, 12])
def test_neutral_is_riccati_bessel(l):
    for rho in [0.05, 0.7, 3.0, 11.0, 37.0]:
        F, Fp, G, Gp = oracle.coulomb(0.0, rho, l)
        jl, jlp = special.spherical_jn(l, rho), special.spherical_jn(l, rho, derivative=True)
        yl, ylp = special.spherical_yn(l, rho), special.spherical_yn(l, rho, derivative=True)
        ref = np.array([rho * jl, jl + rho * jlp, -rho * yl, -(yl + rho * ylp)])
        got = np.array([F, Fp, G, Gp])
        assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_neutral_s_wave_sin_cos():
    for rho in [0.01, 0.5, 2.0, 9.0, 33.0]:
        np.testing.assert_allclose(oracle.coulomb(0.0, rho, 0),
                                   [math.sin(rho), math.cos(rho), math.cos(rho), -math.sin(rho)],
                                   rtol=1e-14, atol=1e-15)


def _coulomb_cases(n, seed):
    rng = np.random.default_rng(seed)
    cases = [(-3000.0, 0.02, 0), (-4454.5, 0.0135, 4), (-515.8, 0.116, 12), (-3001.4, 0.0199, 11),
             (-11.18, 5.367, 12), (-1.0, 40.0, 0), (0.0, 0.3, 3), (-2.0, 30.0, 3)]
    for _ in range(n):
        z = rng.choice([2.0, 5.0])
        a = rng.choice([10.0, 12.0])
        eps = 10 ** rng.uniform(-6, math.log10(8))
        k = math.sqrt(eps)
        cases.append((-z / k, k * a, int(rng.integers(0, 13))))
    return cases


@pytest.mark.parametrize("case", _coulomb_cases(40, 5))
def test_coulomb_vs_mpmath(case):
    eta, rho, l = case
    got = oracle.coulomb(eta, rho, l)
    ref = _mp_coulomb(l, eta, rho)
    scale = np.sqrt(np.sum(ref ** 2))
    assert np.max(np.abs(got - ref)) <= 2e-14 * scale, (got, ref)


def test_coulomb_l_recurrence():
    # DLMF 33.4: R_L u_{L-1} - S_L u_L = u'_L with R_L = sqrt(1+eta^2/L^2), S_L = L/rho + eta/L
    for eta, rho in [(-20.0, 1.5), (-3.0, 8.0), (-200.0, 0.3)]:
        for L in range(1, 10):
            Fm = oracle.coulomb(eta, rho, L - 1)
            F = oracle.coulomb(eta, rho, L)
            RL = math.sqrt(1 + eta * eta / (L * L))
            SL = L / rho + eta / L
            for u_m, u, up in [(Fm[0], F[0], F[1]), (Fm[2], F[2], F[3])]:
                assert abs(RL * u_m - SL * u - up) <= 1e-12 * (abs(RL * u_m) + abs(SL * u) + abs(up))


# ---------------- closed channels ----------------

def test_closed_neutral_s_wave():
    for kap in [0.1, 0.7, 2.5]:
        for r in [3.0, 12.0]:
            assert abs(oracle.closed_logderiv(0.0, -kap * kap, r, 0) + kap) < 1e-14 * max(1, kap)


@pytest.mark.parametrize("l", [0, 1, 3, 6])
def test_closed_neutral_modified_bessel(l):
    # W_{0,l+1/2}(2 kappa r) is proportional to sqrt(r) K_{l+1/2}(kappa r)
    for kap in [0.3, 1.1]:
        for r in [2.0, 10.0]:
            x = kap * r
            ref = 0.5 / r + kap * special.kvp(l + 0.5, x) / special.kv(l + 0.5, x)
            assert abs(oracle.closed_logderiv(0.0, -kap * kap, r, l) - ref) <= 1e-13 * max(1, abs(ref))


@pytest.mark.parametrize("nu,l", [(1, 0), (2, 0), (2, 1), (3, 1), (5, 2), (8, 3), (12, 7), (30, 12)])
def test_closed_hydrogenic(nu, l):
    # integer nu = n >= l+1: W_{n,l+1/2}(x) = (-1)^{n_r} n_r! x^{l+1} e^{-x/2} L_{n_r}^{(2l+1)}(x)
    # Radii are those of the workloads (a >= 10).  Deep inside the centrifugal
    # barrier at an exactly integer nu the decaying solution is the regular one,
    # and inward integration amplifies rounding (about 7e6 x unit roundoff at
    # l = 12, r = 12; far more at r <= 4), so such radii are not pinned here.
    z = 5.0
    kap = z / nu
    nr = nu - l - 1
    for r in [10.0, 12.0, 20.0, 30.0]:
        x = 2 * kap * r
        Lg = special.eval_genlaguerre(nr, 2 * l + 1, x)
        dLg = -special.eval_genlaguerre(nr - 1, 2 * l + 2, x) if nr > 0 else 0.0
        ref = 2 * kap * ((l + 1) / x - 0.5 + dLg / Lg)
        got = oracle.closed_logderiv(z, -kap * kap, r, l)
        # compare the normalised directions (handles zeros of W)
        d1 = np.array([1.0, got]) / math.hypot(1, r * got)
        d2 = np.array([1.0, ref]) / math.hypot(1, r * ref)
        assert np.max(np.abs(d1 - d2) * [1, r]) < 1e-11


def _closed_cases(n, seed):
    rng = np.random.default_rng(seed)
    cases = [(5.0, 12.0, 10, -6.22e-3), (5.0, 12.0, 5, -1e-3), (5.0, 12.0, 0, -1e-6), (5.0, 12.0, 12, -1e-6),
             (5.0, 12.0, 12, -8.0), (2.0, 10.0, 1, -0.2)]
    for _ in range(n):
        cases.append((5.0, 12.0, int(rng.integers(0, 13)), -10 ** rng.uniform(-5, math.log10(8))))
    return cases


@pytest.mark.parametrize("case", _closed_cases(30, 1))
def test_closed_vs_mpmath_whittaker(case):
    z, a, l, eps = case
    mp.mp.dps = 40
    # kappa and nu in full precision from the same double eps (near threshold the
    # direction moves by ~pi nu per unit relative change of nu)
    kap = mp.sqrt(-mp.mpf(eps))
    nu = z / kap
    W = lambda r: mp.whitw(nu, l + 0.5, 2 * kap * r)
    ref = float(mp.diff(W, a) / W(a))
    got = oracle.closed_logderiv(z, eps, a, l)
    d1 = np.array([1.0, got]) / math.hypot(1, a * got)
    d2 = np.array([1.0, ref]) / math.hypot(1, a * ref)
    assert np.max(np.abs(d1 - d2) * [1, a]) < 5e-13, (got, ref)


def test_channel_function_normalisation():
    # open: s'c - s c' = 1 (unit Wronskian in r); closed: e^2 + (a e')^2 = 1, e >= 0
    rng = np.random.default_rng(2)
    for _ in range(200):
        z, a, l = 5.0, 12.0, int(rng.integers(0, 13))
        eps = rng.choice([-1, 1]) * 10 ** rng.uniform(-5, 0.9)
        s, sp, c, cp = oracle.channel(z, eps, a, l)
        if eps > 0:
            assert abs(sp * c - s * cp - 1) < 1e-12
        else:
            assert s == 0 and sp == 0 and c >= 0 and abs(c * c + (a * cp) ** 2 - 1) < 1e-14
