"""Pins for the oracle's R-matrix stage, eq. (rmatrix) of the PSTGF paper
(section "Overview"): R_ij = (1/2a) sum_k w_ik w_jk / (E_k - E)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1909_07321_amd import synth


def _pw(w, Ek, a=2.0, e_thr=None, l=None):
    M, n = w.shape
    e_thr = np.zeros(n) if e_thr is None else np.asarray(e_thr, float)
    targets = np.arange(n, dtype=np.int32)
    return synth.PartialWave(n, M, n, a, 0.0, 1.0, 1.0, e_thr, np.zeros(n, np.int32) if l is None else np.asarray(l, np.int32),
                             targets, np.asarray(Ek, float), np.ascontiguousarray(w, float))


def test_exact_rational():
    # decimal-exact inputs: R computed with fractions.Fraction must match
    rng = np.random.default_rng(3)
    n, M = 3, 7
    w = rng.integers(-8, 9, size=(M, n)) / 4.0
    Ek = np.sort(rng.integers(-40, 40, size=M) / 8.0)
    Ek = np.unique(Ek)
    w = w[: Ek.size]
    a = 2.5
    pw = _pw(w, Ek, a=a)
    E = np.array([0.3125, 1.0625, -2.75])
    R, st = oracle.Oracle(pw).form_R(E)
    assert (st == 0).all()
    for e, Ev in enumerate(E):
        for i in range(n):
            for j in range(n):
                exact = sum(Fraction(w[k, i]) * Fraction(w[k, j]) / (Fraction(Ek[k]) - Fraction(Ev))
                            for k in range(Ek.size)) / (2 * Fraction(a))
                assert R[e, i, j] == float(exact)


def test_rank_one_single_pole():
    w = np.array([[0.7, -1.3, 0.2, 2.0]])
    Ek = np.array([1.5])
    pw = _pw(w, Ek, a=3.0)
    E = np.array([0.25, 2.0])
    R, _ = oracle.Oracle(pw).form_R(E)
    for e, Ev in enumerate(E):
        ref = np.outer(w[0], w[0]) / (2 * 3.0 * (1.5 - Ev))
        np.testing.assert_allclose(R[e], ref, rtol=1e-15, atol=0)


def test_symmetry_and_monotone_diagonal():
    pw, E = synth.config1()
    o = oracle.Oracle(pw)
    R, st = o.form_R(E)
    assert (st == 0).all()
    assert np.array_equal(R, np.transpose(R, (0, 2, 1)))
    # dR/dE = (1/2a) W D^2 W^T is positive semidefinite: between two adjacent
    # poles every diagonal element increases with E
    lo, hi = pw.Ek[np.searchsorted(pw.Ek, 1.0) - 1], pw.Ek[np.searchsorted(pw.Ek, 1.0)]
    Eg = np.linspace(lo + 1e-3, hi - 1e-3, 50)
    Rg, _ = o.form_R(Eg)
    d = np.diagonal(Rg, axis1=1, axis2=2)
    assert (np.diff(d, axis=0) > 0).all()
    # and the smallest eigenvalue of the finite difference is >= 0
    for e in range(len(Eg) - 1):
        assert np.linalg.eigvalsh(Rg[e + 1] - Rg[e]).min() > -1e-12


def test_pole_status_and_nan():
    pw, _ = synth.config1()
    E = np.array([pw.Ek[5], 0.5 * (pw.Ek[5] + pw.Ek[6])])
    R, st = oracle.Oracle(pw).form_R(E)
    assert st[0] == oracle.PT_POLE and np.isnan(R[0]).all()
    assert st[1] == 0 and np.isfinite(R[1]).all()


def test_long_double_vs_compensated_double():
    # independent re-sum of config 2 entries with math.fsum (exactly rounded)
    import math
    pw, E = synth.config2()
    o = oracle.Oracle(pw)
    Es = E[[3, 777, 1500]]
    R, _ = o.form_R(Es)
    rng = np.random.default_rng(0)
    for e, Ev in enumerate(Es):
        for _ in range(6):
            i, j = rng.integers(0, pw.nchan, 2)
            terms = pw.w[:, i] * pw.w[:, j] / (pw.Ek - Ev)
            ref = math.fsum(terms.tolist()) / (2 * pw.a)
            assert abs(R[e, i, j] - ref) <= 1e-13 * np.abs(terms).sum() / (2 * pw.a)
