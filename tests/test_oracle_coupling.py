"""Pins of the oracle's long-range coupling and Numerov propagation (section
"Overview": eq. (radial) with the multipole potentials U_nm, propagated between
the boundary r0 = a and the asymptotic radius r1; Rydberg-unit reading
F'' = (diag(l(l+1)/r^2 - 2z/r - eps) + 2U) F, U_ij = sum_lam cf_ij r^-(lam+1)).

- U = 0: the propagated columns converge at fourth order to the analytic
  Coulomb / Whittaker functions at r = a, and K to the plain r = a matching.
- Coupled: the propagated matrices converge at fourth order to an mpmath
  Taylor-series ODE solution of the coupled equations (30 digits) started from
  the same data at r1.
- K is symmetric, invariant to the recombination of closed columns, and
  block-diagonal when the coupling and amplitudes do not connect two groups.
"""
import numpy as np
import pytest

import oracle
from paper_1909_07321_amd import synth


def _wave():
    return synth.make_partial_wave(1234, 6, 20, z=3.0, a=10.0, thr_range=(0.0, 3.0), pole_range=(-2.0, 40.0),
                                   name="px")


def _cf(n, seed=0, scale=1.0, lamax=2):
    cf = np.random.default_rng(seed).normal(size=(lamax, n, n)) * scale
    return cf + cf.transpose(0, 2, 1)


def _columns(open_row):
    n = open_row.size
    return [i for i in range(n) if not open_row[i]] + [i for i in range(n) if open_row[i]]


def test_uncoupled_propagation_converges_to_analytic():
    pw = _wave()
    E = np.array([0.7, 1.9, 3.3])
    o = oracle.Oracle(pw)
    fg, op, no, _ = o.asymptotic(E)
    n = pw.nchan
    errs = []
    for N in (801, 1601, 3201):
        phi, dphi, op2, no2, st = o.propagate(E, dict(cf=np.zeros((2, n, n)), r1=30.0, npts=N, stab=10 ** 9))
        assert (st == 0).all() and np.array_equal(op, op2)
        worst = 0.0
        for e in range(E.size):
            nc = n - no[e]
            for j, ch in enumerate(_columns(op[e])):
                # off-diagonal entries stay exactly zero without coupling
                assert np.count_nonzero(phi[e, :, j]) == 1
                if j < nc:   # closed: the direction (log derivative) is what is defined
                    ld, ref = dphi[e, ch, j] / phi[e, ch, j], fg[e, ch, 3] / fg[e, ch, 2]
                    worst = max(worst, abs(ld - ref) / abs(ref))
                else:
                    worst = max(worst, abs(phi[e, ch, j] - fg[e, ch, 2]), abs(dphi[e, ch, j] - fg[e, ch, 3]))
            for j in range(no[e]):
                ch = _columns(op[e])[nc + j]
                worst = max(worst, abs(phi[e, ch, n + j] - fg[e, ch, 0]), abs(dphi[e, ch, n + j] - fg[e, ch, 1]))
        errs.append(worst)
    print("uncoupled propagation error vs analytic:", errs)
    assert 10 < errs[0] / errs[1] < 25 and 10 < errs[1] / errs[2] < 25   # fourth order
    assert errs[2] < 3e-8


def test_uncoupled_K_converges_to_plain_matching():
    pw = _wave()
    E = np.array([0.7, 1.9, 3.3])
    o = oracle.Oracle(pw)
    R, _ = o.form_R(E)
    fg, op, no, _ = o.asymptotic(E)
    K0, _, _ = o.solve_K(E, R, fg)
    errs = []
    for N in (801, 3201):
        phi, dphi, *_ = o.propagate(E, dict(cf=np.zeros((1, pw.nchan, pw.nchan)), r1=30.0, npts=N))
        K, _, st = o.solve_K_coupled(E, R, phi, dphi)
        assert (st == 0).all()
        errs.append(max(np.abs(K[e, :no[e], :no[e]] - K0[e, :no[e], :no[e]]).max() / max(1, np.abs(K0[e]).max())
                        for e in range(E.size)))
    print("uncoupled K vs plain matching:", errs)
    assert errs[0] / errs[1] > 100 and errs[1] < 1e-7


def test_coupled_propagation_against_mpmath():
    mpmath = pytest.importorskip("mpmath")
    n, E, r1 = 3, 0.9, 16.0
    e_thr = np.array([0.0, 0.0, 1.5])
    l = np.array([0, 2, 1], np.int32)
    pw = synth.PartialWave(n, 10, 2, 8.0, 0.0, 2.0, 1.0, np.array([0.0, 1.5]), l, np.array([0, 0, 1], np.int32),
                           np.linspace(-1, 20, 10), np.full((10, n), 0.3))
    cf = _cf(n, 3, 0.4)
    mpmath.mp.dps = 30
    eps = [mpmath.mpf(E) - mpmath.mpf(float(x)) for x in e_thr]
    spec = [(2, 0), (0, 1), (1, 1), (0, 2), (1, 2)]   # closed e, open c, open s
    P, D = np.zeros((n, 5)), np.zeros((n, 5))
    for j, (ch, kind) in enumerate(spec):
        f = oracle.channel(pw.z, E - e_thr[ch], r1, int(l[ch]))
        v, dv = (f[0], f[1]) if kind == 2 else (f[2], f[3])
        y0 = [mpmath.mpf(0)] * (2 * n)
        y0[ch], y0[n + ch] = mpmath.mpf(v), -mpmath.mpf(dv)   # in t = r1 - r, dY/dt = -Y'

        def F(t, y):
            r = mpmath.mpf(r1) - t
            out = list(y[n:])
            for i in range(n):
                acc = (mpmath.mpf(int(l[i]) * (int(l[i]) + 1)) / r ** 2 - 2 * mpmath.mpf(pw.z) / r - eps[i]) * y[i]
                for k in range(n):
                    acc += 2 * sum(mpmath.mpf(cf[lam, i, k]) * r ** (-(lam + 2)) for lam in range(2)) * y[k]
                out.append(acc)
            return out
        y = mpmath.odefun(F, 0, y0)(mpmath.mpf(r1 - pw.a))
        P[:, j] = [float(y[i]) for i in range(n)]
        D[:, j] = [-float(y[n + i]) for i in range(n)]
    o = oracle.Oracle(pw)
    errs = []
    for N in (801, 1601, 3201):
        phi, dphi, _, _, st = o.propagate(np.array([E]), dict(cf=cf, r1=r1, npts=N, stab=10 ** 9))
        assert st[0] == 0
        ep = np.max(np.abs(phi[0][:, :5] - P) / np.abs(P).max(axis=0))
        ed = np.max(np.abs(dphi[0][:, :5] - D) / np.abs(D).max(axis=0))
        errs.append(max(ep, ed))
    print("coupled propagation vs mpmath:", errs)
    assert 10 < errs[0] / errs[1] < 25 and 10 < errs[1] / errs[2] < 25
    assert errs[2] < 1e-11


def test_coupled_K_symmetric_and_recombination_invariant():
    pw = _wave()
    E = np.array([0.7, 1.9, 3.3])
    o = oracle.Oracle(pw)
    cf = _cf(pw.nchan, 1)
    res = {stab: o.run_coupled(E, dict(cf=cf, r1=30.0, npts=1601, stab=stab)) for stab in (16, 64)}
    coarse = o.run_coupled(E, dict(cf=cf, r1=30.0, npts=801, stab=64))
    no = oracle.open_count(pw, E)
    asym = lambda K: max(np.abs(K[e, :no[e], :no[e]] - K[e, :no[e], :no[e]].T).max() / max(1, np.abs(K[e]).max())
                         for e in range(E.size))
    # symmetric up to the O(h^4) discretisation of the matching derivative
    a1, a2 = asym(coarse["K"]), asym(res[64]["K"])
    print("K asymmetry at 801 / 1601 points:", a1, a2)
    assert a2 < 5e-9 and 10 < a1 / a2 < 25
    for e in range(E.size):
        K = res[64]["K"][e, :no[e], :no[e]]
        assert np.abs(K - res[16]["K"][e, :no[e], :no[e]]).max() <= 1e-12 * max(1, np.abs(K).max())
    assert np.abs(res[64]["omega"] - res[16]["omega"]).max() <= 1e-12 * res[64]["omega"].max()
    # the coupling changes K (it is not silently dropped)
    K0 = o.run(E)["K"]
    assert np.abs(res[64]["K"][0] - K0[0]).max() > 1e-3


def test_recombination_at_last_allowed_step():
    """npts - 3 and npts - 2 both multiples of the recombination period: the
    last recombination (at step npts - 3, before Z_1 is recorded) must leave K
    as it is without any recombination (the derivative at r0 takes Z_1 and
    Z_-1 from one basis)."""
    pw = _wave()
    E = np.array([0.7, 3.3])
    o = oracle.Oracle(pw)
    cf = _cf(pw.nchan, 4)
    no = oracle.open_count(pw, E)
    ref = o.run_coupled(E, dict(cf=cf, r1=14.0, npts=131, stab=10 ** 9))["K"]
    for npts, stab in ((131, 64), (131, 128), (130, 64), (130, 128)):
        K = o.run_coupled(E, dict(cf=cf, r1=14.0, npts=npts, stab=stab))["K"]
        Kr = ref if npts == 131 else o.run_coupled(E, dict(cf=cf, r1=14.0, npts=npts, stab=10 ** 9))["K"]
        for e in range(E.size):
            d = np.abs(K[e, :no[e], :no[e]] - Kr[e, :no[e], :no[e]]).max() / max(1, np.abs(Kr[e]).max())
            assert d <= 1e-12, (npts, stab, e, d)


def test_block_diagonal_coupling():
    """Two groups of channels connected neither by the coupling nor by the
    amplitudes (disjoint pole sets): K is block diagonal and each block equals
    the problem of its group alone."""
    pw = _wave()
    n = pw.nchan
    A, B = [0, 1, 4], [2, 3, 5]
    w = pw.w.copy()
    half = pw.npole // 2
    w[:half][:, B] = 0.0
    w[half:][:, A] = 0.0
    cf = _cf(n, 2)
    for g1 in A:
        for g2 in B:
            cf[:, g1, g2] = cf[:, g2, g1] = 0.0
    full = synth.PartialWave(n, pw.npole, pw.ntarget, pw.a, pw.b, pw.z, pw.g, pw.e_target, pw.l, pw.target,
                             pw.Ek, w)
    E = np.array([0.7, 2.9])
    cp = dict(r1=25.0, npts=1601, stab=64)
    Kf = oracle.Oracle(full).run_coupled(E, dict(cp, cf=cf))["K"]
    for grp in (A, B):
        sub = synth.PartialWave(len(grp), pw.npole, pw.ntarget, pw.a, pw.b, pw.z, pw.g, pw.e_target, pw.l[grp],
                                pw.target[grp], pw.Ek, np.ascontiguousarray(w[:, grp]))
        Ks = oracle.Oracle(sub).run_coupled(E, dict(cp, cf=np.ascontiguousarray(cf[:, grp][:, :, grp])))["K"]
        for e in range(E.size):
            ef = E[e] - pw.e_thr > 0
            of = [i for i in range(n) if ef[i]]          # open channels of the full wave, ascending
            og = [i for i in grp if ef[i]]
            if not og:
                continue
            rows = [of.index(i) for i in og]
            blk = Kf[e][np.ix_(rows, rows)]
            np.testing.assert_allclose(blk, Ks[e, :len(og), :len(og)], rtol=1e-11, atol=1e-13)
            others = [k for k in range(len(of)) if k not in rows]
            if others:
                assert np.abs(Kf[e][np.ix_(rows, others)]).max() <= 1e-12 * max(1, np.abs(blk).max())
