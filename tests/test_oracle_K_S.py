"""Pins for the oracle's matching/K solve (eq. (match) of the PSTGF paper) and
its S, T and collision-strength stage (Glossary)."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_1909_07321_amd import synth


def _one_channel(z, a, l, Ek, w, b=0.0, g=1.0):
    Ek = np.asarray(Ek, float)
    w = np.asarray(w, float).reshape(-1, 1)
    return synth.PartialWave(1, Ek.size, 1, a, b, z, g, np.array([0.0]), np.array([l], np.int32),
                             np.array([0], np.int32), Ek, w)


def test_neutral_s_wave_closed_form():
    # one open channel, z = 0, l = 0: tan(delta) = (kaR cos ka - sin ka)/(cos ka + kaR sin ka)
    rng = np.random.default_rng(4)
    Ek = np.sort(rng.uniform(-1, 30, 12))
    w = rng.normal(size=12) / math.sqrt(8.0)
    pw = _one_channel(0.0, 8.0, 0, Ek, w)
    E = np.linspace(0.05, 3.0, 57)
    o = oracle.Oracle(pw)
    res = o.run(E, want_S=True)
    R, _ = o.form_R(E)
    for e, Ev in enumerate(E):
        k = math.sqrt(Ev)
        ka, r = k * 8.0, R[e, 0, 0]
        tand = (ka * r * math.cos(ka) - math.sin(ka)) / (math.cos(ka) + ka * r * math.sin(ka))
        assert abs(res["K"][e, 0, 0] - tand) <= 1e-13 * max(1, abs(tand))
        d = math.atan(tand)
        assert abs(res["S"][e, 0, 0] - complex(math.cos(2 * d), math.sin(2 * d))) < 1e-13
        assert abs(res["omega"][e, 0, 0] - 0.5 * 4 * math.sin(d) ** 2) < 1e-13


@pytest.mark.parametrize("l,b,g", [(0, 0.0, 1.0), (1, 0.0, 3.0), (2, 0.7, 2.0)])
def test_single_channel_ion_closed_form(l, b, g):
    # F = s + cK on one open channel and F = R(aF' - bF) give
    # K = (R (a s' - b s) - s) / (c - R (a c' - b c)), with s, c from mpmath
    z, a = 2.0, 10.0
    rng = np.random.default_rng(l)
    Ek = np.sort(rng.uniform(-1, 30, 10))
    w = rng.normal(size=10) / math.sqrt(a)
    pw = _one_channel(z, a, l, Ek, w, b=b, g=g)
    E = np.array([0.013, 0.4, 1.7, 2.9])
    o = oracle.Oracle(pw)
    R, _ = o.form_R(E)
    res = o.run(E)
    mp.mp.dps = 30
    for e, Ev in enumerate(E):
        k = mp.sqrt(mp.mpf(Ev))
        eta, rho = -z / k, k * a
        F = mp.coulombf(l, eta, rho)
        G = mp.coulombg(l, eta, rho)
        Fp = mp.diff(lambda x: mp.coulombf(l, eta, x), rho)
        Gp = mp.diff(lambda x: mp.coulombg(l, eta, x), rho)
        s, c, sp, cp = F / mp.sqrt(k), G / mp.sqrt(k), Fp * mp.sqrt(k), Gp * mp.sqrt(k)
        r = mp.mpf(R[e, 0, 0])
        Kref = float((r * (a * sp - b * s) - s) / (c - r * (a * cp - b * c)))
        assert abs(res["K"][e, 0, 0] - Kref) <= 1e-12 * max(1, abs(Kref))
        assert abs(res["omega"][e, 0, 0] - g / 2 * 4 * Kref ** 2 / (1 + Kref ** 2)) <= 1e-12 * g


def _reduced_K(R, fg, open_mask, a, b):
    """Closed channels eliminated first: R_eff = R_oo + R_oc (theta - R_cc)^-1 R_co
    with theta_c = e_c / (a e'_c - b e_c); then an open-channel-only solve."""
    o = np.where(open_mask)[0]
    c = np.where(~open_mask)[0]
    Reff = R[np.ix_(o, o)].copy()
    if c.size:
        th = fg[c, 2] / (a * fg[c, 3] - b * fg[c, 2])
        Reff += R[np.ix_(o, c)] @ np.linalg.solve(np.diag(th) - R[np.ix_(c, c)], R[np.ix_(c, o)])
    s, sp, cc, cp = fg[o, 0], fg[o, 1], fg[o, 2], fg[o, 3]
    A = np.diag(cc) - Reff * (a * cp - b * cc)[None, :]
    B = Reff * (a * sp - b * s)[None, :] - np.diag(s)
    return np.linalg.solve(A, B)


def test_full_and_reduced_formulations_agree():
    pw, E = synth.config2()
    o = oracle.Oracle(pw)
    sel = E[::97]
    R, _ = o.form_R(sel)
    fg, op, no, st = o.asymptotic(sel)
    K, cond, stk = o.solve_K(sel, R, fg)
    checked = 0
    for e in range(sel.size):
        assert stk[e] == 0
        if no[e] == 0:
            continue
        # the reduced form is solved in plain float64; the matching matrices here
        # have 1-norm condition estimates of 1e5..1e8, yet both forms agree to a
        # few 1e-12 (normwise, relative to max(1, max|K|))
        Kr = _reduced_K(R[e], fg[e], op[e].astype(bool), pw.a, pw.b)
        n0 = no[e]
        err = np.abs(K[e, :n0, :n0] - Kr).max() / max(1, np.abs(Kr).max())
        assert err < 1e-10, (e, err, cond[e])
        checked += 1
    assert checked >= 20


def test_K_symmetric_and_status_clean_config1_config2():
    for cfg in (synth.config1, synth.config2):
        pw, E = cfg()
        sel = E if E.size <= 200 else E[::41]
        res = oracle.Oracle(pw).run(sel)
        assert (res["status"] == 0).all()
        no = oracle.open_count(pw, sel)
        for e in range(sel.size):
            Kb = res["K"][e, : no[e], : no[e]]
            assert np.abs(Kb - Kb.T).max() <= 1e-12 * max(1, np.abs(Kb).max()) * max(1, res["cond"][e] / 1e3)


def test_block_diagonal_W_gives_block_diagonal_K():
    pw, E = synth.config1()
    w = pw.w.copy()
    w[:20, 2:] = 0.0   # poles 0..19 couple only to channels 0, 1
    w[20:, :2] = 0.0   # poles 20..39 couple only to channels 2, 3
    full = synth.PartialWave(4, 40, 2, pw.a, pw.b, pw.z, pw.g, pw.e_target, pw.l, pw.target, pw.Ek, w)
    blk0 = synth.PartialWave(2, 20, 1, pw.a, pw.b, pw.z, pw.g, pw.e_target[:1], pw.l[:2],
                             np.zeros(2, np.int32), pw.Ek[:20], np.ascontiguousarray(w[:20, :2]))
    blk1 = synth.PartialWave(2, 20, 1, pw.a, pw.b, pw.z, pw.g, pw.e_target[1:], pw.l[2:],
                             np.zeros(2, np.int32), pw.Ek[20:], np.ascontiguousarray(w[20:, 2:]))
    Eh = E[E > 0.6][::7]
    Kf = oracle.Oracle(full).run(Eh)["K"]
    K0 = oracle.Oracle(blk0).run(Eh)["K"]
    K1 = oracle.Oracle(blk1).run(Eh)["K"]
    for e in range(Eh.size):
        np.testing.assert_allclose(Kf[e, :2, :2], K0[e], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(Kf[e, 2:, 2:], K1[e], rtol=1e-12, atol=1e-13)
        assert np.abs(Kf[e, :2, 2:]).max() < 1e-13 and np.abs(Kf[e, 2:, :2]).max() < 1e-13
    # below the second threshold the closed block only enters through R_oc = 0
    El = E[E < 0.49][::9]
    Kf = oracle.Oracle(full).run(El)["K"]
    K0 = oracle.Oracle(blk0).run(El)["K"]
    np.testing.assert_allclose(Kf[:, :2, :2], K0, rtol=1e-12, atol=1e-13)


def test_K_continuous_across_R_pole():
    pw, _ = synth.config1()
    o = oracle.Oracle(pw)
    for k in [8, 15, 22]:
        Ek = pw.Ek[k]
        E = np.array([Ek - 1e-7, Ek + 1e-7])
        R, _ = o.form_R(E)
        res = o.run(E)
        assert np.abs(R[0] - R[1]).max() > 1e4          # R itself jumps through the pole
        no = oracle.open_count(pw, E[:1])[0]
        dK = np.abs(res["K"][0, :no, :no] - res["K"][1, :no, :no]).max()
        assert dK < 1e-4 * max(1, np.abs(res["K"][0]).max())


def test_K_invariant_to_closed_channel_scaling():
    pw, E = synth.config2()
    o = oracle.Oracle(pw)
    sel = E[100:2000:211]
    R, _ = o.form_R(sel)
    fg, op, no, _ = o.asymptotic(sel)
    K1, c1, _ = o.solve_K(sel, R, fg)
    fg2 = fg.copy()
    closed = op == 0
    fg2[..., 2][closed] *= -3.7
    fg2[..., 3][closed] *= -3.7
    K2, _, _ = o.solve_K(sel, R, fg2)
    for e in range(sel.size):
        n0 = no[e]
        assert np.abs(K1[e, :n0, :n0] - K2[e, :n0, :n0]).max() <= 1e-13 * max(1, np.abs(K1[e]).max()) * max(1, c1[e] / 1e2)


def test_S_unitary_symmetric_and_T_identity():
    pw, E = synth.config2()
    o = oracle.Oracle(pw)
    sel = E[5::181]
    res = o.run(sel, want_S=True)
    no = oracle.open_count(pw, sel)
    for e in range(sel.size):
        n0 = no[e]
        if n0 == 0:
            continue
        S = res["S"][e, :n0, :n0]
        K = res["K"][e, :n0, :n0]
        I = np.eye(n0)
        assert np.abs(S @ S.conj().T - I).max() < 1e-12
        assert np.abs(S - S.T).max() < 1e-12
        T = S - I
        # sum_j |T_ij|^2 = 2 (1 - Re S_ii) <= 4
        rows = (np.abs(T) ** 2).sum(axis=1)
        np.testing.assert_allclose(rows, 2 * (1 - S.diagonal().real), atol=1e-12)
        assert rows.max() <= 4 + 1e-12
        # |T|^2 = 4 [(Y - I)^2 + (Y K)^2] with Y = (1 + K^2)^-1
        Y = np.linalg.inv(I + K @ K)
        np.testing.assert_allclose(np.abs(T) ** 2, 4 * ((Y - I) ** 2 + (Y @ K) ** 2), atol=1e-11)


def test_omega_properties():
    pw, E = synth.config2()
    o = oracle.Oracle(pw)
    sel = E[7::173]
    res = o.run(sel, want_S=True)
    no = oracle.open_count(pw, sel)
    for e in range(sel.size):
        om = res["omega"][e]
        assert np.abs(om - om.T).max() < 1e-12 and om.min() >= 0
        # targets whose channels are all closed have no collision strength
        open_t = np.unique(pw.target[pw.e_thr < sel[e]])
        closed_t = np.setdiff1d(np.arange(pw.ntarget), open_t)
        assert np.all(om[closed_t, :] == 0) and np.all(om[:, closed_t] == 0)
        # total out of target p: sum_q Omega_pq = (g/2) sum_{i in p} 2 (1 - Re S_ii)
        S = res["S"][e, : no[e], : no[e]]
        tgt = pw.target[: no[e]] if no[e] else np.array([], int)
        idx = np.where(pw.e_thr < sel[e])[0]
        per = np.zeros(pw.ntarget)
        np.add.at(per, pw.target[idx], 0.5 * pw.g * 2 * (1 - S.diagonal().real))
        np.testing.assert_allclose(om.sum(axis=1), per, atol=1e-11)


def test_no_open_channels():
    pw, _ = synth.config2()
    # move every threshold above the energy
    pw2 = synth.PartialWave(pw.nchan, pw.npole, pw.ntarget, pw.a, pw.b, pw.z, pw.g, pw.e_target + 1.0,
                            pw.l, pw.target, pw.Ek, pw.w)
    res = oracle.Oracle(pw2).run(np.array([0.5, 0.9]))
    assert (res["status"] == 0).all() and (res["omega"] == 0).all()


def test_threshold_guard():
    pw, _ = synth.config1()
    res = oracle.Oracle(pw).run(np.array([0.5 + 1e-12, 0.5 + 1e-3]))
    assert res["status"][0] & oracle.PT_THRESHOLD and np.isnan(res["omega"][0]).all()
    assert res["status"][1] == 0


def test_omega_from_T_identity_by_target():
    # Omega_pq = (g/2) sum_{i in p, j in q} |T_ij|^2 with |T|^2 taken from the
    # Cholesky-free identity 4[(Y - I)^2 + (Y K)^2], Y = (1 + K^2)^-1
    pw, E = synth.config2()
    pw = synth.PartialWave(pw.nchan, pw.npole, pw.ntarget, pw.a, pw.b, pw.z, 2.0, pw.e_target, pw.l,
                           pw.target, pw.Ek, pw.w)
    sel = E[11::301]
    res = oracle.Oracle(pw).run(sel)
    for e in range(sel.size):
        idx = np.where(pw.e_thr < sel[e])[0]
        n0 = idx.size
        K = res["K"][e, :n0, :n0]
        Y = np.linalg.inv(np.eye(n0) + K @ K)
        T2 = 4 * ((Y - np.eye(n0)) ** 2 + (Y @ K) ** 2)
        om = np.zeros((pw.ntarget, pw.ntarget))
        np.add.at(om, (pw.target[idx][:, None], pw.target[idx][None, :]), 0.5 * pw.g * T2)
        np.testing.assert_allclose(res["omega"][e], om, atol=1e-10 * max(1, om.max()))


def test_channel_permutation_covariance():
    # relabelling channels permutes K and S among the open channels and leaves
    # Omega unchanged (targets keep their labels)
    pw, E = synth.config2()
    perm = np.random.default_rng(9).permutation(pw.nchan)
    pwp = synth.PartialWave(pw.nchan, pw.npole, pw.ntarget, pw.a, pw.b, pw.z, pw.g, pw.e_target,
                            pw.l[perm], pw.target[perm], pw.Ek, np.ascontiguousarray(pw.w[:, perm]))
    sel = E[40::400]
    r0 = oracle.Oracle(pw).run(sel)
    r1 = oracle.Oracle(pwp).run(sel)
    for e in range(sel.size):
        o0 = np.where(pw.e_thr < sel[e])[0]           # open channels, original labels
        o1 = np.where(pwp.e_thr < sel[e])[0]          # open channels, new labels
        n0 = o0.size
        # new open channel t is original channel perm[o1[t]]
        pos = {c: t for t, c in enumerate(o0)}
        q = np.array([pos[perm[c]] for c in o1], dtype=int)
        K0 = r0["K"][e, :n0, :n0]
        K1 = r1["K"][e, :n0, :n0]
        scale = max(1, np.abs(K0).max())
        assert np.abs(K1 - K0[np.ix_(q, q)]).max() < 1e-9 * scale
        np.testing.assert_allclose(r1["omega"][e], r0["omega"][e], atol=1e-9)


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_cond1_estimate_bounds_true_condition_number(cfg):
    """The oracle's condition estimate of the matching matrix (Hager's method
    for ||A^-1||_1 times ||A||_1) against the exact 1-norm condition number of
    A_im = d_im C_i - R_im (a C'_m - b C_m) (eq. (match)), rebuilt here from
    the oracle's own R and asymptotic values and evaluated by numpy.  Hager's
    estimate is a lower bound of ||A^-1||_1 that is in practice within a small
    factor of it, so the estimate must lie in [0.3, 1] x cond_1(A)."""
    if cfg == "c1":
        pw, E = synth.config1()
        E = E[::17]
    else:
        pw, E = synth.config2()
        E = E[::167]   # 12 energies across [0.01, 6] Ry
    o = oracle.Oracle(pw)
    R, _ = o.form_R(E)
    fg, _, no, _ = o.asymptotic(E)
    _, cond, st = o.solve_K(E, R, fg)
    assert (st == 0).all()
    for e in range(E.size):
        if no[e] == 0:
            assert cond[e] == 0
            continue
        C, Cp = fg[e, :, 2], fg[e, :, 3]
        A = np.diag(C) - R[e] * (pw.a * Cp - pw.b * C)[None, :]
        exact = np.linalg.cond(A, 1)
        assert 0.3 * exact <= cond[e] <= exact * (1 + 1e-12), (E[e], cond[e], exact)
