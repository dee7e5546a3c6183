"""Pins of the oracle's multichannel quantum-defect operation (the stgf
namelist's MQDT variables: iqdt = 1 treats every channel as open through the
unphysical K, imode = -1 solves on a coarse mesh and interpolates on the fine
one, ieq < 0 sets the coarse step, fnumin and iomsw = 1 omit deeply closed
channels).

The pins do not re-use the oracle's arithmetic:
* the energy-analytic Coulomb pair (f, g) against mpmath's Kummer and Tricomi
  functions, and its Wronskian;
* the pair joins the open-channel (s, c) smoothly at the threshold (Taylor
  coefficients fitted on both sides agree), which fixes its normalisation;
* eliminating the closed member channels from the unphysical K reproduces the
  physical K of the direct path at the same energy (an identity that holds
  only with the right pair, sign and tan(pi nu));
* with every point a coarse point the coarse/fine operation is the direct
  path; with fewer, its error falls as the fourth power of the coarse step
  where R is smooth (no pole of eq. (rmatrix) in the mesh range), also where
  the unphysical K itself has a pole (an eigenphase through pi/2), because
  the interpolated quantity is (1 - i Kun)^-1, bounded and smooth."""
import numpy as np
import mpmath as mp
import pytest

import oracle
from paper_1909_07321_amd import synth


def _ref_pair(z, eps, a, l):
    """(f, f', g, g') from closed forms: u = r^(l+1) e^(-kr) M(l+1-nu, 2l+2, 2kr),
    W = e^(-kr) (2kr)^(l+1) U(l+1-nu, 2l+2, 2kr), f = N A^(1/2) u,
    g = -W/Wr(f, W) + f cot(pi nu)."""
    mp.mp.dps = 40
    z, eps, a = mp.mpf(z), mp.mpf(eps), mp.mpf(a)
    kap = mp.sqrt(-eps)
    nu = z / kap
    A = mp.fprod([1 + p * p * eps / z ** 2 for p in range(1, l + 1)])
    N = mp.sqrt(2 * mp.pi * z) * (2 * z) ** l / mp.factorial(2 * l + 1)
    u = lambda r: r ** (l + 1) * mp.exp(-kap * r) * mp.hyp1f1(l + 1 - nu, 2 * l + 2, 2 * kap * r)
    w = lambda r: mp.exp(-kap * r) * (2 * kap * r) ** (l + 1) * mp.hyperu(l + 1 - nu, 2 * l + 2, 2 * kap * r)
    f, fp = N * mp.sqrt(A) * u(a), N * mp.sqrt(A) * mp.diff(u, a)
    e, ep = w(a), mp.diff(w, a)
    W = f * ep - fp * e
    cot = mp.cot(mp.pi * nu)
    return np.array([float(x) for x in (f, fp, -e / W + f * cot, -ep / W + fp * cot)])


CASES = [(5.0, -0.3, 12.0, 0), (5.0, -0.05, 12.0, 3), (3.0, -0.11, 9.0, 2), (5.0, -0.004, 12.0, 7),
         (2.0, -0.02, 10.0, 1), (5.0, -0.0123, 12.0, 15), (1.0, -0.0031, 20.0, 4)]


@pytest.mark.parametrize("z,eps,a,l", CASES)
def test_pair_against_kummer_and_tricomi(z, eps, a, l):
    out, member = oracle.mqdt_channel(z, eps, a, l, 0.0)
    assert member
    ref = _ref_pair(z, eps, a, l)
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
    # Wronskian f g' - f' g = -1, the value of s c' - s' c for open channels
    assert abs(out[0] * out[3] - out[1] * out[2] + 1.0) < 1e-12


def test_member_rule():
    """closed members need nu = z/sqrt(-eps) >= max(fnumin, l + 0.1)"""
    z, a = 5.0, 12.0
    for l, fnumin in [(0, 0.0), (3, 0.0), (3, 6.0), (9, 2.0)]:
        numin = max(fnumin, l + 0.1)
        edge = -(z * z) / (numin * numin)
        assert oracle.mqdt_channel(z, edge * 0.999, a, l, fnumin)[1]
        assert not oracle.mqdt_channel(z, edge * 1.001, a, l, fnumin)[1]
        out, m = oracle.mqdt_channel(z, 0.2, a, l, fnumin)  # open: the Coulomb (s, s', c, c')
        assert m and np.array_equal(out, oracle.channel(z, 0.2, a, l))
        out, m = oracle.mqdt_channel(z, edge * 1.5, a, l, fnumin)  # omitted: the decaying direction
        assert not m and np.array_equal(out, oracle.channel(z, edge * 1.5, a, l))


@pytest.mark.parametrize("l", [0, 2, 5])
def test_pair_continues_the_open_functions_across_threshold(l):
    """f and g below the threshold and s and c above it are one smooth function
    of energy: degree-5 fits on either side agree in value and slope at 0."""
    z, a, h = 5.0, 12.0, 2.113e-3
    xs = np.arange(1, 7) * h

    def fit(x, y):
        return np.polynomial.polynomial.polyfit(x, y, 5)

    lo = np.array([oracle.mqdt_channel(z, -x, a, l, 0.0)[0] for x in xs])
    hi = np.array([oracle.mqdt_channel(z, x, a, l, 0.0)[0] for x in xs])
    for q in range(4):
        cl, ch = fit(-xs, lo[:, q]), fit(xs, hi[:, q])
        scale = np.abs(hi[:, q]).max()
        assert abs(cl[0] - ch[0]) < 1e-11 * scale, (q, cl[0], ch[0])
        assert abs(cl[1] - ch[1]) < 1e-6 * scale, (q, cl[1], ch[1])


def _wave(seed=5, n=12, far=False):
    pr = (20.0, 80.0) if far else (-2.0, 40.0)
    return synth.make_partial_wave(seed, n, 10, z=5.0, a=12.0, thr_range=(0.0, 3.0), pole_range=pr,
                                   npole=15 * n, name="mq")


def test_elimination_reproduces_the_physical_K():
    pw = _wave()
    E = np.array([0.37, 1.23, 2.11, 2.95, 3.4, 0.0913, 1.777])
    o = oracle.Oracle(pw, nthreads=4)
    fnumin = np.sqrt(pw.z * pw.a)
    Ku, nm, st = o.unphysical_K(E, fnumin)
    K, st2 = o.mqdt_eliminate(E, fnumin, Ku, nm)
    ref = o.run(E)
    no = oracle.open_count(pw, E)
    assert (st == 0).all() and (st2 == 0).all() and (ref["status"] == 0).all()
    closed_members = nm - no
    assert closed_members.max() >= 2  # the identity is exercised with closed members present
    for e in range(E.size):
        a, b = K[e, :no[e], :no[e]], ref["K"][e, :no[e], :no[e]]
        assert np.abs(a - b).max() <= 1e-11 * max(1.0, np.abs(b).max()), e
        # the unphysical K is symmetric like the physical one
        k = Ku[e, :nm[e], :nm[e]]
        assert np.abs(k - k.T).max() <= 1e-11 * max(1.0, np.abs(k).max())


def test_without_closed_members_unphysical_is_physical():
    pw = _wave()
    E = np.array([0.8, 2.2])
    o = oracle.Oracle(pw, nthreads=4)
    Ku, nm, st = o.unphysical_K(E, 1e6)
    ref = o.run(E)
    no = oracle.open_count(pw, E)
    assert np.array_equal(nm, no)
    for e in range(E.size):
        assert np.abs(Ku[e, :no[e], :no[e]] - ref["K"][e, :no[e], :no[e]]).max() <= 1e-12 * max(
            1.0, np.abs(ref["K"][e]).max())


def test_coarse_points_and_every_point_coarse():
    pw = _wave(far=True)
    th = np.unique(pw.e_thr)
    E = np.linspace(th[1] + 0.01, th[2] - 0.003, 97)
    o = oracle.Oracle(pw, nthreads=4)
    fnumin = np.sqrt(pw.z * pw.a)
    ref = o.run(E)
    r1 = o.mqdt_run(E, 1, fnumin)
    assert r1["coarse"].all()
    no = oracle.open_count(pw, E)
    for e in range(E.size):
        b = ref["K"][e, :no[e], :no[e]]
        assert np.abs(r1["K"][e, :no[e], :no[e]] - b).max() <= 1e-11 * max(1.0, np.abs(b).max())
    assert np.abs(r1["omega"] - ref["omega"]).max() <= 1e-11 * np.abs(ref["omega"]).max()
    # coarse points: every ieq-th point of each run of equal member count and each run's last point
    _, nm, _ = o.unphysical_K(E, fnumin)
    r5 = o.mqdt_run(E, 5, fnumin)
    want = np.zeros(E.size, bool)
    s0 = 0
    while s0 < E.size:
        s1 = s0 + 1
        while s1 < E.size and nm[s1] == nm[s0]:
            s1 += 1
        want[s0:s1:5] = True
        want[s1 - 1] = True
        s0 = s1
    assert np.array_equal(r5["coarse"], want)
    assert len(np.unique(nm)) >= 2  # the mesh crosses a change of the member set
    # at the coarse points the result is the direct one
    c = np.flatnonzero(want)
    for e in c:
        b = ref["K"][e, :no[e], :no[e]]
        assert np.abs(r5["K"][e, :no[e], :no[e]] - b).max() <= 1e-11 * max(1.0, np.abs(b).max())


def test_interpolation_error_falls_as_fourth_power():
    """No pole of eq. (rmatrix) in the mesh range, so the unphysical K is smooth
    while the physical K carries the Rydberg resonances of the closed members."""
    pw = synth.make_partial_wave(7, 10, 8, z=5.0, a=12.0, thr_range=(0.0, 2.0), pole_range=(20.0, 80.0),
                                 npole=200, name="smooth")
    th = np.unique(pw.e_thr)
    E = np.linspace(th[1] + 0.01, th[2] - 0.005, 401)
    o = oracle.Oracle(pw, nthreads=4)
    fnumin = np.sqrt(pw.z * pw.a)
    ref = o.run(E)
    no = oracle.open_count(pw, E)
    med = []
    for ieq in (4, 8, 16):
        r = o.mqdt_run(E, ieq, fnumin)
        assert (r["status"] == 0).all()
        err = [np.abs(r["K"][e, :no[e], :no[e]] - ref["K"][e, :no[e], :no[e]]).max() /
               max(1.0, np.abs(ref["K"][e, :no[e], :no[e]]).max()) for e in range(E.size) if not r["coarse"][e]]
        med.append(np.median(err))
    assert med[0] < 1e-7
    assert 6.0 < med[1] / med[0] < 40.0 and 6.0 < med[2] / med[1] < 40.0, med


def test_flagged_points_are_not_coarse_and_bad_input_is_refused():
    pw = _wave(far=True)
    th = np.unique(pw.e_thr)
    E = np.linspace(th[1] - 0.02, th[1] + 0.02, 21)
    E[10] = th[1]  # exactly at a threshold
    o = oracle.Oracle(pw, nthreads=2)
    r = o.mqdt_run(E, 4, np.sqrt(pw.z * pw.a))
    assert r["status"][10] & oracle.PT_THRESHOLD and not r["coarse"][10]
    assert np.isnan(r["omega"][10]).all()
    assert (r["status"][np.arange(21) != 10] == 0).all()
    with pytest.raises(ValueError):
        o.mqdt_run(E[::-1], 4, 7.0)
    with pytest.raises(ValueError):
        o.mqdt_run(E, 0, 7.0)


def _minv(K, m):
    """(1 - i K)^-1 of the leading m x m block (numpy), as X + i Y padded to K's shape."""
    X, Y = np.zeros_like(K), np.zeros_like(K)
    if m:
        Mi = np.linalg.inv(np.eye(m) - 1j * K[:m, :m])
        X[:m, :m], Y[:m, :m] = Mi.real, Mi.imag
    return X, Y


def _ku_from_xy(X, Y, m):
    """unphysical K = Y X^-1 of the leading m x m blocks, symmetrised"""
    K = np.zeros_like(X)
    if m:
        Z = np.linalg.solve(X[:m, :m], Y[:m, :m])
        K[:m, :m] = 0.5 * (Z + Z.T)
    return K


def test_fine_point_uses_the_four_surrounding_coarse_points():
    """A fine point between coarse points c_k <= E < c_(k+1) of its run takes the
    cubic through c_(k-1) .. c_(k+2) (shifted inside the run at its ends) of the
    real and imaginary parts of (1 - i Kun)^-1, and Kun = Y X^-1 from them."""
    pw = _wave(far=True)
    th = np.unique(pw.e_thr)
    E = np.linspace(th[1] + 0.01, th[2] - 0.003, 61)
    o = oracle.Oracle(pw, nthreads=4)
    fnumin = np.sqrt(pw.z * pw.a)
    r = o.mqdt_run(E, 6, fnumin)
    Ku, nm, _ = o.unphysical_K(E, fnumin)
    no = oracle.open_count(pw, E)
    ok = []
    for e in range(E.size):
        if r["coarse"][e]:
            continue
        run = np.flatnonzero(nm == nm[e])
        cl = [j for j in run if r["coarse"][j]]
        k = max(q for q in range(len(cl)) if cl[q] <= e)
        w = min(4, len(cl))
        s0 = max(0, min(k - 1, len(cl) - w))
        nodes = cl[s0:s0 + w]
        wts = [np.prod([(E[e] - E[m]) / (E[q] - E[m]) for m in nodes if m != q]) for q in nodes]
        xy = [_minv(Ku[q], nm[q]) for q in nodes]
        X = sum(w * x for w, (x, _) in zip(wts, xy))
        Y = sum(w * y for w, (_, y) in zip(wts, xy))
        Ki = _ku_from_xy(X, Y, nm[e])
        K, st = o.mqdt_eliminate(E[e:e + 1], fnumin, Ki[None], nm[e:e + 1])
        b = K[0, :no[e], :no[e]]
        # on a closed-channel resonance the elimination magnifies the rounding
        # of the interpolant (here in double, there in long double); a wrong
        # stencil moves every point by the interpolation error instead
        ok.append(np.abs(r["K"][e, :no[e], :no[e]] - b).max() <= 1e-11 * max(1.0, np.abs(b).max()))
    assert len(ok) > 40 and np.mean(ok) >= 0.95, np.mean(ok)


def test_interpolation_converges_across_a_pole_of_the_unphysical_K():
    """Below the highest threshold of the quantum-defect workload (scaled down)
    an eigenphase of the unphysical K passes pi/2, so Kun has a pole in the
    mesh; the interpolated (1 - i Kun)^-1 has none, and the median error of K
    still falls as the fourth power of the coarse step."""
    pw, E, _, fnumin = synth.config_mqdt(24, 20, 400)
    o = oracle.Oracle(pw, nthreads=4)
    Ku, nm, st = o.unphysical_K(E, fnumin)
    ok = st == 0
    assert ok.mean() > 0.99
    big = np.array([np.abs(Ku[e, :nm[e], :nm[e]]).max() for e in np.flatnonzero(ok)])
    assert big.max() > 1e2 * np.median(big)  # the pole
    ref = o.run(E)
    no = oracle.open_count(pw, E)
    med = []
    for ieq in (4, 8):
        r = o.mqdt_run(E, ieq, fnumin)
        err = [np.abs(r["K"][e, :no[e], :no[e]] - ref["K"][e, :no[e], :no[e]]).max() /
               max(1.0, np.abs(ref["K"][e, :no[e], :no[e]]).max()) for e in range(E.size) if not r["coarse"][e]]
        med.append(np.median(err))
    assert med[0] < 1e-5 and 6.0 < med[1] / med[0] < 40.0, med


def test_interpolating_K_itself_converges_only_without_poles():
    """iqdt = 2 interpolates the unphysical K: with every point coarse it is the
    direct path; where Ku has no pole in the mesh its error falls with the
    coarse step like the S interpolation's; across a pole of Ku (the
    highest-threshold window) it fails where the S interpolation does not."""
    pw = synth.make_partial_wave(7, 10, 8, z=5.0, a=12.0, thr_range=(0.0, 2.0), pole_range=(20.0, 80.0),
                                 npole=200, name="smooth")
    th = np.unique(pw.e_thr)
    E = np.linspace(th[1] + 0.01, th[2] - 0.005, 401)
    o = oracle.Oracle(pw, nthreads=4)
    fnumin = np.sqrt(pw.z * pw.a)
    ref = o.run(E)
    no = oracle.open_count(pw, E)

    def med(r):
        return np.median([np.abs(r["K"][e, :no[e], :no[e]] - ref["K"][e, :no[e], :no[e]]).max() /
                          max(1.0, np.abs(ref["K"][e, :no[e], :no[e]]).max()) for e in range(E.size)
                          if not r["coarse"][e]])

    r1 = o.mqdt_run(E, 1, fnumin, iqdt=2)
    assert max(np.abs(r1["K"][e] - ref["K"][e]).max() for e in range(E.size)) < 1e-10
    m4, m8 = med(o.mqdt_run(E, 4, fnumin, iqdt=2)), med(o.mqdt_run(E, 8, fnumin, iqdt=2))
    assert m4 < 1e-6 and 6.0 < m8 / m4 < 40.0, (m4, m8)
    pw2, E2, _, fn2 = synth.config_mqdt(24, 20, 400)
    o2 = oracle.Oracle(pw2, nthreads=4)
    ref2 = o2.run(E2)
    no2 = oracle.open_count(pw2, E2)

    def med2(r):
        return np.median([np.abs(r["K"][e, :no2[e], :no2[e]] - ref2["K"][e, :no2[e], :no2[e]]).max() /
                          max(1.0, np.abs(ref2["K"][e, :no2[e], :no2[e]]).max()) for e in range(E2.size)
                          if not r["coarse"][e]])

    assert med2(o2.mqdt_run(E2, 4, fn2, iqdt=2)) > 100 * med2(o2.mqdt_run(E2, 4, fn2, iqdt=1))


def test_qetest_reuses_the_interpolant_within_its_energy_step():
    """A point within qetest z^2 of the last point evaluated at its own energy
    takes the interpolant at that energy (its tan(pi nu) stays its own); other
    points are as without qetest."""
    pw = _wave(far=True)
    th = np.unique(pw.e_thr)
    E = np.linspace(th[1] + 0.01, th[2] - 0.003, 61)
    o = oracle.Oracle(pw, nthreads=4)
    fnumin = np.sqrt(pw.z * pw.a)
    h = E[1] - E[0]
    qe = 1.5 * h / pw.z ** 2  # every other fine point reuses its neighbour's interpolant
    r0 = o.mqdt_run(E, 6, fnumin)
    rq = o.mqdt_run(E, 6, fnumin, qetest=qe)
    assert np.array_equal(r0["coarse"], rq["coarse"])
    Ku, nm, _ = o.unphysical_K(E, fnumin)
    last, reused, same = None, 0, 0
    for e in range(E.size):
        if e == 0 or nm[e] != nm[e - 1]:
            last = None
        if not rq["coarse"][e] and last is not None and abs(E[e] - E[last]) <= qe * pw.z ** 2:
            # interpolant of the point `last`, eliminated at this point's energy
            run = np.flatnonzero(nm == nm[e])
            cl = [j for j in run if rq["coarse"][j]]
            k = max([q for q in range(len(cl)) if cl[q] <= last] or [0])
            w = min(4, len(cl))
            s0 = max(0, min(k - 1, len(cl) - w))
            nodes = cl[s0:s0 + w]
            wts = [np.prod([(E[last] - E[m]) / (E[q] - E[m]) for m in nodes if m != q]) for q in nodes]
            xy = [_minv(Ku[q], nm[q]) for q in nodes]
            Ki = _ku_from_xy(sum(a * x for a, (x, _) in zip(wts, xy)), sum(a * y for a, (_, y) in zip(wts, xy)),
                             nm[e])
            K, _ = o.mqdt_eliminate(E[e:e + 1], fnumin, Ki[None], nm[e:e + 1])
            no = oracle.open_count(pw, E[e:e + 1])[0]
            b = K[0, :no, :no]
            assert np.abs(rq["K"][e, :no, :no] - b).max() <= 1e-9 * max(1.0, np.abs(b).max()), e
            reused += 1
        else:
            assert np.array_equal(rq["K"][e], r0["K"][e]), e
            same += 1
            last = e
    assert reused >= 15 and same >= 15
    with pytest.raises(ValueError):
        o.mqdt_run(E, 6, fnumin, iqdt=3)
    with pytest.raises(ValueError):
        o.mqdt_run(E, 6, fnumin, qetest=-1.0)


def test_s_form_elimination():
    """Omega from the closed members eliminated in S form,
    S = S_oo + S_oc (e^{-2 pi i nu} - S_cc)^-1 S_co of the interpolated
    unphysical S: the direct Omega at every-point-coarse, fourth-order
    convergence where R is smooth, and agreement with the K route to the
    interpolation error."""
    pw = synth.make_partial_wave(7, 10, 8, z=5.0, a=12.0, thr_range=(0.0, 2.0), pole_range=(20.0, 80.0),
                                 npole=200, name="smooth")
    th = np.unique(pw.e_thr)
    E = np.linspace(th[1] + 0.01, th[2] - 0.005, 401)
    o = oracle.Oracle(pw, nthreads=4)
    fn = np.sqrt(pw.z * pw.a)
    ref = o.run(E)

    def oerr(a, b):
        a, b = a.reshape(E.size, -1), b.reshape(E.size, -1)
        top = np.abs(b).max(axis=1, keepdims=True)
        return (np.abs(a - b) / np.maximum(np.abs(b), 1e-12 * top)).max(axis=1)

    r1 = o.mqdt_run(E, 1, fn, sform=True)
    assert (r1["status"] == 0).all() and oerr(r1["omega"], ref["omega"]).max() < 1e-11
    assert not r1["K"].any()  # K is not formed in S form
    med = []
    for q in (8, 16):
        rs, rk = o.mqdt_run(E, q, fn, sform=True), o.mqdt_run(E, q, fn)
        f = ~rs["coarse"]
        med.append(np.median(oerr(rs["omega"], ref["omega"])[f]))
        assert np.median(oerr(rs["omega"], rk["omega"])[f]) < 10 * med[-1] + 1e-14
    assert med[0] < 1e-12 and 6.0 < med[1] / med[0] < 40.0, med
    with pytest.raises(ValueError):
        o.mqdt_run(E, 4, fn, iqdt=2, sform=True)
