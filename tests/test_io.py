"""File boundary (section "Input files": H.DAT, sizeH.dat; section "Output
files": OMEGA): the library's readers against files written by independent
Python code, and its OMEGA writer against an independent Python reader."""
import struct

import numpy as np
import pytest

from paper_1909_07321_amd import synth

import _fortran as F


@pytest.fixture(scope="module")
def rm():
    from paper_1909_07321_amd import rm as m
    return m


def _target(nast=3, lamax=2, lrang2=2):
    rng = np.random.default_rng(5)
    enat = np.concatenate([[-1.25], np.sort(rng.uniform(-1.2, 0.5, nast - 1))])
    return dict(nelc=10, nz=14, lrang2=lrang2, lamax=lamax, enat=enat, lat=np.arange(nast) % 3,
                isat=np.full(nast, 2), ra=11.5, bsto=0.0, coeff=rng.normal(size=(lrang2, 3)),
                butt=[(rng.normal(size=k), rng.normal(size=k)) for k in range(2, 2 + lrang2)])


def _symmetry(seed, nconat, lamax, M):
    rng = np.random.default_rng(seed)
    n = int(sum(nconat))
    cf = rng.normal(size=(lamax, n, n))
    cf = cf + np.transpose(cf, (0, 2, 1))
    return dict(lrgl2=3, nspn2=2, npty2=1, nconat=np.asarray(nconat), l2p=rng.integers(0, 6, n),
                cf=cf, value=np.sort(rng.uniform(-2, 40, M)), wmat=rng.normal(size=(M, n)) / 3.4)


@pytest.mark.parametrize("big", [False, True])
def test_hdat_round_trip(tmp_path, rm, big):
    t = _target()
    syms = [_symmetry(1, [2, 0, 3], 2, 17), _symmetry(2, [1, 2, 2], 2, 9)]
    data = F.hdat_target(t["nelc"], t["nz"], t["lrang2"], t["lamax"], t["enat"], t["lat"], t["isat"], t["ra"],
                         t["bsto"], t["coeff"], t["butt"], big)
    data += F.hdat_symmetry(**syms[0], big=big, split=40)   # large records cut into subrecords
    path = tmp_path / "H.DAT000"
    path.write_bytes(data)
    more = tmp_path / "H.DAT001"
    more.write_bytes(F.hdat_symmetry(**syms[1], more2=1, big=big))
    tgt, got = rm.read_hdat(str(path), [str(more)])
    for k in ("nelc", "nz", "lrang2", "lamax", "ra", "bsto"):
        assert tgt[k] == t[k]
    assert tgt["nast"] == 3 and np.array_equal(tgt["enat"], t["enat"])
    assert np.array_equal(tgt["lat"], t["lat"]) and np.array_equal(tgt["isat"], t["isat"])
    assert len(got) == 2
    for s, g in zip(syms, got):
        for k in ("nconat", "l2p", "cf", "value", "wmat"):
            assert np.array_equal(np.asarray(g[k]), np.asarray(s[k])), k
        pw = g["pw"]
        tg = np.repeat(np.arange(3), s["nconat"])
        assert np.array_equal(pw.target, tg)
        assert np.array_equal(pw.e_target[pw.target], t["enat"][tg] - t["enat"][0])
        assert pw.z == t["nz"] - t["nelc"] and pw.a == t["ra"] and pw.g == 2 * (2 * 3 + 1)
        assert np.array_equal(pw.w, s["wmat"]) and np.array_equal(pw.Ek, s["value"])


def test_hdat_from_synthetic_wave_keeps_every_input(tmp_path, rm):
    """A synthetic partial wave written as H.DAT and read back gives the same
    descriptor: poles, amplitudes (pole-major), l, channel-to-target map and
    thresholds; J coupling (NSPN2 = 0) gives g = 2J + 1."""
    pw, _ = synth.config1()
    counts = np.bincount(pw.target, minlength=pw.ntarget)
    data = F.hdat_target(1, 3, 0, 1, pw.e_target, [0, 1], [0, 0], pw.a, pw.b, np.zeros((0, 3)), [])
    data += F.hdat_symmetry(5, 0, 0, counts, pw.l, np.zeros((1, 4, 4)), pw.Ek, pw.w)
    p = tmp_path / "H.DAT"
    p.write_bytes(data)
    _, got = rm.read_hdat(str(p))
    q = got[0]["pw"]
    assert q.nchan == pw.nchan and q.ntarget == pw.ntarget and q.g == 6.0 and q.z == 2.0
    for k in ("Ek", "w", "l", "target"):
        assert np.array_equal(getattr(q, k), getattr(pw, k)), k
    assert np.array_equal(q.e_target[q.target], pw.e_target[pw.target])


def test_hdat_rejects_damaged_files(tmp_path, rm):
    t = _target()
    good = F.hdat_target(t["nelc"], t["nz"], t["lrang2"], t["lamax"], t["enat"], t["lat"], t["isat"], t["ra"],
                         t["bsto"], t["coeff"], t["butt"])
    s = _symmetry(3, [2, 1, 1], 2, 5)
    cases = {
        "truncated": good[:-7],
        "nconat": good + F.hdat_symmetry(**{**s, "nconat": np.array([2, 1, 2])}),
        "poles": good + F.hdat_symmetry(**{**s, "value": s["value"][::-1].copy()}),
        "markers": good[:-4] + struct.pack("<i", 12345),
        "not_hdat": F.record(F.i4([1, 2, 3])),
    }
    for name, data in cases.items():
        p = tmp_path / f"bad_{name}"
        p.write_bytes(data)
        with pytest.raises(rm.RMError):
            rm.read_hdat(str(p))


def test_sizeh_and_sizebp(tmp_path, rm):
    rows = [(12, 240, 250, 2, 3, 1), (7, 140, 151, 4, 0, 0), (123, 2460, 2471, 0, 13, 1)]
    h = tmp_path / "sizeH.dat"
    # 8X,I5,10X,I6,8X,I6,3(4X,I3)
    h.write_text("".join(f"{'NCHAN =':8s}{a:5d}{'  NCON =  ':10s}{b:6d}{' MNP2 = ':8s}{c:6d}"
                         f"{'  S=':4s}{s:3d}{'  L=':4s}{l:3d}{' PI=':4s}{pi:3d}\n" for a, b, c, s, l, pi in rows))
    got = rm.read_sizeh(str(h), 0)
    assert [tuple(r.values()) for r in got] == rows
    bp = tmp_path / "sizeBP.dat"
    # 3I7,9X,I3,8X,I3
    bp.write_text("".join(f"{a:7d}{b:7d}{c:7d}{' 2J/PI = ':9s}{j:3d}{'  PAR = ':8s}{pi:3d}\n"
                          for a, b, c, _, j, pi in rows) + "\n")
    got = rm.read_sizeh(str(bp), 1)
    assert [(r["nchan"], r["ncon"], r["mnp2"], r["s"], r["l"], r["ipi"]) for r in got] == \
        [(a, b, c, 0, j, pi) for a, b, c, _, j, pi in rows]
    with pytest.raises(rm.RMError):
        rm.read_sizeh(str(tmp_path / "missing.dat"))


def _expected_transitions(nlev, nomwrt, elastic):
    if nomwrt >= 0:
        tr = [(i, j) for i in range(nlev) for j in range(i if elastic else i + 1, nlev)]
    else:
        tr = [(i, j) for j in range(nlev) for i in range(0, j + 1 if elastic else j)]
    return tr[:abs(nomwrt)]


@pytest.mark.parametrize("nomwrt,elastic", [(2 ** 31 - 1, False), (2 ** 31 - 1, True), (4, False), (-5, True)])
def test_omega_writer(tmp_path, rm, nomwrt, elastic):
    rng = np.random.default_rng(9)
    nlev, ne, nz, nel = 4, 6, 26, 23
    om = rng.uniform(0, 3, (ne, nlev, nlev))
    E = np.linspace(0.5, 9.0, ne)
    elev = np.array([0.0, 0.3, 0.71, 1.9])
    S, L = np.array([2, 4, 2, 2]), np.array([0, 1, 2, 1])
    tr = _expected_transitions(nlev, nomwrt, elastic)
    nw = len(tr) if nomwrt >= 0 else -len(tr)
    z2 = (nz - nel) ** 2
    for formatted in (True, False):
        p = tmp_path / ("OMEGA" if formatted else "OMEGAU")
        rm.write_omega(str(p), nz, nel, S, L, elev, E, om, nomwrt=nomwrt, elastic=elastic, formatted=formatted)
        if formatted:
            lines = p.read_text().split("\n")
            assert lines[0].split() == [str(nz), str(nel)]
            assert lines[1].split() == [str(nlev), str(ne), str(nw)]
            assert [int(x) for x in lines[2].split()] == [v for pair in zip(S, L) for v in pair]
            np.testing.assert_array_equal([float(x) for x in lines[3].split()], elev / z2)
            body = [[float(x) for x in ln.split()] for ln in lines[4:4 + ne]]
        else:
            recs = F.read_records(p.read_bytes())
            assert struct.unpack("<2i", recs[0]) == (nz, nel)
            assert struct.unpack("<3i", recs[1]) == (nlev, ne, nw)
            assert list(np.frombuffer(recs[2], "<i4")) == [v for pair in zip(S, L) for v in pair]
            np.testing.assert_array_equal(np.frombuffer(recs[3], "<f8"), elev / z2)
            body = [list(np.frombuffer(r, "<f8")) for r in recs[4:]]
            assert len(recs) == 4 + ne
        for e in range(ne):
            assert body[e][0] == E[e] / z2
            assert body[e][1:] == [om[e, i, j] for i, j in tr]


def test_file_calls_refuse_null_arguments():
    """Every file-boundary call with NULL handle, path and outputs returns
    RM_E_ARG without touching memory; closing a NULL handle is a no-op."""
    import ctypes

    from paper_1909_07321_amd import rm
    for name in ("rm_hdat_open", "rm_hdat_target_info", "rm_hdat_attach", "rm_hdat_next", "rm_hdat_arrays",
                 "rm_hdat_pw_desc", "rm_sizeh_read", "rm_omega_write", "rm_hdat_close"):
        fn = getattr(rm._lib, name)
        args = [0.0 if t is ctypes.c_double else
                None if (t in (ctypes.c_void_p, ctypes.c_char_p) or not isinstance(getattr(t, "_type_", ""), str))
                else 0 for t in fn.argtypes]
        assert fn(*args) == (rm.RM_OK if name == "rm_hdat_close" else rm.RM_E_ARG), name
