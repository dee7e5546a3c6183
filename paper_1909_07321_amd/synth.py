"""Seeded synthetic inputs for the outer-region R-matrix energy loop.

This module only draws numbers: channel thresholds, angular momenta, channel
to target maps, R-matrix poles E_k, surface amplitudes w_ik and energy grids.
It contains none of the method's arithmetic, so both the FP64 oracle and the
HIP library can consume the same inputs.

Random numbers come from splitmix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), evaluated in closed form per
index so that every field has its own reproducible stream; normals use the
Box-Muller transform.  The logical content of one partial wave mirrors the
symmetry record of an H.DAT file (PSTGF paper, section "Input files", H.DAT
table): poles ``Ek`` (VALUE), amplitudes ``w`` written pole by pole (WMAT),
channel angular momenta ``l`` (L2P), channel-to-target map (NCONAT), plus the
target energies, the box radius a, the logarithmic-derivative constant b and
the residual charge z.
"""
from __future__ import annotations

import dataclasses
import math
import zlib

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# grid energies are never placed closer than this to a channel threshold
THRESHOLD_CLEARANCE = 1e-9


def _mix(x: np.ndarray) -> np.ndarray:
    x = x.copy()
    x ^= x >> np.uint64(30)
    x *= _M1
    x ^= x >> np.uint64(27)
    x *= _M2
    x ^= x >> np.uint64(31)
    return x


class Stream:
    """Counter-based splitmix64 stream: value i is mix(seed + (i+1)*gamma)."""

    def __init__(self, seed: int, name: str):
        base = (int(seed) * 0x100000001B3 + zlib.crc32(name.encode())) & 0xFFFFFFFFFFFFFFFF
        self.seed = np.uint64(base)
        self.pos = 0

    def u64(self, n: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            idx = np.arange(self.pos + 1, self.pos + 1 + n, dtype=np.uint64)
            out = _mix(self.seed + idx * _GAMMA)
        self.pos += n
        return out

    def uniform(self, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        u = (self.u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
        return lo + (hi - lo) * u

    def integers(self, n: int, lo: int, hi_inclusive: int) -> np.ndarray:
        span = hi_inclusive - lo + 1
        return lo + np.floor(self.uniform(n) * span).astype(np.int64)

    def normal(self, n: int) -> np.ndarray:
        m = (n + 1) // 2
        u1 = self.uniform(m)
        u2 = self.uniform(m)
        r = np.sqrt(-2.0 * np.log1p(-u1))
        th = 2.0 * math.pi * u2
        out = np.empty(2 * m)
        out[0::2] = r * np.cos(th)
        out[1::2] = r * np.sin(th)
        return out[:n]


@dataclasses.dataclass
class PartialWave:
    """One partial wave's resident inputs (all host numpy arrays)."""

    nchan: int
    npole: int
    ntarget: int
    a: float
    b: float
    z: float
    g: float
    e_target: np.ndarray   # [ntarget] target energies (Ry)
    l: np.ndarray          # [nchan] int32 channel angular momentum
    target: np.ndarray     # [nchan] int32 target index of each channel
    Ek: np.ndarray         # [npole] ascending poles (Ry)
    w: np.ndarray          # [npole, nchan] amplitudes, w[k, i] = w_ik

    @property
    def e_thr(self) -> np.ndarray:
        """Channel thresholds e_i = target energy of the channel's target."""
        return np.ascontiguousarray(self.e_target[self.target], dtype=np.float64)

    def footprint_bytes(self) -> int:
        return self.npole * self.nchan * 12 + self.npole * 8


def _thresholds_clear(e_thr: np.ndarray, energies: np.ndarray) -> bool:
    if energies.size == 0:
        return True
    t = np.unique(e_thr)
    e = np.sort(energies)
    pos = np.searchsorted(e, t)
    for p, tv in zip(pos, t):
        for q in (p - 1, p):
            if 0 <= q < e.size and abs(e[q] - tv) < THRESHOLD_CLEARANCE:
                return False
    return True


def make_partial_wave(seed: int, nchan: int, poles_per_chan: float, *, z: float, a: float,
                      thr_range: tuple[float, float], pole_range: tuple[float, float],
                      lmax: int = 12, b: float = 0.0, g: float = 1.0,
                      avoid_energies: np.ndarray | None = None, npole: int | None = None,
                      name: str = "pw") -> PartialWave:
    """Random partial wave with ceil(n/4) targets, four channels per target.

    Target 0 sits at 0 Ry, the others are sorted uniform in ``thr_range``;
    channel i belongs to target min(i // 4, ntarget - 1); l_i is uniform in
    0..lmax; poles are sorted uniform in ``pole_range``; w_ik ~ N(0,1)/sqrt(a).
    Thresholds are redrawn until no energy of ``avoid_energies`` lies within
    THRESHOLD_CLEARANCE of one.
    """
    ntarget = max(1, -(-nchan // 4))
    M = int(npole if npole is not None else round(poles_per_chan * nchan))
    for attempt in range(1000):
        st = Stream(seed, f"{name}/thresholds/{attempt}")
        e_target = np.concatenate([[0.0], np.sort(st.uniform(ntarget - 1, *thr_range))])
        target = np.minimum(np.arange(nchan) // 4, ntarget - 1).astype(np.int32)
        if avoid_energies is None or _thresholds_clear(e_target[target], avoid_energies):
            break
    else:  # pragma: no cover
        raise RuntimeError("could not place thresholds away from the energy grid")
    l = Stream(seed, f"{name}/l").integers(nchan, 0, lmax).astype(np.int32)
    Ek = np.sort(Stream(seed, f"{name}/poles").uniform(M, *pole_range))
    w = (Stream(seed, f"{name}/w").normal(M * nchan) / math.sqrt(a)).reshape(M, nchan)
    return PartialWave(nchan, M, ntarget, float(a), float(b), float(z), float(g),
                       e_target, l, target, Ek, np.ascontiguousarray(w))


def partial_wave_family(seed: int, npw: int, ntarget: int, chan_per_target,
                        poles_per_chan: float, *, z: float, a: float, thr_range: tuple[float, float],
                        pole_range: tuple[float, float], lmax: int = 12,
                        avoid_energies: np.ndarray | None = None, name: str = "fam") -> list[PartialWave]:
    """Partial waves of one collision problem: they share the targets (target 0
    at 0 Ry, the others sorted uniform in ``thr_range``), and wave w couples each
    target to a uniform number of channels in ``chan_per_target`` (one (lo, hi)
    range for every wave, or a list with one range per wave; channels ordered
    by target, a target may have none), with its own l values, poles and
    amplitudes.  Wave w has statistical weight g = 2w + 1 (a stand-in for
    2J + 1)."""
    for attempt in range(1000):
        e_target = np.concatenate([[0.0], np.sort(Stream(seed, f"{name}/targets/{attempt}").uniform(ntarget - 1,
                                                                                                   *thr_range))])
        if avoid_energies is None or _thresholds_clear(e_target, avoid_energies):
            break
    else:  # pragma: no cover
        raise RuntimeError("could not place thresholds away from the energy grid")
    out = []
    for w in range(npw):
        rng_w = chan_per_target[w] if isinstance(chan_per_target, list) else chan_per_target
        counts = Stream(seed, f"{name}/w{w}/counts").integers(ntarget, *rng_w)
        target = np.repeat(np.arange(ntarget), counts).astype(np.int32)
        n = int(target.size)
        M = int(round(poles_per_chan * n))
        l = Stream(seed, f"{name}/w{w}/l").integers(n, 0, lmax).astype(np.int32)
        Ek = np.sort(Stream(seed, f"{name}/w{w}/poles").uniform(M, *pole_range))
        amp = (Stream(seed, f"{name}/w{w}/amp").normal(M * n) / math.sqrt(a)).reshape(M, n)
        out.append(PartialWave(n, M, ntarget, float(a), 0.0, float(z), float(2 * w + 1), e_target.copy(), l, target,
                               Ek, np.ascontiguousarray(amp)))
    return out


def config_sum(npw: int = 12, nenergy: int = 2000) -> tuple[list[PartialWave], np.ndarray]:
    """Sum over partial waves: 12 waves sharing 60 targets (thresholds in
    [0, 4] Ry), 1..4 channels per target, 30 poles per channel in [-2, 60] Ry,
    z=5, a=12, 2000 energies uniform in [0.01, 6] Ry."""
    E = np.linspace(0.01, 6.0, nenergy)
    return partial_wave_family(config_seed(6), npw, 60, (1, 4), 30, z=5.0, a=12.0, thr_range=(0.0, 4.0),
                               pole_range=(-2.0, 60.0), avoid_energies=E, name="sum"), E


def config_imbalance(npw: int = 16, nenergy: int = 2000) -> tuple[list[PartialWave], np.ndarray]:
    """Load-balance workload: 16 waves of one collision problem sharing 150
    targets (thresholds in [0, 6] Ry), wave w coupling each target to 0..k_w
    channels with k_w = 1 + (w mod 8), so channel counts run from about 75 to
    600; 30 poles per channel in [-2, 60] Ry, z=5, a=12, 2000 energies uniform
    in [0.01, 8] Ry, so the open fraction n_o/n runs from near 0 to 1 across the
    grid (the slow energies are those with n_o ~ n_c)."""
    E = np.linspace(0.01, 8.0, nenergy)
    ranges = [(0, 1 + (w % 8)) for w in range(npw)]
    return partial_wave_family(config_seed(7), npw, 150, ranges, 30, z=5.0, a=12.0, thr_range=(0.0, 6.0),
                               pole_range=(-2.0, 60.0), avoid_energies=E, name="imb"), E


def config_seed(index: int) -> int:
    return 1909 * 1000 + index


def config1() -> tuple[PartialWave, np.ndarray]:
    """Plain method, one partial wave: z=2, a=10, four channels on two targets
    (thresholds 0 and 0.5 Ry, l = 0,1,1,2), 40 poles uniform in [-1, 30] Ry,
    200 energies on a uniform grid in [0.05, 3] Ry."""
    seed = config_seed(1)
    E = np.linspace(0.05, 3.0, 200)
    e_target = np.array([0.0, 0.5])
    target = np.array([0, 0, 1, 1], dtype=np.int32)
    l = np.array([0, 1, 1, 2], dtype=np.int32)
    a = 10.0
    Ek = np.sort(Stream(seed, "c1/poles").uniform(40, -1.0, 30.0))
    w = (Stream(seed, "c1/w").normal(40 * 4) / math.sqrt(a)).reshape(40, 4)
    assert _thresholds_clear(e_target[target], E)
    pw = PartialWave(4, 40, 2, a, 0.0, 2.0, 1.0, e_target, l, target, Ek, np.ascontiguousarray(w))
    return pw, E


def config2() -> tuple[PartialWave, np.ndarray]:
    """200 channels, 30 poles per channel in [-2, 60] Ry, thresholds in [0, 4] Ry,
    z=5, a=12, 2000 energies uniform in [0.01, 6] Ry."""
    E = np.linspace(0.01, 6.0, 2000)
    pw = make_partial_wave(config_seed(2), 200, 30, z=5.0, a=12.0, thr_range=(0.0, 4.0),
                           pole_range=(-2.0, 60.0), avoid_energies=E, name="c2")
    return pw, E


def config3(npw: int = 64, nenergy: int = 5000) -> tuple[list[PartialWave], np.ndarray]:
    """64 partial waves, channel counts uniform in 20..600, 30 poles per channel,
    z=5, a=12, thresholds in [0, 4] Ry, 5000 energies uniform in [0.01, 6] Ry."""
    E = np.linspace(0.01, 6.0, nenergy)
    sizes = Stream(config_seed(3), "c3/sizes").integers(npw, 20, 600)
    pws = [make_partial_wave(config_seed(3), int(n), 30, z=5.0, a=12.0, thr_range=(0.0, 4.0),
                             pole_range=(-2.0, 60.0), avoid_energies=E, name=f"c3/pw{p}")
           for p, n in enumerate(sizes)]
    return pws, E


def config4(nenergy: int = 1000) -> tuple[PartialWave, np.ndarray]:
    """1500 channels, 40 poles per channel (60000) in [-2, 60] Ry, thresholds in
    [0, 8] Ry, z=5, a=12, 1000 energies uniform in [0.01, 8] Ry."""
    E = np.linspace(0.01, 8.0, nenergy)
    pw = make_partial_wave(config_seed(4), 1500, 40, z=5.0, a=12.0, thr_range=(0.0, 8.0),
                           pole_range=(-2.0, 60.0), avoid_energies=E, name="c4")
    return pw, E


@dataclasses.dataclass
class Request:
    pw_index: int
    arrival_s: float
    energies: np.ndarray


def config5_pool(npw: int = 16, nmax: int = 2000) -> list[PartialWave]:
    """Serving pool: channel counts log-uniform in [10, nmax], 30..40 poles per
    channel, thresholds in [0, 8] Ry, poles in [-2, 60] Ry, z=5, a=12."""
    st = Stream(config_seed(5), "c5/sizes")
    sizes = np.exp(st.uniform(npw, math.log(10), math.log(nmax))).round().astype(int)
    ppc = Stream(config_seed(5), "c5/ppc").integers(npw, 30, 40)
    return [make_partial_wave(config_seed(5), int(n), float(p), z=5.0, a=12.0, thr_range=(0.0, 8.0),
                              pole_range=(-2.0, 60.0), name=f"c5/pw{i}")
            for i, (n, p) in enumerate(zip(sizes, ppc))]


def config5_requests(pool: list[PartialWave], nreq: int = 400, rate_hz: float = 1.0,
                     block_range: tuple[int, int] = (100, 20000)) -> list[Request]:
    """Poisson request stream: pw uniform from the pool, block size log-uniform
    in ``block_range``, energies sorted uniform in [0.01, 8] Ry, kept clear of
    the chosen partial wave's thresholds."""
    st = Stream(config_seed(5), "c5/requests")
    pick = st.integers(nreq, 0, len(pool) - 1)
    sizes = np.exp(st.uniform(nreq, math.log(block_range[0]), math.log(block_range[1]))).round().astype(int)
    gaps = -np.log1p(-st.uniform(nreq)) / rate_hz
    t = np.cumsum(gaps)
    reqs = []
    for r in range(nreq):
        es = Stream(config_seed(5), f"c5/req{r}")
        E = np.sort(es.uniform(int(sizes[r]), 0.01, 8.0))
        thr = np.unique(pool[pick[r]].e_thr)
        pos = np.clip(np.searchsorted(thr, E), 1, thr.size - 1) if thr.size > 1 else np.zeros(E.size, int)
        near = np.minimum(np.abs(E - thr[pos]), np.abs(E - thr[np.maximum(pos - 1, 0)]))
        E = np.where(near < THRESHOLD_CLEARANCE, E + 10 * THRESHOLD_CLEARANCE, E)
        reqs.append(Request(int(pick[r]), float(t[r]), np.sort(E)))
    return reqs


def multipole_coefficients(seed: int, nchan: int, lamax: int = 2, scale: float = 0.5,
                           name: str = "cf") -> np.ndarray:
    """Coefficients of the long-range multipole potentials (the H.DAT CF
    record), [lamax][nchan][nchan]: for every order a symmetric matrix with
    N(0, scale^2) entries (the diagonal N(0, 2 scale^2))."""
    x = Stream(seed, f"{name}/{nchan}/{lamax}").normal(lamax * nchan * nchan).reshape(lamax, nchan, nchan) * scale
    return np.ascontiguousarray((x + x.transpose(0, 2, 1)) / math.sqrt(2.0))


def config_coupled(nchan: int = 100, nenergy: int = 1000) -> tuple[PartialWave, dict, np.ndarray]:
    """Coupled wave: 100 channels (25 targets, thresholds in [0, 8] Ry), 20
    poles per channel in [-2, 60] Ry, z=5, a=12, dipole and quadrupole
    potentials (lamax = 2, scale 0.5) propagated to r1 = 30 on the paper's 3201
    points, 1000 energies uniform in [0.01, 8] Ry.  Returns (wave, coupling,
    energies) with coupling = dict(cf, r1, npts, stab)."""
    E = np.linspace(0.01, 8.0, nenergy)
    pw = make_partial_wave(config_seed(8), nchan, 20, z=5.0, a=12.0, thr_range=(0.0, 8.0),
                           pole_range=(-2.0, 60.0), avoid_energies=E, name="cpl")
    cp = dict(cf=multipole_coefficients(config_seed(8), nchan), r1=30.0, npts=3201, stab=64)
    return pw, cp, E


def config_mqdt(nchan: int = 1500, poles_per_chan: float = 40, nenergy: int = 2000,
                seed_index: int = 9) -> tuple[PartialWave, np.ndarray, int, float]:
    """Quantum-defect workload: the Rydberg series below the highest threshold.
    1500 channels (375 targets), z=5, a=12, 40 poles per channel uniform in
    [9.5, 60] Ry; target thresholds uniform in [0, 8] Ry, then the highest
    target moved 0.6 Ry above the next one, so that every other channel is open
    across the mesh.  Fine mesh: 2000 energies from 0.4 Ry to 1e-3 Ry below the
    highest threshold, where that target's closed channels have effective
    quantum numbers 7.9..158 (all members with fnumin = sqrt(z a), except those
    with l + 0.1 above nu early in the mesh).  No pole lies within 0.9 Ry of
    the mesh, so R is smooth across it, as for an inner region whose
    eigenvalues are spaced wider than the mesh.  Coarse step ieq = 8.  Returns
    (wave, energies, ieq, fnumin)."""
    pw = make_partial_wave(config_seed(seed_index), nchan, poles_per_chan, z=5.0, a=12.0, thr_range=(0.0, 8.0),
                           pole_range=(9.5, 60.0), name="mqdt")
    top_t = int(np.argmax(pw.e_target))
    top = float(np.delete(pw.e_target, top_t).max()) + 0.6
    pw.e_target[top_t] = top
    E = np.linspace(top - 0.4, top - 1e-3, nenergy)
    return pw, E, 8, float(np.sqrt(pw.z * pw.a))
