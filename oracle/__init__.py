"""FP64 CPU oracle for the outer-region R-matrix energy loop (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  It wraps ``rmo.c`` (plain long-double C, OpenMP over energies)
with ctypes and shares no code with the HIP library.  See ``rmo.h`` for the
conventions and the paper passages each stage follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "librmo.so")
_SRC = os.path.join(_HERE, "rmo.c")

PT_POLE, PT_THRESHOLD, PT_NOCONV, PT_SINGULAR, PT_NONFINITE = 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/librmo.so."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-std=c11", "-Wall", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _PW(ctypes.Structure):
    _fields_ = [("nchan", ctypes.c_int32), ("npole", ctypes.c_int32), ("ntarget", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("z", ctypes.c_double),
                ("g", ctypes.c_double),
                ("e_thr", ctypes.c_void_p), ("l", ctypes.c_void_p), ("target", ctypes.c_void_p),
                ("Ek", ctypes.c_void_p), ("w", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("RMO_SO")  # a mutant build, used only by the mutation test
        if not path:
            build(force=False)
            path = _SO
        _lib = ctypes.CDLL(path)
        vp, i32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        _lib.rmo_form_R.argtypes = [vp, vp, i32, vp, vp, i32]
        _lib.rmo_asymptotic.argtypes = [vp, vp, i32, d, vp, vp, vp, vp, i32]
        _lib.rmo_solve_K.argtypes = [vp, vp, i32, vp, vp, d, vp, vp, vp, i32]
        _lib.rmo_collision_strengths.argtypes = [vp, vp, i32, vp, d, vp, vp, vp, i32]
        _lib.rmo_run.argtypes = [vp, vp, i32, d, vp, vp, vp, vp, vp, i32]
        _lib.rmo_coulomb.argtypes = [d, d, i32, vp]
        _lib.rmo_closed_logderiv.argtypes = [d, d, d, i32, vp]
        _lib.rmo_channel.argtypes = [d, d, d, i32, vp]
        _lib.rmo_propagate.argtypes = [vp, vp, vp, i32, d, vp, vp, vp, vp, vp, i32]
        _lib.rmo_solve_K_coupled.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, i32]
        _lib.rmo_run_coupled.argtypes = [vp, vp, vp, i32, d, vp, vp, vp, vp, i32]
        _lib.rmo_unphysical_K.argtypes = [vp, vp, i32, d, d, vp, vp, vp, vp, i32]
        _lib.rmo_mqdt_eliminate.argtypes = [vp, vp, i32, d, vp, vp, vp, vp, i32]
        _lib.rmo_mqdt_run.argtypes = [vp, vp, i32, i32, i32, i32, d, d, d, vp, vp, vp, vp, i32]
        _lib.rmo_mqdt_channel.argtypes = [d, d, d, i32, d, vp]
    return _lib


class _Coupling(ctypes.Structure):
    _fields_ = [("lamax", ctypes.c_int32), ("cf", ctypes.c_void_p), ("r1", ctypes.c_double),
                ("npts", ctypes.c_int32), ("stab", ctypes.c_int32)]


def _coupling(cp: dict):
    """cp: dict(cf=[lamax][n][n] array, r1, npts, stab); returns (struct, keep-alive)."""
    cf = np.ascontiguousarray(cp["cf"], dtype=np.float64)
    return _Coupling(cf.shape[0], cf.ctypes.data if cf.size else None, float(cp["r1"]), int(cp["npts"]),
                     int(cp.get("stab", 64))), cf


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """Holds one partial wave; every call returns fresh numpy arrays."""

    def __init__(self, pw, nthreads: int = 0):
        self.pw = pw
        self.nthreads = int(nthreads)
        self._keep = [np.ascontiguousarray(pw.e_thr, dtype=np.float64),
                      np.ascontiguousarray(pw.l, dtype=np.int32),
                      np.ascontiguousarray(pw.target, dtype=np.int32),
                      np.ascontiguousarray(pw.Ek, dtype=np.float64),
                      np.ascontiguousarray(pw.w, dtype=np.float64)]
        self._s = _PW(pw.nchan, pw.npole, pw.ntarget, pw.a, pw.b, pw.z, pw.g,
                      *[k.ctypes.data for k in self._keep])

    @property
    def _p(self):
        return ctypes.byref(self._s)

    def form_R(self, E):
        E = np.ascontiguousarray(E, dtype=np.float64)
        n = self.pw.nchan
        R = np.empty((E.size, n, n))
        st = np.zeros(E.size, np.int32)
        lib().rmo_form_R(self._p, _ptr(E), E.size, _ptr(R), _ptr(st), self.nthreads)
        return R, st

    def asymptotic(self, E, thr_guard: float = 1e-10):
        E = np.ascontiguousarray(E, dtype=np.float64)
        n = self.pw.nchan
        fg = np.empty((E.size, n, 4))
        op = np.empty((E.size, n), np.int8)
        no = np.empty(E.size, np.int32)
        st = np.zeros(E.size, np.int32)
        lib().rmo_asymptotic(self._p, _ptr(E), E.size, thr_guard, _ptr(fg), _ptr(op), _ptr(no),
                             _ptr(st), self.nthreads)
        return fg, op, no, st

    def solve_K(self, E, R, fg, thr_guard: float = 1e-10):
        E = np.ascontiguousarray(E, dtype=np.float64)
        R = np.ascontiguousarray(R, dtype=np.float64)
        fg = np.ascontiguousarray(fg, dtype=np.float64)
        n = self.pw.nchan
        K = np.empty((E.size, n, n))
        cond = np.empty(E.size)
        st = np.zeros(E.size, np.int32)
        lib().rmo_solve_K(self._p, _ptr(E), E.size, _ptr(R), _ptr(fg), thr_guard, _ptr(K),
                          _ptr(cond), _ptr(st), self.nthreads)
        return K, cond, st

    def collision_strengths(self, E, K, thr_guard: float = 1e-10, want_S: bool = False):
        E = np.ascontiguousarray(E, dtype=np.float64)
        K = np.ascontiguousarray(K, dtype=np.float64)
        n, nt = self.pw.nchan, self.pw.ntarget
        om = np.empty((E.size, nt, nt))
        S = np.empty((E.size, n, n, 2)) if want_S else None
        st = np.zeros(E.size, np.int32)
        lib().rmo_collision_strengths(self._p, _ptr(E), E.size, _ptr(K), thr_guard, _ptr(om),
                                      _ptr(S) if want_S else None, _ptr(st), self.nthreads)
        return om, (S[..., 0] + 1j * S[..., 1] if want_S else None), st

    def propagate(self, E, coupling: dict, thr_guard: float = 1e-10):
        """Solution matrices at r0 = a after the Numerov propagation from r1:
        (phi, dphi [ne][n][2n], open, nopen, status)."""
        E = np.ascontiguousarray(E, dtype=np.float64)
        n = self.pw.nchan
        cs, keep = _coupling(coupling)
        phi, dphi = np.empty((E.size, n, 2 * n)), np.empty((E.size, n, 2 * n))
        op = np.empty((E.size, n), np.int8)
        no = np.empty(E.size, np.int32)
        st = np.zeros(E.size, np.int32)
        if lib().rmo_propagate(self._p, ctypes.byref(cs), _ptr(E), E.size, thr_guard, _ptr(phi), _ptr(dphi),
                               _ptr(op), _ptr(no), _ptr(st), self.nthreads):
            raise ValueError("invalid coupling")
        return phi, dphi, op, no, st

    def solve_K_coupled(self, E, R, phi, dphi):
        E = np.ascontiguousarray(E, dtype=np.float64)
        R, phi, dphi = (np.ascontiguousarray(x, dtype=np.float64) for x in (R, phi, dphi))
        n = self.pw.nchan
        K = np.empty((E.size, n, n))
        cond = np.empty(E.size)
        st = np.zeros(E.size, np.int32)
        lib().rmo_solve_K_coupled(self._p, _ptr(E), E.size, _ptr(R), _ptr(phi), _ptr(dphi), _ptr(K), _ptr(cond),
                                  _ptr(st), self.nthreads)
        return K, cond, st

    def run_coupled(self, E, coupling: dict, thr_guard: float = 1e-10):
        E = np.ascontiguousarray(E, dtype=np.float64)
        n, nt = self.pw.nchan, self.pw.ntarget
        cs, keep = _coupling(coupling)
        om = np.empty((E.size, nt, nt))
        K = np.empty((E.size, n, n))
        cond = np.empty(E.size)
        st = np.zeros(E.size, np.int32)
        if lib().rmo_run_coupled(self._p, ctypes.byref(cs), _ptr(E), E.size, thr_guard, _ptr(om), _ptr(K),
                                 _ptr(cond), _ptr(st), self.nthreads):
            raise ValueError("invalid coupling")
        return dict(omega=om, K=K, cond=cond, status=st)

    def unphysical_K(self, E, fnumin: float, thr_guard: float = 1e-10, want_cond: bool = False):
        """Unphysical K over the member channels at each energy: (Ku [ne][n][n]
        with the leading nmember x nmember block set, nmember, status); with
        want_cond also the matching matrix's 1-norm condition estimate."""
        E = np.ascontiguousarray(E, dtype=np.float64)
        n = self.pw.nchan
        Ku = np.empty((E.size, n, n))
        nm = np.empty(E.size, np.int32)
        cond = np.empty(E.size)
        st = np.zeros(E.size, np.int32)
        lib().rmo_unphysical_K(self._p, _ptr(E), E.size, fnumin, thr_guard, _ptr(Ku), _ptr(nm), _ptr(cond), _ptr(st),
                               self.nthreads)
        return (Ku, nm, st, cond) if want_cond else (Ku, nm, st)

    def mqdt_eliminate(self, E, fnumin: float, Ku, nmember):
        """Physical K from unphysical K at the same energies: (K, status)."""
        E = np.ascontiguousarray(E, dtype=np.float64)
        Ku = np.ascontiguousarray(Ku, dtype=np.float64)
        nm = np.ascontiguousarray(nmember, dtype=np.int32)
        n = self.pw.nchan
        K = np.empty((E.size, n, n))
        st = np.zeros(E.size, np.int32)
        lib().rmo_mqdt_eliminate(self._p, _ptr(E), E.size, fnumin, _ptr(Ku), _ptr(nm), _ptr(K), _ptr(st),
                                 self.nthreads)
        return K, st

    def mqdt_run(self, E, ieq: int, fnumin: float, thr_guard: float = 1e-10, iqdt: int = 1, qetest: float = 1e-7,
                 sform: bool = False):
        """Coarse/fine operation on an ascending mesh: dict(omega, K, coarse, status)."""
        E = np.ascontiguousarray(E, dtype=np.float64)
        n, nt = self.pw.nchan, self.pw.ntarget
        om = np.empty((E.size, nt, nt))
        K = np.empty((E.size, n, n))
        co = np.zeros(E.size, np.int8)
        st = np.zeros(E.size, np.int32)
        if lib().rmo_mqdt_run(self._p, _ptr(E), E.size, ieq, iqdt, int(sform), fnumin, qetest, thr_guard, _ptr(om),
                              _ptr(K), _ptr(co), _ptr(st), self.nthreads):
            raise ValueError("ieq >= 1, iqdt 1 or 2, qetest >= 0, z > 0 and an ascending mesh are needed")
        return dict(omega=om, K=K, coarse=co.astype(bool), status=st)

    def run(self, E, thr_guard: float = 1e-10, want_K: bool = True, want_S: bool = False):
        E = np.ascontiguousarray(E, dtype=np.float64)
        n, nt = self.pw.nchan, self.pw.ntarget
        om = np.empty((E.size, nt, nt))
        K = np.empty((E.size, n, n)) if want_K else None
        S = np.empty((E.size, n, n, 2)) if want_S else None
        cond = np.empty(E.size)
        st = np.zeros(E.size, np.int32)
        lib().rmo_run(self._p, _ptr(E), E.size, thr_guard, _ptr(om), _ptr(K) if want_K else None,
                      _ptr(S) if want_S else None, _ptr(cond), _ptr(st), self.nthreads)
        return dict(omega=om, K=K, S=(S[..., 0] + 1j * S[..., 1]) if want_S else None, cond=cond,
                    status=st)


def open_count(pw, E) -> np.ndarray:
    """Number of open channels per energy (eps_i = E - e_i > 0)."""
    E = np.asarray(E, dtype=np.float64)
    return (E[:, None] - pw.e_thr[None, :] > 0).sum(axis=1)


def coulomb(eta: float, rho: float, l: int) -> np.ndarray:
    """(F, dF/drho, G, dG/drho) of the Coulomb functions."""
    out = np.empty(4)
    if lib().rmo_coulomb(float(eta), float(rho), int(l), _ptr(out)):
        raise RuntimeError("coulomb: no convergence")
    return out


def closed_logderiv(z: float, eps: float, r: float, l: int) -> float:
    out = np.empty(1)
    if lib().rmo_closed_logderiv(float(z), float(eps), float(r), int(l), _ptr(out)):
        raise RuntimeError("closed_logderiv: no convergence")
    return float(out[0])


def channel(z: float, eps: float, a: float, l: int) -> np.ndarray:
    out = np.empty(4)
    if lib().rmo_channel(float(z), float(eps), float(a), int(l), _ptr(out)):
        raise RuntimeError("channel: no convergence")
    return out


def mqdt_channel(z: float, eps: float, a: float, l: int, fnumin: float):
    """Channel functions of the unphysical K at r = a and the member flag:
    ((s, s', c, c') | (f, f', g, g') | (0, 0, e, e'), member)."""
    out = np.empty(4)
    m = lib().rmo_mqdt_channel(z, eps, a, l, fnumin, _ptr(out))
    if m < 0:
        raise ArithmeticError("channel function did not converge")
    return out, bool(m)
