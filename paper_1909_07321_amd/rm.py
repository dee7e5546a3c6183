"""Python binding of librm (C ABI in include/rm.h): argument marshalling only.

Every computation runs in the HIP library.  Host inputs/outputs are numpy
arrays; device inputs/outputs may be torch CUDA tensors, in which case the call
is ordered on the tensor's current torch stream (``device_ptrs = 1``).  There is
no fallback: if ``librm.so`` is missing or fails to load, importing this module
raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RM_LIB", os.path.join(_HERE, "librm.so"))

RM_OK, RM_PENDING = 0, 1
RM_E_ARG, RM_E_NOMEM, RM_E_DEVICE, RM_E_NOTFOUND, RM_E_BUSY, RM_E_IO = -1, -2, -3, -4, -5, -6
PT_POLE, PT_THRESHOLD, PT_NOCONV, PT_SINGULAR, PT_NONFINITE = 1, 2, 4, 8, 16
FP64, FP32_SPLIT = 0, 1
NOALLOC_SCRATCH_BYTES = 256 << 20  # RM_NOALLOC_SCRATCH_BYTES of rm.h
PROP_MAX_CHANNELS, PROP_MAX_LAMAX = 128, 8  # RM_PROP_MAX_CHANNELS, RM_PROP_MAX_LAMAX
ORDER_WAVE, ORDER_PERMUTED = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"librm.so not built ({LIB_PATH}); run __graft_entry__.build()")
try:
    # torch carries its own HIP runtime with the same soname as ROCm's; loading
    # it first makes librm bind to that one copy, so a process never holds two
    # HIP runtimes (torch tensors and librm then share device memory and streams)
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is optional for host-array use
    torch = None
_lib = ctypes.CDLL(LIB_PATH)

_vp, _i32, _u64, _d, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t


class Opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("split_delta", _d), ("thr_guard", _d), ("stream", _vp),
                ("device_ptrs", _i32)]


class PWDesc(ctypes.Structure):
    _fields_ = [("nchan", _i32), ("npole", _i32), ("ntarget", _i32), ("a", _d), ("b", _d), ("z", _d),
                ("g", _d), ("e_thr", _vp), ("l", _vp), ("target", _vp), ("Ek", _vp), ("w", _vp)]


class BatchItem(ctypes.Structure):
    _fields_ = [("pw_id", _i32), ("E", _vp), ("ne", _i32), ("omega", _vp), ("K", _vp), ("status", _vp)]


class Request(ctypes.Structure):
    _fields_ = [("pw_id", _i32), ("E", _vp), ("ne", _i32), ("opts", Opts), ("omega", _vp), ("K", _vp),
                ("status", _vp)]


class ReqStats(ctypes.Structure):
    _fields_ = [("t_arrive_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("nblocks", _i32)]


_lib.rm_opts_default.argtypes = [ctypes.POINTER(Opts)]
_lib.rm_create.argtypes = [ctypes.c_int, _sz, ctypes.POINTER(_vp)]
_lib.rm_destroy.argtypes = [_vp]
_lib.rm_last_error.argtypes = [_vp]
_lib.rm_last_error.restype = ctypes.c_char_p
_lib.rm_pw_upload.argtypes = [_vp, ctypes.POINTER(PWDesc), ctypes.POINTER(_i32)]
_lib.rm_pw_release.argtypes = [_vp, _i32]
_lib.rm_pw_footprint.argtypes = [_i32, _i32]
_lib.rm_pw_footprint.restype = _sz
_lib.rm_work_footprint.argtypes = [_i32, _i32, _i32, _i32]
_lib.rm_work_footprint.restype = _sz
_lib.rm_form_R.argtypes = [_vp, _i32, _vp, _i32, ctypes.POINTER(Opts), _vp, _vp]
_lib.rm_asymptotic.argtypes = [_vp, _i32, _vp, _i32, ctypes.POINTER(Opts), _vp, _vp, _vp, _vp]
_lib.rm_solve_K.argtypes = [_vp, _i32, _vp, _i32, _vp, _vp, ctypes.POINTER(Opts), _vp, _vp]
_lib.rm_collision_strengths.argtypes = [_vp, _i32, _vp, _i32, _vp, ctypes.POINTER(Opts), _vp, _vp, _vp]
_lib.rm_run.argtypes = [_vp, _i32, _vp, _i32, ctypes.POINTER(Opts), _vp, _vp, _vp]
_lib.rm_run_noalloc.argtypes = [_vp, _i32, _vp, _i32, ctypes.POINTER(Opts), _vp, _vp, _vp]
_lib.rm_run_batch.argtypes = [_vp, ctypes.POINTER(BatchItem), _i32, ctypes.POINTER(Opts)]
_lib.rm_run_sum.argtypes = [_vp, ctypes.POINTER(_i32), _i32, _vp, _i32, _i32, ctypes.POINTER(Opts), _vp, _vp]
_lib.rm_submit.argtypes = [_vp, ctypes.POINTER(Request), ctypes.POINTER(_u64)]
_lib.rm_poll.argtypes = [_vp, _u64, ctypes.POINTER(ReqStats)]
_lib.rm_drain.argtypes = [_vp]
_lib.rm_prof_enable.argtypes = [_vp, _i32]
_lib.rm_prof_read.argtypes = [_vp, ctypes.c_char_p, ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64)]
_lib.rm_prof_chunks.argtypes = [_vp, ctypes.c_int64, _vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_int64)]
_lib.rm_tile_bucket.argtypes = [_i32]
_lib.rm_tile_bucket.restype = _i32
_lib.rm_tile_count.argtypes = [_i32]
_lib.rm_tile_count.restype = _i32
_lib.rm_tile_shape.argtypes = [_i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
_lib.rm_get_tile.argtypes = [_vp, _i32, _i32, ctypes.POINTER(_i32)]
_lib.rm_set_tile.argtypes = [_vp, _i32, _i32, _i32]
_lib.rm_tune.argtypes = [_vp, _i32, ctypes.POINTER(_i32), _i32, _vp, _i32, _i32, ctypes.c_char_p, _vp]
_lib.rm_tune_load.argtypes = [_vp, ctypes.c_char_p]
_lib.rm_set_graph.argtypes = [_vp, _i32]
_lib.rm_graph_stats.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
_lib.rm_pw_upload_coupled.argtypes = [_vp, ctypes.POINTER(PWDesc), _i32, _vp, _d, ctypes.POINTER(_i32)]
_lib.rm_set_propagation.argtypes = [_vp, _i32, _i32]
_lib.rm_propagate.argtypes = [_vp, _i32, _vp, _i32, ctypes.POINTER(Opts), _vp, _vp, _vp]
_lib.rm_mqdt_unphysical_K.argtypes = [_vp, _i32, _vp, _i32, _d, ctypes.POINTER(Opts), _vp, _vp, _vp]


class MqdtOpts(ctypes.Structure):
    _fields_ = [("ieq", _i32), ("iqdt", _i32), ("fnumin", _d), ("qetest", _d)]


_lib.rm_mqdt_opts_default.argtypes = [ctypes.POINTER(MqdtOpts)]
_lib.rm_run_mqdt.argtypes = [_vp, _i32, _vp, _i32, ctypes.POINTER(MqdtOpts), ctypes.POINTER(Opts), _vp, _vp, _vp,
                             _vp]

EXPORTS = ["rm_opts_default", "rm_create", "rm_destroy", "rm_last_error", "rm_pw_upload", "rm_pw_release",
           "rm_pw_footprint", "rm_work_footprint", "rm_form_R", "rm_asymptotic", "rm_solve_K", "rm_collision_strengths", "rm_run",
           "rm_run_noalloc", "rm_run_batch", "rm_run_sum", "rm_tile_bucket", "rm_tile_count", "rm_tile_shape", "rm_get_tile",
           "rm_set_tile", "rm_tune", "rm_tune_load", "rm_set_graph", "rm_graph_stats",
           "rm_submit", "rm_poll", "rm_drain", "rm_prof_enable", "rm_prof_read", "rm_prof_chunks",
           "rm_pw_upload_coupled", "rm_set_propagation", "rm_propagate", "rm_mqdt_unphysical_K", "rm_run_mqdt", "rm_mqdt_opts_default",
           "rm_hdat_open", "rm_hdat_close", "rm_hdat_error", "rm_hdat_target_info", "rm_hdat_attach", "rm_hdat_next",
           "rm_hdat_arrays", "rm_hdat_pw_desc", "rm_sizeh_read", "rm_omega_write"]


class RMError(RuntimeError):
    pass


# ------------------------------------------------------------ file boundary
class HdatTarget(ctypes.Structure):
    _fields_ = [("nelc", _i32), ("nz", _i32), ("lrang2", _i32), ("lamax", _i32), ("nast", _i32), ("ra", _d),
                ("bsto", _d)]


class HdatSym(ctypes.Structure):
    _fields_ = [("lrgl2", _i32), ("nspn2", _i32), ("npty2", _i32), ("nchan", _i32), ("mnp2", _i32), ("more2", _i32)]


class SizeRow(ctypes.Structure):
    _fields_ = [("nchan", _i32), ("ncon", _i32), ("mnp2", _i32), ("s", _i32), ("l", _i32), ("ipi", _i32)]


_lib.rm_hdat_open.argtypes = [ctypes.c_char_p, ctypes.POINTER(_vp)]
_lib.rm_hdat_close.argtypes = [_vp]
_lib.rm_hdat_error.argtypes = [_vp]
_lib.rm_hdat_error.restype = ctypes.c_char_p
_lib.rm_hdat_target_info.argtypes = [_vp, ctypes.POINTER(HdatTarget), _vp, _vp, _vp]
_lib.rm_hdat_attach.argtypes = [_vp, ctypes.c_char_p]
_lib.rm_hdat_next.argtypes = [_vp, ctypes.POINTER(HdatSym)]
_lib.rm_hdat_arrays.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
_lib.rm_hdat_pw_desc.argtypes = [_vp, ctypes.POINTER(PWDesc)]
_lib.rm_sizeh_read.argtypes = [ctypes.c_char_p, _i32, _i32, ctypes.POINTER(SizeRow), ctypes.POINTER(_i32)]
_lib.rm_omega_write.argtypes = [ctypes.c_char_p, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _i32, _i32]


def read_hdat(path: str, more_files=()):
    """Reads an H.DAT / H.DAT000 file (and further H.DATXXX symmetry files):
    returns (target dict, list of symmetry dicts).  Each symmetry dict holds
    the record values and ``pw``, a partial wave ready for Context.pw_upload
    (thresholds ENAT(target) - ENAT(1), statistical weight from S, L or J)."""
    from . import synth
    h = _vp()
    st = _lib.rm_hdat_open(path.encode(), ctypes.byref(h))
    try:
        if st < 0:
            raise RMError(f"librm status {st}: {_lib.rm_hdat_error(h).decode()}")
        t = HdatTarget()
        _lib.rm_hdat_target_info(h, ctypes.byref(t), None, None, None)
        enat, lat, isat = np.empty(t.nast), np.empty(t.nast, np.int32), np.empty(t.nast, np.int32)
        _lib.rm_hdat_target_info(h, ctypes.byref(t), _ptr(enat), _ptr(lat), _ptr(isat))
        target = dict(nelc=t.nelc, nz=t.nz, lrang2=t.lrang2, lamax=t.lamax, nast=t.nast, ra=t.ra, bsto=t.bsto,
                      enat=enat, lat=lat, isat=isat)
        syms, files = [], list(more_files)
        while True:
            sym = HdatSym()
            st = _lib.rm_hdat_next(h, ctypes.byref(sym))
            if st == RM_E_NOTFOUND:
                if not files:
                    break
                if _lib.rm_hdat_attach(h, files.pop(0).encode()) < 0:
                    raise RMError(_lib.rm_hdat_error(h).decode())
                continue
            if st < 0:
                raise RMError(f"librm status {st}: {_lib.rm_hdat_error(h).decode()}")
            n, M = sym.nchan, sym.mnp2
            nconat, l2p = np.empty(t.nast, np.int32), np.empty(n, np.int32)
            cf, value, wmat = np.empty((t.lamax, n, n)), np.empty(M), np.empty((M, n))
            _lib.rm_hdat_arrays(h, _ptr(nconat), _ptr(l2p), _ptr(cf), _ptr(value), _ptr(wmat))
            d = PWDesc()
            _lib.rm_hdat_pw_desc(h, ctypes.byref(d))
            ethr = np.ctypeslib.as_array(ctypes.cast(d.e_thr, ctypes.POINTER(_d)), (n,)).copy()
            tgt = np.ctypeslib.as_array(ctypes.cast(d.target, ctypes.POINTER(_i32)), (n,)).copy()
            pw = synth.PartialWave(n, M, d.ntarget, d.a, d.b, d.z, d.g, enat - enat[0], l2p.copy(), tgt,
                                   value.copy(), wmat.copy())
            assert np.array_equal(pw.e_target[pw.target], ethr)
            syms.append(dict(lrgl2=sym.lrgl2, nspn2=sym.nspn2, npty2=sym.npty2, nchan=n, mnp2=M, more2=sym.more2,
                             nconat=nconat, l2p=l2p, cf=cf, value=value, wmat=wmat, pw=pw))
        return target, syms
    finally:
        _lib.rm_hdat_close(h)


def read_sizeh(path: str, kind: int = 0):
    """Rows of sizeH.dat (kind 0) or sizeBP.dat (kind 1) as dicts."""
    cnt = _i32()
    st = _lib.rm_sizeh_read(path.encode(), kind, 0, None, ctypes.byref(cnt))
    if st < 0:
        raise RMError(f"librm status {st}: cannot read {path}")
    rows = (SizeRow * max(1, cnt.value))()
    _lib.rm_sizeh_read(path.encode(), kind, cnt.value, rows, ctypes.byref(cnt))
    return [dict(nchan=r.nchan, ncon=r.ncon, mnp2=r.mnp2, s=r.s, l=r.l, ipi=r.ipi) for r in rows[:cnt.value]]


def write_omega(path: str, nz: int, nel: int, S, L, elev, E, omega, nomwrt: int = 2 ** 31 - 1,
                elastic: bool = False, formatted: bool = True):
    """Writes OMEGA (formatted) or OMEGAU (unformatted) from omega [ne][nlev][nlev]."""
    S = np.ascontiguousarray(S, np.int32)
    L = np.ascontiguousarray(L, np.int32)
    elev = np.ascontiguousarray(elev, np.float64)
    E = np.ascontiguousarray(E, np.float64)
    omega = np.ascontiguousarray(omega, np.float64)
    st = _lib.rm_omega_write(path.encode(), int(formatted), nz, nel, S.size, _ptr(S), _ptr(L), _ptr(elev), E.size,
                             _ptr(E), _ptr(omega), int(nomwrt), int(elastic))
    if st < 0:
        raise RMError(f"librm status {st}: cannot write {path}")


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _energies(E):
    """An energy mesh as the library reads it: (array, on_device).  A torch
    tensor is handed over as device memory and must be a contiguous 1-D float64
    tensor on the GPU (anything else would be misread or read past its end);
    other input becomes a contiguous float64 host array."""
    if _is_torch(E):
        if not (E.is_cuda and str(E.dtype) == "torch.float64" and E.dim() == 1 and E.is_contiguous()):
            raise RMError(f"energies on the device must be a contiguous 1-D float64 GPU tensor "
                          f"(got {E.dtype}, shape {tuple(E.shape)}, {E.device})")
        return E, True
    E = np.ascontiguousarray(E, dtype=np.float64)
    if E.ndim != 1:
        raise RMError(f"energies must be 1-D (got shape {E.shape})")
    return E, False


def _check_outputs(call, dev, outs, write=True):
    """Caller-owned buffers: each (name, array, shape, numpy dtype) must be
    device memory when the energies are (host memory otherwise), of that dtype,
    contiguous and of that shape (shape None: not checked), and writeable when
    the library writes it, since the library reads or writes it in full through
    a raw pointer.  A None array passes (the optional ones are checked by the
    library)."""
    for name, a, shape, dt in outs:
        if a is None:
            continue
        if dev:
            ok = (_is_torch(a) and a.is_cuda and str(a.dtype) == "torch." + {np.float64: "float64",
                  np.int32: "int32", np.int8: "int8"}[dt] and a.is_contiguous())
        else:
            ok = (isinstance(a, np.ndarray) and a.dtype == dt and a.flags.c_contiguous
                  and (a.flags.writeable or not write))
        if not ok or (shape is not None and tuple(a.shape) != tuple(shape)):
            where = "GPU tensor" if dev else "writeable host array"
            raise RMError(f"{call}: {name} must be a contiguous {np.dtype(dt).name} {where}"
                          + (f" of shape {tuple(shape)}" if shape is not None else "")
                          + f" (got {type(a).__name__} {getattr(a, 'dtype', '')} {tuple(getattr(a, 'shape', ()))})")


def _ptr(x):
    if x is None:
        return None
    if _is_torch(x):
        return ctypes.c_void_p(x.data_ptr())
    return x.ctypes.data_as(ctypes.c_void_p)


def pw_footprint(nchan: int, npole: int) -> int:
    return int(_lib.rm_pw_footprint(nchan, npole))


def work_footprint(nchan: int, npole: int, ntarget: int, ne: int) -> int:
    return int(_lib.rm_work_footprint(nchan, npole, ntarget, ne))


NBUCKET = 4


def tile_bucket(nchan: int) -> int:
    """Size bucket of a channel count (rm_tile_bucket)."""
    return int(_lib.rm_tile_bucket(nchan))


def tile_shapes(prec: int):
    """[(tile side, energies per task)] of the R-contraction shapes of a precision."""
    out = []
    for sh in range(int(_lib.rm_tile_count(prec))):
        t, e = _i32(), _i32()
        if _lib.rm_tile_shape(prec, sh, ctypes.byref(t), ctypes.byref(e)) != 0:
            raise RMError("rm_tile_shape failed")
        out.append((t.value, e.value))
    return out


class Context:
    """One librm context on a HIP device (rm_create / rm_destroy)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = _vp()
        self._check(_lib.rm_create(device, hbm_budget_bytes, ctypes.byref(h)), None)
        self.h = h
        self.device = device
        self._pw = {}
        self._inflight = {}  # ticket -> the request's host buffers, held until poll() retires it

    def _check(self, st: int, h=...):
        if st < 0:
            msg = _lib.rm_last_error(self.h if h is ... else h)
            raise RMError(f"librm status {st}: {msg.decode() if msg else ''}")
        return st

    def close(self):
        if getattr(self, "h", None):
            _lib.rm_destroy(self.h)
            self.h = None
            self._inflight.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def pw_upload(self, pw, coupling: dict | None = None) -> int:
        """Upload a synth.PartialWave (or any object with the same fields); with
        coupling = dict(cf=[lamax][n][n] multipole coefficients, r1=radius) the
        wave's channels are coupled between a and r1."""
        keep = [np.ascontiguousarray(pw.e_thr, dtype=np.float64), np.ascontiguousarray(pw.l, dtype=np.int32),
                np.ascontiguousarray(pw.target, dtype=np.int32), np.ascontiguousarray(pw.Ek, dtype=np.float64),
                np.ascontiguousarray(pw.w, dtype=np.float64)]
        n, M = int(pw.nchan), int(pw.npole)
        for name, arr, size in zip(("e_thr", "l", "target", "Ek", "w"), keep, (n, n, n, M, M * n)):
            if arr.size < size:  # the library reads size entries; spare ones are harmless
                raise RMError(f"pw_upload: {name} has {arr.size} entries, nchan = {n} and npole = {M} need {size}")
        d = PWDesc(pw.nchan, pw.npole, pw.ntarget, pw.a, pw.b, pw.z, pw.g, *[k.ctypes.data for k in keep])
        pid = _i32()
        if coupling is None:
            self._check(_lib.rm_pw_upload(self.h, ctypes.byref(d), ctypes.byref(pid)))
        else:
            cf = np.ascontiguousarray(coupling["cf"], dtype=np.float64)
            if cf.ndim != 3 or cf.shape[1:] != (pw.nchan, pw.nchan):
                raise ValueError("coupling cf must be [lamax][nchan][nchan]")
            self._check(_lib.rm_pw_upload_coupled(self.h, ctypes.byref(d), cf.shape[0], cf.ctypes.data,
                                                  float(coupling["r1"]), ctypes.byref(pid)))
        self._pw[pid.value] = (pw.nchan, pw.ntarget)
        return pid.value

    def set_propagation(self, npts: int = 3201, stab: int = 64):
        self._check(_lib.rm_set_propagation(self.h, int(npts), int(stab)))

    def propagate(self, pw_id, E, thr_guard=1e-10):
        """phi, dphi [ne][n][2n] at r = a of a coupled wave, and status."""
        E, dev = self._E(E)
        n, _ = self._pw.get(pw_id, (1, 1))
        ne = E.shape[0]
        phi = self._alloc(E, (ne, n, 2 * n), np.float64)
        dphi = self._alloc(E, (ne, n, 2 * n), np.float64)
        st = self._alloc(E, (ne,), np.int32)
        o = self._opts(FP64, 0.05, thr_guard, dev)
        self._check(_lib.rm_propagate(self.h, pw_id, _ptr(E), ne, ctypes.byref(o), _ptr(phi), _ptr(dphi), _ptr(st)))
        return phi, dphi, st

    def pw_release(self, pw_id: int):
        self._check(_lib.rm_pw_release(self.h, pw_id))
        self._pw.pop(pw_id, None)

    def _opts(self, prec, split_delta, thr_guard, dev, stream=None):
        o = Opts()
        _lib.rm_opts_default(ctypes.byref(o))
        o.prec = int(prec)
        o.split_delta = float(split_delta)
        o.thr_guard = float(thr_guard)
        o.device_ptrs = 1 if dev else 0
        if dev:
            import torch
            o.stream = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream().cuda_stream)
        return o

    def _alloc(self, like, shape, dtype):
        if _is_torch(like):
            import torch
            tdt = {np.float64: torch.float64, np.int32: torch.int32, np.int8: torch.int8}[dtype]
            return torch.empty(shape, dtype=tdt, device=like.device)
        return np.empty(shape, dtype=dtype)

    def _E(self, E):
        return _energies(E)

    def _out_shapes(self, pw_id, ne):
        """(omega, K, status) shapes of a wave's results, or Nones for an
        unknown wave (the library reports that)."""
        if pw_id not in self._pw:
            return None, None, None
        n, nt = self._pw[pw_id]
        return (ne, nt, nt), (ne, n, n), (ne,)

    def form_R(self, pw_id, E, prec=FP64, split_delta=0.05, thr_guard=1e-10):
        E, dev = self._E(E)
        n, _ = self._pw.get(pw_id, (1, 1))
        ne = E.shape[0]
        R = self._alloc(E, (ne, n, n), np.float64)
        st = self._alloc(E, (ne,), np.int32)
        o = self._opts(prec, split_delta, thr_guard, dev)
        self._check(_lib.rm_form_R(self.h, pw_id, _ptr(E), ne, ctypes.byref(o), _ptr(R), _ptr(st)))
        return R, st

    def asymptotic(self, pw_id, E, thr_guard=1e-10):
        E, dev = self._E(E)
        n, _ = self._pw.get(pw_id, (1, 1))
        ne = E.shape[0]
        fg = self._alloc(E, (ne, n, 4), np.float64)
        op = self._alloc(E, (ne, n), np.int8)
        no = self._alloc(E, (ne,), np.int32)
        st = self._alloc(E, (ne,), np.int32)
        o = self._opts(FP64, 0.05, thr_guard, dev)
        self._check(_lib.rm_asymptotic(self.h, pw_id, _ptr(E), ne, ctypes.byref(o), _ptr(fg), _ptr(op), _ptr(no),
                                       _ptr(st)))
        return fg, op, no, st

    def solve_K(self, pw_id, E, R, fg, thr_guard=1e-10):
        E, dev = self._E(E)
        n, _ = self._pw.get(pw_id, (1, 1))
        ne = E.shape[0]
        if not dev:
            R = np.ascontiguousarray(R, dtype=np.float64)
            fg = np.ascontiguousarray(fg, dtype=np.float64)
        known = pw_id in self._pw
        _check_outputs("solve_K", dev, [("R", R, (ne, n, n) if known else None, np.float64),
                                        ("fg", fg, (ne, n, 4) if known else None, np.float64)], write=False)
        K = self._alloc(E, (ne, n, n), np.float64)
        st = self._alloc(E, (ne,), np.int32)
        o = self._opts(FP64, 0.05, thr_guard, dev)
        self._check(_lib.rm_solve_K(self.h, pw_id, _ptr(E), ne, _ptr(R), _ptr(fg), ctypes.byref(o), _ptr(K),
                                    _ptr(st)))
        return K, st

    def collision_strengths(self, pw_id, E, K, thr_guard=1e-10, want_S=False):
        E, dev = self._E(E)
        n, nt = self._pw.get(pw_id, (1, 1))
        ne = E.shape[0]
        if not dev:
            K = np.ascontiguousarray(K, dtype=np.float64)
        _check_outputs("collision_strengths", dev, [("K", K, (ne, n, n) if pw_id in self._pw else None, np.float64)],
                       write=False)
        om = self._alloc(E, (ne, nt, nt), np.float64)
        S = self._alloc(E, (ne, n, n, 2), np.float64) if want_S else None
        st = self._alloc(E, (ne,), np.int32)
        o = self._opts(FP64, 0.05, thr_guard, dev)
        self._check(_lib.rm_collision_strengths(self.h, pw_id, _ptr(E), ne, _ptr(K), ctypes.byref(o), _ptr(om),
                                                _ptr(S), _ptr(st)))
        if want_S and not dev:
            S = S[..., 0] + 1j * S[..., 1]
        return om, S, st

    def run(self, pw_id, E, prec=FP64, split_delta=0.05, thr_guard=1e-10, want_K=True, out=None, stream=None):
        """Fused R -> asymptotics -> K -> Omega for a block of energies."""
        E, dev = self._E(E)
        n, nt = self._pw.get(pw_id, (1, 1))
        ne = E.shape[0]
        if out is None:
            om = self._alloc(E, (ne, nt, nt), np.float64)
            K = self._alloc(E, (ne, n, n), np.float64) if want_K else None
            st = self._alloc(E, (ne,), np.int32)
        else:
            om, K, st = out
            so, sk, ss = self._out_shapes(pw_id, ne)
            _check_outputs("run", dev, [("omega", om, so, np.float64), ("K", K, sk, np.float64),
                                        ("status", st, ss, np.int32)])
        o = self._opts(prec, split_delta, thr_guard, dev, stream)
        self._check(_lib.rm_run(self.h, pw_id, _ptr(E), ne, ctypes.byref(o), _ptr(om), _ptr(K), _ptr(st)))
        return om, K, st

    def mqdt_unphysical_K(self, pw_id, E, fnumin, prec=FP64, split_delta=0.05, thr_guard=1e-10):
        """rm_mqdt_unphysical_K: (Ku [ne][n][n], nmember [ne], status [ne])."""
        E, dev = self._E(E)
        n, _ = self._pw.get(pw_id, (1, 1))
        ne = E.shape[0]
        Ku = self._alloc(E, (ne, n, n), np.float64)
        nm = self._alloc(E, (ne,), np.int32)
        st = self._alloc(E, (ne,), np.int32)
        o = self._opts(prec, split_delta, thr_guard, dev)
        self._check(_lib.rm_mqdt_unphysical_K(self.h, pw_id, _ptr(E), ne, float(fnumin), ctypes.byref(o), _ptr(Ku),
                                              _ptr(nm), _ptr(st)))
        return Ku, nm, st

    def run_mqdt(self, pw_id, E, ieq, fnumin, iqdt=1, qetest=1e-7, prec=FP64, split_delta=0.05, thr_guard=1e-10,
                 want_K=True, stream=None):
        """rm_run_mqdt on an ascending mesh: (omega, K or None, coarse mask, status)."""
        E, dev = self._E(E)
        n, nt = self._pw.get(pw_id, (1, 1))
        ne = E.shape[0]
        om = self._alloc(E, (ne, nt, nt), np.float64)
        K = self._alloc(E, (ne, n, n), np.float64) if want_K else None
        co = self._alloc(E, (ne,), np.int8)
        st = self._alloc(E, (ne,), np.int32)
        o = self._opts(prec, split_delta, thr_guard, dev, stream)
        mq = MqdtOpts(int(ieq), int(iqdt), float(fnumin), float(qetest))
        self._check(_lib.rm_run_mqdt(self.h, pw_id, _ptr(E), ne, ctypes.byref(mq), ctypes.byref(o), _ptr(om),
                                     _ptr(K), _ptr(co), _ptr(st)))
        return om, K, co, st

    def run_noalloc(self, pw_id, E, out, prec=FP64, split_delta=0.05, thr_guard=1e-10, stream=None):
        """rm_run_noalloc: E and out = (omega, K or None, status) are device
        tensors the caller allocated; the library allocates nothing."""
        E, dev = self._E(E)
        if not dev:
            raise RMError("run_noalloc takes device tensors")
        om, K, st = out
        so, sk, ss = self._out_shapes(pw_id, E.shape[0])
        _check_outputs("run_noalloc", True, [("omega", om, so, np.float64), ("K", K, sk, np.float64),
                                             ("status", st, ss, np.int32)])
        o = self._opts(prec, split_delta, thr_guard, True, stream)
        self._check(_lib.rm_run_noalloc(self.h, pw_id, _ptr(E), E.shape[0], ctypes.byref(o), _ptr(om), _ptr(K),
                                        _ptr(st)))
        return om, K, st

    def run_batch(self, items, prec=FP64, split_delta=0.05, thr_guard=1e-10, want_K=False):
        """items: list of (pw_id, E).  All partial waves in one rm_run_batch call;
        returns a list of (omega, K or None, status) per item."""
        keep, outs = [], []
        arr = (BatchItem * max(1, len(items)))()
        dev = False
        for k, (pid, E) in enumerate(items):
            E, d = self._E(E)
            if k and d != dev:
                raise RMError("run_batch: energies must be all on the device or all on the host")
            dev = d
            n, nt = self._pw.get(pid, (1, 1))
            ne = E.shape[0]
            om = self._alloc(E, (ne, nt, nt), np.float64)
            K = self._alloc(E, (ne, n, n), np.float64) if want_K else None
            st = self._alloc(E, (ne,), np.int32)
            keep.append(E)
            outs.append((om, K, st))
            arr[k] = BatchItem(pid, _ptr(E), ne, _ptr(om), _ptr(K), _ptr(st))
        o = self._opts(prec, split_delta, thr_guard, dev)
        self._check(_lib.rm_run_batch(self.h, arr, len(items), ctypes.byref(o)))
        return outs

    def run_sum(self, pw_ids, E, prec=FP64, order=ORDER_PERMUTED, split_delta=0.05, thr_guard=1e-10):
        """Omega summed over the partial waves pw_ids (same targets), added in
        that order; returns (omega [ne][nt][nt], status [ne])."""
        E, dev = self._E(E)
        ne = E.shape[0]
        nt = self._pw.get(pw_ids[0], (1, 1))[1]
        om = self._alloc(E, (ne, nt, nt), np.float64)
        st = self._alloc(E, (ne,), np.int32)
        ids = (_i32 * len(pw_ids))(*pw_ids)
        o = self._opts(prec, split_delta, thr_guard, dev)
        self._check(_lib.rm_run_sum(self.h, ids, len(pw_ids), _ptr(E), ne, order, ctypes.byref(o), _ptr(om),
                                    _ptr(st)))
        return om, st

    # ------------------------------------------------------------ serving
    def submit(self, pw_id, E, prec=FP64, split_delta=0.05, thr_guard=1e-10, want_K=False):
        """Queue a request; returns (ticket, outputs dict).  The output arrays
        belong to the request until poll() reports it done."""
        n, nt = self._pw.get(pw_id, (1, 1))
        E, dev = _energies(E)
        if dev:
            raise RMError("submit takes host energies (the request's results come back in host memory)")
        ne = E.shape[0]
        outs = dict(omega=np.empty((ne, nt, nt)), K=np.empty((ne, n, n)) if want_K else None,
                    status=np.zeros(ne, np.int32), E=E)
        o = self._opts(prec, split_delta, thr_guard, False)
        rq = Request(pw_id, E.ctypes.data, ne, o, outs["omega"].ctypes.data,
                     outs["K"].ctypes.data if want_K else None, outs["status"].ctypes.data)
        t = _u64()
        self._check(_lib.rm_submit(self.h, ctypes.byref(rq), ctypes.byref(t)))
        self._inflight[t.value] = outs
        return t.value, outs

    def poll(self, ticket):
        """Returns None while pending, else the request's timing stats (ns)."""
        s = ReqStats()
        st = _lib.rm_poll(self.h, ticket, ctypes.byref(s))
        if st == RM_PENDING:
            return None
        self._inflight.pop(ticket, None)
        self._check(st)
        return dict(t_arrive_ns=s.t_arrive_ns, t_admit_ns=s.t_admit_ns, t_start_ns=s.t_start_ns,
                    t_done_ns=s.t_done_ns, nblocks=s.nblocks)

    def drain(self):
        self._check(_lib.rm_drain(self.h))

    # ------------------------------------------------------- graph mode
    def set_graph(self, on: bool):
        self._check(_lib.rm_set_graph(self.h, 1 if on else 0))

    def graph_stats(self):
        """(captured, replayed) stage-group graphs since the context was made."""
        c, r = ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.rm_graph_stats(self.h, ctypes.byref(c), ctypes.byref(r)))
        return c.value, r.value

    # ------------------------------------------------------ tile autotuner
    def get_tile(self, prec, bucket):
        sh = _i32()
        self._check(_lib.rm_get_tile(self.h, prec, bucket, ctypes.byref(sh)))
        return sh.value

    def set_tile(self, prec, bucket, shape):
        self._check(_lib.rm_set_tile(self.h, prec, bucket, shape))

    def tune(self, prec, pw_ids, E, reps=2, cache_path=None):
        """Times every R tile shape of prec on the waves pw_ids for the energies
        E, keeps the fastest per size bucket; returns the times [npw][nshapes] (ms)."""
        E = np.ascontiguousarray(E, dtype=np.float64)
        ids = (_i32 * len(pw_ids))(*pw_ids)
        ms = np.zeros((len(pw_ids), len(tile_shapes(prec))))
        path = cache_path.encode() if cache_path else None
        self._check(_lib.rm_tune(self.h, prec, ids, len(pw_ids), _ptr(E), E.shape[0], reps, path, _ptr(ms)))
        return ms

    def tune_load(self, cache_path):
        self._check(_lib.rm_tune_load(self.h, cache_path.encode()))

    # ---------------------------------------------------------- profiling
    def prof_enable(self, on: bool = True):
        self._check(_lib.rm_prof_enable(self.h, 1 if on else 0))

    def prof_read(self, stage: str):
        """(total_ms, launches, energies) of a stage since the last read."""
        ms, nl, ne = _d(), ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.rm_prof_read(self.h, stage.encode(), ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(ne)))
        return ms.value, nl.value, ne.value

    def prof_chunks(self, cap: int = 65536):
        """Per-chunk records since the last read: dict of arrays ms, model_flops,
        open_frac, energies (issue order)."""
        ms, fl, of = np.empty(cap), np.empty(cap), np.empty(cap)
        ne, cnt = np.empty(cap, np.int64), ctypes.c_int64()
        self._check(_lib.rm_prof_chunks(self.h, cap, _ptr(ms), _ptr(fl), _ptr(of), _ptr(ne), ctypes.byref(cnt)))
        k = cnt.value
        return dict(ms=ms[:k], model_flops=fl[:k], open_frac=of[:k], energies=ne[:k])
