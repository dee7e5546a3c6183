"""The C-ABI library loads and exports every function include/rm.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1909_07321_amd", "librm.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rm_[A-Za-z_0-9]+)\s*\(", src)))


def test_header_parsed():
    names = declared_functions()
    for must in ["rm_create", "rm_form_R", "rm_asymptotic", "rm_solve_K", "rm_collision_strengths", "rm_submit",
                 "rm_poll"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="librm.so not built")
def test_binding_lists_every_symbol():
    from paper_1909_07321_amd import rm
    assert sorted(rm.EXPORTS) == declared_functions()


def test_oracle_not_linked_into_library():
    # the product library must not depend on the oracle
    if not os.path.exists(LIB):
        pytest.skip("librm.so not built")
    data = open(LIB, "rb").read()
    assert b"rmo_" not in data and b"librmo" not in data


@pytest.mark.skipif(not os.path.exists(LIB), reason="librm.so not built")
def test_tile_shape_table():
    # host-only queries of the R tile shapes (no device call)
    from paper_1909_07321_amd import rm
    assert [rm.tile_bucket(n) for n in (1, 64, 65, 192, 193, 512, 513, 16384)] == [0, 0, 1, 1, 2, 2, 3, 3]
    for prec in (0, 1):
        shapes = rm.tile_shapes(prec)
        assert shapes[0] == (32, 4)  # the default shape
        assert len(set(shapes)) == len(shapes) >= 2
        for tile, eb in shapes:
            assert tile in (16, 32, 64) and 1 <= eb <= 8
    assert rm.tile_shapes(7) == []


def test_mqdt_option_defaults():
    """rm_mqdt_opts_default: every point coarse (the direct result), the unphysical S
    interpolated, no fnumin floor, the paper's qetest of 1e-7."""
    from paper_1909_07321_amd import rm
    o = rm.MqdtOpts()
    rm._lib.rm_mqdt_opts_default(ctypes.byref(o))
    assert (o.ieq, o.iqdt, o.fnumin, o.qetest) == (1, 1, 0.0, 1e-7)


def test_binding_fails_loudly_without_the_library():
    """No fallback: importing the binding without librm.so raises."""
    import subprocess
    import sys

    env = dict(os.environ, RM_LIB=os.path.join(ROOT, "no_such_dir", "librm.so"))
    r = subprocess.run([sys.executable, "-c", "from paper_1909_07321_amd import rm"], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0 and "ImportError: librm.so not built" in r.stderr


@pytest.mark.skipif(not os.path.exists(LIB), reason="librm.so not built")
def test_create_without_a_device_names_the_failed_call():
    """rm_create on a host without a HIP device returns RM_E_DEVICE and no
    context; rm_last_error(NULL) names the failed HIP call and HIP's text."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a HIP device is present")
    from paper_1909_07321_amd import rm
    h = ctypes.c_void_p()
    assert rm._lib.rm_create(0, 0, ctypes.byref(h)) == rm.RM_E_DEVICE and h.value is None
    msg = rm._lib.rm_last_error(None).decode()
    assert msg.startswith("rm_create(device 0): hipSetDevice: ") and len(msg) > len("rm_create(device 0): hipSetDevice: ")
    with pytest.raises(rm.RMError, match="hipSetDevice"):
        rm.Context(0)


@pytest.mark.skipif(not os.path.exists(LIB), reason="librm.so not built")
def test_binding_checks_what_it_hands_over():
    """The binding refuses energies and caller-owned outputs that the library
    would misread or write past (host-side checks; no device call)."""
    import numpy as np
    import torch

    from paper_1909_07321_amd import rm
    E, dev = rm._energies([0.1, 0.2, 0.3])
    assert E.dtype == np.float64 and E.flags.c_contiguous and not dev
    with pytest.raises(rm.RMError, match="1-D"):
        rm._energies(np.zeros((2, 3)))
    for bad in (torch.zeros(4, dtype=torch.float64), torch.zeros(4, dtype=torch.float32)):  # not GPU tensors
        with pytest.raises(rm.RMError, match="float64 GPU tensor"):
            rm._energies(bad)
    ne, n, nt = 5, 4, 2
    good = [("omega", np.empty((ne, nt, nt)), (ne, nt, nt), np.float64),
            ("K", None, (ne, n, n), np.float64),
            ("status", np.empty(ne, np.int32), (ne,), np.int32)]
    rm._check_outputs("run", False, good)
    rm._check_outputs("run", False, [(a, b, None, d) for a, b, _, d in good])  # unknown wave: shape unchecked
    ro = np.empty(ne, np.int32)
    ro.setflags(write=False)
    for name, arr in [("omega", np.empty((ne, nt, nt), np.float32)),      # wrong dtype
                      ("omega", np.empty((ne - 1, nt, nt))),               # too short
                      ("omega", np.empty((ne, nt, 2 * nt))[:, :, ::2]),    # not contiguous
                      ("status", ro)]:                                     # read-only
        outs = [(a, arr if a == name else b, s, d) for a, b, s, d in good]
        with pytest.raises(rm.RMError, match=f"run: {name} must be"):
            rm._check_outputs("run", False, outs)
    with pytest.raises(rm.RMError, match="omega must be a contiguous float64 GPU tensor"):
        rm._check_outputs("run", True, good)  # host arrays beside device energies
    rm._check_outputs("solve_K", False, [("R", ro, (ne,), np.int32)], write=False)  # inputs may be read-only
    with pytest.raises(rm.RMError, match="solve_K: fg must be"):
        rm._check_outputs("solve_K", False, [("fg", np.empty((ne, n, 2)), (ne, n, 4), np.float64)], write=False)


@pytest.mark.skipif(not os.path.exists(LIB), reason="librm.so not built")
def test_upload_checks_field_sizes_before_any_device_call():
    """A wave whose arrays disagree with nchan / npole is refused by the binding
    (the library would read past them); the check needs no device."""
    import dataclasses

    import numpy as np

    from paper_1909_07321_amd import rm, synth
    pw, _ = synth.config1()
    ctx = rm.Context.__new__(rm.Context)  # no rm_create: the refusal comes first
    ctx.h, ctx._pw = None, {}
    for field, bad in [("l", pw.l[:-1]), ("Ek", pw.Ek[:-1]), ("w", pw.w[:, :-1])]:
        with pytest.raises(rm.RMError, match=f"pw_upload: {field} has"):
            ctx.pw_upload(dataclasses.replace(pw, **{field: bad}))
    assert np.asarray(pw.w).shape == (pw.npole, pw.nchan)


def test_every_context_call_refuses_a_null_context():
    """Each entry point that takes a context returns RM_E_ARG for a null one,
    through the wrapper that keeps exceptions from the C caller, before any
    device call (runs without a GPU)."""
    from paper_1909_07321_amd import rm
    text = open(os.path.join(ROOT, "include", "rm.h")).read()
    names = sorted(set(re.findall(r"rm_status\s+(rm_\w+)\s*\(\s*(?:const\s+)?rm_ctx\s*\*", text)))
    assert len(names) >= 28, names
    zero = {ctypes.c_double: 0.0, ctypes.c_float: 0.0}
    for name in names:
        fn = getattr(rm._lib, name)
        assert fn.argtypes, f"{name}: binding sets no argument types"
        args = [zero.get(t, None if (t in (ctypes.c_void_p, ctypes.c_char_p) or hasattr(t, "_type_")
                                     and not isinstance(t._type_, str)) else 0) for t in fn.argtypes]
        assert fn(*args) == rm.RM_E_ARG, name
