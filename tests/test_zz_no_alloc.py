"""rm_run_noalloc: the fused path with its workspace in the library's fixed
device array instead of allocated memory.  Its results must equal rm_run's
bitwise (each energy's arithmetic does not depend on the chunk it rides in), on
two calls in a row, the second smaller, and it must refuse a partial wave whose
one-energy workspace exceeds the array."""
import numpy as np
import pytest

from paper_1909_07321_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def test_noalloc_equals_run():
    import torch

    from paper_1909_07321_amd import rm
    pw, E = synth.config2()
    with rm.Context(0) as ctx:
        pid = ctx.pw_upload(pw)
        calls = 0
        for prec in (rm.FP64, rm.FP32_SPLIT):
            for sel in (E[::4], E[::53]):   # 500 energies, then 38
                _say("noalloc", "fp64" if prec == rm.FP64 else "split", sel.size, "energies of", pw.nchan, "channels")
                Ed = torch.tensor(sel, dtype=torch.float64, device="cuda")
                om = torch.empty((sel.size, pw.ntarget, pw.ntarget), dtype=torch.float64, device="cuda")
                K = torch.empty((sel.size, pw.nchan, pw.nchan), dtype=torch.float64, device="cuda")
                st = torch.empty(sel.size, dtype=torch.int32, device="cuda")
                torch.cuda.synchronize()
                free0 = torch.cuda.mem_get_info()[0]
                ctx.run_noalloc(pid, Ed, (om, K, st), prec=prec)
                torch.cuda.synchronize()
                free1 = torch.cuda.mem_get_info()[0]
                ref = ctx.run(pid, Ed, prec=prec)
                torch.cuda.synchronize()
                assert torch.equal(st, ref[2]) and (st.cpu().numpy() == 0).all()
                assert torch.equal(om, ref[0]) and torch.equal(K, ref[1])
                _say(f"  bitwise equal to rm_run; device free memory {free0 >> 20} -> {free1 >> 20} MiB")
                # the process's first launches may let the HIP runtime set itself
                # up; every later call must leave the device's free memory as it was
                if calls:
                    assert free1 == free0
                calls += 1
        ctx.pw_release(pid)


def test_noalloc_coupled_wave_equals_run():
    """A coupled wave (its propagation matrices also carved from the array)."""
    import torch

    from paper_1909_07321_amd import rm
    E = np.linspace(0.2, 7.8, 96)
    pw = synth.make_partial_wave(synth.config_seed(8) + 60, 90, 20, z=5.0, a=12.0, thr_range=(0.0, 8.0),
                                 pole_range=(-2.0, 60.0), avoid_energies=E, name="noalloc-cpl")
    cp = dict(cf=synth.multipole_coefficients(synth.config_seed(8) + 60, pw.nchan), r1=30.0)
    with rm.Context(0) as ctx:
        ctx.set_propagation(801, 64)
        pid = ctx.pw_upload(pw, cp)
        for sel in (E, E[::7]):
            _say("noalloc coupled", sel.size, "energies of", pw.nchan, "channels")
            Ed = torch.tensor(sel, dtype=torch.float64, device="cuda")
            om = torch.empty((sel.size, pw.ntarget, pw.ntarget), dtype=torch.float64, device="cuda")
            K = torch.empty((sel.size, pw.nchan, pw.nchan), dtype=torch.float64, device="cuda")
            st = torch.empty(sel.size, dtype=torch.int32, device="cuda")
            ctx.run_noalloc(pid, Ed, (om, K, st))
            ref = ctx.run(pid, Ed)
            torch.cuda.synchronize()
            assert torch.equal(st, ref[2]) and (st.cpu().numpy() == 0).all()
            assert torch.equal(om, ref[0]) and torch.equal(K, ref[1])
        ctx.pw_release(pid)


def test_noalloc_refuses_oversized_wave():
    import torch

    from paper_1909_07321_amd import rm
    pw = synth.make_partial_wave(synth.config_seed(5) + 300, 3000, 1, z=5.0, a=12.0, thr_range=(0.0, 8.0),
                                 pole_range=(-2.0, 60.0), name="noalloc-big")
    assert rm.work_footprint(pw.nchan, pw.npole, pw.ntarget, 1) > rm.NOALLOC_SCRATCH_BYTES
    with rm.Context(0) as ctx:
        pid = ctx.pw_upload(pw)
        Ed = torch.tensor([1.0], dtype=torch.float64, device="cuda")
        om = torch.empty((1, pw.ntarget, pw.ntarget), dtype=torch.float64, device="cuda")
        st = torch.empty(1, dtype=torch.int32, device="cuda")
        with pytest.raises(rm.RMError, match="no-alloc scratch"):
            ctx.run_noalloc(pid, Ed, (om, None, st))
        with pytest.raises(rm.RMError):
            ctx.run_noalloc(pid, np.array([1.0]), (om, None, st))   # host energies are refused
        ctx.pw_release(pid)
