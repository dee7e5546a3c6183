"""Sum over partial waves (rm_run_sum): Omega summed over the waves of one
collision problem, in the order given.  It must equal, bitwise, the sum of
rm_run over each wave taken in that order, whatever the chunk order, and match
the oracle's per-wave results summed."""
import numpy as np
import pytest

import oracle
from paper_1909_07321_amd import synth

from _metrics import gate, omega_elementwise, stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1909_07321_amd import rm
    c = rm.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def family():
    E = np.linspace(0.01, 6.0, 37)
    fam = synth.partial_wave_family(synth.config_seed(6) + 1, 4, 6, (1, 3), 30, z=5.0, a=12.0,
                                    thr_range=(0.0, 4.0), pole_range=(-2.0, 60.0), avoid_energies=E, name="tsum")
    return fam, E


def test_sum_equals_waves_added_in_order(ctx, family):
    from paper_1909_07321_amd import rm
    fam, E = family
    ids = [ctx.pw_upload(p) for p in fam]
    alone = [ctx.run(i, E, prec=rm.FP64, want_K=False)[0] for i in ids]
    ref = np.zeros_like(alone[0])
    for om in alone:
        ref = ref + om
    for order in (rm.ORDER_WAVE, rm.ORDER_PERMUTED):
        om, st = ctx.run_sum(ids, E, prec=rm.FP64, order=order)
        assert (st == 0).all()
        assert np.array_equal(om, ref), order
    # a different wave order is a different (equally valid) rounding order
    om_r, _ = ctx.run_sum(ids[::-1], E, prec=rm.FP64)
    np.testing.assert_allclose(om_r, ref, rtol=1e-14, atol=0)
    for i in ids:
        ctx.pw_release(i)


def test_sum_matches_oracle(ctx, family):
    fam, E = family
    ids = [ctx.pw_upload(p) for p in fam]
    om, st = ctx.run_sum(ids, E)
    ref = np.zeros_like(om)
    cond = np.ones(E.size)
    for p in fam:
        r = oracle.Oracle(p).run(E, want_K=False)
        assert (r["status"] == 0).all()
        ref += r["omega"]
        cond = np.maximum(cond, np.nan_to_num(r["cond"], nan=1.0))
    g = gate(cond)
    err = omega_elementwise(om, ref)
    print(f"sum over {len(fam)} waves: Omega elementwise {stats(err)}, max cond {cond.max():.1e}")
    assert (err <= g).all()
    assert np.allclose(om, np.transpose(om, (0, 2, 1)), rtol=1e-12, atol=0)
    for i in ids:
        ctx.pw_release(i)


def test_sum_device_pointers_and_flags(ctx, family):
    import torch

    from paper_1909_07321_amd import rm
    fam, E = family
    ids = [ctx.pw_upload(p) for p in fam]
    # one energy exactly on a pole of wave 2: that wave flags it, so the sum does
    Ex = np.sort(np.concatenate([E[:10], [fam[2].Ek[fam[2].Ek > 0.5][0]]]))
    om_h, st_h = ctx.run_sum(ids, Ex)
    Ed = torch.tensor(Ex, dtype=torch.float64, device="cuda")
    om_d, st_d = ctx.run_sum(ids, Ed)
    assert np.array_equal(om_d.cpu().numpy(), om_h, equal_nan=True)
    assert np.array_equal(st_d.cpu().numpy(), st_h)
    k = int(np.nonzero(Ex == fam[2].Ek[fam[2].Ek > 0.5][0])[0][0])
    assert st_h[k] & rm.PT_POLE and np.isnan(om_h[k]).all()
    assert (np.delete(st_h, k) == 0).all()
    for i in ids:
        ctx.pw_release(i)


def test_sum_rejects_different_targets(ctx, family):
    from paper_1909_07321_amd import rm
    fam, E = family
    other = synth.make_partial_wave(5, 40, 10, z=5.0, a=12.0, thr_range=(0.0, 4.0), pole_range=(-2.0, 60.0))
    ids = [ctx.pw_upload(fam[0]), ctx.pw_upload(other)]
    assert other.ntarget != fam[0].ntarget
    with pytest.raises(rm.RMError):
        ctx.run_sum(ids, E)
    for i in ids:
        ctx.pw_release(i)


def test_sum_with_uncoupled_targets_and_chunk_records(ctx):
    """Waves of very different sizes where some targets have no channel in a
    wave (their Omega rows and columns are zero in that wave): the sum matches
    the oracle, both chunk orders give the same bits, and the per-chunk profile
    records cover every (wave, energy) point."""
    from paper_1909_07321_amd import rm
    E = np.linspace(0.01, 8.0, 41)
    fam = synth.partial_wave_family(synth.config_seed(7) + 1, 4, 20, [(0, 1), (0, 2), (0, 4), (1, 4)], 30, z=5.0,
                                    a=12.0, thr_range=(0.0, 6.0), pole_range=(-2.0, 60.0), avoid_energies=E,
                                    name="timb")
    assert any(np.bincount(p.target, minlength=p.ntarget).min() == 0 for p in fam)
    ids = [ctx.pw_upload(p) for p in fam]
    ref = np.zeros((E.size, fam[0].ntarget, fam[0].ntarget))
    cond = np.ones(E.size)
    for p in fam:
        r = oracle.Oracle(p).run(E, want_K=False)
        assert (r["status"] == 0).all()
        ref += r["omega"]
        cond = np.maximum(cond, np.nan_to_num(r["cond"], nan=1.0))
    outs = {}
    for order in (rm.ORDER_WAVE, rm.ORDER_PERMUTED):
        ctx.prof_chunks()
        ctx.prof_enable(True)
        om, st = ctx.run_sum(ids, E, prec=rm.FP64, order=order)
        ctx.prof_enable(False)
        ch = ctx.prof_chunks()
        for s_ in ("rform", "nearpole", "asym", "ksolve", "somega", "chunk"):
            ctx.prof_read(s_)
        assert (st == 0).all()
        assert ch["energies"].sum() == len(fam) * E.size and (ch["ms"] > 0).all()
        assert ((ch["open_frac"] >= 0) & (ch["open_frac"] <= 1)).all()
        outs[order] = om
    assert np.array_equal(outs[rm.ORDER_WAVE], outs[rm.ORDER_PERMUTED])
    err = omega_elementwise(outs[rm.ORDER_WAVE], ref)
    print(f"uncoupled-target family: Omega elementwise {stats(err)}", flush=True)
    assert (err <= gate(cond)).all()
    for i in ids:
        ctx.pw_release(i)
