"""Graph mode: the chunk pipeline of rm_run / rm_run_batch runs as captured HIP
graphs (one per stage group), captured once per chunk shape and replayed while
it repeats.  Each replay must give, bitwise, what direct launches give, also
with eager work of the same context between the replays."""
import numpy as np
import pytest

from paper_1909_07321_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rm():
    from paper_1909_07321_amd import rm as m
    return m


@pytest.fixture(scope="module")
def waves():
    sizes = [30, 97, 260]
    E = np.linspace(0.01, 6.0, 37)
    pws = [synth.make_partial_wave(synth.config_seed(3) + 120 + i, n, 20, z=5.0, a=12.0, thr_range=(0.0, 4.0),
                                   pole_range=(-2.0, 60.0), avoid_energies=E, name=f"graph{i}")
           for i, n in enumerate(sizes)]
    return pws, E


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replays_equal_direct(rm, waves, prec):
    pws, E = waves
    with rm.Context(0) as ctx:
        ids = [ctx.pw_upload(p) for p in pws]
        ctx.set_graph(False)
        c0, r0 = ctx.graph_stats()
        direct = ctx.run(ids[2], E, prec=prec)
        direct_b = ctx.run_batch([(i, E[k::2]) for k, i in enumerate(ids)], prec=prec, want_K=True)
        assert ctx.graph_stats() == (c0, r0)  # nothing captured with graphs off
        ctx.set_graph(True)
        for rep in range(3):
            om, K, st = ctx.run(ids[2], E, prec=prec)
            c, r = ctx.graph_stats()
            print(f"prec={prec} replay {rep}: captures {c} replays {r}", flush=True)
            for a, b in zip((om, K, st), direct):
                assert np.array_equal(a, b, equal_nan=True), rep
            if rep > 0:
                assert r > r0, "the repeated chunk shape must replay its graphs"
            r0 = r
            # eager work of the same context between replays
            ctx.set_graph(False)
            again = ctx.run(ids[0], E[::3], prec=prec)
            ctx.set_graph(True)
            assert (again[2] == 0).all()
        outs = ctx.run_batch([(i, E[k::2]) for k, i in enumerate(ids)], prec=prec, want_K=True)
        for (om, K, st), (om2, K2, st2) in zip(outs, direct_b):
            assert np.array_equal(om, om2, equal_nan=True)
            assert np.array_equal(K, K2, equal_nan=True)
            assert np.array_equal(st, st2)
        c, r = ctx.graph_stats()
        assert c > 0
        # Omega does not depend on whether K is also returned
        om_noK, K_none, st_noK = ctx.run(ids[2], E, prec=prec, want_K=False)
        assert K_none is None
        assert np.array_equal(om_noK, direct[0], equal_nan=True) and np.array_equal(st_noK, direct[2])


def test_graph_recapture_on_shape_change(rm, waves):
    """Chunks of new shapes (more energies, so the workspace grows and moves)
    recapture their graphs; going back to an old shape is correct too."""
    pws, E = waves
    with rm.Context(0) as ctx:
        pid = ctx.pw_upload(pws[1])
        blocks = [E[:7], np.linspace(0.02, 5.9, 300), E[:7], E[::2]]
        ctx.set_graph(False)
        ref = [ctx.run(pid, b, prec=1) for b in blocks]
        ctx.set_graph(True)
        for rep in range(2):
            for b, (om0, K0, st0) in zip(blocks, ref):
                om, K, st = ctx.run(pid, b, prec=1)
                print(f"rep {rep} ne={b.size}: captures/replays {ctx.graph_stats()}", flush=True)
                assert np.array_equal(om, om0, equal_nan=True) and np.array_equal(K, K0, equal_nan=True)
                assert np.array_equal(st, st0)


def test_tile_and_graph_argument_errors(rm, waves):
    pws, E = waves
    with rm.Context(0) as ctx:
        with pytest.raises(rm.RMError):
            ctx.set_tile(0, rm.NBUCKET, 0)
        with pytest.raises(rm.RMError):
            ctx.set_tile(1, 0, len(rm.tile_shapes(1)))
        with pytest.raises(rm.RMError):
            ctx.get_tile(5, 0)
        with pytest.raises(rm.RMError):
            ctx.tune(0, [12345], E[:4])  # unknown partial wave
        pid = ctx.pw_upload(pws[0])
        with pytest.raises(rm.RMError):
            ctx.tune(0, [pid], E[:4], reps=0)
        assert ctx.get_tile(0, rm.tile_bucket(pws[0].nchan)) == 0  # nothing changed
