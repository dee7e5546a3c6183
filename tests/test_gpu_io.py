"""The file path end to end: partial waves written as H.DAT files, read by the
library, run on the GPU (Omega summed over the waves) and written as OMEGA.
Results must equal, bitwise, the same waves uploaded directly."""
import numpy as np
import pytest

from paper_1909_07321_amd import synth

import _fortran as F

pytestmark = pytest.mark.gpu


def test_hdat_to_omega(tmp_path):
    from paper_1909_07321_amd import rm
    E = np.linspace(0.01, 6.0, 40)
    fam = synth.partial_wave_family(synth.config_seed(6) + 9, 3, 5, (1, 3), 20, z=3.0, a=10.0,
                                    thr_range=(0.0, 4.0), pole_range=(-2.0, 50.0), avoid_energies=E, name="io")
    # H.DAT000 holds the target and the first wave, H.DAT001/002 one wave each; NELC = 7, NZ = 10
    enat = fam[0].e_target - 0.8
    files = []
    for k, pw in enumerate(fam):
        data = b""
        if k == 0:
            data += F.hdat_target(7, 10, 0, 2, enat, np.arange(5) % 2, np.full(5, 2), pw.a, 0.0,
                                  np.zeros((0, 3)), [])
        counts = np.bincount(pw.target, minlength=pw.ntarget)
        data += F.hdat_symmetry(k, 0, k % 2, counts, pw.l, np.zeros((2, pw.nchan, pw.nchan)), pw.Ek, pw.w,
                                more2=int(k + 1 < len(fam)))
        p = tmp_path / f"H.DAT{k:03d}"
        p.write_bytes(data)
        files.append(str(p))
    tgt, syms = rm.read_hdat(files[0], files[1:])
    assert len(syms) == len(fam)
    with rm.Context(0) as ctx:
        ids_file = [ctx.pw_upload(s["pw"]) for s in syms]
        # the same waves directly, with the weights the file implies (J coupling, g = 2J + 1 with 2J = k)
        direct = [synth.PartialWave(p.nchan, p.npole, p.ntarget, p.a, p.b, p.z, float(k + 1), p.e_target, p.l,
                                    p.target, p.Ek, p.w) for k, p in enumerate(fam)]
        ids_direct = [ctx.pw_upload(p) for p in direct]
        om_f, st_f = ctx.run_sum(ids_file, E)
        om_d, st_d = ctx.run_sum(ids_direct, E)
        assert (st_f == 0).all() and np.array_equal(st_f, st_d)
        assert np.array_equal(om_f, om_d)
    out = tmp_path / "OMEGAU"
    rm.write_omega(str(out), tgt["nz"], tgt["nelc"], tgt["isat"], tgt["lat"], tgt["enat"] - tgt["enat"][0], E, om_f,
                   formatted=False)
    recs = F.read_records(out.read_bytes())
    ntr = 5 * 4 // 2
    assert len(recs) == 4 + E.size
    first = np.frombuffer(recs[4], "<f8")
    assert first.size == ntr + 1 and first[0] == E[0] / 9.0
    assert first[1] == om_f[0, 0, 1] and first[-1] == om_f[0, 3, 4]
