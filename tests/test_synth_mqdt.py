"""The quantum-defect workload has the structure its description states: the
highest target 0.6 Ry above the next, every other channel open across the
mesh, the top target's channels closed there with effective quantum numbers
from about 7.9 to 158, no pole of eq. (rmatrix) within 0.9 Ry of the mesh,
and few runs of equal member set."""
import numpy as np

from paper_1909_07321_amd import synth


def test_quantum_defect_workload_structure():
    pw, E, ieq, fnumin = synth.config_mqdt()
    assert (pw.nchan, pw.npole, E.size, ieq) == (1500, 60000, 2000, 8)
    assert np.all(np.diff(E) > 0)
    et = np.sort(pw.e_target)
    top = et[-1]
    assert abs(top - et[-2] - 0.6) < 1e-12
    assert abs(E[0] - (top - 0.4)) < 1e-12 and abs(E[-1] - (top - 1e-3)) < 1e-12
    eps = E[:, None] - pw.e_thr[None, :]
    top_ch = pw.e_thr == top
    assert (eps[:, ~top_ch] > 0).all()  # every other channel open across the mesh
    assert (eps[:, top_ch] < 0).all()
    nu = pw.z / np.sqrt(-eps[:, top_ch])
    assert abs(nu.min() - pw.z / np.sqrt(0.4)) < 1e-9 and abs(nu.max() - pw.z / np.sqrt(1e-3)) < 1e-9
    assert np.abs(pw.Ek[:, None] - E[None, :]).min() > 0.9  # R smooth across the mesh
    assert abs(fnumin - np.sqrt(pw.z * pw.a)) < 1e-12
    # member count per energy (open, or closed with nu >= max(fnumin, l + 0.1)): few runs
    numin = np.maximum(fnumin, pw.l + 0.1)
    member = (eps > 0) | (pw.z / np.sqrt(np.abs(eps)) >= numin[None, :])
    runs = 1 + np.count_nonzero(np.diff(member.sum(axis=1)))
    assert 1 <= runs <= 5


def test_smaller_quantum_defect_workloads_keep_the_structure():
    for n, ppc in ((16, 12), (24, 20), (60, 20)):
        pw, E, _, _ = synth.config_mqdt(n, ppc, 50)
        top = pw.e_target.max()
        eps = E[:, None] - pw.e_thr[None, :]
        assert (eps[:, pw.e_thr != top] > 0).all() and (eps[:, pw.e_thr == top] < 0).all()
