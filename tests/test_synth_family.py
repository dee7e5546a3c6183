"""Partial-wave families (inputs of the sum over partial waves): the waves share
their targets, couple every target to 1..4 channels ordered by target, carry
g = 2w + 1, and are reproducible from the seed."""
import numpy as np

from paper_1909_07321_amd import synth


def test_family_shares_targets_and_orders_channels():
    E = np.linspace(0.01, 6.0, 50)
    fam = synth.partial_wave_family(77, 5, 9, (1, 4), 20, z=5.0, a=12.0, thr_range=(0.0, 4.0),
                                    pole_range=(-2.0, 60.0), avoid_energies=E, name="t")
    assert len(fam) == 5
    for w, pw in enumerate(fam):
        assert pw.ntarget == 9
        np.testing.assert_array_equal(pw.e_target, fam[0].e_target)
        assert pw.e_target[0] == 0.0 and np.all(np.diff(pw.e_target) >= 0)
        counts = np.bincount(pw.target, minlength=9)
        assert counts.min() >= 1 and counts.max() <= 4
        assert np.all(np.diff(pw.target) >= 0)
        assert pw.nchan == counts.sum() and pw.w.shape == (pw.npole, pw.nchan)
        assert pw.npole == 20 * pw.nchan and np.all(np.diff(pw.Ek) >= 0)
        assert pw.g == 2 * w + 1
        assert synth._thresholds_clear(pw.e_thr, E)
    again = synth.partial_wave_family(77, 5, 9, (1, 4), 20, z=5.0, a=12.0, thr_range=(0.0, 4.0),
                                      pole_range=(-2.0, 60.0), avoid_energies=E, name="t")
    for a_, b_ in zip(fam, again):
        np.testing.assert_array_equal(a_.w, b_.w)
        np.testing.assert_array_equal(a_.target, b_.target)
    # waves differ from each other
    assert not np.array_equal(fam[0].target, fam[1].target) or not np.array_equal(fam[0].l, fam[1].l)
