"""MI355X-native outer-region R-matrix energy loop (PSTGF method).

The compute path lives in the HIP library ``librm.so`` (C ABI declared in
``include/rm.h``); :mod:`paper_1909_07321_amd.rm` is its Python binding and
:mod:`paper_1909_07321_amd.synth` draws seeded synthetic inputs.
"""
