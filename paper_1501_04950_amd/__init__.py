"""alpha-Moebius domain-wall propagators on MI355X (gfx950).

The compute path is the HIP library ``libdwa.so`` built from ``csrc/`` and
reached through :mod:`paper_1501_04950_amd.dwa` (a ctypes binding with the same
names as the C-ABI).  :mod:`paper_1501_04950_amd.synth` generates seeded inputs.
"""
