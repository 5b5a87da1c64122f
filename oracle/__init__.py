"""CPU oracle for the ENUF hot path (test infrastructure only).

``ewald``       plain FP64 Ewald sum over explicit k-vectors (C + OpenMP)
``enuf_mirror`` the ENUF gridding steps in plain numpy FP64
``dpd``         the ENUF-DPD real-space sum of Slater-smeared charges

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package; the HIP library never imports, links or calls it.
"""
