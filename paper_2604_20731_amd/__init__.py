"""MI355X-native hot path of the IGA-ADS-CRVPINN hybrid CO2 solver.

The compute path is the C-ABI library ``libcrv.so`` (hand-written HIP kernels
for gfx950) declared in ``include/crv.h``; ``paper_2604_20731_amd.crv`` is its
thin ctypes binding.  ``inputs`` draws seeded synthetic problem data.
Submodules are imported lazily so that loading the input generators never
touches the GPU library.
"""
