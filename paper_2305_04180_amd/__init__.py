"""MI355X-native vectorized Sparrow step (arXiv 2305.04180): binding package.

The compute lives in ``libsparrow.so`` (HIP kernels for gfx950 behind a C-ABI,
declared in ``include/sparrow.h``); ``sparrow.py`` marshals arguments to it.
``inputs.py`` generates seeded synthetic workloads.
"""
