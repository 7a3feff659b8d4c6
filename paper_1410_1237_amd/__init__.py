"""MI355X-native synchronous parallel Louvain (Lu, Halappanavar, Kalyanaraman,
"Parallel Heuristics for Scalable Community Detection").

The compute path lives in ``liblouvain.so`` (HIP kernels for gfx950 behind a
C ABI declared in ``include/louvain.h``); ``louvain`` is a thin ctypes binding
over it.  ``graphs`` makes seeded synthetic inputs.
"""
