"""MI355X-native Downstream tracking + two-track vertexing (arXiv:2503.13092).

``ds`` is the binding of the HIP library (include/ds.h); ``synth`` generates
seeded synthetic events; ``serve`` is the continuous-batching request loop.
"""
