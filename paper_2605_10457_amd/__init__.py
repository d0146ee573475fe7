"""MI355X-native emitter-centric closest-hit LiDAR ray casting (GRCA).

The hot path lives in ``libgrca.so`` (hand-written HIP for gfx950) behind the
C ABI declared in ``include/grca.h``; ``grca`` is its thin ctypes binding.
Importing this package loads nothing: the library is opened on first use and
raises if it has not been built.
"""
__all__ = ["grca", "synth"]
