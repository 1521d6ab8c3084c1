"""MI355X-native megakernel and wavefront path tracing (libptmi).

`scenes` holds the seeded synthetic scene generators; `ptmi` is the binding
of the HIP library (it raises ImportError when the library is not built).
"""
from . import scenes  # noqa: F401

__all__ = ["scenes"]
