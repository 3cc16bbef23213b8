"""MI355X (gfx950) unstructured S_N transport sweep.

Modules: ``snx`` (binding of the HIP library libsnx.so), ``inputs`` (seeded
synthetic problems), ``build`` (in-tree hipcc build).
"""
__all__ = ["snx", "inputs", "build"]
