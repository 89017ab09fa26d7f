"""Even-odd Wilson fermion operator on MI355X (gfx950).

The compute path lives in the HIP library ``libwilson_eo.so`` built from
``csrc/``; ``wilson_eo`` is its ctypes binding and ``ops``/``autograd`` the
torch-facing layer.  Nothing here falls back to a CPU implementation: if the
library is missing, loading it raises.
"""
__all__ = ["inputs"]
