"""Element tensors in the tensor representation A^K = A^0 : G_K on AMD MI355X (gfx950).

* ``capi``     -- ctypes binding of libffc_hip.so (the C-ABI in include/ffc_hip.h)
* ``forms``    -- Form / Batch / compute_geometry over torch CUDA tensors
* ``meshgen``  -- seeded synthetic meshes and coefficient fields (inputs only)
"""
__all__ = ["capi", "forms", "meshgen"]


def __getattr__(name):
    if name in ("Form", "Batch", "compute_geometry"):
        from . import forms

        return getattr(forms, name)
    raise AttributeError(name)
