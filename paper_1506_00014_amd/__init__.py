"""Log-polar Radon transform R, back-projection R# and FBP on AMD MI355X (gfx950).

The operators run in hand-written HIP kernels behind the C-ABI library libradonlp.so
(include/radonlp.h); this package binds them to PyTorch tensors.  Importing the package
does not load the library; the first plan does, and fails loudly if it is missing.
"""

__all__ = ["RadonPlan", "radon_fwd", "radon_adj", "radon_transpose", "fbp", "radon_bp_lp", "fbp_lp", "RadonFn", "radon",
           "RadonAdjFn", "back_project",
           "RaggedBatch"]


def __getattr__(name):
    if name in __all__:
        from . import api

        return getattr(api, name)
    raise AttributeError(name)
