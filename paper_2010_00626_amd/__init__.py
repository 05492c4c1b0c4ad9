"""MI355X-native kappa-cycle multigrid (Avnat & Yavneh) for the 2D rotated
anisotropic diffusion equation.  The compute path lives in the HIP library
``libkcycle.so`` (C-ABI declared in ``include/kcycle.h``); the Python modules
here only marshal arguments.  Submodules are imported on demand so that
``inputs`` and ``model`` stay usable without a GPU or torch."""

__all__ = ["inputs", "model", "kcycle", "autograd", "autotune"]
