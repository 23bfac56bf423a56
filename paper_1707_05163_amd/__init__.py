"""MI355X-native Lagrangian particle advection (HIP kernels for gfx950 behind a C ABI).

``FieldSet`` and ``ParticleSet`` load the in-tree HIP library on first use and raise
ImportError if it has not been built; nothing here computes on the CPU.
"""

__all__ = ["FieldSet", "ParticleSet", "SEED", "philox_normals", "execute_batch",
           "autotune_batch", "Surrogate", "surrogate_features", "surrogate_check"]


def __getattr__(name):
    if name in __all__:
        from . import core
        return getattr(core, name)
    raise AttributeError(name)
