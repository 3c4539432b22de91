"""Dark-siren hierarchical population log-likelihood on MI355X (gfx950).

The GPU path lives in ``libdsl.so`` (HIP kernels behind a C ABI declared in
``include/dsl.h``); ``paper_2605_23538_amd.binding`` is its thin ctypes
binding and ``paper_2605_23538_amd.synth`` generates seeded inputs.  Importing
the package loads nothing: the binding is imported on first attribute access.
"""
_LAZY = ("DarkSirenLikelihood", "LogLFunction", "load_library", "DSLError")


def __getattr__(name):
    if name in _LAZY:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
