"""MI355X-native FAST-HALS (PL-NMF hot path): C-ABI library + thin binding.

``Plan`` (dense or CSR A) runs FAST-HALS sweeps on one GPU; ``Mlp`` is the
fold-in warm-start network.  The compiled library is libplnmf.so in this
directory (build with ``__graft_entry__.build()``).
"""
from ._lib import NativeLibraryMissing, NmfError, lib  # noqa: F401


def __getattr__(name):
    if name in ("Plan", "Matrix", "Mlp"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
