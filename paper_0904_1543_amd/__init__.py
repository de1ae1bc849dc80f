"""MI355X-native local Hamiltonian of the Daubechies-wavelet Kohn-Sham method.

The compute path lives in ``libwvl.so`` (hand-written HIP for gfx950 behind
the C ABI declared in ``include/wvl.h``).  ``paper_0904_1543_amd.lib`` is the
thin ctypes binding with the same names; ``ops`` wraps it for torch tensors;
``autograd`` adds the energy functional with its hand-written backward.
Submodules are imported lazily so that ``inputs`` can be used without a GPU.
"""

import importlib

__all__ = ["inputs", "lib", "ops", "autograd", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
