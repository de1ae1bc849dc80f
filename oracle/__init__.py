"""Float64 CPU oracle of the local Hamiltonian path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or execute anything in this package.  The GPU
library never does: it derives its own filters and shares no code with it.

Every function is pinned by tests under ``tests/test_oracle_*.py`` against
mathematics (closed forms, invariants, brute-force dense matrices, Fourier
identities, exact finite differences); none is "parity unpinned".
"""

from . import boundary, compress, filters, precond, wavelet  # noqa: F401
