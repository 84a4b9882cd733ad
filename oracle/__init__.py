"""FP64 CPU oracle for the non-Fourier SENSE hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the tests, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` use it.  It
shares no code with the GPU library and does not import it.

Every function is pinned by a CPU test against something other than itself
(brute-force sums, the Cartesian DFT special case, the adjoint identity,
dense solves, finite differences); see ``tests/test_oracle_pins.py``.
"""
from .nfs_oracle import (  # noqa: F401
    phase,
    apply_E,
    apply_EH,
    apply_EHE,
    cg_solve,
    encode_grads,
    dense_E,
)
from .bruteforce import E_brute, EH_brute  # noqa: F401
