"""CPU oracle (test infrastructure, not product code).

Plain, slow, FP64 numpy implementation of the fast spectral Boltzmann
collision operator of Dimarco, Loubere, Narski and Rey (Sections 3.2-3.3 of
the paper), of its conservation projection and of the FKS transport shift.
It exists to check the HIP path: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code
with the HIP library and never imports it.

Parity status of each function is stated in its docstring; the pins live in
``tests/test_oracle_pins.py``.
"""
from .fks_oracle import *  # noqa: F401,F403
from . import fks_oracle2d  # noqa: F401  (two-dimensional Maxwell molecules)
from . import fks_oracle_bgk  # noqa: F401  (BGK with the conservative discrete Maxwellian)
from . import fks_oracle_dealias  # noqa: F401  (zero-padded, de-aliased variant of the fast form)
