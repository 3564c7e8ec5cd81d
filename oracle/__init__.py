"""Plain FP64 CPU oracle of the per-patch CTU+CT MHDTVD update.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product path never imports it.
It shares no code with the HIP library; the two meet only through the seeded
input generators (``paper_1701_07452_amd.inputs``), which hold none of the
method's arithmetic.
"""
from .oracle import (  # noqa: F401
    OracleParams,
    OracleSim,
    build_oracle,
    default_params,
    eigensystem,
    floor_state,
    hll_flux,
    line_fluxes,
    phys_flux,
)
