"""Stochastic Kraus-trajectory ensembles of noisy circuits on MI355X (gfx950).

The product path is the C-ABI library libstn.so (include/stn.h, sources in
csrc/) and the thin ctypes binding in ``binding``.  Importing this package
does not load the library; ``binding.load()`` does, and raises if it has not
been built (``python -m paper_2210_15874_amd.build``).
"""
from .binding import (OUT_DIAG, OUT_ENERGY, OUT_RHO, OUT_STATES, PLAN_AUTO, PLAN_LIGHTCONE, PLAN_SV_GATES,
                      PLAN_SV_LDS, PLAN_SV_TILED, Accum, Batch, Plan, Server, StnError, contract_many, load,
                      simulate_batch_ensemble)

__all__ = ["Plan", "Batch", "Accum", "Server", "StnError", "load", "simulate_batch_ensemble", "contract_many",
           "OUT_RHO", "OUT_DIAG",
           "OUT_ENERGY", "OUT_STATES", "PLAN_AUTO", "PLAN_SV_LDS", "PLAN_SV_TILED", "PLAN_LIGHTCONE",
           "PLAN_SV_GATES"]
