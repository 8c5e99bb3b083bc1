"""GPU-resident refactorization + FGMRES-IR solver for sequences of sparse KKT systems
(MI355X / gfx950).  The compute lives in libkkt.so; see kkt.py for the binding."""
from .kkt import (KKTError, Solver, default_opts, lib, PREC_FP64, PREC_MIXED, GUARD_PERTURB,  # noqa: F401
                  GUARD_FAIL, STOP_PAPER, STOP_NRBE, KKT_OK, KKT_EINVAL, KKT_ENOMEM, KKT_ESINGULAR,
                  KKT_ENOCONV, KKT_EDEVICE, KKT_ESTATE, EXPORTS, ORDER_MD, ORDER_ND,
                  IR_FGMRES, IR_RICHARDSON, IR_ERROR_FGMRES, RESID_FP64, RESID_DD, GS_CGS2, GS_DCGS2, Server,
                  refactor_batch, HyKKT)
