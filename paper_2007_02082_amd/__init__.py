"""MI355X (gfx950) IPCS + BCE-IB finite-element time step.

The compute path is the HIP library libibfe.so (C ABI in include/ibfe.h); this
package only builds it and binds it.  Importing the package does not load the
library; `load()` (or creating a Plan/Solver) does and raises if it is missing.
"""
from ._lib import (FIELD_PHI, FIELD_UIB, FIELD_USTAR, FLAG_DU, FLAG_F, FLAG_P,  # noqa: F401
                   FLAG_HANG, FLAG_PDIR, OP_ADVDIFF, OP_DIV, OP_GRAD, OP_INTERP, OP_MASS, OP_SPREAD,
                   OP_STIFF, REQ_DONE, REQ_FAILED, REQ_QUEUED, REQ_RUNNING, SIGNATURES,
                   Batcher, IbfeError, Plan, Server, Solver, inputs_from_case, load, request_footprint)
