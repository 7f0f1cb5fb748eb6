"""MI355X (gfx950) PARAFAC2-ALS hot path (SPARTan, KDD'17) behind a C ABI.

The compute lives in libparafac2.so (hand-written HIP); `binding` marshals
torch device tensors into its C calls.
"""
from . import binding  # noqa: F401
from .binding import (  # noqa: F401
    Context,
    DeviceSlices,
    Model,
    Parafac2Error,
    parafac2_get_mttkrp,
    parafac2_get_q,
    parafac2_init,
    parafac2_iterate,
    parafac2_model_create,
    parafac2_project,
)
