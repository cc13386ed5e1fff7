"""MI355X (gfx950) range guard: batched pointer validation and guarded kernels over a
device-resident allocation table (the protected memory model of AgileOS, arXiv 2606.06697).

The compute path is libagile_guard.so (hand-written HIP kernels behind a C ABI, see
``include/agile_guard.h``); ``guard`` binds it, ``embedding`` puts the guarded gather and its
scatter-add backward behind ``torch.autograd.Function``, ``serving`` runs the multi-client
request loop.
"""
from . import guard  # noqa: F401
from .guard import *  # noqa: F401,F403
from . import embedding  # noqa: F401
