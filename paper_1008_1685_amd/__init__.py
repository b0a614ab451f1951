"""MI355X-native 1D3V particle-in-cell hot path with radiation reaction.

The computation lives in the HIP library ``libpic.so`` (C ABI in
include/pic.h); this package only marshals arguments to it.
"""
from ._native import PicError, load  # noqa: F401
from .run import Run, make_config, workspace_bytes  # noqa: F401
