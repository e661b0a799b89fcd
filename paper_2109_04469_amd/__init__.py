"""MI355X-native explicit 1D3V electrostatic PIC/MCC particle step.

The method is the six-step cycle of arXiv:2109.04469 (Sec. 2). The compute
path is libpic.so (hand-written HIP for gfx950) behind the C ABI declared in
include/pic.h; this package only marshals arguments to it and uses PyTorch
for device memory and streams.
"""
from . import capi  # noqa: F401
from .capi import PicError  # noqa: F401


def __getattr__(name):
    # torch is imported lazily so that the C ABI can be inspected without it
    if name in ("Discharge", "Batch", "Mlp", "step_many", "selftest_philox", "selftest_sqrt",
                "selftest_copy", "mlp_forward_static"):
        from . import discharge

        return getattr(discharge, name)
    raise AttributeError(name)
