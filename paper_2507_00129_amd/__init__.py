"""MI355X-native Lyman-alpha pixel-pair accumulation (xi, distortion matrix,
xi gradient) behind a small C ABI (include/lya.h).

The computation runs in the HIP library ``_lib/liblya.so``; this package only
marshals arguments to it.  Build it with ``python -m paper_2507_00129_amd.build``.
"""
from .lya import (  # noqa: F401
    DeviceForests,
    Library,
    LyaError,
    load_library,
    LYA_OK, LYA_E_INVALID, LYA_E_NOMEM, LYA_E_DEVICE, LYA_E_UNSUPPORTED,
)


def differentiable_xi(*args, **kwargs):
    """torch-differentiable xi (see paper_2507_00129_amd.autograd.xi)."""
    from .autograd import xi
    return xi(*args, **kwargs)
