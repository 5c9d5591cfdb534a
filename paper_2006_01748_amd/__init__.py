"""MI355X (gfx950) library for the explicit finite-volume step of the anisotropic,
heterogeneous Gatenby-Gawlinski model (Mascia, Pera, Simeoni; Section 2, eq. (3)).

The compute path is the HIP library ``libggfv.so`` behind the C ABI of
``include/ggfv.h`` (and ``include/ggfv3.h`` for the three-dimensional form);
this package is its thin binding.  Importing the package does
not load the library: the first ``Context`` does, and it raises if the library
was not built (``python -m paper_2006_01748_amd.build``).
"""
from ._binding import (  # noqa: F401
    Context, Context3, Batch, GGFVError, Params, Diag, lib, exported_names, front_speed, diagnostics_noalloc,
    GGFV_OK, GGFV_EINVAL, GGFV_ENOMEM, GGFV_EHIP, GGFV_ESTATE, GGFV_EUNSTABLE,
    GGFV_F32, GGFV_F64, GGFV_F32C, GGFV_HOST, GGFV_DEVICE,
)
