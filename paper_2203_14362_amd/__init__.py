"""Canvas-based point-in-polygon selection and aggregation joins for AMD
MI355X (gfx950): HIP kernels behind the C ABI of include/spade.h, with a thin
ctypes binding (``spade.Context``)."""
from .spade import (Batch, Canvas, Context, DevicePolys, HostTable, SpadeError, Table, load_library,  # noqa: F401
                    SPADE_OK, SPADE_E_INVALID, SPADE_E_CAPACITY, SPADE_E_NOMEM,
                    SPADE_E_HIP, SPADE_E_UNSUPPORTED, SPADE_E_TOO_LARGE, EXPORTS, LIB_PATH)
