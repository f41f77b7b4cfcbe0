"""MI355X-native CTMRG (corner transfer matrix renormalization group) library.

The computation lives in the HIP library ``libctm.so`` (C ABI in include/ctm.h);
this package only builds it (``build``) and binds it (``_binding``).
"""
from ._binding import (CTM_DOWN, CTM_LEFT, CTM_RIGHT, CTM_UP, EXPORTS, Ctm, CtmError, Queue,  # noqa: F401
                       SimpleUpdate, ctm_footprint_bytes, load, make_config)
