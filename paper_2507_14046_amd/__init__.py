"""MI355X (gfx950) library for the per-frame DIP fitting iteration of D2IP
(arXiv 2507.14046): 3D residual U-Net forward from a fixed noise input, the
linearised sensitivity operator J, the data-fit loss, J^T, the network
backward and Adam, with parameters carried from frame to frame.

The compute lives in libd2ip.so (hand-written HIP kernels behind the C-ABI of
include/d2ip.h); this package only marshals arguments.  The library is loaded
on first use (``load()``, any Context or query) and that raises if it is not
built: there is no other execution path.
"""
from . import _lib
from ._lib import D2ipError, LIB_PATH
from ._lib import load
from .context import Context, ModuleFit, check_launches, module_param_count, param_count, workspace_bytes

__all__ = ["Context", "ModuleFit", "module_param_count", "check_launches", "param_count", "workspace_bytes", "D2ipError", "LIB_PATH", "load"]
