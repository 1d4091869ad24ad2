"""MI355X (gfx950) complex finite-element Helmholtz solver.

The compute path is the HIP library ``libhz.so`` (C ABI: ``include/hz.h``);
this package is its Python binding (``hz``) and a torch autograd wrapper of
the adjoint gradient (``autograd``).
"""
from .hz import (Helmholtz, HzError, lib, make_opts, header_symbols, dd_alpha, node_order,  # noqa: F401
                 HZ_OK, HZ_NOT_CONVERGED, HZ_BREAKDOWN, HZ_ERR_INVALID, HZ_ERR_HIP,
                 HZ_ERR_OOM, HZ_ERR_STATE)
