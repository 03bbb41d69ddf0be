"""MI355X (gfx950) multi-level greedy RBF mesh deformation.

The product is the HIP library ``librbfdef.so`` behind the C ABI of ``include/rbfdef.h``;
``rbfdef`` is its ctypes binding (same function names). Build with ``__graft_entry__.build()``
or ``python -m paper_2107_13887_amd.build``.
"""
from . import rbfdef  # noqa: F401
from .rbfdef import (Context, RbfError, rbf_ctx_create, rbf_ctx_destroy, rbf_evaluate,  # noqa: F401
                     rbf_geom_create, rbf_geom_release, rbf_greedy_select, rbf_poll,
                     rbf_solve_weights, rbf_submit, rbf_volume_update, rbf_wait)
