"""Filter / group-by / aggregate queries on lightweight-compressed columns,
run by hand-written HIP kernels on MI355X (gfx950).  See include/ccq.h for
the C-ABI; ``ccq`` is its Python binding."""
from . import ccq  # noqa: F401
from .ccq import CcqError, Context, Plan, Result, Table, plan_check, to_device  # noqa: F401
