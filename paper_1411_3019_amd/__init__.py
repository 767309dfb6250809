"""MI355X-native molecular dynamics on implicit surfaces (RATTLE + Langevin).

The computation lives in the HIP library libmd.so (C ABI: include/md.h);
`md` is its Python binding.
"""
from . import md  # noqa: F401
from .md import MDError, Params, Pool, System, footprint  # noqa: F401
