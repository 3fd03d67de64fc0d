"""MI355X implementation of the two-fluid kinetic scheme for dilute polymer
solutions (arXiv:2201.10132): Python binding of the C ABI in include/tpl.h.

Every step of the method runs in the HIP kernels of ``libtpl.so``; this
package only marshals arguments.  Importing it fails loudly when the library
has not been built.
"""
from .tpl import (TPL_BF16, TPL_FP32, TPL_FP64, TPL_NFIELDS, TPL_POLYMER, TPL_SOLVENT,  # noqa: F401
                  Batch, Mlp, TplError, Tpl, lib, lib_path, tpl_last_error)
