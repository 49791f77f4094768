"""MI355X (gfx950) finite element cell kernels and CSR assembly.

The compute path is ``libfe.so`` (hand-written HIP, see ``csrc/``) behind the
C ABI of ``include/fe.h``; this package is its thin Python binding.
"""
from ._lib import FeError, FeLibraryError, load  # noqa: F401
from .api import (  # noqa: F401
    Assembly,
    MeshView,
    fe_assemble_csr,
    fe_cell_kernels,
    fe_form_prepare,
    fe_get_device_status,
    fe_tabulate,
    form_desc,
)
