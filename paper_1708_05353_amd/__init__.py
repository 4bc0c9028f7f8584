"""occk: far-field occupied exchange of occ-FMM-K (arXiv:1708.05353) on MI355X.

The compute path is the HIP library ``libocck.so`` (built in-tree by
``paper_1708_05353_amd.build``) behind the C ABI declared in include/occk.h;
``paper_1708_05353_amd.occk`` is its Python binding.
"""
from .occk import (OcckError, Tree, far_K, lib, PREC_FP64, PREC_FP32, PREC_BF16X3, PREC_BF16X6,  # noqa: F401
                   RANK_FIXED, RANK_LEARNED)
