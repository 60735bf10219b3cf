"""MI355X-native BTTB gravity/magnetic operators and joint RRCG inversion.

Implements the hot path of Vatankhah, Renaut, Huang, Mickus, Gharloghi, "Large-scale
focusing joint inversion of gravity and magnetic data with Gramian constraint"
(arXiv:2112.15562): the per-depth-layer BTTB products y = A m and z = A^T r computed
through BCCB embeddings with FFT2 (Sec. 2.7.1), and the joint RRCG iteration with L1
reweighting and the Gramian coupling (Sec. 2.4-2.8).  All arithmetic runs in the HIP
library ``libbttb.so`` (C ABI: ``include/bttb.h``); importing this package fails if the
library is not built.
"""
import os as _os

from . import _lib
from ._lib import BTTBError, MAX_TRANSFORM

if not _os.path.exists(_lib.LIB_PATH):  # no fallback path: fail loudly without the HIP library
    raise ImportError(f"{_lib.LIB_PATH} is not built; run `python paper_2112_15562_amd/build.py`")

from .operator import GRAVITY, MAGNETIC, Group, Operator, pointer_array, prism_kernels  # noqa: E402
from .autograd import BTTBFunction, BTTBTransposeFunction, ForwardModel  # noqa: E402
from .rrcg import JointRRCG, JointRRCGGroup  # noqa: E402
from .scan import lambda_scan  # noqa: E402

__all__ = ["Operator", "Group", "pointer_array", "prism_kernels", "GRAVITY", "MAGNETIC", "BTTBFunction", "BTTBTransposeFunction",
           "ForwardModel", "JointRRCG", "JointRRCGGroup", "lambda_scan", "BTTBError", "MAX_TRANSFORM"]
