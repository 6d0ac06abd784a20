"""MI355X-native cone-beam CT projectors (TIGRE v3, arXiv 2412.10129):
Siddon and interpolated forward projectors, their exact transposes, FDK,
CGLS and OS-SART on hand-written HIP kernels for gfx950 (libctmi.so)."""
from . import _lib
from ._lib import CtmiError
from .ops import Plan, geometry_check, view_table, dot, axpby, stream_check
from .algs import (fdk, cgls, os_sart, OSSART, mlem, osem, OSEM, asd_pocs, ASDPOCS, psnr_from_sq_err, pnp_cgls,
                   save_state, load_state)
from .projector import Projector, create_pytorch_operator
from .unet import UNet

__all__ = ["Plan", "geometry_check", "view_table", "dot", "axpby", "stream_check", "fdk", "cgls", "os_sart", "OSSART", "mlem", "osem", "OSEM", "asd_pocs", "ASDPOCS",
           "psnr_from_sq_err", "Projector", "create_pytorch_operator", "CtmiError", "UNet", "pnp_cgls",
           "save_state", "load_state"]


def library():
    """The loaded libctmi (raises ImportError if it is not built)."""
    return _lib.lib()


library()
