"""MI355X (gfx950) time stepper for the eigenfunction-segregation partition
method of Elliott & Ranner (arXiv 1408.2355).

The work runs in the HIP library libsegpart.so (C ABI in include/segpart.h);
``segpart`` is its ctypes binding.  Build with
``python -m paper_1408_2355_amd.build``.
"""
from .segpart import (Mesh, State, Server, SegpartError, params, solve,  # noqa: F401
                      SP_FP64, SP_MIXED, SP_MAT_M, SP_MAT_A, SP_STAGE_HEAT,
                      SP_STAGE_NODE, SP_STAGE_NORM, SP_OK, SP_ENOCONV)
