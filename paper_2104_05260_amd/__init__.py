"""MI355X (gfx950) HSMA hot path: Python binding of the C-ABI library.

The binding only marshals arguments; every step of the method runs in the
HIP kernels of libhsma.so.  Importing works without a GPU; plan creation
needs one (HSMA_ERR_NO_DEVICE otherwise).
"""
from .hsma import (  # noqa: F401
    HSMAError, Params, Plan, HostPlan, Server, MD, ReplicaEnsemble, lib_path, load_library, solid_harmonics, hilbert_key,
    STATUS, GEOM_3D, GEOM_2D, FP64, FP32C,
)
