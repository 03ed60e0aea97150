"""MI355X FDLB solver for the simplified Enskog-Shakhov model (arXiv 2211.16933).

Thin Python binding of libelb.so (include/elb.h).  Every step of the method runs in the
library's HIP kernels; this module only marshals arguments.  PyTorch provides the device
workspace and the stream.  The library must be built (python -m
paper_2211_16933_amd.build); importing the solver without it raises.
"""
from .binding import (  # noqa: F401
    ELB_OK, ELB_EINVAL, ELB_ENOMEM, ELB_EHIP, ELB_ENONFINITE, ELB_ESTATE, ELB_EUNSUPPORTED,
    BC_PERIODIC, BC_EQUILIBRIUM, PR_CONST, PR_ENSKOG, FP64, FP32, FP32_MIXED, CHI_SET, CHI_RETFM,
    ElbError, Params, Solver, BatchSolver, lib, library_path, quadrature, derived, workspace_bytes,
    supported_q, params_from_workload, mlp_param_count, mlp_norm_count, mlp_workspace_bytes,
    projection, mlp_normaliser, closure_sample, mlp_forward, mlp_loss, mlp_backward, mlp_adam,
    mlp_round, mlp_loss_noalloc, lift, closure_lift,
)
