"""FP64 CPU oracle for the differentiable particle-mesh forward model and its adjoint.

TEST INFRASTRUCTURE ONLY: used by tests/, by the smoke check and by the benchmark's
CPU-baseline leg. The product (the HIP library and its binding) never imports it.
"""
from . import cosmology, lbfgs, mesh, model, stats  # noqa: F401
