"""MI355X-native ensemble ODE solver with discrete-adjoint gradients.

Adaptive explicit Runge--Kutta integration (Dopri5, Tsit5, Verner 7) of very
many small independent ODE systems, one trajectory per GPU lane, with the
gradient of scalar losses through a checkpointed discrete adjoint.  The
compute lives in the HIP library ``libgradsolve.so`` built from ``csrc/``;
this package only binds it (``api``) and wraps it for autograd
(``autograd``).  ``inputs`` holds the seeded workload generators.

Submodules are imported lazily so that the input generators can be used on a
machine without a GPU or torch.
"""

__all__ = ["api", "autograd", "inputs", "build"]
