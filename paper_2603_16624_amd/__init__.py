"""MI355X-native ECsim particle hot path: mover, moment gather, mass-matrix apply.

Submodules are imported on demand: ``inputs`` (seeded synthetic plasmas),
``ecsim`` (the Python binding of the C-ABI library ``libecsim.so``) and
``autograd`` (the differentiable mover + moments).
"""
__all__ = ["inputs", "ecsim", "autograd"]
