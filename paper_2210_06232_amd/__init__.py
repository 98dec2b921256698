"""EI-FP (exponential-integrator Fourier pseudospectral) time stepping for 3-D Maxwell's
equations on one MI355X.  The compute path is the HIP library ``libeifp.so`` built from
``csrc/``; ``eifp`` holds its thin Python binding (imported lazily so that the input
generators can be used without a GPU)."""
__all__ = ["inputs"]
