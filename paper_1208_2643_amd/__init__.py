"""MI355X-native nonlinear FAS multigrid time stepper for the modified phase
field crystal equation (both convex-splitting schemes of Baskaran et al.).

Submodules: ``api`` (PyTorch-facing stepper), ``_lib`` (ctypes binding of
libmpfc.so), ``inputs`` (seeded synthetic initial data), ``build`` (hipcc
build of the library).  Nothing is imported eagerly, so ``inputs`` can be
used without a GPU or a built library.
"""
__all__ = ["api", "inputs", "build"]
