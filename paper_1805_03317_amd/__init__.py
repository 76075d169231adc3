"""MI355X-native Subsampling SMC hot path for Bayesian GLMs.

The compute path is the HIP library built from csrc/ (C ABI declared in
include/subsmc.h); `binding` marshals arguments to it. Importing this package
does not load the library; the first call into `binding` does, and raises if
the library has not been built.
"""
