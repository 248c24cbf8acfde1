"""MI355X-native global SPAI iterations (MR / CG / LOMR with sparse matrix iterates)
and the SPAI-preconditioned CG solve, as a HIP library (libspai.so) with a thin
Python binding.

Submodules: ``spai`` (binding of the C ABI in include/spai.h), ``build`` (hipcc
build of the library), ``workloads`` (seeded synthetic inputs).  Importing the
package loads nothing; ``spai.load()`` loads the library and raises if it is missing.
"""
__all__ = ["spai", "build", "workloads"]
