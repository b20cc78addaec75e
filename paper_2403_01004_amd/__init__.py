"""MI355X-native parabolic-operator advance (field-aligned conduction and
viscosity on a spherical shell; RKL2/RKG2 super time stepping and Backward
Euler + Jacobi PCG, cycled at the practical time step limit).

The compute path is libparadv.so (hand-written HIP for gfx950) behind the
C ABI in include/paradv.h; `paradv` is its ctypes binding.  Importing this
package loads nothing; `paradv.load()` loads the library.
"""
__all__ = ["paradv", "inputs"]
