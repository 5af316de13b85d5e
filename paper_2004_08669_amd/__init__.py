"""MI355X-native CTMRG step for q-state vector-spin (polyhedron) models.

The HIP library (libctmrg.so, C ABI in include/ctmrg.h) runs every step of the
method on the GPU; `ctmrg` is its Python binding.
"""
