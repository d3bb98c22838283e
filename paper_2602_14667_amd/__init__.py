"""MI355X-native recursive regularised lattice Boltzmann MHD (D2Q9 + D2Q5).

The compute path is the HIP library ``librrmhd.so`` (built from ``csrc/``);
``rrmhd`` is its ctypes binding.  Importing the package loads nothing: the
binding loads the library on first use and raises if it is missing.
"""
__all__ = ["rrmhd", "inputs"]
