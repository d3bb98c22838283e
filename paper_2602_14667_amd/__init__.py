"""MI355X-native recursive regularised lattice Boltzmann MHD (D2Q9 + D2Q5).

The compute path is the HIP library ``librrmhd.so`` (built from ``csrc/``);
``rrmhd`` is its ctypes binding.  Importing the package loads nothing: the
binding loads the library on first use and raises if it is missing.
"""
__all__ = ["rrmhd", "inputs"]

# Sources of the step kernels; their hash tags measured traffic figures so a
# figure taken on another kernel version is not reported.
KERNEL_SOURCES = ("csrc/rr_node.h", "csrc/rr_pull.h", "csrc/rr_kernels.hip")
KERNEL3D_SOURCES = ("csrc/rr_node.h", "csrc/rr_pull.h", "csrc/rr_3d.hip")
BATCH_SOURCES = ("csrc/rr_node.h", "csrc/rr_pull.h", "csrc/rr_batch.hip")


def kernel_hash(sources=KERNEL_SOURCES) -> str:
    import hashlib
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(here, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel3d_hash() -> str:
    return kernel_hash(KERNEL3D_SOURCES)


def batch_hash() -> str:
    return kernel_hash(BATCH_SOURCES)
