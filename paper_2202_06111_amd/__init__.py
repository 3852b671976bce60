"""MI355X-native graph-construction path of the graph-based invariant set (GIS)
algorithm (Decardi-Nelson & Liu, arXiv 2202.06111).

The compute path lives in the HIP library libgis.so (paper_2202_06111_amd/csrc,
C-ABI declared in include/gis.h); `paper_2202_06111_amd.gis` is the thin
ctypes binding over it and `paper_2202_06111_amd.workloads` describes the
seeded synthetic workloads.  Importing the package loads nothing.
"""
__all__ = ["gis", "workloads"]
