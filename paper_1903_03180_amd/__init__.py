"""SCPL video retargeting (Seam Carving with Parental Labeling) on MI355X.

The compute path is the HIP library `libscpl.so` (C ABI declared in
include/scpl.h); `paper_1903_03180_amd.scpl` is its Python binding and
`paper_1903_03180_amd.synth` draws seeded synthetic inputs.  Submodules are
imported lazily so that the input generator works without the library.
"""
__all__ = ["scpl", "synth"]
