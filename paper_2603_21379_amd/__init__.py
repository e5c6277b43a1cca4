"""tkmi: randomized (H-)Tucker decomposition on MI355X.

The compute path is libtkmi.so (hand-written HIP kernels for gfx950 behind a
C ABI, see include/tkmi.h); `binding` marshals torch tensors into it and
`tucker` chains the entry points into the Sub-R-HOSVD / Sub-R-RtL-HT
pipelines.  Importing this package does not load the library; the first
call does, and raises if it has not been built.
"""
__all__ = ["binding", "tucker"]
