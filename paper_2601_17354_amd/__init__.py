"""MI355X (gfx950) differentiable tile-based Gaussian splatting.

The hot path of PocketGS's training operator T (arXiv 2601.17354): EWA
projection, tile binning with a 64-bit (tile, depth) key radix sort,
front-to-back compositing with the forward replay trace S = {id, C_in, alpha},
the backward that replays it, and the index-mapped scatter of gradients to
the canonical parameter buffer.  All of it runs in hand-written HIP kernels
behind the C ABI of include/pocketgs.h (libpocketgs.so, built in-tree by
`python -m paper_2601_17354_amd.build`); this package only marshals
arguments and owns buffers through PyTorch.
"""

from ._lib import LIB_PATH, load  # noqa: F401

__all__ = ["LIB_PATH", "load"]
