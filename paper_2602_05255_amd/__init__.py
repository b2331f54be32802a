"""lrx: batched low-rank determinant and Pfaffian updates on MI355X (gfx950).

The compute path is the C-ABI library ``liblrx.so`` (HIP kernels); the Python
side only marshals arguments.  Import ``paper_2602_05255_amd.lrx`` for the
binding; this package initialiser loads nothing so that the input generators
can be imported on machines without the built library.
"""
__all__ = ["inputs"]
