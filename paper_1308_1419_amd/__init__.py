"""tdmap: triangular-domain EDM kernels for MI355X (gfx950).

Importing the package does not load the HIP library; the first call into
``paper_1308_1419_amd.tdmap`` does, and fails loudly when it is missing.
"""
__all__ = ["synth"]
