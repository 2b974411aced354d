"""MI355X (gfx950) implementation of the differentiable Randers-Finsler
fast-sweeping eikonal solve (arXiv 2603.00035): HIP kernels behind the C ABI
in include/eik.h, with a thin PyTorch binding. Importing the package does not
load the library; ``paper_2603_00035_amd.eikonal`` does."""

__all__ = ["eikonal"]
