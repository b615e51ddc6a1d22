"""MI355X (gfx950) rejection sampler for the truncated-KdV Gibbs measure.

Implements the data-parallel hot path of N. J. Moore & B. Foerster, "In search
of rogue waves: a novel proposal distribution for parallelized rejection
sampling of the truncated KdV Gibbs measure" (arXiv 2411.16952): batched
rejection sampling on the energy sphere S^{2K-1} with the paper's anisotropic
Gaussian proposal (and the uniform proposal as the baseline).

The compute path is the C-ABI library ``libtkdv.so`` (``include/tkdv.h``),
hand-written HIP for gfx950; ``paper_2411_16952_amd.tkdv`` is its ctypes
binding.  ``paper_2411_16952_amd.workloads`` holds the seeded parameter
points of the benchmark configurations (no arithmetic of the method).
"""
