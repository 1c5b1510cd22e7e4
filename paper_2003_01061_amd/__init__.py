"""MI355X-native feature-aware SPH relaxation (arXiv 2003.01061).

``paper_2003_01061_amd.binding`` wraps the C-ABI library ``libsphmesh.so``
(hand-written gfx950 HIP kernels); ``paper_2003_01061_amd.workload`` draws the
seeded synthetic inputs.  Importing the package loads neither.
"""
