"""MI355X-native matrix-free multigrid for the Poisson problem on locally
refined hexahedral meshes (arXiv 2203.12292): the HIP library ``libmfmg.so``
and its ctypes binding ``paper_2203_12292_amd.mfmg``."""
