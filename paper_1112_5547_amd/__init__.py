"""MI355X-native two-component Shan-Chen lattice Boltzmann library.

Implements the multicomponent Shan-Chen BGK time step of Scarbolo et al.,
"Unified framework for a side-by-side comparison of different multicomponent
algorithms: lattice Boltzmann vs. phase field model" (Sec. 2.1) on periodic
D2Q9 and D3Q19 lattices as hand-written HIP kernels for gfx950, behind the C
ABI of include/lbm_sc.h.  This package is the thin Python binding: argument
marshalling, with PyTorch supplying device memory and streams.
"""
from ._abi import (LBM_BATCH_FUSED, LBM_BATCH_PER_LATTICE, LBM_BATCH_PERSISTENT, LBM_D2Q9,
                   LBM_D3Q19, LBM_FP32_SHIFTED, LBM_FP64, LbmError, lib)
from .batch import Batch
from .lattice import Lattice, bytes_needed, copy_bench, tiles

D2Q9, D3Q19 = LBM_D2Q9, LBM_D3Q19

__all__ = ["Lattice", "Batch", "LbmError", "lib", "tiles", "bytes_needed", "copy_bench", "D2Q9",
           "D3Q19", "LBM_FP64", "LBM_FP32_SHIFTED", "LBM_BATCH_PER_LATTICE", "LBM_BATCH_FUSED",
           "LBM_BATCH_PERSISTENT"]
