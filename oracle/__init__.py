"""FP64 oracle for the ADMM-consensus Gaussian-splatting training step.

TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this package; the product path
never does.  It shares no code with the GPU implementation: the rasterizer is
plain C (``orc.c``, per-pixel brute force in FP64), the optimiser and the
consensus step are plain NumPy in FP64 (``admm.py``), the structural
similarity term of the loss is NumPy in FP64 (``ssim.py``), the scene
splitting is plain Python (``split.py``), and the tile-binning reference is a
stable sort (``binning.py``).

Every function says which passage of the paper it follows.  Pinned by the
``-m "not gpu"`` tests (closed forms, invariants, library routines, finite
differences); see the individual docstrings.
"""
from .raster import (Camera, RasterConfig, project, render, backward, sh_basis,  # noqa: F401
                     quat_rotation, l1_loss_and_grad, FLAG_NAMES, load_library)
from .admm import (adam_admm, adaptive_rho, consensus, consensus_full, penalty_groups,  # noqa: F401
                   rescale_duals, residual_sums, scaled_lagrangian, unscaled_lagrangian)
from .binning import bin_reference  # noqa: F401
from . import split, ssim  # noqa: F401
