"""MI355X-native black-box multigrid (BoxMG) V-cycle for 2D variable-coefficient
diffusion on vertex-centred grids.

The solver itself is the HIP library declared in ``include/bmg.h``; the Python
binding lives in :mod:`paper_2502_05279_amd.boxmg` and loads the library on first
use.  :mod:`paper_2502_05279_amd.inputs` holds the seeded problem generators.
"""

__all__ = ["boxmg", "inputs", "build"]
