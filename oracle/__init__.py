"""CPU oracle for the BoxMG V-cycle — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP library: the C
tier (``bmg_oracle.c`` via ``ref``) follows the method step by step in FP64 (and
FP32 for the refinement preconditioner) in the paper's order of operations, and
the matrix tier (``dense``) restates the same objects as sparse/dense matrices
for small grids, so that each can be checked against the mathematics.
"""
