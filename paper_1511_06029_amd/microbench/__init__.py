"""Microbenchmarks of the device the kernels are measured against.

``python -m paper_1511_06029_amd.microbench`` builds ``mfma_f64_rate.hip``
for gfx950 (in-tree, into ``microbench/_build``) and runs it: the
register-only rate of the FP64 matrix instructions, with the operand
pattern of the fused-pair core-step kernel, printed as one JSON line.
"""
