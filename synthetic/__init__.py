"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only draws random numbers and evaluates the analytic test
signals; it holds none of the QTT method's arithmetic (no SVD, no
convolution, no kernel sampling).  Every generator is deterministic for a
given seed and states its draw order, so the CPU oracle and the HIP path see
bit-identical inputs.
"""

from .generators import (  # noqa: F401
    WORKLOADS,
    gaussian_bumps_1d,
    scatterers_1d,
    sar_image_2d,
    batch_lines,
    diff_workload,
    paper_example1,
    paper_example2,
    paper_example3,
    closed_form_signal,
)
