"""FP64 CPU oracle for the QTT denoising-convolution pipeline.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of the method of Chertock, Leonard, Tsynkov and Utyuzhnikov,
"Denoising Convolution Algorithms and Applications to SAR Signal
Processing" (arXiv 2301.13339), written with numpy/LAPACK in float64.  Only
the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product path (the HIP library and its Python binding) never
does, and shares no code with it.

Modules
-------
``tt``        TT-SVD (Algorithm 1), Full (Algorithm 3), TT-rounding, QTT maps.
``conv``      discrete convolution (2.2), DFT route (Section 2), sinc kernel
              (3.1)/(7.2)/(7.3) and its Toeplitz generator.
``pipeline``  the composed pipeline (Algorithm 2 with an exact convolution
              and TT-rounding), the error metric (7.1).
``rsvd``      range finder and randomized SVD (Algorithms 4 and 5).
``ttm``       TT-SVD and max-rank TT-RSVD for mode sizes other than 2.
``grads``     gradients of the convolution + reconstruction loss.
``qfft``      QTT-FFT / QTT-iFFT (radix-2 stages with rounding), Hadamard
              product and the QTT-FFT convolution route (Algorithm 2, Step 3).

Readings of passages that are ambiguous or garbled are listed in each
function's docstring.
"""

from . import tt, conv  # noqa: F401
