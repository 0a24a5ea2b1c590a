"""FP64 CPU oracle for the DISK sparse kernel complex.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything here; the
product library never calls into it, and this package imports nothing from the
product (it shares no kernels, helpers, tables or constants with it).  Inputs
come from ``synth`` (seeded generators that contain none of the method's
arithmetic).

What it computes, following "DISK: Differentiable Sparse Kernel Complex for
Efficient Spatially-Variant Convolution" (Wu, Cao, Huo; ICLR 2026):

* ``sparse``  - bilinear read, one sparse layer (Eq. 2), the nested chain
                (Eq. 3 / Eq. 4) and the impulse response (Eq. 10);
* ``loss``    - normalised MSE, PSNR, Charbonnier (Eq. 11);
* ``adjoint`` - gradients of the loss w.r.t. every offset, weight and the input
                (the end-to-end differentiation of Sec. 4.1);
* ``adam``    - Adam with linear learning-rate decay and the optimisation loop
                (Sec. 5.1 implementation paragraph);
* ``init``    - radial initialisation (Eq. 6), sparse-sampling initialisation
                (Eq. 7), random initialisation (Sec. 4.2);
* ``interp``  - filter-space interpolation (Eq. 8, Eq. 9);
* ``svfilter``- the spatially varying sparse chain (Sec. 4.3);
* ``dense``   - dense convolution (Eq. 1), uniform and spatially varying, used
                as the quality reference;
* ``net``     - the learned initialiser's conv/MLP network evaluated in FP64
                on BF16-rounded operands, with its gradients.

Everything is plain numpy in float64, looping over taps and vectorised over
pixels; no blocking, fusion or reordering beyond the definitions.

Pins: every function is checked in ``tests/test_oracle_*.py`` against closed
forms, invariants, library routines (scipy, torch CPU) or brute force.  Parity
that no pin fixes is stated as "parity unpinned" in the function's docstring.
"""
