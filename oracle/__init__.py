"""Plain FP64 CPU oracle of the MUJICA hot path (arXiv 2604.26823).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference against which the HIP implementation is checked.  Only the test
suite, the smoke check in ``__graft_entry__`` and the CPU-baseline leg of
``bench.py`` may import or run it; the product path never does, and it shares
no code with the HIP library or its Python binding (the seeded input
generators are the only module both sides use, and they hold none of the
method's arithmetic).

Modules, each following the paper's notation:

* ``cosmology``  - background, linear/second-order growth, BBKS P(k),
                   FastPM kick/drift factors (paper section 2.2.1, item 2).
* ``fourier``    - real-FFT conventions and k-space multiplier operators.
* ``cic``        - cloud-in-cell paint / readout and their derivatives.
* ``model``      - white noise -> 2LPT -> KDK PM -> RSD -> bias, selection
                   -> masked Gaussian chi^2 + prior; hand VJP and JVP.
* ``philox``     - Philox4x64-10 counter-based generator and the draws built
                   on it (Salmon et al. 2011).
* ``projection`` - z-score + clip/reset projection P (paper section 2.3.1).
* ``rom``        - rank-order matching, real and Fourier space (section 2.3.2).
* ``lbfgs``      - projected L-BFGS with backtracking line search
                   (section 2.3.1; Nocedal & Wright two-loop recursion).

Floating point is FP64 throughout; integer work is exact.
"""
