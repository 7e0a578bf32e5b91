"""FP64 CPU oracle for the three-phonon linewidth path.

TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously-correct NumPy/SciPy
implementation of what the GPU library computes, written from the paper's
equations.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import it; the GPU library never does, and the oracle
imports nothing from the GPU package.
"""
