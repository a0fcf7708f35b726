"""CPU FP64 oracle for randomized POD (test infrastructure only).

This package is the slow, plain reference that the GPU library is checked
against. Only the test-suite, the smoke entry point and the CPU-baseline leg
of the benchmark may import it; the product path (the HIP library and its
Python binding) never does, and the two share no code.

Contents
--------
philox   Philox4x32-10 counter-based generator and the Box-Muller map that
         turns it into the Gaussian sketch (Sec. 4.2: N(0,1) entries).
pod      O1: deterministic POD by the thin SVD of the snapshot matrix
         (Sec. 4.1, the SVD equation), plus the method of snapshots and a
         streaming TSQR route for large inputs.
rpod     O2: randomized POD, Alg. 1 of Sec. 4.2 (stable form with
         re-orthonormalisation after every product), and the literal form.
metrics  sign-invariant comparison metrics (principal angles, sigma errors).
energy   the energy of the leading modes and the rank rule (Sec. 4.1).
reconstruct  reduced-order fields (Sec. 4) and the relative L2 error of
         time-averaged fields (Sec. 5).
center   fluctuation snapshots (Sec. 4.1): each snapshot minus the time
         average of its parameter's block of columns.
warm     the learned warm start (an extension of Alg. 1, not in the paper):
         network forward, loss, analytic gradient and Adam step, the bank
         Grams and targets, the predicted subspace and the warm-started
         rPOD with its residual check.

Parity status: every function here is pinned by a CPU test against a closed
form, a published known-answer vector, brute force or a theorem's bound.
"""
