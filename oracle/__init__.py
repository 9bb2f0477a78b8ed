"""CPU oracle for the H^2 VIE hot path.  TEST INFRASTRUCTURE ONLY.

Plain, slow, complex128 NumPy implementations of what the HIP path computes,
written from the paper (Omar & Jiao, "O(N) iterative and O(NlogN) fast direct
VIE solvers with a minimal-rank H^2-representation"):

* kernel.py    - g(r) = exp(-jkr)/(4 pi r) (eq. (1)) and the equal-volume
                 sphere self term; brute-force dense G and Z products;
* matvec.py    - the H^2 matrix-vector product of Sec. IV.B: forward
                 transformation, coupling multiplication, backward
                 transformation, plus the full products of the inadmissible
                 blocks, followed by Z x = x + sigma k^2 V G (chi . x);
* partition.py - a plain recursive block-cluster partition (eq. (4)) used to
                 pin the generator's partition;
* krylov.py    - restarted GMRES / flexible GMRES with classical Gram-Schmidt
                 applied twice, Givens rotations and a true-residual check,
                 and GMRES-based iterative refinement; BiCGStab (the paper's
                 iterative solver, Sec. V);
* precision.py - emulation of the FP32 and BF16 hi+lo storage tiers;
* mlp.py       - the per-leaf MLP preconditioner's forward/backward/Adam.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may
import this package.  It shares no code with the HIP path or with the input
generators beyond the arrays those generators produce.

Parity status: every function here is pinned by the `-m "not gpu"` tests in
tests/test_oracle_*.py against closed forms, library routines, brute force
or invariants, except where a docstring says "parity unpinned".
"""
