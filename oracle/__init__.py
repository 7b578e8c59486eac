"""CPU FP64 oracle for the D-VQLS hot path (arXiv 2604.14435).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the GPU path computes.  Only the test suite, the
package's smoke check and the benchmark's CPU-baseline leg may import it; the
product path never calls it and shares no code with it.

Modules
  pauli    -- Pauli coefficients c = Tr(P^dagger A)/N (Section II-B, Eq. (5)):
              brute force over explicit Kronecker products, and a plain FWHT;
              magnitude pruning (tau threshold / top-L) and the Frobenius error.
  circuit  -- gate-by-gate state-vector simulation of every Hadamard-test
              circuit (Section II-A/II-C) on n system qubits + 1 ancilla.
  cost     -- cost assembly from the terms (Eq. (1), Eq. (4), Section II-C
              stage iii), the dense-matrix definitions, parameter-shift and
              finite-difference gradients, gradient descent.
  linalg   -- classical solutions, fidelity, the perturbation bound (Eq. (6)),
              the pruning-accuracy study (Section III-B).
  mlp      -- FP64 reference of the warm-start MLP (forward, backward, Adam).

Parity status of each function is stated in its module docstring; every
function is pinned by a ``-m "not gpu"`` test against values the paper prints,
closed forms, invariants or brute force, except where a docstring says
"parity unpinned".
"""
