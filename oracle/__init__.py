"""CPU oracle for the tensor-network circuit contraction path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
calls this package; only the test-suite, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP library: the gate
matrices, the state-vector simulator, the tensor-network builder and the
contraction orders here are all written independently, in complex128.

Parts (each module cites the passage of the paper it follows):

* ``gates``        gate matrices and their angle derivatives;
* ``statevector``  O1: dense state vector, amplitudes, Pauli expectations,
                   weighted energies, adjoint gradient, parameter shift and
                   central finite differences;
* ``brute``        O3: the full 2^n x 2^n unitary, n <= 8;
* ``tn``           O2: an einsum-style pairwise tensor-network contraction
                   with its own network builder and sweep orders;
* ``mpo``          operators given as matrix product operators: the dense
                   matrix and the application to a state vector.
"""
from . import gates, statevector, brute, tn, mpo  # noqa: F401
