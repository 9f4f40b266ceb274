"""O3: brute-force full unitary, n <= 8 (oracle; test infrastructure).

Section "Circuits and gates / Basic circuits and outputs": the circuit's
unitary is the ordered product of its gates, each embedded into the full
2^n space; an amplitude <bits|U|0...0> is the entry U[bits, 0].  Embedding
here is by explicit index arithmetic over all basis states (not by the
tensordot used in O1), so the two share no contraction code.
"""
from __future__ import annotations

import numpy as np

from . import gates as G

MAX_QUBITS = 8


def embed(mat: np.ndarray, qubits, n: int) -> np.ndarray:
    """The 2^n x 2^n matrix of a k-qubit gate acting on `qubits`."""
    if n > MAX_QUBITS:
        raise ValueError("brute force limited to 8 qubits")
    k = len(qubits)
    dim = 1 << n
    full = np.zeros((dim, dim), dtype=np.complex128)
    shifts = [n - 1 - q for q in qubits]   # qubit 0 = most significant bit
    for col in range(dim):
        sub_in = 0
        for s in shifts:
            sub_in = (sub_in << 1) | ((col >> s) & 1)
        rest = col
        for s in shifts:
            rest &= ~(1 << s)
        for sub_out in range(1 << k):
            row = rest
            for j, s in enumerate(shifts):
                if (sub_out >> (k - 1 - j)) & 1:
                    row |= 1 << s
            full[row, col] += mat[sub_out, sub_in]
    return full


def unitary(circ, params) -> np.ndarray:
    n = circ.n_qubits
    params = np.asarray(params, dtype=np.float64)
    u = np.eye(1 << n, dtype=np.complex128)
    for g in circ.gates:
        u = embed(G.matrix(g, params), g.qubits, n) @ u
    return u


def bits_index(bits) -> int:
    idx = 0
    for b in bits:
        idx = (idx << 1) | int(b)
    return idx


def amplitude(circ, params, bits=None) -> complex:
    u = unitary(circ, params)
    if bits is None:
        bits = (0,) * circ.n_qubits
    return complex(u[bits_index(bits), 0])


def pauli_dense(structure) -> np.ndarray:
    m = np.array([[1.0 + 0j]])
    for s in structure:
        m = np.kron(m, G.PAULI[int(s)])
    return m


def energy(circ, params, obs) -> complex:
    psi = unitary(circ, params)[:, 0]
    re = im = 0.0
    for a, s in zip(obs.weights, obs.structures):
        v = complex(np.conj(psi) @ (pauli_dense(s) @ psi))
        re += float(a) * v.real
        im += float(a) * v.imag
    return complex(re, im)
