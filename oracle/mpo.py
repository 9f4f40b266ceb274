"""Operators given as matrix product operators (oracle; test infrastructure).

Section "Expectations of Hamiltonians via operator_expectation" (MPO input)
and section "QuOperator and QuVector": a matrix product operator is

    M[i_1 ... i_n ; j_1 ... j_n] = sum over the bond indices b_1 ... b_{n-1}
                                   of prod_k T_k[b_{k-1}, b_k, i_k, j_k],

with b_0 and b_n of dimension one (row index i_k, column index j_k, the
out-edge before the in-edge as in the paper's QuOperator convention); the
section "QuOperator as the operator to be measured" measures <psi|M|psi>.

Here a site tensor is a numpy array of shape (D_left, D_right, 2, 2).  The
two functions below are that sum written out two ways: ``dense`` builds the
2^n x 2^n matrix (small n), ``apply`` applies M to a state vector site by
site, carrying the open bond index.
"""
from __future__ import annotations

import numpy as np


def check(tensors, n_qubits=None):
    if n_qubits is not None and len(tensors) != n_qubits:
        raise ValueError("one site tensor per qubit")
    for k, t in enumerate(tensors):
        t = np.asarray(t)
        if t.ndim != 4 or t.shape[2:] != (2, 2):
            raise ValueError(f"site {k}: shape (Dl, Dr, 2, 2) expected")
        if k == 0 and t.shape[0] != 1:
            raise ValueError("the first site has a left bond of dimension 1")
        if k == len(tensors) - 1 and t.shape[1] != 1:
            raise ValueError("the last site has a right bond of dimension 1")
        if k > 0 and t.shape[0] != np.asarray(tensors[k - 1]).shape[1]:
            raise ValueError(f"bond {k} dimensions do not match")


def dense(tensors) -> np.ndarray:
    """The matrix: for every right bond value r of the sites so far, the
    partial operator sum_l partial[l] (x) T_k[l, r]."""
    check(tensors)
    partial = [np.ones((1, 1), dtype=np.complex128)]
    for t in tensors:
        t = np.asarray(t, dtype=np.complex128)
        dl, dr = t.shape[:2]
        partial = [sum(np.kron(partial[l], t[l, r]) for l in range(dl)) for r in range(dr)]
    return partial[0]


def apply(psi: np.ndarray, tensors) -> np.ndarray:
    """M psi for psi held as a (2,)*n array (axis q = qubit q)."""
    n = psi.ndim
    check(tensors, n)
    acc = psi[None, ...]                       # (bond, q_0, ..., q_{n-1})
    for k, t in enumerate(tensors):
        t = np.asarray(t, dtype=np.complex128)
        # contract the left bond and the in-edge of site k
        acc = np.tensordot(t, acc, axes=([0, 3], [0, k + 1]))
        # axes now (right bond, out-edge k, q_0..q_{k-1}, q_{k+1}..); put the
        # out-edge back at qubit k's place
        acc = np.moveaxis(acc, 1, k + 1)
    return acc[0]


def expectation(psi: np.ndarray, tensors) -> complex:
    return complex(np.vdot(psi, apply(psi, tensors)))
