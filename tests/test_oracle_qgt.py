"""Pins for the oracle's state Jacobian and geometric tensor (no GPU).

G_ij = <d_i psi|d_j psi> - <d_i psi|psi><psi|d_j psi> (section "Advanced
automatic differentiation"; QFI = 4 Re G).  Sources of truth:
* central finite differences of the state vector (h = 1e-5);
* closed forms: RX(t)|0> has G = 1/4 at every t; RX on distinct qubits
  gives G = I/4; a gate whose generator commutes with the state
  (RZ on |0>) has G = 0;
* invariants: G is Hermitian and positive semi-definite, and a slot shared
  by two gates gets the sum of both uses' derivatives;
* the paper's example ansatz (6 qubits, 3 layers of RX on every qubit with
  one shared angle per layer and a CNOT ladder) through the same checks.
"""
import math

import numpy as np
import pytest

import tcgen
from oracle import statevector as sv


def fd_jacobian(circ, p, h=1e-5):
    cols = []
    for s in range(circ.n_params):
        q = p.copy()
        q[s] += h
        a = sv.state(circ, q)
        q[s] -= 2 * h
        b = sv.state(circ, q)
        cols.append((a - b) / (2 * h))
    return np.stack(cols, axis=1)


def paper_ansatz(n=6, layers=3):
    c = tcgen.Circuit(n, layers)
    for j in range(layers):
        for i in range(n):
            c.add("rx", (i,), (j,))
        for i in range(n - 1):
            c.add("cnot", (i, i + 1))
    return c


@pytest.mark.parametrize("seed", [0, 1])
def test_jacobian_matches_finite_differences(seed):
    circ = tcgen.random_circuit(4, 18, seed, kinds=["rx", "ry", "rz", "rzz", "fsim", "cnot", "h"])
    p = np.random.default_rng(seed).uniform(-3, 3, circ.n_params)
    np.testing.assert_allclose(sv.jacobian(circ, p), fd_jacobian(circ, p), atol=1e-8)


def test_single_rx_closed_form():
    c = tcgen.Circuit(1, 1).add("rx", (0,), (0,))
    for t in (0.0, 0.3, 2.0):
        g = sv.geometric_tensor(c, np.array([t]))
        assert abs(g[0, 0] - 0.25) < 1e-14


def test_product_of_rx_is_quarter_identity_and_rz_on_zero_is_zero():
    c = tcgen.Circuit(3, 4)
    for q in range(3):
        c.add("rx", (q,), (q,))
    g = sv.geometric_tensor(c, np.array([0.4, 1.1, 2.5, 0.0]))
    np.testing.assert_allclose(g[:3, :3], np.eye(3) / 4, atol=1e-14)
    z = tcgen.Circuit(1, 1).add("rz", (0,), (0,))
    assert abs(sv.geometric_tensor(z, np.array([0.9]))[0, 0]) < 1e-14


def test_paper_ansatz_shared_slots_hermitian_psd():
    circ = paper_ansatz()
    p = np.array([0.1, 0.2, 0.3])
    g = sv.geometric_tensor(circ, p)
    np.testing.assert_allclose(g, g.conj().T, atol=1e-13)
    assert np.min(np.linalg.eigvalsh(g)) > -1e-12
    # the same tensor from the finite-difference Jacobian
    jac = fd_jacobian(circ, p)
    psi = sv.state(circ, p)
    ov = jac.conj().T @ psi
    np.testing.assert_allclose(g, jac.conj().T @ jac - np.outer(ov, ov.conj()), atol=1e-8)
    # the first layer acts on |0...0> with one shared angle: 6 independent
    # RX derivatives, so G_00 = 6 / 4
    assert abs(g[0, 0] - 1.5) < 1e-12
