"""Pins for the oracle's MPO operators (no GPU).

Sources of truth, none of which is ``oracle.mpo`` itself:
* the paper's printed values: the dense matrix of X0 X1 - Z0 - Z1 (section
  "Expectations of Hamiltonians via operator_expectation", dense input;
  its printed matrix, last entry 2) and <Z0 Z1> = -1 for the QuOperator
  Z (x) Z measured after X on qubit 0 (section "QuOperator as the operator
  to be measured");
* the dense Pauli sum built by Kronecker products in O3 (``brute``): the
  TFIM MPO's matrix must equal it entry by entry;
* the Pauli-sum energies and adjoint gradients of O1 on random circuits;
* a closed form: on |0...0> the TFIM energy is j (n - 1).
"""
import numpy as np
import pytest

import tcgen
from oracle import brute, mpo
from oracle import statevector as sv

X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)


def site(*ops_by_bond, dl, dr):
    """A site tensor from (l, r, 2x2 operator) triples."""
    t = np.zeros((dl, dr, 2, 2), dtype=np.complex128)
    for l, r, op in ops_by_bond:
        t[l, r] = op
    return t


def test_paper_dense_matrix_of_x0x1_minus_z0_minus_z1():
    # H = X (x) X + (-Z) (x) I + I (x) (-Z) through a bond of dimension 3
    t0 = site((0, 0, X), (0, 1, -Z), (0, 2, I2), dl=1, dr=3)
    t1 = site((0, 0, X), (1, 0, I2), (2, 0, -Z), dl=3, dr=1)
    printed = np.array([[-2, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0], [1, 0, 0, 2]], dtype=float)
    np.testing.assert_array_equal(mpo.dense([t0, t1]), printed)


def test_paper_quoperator_zz_after_x_is_minus_one():
    ops = [site((0, 0, Z), dl=1, dr=1), site((0, 0, Z), dl=1, dr=1)]
    c = tcgen.Circuit(2, 0).add("x", (0,))
    psi = sv.run(c, np.zeros(0))
    assert abs(mpo.expectation(psi, ops) - (-1.0)) < 1e-15


@pytest.mark.parametrize("n,g,j", [(1, 0.7, 1.0), (2, 1.0, 1.0), (3, 0.6, -1.3), (5, 1.2, 1.0),
                                   (7, 0.5, 0.8)])
def test_tfim_mpo_dense_equals_pauli_sum(n, g, j):
    obs = tcgen.tfim_mpo(n, g, j)
    pauli = tcgen.tfim_zz_x(n, g)
    want = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for w, s in zip(pauli.weights, pauli.structures):
        coeff = j if np.count_nonzero(s == 3) == 2 else w
        want += coeff * brute.pauli_dense(s)
    np.testing.assert_allclose(mpo.dense(obs.mpo), want, atol=1e-14)


def test_apply_matches_dense_on_random_mpos():
    """Random complex site tensors with uneven bonds (1, 3, 2, 4, 1): the
    site-by-site application equals the dense matrix times the vector."""
    rng = np.random.default_rng(3)
    dims = [1, 3, 2, 4, 2, 1]
    ts = [rng.normal(size=(dims[k], dims[k + 1], 2, 2)) +
          1j * rng.normal(size=(dims[k], dims[k + 1], 2, 2)) for k in range(5)]
    psi = rng.normal(size=(2,) * 5) + 1j * rng.normal(size=(2,) * 5)
    got = mpo.apply(psi, ts).reshape(-1)
    want = mpo.dense(ts) @ psi.reshape(-1)
    np.testing.assert_allclose(got, want, atol=1e-12)


def test_tfim_mpo_on_zero_state_closed_form():
    n, g, j = 9, 0.8, 1.1
    psi = sv.zero_state(n)
    assert abs(mpo.expectation(psi, tcgen.tfim_mpo(n, g, j).mpo) - j * (n - 1)) < 1e-13


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mpo_energy_and_gradient_equal_the_pauli_sum(seed):
    n, layers = 8, 3
    circ = tcgen.chain_ladder(n, layers)
    p = tcgen.draw_angles(seed, (circ.n_params,)).astype(np.float64)
    g = 0.5 + 0.25 * seed
    e_mpo = sv.energy(circ, p, tcgen.tfim_mpo(n, g))
    e_ps = sv.energy(circ, p, tcgen.tfim_zz_x(n, g))
    assert abs(e_mpo - e_ps) < 1e-12
    em, gm = sv.energy_grad(circ, p, tcgen.tfim_mpo(n, g))
    ep, gp = sv.energy_grad(circ, p, tcgen.tfim_zz_x(n, g))
    assert abs(em - ep) < 1e-12
    np.testing.assert_allclose(gm, gp, atol=1e-11)


def test_planted_wrong_site_order_fails():
    """A mistake the pins must see: applying the sites in reverse order
    (the tensors of a non-symmetric operator) changes M psi."""
    rng = np.random.default_rng(5)
    dims = [1, 2, 3, 1]
    ts = [rng.normal(size=(dims[k], dims[k + 1], 2, 2)) for k in range(3)]
    psi = rng.normal(size=(2, 2, 2)) + 0j
    want = mpo.dense(ts) @ psi.reshape(-1)
    rev = [np.transpose(t, (1, 0, 2, 3)) for t in ts[::-1]]
    assert np.max(np.abs(mpo.apply(psi, rev).reshape(-1) - want)) > 1e-3
