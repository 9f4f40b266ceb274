"""Pins for the oracle's gate matrices (no GPU).

Each gate is checked against something other than its own formula: a matrix
exponential of its generator (scipy), algebraic identities (squares,
unitarity, truth tables), the paper's printed matrices, and numerical
derivatives.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import tcgen
from oracle import brute
from oracle import gates as G

RNG = np.random.default_rng(1234)
ANGLES = list(RNG.uniform(-7.0, 7.0, size=6)) + [0.0, math.pi, math.pi / 2]


def g1(kind, t=None):
    return tcgen.Gate(kind, (0,), (-1,) if t is not None else (),
                      (t,) if t is not None else ())


def g2(kind, *ts):
    return tcgen.Gate(kind, (0, 1), tuple(-1 for _ in ts), tuple(ts))


@pytest.mark.parametrize("kind,gen", [("rx", G.X), ("ry", G.Y), ("rz", G.Z)])
@pytest.mark.parametrize("t", ANGLES)
def test_single_qubit_rotations_are_half_angle_exponentials(kind, gen, t):
    # reading: R_G(t) = exp(-i t G / 2)
    np.testing.assert_allclose(G.matrix(g1(kind, t), []), expm(-0.5j * t * gen),
                               atol=1e-14)


@pytest.mark.parametrize("kind,gen", [("rzz", np.kron(G.Z, G.Z)),
                                      ("rxx", np.kron(G.X, G.X)),
                                      ("ryy", np.kron(G.Y, G.Y))])
@pytest.mark.parametrize("t", ANGLES)
def test_two_qubit_rotations_are_half_angle_exponentials(kind, gen, t):
    np.testing.assert_allclose(G.matrix(g2(kind, t), []), expm(-0.5j * t * gen),
                               atol=1e-14)


def test_zz_matrix_of_the_exp1_example():
    # section "Circuits and gates", exponential gates: Z (x) Z is diag(1,-1,-1,1)
    np.testing.assert_array_equal(np.kron(G.Z, G.Z).real,
                                  np.diag([1.0, -1.0, -1.0, 1.0]))


@pytest.mark.parametrize("t", ANGLES)
def test_exp1_form_relates_to_rzz(t):
    # exp(i t ZZ) (the paper's exp1 form) equals RZZ(-2t) under our reading
    np.testing.assert_allclose(expm(1j * t * np.kron(G.Z, G.Z)),
                               G.matrix(g2("rzz", -2.0 * t), []), atol=1e-14)


@pytest.mark.parametrize("t", ANGLES)
@pytest.mark.parametrize("p", ANGLES[:4])
def test_fsim_is_swap_rotation_times_controlled_phase(t, p):
    # fSim(t, p) = exp(-i t (XX + YY)/2) . diag(1, 1, 1, e^{-i p})
    h = 0.5 * (np.kron(G.X, G.X) + np.kron(G.Y, G.Y))
    ref = expm(-1j * t * h) @ np.diag([1, 1, 1, np.exp(-1j * p)])
    np.testing.assert_allclose(G.matrix(g2("fsim", t, p), []), ref, atol=1e-14)


@pytest.mark.parametrize("kind,target", [("sqrt_x", G.X), ("sqrt_y", G.Y),
                                         ("sqrt_w", (G.X + G.Y) / math.sqrt(2))])
def test_square_roots_square_to_their_gate(kind, target):
    m = G.matrix(g1(kind), [])
    np.testing.assert_allclose(m @ m, target, atol=1e-15)
    np.testing.assert_allclose(m.conj().T @ m, np.eye(2), atol=1e-15)


def test_sqrt_w_printed_form():
    # principal root read as 1/2 [[1+i, -i sqrt2], [sqrt2, 1+i]]
    m = G.matrix(g1("sqrt_w"), [])
    s2 = math.sqrt(2)
    np.testing.assert_allclose(m, 0.5 * np.array([[1 + 1j, -1j * s2],
                                                  [s2, 1 + 1j]]), atol=1e-15)


def test_clifford_identities_and_truth_tables():
    h = G.matrix(g1("h"), [])
    s = G.matrix(g1("s"), [])
    np.testing.assert_allclose(h @ h, np.eye(2), atol=1e-15)
    np.testing.assert_allclose(s @ s, G.Z, atol=1e-15)
    np.testing.assert_allclose(h @ G.Z @ h, G.X, atol=1e-15)
    cx = G.matrix(g2("cnot"), [])
    # control = qubits[0] (most significant): |10> -> |11>, |11> -> |10>
    for col, row in [(0, 0), (1, 1), (2, 3), (3, 2)]:
        e = np.zeros(4)
        e[col] = 1
        assert np.argmax(np.abs(cx @ e)) == row
    np.testing.assert_array_equal(G.matrix(g2("cz"), []).real,
                                  np.diag([1.0, 1, 1, -1]))


@pytest.mark.parametrize("kind", ["rx", "ry", "rz", "rzz", "rxx", "ryy", "fsim"])
def test_angle_derivatives_match_numerical_derivatives(kind):
    nq, na = tcgen.GATE_ARITY[kind]
    ts = list(RNG.uniform(-3, 3, size=na))
    h = 1e-6
    for which in range(na):
        g = tcgen.Gate(kind, tuple(range(nq)), (-1,) * na, tuple(ts))
        tp = list(ts)
        tp[which] += h
        tm = list(ts)
        tm[which] -= h
        gp = tcgen.Gate(kind, g.qubits, g.params, tuple(tp))
        gm = tcgen.Gate(kind, g.qubits, g.params, tuple(tm))
        num = (G.matrix(gp, []) - G.matrix(gm, [])) / (2 * h)
        np.testing.assert_allclose(G.dmatrix(g, [], which), num, atol=1e-9)


def test_user_operator_2x_plus_3z():
    # section "Basic circuits and outputs": 2X + 3Z is [[3, 2], [2, -3]]
    m = 2 * brute.pauli_dense([1]) + 3 * brute.pauli_dense([3])
    np.testing.assert_array_equal(m.real, [[3, 2], [2, -3]])


def test_dense_pauli_sum_printed_matrix():
    # section "Expectations of Hamiltonians via operator_expectation":
    # X0 X1 - Z0 - Z1, printed as a 4x4 matrix (the printed matrix ends in 2;
    # the code literal next to it has a garbled last row)
    m = brute.pauli_dense([1, 1]) - brute.pauli_dense([3, 0]) - \
        brute.pauli_dense([0, 3])
    np.testing.assert_array_equal(m.real, [[-2, 0, 0, 1], [0, 0, 1, 0],
                                           [0, 1, 0, 0], [1, 0, 0, 2]])
    assert np.all(m.imag == 0)
