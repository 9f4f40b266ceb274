"""Pins for the oracle's circuits, expectations and gradients (no GPU).

Sources of truth, none of which is the oracle itself:
* worked examples of the paper (values it prints, or derive by hand from
  its examples: sections "Basic circuits and outputs", "Batched VQE",
  "QuOperator and QuVector");
* closed forms (GHZ, Bell, Hadamard layer, product states under RX, the
  one-layer forms of the two chain ansatze);
* invariants (unit norm, exact zeros of the gradient);
* brute force over full unitaries for n <= 8 (O3) and agreement of the
  three independent simulators O1, O2, O3;
* the exact parameter-shift rule and central finite differences for the
  adjoint gradient.
"""
import cmath
import json
import math
import os

import numpy as np
import pytest

import tcgen
from oracle import brute, tn
from oracle import statevector as sv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def close(a, b, tol):
    return abs(complex(a) - complex(b)) <= tol


# ---------------------------------------------------------------- paper examples

def test_paper_h_cnot_rx_state():
    # section "Basic circuits and outputs": H(0), CNOT(0,1), RX(0.2) on q1;
    # by hand: [cos .1, -i sin .1, -i sin .1, cos .1] / sqrt 2
    with open(os.path.join(GOLDEN, "paper_examples.json")) as f:
        ref = json.load(f)["h_cnot_rx02_state"]
    c = tcgen.Circuit(2, 0).add("h", (0,)).add("cnot", (0, 1)) \
        .add("rx", (1,), fixed=(0.2,))
    want = np.array([complex(*z) for z in ref["value"]])
    for got in (sv.state(c, []), brute.unitary(c, [])[:, 0]):
        np.testing.assert_allclose(got, want, atol=5e-7)
    np.testing.assert_allclose(sv.state(c, []),
                               np.array([math.cos(.1), -1j * math.sin(.1),
                                         -1j * math.sin(.1), math.cos(.1)]) / math.sqrt(2),
                               atol=1e-15)


def test_paper_zz_after_x_is_minus_one():
    # section "QuOperator as the operator to be measured": X(0), <Z0 Z1> = -1
    c = tcgen.Circuit(2, 0).add("x", (0,))
    obs = tcgen.pauli_string(2, z=(0, 1))
    assert close(sv.energy(c, [], obs), -1.0, 1e-15)
    assert close(brute.energy(c, [], obs), -1.0, 1e-15)
    assert close(tn.energy(c, [], obs), -1.0, 1e-15)


def test_paper_mps_input_111_then_x0():
    # section "QuVector as the input state": |111>, X(0), <Z0> = 1
    c = tcgen.Circuit(3, 0).add("x", (0,))
    psi = np.zeros((2, 2, 2), np.complex128)
    psi[1, 1, 1] = 1
    out = sv.run(c, [], psi)
    assert close(sv.pauli_expectation(out, [3, 0, 0]), 1.0, 1e-15)


def test_paper_batched_vqe_toy():
    # section "Batched VQE": RX(w0) q0, CNOT, RX(w1) q1, <Z0 Z1>.
    # By hand f = cos(w1): the CNOT maps Z0 Z1 back to Z1, whose value
    # after RX(w1) on |0> is cos w1; df/dw0 = 0, df/dw1 = -sin w1.
    with open(os.path.join(GOLDEN, "paper_examples.json")) as f:
        ref = json.load(f)["batched_vqe_toy"]
    c = tcgen.Circuit(2, 2).add("rx", (0,), (0,)).add("cnot", (0, 1)) \
        .add("rx", (1,), (1,))
    obs = tcgen.pauli_string(2, z=(0, 1))
    for w, fv in zip(ref["W"], ref["f"]):
        e, g = sv.energy_grad(c, w, obs)
        assert abs(e - fv) < 5e-8
        assert abs(e - math.cos(w[1])) < 1e-14
        np.testing.assert_allclose(g, [0.0, -math.sin(w[1])], atol=1e-14)


def test_paper_quoperator_all_ones_contraction():
    # section "QuOperator and QuVector": n1, n2 (2x2x2), n3 (2x2) of ones,
    # n1[2]-n2[2], n2[1]-n3[0]; operator (out n1[0], n2[0]; in n1[1], n3[1])
    # applied to the product of two all-ones vectors gives [16]*4.
    ones = lambda *s: np.ones(s, np.complex128)  # noqa: E731
    ts = [tn.T(ones(2, 2, 2), (0, 1, 2), ()), tn.T(ones(2, 2, 2), (3, 4, 2), ()),
          tn.T(ones(2, 2), (4, 5), ()), tn.T(ones(2), (1,), ()),
          tn.T(ones(2), (5,), ())]
    arr, labels = tn.contract_in_order(ts)
    assert sorted(labels) == [0, 3]
    np.testing.assert_array_equal(arr.reshape(-1), [16, 16, 16, 16])


# ---------------------------------------------------------------- closed forms

def ghz(n):
    c = tcgen.Circuit(n, 0).add("h", (0,))
    for i in range(n - 1):
        c.add("cnot", (i, i + 1))
    return c


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_ghz_amplitudes_and_correlators(n):
    c = ghz(n)
    r2 = 1 / math.sqrt(2)
    for sim in ("sv", "tn", "tn_split", "brute"):
        if sim == "brute" and n > 8:
            continue
        amp = {"sv": lambda b: sv.amplitude(c, [], b),
               "tn": lambda b: tn.amplitude(c, [], b),
               "tn_split": lambda b: tn.amplitude(c, [], b, split=True),
               "brute": lambda b: brute.amplitude(c, [], b)}[sim]
        assert close(amp((0,) * n), r2, 1e-14)
        assert close(amp((1,) * n), r2, 1e-14)
        assert close(amp((1,) + (0,) * (n - 1)), 0.0, 1e-14)
    for i in range(n):
        for j in range(i + 1, n):
            obs = tcgen.pauli_string(n, z=(i, j))
            assert close(sv.energy(c, [], obs), 1.0, 1e-14)
            assert close(tn.energy(c, [], obs), 1.0, 1e-14)
    assert close(sv.energy(c, [], tcgen.pauli_string(n, x=range(n))), 1.0, 1e-14)
    assert close(tn.energy(c, [], tcgen.pauli_string(n, x=range(n))), 1.0, 1e-14)


def test_bell_state():
    c = ghz(2)
    np.testing.assert_allclose(sv.state(c, []), [2 ** -.5, 0, 0, 2 ** -.5],
                               atol=1e-15)


@pytest.mark.parametrize("n", [1, 4, 9])
def test_hadamard_layer_amplitudes(n):
    c = tcgen.Circuit(n, 0)
    for q in range(n):
        c.add("h", (q,))
    rng = np.random.default_rng(n)
    for _ in range(4):
        bits = tuple(int(b) for b in rng.integers(0, 2, n))
        assert close(sv.amplitude(c, [], bits), 2 ** (-n / 2), 1e-14)
        assert close(tn.amplitude(c, [], bits), 2 ** (-n / 2), 1e-14)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_unit_norm_through_identity_observable(seed):
    c = tcgen.random_circuit(6, 40, seed,
                             kinds=[k for k in tcgen.UNITARY_KINDS if k not in ("u1", "u2")])
    p = np.random.default_rng(seed).uniform(0, 2 * math.pi, c.n_params)
    ident = tcgen.pauli_string(6)
    assert close(sv.energy(c, p, ident), 1.0, 1e-13)
    assert close(tn.energy(c, p, ident, order="time"), 1.0, 1e-13)
    assert abs(np.linalg.norm(sv.state(c, p)) - 1) < 1e-13


def test_rx_layer_z_expectations():
    n = 5
    th = np.random.default_rng(3).uniform(0, 2 * math.pi, n)
    c = tcgen.Circuit(n, n)
    for q in range(n):
        c.add("rx", (q,), (q,))
    for q in range(n):
        assert close(sv.energy(c, th, tcgen.pauli_string(n, z=(q,))),
                     math.cos(th[q]), 1e-14)
        assert close(sv.energy(c, th, tcgen.pauli_string(n, x=(q,))), 0.0, 1e-14)


def test_brickwork_one_layer_amplitude_closed_form():
    # <0^n| RZZ(even bonds) RX |0^n> = exp(-i sum_b phi_b / 2) prod_i cos(theta_i/2)
    n = 10
    c = tcgen.chain_brickwork(n, 1)
    p = tcgen.draw_angles(11, (1, 2, n)).reshape(-1).astype(np.float64)
    th = p[:n]
    phi = [p[n + i] for i in range(0, n - 1, 2)]
    want = cmath.exp(-0.5j * sum(phi)) * np.prod(np.cos(th / 2))
    assert close(sv.amplitude(c, p), want, 1e-14)
    assert close(tn.amplitude(c, p), want, 1e-14)
    assert close(tn.amplitude(c, p, split=True), want, 1e-14)


def test_ladder_one_layer_energy_and_gradient_closed_form():
    # L = 1: RZZ on |0^n> is a global phase, so E = sum_i cos t_i cos t_{i+1}
    # (<X_i> = 0), dE/dt_i = -sin t_i (cos t_{i-1} + cos t_{i+1}), dE/dphi = 0.
    n = 7
    c = tcgen.chain_ladder(n, 1)
    obs = tcgen.tfim_zz_x(n, 1.0)
    p = tcgen.draw_angles(12, (1, 2, n)).reshape(-1).astype(np.float64)
    th = p[n:]
    e_want = sum(math.cos(th[i]) * math.cos(th[i + 1]) for i in range(n - 1))
    e, g = sv.energy_grad(c, p, obs)
    assert abs(e - e_want) < 1e-13
    assert abs(tn.energy(c, p, obs).real - e_want) < 1e-13
    gw = np.zeros(2 * n)
    for i in range(n):
        nb = (math.cos(th[i - 1]) if i > 0 else 0) + \
             (math.cos(th[i + 1]) if i < n - 1 else 0)
        gw[n + i] = -math.sin(th[i]) * nb
    np.testing.assert_allclose(g, gw, atol=1e-13)


def test_vqe_chain_gradient_exact_zeros():
    # first RZZ layer acts on |0^n>: its gradient is exactly zero; the unused
    # slot phi[l][n-1] of every layer is zero too (n + L - 1 zeros)
    n, L = 8, 3
    c = tcgen.chain_ladder(n, L)
    obs = tcgen.tfim_zz_x(n)
    p = tcgen.draw_angles(13, (L, 2, n)).reshape(-1)
    _, g = sv.energy_grad(c, p, obs)
    g = g.reshape(L, 2, n)
    assert np.all(np.abs(g[0, 0, :]) < 1e-13)
    assert np.all(g[:, 0, n - 1] == 0.0)
    assert np.all(np.abs(g[1:, 0, :n - 1]) > 1e-6)


def test_brickwork_last_zz_layer_commutes_with_z0z1():
    n, L = 10, 4
    c = tcgen.chain_brickwork(n, L)
    obs = tcgen.pauli_string(n, z=(0, 1))
    p = tcgen.draw_angles(1, (L, 2, n)).reshape(-1)
    _, g = sv.energy_grad(c, p, obs)
    assert np.all(np.abs(g.reshape(L, 2, n)[3, 1, :]) < 1e-13)


# ---------------------------------------------------------------- O1 vs O3 vs O2

ALL_KINDS = list(tcgen.GATE_ARITY)


@pytest.mark.parametrize("seed", range(6))
def test_statevector_matches_brute_force(seed):
    n = 3 + seed % 4
    c = tcgen.random_circuit(n, 25, seed)
    p = np.random.default_rng(100 + seed).uniform(-4, 4, c.n_params)
    rng = np.random.default_rng(seed)
    for _ in range(3):
        bits = tuple(int(b) for b in rng.integers(0, 2, n))
        assert close(sv.amplitude(c, p, bits), brute.amplitude(c, p, bits), 1e-12)
    s = rng.integers(0, 4, size=(4, n)).astype(np.uint8)
    obs = tcgen.Observable("pauli_sum", structures=s, weights=rng.normal(size=4))
    assert close(sv.energy(c, p, obs), brute.energy(c, p, obs), 1e-12)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("order,split", [("col", False), ("col", True),
                                         ("time", False), ("row", True)])
def test_tensor_network_matches_statevector(seed, order, split):
    n = 4 + seed
    c = tcgen.random_circuit(n, 30, seed)
    p = np.random.default_rng(200 + seed).uniform(-4, 4, c.n_params)
    bits = tuple(int(b) for b in np.random.default_rng(seed).integers(0, 2, n))
    assert close(tn.amplitude(c, p, bits, order, split), sv.amplitude(c, p, bits), 1e-12)
    s = np.random.default_rng(seed).integers(0, 4, size=(3, n)).astype(np.uint8)
    obs = tcgen.Observable("pauli_sum", structures=s, weights=np.array([1.0, -0.5, 2.0]))
    assert close(tn.energy(c, p, obs, order, split), sv.energy(c, p, obs), 1e-12)


def test_forward_chain_workload_o1_vs_o2():
    circ, p, zz, amp = tcgen.workload_forward_chain()
    assert close(sv.amplitude(circ, p), tn.amplitude(circ, p, split=True), 1e-12)
    assert close(sv.amplitude(circ, p), tn.amplitude(circ, p), 1e-12)
    assert close(sv.energy(circ, p, zz), tn.energy(circ, p, zz, split=True), 1e-12)


def test_vqe_chain_workload_o1_vs_o2_all_terms():
    circ, p, obs = tcgen.workload_vqe_chain()
    v1 = sv.term_values(circ, p, obs)
    for j, s in enumerate(obs.structures):
        v2 = tn.expectation(circ, p, s, order="col", split=True)
        assert close(v1[j], v2, 1e-12), j
        assert abs(v2.imag) < 1e-12


@pytest.mark.parametrize("rows,cols", [(2, 4), (3, 3), (4, 4)])
def test_grid_generator_o1_vs_o2_two_orders(rows, cols):
    circ, p, obs = tcgen.workload_grid_amplitude(rows, cols, 8)
    a1 = sv.amplitude(circ, p)
    assert close(tn.amplitude(circ, p, order="col"), a1, 1e-12 * max(1, abs(a1)))
    assert close(tn.amplitude(circ, p, order="row"), a1, 1e-12 * max(1, abs(a1)))


# ---------------------------------------------------------------- gradients

def test_adjoint_gradient_matches_parameter_shift_and_fd():
    n, L = 6, 3
    c = tcgen.chain_ladder(n, L)
    obs = tcgen.tfim_zz_x(n, 0.7)
    p = tcgen.draw_angles(21, (L, 2, n)).reshape(-1)
    e, g = sv.energy_grad(c, p, obs)
    assert abs(e - sv.energy(c, p, obs).real) < 1e-13
    np.testing.assert_allclose(g, sv.param_shift_grad(c, p, obs), atol=1e-10)
    fd = sv.finite_diff_grad(c, p, obs, h=1e-3)
    assert np.linalg.norm(g - fd) / max(np.linalg.norm(g), 1) < 1e-6


def test_adjoint_gradient_with_shared_slots_and_fsim():
    c = tcgen.Circuit(4, 3)
    c.add("h", (0,)).add("rx", (1,), (0,)).add("fsim", (0, 1), (1, 2))
    c.add("rzz", (1, 2), (0,)).add("sqrt_w", (3,)).add("fsim", (2, 3), (2, 1))
    c.add("ry", (0,), (0,))
    obs = tcgen.tfim_zz_x(4, 1.3)
    p = np.array([0.3, 1.1, -0.4])
    _, g = sv.energy_grad(c, p, obs)
    fd = sv.finite_diff_grad(c, p, obs, h=1e-4)
    np.testing.assert_allclose(g, fd, atol=1e-7)
