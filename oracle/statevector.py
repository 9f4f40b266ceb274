"""O1: dense complex128 state-vector simulator (oracle; test infrastructure).

Follows the paper's definitions directly:

* section "Circuits and gates / Basic circuits and outputs": the circuit acts
  on |0...0>, the wavefunction is indexed with qubit 0 most significant, an
  amplitude is one entry of it;
* section "Pauli string expectation / Pauli structures and weights" and the
  Hamiltonian written as a weighted sum of Pauli strings in the introduction:
  E = sum_j alpha_j <psi|P_j|psi>, summed here in float64 in term order;
* section "Expectations of Hamiltonians via operator_expectation": an
  operator given as an MPO is applied to the state by ``oracle.mpo``;
* section "Gradients, optimization and variational algorithms": dE/dtheta,
  computed here with the adjoint method (Jones & Gacon, arXiv:2009.02823):
  with psi_g = U_g psi_{g-1} and lambda_g = (U_G ... U_{g+1})^dagger H psi_G,
  dE/dtheta_g = 2 Re <lambda_g| dU_g/dtheta |psi_{g-1}>.

The state is held as an n-dimensional (2,)*n array whose axis q is qubit q.
"""
from __future__ import annotations

import math

import numpy as np

from . import gates as G
from . import mpo


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    return psi


def apply(psi: np.ndarray, mat: np.ndarray, qubits) -> np.ndarray:
    """Apply a k-qubit matrix to the listed axes of psi."""
    k = len(qubits)
    t = mat.reshape((2,) * (2 * k))
    # contract the input legs of t (last k axes) with the target axes of psi
    out = np.tensordot(t, psi, axes=(list(range(k, 2 * k)), list(qubits)))
    # the k new axes sit in front; move them back to their qubit positions
    return np.moveaxis(out, list(range(k)), list(qubits))


def run(circ, params, psi=None) -> np.ndarray:
    params = np.asarray(params, dtype=np.float64)
    if psi is None:
        psi = zero_state(circ.n_qubits)
    for g in circ.gates:
        psi = apply(psi, G.matrix(g, params), g.qubits)
    return psi


def state(circ, params) -> np.ndarray:
    return run(circ, params).reshape(-1)


def amplitude(circ, params, bits=None) -> complex:
    psi = run(circ, params)
    if bits is None:
        bits = (0,) * circ.n_qubits
    return complex(psi[tuple(bits)])


def apply_pauli(psi: np.ndarray, structure) -> np.ndarray:
    out = psi
    for q, s in enumerate(structure):
        if s:
            out = apply(out, G.PAULI[int(s)], (q,))
    return out


def pauli_expectation(psi: np.ndarray, structure) -> complex:
    return complex(np.vdot(psi, apply_pauli(psi, structure)))


def term_values(circ, params, obs) -> np.ndarray:
    """<psi|P_j|psi> for every term j (complex128)."""
    psi = run(circ, params)
    return np.array([pauli_expectation(psi, s) for s in obs.structures])


def energy(circ, params, obs) -> complex:
    """sum_j alpha_j <P_j>, accumulated in float64 in term order; for an
    operator given as an MPO, <psi|M|psi>."""
    if obs.kind == "mpo":
        return mpo.expectation(run(circ, params), obs.mpo)
    vals = term_values(circ, params, obs)
    re = 0.0
    im = 0.0
    for a, v in zip(obs.weights, vals):
        re += float(a) * v.real
        im += float(a) * v.imag
    return complex(re, im)


def apply_hamiltonian(psi: np.ndarray, obs) -> np.ndarray:
    if obs.kind == "mpo":
        return mpo.apply(psi, obs.mpo)
    out = np.zeros_like(psi)
    for a, s in zip(obs.weights, obs.structures):
        out = out + float(a) * apply_pauli(psi, s)
    return out


def energy_grad(circ, params, obs):
    """(E, dE/dparams) by the adjoint method; unused slots get exactly 0."""
    params = np.asarray(params, dtype=np.float64)
    psi = run(circ, params)
    lam = apply_hamiltonian(psi, obs)
    e = float(np.vdot(psi, lam).real)
    grad = np.zeros(circ.n_params, dtype=np.float64)
    for g in reversed(circ.gates):
        u = G.matrix(g, params)
        udag = u.conj().T
        psi = apply(psi, udag, g.qubits)          # psi_{g-1}
        for which, s in enumerate(g.params):
            if s < 0:
                continue
            du = G.dmatrix(g, params, which)
            grad[s] += 2.0 * float(np.vdot(lam, apply(psi, du, g.qubits)).real)
        lam = apply(lam, udag, g.qubits)          # lambda_{g-1}
    return e, grad


def _with_gate_angle(circ, params, gi, which, delta):
    """A copy of circ in which angle `which` of gate number gi is fixed at
    its current value + delta (only that gate use moves, even if its slot is
    shared with other gates)."""
    from tcgen import Circuit, Gate
    gates = list(circ.gates)
    g = gates[gi]
    ps = list(g.params)
    fx = list(g.fixed)
    fx[which] = G.gate_angles(g, params)[which] + delta
    ps[which] = -1
    gates[gi] = Gate(g.kind, g.qubits, tuple(ps), tuple(fx), g.matrix)
    return Circuit(circ.n_qubits, circ.n_params, gates, circ.coords)


def param_shift_grad(circ, params, obs) -> np.ndarray:
    """Exact two-point shift rule, one shift pair per gate use, summed into
    its slot.  Valid for exp(-i t G/2) gates with G^2 = I only."""
    params = np.asarray(params, dtype=np.float64)
    grad = np.zeros(circ.n_params, dtype=np.float64)
    for gi, g in enumerate(circ.gates):
        for which, s in enumerate(g.params):
            if s < 0:
                continue
            if not G.shift_rule_ok(g.kind):
                raise ValueError(f"no exact shift rule for {g.kind}")
            ep = energy(_with_gate_angle(circ, params, gi, which, math.pi / 2), params, obs).real
            em = energy(_with_gate_angle(circ, params, gi, which, -math.pi / 2), params, obs).real
            grad[s] += 0.5 * (ep - em)
    return grad


def finite_diff_grad(circ, params, obs, h: float = 1e-3) -> np.ndarray:
    """Central differences [E(t+h) - E(t-h)] / 2h on every slot."""
    params = np.asarray(params, dtype=np.float64)
    grad = np.zeros(circ.n_params, dtype=np.float64)
    for s in range(circ.n_params):
        p = params.copy()
        p[s] += h
        ep = energy(circ, p, obs).real
        p[s] -= 2 * h
        em = energy(circ, p, obs).real
        grad[s] = (ep - em) / (2 * h)
    return grad


def jacobian(circ, params) -> np.ndarray:
    """J[:, j] = d psi / d theta_j as a (2^n, n_params) matrix: for every
    use of slot j (a gate angle reading it), the circuit run with that gate
    replaced by its derivative, summed over the slot's uses (the product
    rule written out).  Section "Advanced automatic differentiation":
    the Jacobian of the output state."""
    params = np.asarray(params, dtype=np.float64)
    n = circ.n_qubits
    jac = np.zeros((1 << n, circ.n_params), dtype=np.complex128)
    for gi, g in enumerate(circ.gates):
        for which, s in enumerate(g.params):
            if s < 0:
                continue
            psi = zero_state(n)
            for gk, h in enumerate(circ.gates):
                m = G.dmatrix(h, params, which) if gk == gi else G.matrix(h, params)
                psi = apply(psi, m, h.qubits)
            jac[:, s] += psi.reshape(-1)
    return jac


def geometric_tensor(circ, params) -> np.ndarray:
    """G_ij = <d_i psi|d_j psi> - <d_i psi|psi><psi|d_j psi> (section
    "Advanced automatic differentiation", the quantity behind the QFI and
    the quantum natural gradient; the QFI is 4 Re G)."""
    psi = state(circ, params)
    jac = jacobian(circ, params)
    overlap = jac.conj().T @ psi          # <d_i psi|psi>
    return jac.conj().T @ jac - np.outer(overlap, overlap.conj())
