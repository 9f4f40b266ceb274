"""GPU parity of resident term launches (plan exec_mode 3): one workgroup
per term runs the term's leaves, forward pass and reverse sweep in a single
kernel, with the tensors the planner places there held in the workgroup's
LDS.  Checked against the oracle (O1 state vector, complex128) at the
complex64 tolerance, against level launches of the same network, and on
the forward-only call of a gradient plan."""
import numpy as np
import pytest

import tcgen
from oracle import statevector as sv
from paper_2205_10091_amd import _lib as L
from paper_2205_10091_amd import api
from gpu_common import TOL_C64, assert_grad, device_params, rel_err

pytestmark = pytest.mark.gpu

RESIDENT = 4  # tc_plan_info.exec_mode of a plan with resident term launches


def test_resident_headline_chain_energy_and_gradient():
    circ, p, obs = tcgen.workload_vqe_chain()
    plan = api.compile(circ, obs, want_grad=True, n_trials=64, seed=1, exec_mode=3)
    info = plan.info()
    assert info.exec_mode == RESIDENT
    assert info.n_launches == 2 and info.n_grad_launches == 2  # term + root, term + grad
    e, g = plan.contract_grad(device_params(p))
    e_ref, g_ref = sv.energy_grad(circ, p, obs)
    print(f"resident 20-qubit chain: |dE| {abs(e[0] - e_ref):.2e}, "
          f"max |dg| {np.max(np.abs(g[0] - g_ref)):.2e}")
    assert rel_err(e[0], e_ref, 1.0) < TOL_C64
    assert_grad(g[0], g_ref, TOL_C64, "resident chain")
    # the forward-only call of the same plan runs the forward groups alone
    v = plan.contract(device_params(p))[0]
    assert abs(v - e[0]) <= 1e-6 * max(1.0, abs(e[0]))


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("caller_matrices", [False, True])
def test_resident_all_gate_kinds_against_oracle_and_level_launches(seed, caller_matrices):
    """Every gate kind; with caller matrices (u1/u2, random and not unitary)
    the energy is checked against the oracle and the gradient against level
    launches only (the oracle's adjoint gradient assumes unitary gates)."""
    n = 6
    kinds = [k for k in tcgen.UNITARY_KINDS if caller_matrices or k not in ("u1", "u2")]
    circ = tcgen.random_circuit(n, 50, seed, kinds)
    p = np.random.default_rng(seed).uniform(-3, 3, circ.n_params).astype(np.float32)
    rng = np.random.default_rng(10 + seed)
    s = rng.integers(0, 4, size=(5, n)).astype(np.uint8)
    obs = tcgen.Observable("pauli_sum", structures=s, weights=rng.normal(size=5))
    res = api.compile(circ, obs, want_grad=True, exec_mode=3)
    lev = api.compile(circ, obs, want_grad=True, exec_mode=1)
    assert res.info().exec_mode == RESIDENT
    e3, g3 = res.contract_grad(device_params(p))
    e1, g1 = lev.contract_grad(device_params(p))
    e_ref, g_ref = sv.energy_grad(circ, p.astype(np.float64), obs)
    scale = max(1.0, float(np.sum(np.abs(obs.weights))))
    assert abs(e3[0] - e_ref) / scale < TOL_C64
    if not caller_matrices:
        assert_grad(g3[0] / scale, g_ref / scale, TOL_C64, "resident")
    gs = max(1.0, float(np.max(np.abs(g1[0]))))
    assert abs(e3[0] - e1[0]) / scale < 2e-6
    assert_grad(g3[0] / gs, g1[0] / gs, 2e-6, "resident vs level")


def test_resident_checkpointed_sweep_and_amplitude():
    circ, p, obs = tcgen.workload_vqe_chain(n=12, layers=4)
    plan = api.compile(circ, obs, want_grad=True, exec_mode=3, checkpoint_every=2)
    info = plan.info()
    assert info.exec_mode == RESIDENT and info.checkpoint_every == 2
    e, g = plan.contract_grad(device_params(p))
    e_ref, g_ref = sv.energy_grad(circ, p, obs)
    assert rel_err(e[0], e_ref, 1.0) < TOL_C64
    assert_grad(g[0], g_ref, TOL_C64, "resident checkpointed")
    n = circ.n_qubits
    bits = tuple(int(b) for b in np.random.default_rng(3).integers(0, 2, n))
    amp = api.compile(circ, tcgen.amplitude(n, bits), exec_mode=3)
    a = amp.contract(device_params(p))[0]
    assert rel_err(a, sv.amplitude(circ, p, bits), 2 ** (-n / 2)) < TOL_C64


def test_resident_repeated_calls_are_bitwise_equal():
    circ, p, obs = tcgen.workload_vqe_chain(n=14, layers=5)
    plan = api.compile(circ, obs, want_grad=True, exec_mode=3)
    e1, g1 = plan.contract_grad(device_params(p))
    for _ in range(3):
        e2, g2 = plan.contract_grad(device_params(p))
        assert np.array_equal(e1, e2) and np.array_equal(g1, g2)


def test_resident_mode_errors():
    circ, p, obs = tcgen.workload_vqe_chain(n=8, layers=2)
    with pytest.raises(L.TcxError) as ex:
        api.compile(circ, obs, batch=2, exec_mode=3)
    assert ex.value.status == L.TC_ERR_UNSUPPORTED
