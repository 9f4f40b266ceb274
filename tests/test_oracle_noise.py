"""Pins for the oracle's channels with externalised randomness (no GPU).

Sections "Externalizing the randomness", "Batched Monte Carlo trajectory
noise simulation" and "Demonstration of barren plateaus": a status x in
[0,1) picks one operator of a channel by intervals whose lengths are the
outcome probabilities.  Sources of truth:
* the paper's interval rule for its (px, py, pz) = (0.1, 0.2, 0.3)
  example, by hand: [0, 0.4) I, [0.4, 0.5) X, [0.5, 0.7) Y, [0.7, 1) Z;
  and for the RX/RY/RZ choice, thirds;
* the density-matrix channel rho -> sum_i p_i P_i rho P_i written with the
  Pauli matrices of O3 (``brute``): the probability-weighted sum of the
  trajectories (one status inside each interval) equals it exactly, and the
  closed forms <Z> = 1 - 2 (px + py) on |0>, <X> = 1 - 2 (py + pz) on |+>;
* a Monte Carlo mean over uniform statuses converges to the channel (5
  standard errors);
* the float32 cut points: a status equal to a cut falls in the next
  interval.
"""
import numpy as np
import pytest

import tcgen
from oracle import brute
from oracle import gates as G
from oracle import statevector as sv

PX, PY, PZ = 0.1, 0.2, 0.3


def depol(status, probs=(PX, PY, PZ)):
    return tcgen.Gate("depol", (0,), (-1,), (float(status),), tuple(probs))


@pytest.mark.parametrize("x,k", [(0.0, 0), (0.2, 0), (0.39, 0), (0.41, 1), (0.49, 1), (0.51, 2),
                                 (0.69, 2), (0.71, 3), (0.999, 3)])
def test_paper_intervals_by_hand(x, k):
    np.testing.assert_array_equal(G.matrix(depol(x), []), brute.pauli_dense([k]))


def test_rswitch_thirds_are_rx_ry_rz():
    t = 0.7
    for x, kind in ((0.1, "rx"), (0.5, "ry"), (0.9, "rz")):
        g = tcgen.Gate("rswitch", (0,), (-1, -1), (t, x))
        ref = G.matrix(tcgen.Gate(kind, (0,), (-1,), (t,)), [])
        np.testing.assert_allclose(G.matrix(g, []), ref, atol=1e-15)
        np.testing.assert_allclose(G.dmatrix(g, [], 0),
                                   G.dmatrix(tcgen.Gate(kind, (0,), (-1,), (t,)), [], 0), atol=1e-15)
        assert np.all(G.dmatrix(g, [], 1) == 0)


def test_float32_cut_points():
    p0 = np.float32(np.float32(np.float32(np.float32(1.0) - np.float32(PX)) - np.float32(PY)) - np.float32(PZ))
    np.testing.assert_array_equal(G.matrix(depol(float(p0)), []), brute.pauli_dense([1]))
    below = np.nextafter(p0, np.float32(0.0))
    np.testing.assert_array_equal(G.matrix(depol(float(below)), []), brute.pauli_dense([0]))


def channel_expectation(prep, obs_structure, probs):
    """Tr(O E(rho)) with E(rho) = sum_i p_i P_i rho P_i (dense, by hand)."""
    psi = sv.state(prep, np.zeros(prep.n_params))
    rho = np.outer(psi, psi.conj())
    ps = [1 - sum(probs)] + list(probs)
    out = sum(p * brute.pauli_dense([k]) @ rho @ brute.pauli_dense([k]) for k, p in enumerate(ps))
    return float(np.trace(brute.pauli_dense(obs_structure) @ out).real)


@pytest.mark.parametrize("prep_h,obs", [(False, 3), (True, 1), (True, 2)])
def test_trajectory_weighted_sum_equals_the_channel(prep_h, obs):
    probs = (PX, PY, PZ)
    mids = [0.2, 0.45, 0.6, 0.85]                 # one status inside each interval
    weights = [1 - sum(probs), PX, PY, PZ]
    prep = tcgen.Circuit(1, 0)
    if prep_h:
        prep.add("h", (0,))
    o = tcgen.pauli_string(1, **{"x" if obs == 1 else "y" if obs == 2 else "z": (0,)})
    acc = 0.0
    for w, x in zip(weights, mids):
        c = tcgen.Circuit(1, 1, list(prep.gates) + [depol(x)])
        acc += w * sv.energy(c, np.zeros(1), o).real
    assert abs(acc - channel_expectation(prep, [obs], probs)) < 1e-14
    if not prep_h and obs == 3:
        assert abs(acc - (1 - 2 * (PX + PY))) < 1e-14
    if prep_h and obs == 1:
        assert abs(acc - (1 - 2 * (PY + PZ))) < 1e-14


def test_monte_carlo_mean_converges_to_the_channel():
    rng = np.random.default_rng(0)
    xs = rng.uniform(0, 1, 4000).astype(np.float32)
    c = tcgen.Circuit(1, 1, [tcgen.Gate("h", (0,)), tcgen.Gate("depol", (0,), (0,), (0.0,), (PX, PY, PZ))])
    o = tcgen.pauli_string(1, x=(0,))
    vals = np.array([sv.energy(c, np.array([x], np.float64), o).real for x in xs])
    want = 1 - 2 * (PY + PZ)
    assert abs(vals.mean() - want) < 5 * vals.std() / np.sqrt(len(vals))
