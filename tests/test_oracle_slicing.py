"""Pins for the slicing branch of the oracle's sweep contraction (no GPU).

Slicing replaces one contraction by the plain sum, over every value of a
fixed set of labels, of the networks with those labels pinned (the index
sum of section "Tensor network engine", written out; the paper names
slicing as the way past memory limits in its outlook).  These tests force
``oracle.tn.fold_sliced`` to slice by giving it a memory limit below the
sweep's peak, then compare with things the slicing code does not share:

* a closed form: trace(A B) of two non-symmetric matrices, and a three-index
  chain whose sum ``numpy.einsum`` writes out;
* the state-vector oracle (O1) on grid amplitudes and on Pauli expectations of
  random circuits over every gate kind, at 1e-12;
* the number of slices visited (the product of the sliced dimensions).

A planted mistake (the slice taken on the wrong axis) is shown to fail the
same comparison, so the pins are not blind to it.
"""
import numpy as np
import pytest

import tcgen
from oracle import statevector as sv
from oracle import tn


def _fold_forced(ts, drop_log2):
    """fold_sliced with a limit 2^drop_log2 below the sweep's own peak;
    returns (value, sliced labels, slices visited)."""
    peak = tn.peak_log2(ts)
    limit = 1 << max(peak - drop_log2, 1)
    labels = tn.choose_slices(ts, limit)
    seen = []
    v = tn.fold_sliced(ts, limit, progress=lambda idx, shape: seen.append(idx))
    return v, labels, len(seen)


def test_slice_trace_of_two_matrices_closed_form():
    rng = np.random.default_rng(0)
    a = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    b = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    # label 0 is A's row and B's column: slicing it must take A's axis 0
    # and B's axis 1
    ts = [tn.T(a, (0, 1), (0, 0, 0, 0)), tn.T(b, (1, 0), (0, 1, 0, 1))]
    want = np.trace(a @ b)
    labels = tn.choose_slices(ts, 1)
    assert labels, "a limit of one element must slice"
    got = tn.fold_sliced(ts, 1)
    assert abs(got - want) < 1e-14 * max(1.0, abs(want))


def test_slice_three_index_chain_matches_einsum():
    rng = np.random.default_rng(1)
    a = rng.normal(size=(2, 2, 2)) + 1j * rng.normal(size=(2, 2, 2))
    b = rng.normal(size=(2, 2, 2)) + 1j * rng.normal(size=(2, 2, 2))
    c = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    # labels: a(i, j, k), b(k, l, i), c(l, j)
    ts = [tn.T(a, (0, 1, 2), (0, 0, 0, 0)), tn.T(b, (2, 3, 0), (0, 1, 0, 1)),
          tn.T(c, (3, 1), (0, 2, 0, 2))]
    want = np.einsum("ijk,kli,lj->", a, b, c)
    for limit in (8, 4, 2):
        got = tn.fold_sliced(ts, limit)
        assert abs(got - want) < 1e-13 * max(1.0, abs(want)), limit
    assert len(tn.choose_slices(ts, 2)) >= 2


@pytest.mark.parametrize("rows,cols,drop", [(3, 3, 2), (2, 4, 2), (3, 3, 1)])
def test_sliced_grid_amplitude_matches_statevector(rows, cols, drop):
    circ, p, _ = tcgen.workload_grid_amplitude(rows, cols, 8)
    a1 = sv.amplitude(circ, p)
    for order in ("col", "row2"):
        ts = sorted(tn.amplitude_network(circ, p), key=tn._sort_key(order))
        v, labels, n_slices = _fold_forced(ts, drop)
        assert len(labels) >= 1
        assert n_slices == 2 ** len(labels)
        assert abs(v - a1) <= 1e-12 * max(abs(a1), 2 ** (-circ.n_qubits / 2)), order


@pytest.mark.parametrize("seed", range(3))
def test_sliced_expectations_of_random_circuits_match_statevector(seed):
    n = 6
    circ = tcgen.random_circuit(n, 40, seed)
    p = np.random.default_rng(300 + seed).uniform(-3, 3, circ.n_params)
    rng = np.random.default_rng(seed)
    s = rng.integers(0, 4, size=(3, n)).astype(np.uint8)
    s[:, 0] = (1, 2, 3)   # every Pauli kind on the first qubit
    for split in (False, True):
        for st in s:
            want = sv.energy(circ, p, tcgen.Observable(
                "pauli_sum", structures=st[None, :], weights=np.array([1.0])))
            ts = sorted(tn.expectation_network(circ, p, st, split=split),
                        key=tn._sort_key("time"))
            v, labels, _ = _fold_forced(ts, 2)
            assert labels
            assert abs(v - want) < 1e-12, (split, st)


def test_sliced_vqe_terms_match_statevector():
    circ, p, obs = tcgen.workload_vqe_chain(n=10, layers=3)
    v1 = sv.term_values(circ, p, obs)
    for j in (0, 4, 8, 9, 15):
        ts = sorted(tn.expectation_network(circ, p, obs.structures[j], split=True),
                    key=tn._sort_key("time"))
        v, labels, _ = _fold_forced(ts, 2)
        assert labels
        assert abs(v - v1[j]) < 1e-12, j


def _wrong_axis_fix(tensors, label, value):
    """The slice taken on the neighbouring axis of each tensor."""
    out = []
    for t in tensors:
        if label in t.labels:
            ax = t.labels.index(label)
            bad = (ax + 1) % t.data.ndim
            out.append(tn.T(np.take(t.data, value, axis=bad),
                            t.labels[:ax] + t.labels[ax + 1:], t.key))
        else:
            out.append(t)
    return out


def test_planted_wrong_axis_is_caught(monkeypatch):
    """The comparisons above fail when the slice is taken on the wrong axis
    of a tensor (the mistake a reader would look for in the slicing code).
    Generic tensors are needed to see it: fSim is symmetric under swapping
    its two qubits and sqrt(X) is a symmetric matrix, so a grid of those can
    hide it; random tensors and random U1/U2 matrices cannot."""
    rng = np.random.default_rng(1)
    a = rng.normal(size=(2, 2, 2)) + 1j * rng.normal(size=(2, 2, 2))
    b = rng.normal(size=(2, 2, 2)) + 1j * rng.normal(size=(2, 2, 2))
    c = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    ts3 = [tn.T(a, (0, 1, 2), (0, 0, 0, 0)), tn.T(b, (2, 3, 0), (0, 1, 0, 1)),
           tn.T(c, (3, 1), (0, 2, 0, 2))]
    want3 = np.einsum("ijk,kli,lj->", a, b, c)

    circ = tcgen.random_circuit(6, 40, 0)
    p = np.random.default_rng(300).uniform(-3, 3, circ.n_params)
    st = np.array([1, 2, 3, 0, 1, 3], np.uint8)
    want = sv.energy(circ, p, tcgen.Observable(
        "pauli_sum", structures=st[None, :], weights=np.array([1.0])))
    ts = sorted(tn.expectation_network(circ, p, st), key=tn._sort_key("time"))

    assert abs(tn.fold_sliced(ts3, 2) - want3) < 1e-13
    assert abs(_fold_forced(ts, 2)[0] - want) < 1e-12
    monkeypatch.setattr(tn, "_fix", _wrong_axis_fix)
    assert abs(tn.fold_sliced(ts3, 2) - want3) > 1e-3
    assert abs(_fold_forced(ts, 2)[0] - want) > 1e-6
