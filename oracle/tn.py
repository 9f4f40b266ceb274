"""O2: einsum-style pairwise tensor-network contraction (oracle; test infra).

Section "Tensor network engine": a circuit's diagram is a tensor network;
an amplitude or an expectation value is obtained by contracting edges until
one node is left, and the order of contraction changes cost but not the
result.  Section "Custom contraction settings" computes <Z_{n/2}> as a single
network (the ``reuse=False`` form) rather than from the state, and section
"Very large circuit simulation" splits two-qubit gates into two connected
three-leg tensors by an SVD.

This module builds its own network (independent of the GPU library's
builder) and contracts it with ``numpy.tensordot`` in a fixed *sweep* order,
never with a path finder:

* ``order="col"``: tensors sorted by (column, row, phase, time) of the qubit
  they sit on, where a two-qubit gate sits on its later qubit; a chain's
  column is its qubit index;
* ``order="row"``: the same with rows and columns exchanged;
* ``order="col2"``/``"row2"``: as "col"/"row", but the multi-qubit tensors
  a qubit owns are absorbed before that qubit's single-qubit tensors;
* ``order="time"``: tensors in the order they were created.

The expectation <psi|P|psi> is built as one network: the ket (|0> vectors,
gates), the Pauli matrices on the measured qubits, and the bra, which is the
entrywise complex conjugate of the ket network whose open legs meet the
Pauli matrices' output legs.  ``split=True`` replaces every two-qubit gate
by the two factors of its operator-Schmidt decomposition (numpy SVD, exact
rank), as in the paper's split option without truncation.

Where a sweep's largest intermediate is too big, ``max_elements`` lets the
fold *slice*: labels are fixed one value at a time and the sliced networks'
scalars are summed (the plain sum over that index, written out).  Labels are
chosen one by one, each time the one whose removal lowers the sweep's peak
the most, until the peak fits.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

from . import gates as G


@dataclass
class T:
    data: np.ndarray
    labels: Tuple[int, ...]
    key: Tuple               # (row, col, phase, time) of its owning qubit


class _Builder:
    def __init__(self, circ, split: bool):
        self.circ = circ
        self.split = split
        self.next_label = 0
        self.tensors: List[T] = []
        self.time = 0

    def label(self) -> int:
        self.next_label += 1
        return self.next_label - 1

    def rc(self, q):
        if self.circ.coords is not None:
            return self.circ.coords[q]
        return (0, q)

    def owner(self, qubits):
        # a multi-qubit tensor belongs to its latest qubit in (col, row) order
        return max(qubits, key=lambda q: (self.rc(q)[1], self.rc(q)[0]))

    def add(self, data, labels, qubit, phase):
        r, c = self.rc(qubit)
        self.tensors.append(T(np.asarray(data, np.complex128), tuple(labels),
                              (r, c, phase, self.time)))
        self.time += 1

    def ket(self, params, conj: bool, phase: int, final=None):
        """Add |0> vectors and gates; return the open label of every qubit.
        With conj=True all entries are conjugated (the bra half).  `final`
        optionally fixes the labels of the open legs."""
        n = self.circ.n_qubits
        cur = [self.label() for _ in range(n)]
        for q in range(n):
            self.add(np.array([1.0, 0.0]), (cur[q],), q, phase)
        gl = list(self.circ.gates)
        last_use = {}
        for gi, g in enumerate(gl):
            for q in g.qubits:
                last_use[q] = gi
        for gi, g in enumerate(gl):
            m = G.matrix(g, params)
            if conj:
                m = m.conj()
            k = len(g.qubits)
            outs = []
            for q in g.qubits:
                if final is not None and last_use[q] == gi:
                    outs.append(final[q])
                else:
                    outs.append(self.label())
            ins = [cur[q] for q in g.qubits]
            if k == 2 and self.split:
                self._add_split(m, outs, ins, g.qubits, phase)
            else:
                self.add(m.reshape((2,) * (2 * k)), outs + ins,
                         self.owner(g.qubits), phase)
            for q, o in zip(g.qubits, outs):
                cur[q] = o
        if final is not None:
            # qubits with no gate: their |0> leg is the open leg
            for q in range(n):
                if q not in last_use:
                    self._relabel(cur[q], final[q])
                    cur[q] = final[q]
        return cur

    def _relabel(self, old, new):
        for t in self.tensors:
            if old in t.labels:
                t.labels = tuple(new if x == old else x for x in t.labels)

    def _add_split(self, m, outs, ins, qubits, phase):
        # operator-Schmidt: m[(oa ob),(ia ib)] -> M[(oa ia),(ob ib)]
        mm = m.reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)
        u, s, vh = np.linalg.svd(mm)
        r = int(np.sum(s > 1e-13 * max(s[0], 1e-300)))
        r = max(r, 1)
        a = (u[:, :r] * s[:r]).reshape(2, 2, r)      # (oa, ia, bond)
        b = vh[:r, :].reshape(r, 2, 2)               # (bond, ob, ib)
        bond = self.label()
        self.add(a, (outs[0], ins[0], bond), qubits[0], phase)
        self.add(b, (bond, outs[1], ins[1]), qubits[1], phase)


def _sort_key(order):
    # "col2"/"row2": like "col"/"row", but on each qubit the multi-qubit
    # tensors it owns (their other legs are already in the accumulator) are
    # absorbed before its single-qubit tensors, which keeps the growth while
    # a qubit is processed to one leg.
    if order == "col2":
        return lambda t: (t.key[1], t.key[0], t.data.ndim <= 2, t.key[2], t.key[3])
    if order == "row2":
        return lambda t: (t.key[0], t.key[1], t.data.ndim <= 2, t.key[2], t.key[3])
    if order == "col":
        return lambda t: (t.key[1], t.key[0], t.key[2], t.key[3])
    if order == "row":
        return lambda t: (t.key[0], t.key[1], t.key[2], t.key[3])
    if order == "time":
        return lambda t: (t.key[2], t.key[3])
    raise ValueError(order)


def _fold(tensors: List[T], max_elements: int) -> complex:
    """Contract left to right; raise if an intermediate would exceed
    max_elements (checked on labels before any arithmetic)."""
    # symbolic pass
    peak = 1 << peak_log2(tensors)
    if peak > max_elements:
        raise MemoryError(f"sweep peak 2^{peak.bit_length() - 1} elements "
                          f"exceeds the limit")
    acc_t, acc_l = contract_in_order(tensors)
    assert acc_t.ndim == 0, "network left open legs"
    return complex(acc_t)


def contract_in_order(tensors: List[T]):
    """Fold the list left to right with tensordot over shared labels;
    returns (array, labels) of whatever legs remain open."""
    acc_t = tensors[0].data
    acc_l = list(tensors[0].labels)
    for t in tensors[1:]:
        shared = [x for x in acc_l if x in t.labels]
        ia = [acc_l.index(x) for x in shared]
        ib = [t.labels.index(x) for x in shared]
        acc_t = np.tensordot(acc_t, t.data, axes=(ia, ib))
        acc_l = [x for x in acc_l if x not in shared] + \
            [x for x in t.labels if x not in shared]
    return acc_t, acc_l


def peak_log2(tensors: List[T]) -> int:
    """log2 of the largest intermediate of the left fold (all dims are
    powers of two)."""
    dims = {}
    for t in tensors:
        for l, d in zip(t.labels, t.data.shape):
            dims[l] = d.bit_length() - 1
    acc = set()
    peak = 0
    for t in tensors:
        shared = acc & set(t.labels)
        acc = (acc | set(t.labels)) - shared
        peak = max(peak, sum(dims[l] for l in acc))
    return peak


def amplitude_network(circ, params, bits=None, split=False) -> List[T]:
    params = np.asarray(params, np.float64)
    b = _Builder(circ, split)
    n = circ.n_qubits
    bits = (0,) * n if bits is None else tuple(bits)
    fin = b.ket(params, conj=False, phase=0)
    for q in range(n):
        v = np.zeros(2)
        v[int(bits[q])] = 1.0
        b.add(v, (fin[q],), q, 1)
    return b.tensors


def expectation_network(circ, params, structure, split=False) -> List[T]:
    params = np.asarray(params, np.float64)
    b = _Builder(circ, split)
    n = circ.n_qubits
    ket_out = b.ket(params, conj=False, phase=0)
    bra_out = list(ket_out)
    for q in range(n):
        s = int(structure[q])
        if s:
            o = b.label()
            # P[out, in]: in = ket leg, out = bra leg
            b.add(G.PAULI[s], (o, ket_out[q]), q, 1)
            bra_out[q] = o
    b.ket(params, conj=True, phase=2, final=bra_out)
    return b.tensors


def _peak_without(tensors: List[T], removed) -> int:
    dims = {}
    for t in tensors:
        for l, d in zip(t.labels, t.data.shape):
            dims[l] = d.bit_length() - 1
    acc = set()
    peak = 0
    for t in tensors:
        ls = set(t.labels) - removed
        shared = acc & ls
        acc = (acc | ls) - shared
        peak = max(peak, sum(dims[l] for l in acc))
    return peak


def choose_slices(tensors: List[T], max_elements: int, max_slices: int = 16):
    """Labels to slice so that the fold's peak fits max_elements."""
    removed = set()
    labels = sorted({l for t in tensors for l in t.labels})
    limit = max_elements.bit_length() - 1
    while _peak_without(tensors, removed) > limit:
        if len(removed) >= max_slices:
            raise MemoryError("too many slices needed")
        best = min((l for l in labels if l not in removed),
                   key=lambda l: (_peak_without(tensors, removed | {l}), l))
        removed.add(best)
    return sorted(removed)


def _fix(tensors: List[T], label: int, value: int) -> List[T]:
    out = []
    for t in tensors:
        if label in t.labels:
            ax = t.labels.index(label)
            out.append(T(np.take(t.data, value, axis=ax),
                         t.labels[:ax] + t.labels[ax + 1:], t.key))
        else:
            out.append(t)
    return out


def fold_sliced(tensors: List[T], max_elements: int, progress=None) -> complex:
    """Sum over all values of the chosen slice labels of the left fold."""
    sl = choose_slices(tensors, max_elements)
    if not sl:
        return _fold(tensors, max_elements)
    dims = {}
    for t in tensors:
        for l, d in zip(t.labels, t.data.shape):
            dims[l] = d
    total = 0j
    shape = [dims[l] for l in sl]
    for idx in np.ndindex(*shape):
        ts = tensors
        for l, v in zip(sl, idx):
            ts = _fix(ts, l, v)
        total += _fold(ts, max_elements)
        if progress is not None:
            progress(idx, shape)
    return total


def amplitude(circ, params, bits=None, order="col", split=False,
              max_elements=1 << 27, progress=None) -> complex:
    ts = amplitude_network(circ, params, bits, split)
    return fold_sliced(sorted(ts, key=_sort_key(order)), max_elements, progress)


def expectation(circ, params, structure, order="col", split=False,
                max_elements=1 << 27) -> complex:
    ts = expectation_network(circ, params, structure, split)
    return fold_sliced(sorted(ts, key=_sort_key(order)), max_elements)


def energy(circ, params, obs, order="col", split=False,
           max_elements=1 << 27) -> complex:
    re = im = 0.0
    for a, s in zip(obs.weights, obs.structures):
        v = expectation(circ, params, s, order, split, max_elements)
        re += float(a) * v.real
        im += float(a) * v.imag
    return complex(re, im)
