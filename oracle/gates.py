"""Gate matrices in complex128 (oracle; test infrastructure only).

Paper, section "Circuits and gates": qubit 0 is the most significant position,
a two-qubit gate on (q0, q1) is a 4x4 matrix indexed by 2*b(q0) + b(q1), and
``exp1`` gates have the form exp(i theta G) with G^2 = I.  The paper never
writes out its rotation gates; this oracle reads them as the standard
half-angle rotations R_G(theta) = exp(-i theta G / 2) for
G in {X, Y, Z, ZZ, XX, YY}, so that a shift of +-pi/2 gives the exact
parameter-shift gradient.

Gates absent from the paper follow their usual published definitions:

* sqrt(G) for a Pauli-like G (G^2 = I): the principal square root
  ((1+i)/2) I + ((1-i)/2) G, with W = (X + Y)/sqrt(2);
* fSim(theta, phi) (Foxen et al., PRL 125, 120504 (2020)):
  [[1,0,0,0],[0,cos t,-i sin t,0],[0,-i sin t,cos t,0],[0,0,0,e^{-i phi}]].

Channels with externalised randomness (sections "Externalizing the
randomness", "Batched Monte Carlo trajectory noise simulation",
"Demonstration of barren plateaus"): a status x in [0,1) is cut into
contiguous intervals whose lengths are the outcome probabilities, in the
listed order, and the operator of the interval holding x is applied:

* "depol" (probabilities (px, py, pz) in ``matrix``; status = angle 0):
  I, X, Y, Z with probabilities 1 - px - py - pz, px, py, pz;
* "rswitch" (angle 0 = t, angle 1 = status): RX(t), RY(t), RZ(t), a third
  each.

The cut points are computed and compared in float32 (the status arrives as
a float32 parameter), in the order written in ``_choice``, so that a
status next to a cut falls on the same side as in any float32
implementation of the same rule.  The status itself has no derivative.
"""
from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
W = (X + Y) / np.sqrt(2.0)
PAULI = [I2, X, Y, Z]          # structure values 0, 1, 2, 3


def _sqrt_pauli_like(g: np.ndarray) -> np.ndarray:
    return 0.5 * (1 + 1j) * I2 + 0.5 * (1 - 1j) * g


def _rot(gen: np.ndarray, t: float) -> np.ndarray:
    # exp(-i t G / 2) for G^2 = I
    d = gen.shape[0]
    return np.cos(t / 2) * np.eye(d, dtype=np.complex128) - 1j * np.sin(t / 2) * gen


def _drot(gen: np.ndarray, t: float) -> np.ndarray:
    d = gen.shape[0]
    return -0.5 * np.sin(t / 2) * np.eye(d, dtype=np.complex128) \
        - 0.5j * np.cos(t / 2) * gen


def _fsim(t: float, p: float) -> np.ndarray:
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = 1
    m[1, 1] = m[2, 2] = np.cos(t)
    m[1, 2] = m[2, 1] = -1j * np.sin(t)
    m[3, 3] = np.exp(-1j * p)
    return m


def _dfsim(t: float, p: float, which: int) -> np.ndarray:
    m = np.zeros((4, 4), dtype=np.complex128)
    if which == 0:
        m[1, 1] = m[2, 2] = -np.sin(t)
        m[1, 2] = m[2, 1] = -1j * np.cos(t)
    else:
        m[3, 3] = -1j * np.exp(-1j * p)
    return m


ZZ = np.kron(Z, Z)
XX = np.kron(X, X)
YY = np.kron(Y, Y)

_FIXED = {
    "h": np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0),
    "x": X, "y": Y, "z": Z,
    "s": np.array([[1, 0], [0, 1j]], dtype=np.complex128),
    "sqrt_x": _sqrt_pauli_like(X),
    "sqrt_y": _sqrt_pauli_like(Y),
    "sqrt_w": _sqrt_pauli_like(W),
    "cnot": np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]],
                     dtype=np.complex128),
    "cz": np.diag([1, 1, 1, -1]).astype(np.complex128),
}

_ROT_GEN = {"rx": X, "ry": Y, "rz": Z, "rzz": ZZ, "rxx": XX, "ryy": YY}


def _choice(status: float, cuts) -> int:
    """Index of the interval of [0,1) holding the status, for the interval
    ends `cuts` (float32; the last interval runs to 1)."""
    x = np.float32(status)
    for i, c in enumerate(cuts):
        if x < c:
            return i
    return len(cuts)


def _depol_cuts(g):
    # p0 = ((1 - px) - py) - pz, then p0 + px, then (p0 + px) + py, in float32
    px, py, pz = (np.float32(v) for v in g.matrix)
    p0 = np.float32(np.float32(np.float32(np.float32(1.0) - px) - py) - pz)
    c1 = np.float32(p0 + px)
    return [p0, c1, np.float32(c1 + py)]


_RSWITCH = [X, Y, Z]
_RSWITCH_CUTS = [np.float32(1.0) / np.float32(3.0), np.float32(2.0) / np.float32(3.0)]


def gate_angles(g, params) -> list:
    """Angles of gate g: params[slot] where slot >= 0, else the fixed value."""
    return [float(params[s]) if s >= 0 else float(f)
            for s, f in zip(g.params, g.fixed)]


def matrix(g, params) -> np.ndarray:
    """The 2^k x 2^k matrix of gate g (k = number of qubits)."""
    k = g.kind
    if k in _FIXED:
        return _FIXED[k].copy()
    if k in _ROT_GEN:
        (t,) = gate_angles(g, params)
        return _rot(_ROT_GEN[k], t)
    if k == "fsim":
        t, p = gate_angles(g, params)
        return _fsim(t, p)
    if k in ("u1", "u2"):
        d = 2 if k == "u1" else 4
        return np.array([complex(a, b) for a, b in g.matrix],
                        dtype=np.complex128).reshape(d, d)
    if k == "depol":
        (x,) = gate_angles(g, params)
        return PAULI[_choice(x, _depol_cuts(g))].copy()
    if k == "rswitch":
        t, x = gate_angles(g, params)
        return _rot(_RSWITCH[_choice(x, _RSWITCH_CUTS)], t)
    raise ValueError(f"unknown gate kind {k!r}")


def dmatrix(g, params, which: int) -> np.ndarray:
    """d(matrix)/d(angle number `which`) of gate g."""
    k = g.kind
    if k in _ROT_GEN:
        (t,) = gate_angles(g, params)
        return _drot(_ROT_GEN[k], t)
    if k == "fsim":
        t, p = gate_angles(g, params)
        return _dfsim(t, p, which)
    if k == "depol":
        return np.zeros((2, 2), dtype=np.complex128)
    if k == "rswitch":
        t, x = gate_angles(g, params)
        if which == 1:
            return np.zeros((2, 2), dtype=np.complex128)
        return _drot(_RSWITCH[_choice(x, _RSWITCH_CUTS)], t)
    raise ValueError(f"gate kind {k!r} has no angle")


def shift_rule_ok(kind: str) -> bool:
    """True for gates exp(-i t G/2) with G^2 = I, for which the two-point
    shift rule at +-pi/2 is exact."""
    return kind in _ROT_GEN
