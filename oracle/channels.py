"""Kraus sets of the noise channels, selection probabilities and thresholds.

Kraus sets (Sec. III-F, the operator sum of Eq.(1)):
  bitflip(p)     [sqrt(p) X, sqrt(1-p) I]                    (listed order kept)
  depol1(lam)    [sqrt(1-3lam/4) I, sqrt(lam/4) X, sqrt(lam/4) Y, sqrt(lam/4) Z]
  depol2(lam)    16 Pauli products P_a (x) P_b, index 4a+b, P_a on the gate's
                 first qubit: weight 1-15lam/16 for I(x)I and lam/16 otherwise.
                 Reading: the paper names a two-qubit depolarizing rate but no
                 Kraus set; this is the two-qubit analogue of its one-qubit set,
                 E(rho) = (1-lam) rho + lam I/4.
  ampdamp(g)     [[1,0],[0,sqrt(1-g)]], [[0,sqrt(g)],[0,0]]
  kraus          an explicit list.

Selection (Sec. III-G: a uniform number picks a Kraus operator, and the
operator it names is inserted).  The paper does not state the selection
probabilities; the reading used is q_j = Tr(K_j^dagger K_j) / d, which is the
squared coefficient of each Pauli for the mixed-unitary channels above, and the
operator inserted is K_j / sqrt(q_j), so that sum_j q_j (K_j/sqrt q_j) rho
(K_j/sqrt q_j)^dagger = E(rho) exactly (an unbiased estimator).

Integer thresholds: with c_j = q_0 + ... + q_j summed left to right in binary64,
T_j = min(2^32, floor(c_j * 2^32)) and T_{J-1} = 2^32; a 32-bit draw r selects
j = min{ j : r < T_j }.  For the named channels q_j is taken from the closed
forms below (same expressions, same evaluation order as the product path's
planner) so the thresholds are bit-identical on both sides.
"""
import math

import numpy as np

from .gates import I2, X, Y, Z, pauli_string


def selection_probs(ch):
    """q_j of a workloads.Channel, in the channel's Kraus order."""
    k, lam = ch.kind, ch.param
    if k == "bitflip":
        return [lam, 1.0 - lam]
    if k == "depol1":
        qp = lam / 4.0
        return [1.0 - 3.0 * qp, qp, qp, qp]
    if k == "depol2":
        qp = lam / 16.0
        return [1.0 - 15.0 * qp] + [qp] * 15
    if k == "ampdamp":
        return [1.0 - lam / 2.0, lam / 2.0]
    if k == "kraus":
        d = int(round(math.sqrt(len(ch.kraus[0]))))
        out = []
        for op in ch.kraus:
            s = 0.0
            for v in op:  # row-major, left to right
                v = complex(v)
                s = s + (v.real * v.real + v.imag * v.imag)
            out.append(s / d)
        return out
    raise ValueError(f"unknown channel kind {k!r}")


def kraus_ops(ch):
    """Kraus matrices of a workloads.Channel (local little-endian basis)."""
    k, lam = ch.kind, ch.param
    if k == "bitflip":
        return [math.sqrt(lam) * X, math.sqrt(1.0 - lam) * I2]
    if k == "depol1":
        return [math.sqrt(1.0 - 3.0 * lam / 4.0) * I2, math.sqrt(lam / 4.0) * X,
                math.sqrt(lam / 4.0) * Y, math.sqrt(lam / 4.0) * Z]
    if k == "depol2":
        ops = []
        for j in range(16):
            a, b = j // 4, j % 4
            w = 1.0 - 15.0 * lam / 16.0 if j == 0 else lam / 16.0
            ops.append(math.sqrt(w) * pauli_string([a, b]))
        return ops
    if k == "ampdamp":
        return [np.array([[1.0, 0.0], [0.0, math.sqrt(1.0 - lam)]], dtype=np.complex128),
                np.array([[0.0, math.sqrt(lam)], [0.0, 0.0]], dtype=np.complex128)]
    if k == "kraus":
        d = int(round(math.sqrt(len(ch.kraus[0]))))
        return [np.array(op, dtype=np.complex128).reshape(d, d) for op in ch.kraus]
    raise ValueError(f"unknown channel kind {k!r}")


def thresholds(q):
    """uint64 thresholds T_j for selection probabilities q (see module doc)."""
    out = []
    c = 0.0
    for j, qj in enumerate(q):
        c = c + qj
        if j == len(q) - 1:
            out.append(1 << 32)
        else:
            out.append(min(1 << 32, int(math.floor(c * 4294967296.0))))
    return out


def select(r, T):
    """Index j = min{ j : r < T_j } for a 32-bit draw r."""
    for j, t in enumerate(T):
        if r < t:
            return j
    raise AssertionError("last threshold is 2^32")
