"""Plain statevector and density-matrix evolution (complex128).

A state on n qubits is stored as a numpy tensor of shape (2,)*n whose C-order
flattening is the basis index (qubit q = bit q), so qubit q lives on tensor
axis n-1-q.  A density matrix rho[i, j] = <i|rho|j> is a tensor of shape
(2,)*(2n): the first n axes carry the row (ket) bits, the last n the column
(bra) bits.

Every k-qubit operator is applied as a tensor contraction of its 2^k x 2^k
matrix with the k tensor axes it acts on.
"""
import numpy as np


def apply_matrix(t, M, axes):
    """Apply the 2^d x 2^d matrix M (local index = sum_t bit_t << t) to the
    tensor axes `axes` (axes[t] carries local bit t) of tensor t:
    out[..o..] = sum_i M[o, i] t[..i..], as one tensordot over the d axes."""
    d = len(axes)
    Mt = np.asarray(M, dtype=np.complex128).reshape((2,) * (2 * d))
    # Mt axes: output bits d-1..0, then input bits d-1..0 (C order of the local index)
    in_axes = [axes[d - 1 - i] for i in range(d)]
    r = np.tensordot(Mt, t, axes=(list(range(d, 2 * d)), in_axes))
    return np.ascontiguousarray(np.moveaxis(r, list(range(d)), in_axes))


def zero_state(n):
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    return psi


def apply_to_state(psi, M, qubits):
    n = psi.ndim
    return apply_matrix(psi, M, [n - 1 - q for q in qubits])


def apply_to_rho(rho, M, qubits):
    """rho -> M rho M^dagger."""
    n = rho.ndim // 2
    r = apply_matrix(rho, M, [n - 1 - q for q in qubits])
    return apply_matrix(r, np.conj(M), [2 * n - 1 - q for q in qubits])


def apply_kraus_sum(rho, ops, qubits):
    """Eq.(1) literally: sum_j K_j rho K_j^dagger."""
    acc = None
    for K in ops:
        t = apply_to_rho(rho, K, qubits)
        acc = t if acc is None else acc + t
    return acc


def superoperator(ops):
    """S = sum_j conj(K_j) (x) K_j, acting on the local index
    (ket bits) + (bra bits) << d, so that vec(E(rho)) = S vec(rho) on the
    2d axes (ket qubits, bra qubits): the operator sum of Eq.(1) regrouped."""
    S = None
    for K in ops:
        t = np.kron(np.conj(K), K)
        S = t if S is None else S + t
    return S


def apply_superoperator(rho, S, qubits):
    n = rho.ndim // 2
    axes = [n - 1 - q for q in qubits] + [2 * n - 1 - q for q in qubits]
    return apply_matrix(rho, S, axes)


def rho_matrix(rho):
    n = rho.ndim // 2
    return rho.reshape(1 << n, 1 << n)
