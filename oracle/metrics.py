"""Distances between the ensemble estimate and the exact noisy state.

* ``paper_error``: Eq.(2), 1 - |<sqrt(sigma_approx), sqrt(sigma_exact)>|^2 on the
  probability vectors (diagonals), Sec. III-G.
* ``uhlmann_fidelity``: (Tr |sqrt(rho) sqrt(sigma)|)^2 on full density matrices.
* ``trace_distance``: (1/2) ||rho - sigma||_1.
* ``frobenius``: ||rho - sigma||_F.
"""
import numpy as np


def paper_error(sigma_approx, sigma_exact):
    a = np.sqrt(np.clip(np.real(sigma_approx), 0.0, None))
    b = np.sqrt(np.clip(np.real(sigma_exact), 0.0, None))
    return float(1.0 - abs(np.dot(a, b)) ** 2)


def _psd_sqrt(rho):
    w, V = np.linalg.eigh((rho + rho.conj().T) / 2)
    w = np.clip(w, 0.0, None)
    return (V * np.sqrt(w)) @ V.conj().T


def uhlmann_fidelity(rho, sigma):
    """(sum of sqrt eigenvalues of sqrt(rho) sigma sqrt(rho))^2."""
    s = _psd_sqrt(rho)
    m = s @ sigma @ s
    w = np.linalg.eigvalsh((m + m.conj().T) / 2)
    return float(np.sum(np.sqrt(np.clip(w, 0.0, None))) ** 2)


def uhlmann_fidelity_from_states(rho, Psi, K):
    """F(rho, (1/K) Psi^T Psi^*) for Psi = [K, 2^n] via the singular values of
    sqrt(rho) Psi^T / sqrt(K), avoiding the square root of the rank-deficient
    estimate."""
    s = _psd_sqrt(rho)
    sv = np.linalg.svd(s @ Psi.T / np.sqrt(K), compute_uv=False)
    return float(np.sum(sv) ** 2)


def trace_distance(rho, sigma):
    d = rho - sigma
    w = np.linalg.eigvalsh((d + d.conj().T) / 2)
    return float(0.5 * np.sum(np.abs(w)))


def frobenius(rho, sigma):
    return float(np.linalg.norm(rho - sigma))
