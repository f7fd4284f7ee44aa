"""Bitstring samples from the ensemble's probability vector (test infrastructure).

Sec. III-G averages the trajectories' probability vectors into sigma_approx, a
distribution over the 2^n computational-basis bitstrings.  A sampler of that
distribution returns basis index x with probability sigma(x) / sum(sigma).

``sample_bitstrings`` is inverse-transform sampling written out: with the
running sums F(x) = sigma(0) + ... + sigma(x) (in index order, float64) and a
uniform u in [0, 1), the sample is the smallest x with F(x) > u * F(2^n - 1).
When rounding leaves no such x (u * F(last) == F(last)), the sample is the
smallest x with F(x) >= u * F(last), i.e. the last index of positive mass.
Indices of zero mass are never returned.  Basis index x carries qubit q in
bit q, the order of sigma itself.

Pins (tests/test_oracle_sampling.py): hand-computed samples at and around the
cumulative boundaries of small vectors, stratified uniforms reproducing the
distribution's counts to within one, and a chi-square check of random draws.
"""
import numpy as np


def sample_bitstrings(sigma, u):
    sigma = np.asarray(sigma, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    F = np.cumsum(sigma)
    t = u * F[-1]
    out = np.empty(u.shape, dtype=np.int64)
    for i, ti in np.ndenumerate(t):
        x = int(np.argmax(F > ti)) if F[-1] > ti else int(np.argmax(F >= ti))
        out[i] = x
    return out
