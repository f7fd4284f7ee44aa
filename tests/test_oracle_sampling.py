"""Pins of oracle.sampling against hand-computed samples and the distribution it draws from."""
import numpy as np
import pytest

from oracle.sampling import sample_bitstrings


def test_hand_computed_boundaries():
    # sigma = (1/4, 0, 1/2, 1/4): x=0 on [0, 1/4), x=2 on [1/4, 3/4), x=3 on [3/4, 1); x=1 never
    sigma = [0.25, 0.0, 0.5, 0.25]
    u = [0.0, 0.1, 0.2499, 0.25, 0.5, 0.7499, 0.75, 0.9999]
    assert sample_bitstrings(sigma, u).tolist() == [0, 0, 0, 2, 2, 2, 3, 3]


def test_unnormalised_vector_and_leading_zero():
    # an unnormalised vector (trace 2) samples like its normalisation; zero mass at x=0 is skipped at u=0
    sigma = [0.0, 1.0, 0.0, 0.5, 0.5]
    assert sample_bitstrings(sigma, [0.0, 0.49, 0.5, 0.74, 0.75, 0.99]).tolist() == [1, 1, 3, 3, 4, 4]


def test_top_end_returns_last_positive_mass():
    sigma = [0.5, 0.5, 0.0, 0.0]
    u = np.nextafter(1.0, 0.0)
    assert sample_bitstrings(sigma, [u]).tolist() == [1]
    assert sample_bitstrings([1.0], [0.0, 0.5, u]).tolist() == [0, 0, 0]


def test_stratified_counts_match_the_distribution():
    # u_i = (i + 1/2)/M hits each x about M sigma(x) times (within one)
    rng = np.random.default_rng(7)
    sigma = rng.random(64) ** 3
    sigma[[3, 17, 40]] = 0.0
    M = 100000
    x = sample_bitstrings(sigma, (np.arange(M) + 0.5) / M)
    counts = np.bincount(x, minlength=64)
    np.testing.assert_array_less(np.abs(counts - M * sigma / sigma.sum()), 1.0 + 1e-9)
    assert counts[[3, 17, 40]].sum() == 0


def test_random_draws_chi_square():
    rng = np.random.default_rng(11)
    sigma = rng.random(32)
    p = sigma / sigma.sum()
    M = 200000
    counts = np.bincount(sample_bitstrings(sigma, rng.random(M)), minlength=32)
    chi2 = float(((counts - M * p) ** 2 / (M * p)).sum())
    assert chi2 < 31 + 6 * np.sqrt(2 * 31)   # 31 degrees of freedom, about a 6-sigma bound


@pytest.mark.parametrize("n", [1, 3, 6])
def test_basis_state_always_sampled(n):
    sigma = np.zeros(1 << n)
    x0 = (1 << n) - 1 - (n // 2)
    sigma[x0] = 0.7
    u = np.linspace(0.0, np.nextafter(1.0, 0.0), 101)
    assert (sample_bitstrings(sigma, u) == x0).all()
