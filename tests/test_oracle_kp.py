"""Pins of the oracle's Kennedy-Pendleton SU(2) sampler against closed forms:
the histogram of a0 against the exact density sqrt(1-a0^2) exp(alpha a0)
(chi-square over 50 bins), the mean I2/I1, the isotropy of the direction and
the one-attempt acceptance sqrt(2 pi alpha) exp(-alpha) I1(alpha)."""
import numpy as np
import pytest
from scipy import stats

from closed_forms import kp_acceptance, kp_bin_probs, kp_mean
from oracle import su3ref

ALPHAS = [0.5, 2.0, 8.0, 13.0, 30.0]
N = 300_000


@pytest.mark.parametrize("alpha", ALPHAS)
def test_kp_histogram_matches_exact_density(alpha):
    a, over, _ = su3ref.kp_draws(alpha, seed=1000 + int(alpha * 10), n=N, cap=10000)
    assert over == 0
    a0 = a[:, 0]
    edges = np.linspace(-1, 1, 51)
    probs, total = kp_bin_probs(edges, alpha)
    assert abs(total - 1) < 1e-9  # the bin integrals reproduce pi I1(alpha)/alpha
    counts, _ = np.histogram(a0, bins=edges)
    exp = probs * N
    keep = exp > 5
    chi2 = (((counts - exp) ** 2 / exp)[keep]).sum()
    dof = keep.sum() - 1
    assert stats.chi2.sf(chi2, dof) > 1e-4, (chi2, dof)
    err = a0.std() / np.sqrt(N)
    assert abs(a0.mean() - kp_mean(alpha)) < 5 * err


@pytest.mark.parametrize("alpha", [2.0, 13.0])
def test_kp_direction_isotropic_and_unit(alpha):
    a, _, _ = su3ref.kp_draws(alpha, seed=7, n=N, cap=10000)
    assert np.abs((a ** 2).sum(axis=1) - 1).max() < 1e-14
    vec = a[:, 1:]
    nrm = np.linalg.norm(vec, axis=1)
    n = vec[nrm > 1e-6] / nrm[nrm > 1e-6, None]
    m = len(n)
    assert np.all(np.abs(n.mean(axis=0)) < 5 / np.sqrt(3 * m))
    assert np.all(np.abs((n ** 2).mean(axis=0) - 1 / 3) < 5 * np.sqrt(4 / 45 / m))
    # cos(theta) = n3 is uniform on [-1, 1]
    assert stats.kstest(n[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-4


@pytest.mark.parametrize("alpha", ALPHAS)
def test_kp_one_attempt_acceptance(alpha):
    a, over, tries = su3ref.kp_draws(alpha, seed=55, n=N, cap=1)
    assert tries == N
    acc = 1 - over / N
    p = kp_acceptance(alpha)
    assert abs(acc - p) < 5 * np.sqrt(p * (1 - p) / N)
    # rejected draws are reported as NaN, accepted ones as unit quaternions
    assert np.isnan(a[:, 0]).sum() == over
