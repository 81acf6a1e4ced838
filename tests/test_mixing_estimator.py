"""The integrated-autocorrelation estimator of paper_2301_11735_amd.mixing on
series with a closed-form answer (CPU only): an AR(1) process
x_t = phi x_{t-1} + noise has tau_int = (1 + phi) / (2 (1 - phi)); white noise
has 1/2."""
import numpy as np
import pytest

from paper_2301_11735_amd.mixing import tau_int


@pytest.mark.parametrize("phi", [0.0, 0.5, 0.8, 0.95])
def test_tau_int_of_ar1(phi):
    rng = np.random.default_rng(int(100 * phi) + 1)
    taus = []
    for _ in range(20):
        e = rng.standard_normal(20000)
        x = np.empty_like(e)
        x[0] = e[0] / np.sqrt(1 - phi * phi)
        for t in range(1, e.size):
            x[t] = phi * x[t - 1] + e[t]
        taus.append(tau_int(x))
    exact = (1 + phi) / (2 * (1 - phi))
    est, err = np.mean(taus), np.std(taus, ddof=1) / np.sqrt(len(taus))
    # Sokal's window truncates a tail of relative size ~exp(-c) (c = 6)
    assert abs(est - exact) < 4 * err + 0.01 * exact, (est, err, exact)


def test_tau_int_of_constant_series():
    assert tau_int(np.ones(100)) == 0.5
