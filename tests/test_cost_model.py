"""Host-only pins of the Eq. 2 cost-model fit (Sec. 3.2: alpha, beta, gamma
by least squares on measured multiplications, plus a per-product delta)."""
import numpy as np
import pytest
from scipy.optimize import nnls


@pytest.fixture(scope="module")
def atp():
    import os
    import paper_2201_04058_amd as atp
    if not os.path.exists(atp.LIB_PATH):
        from paper_2201_04058_amd import build
        build.build()
    atp.lib()
    return atp


def design(rng, n):
    nnz_x = rng.uniform(1e3, 1e7, n)
    n_op = nnz_x * rng.uniform(1, 300, n)
    nnz_z = n_op / rng.uniform(1, 12, n)
    return nnz_x, n_op, nnz_z


@pytest.mark.parametrize("seed", range(10))
def test_noiseless_data_recover_the_coefficients(atp, seed):
    rng = np.random.default_rng(seed)
    x, o, z = design(rng, 40)
    truth = rng.uniform(0.1, 5.0, 4) * np.array([1e-6, 1e-7, 1e-6, 1e-2])
    t = truth[0] * x + truth[1] * o + truth[2] * z + truth[3]
    coef, r2 = atp.cost_fit(x, o, z, t)
    assert np.allclose(coef, truth, rtol=1e-6, atol=0)
    assert r2 == pytest.approx(1.0, abs=1e-9)


@pytest.mark.parametrize("seed", range(10))
def test_noisy_fit_equals_nonnegative_least_squares(atp, seed):
    """Against scipy's NNLS on the same design; the cases are those where
    dropping the most negative unconstrained coefficient reaches the NNLS
    optimum (at most one coefficient at its bound)."""
    rng = np.random.default_rng(100 + seed)
    x, o, z = design(rng, 60)
    truth = np.array([2e-6, 1e-7, 3e-6, 0.05]) * rng.uniform(0.5, 2.0, 4)
    if seed % 2:
        truth[seed % 4] = 0.0
    t = truth[0] * x + truth[1] * o + truth[2] * z + truth[3]
    t = t * rng.uniform(0.9, 1.1, t.shape)
    A = np.stack([x, o, z, np.ones_like(x)], 1)
    s = np.linalg.norm(A, axis=0)
    ref, _ = nnls(A / s, t)
    ref = ref / s
    if (ref == 0).sum() > 1:
        pytest.skip("NNLS optimum with several coefficients at zero")
    coef, r2 = atp.cost_fit(x, o, z, t)
    assert np.all(np.asarray(coef) >= 0)
    assert np.allclose(coef, ref, rtol=1e-5, atol=1e-12)
    pred = A @ np.asarray(coef)
    assert r2 == pytest.approx(1 - ((t - pred) ** 2).sum() / ((t - t.mean()) ** 2).sum(), rel=1e-9)


def test_bad_arguments(atp):
    import ctypes
    L = atp.lib()
    out = (ctypes.c_double * 4)()
    assert L.atp_cost_fit(0, None, None, None, None, out, None) == atp.ATP_EINVAL
    assert L.atp_get_cost_model(None, out) == atp.ATP_EINVAL
    assert L.atp_set_cost_model(None, out) == atp.ATP_EINVAL
    assert L.atp_calibrate_cost_model(None, None, 1, out, None, None) == atp.ATP_EINVAL
