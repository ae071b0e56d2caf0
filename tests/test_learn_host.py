"""Host-side logic of paper_2503_20907_amd.learn that runs without a GPU."""
import numpy as np
import pytest


def test_nnls_gram_matches_scipy_nnls():
    from scipy.optimize import nnls
    from paper_2503_20907_amd import learn
    rng = np.random.default_rng(40)
    for trial in range(20):
        n = int(rng.integers(1, 6))
        A = rng.normal(size=(3 * n + 2, n))
        y = rng.normal(size=3 * n + 2)
        ref, _ = nnls(A, y)
        got = learn._nnls_gram(A.T @ A, A.T @ y)
        assert np.all(got >= 0)
        f_ref = np.linalg.norm(A @ ref - y)
        f_got = np.linalg.norm(A @ got - y)
        assert f_got <= f_ref * (1 + 1e-9) + 1e-12
        assert np.allclose(got, ref, atol=1e-7)
