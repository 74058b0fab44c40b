"""The OpenMP build of the oracle (all-cores CPU baseline only) against the
plain build: the row product is computed row by row in both (bitwise); the
transposed product adds the same terms per row shard and then over the
shards (1e-14 relative); adaptive steps agree to rounding with the same
decisions.  The tests themselves use the plain build."""
import numpy as np
import pytest

import lpgen
import oracle


@pytest.fixture
def both():
    oracle.set_threaded(False)
    yield
    oracle.set_threaded(False)


def test_threaded_build_matches_the_plain_oracle(both):
    lp = lpgen.planted_skewed(40000, 50000, seed=5, n_dense=40)
    v = oracle.LPView.of(lp)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    a0, t0 = oracle.spmv(v, x), oracle.spmv_t(v, y)
    s0 = oracle.Solver(lp)
    s0.iterate(6)
    oracle.set_threaded(True)
    a1, t1 = oracle.spmv(v, x), oracle.spmv_t(v, y)
    s1 = oracle.Solver(lp)
    s1.iterate(6)
    assert np.array_equal(a0, a1)
    scale = np.abs(lp.csr()).T @ np.abs(y)
    assert np.all(np.abs(t1 - t0) <= 1e-14 * scale + 1e-300)
    assert s0.counters()["attempts"] == s1.counters()["attempts"]
    for k in ("x", "y", "ax", "aty"):
        a, b = getattr(s1, k), getattr(s0, k)
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b), k
