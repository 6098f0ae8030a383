"""Pins of the oracle's tabulated-weights variant (the mapping functions'
table of coefficient values, paper Section 3.1): exact where every fraction
is a table node, and an error that falls as 1 / T otherwise."""
import numpy as np

from oracle import oracle as o


def test_table_is_exact_on_table_nodes():
    # h = 1 and P = 5: the stencil fraction is frac(x - lo - 1.5); with
    # x = lo + m + 1.5 + i / 8 every fraction is i / 8, a node of T = 8
    rng = np.random.default_rng(3)
    n, K = 40, 12
    m = rng.integers(0, K, size=(n, 3))
    i = rng.integers(0, 8, size=(n, 3))
    pos = m + 1.5 + i / 8.0
    q = rng.normal(size=n)
    exact = o.pppm(pos, q, (0, 0, 0), (K,) * 3, (K,) * 3, 5, 0.8, 1.0, "ad")
    tab = o.pppm(pos, q, (0, 0, 0), (K,) * 3, (K,) * 3, 5, 0.8, 1.0, "ad", table=8)
    assert np.array_equal(exact["rho"], tab["rho"])
    assert np.array_equal(exact["forces"], tab["forces"])


def test_table_error_falls_as_one_over_size():
    rng = np.random.default_rng(4)
    n, L, K = 300, 12.0, 16
    pos = rng.uniform(0, L, size=(n, 3))
    q = rng.normal(size=n)
    q -= q.mean()
    exact = o.pppm(pos, q, (0, 0, 0), (L,) * 3, (K,) * 3, 5, 0.5, 1.0, "ik")
    err = {}
    for T in (500, 5000):
        r = o.pppm(pos, q, (0, 0, 0), (L,) * 3, (K,) * 3, 5, 0.5, 1.0, "ik", table=T)
        err[T] = np.sqrt(((r["forces"] - exact["forces"]) ** 2).sum() / (exact["forces"] ** 2).sum())
        # a weight moves by at most max|dw/df| / (2T) < 1 / T
        assert np.abs(r["rho"] - exact["rho"]).max() <= 3 * np.abs(q).sum() / T
    assert 0 < err[5000] < err[500]
    assert 5.0 < err[500] / err[5000] < 20.0


def test_table_charge_gradient_close_to_exact():
    # dE/dq = phi(r) - ... interpolated with the tabulated weights stays
    # within the table's resolution of the exact adjoint
    rng = np.random.default_rng(5)
    n, L, K = 50, 10.0, 12
    pos = rng.uniform(0, L, size=(n, 3))
    q = rng.normal(size=n)
    g = o.energy_gradients(pos, q, (0, 0, 0), (L,) * 3, (K,) * 3, 4, 0.6, 1.0, "ad", table=1000)
    ge = o.energy_gradients(pos, q, (0, 0, 0), (L,) * 3, (K,) * 3, 4, 0.6, 1.0, "ad")
    rel = np.sqrt(((g["grad_q"] - ge["grad_q"]) ** 2).sum() / (ge["grad_q"] ** 2).sum())
    assert rel < 1e-2
