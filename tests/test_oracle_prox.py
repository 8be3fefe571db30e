"""Pins of the oracle's proximity operators (eq. (10) and the Schatten MPO of Sec. 4)."""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle import segsalsa_ref as R
import pinlib
from test_oracle_operators import golden


def test_data_prox_hand_examples():
    g = golden("prox_data")
    for tag in ("a", "b"):
        p = g["p_" + tag].reshape(2, 1, 1)
        v = g["v_" + tag].reshape(2, 1, 1)
        np.testing.assert_allclose(R.prox_data(v, p, 1.0).reshape(-1), g["u_" + tag], atol=1e-15)


@pytest.mark.parametrize("mu", [0.3, 1.0, 4.0])
def test_data_prox_kkt_and_generic_minimiser(mu):
    rng = np.random.default_rng(int(mu * 10))
    K = 5
    p = rng.uniform(0.01, 1.0, size=(K, 4, 4))
    v = 2.0 * rng.standard_normal((K, 4, 4))    # both signs of p^T v
    u = R.prox_data(v, p, mu)
    t = np.sum(p * u, axis=0)
    assert np.all(t > 0)
    kkt = -p / t + mu * (u - v)
    assert np.max(np.abs(kkt)) < 1e-12
    # generic minimiser on a few pixels
    for (r, q) in [(0, 0), (1, 3), (3, 2)]:
        pv, vv = p[:, r, q], v[:, r, q]

        def f(x):
            s = pv @ x
            return np.inf if s <= 0 else -math.log(s) + 0.5 * mu * np.sum((x - vv) ** 2)

        def grad(x):
            return -pv / (pv @ x) + mu * (x - vv)
        x0 = vv + pv * (abs(pv @ vv) + 1.0) / (pv @ pv)      # feasible start, p^T x0 > 0
        res = optimize.minimize(f, x0, jac=grad, method="BFGS", options=dict(gtol=1e-13, maxiter=10000))
        assert np.max(np.abs(res.x - u[:, r, q])) < 1e-7


def test_data_prox_scale_invariance():
    """Per-pixel positive scaling of p leaves the prox unchanged (the prox of f + const)."""
    rng = np.random.default_rng(11)
    p = rng.uniform(0.01, 1.0, size=(4, 3, 3))
    v = rng.standard_normal((4, 3, 3))
    scale = rng.uniform(0.1, 30.0, size=(1, 3, 3))
    np.testing.assert_allclose(R.prox_data(v, p * scale, 1.7), R.prox_data(v, p, 1.7), atol=1e-14)


@pytest.mark.parametrize("p", [1.0, 2.0, math.inf])
def test_schatten_shrink_hand_example(p):
    g = golden("schatten_2x2")
    key = {1.0: "p1", 2.0: "p2", math.inf: "pinf"}[p]
    out = R.schatten_shrink(g["sigma"][None], g["tau"][0], p)[0]
    np.testing.assert_allclose(out, g[key], atol=1e-15)


@pytest.mark.parametrize("p", [1.0, 2.0, math.inf])
@pytest.mark.parametrize("M,K", [(1, 3), (2, 2), (0, 4)])
def test_schatten_prox_eigh_matches_svd(p, M, K):
    rng = np.random.default_rng(M * 7 + K)
    L = (2 * M + 1) ** 2
    Y = rng.standard_normal((L, 2, K, 5, 6))
    # include rank-1 and zero pixels (degenerate singular values)
    Y[:, 1, :, 0, 0] = 0.7 * Y[:, 0, :, 0, 0]
    Y[:, :, :, 1, 1] = 0.0
    Y[:, 1, :, 2, 2] = Y[:, 0, :, 2, 2] * 0
    for tau in (0.05, 0.8, 3.0):
        a = R.prox_schatten(Y, tau, p)
        b = R.prox_schatten_svd(Y, tau, p)
        assert np.max(np.abs(a - b)) < 1e-12


@pytest.mark.parametrize("p", [1.0, 2.0, math.inf])
def test_schatten_prox_generic_minimiser(p):
    """prox of tau ||X||_{S_p} for 2x2 X versus Nelder-Mead on the 4 entries."""
    rng = np.random.default_rng(5)
    tau = 0.6
    for trial in range(3):
        Y = rng.standard_normal((2, 2))

        def snorm(X):
            s = np.linalg.svd(X, compute_uv=False)
            return s.sum() if p == 1 else (np.linalg.norm(s) if p == 2 else s.max())

        def f(x):
            X = x.reshape(2, 2)
            return tau * snorm(X) + 0.5 * np.sum((X - Y) ** 2)
        best = None
        for start in (Y.reshape(-1), np.zeros(4), 0.5 * Y.reshape(-1)):
            res = optimize.minimize(f, start, method="Nelder-Mead",
                                    options=dict(xatol=1e-12, fatol=1e-15, maxiter=40000, maxfev=40000))
            if best is None or res.fun < best.fun:
                best = res
        # (LK) x 2 block with L = 1, K = 2
        Yb = np.empty((1, 2, 2, 1, 1))
        Yb[0, :, :, 0, 0] = Y.T            # entry [j,h,k] = Y[k, h]
        out = R.prox_schatten_svd(Yb, tau, p)[0, :, :, 0, 0].T
        assert f(out.reshape(-1)) <= best.fun + 1e-10
        assert np.max(np.abs(out - best.x.reshape(2, 2))) < 1e-5


def test_l1_ball_projection_vs_bisection():
    rng = np.random.default_rng(9)
    for _ in range(20):
        v = np.abs(rng.standard_normal(2)) * 3
        r = rng.uniform(0.1, 4.0)
        proj = R.project_l1_ball(v[None], r)[0]
        ref = v if v.sum() <= r else np.maximum(v - pinlib._l1_theta(v, r), 0.0)
        np.testing.assert_allclose(proj, ref, atol=1e-12)


def test_positive_and_sum_to_one():
    rng = np.random.default_rng(2)
    v = rng.standard_normal((5, 3, 4))
    u3 = R.prox_positive(v)
    assert np.all(u3 >= 0) and np.all((u3 == v) | (u3 == 0))
    u4 = R.prox_sum_to_one(v)
    np.testing.assert_allclose(u4.sum(axis=0), 1.0, atol=1e-14)
    diff = u4 - v                      # correction is a multiple of 1_K
    np.testing.assert_allclose(diff, np.broadcast_to(diff[:1], diff.shape), atol=1e-15)


def test_simplex_projection_vs_bisection():
    rng = np.random.default_rng(4)
    z = 2 * rng.standard_normal((6, 3, 3))
    P = R.project_simplex(z)
    for r in range(3):
        for q in range(3):
            np.testing.assert_allclose(P[:, r, q], pinlib.simplex_proj_vec(z[:, r, q]), atol=1e-12)
