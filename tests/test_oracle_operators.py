"""Pins of the oracle's linear operators: J, J^T, G^T G and the z-update solve."""
import math
import os

import numpy as np
import pytest

from oracle import segsalsa_ref as R
import pinlib

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.txt")


def golden(block):
    out, cur = {}, None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line[1:-1]
            continue
        if cur == block:
            k, v = line.split("=")
            out[k.strip()] = np.array([float(x) for x in v.split()])
    return out


def test_forward_difference_hand_example():
    g = golden("diff_1x3")
    z = g["z"].reshape(1, 1, 3)
    np.testing.assert_array_equal(R.diff_h(z).reshape(-1), g["dh"])
    np.testing.assert_array_equal(R.diff_h_adj(R.diff_h(z)).reshape(-1), g["dht_dh"])


def test_jacobian_hand_example_and_structure_tensor():
    g = golden("jac_2x3")
    z = g["z"].reshape(1, 2, 3)
    Jz = R.jacobian(z, np.array([1.0]), 0)
    np.testing.assert_array_equal(Jz[0, 0, 0].reshape(-1), g["dh"])
    np.testing.assert_array_equal(Jz[0, 1, 0].reshape(-1), g["dv"])
    pr = R.Problem(np.array([1.0]), 0, 1.0, 1.0, 1.0)
    np.testing.assert_allclose(R.schatten_norms(z, pr).reshape(2, 3)[0, 0], g["snorm00"][0], rtol=1e-15)


@pytest.mark.parametrize("H,W,K,M", [(5, 6, 2, 1), (4, 5, 3, 0), (6, 5, 1, 2)])
def test_jacobian_matches_dense_index_arithmetic(H, W, K, M):
    rng = np.random.default_rng(H * 100 + W)
    L = (2 * M + 1) ** 2
    c = rng.uniform(0.2, 1.5, size=L)            # asymmetric weights: direction matters
    z = rng.standard_normal((K, H, W))
    Jm = pinlib.dense_jacobian(H, W, K, c, M)
    np.testing.assert_allclose(R.jacobian(z, c, M).reshape(-1), Jm @ z.reshape(-1), atol=1e-13)
    w = rng.standard_normal((L, 2, K, H, W))
    np.testing.assert_allclose(R.jacobian_adj(w, c, M).reshape(-1), Jm.T @ w.reshape(-1), atol=1e-13)


def test_adjoint_dot_product():
    rng = np.random.default_rng(7)
    K, H, W, M = 3, 6, 7, 1
    c = rng.uniform(0.1, 1.0, size=9)
    x = rng.standard_normal((K, H, W))
    Y = rng.standard_normal((9, 2, K, H, W))
    lhs = np.sum(R.jacobian(x, c, M) * Y)
    rhs = np.sum(x * R.jacobian_adj(Y, c, M))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_jtj_is_weighted_laplacian():
    """J^T J = (sum_j c_j^2) (D_h^T D_h + D_v^T D_v): periodic shifts are orthogonal."""
    rng = np.random.default_rng(8)
    K, H, W, M = 2, 7, 9, 2
    c = rng.uniform(0.1, 1.0, size=25)
    x = rng.standard_normal((K, H, W))
    lap = R.diff_h_adj(R.diff_h(x)) + R.diff_v_adj(R.diff_v(x))
    np.testing.assert_allclose(R.gtg_apply(x, c, M), 3 * x + np.sum(c * c) * lap, atol=1e-12)


@pytest.mark.parametrize("H,W", [(8, 8), (5, 7), (1, 6)])
def test_symbol_closed_form(H, W):
    """Eigenvalues of 3I + W (D_h^T D_h + D_v^T D_v): 3 + W (4 sin^2(pi kx/W) + 4 sin^2(pi ky/H))."""
    c = np.array([0.3, 0.9, 0.2, 0.5, 1.0, 0.4, 0.7, 0.1, 0.6])
    Wt = float(np.sum(c * c))
    ky = np.arange(H)[:, None]
    kx = np.arange(W)[None, :]
    closed = 3 + Wt * (4 * np.sin(math.pi * kx / W) ** 2 + 4 * np.sin(math.pi * ky / H) ** 2)
    np.testing.assert_allclose(R.gtg_symbol(H, W, c, 1), closed, atol=1e-12)


@pytest.mark.parametrize("H,W,K,M", [(4, 5, 2, 1), (3, 3, 3, 1), (6, 4, 1, 0)])
def test_solve_methods_agree_and_satisfy_stencil(H, W, K, M):
    rng = np.random.default_rng(H + 10 * W)
    L = (2 * M + 1) ** 2
    c = rng.uniform(0.2, 1.0, size=L)
    rhs = rng.standard_normal((K, H, W))
    zf = R.solve_gtg(rhs, c, M, "fft")
    zd = R.solve_gtg(rhs, c, M, "dft")
    zD = R.solve_gtg(rhs, c, M, "dense")
    np.testing.assert_allclose(zf, zD, atol=1e-12)
    np.testing.assert_allclose(zd, zD, atol=1e-12)
    # explicit 5-point stencil of 3 + Wt * (-Laplacian), periodic
    Wt = float(np.sum(c * c))
    sten = (3 + 4 * Wt) * zf - Wt * (np.roll(zf, 1, -1) + np.roll(zf, -1, -1) + np.roll(zf, 1, -2)
                                     + np.roll(zf, -1, -2))
    np.testing.assert_allclose(sten, rhs, atol=1e-12)
    # least squares on the dense stacked operator G (eq. (12)) gives the same z
    G = pinlib.dense_G(H, W, K, c, M)
    b = G @ zD.reshape(-1)
    z_ls = np.linalg.lstsq(G, b, rcond=None)[0]
    np.testing.assert_allclose(z_ls, zD.reshape(-1), atol=1e-11)


def test_gtg_is_normal_matrix_of_dense_G():
    rng = np.random.default_rng(3)
    H, W, K, M = 4, 5, 2, 1
    c = rng.uniform(0.2, 1.0, size=9)
    G = pinlib.dense_G(H, W, K, c, M)
    x = rng.standard_normal((K, H, W))
    np.testing.assert_allclose(R.gtg_apply(x, c, M).reshape(-1), G.T @ (G @ x.reshape(-1)), atol=1e-12)
