"""Pins of the oracle's Schatten-p shrink for general p (the norm of Sec. 3 for p other than 1, 2, inf).

The shrink is checked against things it is not built from:
  * a generic minimiser of 1/2 ||x - sigma||^2 + tau ||x||_p;
  * the optimality condition: sigma - x = tau grad ||x||_p when x != 0, and
    ||sigma||_q <= tau (dual norm) when x = 0;
  * the closed forms: the general code at p = 2 equals the group shrink, and
    it tends to the soft threshold (p -> 1) and to the l_inf shrink (p -> inf);
  * one full round with general p equals the literal eqs. (12)-(14) loop
    whose singular values are shrunk by the generic minimiser.
"""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle import segsalsa_ref as R
import pinlib
import synth


def general(sig, tau, p):
    q = p / (p - 1.0)
    sig = np.asarray(sig, dtype=np.float64)
    return np.maximum(sig - tau * R.project_lq_ball(sig / tau, q), 0.0)


def minimise(sig, tau, p):
    f = lambda x: 0.5 * np.sum((x - sig) ** 2) + tau * np.sum(np.abs(x) ** p) ** (1.0 / p)
    best = None
    for x0 in (sig, 0.5 * sig, sig * 0 + 1e-3):
        r = optimize.minimize(f, x0, method="Nelder-Mead", options=dict(xatol=1e-12, fatol=1e-15, maxiter=20000))
        if best is None or r.fun < best.fun:
            best = r
    return best.x


@pytest.mark.parametrize("p", [1.5, 3.0, 4.7])
def test_general_shrink_matches_minimiser_and_kkt(p):
    rng = np.random.default_rng(int(p * 10))
    q = p / (p - 1.0)
    sig = np.sort(rng.random((40, 2)) * 3.0, axis=1)[:, ::-1]
    sig[0] = [1.0, 1.0]          # merged singular values
    sig[1] = [2.0, 0.0]          # rank one
    tau = 0.7
    x = R.schatten_shrink(sig, tau, p)
    for i in range(len(sig)):
        xm = minimise(sig[i], tau, p)
        assert np.max(np.abs(x[i] - np.maximum(xm, 0))) < 1e-6
        if np.sum(x[i]) > 0:
            g = x[i] ** (p - 1.0) / np.sum(x[i] ** p) ** ((p - 1.0) / p)
            assert np.max(np.abs(sig[i] - x[i] - tau * g)) < 1e-10
        else:
            assert np.sum(sig[i] ** q) ** (1.0 / q) <= tau + 1e-12


def test_general_code_at_p2_and_limits():
    rng = np.random.default_rng(3)
    sig = np.sort(rng.random((30, 2)) * 3.0, axis=1)[:, ::-1]
    tau = 0.8
    assert np.max(np.abs(general(sig, tau, 2.0) - R.schatten_shrink(sig, tau, 2.0))) < 1e-12
    assert np.max(np.abs(general(sig, tau, 1.0 + 1e-6) - R.schatten_shrink(sig, tau, 1.0))) < 1e-4
    assert np.max(np.abs(general(sig, tau, 1e4) - R.schatten_shrink(sig, tau, math.inf))) < 1e-3


def test_general_p_round_matches_literal_loop():
    probs, _, _ = synth.make_image(4, 5, 3, 25, 1.0, 1.5)
    p = 3.0
    pr = R.Problem(synth.gaussian_patch_multipliers(1, 1.0), 1, p, 0.7, 1.3)
    N = 3
    z_lit = pinlib.literal_salsa(probs / probs.sum(0), pr.c, pr.M, p, pr.lam, pr.mu, N + 1)
    z_red = R.solve(probs, pr, N, solve_method="dense", prox2="svd")
    assert np.max(np.abs(z_lit - z_red)) < 1e-8
    z_eig = R.solve(probs, pr, N)
    assert np.max(np.abs(z_eig - z_red)) < 1e-12


@pytest.mark.parametrize("p,key", [(1.0, "sum_p1"), (2.0, "sum_p2"), (math.inf, "sum_pinf"), (3.0, "sum_p3"),
                                   (1.5, "sum_p1_5")])
def test_schatten_norm_hand_example(p, key):
    """The per-pixel Schatten-p norm (eq. (6)) on a hand-worked 2x2, K = 2 field, for general p too."""
    from test_oracle_operators import golden
    g = golden("snorm_2x2")
    z = g["z"].reshape(2, 2, 2)
    pr = R.Problem(np.array([1.0]), 0, p, 1.0, 1.0)
    nrm = R.schatten_norms(z, pr).reshape(2, 2)
    assert abs(float(np.sum(nrm)) - float(g[key][0])) < 1e-12
    if p == 3.0:
        assert abs(float(nrm[0, 0]) - float(g["n00_p3"][0])) < 1e-13
        assert abs(float(nrm[1, 1]) - float(g["n00_p3"][0])) < 1e-13
    if p == 1.5:
        assert abs(float(nrm[0, 0]) - float(g["n00_p1_5"][0])) < 1e-13


def test_objective_hand_example_general_p():
    """Objective of eq. (7) at a feasible-looking field, p = 3, against its hand-worked value."""
    from test_oracle_operators import golden
    g = golden("snorm_2x2")
    z = 0.05 * g["z"].reshape(2, 2, 2) + 0.25
    ph = np.full((2, 2, 2), 0.5)
    pr = R.Problem(np.array([1.0]), 0, 3.0, 0.8, 1.0)
    assert abs(R.objective(z, ph, pr, project=False) - float(g["objective_p3"][0])) < 1e-12


@pytest.mark.parametrize("p", [1.25, 3.0, 4.7])
def test_objective_matches_dense_evaluation(p):
    """The oracle's objective equals an independent evaluation (dense J by index arithmetic,
    LAPACK singular values, the l_p norm written out) at random fields, for general p."""
    rng = np.random.default_rng(int(10 * p))
    K, H, W, M = 3, 4, 5, 1
    c = synth.gaussian_patch_multipliers(M, 1.0)
    Jm = pinlib.dense_jacobian(H, W, K, c, M)
    for _ in range(3):
        z = rng.random((K, H, W))
        ph = rng.random((K, H, W))
        ph /= ph.sum(0)
        pr = R.Problem(c, M, p, 0.7, 1.0)
        ref = pinlib.objective_dense(z.reshape(-1), ph, Jm, K, H * W, (2 * M + 1) ** 2, 0.7, p)
        assert abs(R.objective(z, ph, pr, project=False) - ref) < 1e-12 * abs(ref)


def test_limit_matches_pdhg_general_p():
    """p = 3: the ADMM limit objective equals the minimum found by an independently written
    Chambolle-Pock solver (dual prox through its own l_q-ball projection).  At mu = 5 the
    iteration is feasible to 1e-9 after 500 rounds (the general-p shrink makes it slow to run)."""
    probs, _, _ = synth.make_image(5, 5, 3, 33, 1.0, 1.0)
    ph = probs / probs.sum(0)
    c = synth.gaussian_patch_multipliers(1, 1.0)
    pr = R.Problem(c, 1, 3.0, 0.6, 5.0)
    st, _ = R.solve(probs, pr, 500, return_state=True)
    z = st.z
    assert np.max(np.abs(z.sum(0) - 1)) < 1e-8 and z.min() > -1e-8
    obj = R.objective(z, ph, pr)
    _, obj_pd = pinlib.pdhg(ph, c, 1, 3.0, 0.6, 3000)
    assert abs(obj_pd - obj) < 1e-6 * abs(obj)
