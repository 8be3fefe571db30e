"""Pins of the oracle's SALSA round: the literal eqs. (12)-(14) loop and invariances."""
import math

import numpy as np
import pytest

from oracle import segsalsa_ref as R
import pinlib
import synth


def small_problem(H, W, K, M, seed, p=1.0, lam=0.7, mu=1.3):
    probs, _, _ = synth.make_image(H, W, K, seed, 1.0, 1.5)
    c = synth.gaussian_patch_multipliers(M, 1.0)
    return probs, R.Problem(c, M, p, lam, mu)


@pytest.mark.parametrize("p", [1.0, 2.0, math.inf])
def test_reduced_rounds_equal_literal_salsa(p):
    """N reduced rounds == N+1 z-updates of the literal loop (round-order reading)."""
    probs, pr = small_problem(4, 5, 3, 1, seed=21, p=p)
    N = 4
    z_lit = pinlib.literal_salsa(probs / probs.sum(0), pr.c, pr.M, p, pr.lam, pr.mu, N + 1)
    z_red = R.solve(probs, pr, N, solve_method="dense", prox2="svd")
    assert np.max(np.abs(z_lit - z_red)) < 1e-12
    z_fft = R.solve(probs, pr, N)
    assert np.max(np.abs(z_fft - z_red)) < 1e-12


def test_round_with_asymmetric_weights_matches_literal():
    probs, pr = small_problem(5, 4, 2, 1, seed=22)
    pr.c = np.array([0.1, 0.9, 0.3, 0.5, 1.0, 0.2, 0.8, 0.4, 0.6])
    z_lit = pinlib.literal_salsa(probs / probs.sum(0), pr.c, pr.M, 1.0, pr.lam, pr.mu, 4)
    z_red = R.solve(probs, pr, 3)
    assert np.max(np.abs(z_lit - z_red)) < 1e-12


def test_translation_equivariance():
    probs, pr = small_problem(9, 11, 4, 1, seed=23)
    z = R.solve(probs, pr, 10)
    sh = (4, 7)
    z2 = R.solve(np.roll(probs, sh, axis=(1, 2)), pr, 10)
    assert np.max(np.abs(np.roll(z, sh, axis=(1, 2)) - z2)) < 1e-13


def test_class_permutation_equivariance():
    probs, pr = small_problem(8, 7, 5, 1, seed=24)
    perm = np.array([3, 0, 4, 1, 2])
    z = R.solve(probs, pr, 8)
    z2 = R.solve(probs[perm], pr, 8)
    assert np.max(np.abs(z[perm] - z2)) < 1e-13


def test_transpose_equivariance():
    """Swapping image axes swaps D_h and D_v; the singular values are unchanged."""
    probs, pr = small_problem(6, 9, 3, 1, seed=25)
    c2 = pr.c.reshape(3, 3).T.reshape(-1)
    z = R.solve(probs, pr, 8)
    zt = R.solve(probs.transpose(0, 2, 1), R.Problem(c2, pr.M, pr.p, pr.lam, pr.mu), 8)
    assert np.max(np.abs(z.transpose(0, 2, 1) - zt)) < 1e-13


def test_probability_scale_invariance():
    """Per-pixel positive scaling of p leaves every iterate unchanged."""
    probs, pr = small_problem(7, 6, 3, 1, seed=26)
    rng = np.random.default_rng(1)
    scaled = probs * rng.uniform(0.01, 100.0, size=(1, 7, 6))
    z = R.solve(probs, pr, 12)
    st_s = R.init_state(probs / probs.sum(0), 9)
    ph_unnorm = scaled   # the prox of g1 with unnormalised p gives the same iterate
    for _ in range(12):
        st_s = R.salsa_round(st_s, ph_unnorm, pr)
    assert np.max(np.abs(z - st_s.z)) < 1e-13


def test_logits_input_is_softmax():
    probs, logits, _ = synth.make_image(6, 6, 4, 27, 1.0, 1.5)
    pr = R.Problem(synth.gaussian_patch_multipliers(1, 1.0), 1, 1.0, 1.0, 1.0)
    np.testing.assert_allclose(R.solve(logits, pr, 5, is_logits=True), R.solve(probs, pr, 5), atol=1e-14)


def test_residuals_match_definitions():
    probs, pr = small_problem(6, 5, 3, 1, seed=28)
    ph = probs / probs.sum(0)
    st = R.init_state(ph, 9)
    for _ in range(3):
        st = R.salsa_round(st, ph, pr)
    new, rp, rd = R.salsa_round(st, ph, pr, want_residuals=True)
    G = pinlib.dense_G(6, 5, 3, pr.c, pr.M)
    # u = d_new + v with v = G z - d_old; primal residual ||G z - u||
    z = st.z.reshape(-1)
    d_old = np.concatenate([st.d1.reshape(-1), st.d2.reshape(-1), st.d3.reshape(-1), st.d4.reshape(-1)])
    d_new = np.concatenate([new.d1.reshape(-1), new.d2.reshape(-1), new.d3.reshape(-1), new.d4.reshape(-1)])
    u = d_new + (G @ z - d_old)
    assert abs(rp - np.linalg.norm(G @ z - u)) < 1e-12 * (1 + rp)
    assert abs(rd - pr.mu * np.linalg.norm(G @ (new.z.reshape(-1) - z))) < 1e-12 * (1 + rd)


@pytest.mark.parametrize("p", [1.0, math.inf])
def test_simplex_g4_rounds_equal_literal_salsa(p):
    """g4 read as the probability-simplex projection (Sec. 4 text): reduced rounds == literal loop."""
    probs, _, _ = synth.make_image(4, 5, 4, 24, 2.0, 4.0)   # peaked probabilities: v4 leaves the simplex
    pr = R.Problem(synth.gaussian_patch_multipliers(1, 1.0), 1, p, 0.7, 1.3, g4="simplex")
    N = 4
    z_lit = pinlib.literal_salsa(probs / probs.sum(0), pr.c, pr.M, p, pr.lam, pr.mu, N + 1, g4="simplex")
    z_red = R.solve(probs, pr, N, solve_method="dense", prox2="svd")
    assert np.max(np.abs(z_lit - z_red)) < 1e-12
    # the two readings differ once some v4 leaves the simplex
    pr.g4 = "affine"
    z_aff = R.solve(probs, pr, N, solve_method="dense", prox2="svd")
    assert np.max(np.abs(z_aff - z_red)) > 1e-6
