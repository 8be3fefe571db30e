"""Convergence pins: the oracle's iteration reaches the minimiser of eq. (7).

The iteration is convex ADMM (Sec. 4), so its limit must not depend on mu, must
match an independent primal-dual solver and brute force, and must reduce to
the known closed-form minimisers in special cases.
"""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle import segsalsa_ref as R
import pinlib
import synth


def test_lambda_zero_gives_vertices():
    """lam = 0: the minimiser of sum -ln(p_i^T z_i) on the simplex is e_{argmax p_i}."""
    probs, _, _ = synth.make_image(8, 8, 4, 31, 1.0, 1.5)
    pr = R.Problem(synth.gaussian_patch_multipliers(1, 1.0), 1, 1.0, 0.0, 0.3)
    z = R.solve(probs, pr, 3000)
    vert = (np.arange(4)[:, None, None] == np.argmax(probs, axis=0)[None]).astype(float)
    assert np.max(np.abs(z - vert)) < 1e-9


def test_constant_field_gives_constant_vertex():
    """A constant p field: z = e_{argmax p} everywhere has zero prior and optimal data term."""
    p = np.broadcast_to(np.array([0.1, 0.6, 0.3])[:, None, None], (3, 6, 7)).copy()
    pr = R.Problem(synth.gaussian_patch_multipliers(1, 1.0), 1, 1.0, 2.0, 0.3)
    z = R.solve(p, pr, 3000)
    vert = np.zeros_like(p)
    vert[1] = 1.0
    assert np.max(np.abs(z - vert)) < 1e-9


def test_one_pixel_patch_frobenius_is_vector_tv():
    """L = 1 with the Schatten-2 norm is SegSALSA with the vector-TV prior: iterates agree."""
    probs, _, _ = synth.make_image(7, 9, 3, 32, 1.0, 1.5)
    ph = probs / probs.sum(0)
    pr = R.Problem(np.array([1.0]), 0, 2.0, 0.8, 1.1)
    z = R.solve(probs, pr, 25)
    z_vtv = pinlib.vtv_salsa(ph, 0.8, 1.1, 25)
    assert np.max(np.abs(z - z_vtv)) < 1e-12


def _converged(probs, pr, rounds):
    st, ph = R.solve(probs, pr, rounds, return_state=True)
    return st.z, ph


@pytest.mark.parametrize("p,lam", [(1.0, 0.6), (math.inf, 0.6), (2.0, 0.6)])
def test_limit_independent_of_mu_and_matches_pdhg(p, lam):
    probs, _, _ = synth.make_image(5, 5, 3, 33, 1.0, 1.0)
    ph = probs / probs.sum(0)
    c = synth.gaussian_patch_multipliers(1, 1.0)
    objs = []
    for mu in (5.0, 10.0, 20.0):
        pr = R.Problem(c, 1, p, lam, mu)
        z, _ = _converged(probs, pr, 2000)
        assert np.max(np.abs(z.sum(0) - 1)) < 1e-8 and z.min() > -1e-8   # feasible at convergence
        objs.append(R.objective(z, ph, pr))
    assert max(objs) - min(objs) < 1e-9 * abs(objs[0])
    zp, obj_pd = pinlib.pdhg(ph, c, 1, p, lam, 3000)
    assert abs(obj_pd - objs[0]) < 1e-6 * abs(objs[0])


def test_two_pixel_two_class_brute_force():
    """2 x 2 image, K = 2: z_i = (t_i, 1 - t_i); minimise over t in [0,1]^4 by Nelder-Mead."""
    p = np.array([[[0.7, 0.4], [0.45, 0.2]], [[0.3, 0.6], [0.55, 0.8]]])
    c = np.array([1.0])
    lam = 0.35
    pr = R.Problem(c, 0, 1.0, lam, 1.0)
    z, ph = _converged(p, pr, 8000)
    obj_admm = R.objective(z, ph, pr)

    def f(t):
        t = np.clip(t, 0.0, 1.0)
        zz = np.stack([t.reshape(2, 2), 1 - t.reshape(2, 2)])
        return R.objective(zz, ph, pr, project=False)
    best = math.inf
    grid = np.linspace(0.05, 0.95, 4)
    for a in grid:
        for b in grid:
            res = optimize.minimize(f, np.array([a, b, a, b]), method="Nelder-Mead",
                                    options=dict(xatol=1e-11, fatol=1e-13, maxiter=20000, maxfev=20000))
            best = min(best, res.fun)
    assert obj_admm <= best + 1e-8
    assert abs(obj_admm - best) < 1e-7 * abs(best)


@pytest.mark.parametrize("p", [1.0, math.inf])
def test_simplex_g4_reaches_the_same_minimiser(p):
    """Both readings of g4 split the same feasible set (with g3), so the limits coincide."""
    probs, _, _ = synth.make_image(5, 5, 3, 33, 1.0, 1.0)
    ph = probs / probs.sum(0)
    c = synth.gaussian_patch_multipliers(1, 1.0)
    objs = []
    for g4 in ("affine", "simplex"):
        pr = R.Problem(c, 1, p, 0.6, 5.0, g4=g4)
        z, _ = _converged(probs, pr, 2000)
        assert np.max(np.abs(z.sum(0) - 1)) < 1e-8 and z.min() > -1e-8
        objs.append(R.objective(z, ph, pr))
    assert abs(objs[0] - objs[1]) < 1e-9 * abs(objs[0])
