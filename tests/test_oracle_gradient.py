"""Pins of the FP64 reference gradient (oracle/segsalsa_torch_ref.py), on the CPU.

The reference gradient is PyTorch autograd through a differentiable
restatement of the rounds.  It is pinned to things other than itself:
  * its forward equals the numpy oracle's rounds (which the other oracle tests
    pin to the paper's definitions) for p in {1, 2, inf}, M in {0, 1, 2},
    probabilities and logits;
  * its gradient equals central finite differences of the numpy oracle's own
    forward (not of itself) along random directions, for the input, lambda
    and the patch multipliers;
  * invariances of the input normalisation: the loss depends on p only
    through p / 1^T p, so <dL/dp_i, p_i> = 0 per pixel, and on logits only up
    to a per-pixel constant, so sum_k dL/dlogit_ki = 0.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import segsalsa_ref as R
from oracle import segsalsa_torch_ref as TR

P_VALUES = [1.0, 2.0, math.inf]


def loss_np(z, labels, floor=1e-6):
    H, W = labels.shape
    zy = z[labels, np.arange(H)[:, None], np.arange(W)[None, :]]
    return float(-np.mean(np.log(np.maximum(zy, floor))))


def ref_grad(x, labels, c, M, p, lam, mu, iters, logits):
    xt = torch.from_numpy(x).clone().requires_grad_(True)
    ct = torch.tensor(np.asarray(c, dtype=np.float64), requires_grad=True)
    lt = torch.tensor(float(lam), dtype=torch.float64, requires_grad=True)
    ph = TR.softmax_input(xt) if logits else TR.normalise_input(xt)
    z = TR.solve_torch(ph, ct, M, p, lt, mu, iters)
    loss = TR.ce_loss(z, torch.from_numpy(labels))
    gx, gc, gl = torch.autograd.grad(loss, (xt, ct, lt), allow_unused=True, materialize_grads=True)
    return float(loss), gx.numpy(), gc.numpy(), float(gl)


@pytest.mark.parametrize("p", P_VALUES, ids=["p1", "p2", "pinf"])
@pytest.mark.parametrize("M", [0, 1, 2])
def test_forward_equals_numpy_oracle(p, M):
    x, logits, _ = synth.make_image(11, 13, 4, 20 + M, 1.0, 1.5)
    c = synth.gaussian_patch_multipliers(M, 1.0)
    for inp, is_logits in ((x, False), (logits, True)):
        zo = R.solve(inp, R.Problem(np.asarray(c), M, p, 0.8, 1.4), 7, is_logits=is_logits)
        xt = torch.from_numpy(inp)
        ph = TR.softmax_input(xt) if is_logits else TR.normalise_input(xt)
        zt = TR.solve_torch(ph, torch.tensor(c), M, p, torch.tensor(0.8, dtype=torch.float64), 1.4, 7).numpy()
        assert np.max(np.abs(zt - zo)) <= 1e-12


@pytest.mark.parametrize("p", P_VALUES, ids=["p1", "p2", "pinf"])
def test_gradient_matches_finite_differences_of_the_oracle(p):
    M, mu, iters, lam = 1, 1.5, 10, 0.6
    x, logits, labels = synth.make_image(10, 12, 4, 31, 1.0, 1.5)
    c = np.asarray(synth.gaussian_patch_multipliers(M, 1.0))
    _, gx, gc, gl = ref_grad(logits, labels, c, M, p, lam, mu, iters, True)

    def f(lg, cc, ll):
        return loss_np(R.solve(lg, R.Problem(cc, M, p, ll, mu), iters, is_logits=True), labels)

    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(2):
        d = rng.standard_normal(logits.shape)
        fd = (f(logits + h * d, c, lam) - f(logits - h * d, c, lam)) / (2 * h)
        assert abs(np.sum(gx * d) - fd) <= 1e-5 * abs(fd) + 1e-9
        dc = rng.standard_normal(c.shape)
        fd = (f(logits, c + h * dc, lam) - f(logits, c - h * dc, lam)) / (2 * h)
        assert abs(np.sum(gc * dc) - fd) <= 1e-5 * abs(fd) + 1e-9
    fd = (f(logits, c, lam + h) - f(logits, c, lam - h)) / (2 * h)
    assert abs(gl - fd) <= 1e-5 * abs(fd) + 1e-9


def test_normalisation_invariances():
    M, p = 1, 1.0
    x, logits, labels = synth.make_image(9, 10, 5, 41, 1.0, 1.5)
    c = synth.gaussian_patch_multipliers(M, 1.0)
    _, gx, _, _ = ref_grad(x, labels, c, M, p, 0.7, 1.2, 6, False)
    assert np.max(np.abs(np.sum(gx * x, axis=0))) <= 1e-12
    _, gl, _, _ = ref_grad(logits, labels, c, M, p, 0.7, 1.2, 6, True)
    assert np.max(np.abs(np.sum(gl, axis=0))) <= 1e-12
    assert np.max(np.abs(gl)) > 1e-6


def test_zero_rounds_is_the_normalisation_only():
    """With no rounds z = p_hat: the gradient is the loss gradient through softmax alone."""
    x, logits, labels = synth.make_image(6, 7, 3, 43, 1.0, 1.5)
    c = synth.gaussian_patch_multipliers(1, 1.0)
    _, gx, gc, gl = ref_grad(logits, labels, c, 1, 1.0, 0.7, 1.2, 0, True)
    ph = synth.softmax_fp64(logits)
    onehot = np.zeros_like(ph)
    H, W = labels.shape
    onehot[labels, np.arange(H)[:, None], np.arange(W)[None, :]] = 1.0
    expect = -(onehot - ph) / (H * W)     # d/dlogits of -(1/n) ln softmax_y
    assert np.max(np.abs(gx - expect)) <= 1e-15
    assert np.max(np.abs(gc)) == 0.0 and gl == 0.0
