"""GPU parity of the method's variants against the FP64 oracle.

* g4 read as the probability-simplex projection (Sec. 4's wording) instead
  of the affine projection of the definition (eq. (10)): FP64 within 1e-9,
  FP32 within 2e-4, single and batched solves, and the 145x145 workload.
* General Schatten p (1.25, 1.5, 3, 4.7, 10): FP64 within 1e-9, FP32 within
  2e-4, residuals and objective, the 145x145 workload.
"""
import math

import numpy as np
import pytest
import torch

from gpu_common import check_err, FP32_TOL, FP64_TOL, MARGIN, need_gpu, rounded_input, say, weights_as_seen
import synth
from oracle import segsalsa_ref as R

pytestmark = pytest.mark.gpu


def solve_variant(S, x_np, c, M, p, lam, mu, iters, dtype, **kw):
    K, H, W = x_np.shape
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(device="cuda", dtype=dtype)
    pr = S.Problem(K, H, W, M, c, p, lam, mu, iters, **kw)
    ws = torch.empty(S.segsalsa_str_workspace_size(pr, S._prec(dtype)), dtype=torch.uint8, device="cuda")
    z = torch.empty_like(x)
    st = S.segsalsa_str_solve(pr, x, z, ws, stats=kw.get("residual_every", 0) > 0)
    torch.cuda.synchronize()
    return z, st


def oracle_variant(x_np, c, M, p, lam, mu, iters, g4="affine"):
    return R.solve(x_np, R.Problem(np.asarray(c, dtype=np.float64), M, p, lam, mu, g4=g4), iters)


# (H, W, K, M, p, iters): several tiles and ragged tails; peaked probabilities so v4 leaves the simplex
SIMPLEX_CASES = [
    (9, 7, 4, 1, 1.0, 8),
    (33, 45, 6, 1, math.inf, 8),
    (40, 52, 16, 2, 1.0, 6),
    (29, 31, 3, 0, 2.0, 8),
    (70, 33, 9, 1, 1.0, 6),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("H,W,K,M,p,iters", SIMPLEX_CASES)
def test_simplex_g4_small(H, W, K, M, p, iters, dtype):
    S = need_gpu()
    say(f"case g4=simplex H={H} W={W} K={K} M={M} p={p} iters={iters} {dtype}")
    probs, _, _ = synth.make_image(H, W, K, 700 + H, 2.0, 4.0)
    c = synth.gaussian_patch_multipliers(M, 1.0)
    z, _ = solve_variant(S, probs, c, M, p, 0.7, 1.3, iters, dtype, g4_simplex=True)
    zo = oracle_variant(rounded_input(probs, dtype), weights_as_seen(c, dtype), M, p, 0.7, 1.3, iters, "simplex")
    za = oracle_variant(probs, c, M, p, 0.7, 1.3, iters, "affine")
    err = float(np.max(np.abs(z.double().cpu().numpy() - zo)))
    gap = float(np.max(np.abs(zo - za)))
    say(f"  max|z_gpu - z_oracle| = {err:.3e} (simplex vs affine reading: {gap:.2e})")
    assert gap > 1e-4, "the case should exercise the simplex projection"
    check_err(err, dtype)


def test_simplex_g4_residuals_match_oracle():
    S = need_gpu()
    probs, _, _ = synth.make_image(24, 28, 5, 91, 2.0, 4.0)
    c = synth.gaussian_patch_multipliers(1, 1.0)
    _, st = solve_variant(S, probs, c, 1, 1.0, 0.7, 1.3, 9, torch.float64, g4_simplex=True, residual_every=9)
    pr = R.Problem(np.asarray(c), 1, 1.0, 0.7, 1.3, g4="simplex")
    ph = R.normalize_input(probs, False)
    sto = R.init_state(ph, 9)
    for _ in range(8):
        sto = R.salsa_round(sto, ph, pr)
    _, rp, rd = R.salsa_round(sto, ph, pr, want_residuals=True)
    say(f"  primal {st['primal_res']:.6e} vs {rp:.6e}, dual {st['dual_res']:.6e} vs {rd:.6e}")
    assert abs(st["primal_res"] - rp) <= 1e-9 * rp and abs(st["dual_res"] - rd) <= 1e-9 * rd


def test_simplex_g4_batch_equals_single():
    S = need_gpu()
    shapes = [(37, 53, 4), (61, 29, 9), (16, 16, 8)]
    probs = [synth.make_image(H, W, K, 800 + i, 2.0, 4.0)[0] for i, (H, W, K) in enumerate(shapes)]
    c = synth.gaussian_patch_multipliers(1, 1.0)
    imgs, total = S.image_table([(K, H, W) for (H, W, K) in shapes], [0.7] * 3, [1.3] * 3)
    params = S.BatchParams(1, c, 1.0, 7, g4_simplex=True)
    packed = torch.cat([torch.from_numpy(x).reshape(-1) for x in probs]).cuda()
    z = torch.empty_like(packed)
    ws = torch.empty(S.segsalsa_str_batch_workspace_size(imgs, params, S.SEGSALSA_FP64), dtype=torch.uint8,
                     device="cuda")
    S.segsalsa_str_solve_batch(imgs, params, packed, z, ws)
    torch.cuda.synchronize()
    off = 0
    for (H, W, K), x in zip(shapes, probs):
        zs, _ = solve_variant(S, x, c, 1, 1.0, 0.7, 1.3, 7, torch.float64, g4_simplex=True)
        assert torch.equal(z[off:off + K * H * W].reshape(K, H, W), zs)
        off += K * H * W


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_simplex_g4_pines_145(dtype):
    """145x145, K = 16, 5x5 patch, lambda = mu = 2, 20 rounds, simplex g4."""
    S = need_gpu()
    wl = synth.WORKLOADS["pines_145x145_k16"]
    d = synth.make_workload(wl)
    iters = 20
    say(f"case {wl.name} g4=simplex {iters} rounds {dtype}")
    z, _ = solve_variant(S, d["probs"], d["weights"], wl.M, 1.0, wl.lam, wl.mu, iters, dtype, g4_simplex=True)
    zo = oracle_variant(rounded_input(d["probs"], dtype), weights_as_seen(d["weights"], dtype), wl.M, 1.0, wl.lam,
                        wl.mu, iters, "simplex")
    zg = z.double().cpu().numpy()
    err = float(np.max(np.abs(zg - zo)))
    say(f"  max err {err:.3e}")
    check_err(err, dtype)
    srt = np.sort(zo, axis=0)
    sure = (srt[-1] - srt[-2]) > MARGIN
    assert np.array_equal(np.argmax(zg, axis=0)[sure], np.argmax(zo, axis=0)[sure])


# general Schatten p (Sec. 3's norm for p other than 1, 2, inf): per-pixel Newton solve in the kernel,
# Moreau decomposition with a nested-bisection l_q projection in the oracle
GENERAL_P_CASES = [
    (9, 7, 4, 1, 1.5, 8),
    (33, 45, 6, 1, 3.0, 8),
    (40, 52, 16, 2, 4.7, 5),
    (29, 31, 3, 0, 1.25, 8),
    (47, 53, 5, 1, 10.0, 5),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("H,W,K,M,p,iters", GENERAL_P_CASES)
def test_general_p_small(H, W, K, M, p, iters, dtype):
    S = need_gpu()
    say(f"case general p={p} H={H} W={W} K={K} M={M} iters={iters} {dtype}")
    probs, _, _ = synth.make_image(H, W, K, 900 + H, 1.0, 1.5)
    c = synth.gaussian_patch_multipliers(M, 1.0)
    z, _ = solve_variant(S, probs, c, M, p, 0.8, 1.3, iters, dtype)
    zo = oracle_variant(rounded_input(probs, dtype), weights_as_seen(c, dtype), M, p, 0.8, 1.3, iters)
    err = float(np.max(np.abs(z.double().cpu().numpy() - zo)))
    say(f"  max|z_gpu - z_oracle| = {err:.3e}")
    check_err(err, dtype)


def test_general_p_residuals_and_objective():
    S = need_gpu()
    p = 3.0
    probs, _, _ = synth.make_image(24, 28, 5, 93, 1.0, 1.5)
    c = synth.gaussian_patch_multipliers(1, 1.0)
    z, st = solve_variant(S, probs, c, 1, p, 0.7, 1.3, 9, torch.float64, residual_every=9)
    pr = R.Problem(np.asarray(c), 1, p, 0.7, 1.3)
    ph = R.normalize_input(probs, False)
    sto = R.init_state(ph, 9)
    for _ in range(8):
        sto = R.salsa_round(sto, ph, pr)
    sto, rp, rd = R.salsa_round(sto, ph, pr, want_residuals=True)
    obj = R.objective(sto.z, ph, pr)
    say(f"  primal {st['primal_res']:.6e} vs {rp:.6e}, dual {st['dual_res']:.6e} vs {rd:.6e}, "
        f"objective {st['objective']:.10e} vs {obj:.10e}")
    assert abs(st["primal_res"] - rp) <= 1e-9 * rp and abs(st["dual_res"] - rd) <= 1e-9 * rd
    assert abs(st["objective"] - obj) <= 1e-9 * abs(obj)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_general_p_pines_145(dtype):
    """145x145, K = 16, 5x5 patch, lambda = mu = 2, Schatten-3, 4 rounds (the oracle's l_q projection is slow)."""
    S = need_gpu()
    wl = synth.WORKLOADS["pines_145x145_k16"]
    d = synth.make_workload(wl)
    iters = 4
    say(f"case {wl.name} p=3 {iters} rounds {dtype}")
    z, _ = solve_variant(S, d["probs"], d["weights"], wl.M, 3.0, wl.lam, wl.mu, iters, dtype)
    zo = oracle_variant(rounded_input(d["probs"], dtype), weights_as_seen(d["weights"], dtype), wl.M, 3.0, wl.lam,
                        wl.mu, iters)
    err = float(np.max(np.abs(z.double().cpu().numpy() - zo)))
    say(f"  max err {err:.3e}")
    check_err(err, dtype)
