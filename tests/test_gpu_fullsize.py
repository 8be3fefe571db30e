"""Full-size GPU checks, in the launch configuration the benchmark times.

* 145x145, K = 16, 5x5 patch, 300 rounds: z against the FP64 oracle element
  by element (FP64 <= 1e-9, FP32 <= 2e-4), labels where the margin > 1e-3.
* 610x340, K = 9, 5x5 patch: the whole field against the FP64 oracle
  element by element after 8 rounds (the oracle takes ~4 s a round here).
* 610x340 (K = 9) and 2048x2048 (K = 16), 500 rounds: too long (or, at
  2048x2048, too large) for the oracle, so (a) FP32 z within 2e-4 (and the
  1e-5 rounding envelope) of FP64 z over all rounds and
  (b) one round checked locally at sampled pixels: from the exported state
  before and after the round, every multiplier update and the z-update's
  normal equations A z_new = G^T (u + d) are recomputed with the oracle's
  functions on small periodic windows around each pixel (the round is local
  except for the solve, whose 5-point stencil is local).
"""
import math

import numpy as np
import pytest
import torch

from gpu_common import check_err, FP32_TOL, FP64_TOL, MARGIN, need_gpu, oracle_solve, rounded_input, say, weights_as_seen
import synth
from oracle import segsalsa_ref as R

pytestmark = pytest.mark.gpu


def run(S, wl, d, dtype, iters=None):
    x = torch.from_numpy(d["probs"]).to(device="cuda", dtype=dtype)
    pr = S.Problem(wl.K, wl.H, wl.W, wl.M, d["weights"], wl.schatten_p, wl.lam, wl.mu,
                   wl.iters if iters is None else iters)
    ws = torch.empty(S.segsalsa_str_workspace_size(pr, S._prec(dtype)), dtype=torch.uint8, device="cuda")
    z = torch.empty_like(x)
    S.segsalsa_str_solve(pr, x, z, ws)
    torch.cuda.synchronize()
    return z, ws, pr


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_pines_145_full_against_oracle(dtype):
    S = need_gpu()
    wl = synth.WORKLOADS["pines_145x145_k16"]
    d = synth.make_workload(wl)
    say(f"case {wl.name} {dtype}: GPU {wl.iters} rounds")
    z, ws, _ = run(S, wl, d, dtype)
    zg = z.double().cpu().numpy()
    del ws
    say("  oracle running (about a minute)")
    zo = oracle_solve(rounded_input(d["probs"], dtype), weights_as_seen(d["weights"], dtype), wl.M, wl.schatten_p,
                      wl.lam, wl.mu, wl.iters)
    err = float(np.max(np.abs(zg - zo)))
    say(f"  max |z_gpu - z_oracle| = {err:.3e}")
    check_err(err, dtype)
    srt = np.sort(zo, axis=0)
    sure = (srt[-1] - srt[-2]) > MARGIN
    assert np.array_equal(np.argmax(zg, axis=0)[sure], np.argmax(zo, axis=0)[sure])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_scene_610x340_whole_field_against_oracle(dtype):
    S = need_gpu()
    wl = synth.WORKLOADS["scene_610x340_k9"]
    d = synth.make_workload(wl)
    iters = 8
    say(f"case {wl.name} {dtype}: GPU and oracle, {iters} rounds, whole field")
    z, ws, _ = run(S, wl, d, dtype, iters=iters)
    zg = z.double().cpu().numpy()
    del ws
    say("  oracle running (about half a minute)")
    zo = oracle_solve(rounded_input(d["probs"], dtype), weights_as_seen(d["weights"], dtype), wl.M, wl.schatten_p,
                      wl.lam, wl.mu, iters)
    err = float(np.max(np.abs(zg - zo)))
    say(f"  max |z_gpu - z_oracle| = {err:.3e} over {zo.size} values")
    check_err(err, dtype)
    srt = np.sort(zo, axis=0)
    sure = (srt[-1] - srt[-2]) > MARGIN
    assert np.array_equal(np.argmax(zg, axis=0)[sure], np.argmax(zo, axis=0)[sure])


def gather(t, rows, cols):
    """t[..., rows, cols] for wrapped index vectors, on the device, returned to the host."""
    return t[..., rows[:, None], cols[None, :]].double().cpu().numpy()


def export(S, pr, ws, dtype):
    K, H, W = pr.K, pr.H, pr.W
    L = (2 * pr.patch_radius + 1) ** 2
    d1 = torch.empty(K, H, W, dtype=dtype, device="cuda")
    d3 = torch.empty_like(d1)
    d4 = torch.empty_like(d1)
    d2 = torch.empty(L, 2, K, H, W, dtype=dtype, device="cuda")
    S.segsalsa_str_state_export(pr, ws, d1, d2, d3, d4)
    torch.cuda.synchronize()
    return d1, d2, d3, d4


def local_round_check(wl, c, phat_dev, zo, old, zn, new, pixels, tol):
    """Recompute one round at the given pixels from the exported states (see module docstring)."""
    M = wl.M
    C = 2 * M + 1          # window centre; the window spans offsets -2M-1 .. 2M+1
    tau = wl.lam / wl.mu
    pr = R.Problem(np.asarray(c, dtype=np.float64), M, wl.schatten_p, wl.lam, wl.mu)
    Wt = float(np.sum(pr.c ** 2))
    worst = 0.0
    for (r, q) in pixels:
        rows = torch.tensor([(r + o) % wl.H for o in range(-C, C + 1)], device="cuda")
        cols = torch.tensor([(q + o) % wl.W for o in range(-C, C + 1)], device="cuda")
        z_w = gather(zo, rows, cols)
        d2o_w = gather(old[1], rows, cols)
        d2n_w = gather(new[1], rows, cols)
        Y_w = R.jacobian(z_w, pr.c, M) - d2o_w          # valid at offsets -M-1 .. M
        # g2 prox at the centre pixel
        u2 = R.prox_schatten(Y_w[..., C:C + 1, C:C + 1], tau, wl.schatten_p)
        e2 = np.max(np.abs((u2 - Y_w[..., C:C + 1, C:C + 1]) - d2n_w[..., C:C + 1, C:C + 1]))
        # g1, g3, g4 at the centre pixel
        ph = phat_dev[:, r, q].double().cpu().numpy()[:, None, None]
        zc = z_w[:, C:C + 1, C:C + 1]
        d1o, d3o, d4o = (old[i][:, r, q].double().cpu().numpy()[:, None, None] for i in (0, 2, 3))
        d1n, d3n, d4n = (new[i][:, r, q].double().cpu().numpy()[:, None, None] for i in (0, 2, 3))
        v1, v3, v4 = zc - d1o, zc - d3o, zc - d4o
        e1 = np.max(np.abs((R.prox_data(v1, ph, wl.mu) - v1) - d1n))
        e3 = np.max(np.abs((R.prox_positive(v3) - v3) - d3n))
        e4 = np.max(np.abs((R.prox_sum_to_one(v4) - v4) - d4n))
        # normal equations of the z-update at the centre: A z_new = G^T (u + d)
        a2_w = 2.0 * d2n_w + Y_w
        rhs = (v1 + 2 * d1n) + np.abs(v3) + (v4 + 2 * d4n) + R.jacobian_adj(a2_w, pr.c, M)[:, C:C + 1, C:C + 1]
        zn_w = gather(zn, rows[C - 1:C + 2], cols[C - 1:C + 2])
        sten = (3 + 4 * Wt) * zn_w[:, 1, 1] - Wt * (zn_w[:, 0, 1] + zn_w[:, 2, 1] + zn_w[:, 1, 0] + zn_w[:, 1, 2])
        e5 = np.max(np.abs(sten - rhs[:, 0, 0]))
        worst = max(worst, e1, e2, e3, e4, e5)
    say(f"  local round check over {len(pixels)} pixels: worst {worst:.2e}")
    assert worst <= tol


def sample_pixels(H, W, n, seed):
    rng = np.random.default_rng(seed)
    pts = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, 0), (0, W // 2)]
    pts += [(int(rng.integers(0, H)), int(rng.integers(0, W))) for _ in range(n)]
    return pts


@pytest.mark.parametrize("name", ["scene_610x340_k9", "large_2048x2048_k16"])
def test_fullsize_fp32_vs_fp64_and_local_round(name):
    S = need_gpu()
    wl = synth.WORKLOADS[name]
    d = synth.make_workload(wl)
    say(f"case {name}: FP64 and FP32 GPU, {wl.iters} rounds")
    z64, ws, pr = run(S, wl, d, torch.float64)
    z32, ws32, _ = run(S, wl, d, torch.float32)
    del ws32
    err = float(torch.max(torch.abs(z64 - z32.double())).item())
    say(f"  max |z_fp32 - z_fp64| = {err:.3e}")
    check_err(err, torch.float32, "max |z_fp32 - z_fp64|")
    del z32
    torch.cuda.empty_cache()
    # one more round from the final FP64 state, checked locally
    old = export(S, pr, ws, torch.float64)
    zo = z64.clone()
    phat = torch.from_numpy(d["probs"]).to(device="cuda", dtype=torch.float64)
    one = S.Problem(wl.K, wl.H, wl.W, wl.M, d["weights"], wl.schatten_p, wl.lam, wl.mu, 1, warm_start=True)
    S.segsalsa_str_solve(one, None, z64, ws)
    torch.cuda.synchronize()
    new = export(S, pr, ws, torch.float64)
    local_round_check(wl, d["weights"], phat, zo, old, z64, new, sample_pixels(wl.H, wl.W, 40, 7), 1e-9)
