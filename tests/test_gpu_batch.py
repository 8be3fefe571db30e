"""Batched solves (many images of uneven sizes and class counts) and whole-solve hipGraphs."""
import math

import numpy as np
import pytest
import torch

from gpu_common import check_err, FP32_TOL, FP64_TOL, need_gpu, oracle_many, oracle_solve, rounded_input, say
import synth

pytestmark = pytest.mark.gpu

# uneven shapes: prime sides, K not a power of two, one tiny and one tall image
SHAPES = [(37, 53, 4), (61, 29, 9), (16, 16, 8), (97, 31, 16), (5, 7, 3), (128, 40, 5)]


def make_inputs(shapes, seed0=100):
    return [synth.make_image(H, W, K, seed0 + i, 1.0, 1.5)[0] for i, (H, W, K) in enumerate(shapes)]


def run_batch(S, shapes, probs, c, M, p, lams, mus, iters, dtype, graph=False, every=0, tol=0.0, ws=None):
    imgs, total = S.image_table([(K, H, W) for (H, W, K) in shapes], lams, mus)
    params = S.BatchParams(M, c, p, iters, residual_every=every, tol=tol, use_graph=graph)
    packed = torch.cat([torch.from_numpy(x).reshape(-1) for x in probs]).to(device="cuda", dtype=dtype)
    z = torch.empty_like(packed)
    need = S.segsalsa_str_batch_workspace_size(imgs, params, S._prec(dtype))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    st = S.segsalsa_str_solve_batch(imgs, params, packed, z, ws, stats=every > 0)
    torch.cuda.synchronize()
    out, off = [], 0
    for (H, W, K) in shapes:
        out.append(z[off:off + K * H * W].reshape(K, H, W))
        off += K * H * W
    return out, st, ws


def run_single(S, x, c, M, p, lam, mu, iters, dtype, graph=False, every=0, tol=0.0):
    K, H, W = x.shape
    xt = torch.from_numpy(x).to(device="cuda", dtype=dtype)
    pr = S.Problem(K, H, W, M, c, p, lam, mu, iters, residual_every=every, tol=tol, use_graph=graph)
    ws = torch.empty(S.segsalsa_str_workspace_size(pr, S._prec(dtype)), dtype=torch.uint8, device="cuda")
    z = torch.empty_like(xt)
    st = S.segsalsa_str_solve(pr, xt, z, ws, stats=every > 0)
    torch.cuda.synchronize()
    return z, st


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_batch_equals_single_solves_and_oracle(dtype):
    S = need_gpu()
    M, p, iters = 1, 1.0, 9
    c = synth.gaussian_patch_multipliers(M, 1.0)
    probs = make_inputs(SHAPES)
    lams = [0.5 + 0.2 * i for i in range(len(SHAPES))]
    mus = [1.0 + 0.1 * i for i in range(len(SHAPES))]
    zb, _, _ = run_batch(S, SHAPES, probs, c, M, p, lams, mus, iters, dtype)
    for i, x in enumerate(probs):
        zs, _ = run_single(S, x, c, M, p, lams[i], mus[i], iters, dtype)
        assert torch.equal(zb[i], zs), f"image {i} differs from its single solve"
        if dtype == torch.float64:
            zo = oracle_solve(x, c, M, p, lams[i], mus[i], iters)
            err = float(np.max(np.abs(zb[i].cpu().numpy() - zo)))
            say(f"  image {i} {x.shape}: max err vs oracle {err:.2e}")
            assert err <= FP64_TOL


def test_batch_graph_replays_match_direct():
    S = need_gpu()
    M, iters = 2, 6
    c = synth.gaussian_patch_multipliers(M, 1.5)
    shapes = SHAPES[:4]
    probs = make_inputs(shapes, 200)
    lams, mus = [1.0] * 4, [1.3] * 4
    direct, _, _ = run_batch(S, shapes, probs, c, M, math.inf, lams, mus, iters, torch.float32)
    ref = [t.clone() for t in direct]
    ws = None
    for rep in range(3):
        zg, _, ws = run_batch(S, shapes, probs, c, M, math.inf, lams, mus, iters, torch.float32, graph=True, ws=ws)
        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        for a, b in zip(zg, ref):
            assert torch.equal(a, b), f"replay {rep} differs"


def test_single_solve_graph_replays_match_direct():
    S = need_gpu()
    wl = synth.WORKLOADS["pines_145x145_k16"]
    d = synth.make_workload(wl)
    z_direct, _ = run_single(S, d["probs"], d["weights"], wl.M, 1.0, wl.lam, wl.mu, 20, torch.float32)
    x = torch.from_numpy(d["probs"]).to(device="cuda", dtype=torch.float32)
    pr = S.Problem(wl.K, wl.H, wl.W, wl.M, d["weights"], 1.0, wl.lam, wl.mu, 20, use_graph=True)
    ws = torch.empty(S.segsalsa_str_workspace_size(pr, S.SEGSALSA_FP32), dtype=torch.uint8, device="cuda")
    z = torch.empty_like(x)
    for rep in range(3):
        z.fill_(0.0)
        S.segsalsa_str_solve(pr, x, z, ws)
        torch.cuda.synchronize()
        assert torch.equal(z, z_direct), f"replay {rep}"
        _ = (torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")).sum().item()


def test_batch_early_exit_matches_single_solves():
    S = need_gpu()
    M, every, tol, iters = 1, 5, 1e-2, 400
    c = synth.gaussian_patch_multipliers(M, 1.0)
    shapes = [(16, 18, 3), (21, 13, 4), (9, 30, 5)]
    probs = make_inputs(shapes, 300)
    lams, mus = [0.5, 0.4, 0.6], [2.0, 1.5, 2.5]
    zb, stb, _ = run_batch(S, shapes, probs, c, M, 1.0, lams, mus, iters, torch.float64, every=every, tol=tol)
    rounds = []
    for i, x in enumerate(probs):
        zs, sts = run_single(S, x, c, M, 1.0, lams[i], mus[i], iters, torch.float64, every=every, tol=tol)
        say(f"  image {i}: batch stopped after {stb[i]['rounds_done']}, single after {sts['rounds_done']}")
        assert stb[i]["rounds_done"] == sts["rounds_done"]
        assert torch.equal(zb[i], zs)
        rounds.append(sts["rounds_done"])
    assert len(set(rounds)) > 1, "the images should stop at different rounds"


def test_batch_workload_fp32_vs_fp64():
    """The 64-image batch (sides 96..512, K in {4, 8, 9, 16}, 3x3 patch, 200 rounds)."""
    S = need_gpu()
    B = synth.BATCH
    shapes = synth.batch_shapes()
    probs = [t[0] for t in synth.make_batch(shapes)]
    c = synth.gaussian_patch_multipliers(B["M"], B["patch_sigma"])
    lams, mus = [B["lam"]] * len(shapes), [B["mu"]] * len(shapes)
    say(f"case batch of {len(shapes)} images, {B['iters']} rounds")
    z64, _, _ = run_batch(S, shapes, probs, c, B["M"], 1.0, lams, mus, B["iters"], torch.float64)
    z32, _, _ = run_batch(S, shapes, probs, c, B["M"], 1.0, lams, mus, B["iters"], torch.float32, graph=True)
    err = max(float(torch.max(torch.abs(a - b.double())).item()) for a, b in zip(z64, z32))
    say(f"  max |z_fp32 - z_fp64| over the batch = {err:.2e}")
    check_err(err, torch.float32, "max |z_fp32 - z_fp64|")
    # two images of the batch against their own single solves (the same kernels: bit for bit)
    for i in (0, len(shapes) - 1):
        zs, _ = run_single(S, probs[i], c, B["M"], 1.0, lams[i], mus[i], B["iters"], torch.float64)
        assert torch.equal(z64[i], zs)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_batch_workload_every_image_against_oracle(dtype):
    """Every image of the 64-image batch against the FP64 oracle after 2 rounds, element by element
    (the oracle runs in parallel CPU processes)."""
    S = need_gpu()
    B = synth.BATCH
    shapes = synth.batch_shapes()
    probs = [t[0] for t in synth.make_batch(shapes)]
    c = synth.gaussian_patch_multipliers(B["M"], B["patch_sigma"])
    lams, mus = [B["lam"]] * len(shapes), [B["mu"]] * len(shapes)
    iters = 2
    say(f"case batch of {len(shapes)} images {dtype}: {iters} rounds, every image against the oracle")
    zb, _, _ = run_batch(S, shapes, probs, c, B["M"], 1.0, lams, mus, iters, dtype)
    cw = np.asarray(c, dtype=np.float32).astype(np.float64) if dtype == torch.float32 else np.asarray(c)
    jobs = [(rounded_input(x, dtype), cw, B["M"], 1.0, lams[i], mus[i], iters, False) for i, x in enumerate(probs)]
    say("  oracle running in parallel processes")
    zo = oracle_many(jobs)
    errs = [float(np.max(np.abs(a.double().cpu().numpy() - b))) for a, b in zip(zb, zo)]
    worst = int(np.argmax(errs))
    say(f"  worst image {worst} {shapes[worst]}: max |z_gpu - z_oracle| = {errs[worst]:.3e}")
    check_err(max(errs), dtype)
