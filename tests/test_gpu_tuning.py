"""Tuned launch shapes on the GPU: any shape the tuning table accepts gives the same z as the
oracle (to the same tolerances), and the autotuner's choice does too.

The table changes only the tile grid, the classes per wavefront and the FFT blocking; the
arithmetic of each round is fixed by eqs. (12)-(14)."""
import numpy as np
import pytest
import torch

from gpu_common import check_err, gpu_solve, need_gpu, oracle_solve, problem_inputs, rounded_input, say, weights_as_seen

pytestmark = pytest.mark.gpu


@pytest.fixture()
def table():
    S = need_gpu()
    S.segsalsa_tuning_clear()
    yield S
    S.segsalsa_tuning_clear()
    import os
    if os.path.exists(S.DEFAULT_TUNING_CACHE):
        S.segsalsa_tuning_load(S.DEFAULT_TUNING_CACHE)


CASES = [
    # (H, W, K, M, tuning)
    (8, 300, 2, 0, dict(tile_rows=2, tile_cols=300)),                        # grown tile 301 columns wide
    (300, 9, 3, 1, dict(tile_rows=300, tile_cols=3, classes_per_wave=1)),    # and 303 rows tall
    (37, 61, 6, 1, dict(tile_rows=5, tile_cols=12, classes_per_wave=2, rows_per_block=3, row_threads=64,
                        cols_per_block=16, col_threads=128)),
    (53, 47, 9, 2, dict(tile_rows=4, tile_cols=8, classes_per_wave=4, rows_per_block=1, row_threads=1024,
                        cols_per_block=1, col_threads=64)),
    # Bluestein columns by DFTs in the general kernels (in LDS) and on the fixed-structure engine (M = 256:
    # 16 threads per column)
    (101, 40, 5, 1, dict(generic_fft=1, col_dft=1, rows_per_block=2, row_threads=192, cols_per_block=8,
                         col_threads=512)),
    (101, 40, 5, 1, dict(col_dft=1, rows_per_block=2, row_threads=192, cols_per_block=12, col_threads=192)),
    # the tridiagonal column pass with more threads than chunks, and with one column per workgroup
    (150, 33, 4, 1, dict(cols_per_block=3, col_threads=320)),
    (70, 9, 3, 2, dict(cols_per_block=1, col_threads=64)),
    (43, 131, 3, 1, dict(rows_per_block=6, row_threads=192, cols_per_block=5, col_threads=320)),   # M = 512 rows
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_tuned_shapes_match_oracle(table, case, dtype):
    S = table
    H, W, K, M, tn = CASES[case]
    prec = S._prec(dtype)
    S.segsalsa_tuning_set(K, H, W, M, prec, tn)
    plan, tuned = S.segsalsa_tuning_get(K, H, W, M, prec)
    assert tuned
    say(f"case {H}x{W} K={K} M={M} {dtype}: tuned plan {plan}")
    probs, _, _, c = problem_inputs(H, W, K, M, seed=300 + case)
    iters = 7
    z, _, _, _ = gpu_solve(S, probs, c, M, 1.0, 0.8, 1.1, iters, dtype)
    zo = oracle_solve(rounded_input(probs, dtype), weights_as_seen(c, dtype), M, 1.0, 0.8, 1.1, iters)
    err = float(np.max(np.abs(z.double().cpu().numpy() - zo)))
    say(f"  max |z_gpu - z_oracle| = {err:.3e}")
    check_err(err, dtype)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["fp32", "fp64"])
def test_autotune_then_solve_matches_oracle(table, dtype):
    S = table
    H, W, K, M = 45, 70, 5, 1
    probs, _, _, c = problem_inputs(H, W, K, M, seed=321)
    x = torch.from_numpy(probs).to(device="cuda", dtype=dtype)
    pr = S.Problem(K, H, W, M, c, 1.0, 0.9, 1.2, 10)
    ws = torch.empty(S.segsalsa_str_autotune_workspace_size(pr, S._prec(dtype)), dtype=torch.uint8, device="cuda")
    zs = torch.empty_like(x)
    say(f"case autotune {H}x{W} K={K} M={M} {dtype}")
    best = S.segsalsa_str_autotune(pr, x, zs, ws, rounds=3)
    torch.cuda.synchronize()
    say(f"  tuned: {best}")
    assert best["us_per_round"] > 0
    plan, tuned = S.segsalsa_tuning_get(K, H, W, M, S._prec(dtype))
    assert tuned and {k: plan[k] for k in plan if k != "us_per_round"} == \
        {k: best[k] for k in best if k != "us_per_round"}
    z, _, _, _ = gpu_solve(S, probs, c, M, 1.0, 0.9, 1.2, 10, dtype)
    zo = oracle_solve(rounded_input(probs, dtype), weights_as_seen(c, dtype), M, 1.0, 0.9, 1.2, 10)
    err = float(np.max(np.abs(z.double().cpu().numpy() - zo)))
    say(f"  max |z_gpu - z_oracle| = {err:.3e}")
    check_err(err, dtype)


PF_CASES = [(64, 96, 16, 2), (45, 70, 9, 2), (37, 61, 6, 1), (29, 40, 5, 0)]


@pytest.mark.parametrize("case", range(len(PF_CASES)))
def test_prefetching_prox_build_matches_oracle(table, case):
    """FP32 prox kernel that loads step s + 1 during step s (two classes per wavefront, odd K pads)."""
    S = table
    H, W, K, M = PF_CASES[case]
    S.segsalsa_tuning_set(K, H, W, M, S.SEGSALSA_FP32, dict(classes_per_wave=2, prefetch=1, tile_rows=8,
                                                             tile_cols=16))
    plan, tuned = S.segsalsa_tuning_get(K, H, W, M, S.SEGSALSA_FP32)
    assert tuned and plan["prefetch"] == 1
    probs, _, _, c = problem_inputs(H, W, K, M, seed=400 + case)
    iters = 9
    say(f"case prefetch {H}x{W} K={K} M={M}: {plan}")
    z, _, _, _ = gpu_solve(S, probs, c, M, 1.0, 0.8, 1.1, iters, torch.float32)
    zo = oracle_solve(rounded_input(probs, torch.float32), weights_as_seen(c, torch.float32), M, 1.0, 0.8, 1.1, iters)
    err = float(np.max(np.abs(z.double().cpu().numpy() - zo)))
    say(f"  max |z_gpu - z_oracle| = {err:.3e}")
    check_err(err, torch.float32)
    # the same plan without the prefetch gives the same z bit for bit (same arithmetic, same order)
    S.segsalsa_tuning_set(K, H, W, M, S.SEGSALSA_FP32, dict(classes_per_wave=2, prefetch=0, tile_rows=8,
                                                             tile_cols=16))
    z2, _, _, _ = gpu_solve(S, probs, c, M, 1.0, 0.8, 1.1, iters, torch.float32)
    assert torch.equal(z, z2)


def test_batch_of_several_images_ignores_table(table):
    """Batches of more than one image keep the planner's shapes: an entry for one of their shapes
    leaves the batch's z bit for bit as it was, while a solve of that image alone takes it."""
    S = table
    from test_gpu_batch import make_inputs, run_batch, run_single
    import synth
    shapes = [(37, 53, 4), (61, 29, 9)]
    M, p, iters = 1, 1.0, 6
    c = synth.gaussian_patch_multipliers(M, 1.0)
    probs = make_inputs(shapes, 400)
    lams, mus = [0.7, 0.9], [1.1, 1.2]
    ref, _, _ = run_batch(S, shapes, probs, c, M, p, lams, mus, iters, torch.float32)
    ref = [t.clone() for t in ref]
    H, W, K = shapes[0]
    S.segsalsa_tuning_set(K, H, W, M, S.SEGSALSA_FP32, dict(tile_rows=3, tile_cols=7, classes_per_wave=1,
                                                          rows_per_block=1, row_threads=64))
    got, _, _ = run_batch(S, shapes, probs, c, M, p, lams, mus, iters, torch.float32)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    zs, _ = run_single(S, probs[0], c, M, p, lams[0], mus[0], iters, torch.float32)
    zo = oracle_solve(rounded_input(probs[0], torch.float32), weights_as_seen(c, torch.float32), M, p, lams[0], mus[0],
                      iters)
    err = float(np.max(np.abs(zs.double().cpu().numpy() - zo)))
    say(f"  tuned single solve: max |z - z_oracle| = {err:.3e}")
    check_err(err, torch.float32)
