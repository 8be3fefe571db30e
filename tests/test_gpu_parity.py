"""GPU parity: the HIP path against the FP64 oracle, element by element.

FP64 runs must match the oracle within 1e-9 max-abs; FP32 runs within 2e-4
(the oracle consumes the FP32-rounded input and multipliers); labels must be
identical wherever the oracle's top-two margin exceeds 1e-3.
"""
import math

import numpy as np
import pytest
import torch

from gpu_common import (check_err, FP32_TOL, FP64_TOL, MARGIN, gpu_solve, need_gpu, oracle_solve, problem_inputs,
                        rounded_input, say, weights_as_seen)
import synth

pytestmark = pytest.mark.gpu

# (H, W, K, M, p, iters): several tiles, ragged tails, odd/prime sides, degenerate sizes
SMALL_CASES = [
    (5, 7, 3, 1, 1.0, 6),
    (4, 4, 2, 0, 2.0, 6),
    (8, 5, 4, 2, math.inf, 6),
    (1, 6, 3, 1, 1.0, 5),
    (6, 1, 2, 1, 1.0, 5),
    (13, 11, 3, 2, 1.0, 8),
    (17, 67, 5, 1, 1.0, 8),
    (29, 131, 9, 2, 1.0, 6),
    (70, 33, 16, 1, math.inf, 5),
    (37, 41, 7, 3, 2.0, 4),
    (47, 53, 4, 1, 1.0, 5),      # both sides prime: direct 47- and 53-point stages
    (97, 509, 3, 1, 1.0, 4),     # a direct 97-point stage; Bluestein (M = 1024) for 509
    (122, 86, 5, 2, math.inf, 4),  # 2 x 61 and 2 x 43
    (211, 101, 2, 1, 1.0, 3),    # primes just above the direct-stage limit: Bluestein both ways
    # Bluestein on the fixed-structure engine: convolution lengths 256 .. 4096, an odd K (a lone class
    # in the last pair), ragged last row and column blocks
    (113, 227, 5, 1, 1.0, 4),    # M = 256 columns, 512 rows
    (1031, 6, 3, 1, 2.0, 3),     # M = 4096 columns (one column of 256 threads per workgroup)
    (7, 1031, 4, 2, 1.0, 3),     # M = 4096 rows
    (606, 37, 3, 0, math.inf, 3),  # 606 = 2 x 3 x 101: M = 2048 columns
    # power-of-two sides (the fixed-structure kernels, 64 .. 4096), alone or next to a general side
    (64, 128, 5, 1, 1.0, 5),
    (128, 64, 16, 2, math.inf, 4),
    (256, 512, 3, 1, 2.0, 3),
    (64, 96, 4, 1, 1.0, 4),
    (100, 256, 6, 0, 1.0, 4),
    (1024, 8, 2, 1, 1.0, 3),     # 1024-point columns (three stages: 16, 16, 4)
    (8, 4096, 3, 1, 1.0, 3),     # 4096-point rows (16, 16, 16)
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("H,W,K,M,p,iters", SMALL_CASES)
def test_small_grids(H, W, K, M, p, iters, dtype):
    S = need_gpu()
    say(f"case H={H} W={W} K={K} M={M} p={p} iters={iters} {dtype}")
    probs, _, _, c = problem_inputs(H, W, K, M, seed=H * 131 + W * 7 + K)
    z, *_ = gpu_solve(S, probs, c, M, p, 0.8, 1.3, iters, dtype)
    zo = oracle_solve(rounded_input(probs, dtype), weights_as_seen(c, dtype), M, p, 0.8, 1.3, iters)
    err = np.max(np.abs(z.double().cpu().numpy() - zo))
    say(f"  max|z_gpu - z_oracle| = {err:.3e}")
    check_err(err, dtype)


# the column pass by DFTs (the planner's default is the tridiagonal recursions): general mixed-radix
# and direct prime stages, Bluestein in LDS and on the fixed-structure engine, power-of-two lengths
DFT_COLUMN_CASES = [
    (47, 53, 4, 1, 1.0, 5, 0),
    (122, 86, 5, 2, math.inf, 4, 0),
    (97, 509, 3, 1, 1.0, 4, 0),
    (211, 101, 2, 1, 1.0, 3, 0),
    (211, 101, 2, 1, 1.0, 3, 1),     # the general kernels' Bluestein (in LDS)
    (606, 37, 3, 0, math.inf, 3, 0),
    (1031, 6, 3, 1, 2.0, 3, 0),
    (128, 64, 16, 2, math.inf, 4, 0),
    (1024, 8, 2, 1, 1.0, 3, 0),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("H,W,K,M,p,iters,generic", DFT_COLUMN_CASES)
def test_small_grids_dft_columns(H, W, K, M, p, iters, generic, dtype):
    S = need_gpu()
    prec = S._prec(dtype)
    S.segsalsa_tuning_set(K, H, W, M, prec, dict(col_dft=1, generic_fft=generic))
    try:
        plan, tuned = S.segsalsa_tuning_get(K, H, W, M, prec)
        assert tuned and plan["col_dft"] == 1
        say(f"case DFT columns H={H} W={W} K={K} M={M} p={p} iters={iters} {dtype}: {plan}")
        probs, _, _, c = problem_inputs(H, W, K, M, seed=H * 131 + W * 7 + K)
        z, *_ = gpu_solve(S, probs, c, M, p, 0.8, 1.3, iters, dtype)
    finally:
        S.segsalsa_tuning_set(K, H, W, M, prec, None)
    zo = oracle_solve(rounded_input(probs, dtype), weights_as_seen(c, dtype), M, p, 0.8, 1.3, iters)
    err = np.max(np.abs(z.double().cpu().numpy() - zo))
    say(f"  max|z_gpu - z_oracle| = {err:.3e}")
    check_err(err, dtype)


def engine_length(n):
    """The fixed-structure engine's length for a side: n for powers of two 64 .. 4096, the Bluestein
    length (the power of two >= 2n - 1) for sides with a prime factor above 100, else None."""
    if 64 <= n <= 4096 and n & (n - 1) == 0:
        return n
    m, f, big = n, 2, 1
    while f * f <= m:
        while m % f == 0:
            big, m = max(big, f), m // f
        f += 1
    big = max(big, m)
    if big <= 100:
        return None
    L = 1
    while L < 2 * n - 1:
        L *= 2
    return L if 64 <= L <= 4096 else None


# the fixed-structure engine, forced by tuned blocking: single images this small take the general
# kernels by default (the engine's 16 values per thread would leave the GPU mostly idle)
ENGINE_CASES = [
    (64, 128, 5, 1, 1.0, 5),
    (128, 64, 16, 2, math.inf, 4),
    (256, 512, 3, 1, 2.0, 3),
    (100, 256, 6, 0, 1.0, 4),
    (1024, 8, 2, 1, 1.0, 3),
    (8, 4096, 3, 1, 1.0, 3),
    (97, 509, 3, 1, 1.0, 4),
    (211, 101, 2, 1, 1.0, 3),
    (113, 227, 5, 1, 1.0, 4),
    (7, 1031, 4, 2, 1.0, 3),
    (606, 37, 3, 0, math.inf, 3),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("H,W,K,M,p,iters", ENGINE_CASES)
def test_small_grids_engine_forced(H, W, K, M, p, iters, dtype):
    S = need_gpu()
    prec = S._prec(dtype)
    lr, lc = engine_length(W), engine_length(H)
    tn = dict(col_dft=1)
    if lr:
        tn["rows_per_block"] = max(1, 64 // (lr // 16))
    if lc:
        tn["cols_per_block"] = max(1, 64 // (lc // 16))
    S.segsalsa_tuning_set(K, H, W, M, prec, tn)
    try:
        plan, tuned = S.segsalsa_tuning_get(K, H, W, M, prec)
        assert tuned and plan["generic_fft"] == 0
        say(f"case engine H={H} W={W} K={K} M={M} p={p} iters={iters} {dtype}: {plan}")
        probs, _, _, c = problem_inputs(H, W, K, M, seed=H * 131 + W * 7 + K)
        z, *_ = gpu_solve(S, probs, c, M, p, 0.8, 1.3, iters, dtype)
    finally:
        S.segsalsa_tuning_set(K, H, W, M, prec, None)
    zo = oracle_solve(rounded_input(probs, dtype), weights_as_seen(c, dtype), M, p, 0.8, 1.3, iters)
    err = np.max(np.abs(z.double().cpu().numpy() - zo))
    say(f"  max|z_gpu - z_oracle| = {err:.3e}")
    check_err(err, dtype)


# the column recursions across the range of Wsum = sum c_j^2: rho = 0 (no patch weights: the prior
# vanishes and the solve is z = rhs / 3), the largest rho FP32 solves take them at (Wsum = 256:
# 1 - rho = 0.103), rho near 1 (Wsum = 1e4: the periodic closure carries the column; FP64 only, FP32
# plans the DFT pass there), and a column length with a short last chunk (H = 70: 32 + 32 + 6)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("scale", [0.0, 10.0, 16.0, 100.0])
def test_column_recursions_across_weight_scales(scale, dtype):
    S = need_gpu()
    H, W, K, M, iters = 70, 45, 3, 1, 5
    probs, _, _, c = problem_inputs(H, W, K, M, seed=900 + int(scale))
    c = np.asarray(c) * scale
    say(f"case weights x{scale} (Wsum = {float(np.sum(c ** 2)):.3g}) {dtype}")
    z, *_ = gpu_solve(S, probs, c, M, 1.0, 0.6, 1.2, iters, dtype)
    zo = oracle_solve(rounded_input(probs, dtype), weights_as_seen(c, dtype), M, 1.0, 0.6, 1.2, iters)
    err = float(np.max(np.abs(z.double().cpu().numpy() - zo)))
    say(f"  max|z_gpu - z_oracle| = {err:.3e}")
    # (FP32 at Wsum = 1e4 plans the DFT column pass: 1 - rho = 0.017 there, and the recursions' FP32
    # rounding grows like eps / (1 - rho): 2.3e-5 against the DFT pass's 3.7e-6 on this case)
    check_err(err, dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_plain_64x64(dtype):
    """The 64x64, K = 4, 3x3 patch, Schatten-1, 100-round workload."""
    S = need_gpu()
    wl = synth.WORKLOADS["plain_64x64_k4"]
    d = synth.make_workload(wl)
    say(f"case {wl.name} {dtype}")
    z, *_ = gpu_solve(S, d["probs"], d["weights"], wl.M, wl.schatten_p, wl.lam, wl.mu, wl.iters, dtype)
    zo = oracle_solve(rounded_input(d["probs"], dtype), weights_as_seen(d["weights"], dtype), wl.M,
                      wl.schatten_p, wl.lam, wl.mu, wl.iters)
    zg = z.double().cpu().numpy()
    err = np.max(np.abs(zg - zo))
    say(f"  max err {err:.3e}")
    check_err(err, dtype)
    srt = np.sort(zo, axis=0)
    sure = (srt[-1] - srt[-2]) > MARGIN
    assert np.array_equal(np.argmax(zg, axis=0)[sure], np.argmax(zo, axis=0)[sure])


@pytest.mark.parametrize("p", [1.0, 2.0, math.inf])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_pines_145_short(p, dtype):
    """145x145, K = 16, 5x5 patch, lambda = mu = 2: the first 12 rounds, every Schatten p."""
    S = need_gpu()
    wl = synth.WORKLOADS["pines_145x145_k16"]
    d = synth.make_workload(wl)
    iters = 12
    say(f"case {wl.name} p={p} iters={iters} {dtype}")
    z, *_ = gpu_solve(S, d["probs"], d["weights"], wl.M, p, wl.lam, wl.mu, iters, dtype)
    zo = oracle_solve(rounded_input(d["probs"], dtype), weights_as_seen(d["weights"], dtype), wl.M, p,
                      wl.lam, wl.mu, iters)
    err = np.max(np.abs(z.double().cpu().numpy() - zo))
    say(f"  max err {err:.3e}")
    check_err(err, dtype)


def test_logits_and_asymmetric_weights():
    S = need_gpu()
    probs, logits, _, _ = problem_inputs(23, 19, 5, 1, seed=77)
    c = np.array([0.1, 0.9, 0.3, 0.5, 1.0, 0.2, 0.8, 0.4, 0.6])
    z, *_ = gpu_solve(S, logits, c, 1, 1.0, 0.7, 1.1, 9, torch.float64, logits=True)
    zo = oracle_solve(logits, c, 1, 1.0, 0.7, 1.1, 9, logits=True)
    assert np.max(np.abs(z.cpu().numpy() - zo)) <= FP64_TOL


def test_zero_rounds_returns_normalised_input():
    S = need_gpu()
    probs, _, _, c = problem_inputs(9, 10, 3, 1, seed=5)
    scaled = probs * 3.7
    z, *_ = gpu_solve(S, scaled, c, 1, 1.0, 1.0, 1.0, 0, torch.float64)
    assert np.max(np.abs(z.cpu().numpy() - probs)) <= 1e-14


def test_lambda_zero_identity_prox():
    S = need_gpu()
    probs, _, _, c = problem_inputs(12, 14, 4, 1, seed=6)
    z, *_ = gpu_solve(S, probs, c, 1, 1.0, 0.0, 0.5, 7, torch.float64)
    zo = oracle_solve(probs, c, 1, 1.0, 0.0, 0.5, 7)
    assert np.max(np.abs(z.cpu().numpy() - zo)) <= FP64_TOL


# edges of the interface: the most classes (K = 64), an odd K above 32 (17 class pairs), the longest
# sides (4096 = 8^4 transforms) in both orientations; FP32 also at the largest K its register budget
# allows with a 3x3 (K = 64) and a 5x5 patch (K = 32)
EDGE_CASES = [
    (5, 6, 64, 0, 1.0, 4, None),
    (9, 11, 33, 0, 1.0, 3, None),
    (4096, 3, 2, 0, 2.0, 3, None),
    (3, 4096, 3, 1, math.inf, 3, None),
    (5, 6, 64, 1, 1.0, 4, torch.float32),
    (7, 9, 32, 2, 1.0, 3, torch.float32),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("H,W,K,M,p,iters,only", EDGE_CASES)
def test_interface_edges(H, W, K, M, p, iters, only, dtype):
    if only is not None and dtype != only:
        pytest.skip("beyond the FP64 register budget of one workgroup (UNSUPPORTED by design)")
    S = need_gpu()
    say(f"case edge H={H} W={W} K={K} M={M} p={p} iters={iters} {dtype}")
    probs, _, _, c = problem_inputs(H, W, K, M, seed=H * 17 + W * 3 + K)
    z, *_ = gpu_solve(S, probs, c, M, p, 0.8, 1.3, iters, dtype)
    zo = oracle_solve(rounded_input(probs, dtype), weights_as_seen(c, dtype), M, p, 0.8, 1.3, iters)
    err = np.max(np.abs(z.double().cpu().numpy() - zo))
    say(f"  max|z_gpu - z_oracle| = {err:.3e}")
    check_err(err, dtype)


# the vector fold (16-byte loads of adjacent columns of one tile column), taken when every tile column
# has the same width, a multiple of 4 (FP32) or 2 (FP64), and at least 2M + 2: one, two and many tile
# columns (the neighbours are then the tile itself or one other tile), M = 0 .. 3, an odd K, tiles
# shorter than the halo (rows covered by more than two tiles), a Bluestein row length (404 = 4 x 101);
# in the general row kernel and, by tuned blocking, on the fixed-structure engine.
# (H, W, K, M, tile_rows, tile_cols, iters)
VFOLD_CASES = [
    (64, 128, 5, 1, 8, 16, 4),
    (70, 64, 3, 2, 16, 64, 4),
    (33, 256, 4, 3, 6, 128, 3),
    (40, 64, 2, 0, 8, 8, 4),
    (30, 128, 3, 3, 3, 16, 3),
    (20, 404, 3, 1, 10, 4, 3),
]


def vfold_applies(W, M, tile_cols, vec):
    ntc = -(-W // min(tile_cols, W))
    tc = -(-W // ntc)
    return W % ntc == 0 and tc % vec == 0 and tc >= 2 * M + 2


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("engine", [True, False], ids=["engine", "general"])
@pytest.mark.parametrize("H,W,K,M,tr,tc,iters", VFOLD_CASES)
def test_vector_fold(H, W, K, M, tr, tc, iters, engine, dtype):
    S = need_gpu()
    prec = S._prec(dtype)
    assert vfold_applies(W, M, tc, 4 if dtype == torch.float32 else 2)
    tn = dict(tile_rows=tr, tile_cols=tc)
    if engine:
        tn["rows_per_block"] = max(1, 64 // (engine_length(W) // 16))
    else:
        tn["generic_fft"] = 1
    S.segsalsa_tuning_set(K, H, W, M, prec, tn)
    try:
        plan, tuned = S.segsalsa_tuning_get(K, H, W, M, prec)
        assert tuned and plan["generic_fft"] == (0 if engine else 1)
        say(f"case vector fold H={H} W={W} K={K} M={M} tiles {tr}x{tc} iters={iters} {dtype}: {plan}")
        probs, _, _, c = problem_inputs(H, W, K, M, seed=H * 17 + W + M)
        z, *_ = gpu_solve(S, probs, c, M, 1.0, 0.8, 1.3, iters, dtype)
    finally:
        S.segsalsa_tuning_set(K, H, W, M, prec, None)
    zo = oracle_solve(rounded_input(probs, dtype), weights_as_seen(c, dtype), M, 1.0, 0.8, 1.3, iters)
    err = np.max(np.abs(z.double().cpu().numpy() - zo))
    say(f"  max|z_gpu - z_oracle| = {err:.3e}")
    check_err(err, dtype)
