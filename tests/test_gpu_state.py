"""GPU checks of the solver state: export/import, warm start, determinism,
labels and the device-side input check."""
import math

import numpy as np
import pytest
import torch

from gpu_common import FP32_TOL, FP64_TOL, gpu_solve, need_gpu, problem_inputs, say
import synth
from oracle import segsalsa_ref as R

pytestmark = pytest.mark.gpu


def export_state(S, pr, ws, dtype):
    K, H, W = pr.K, pr.H, pr.W
    L = (2 * pr.patch_radius + 1) ** 2
    d1 = torch.empty(K, H, W, dtype=dtype, device="cuda")
    d3 = torch.empty_like(d1)
    d4 = torch.empty_like(d1)
    d2 = torch.empty(L, 2, K, H, W, dtype=dtype, device="cuda")
    S.segsalsa_str_state_export(pr, ws, d1, d2, d3, d4)
    torch.cuda.synchronize()
    return [t.double().cpu().numpy() for t in (d1, d2, d3, d4)]


@pytest.mark.parametrize("H,W,K,M,p", [(19, 23, 4, 1, 1.0), (31, 17, 6, 2, math.inf), (12, 40, 3, 0, 2.0)])
def test_state_export_matches_oracle(H, W, K, M, p):
    S = need_gpu()
    say(f"case export H={H} W={W} K={K} M={M} p={p}")
    probs, _, _, c = problem_inputs(H, W, K, M, seed=H + W + K)
    z, ws, pr, _ = gpu_solve(S, probs, c, M, p, 0.9, 1.4, 7, torch.float64)
    d1, d2, d3, d4 = export_state(S, pr, ws, torch.float64)
    st, _ = R.solve(probs, R.Problem(c, M, p, 0.9, 1.4), 7, return_state=True)
    for name, a, b in (("z", z.cpu().numpy(), st.z), ("d1", d1, st.d1), ("d2", d2, st.d2), ("d3", d3, st.d3),
                       ("d4", d4, st.d4)):
        err = np.max(np.abs(a - b))
        say(f"  {name}: {err:.2e}")
        assert err <= FP64_TOL, name


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("p", [1.0, 2.0, math.inf])
def test_import_random_state_one_round(dtype, p):
    """One round from an arbitrary imported state (all multipliers non-zero) against the oracle's round."""
    S = need_gpu()
    H, W, K, M = 21, 26, 5, 2
    L = (2 * M + 1) ** 2
    probs, _, _, c = problem_inputs(H, W, K, M, seed=3)
    z0, d1, d3, d4, d2 = synth.random_state(K, H, W, L, seed=9, scale=0.2)
    if dtype == torch.float32:   # the oracle consumes exactly what the GPU holds
        probs, z0, d1, d2, d3, d4, c = (np.asarray(t, dtype=np.float32).astype(np.float64)
                                        for t in (probs, z0, d1, d2, d3, d4, c))
    pr = S.Problem(K, H, W, M, c, p, 1.1, 0.8, 1, warm_start=True)
    ws = torch.empty(S.segsalsa_str_workspace_size(pr, S._prec(dtype)), dtype=torch.uint8, device="cuda")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)
    S.segsalsa_str_state_import(pr, ws, dev(probs), dev(d1), dev(d2), dev(d3), dev(d4))
    z = dev(z0)
    S.segsalsa_str_solve(pr, None, z, ws)
    torch.cuda.synchronize()
    g1, g2, g3, g4 = export_state(S, pr, ws, dtype)
    ref = R.salsa_round(R.State(z0, d1, d2, d3, d4), probs, R.Problem(c, M, p, 1.1, 0.8))
    tol = FP64_TOL if dtype == torch.float64 else 5e-5
    for name, a, b in (("z", z.double().cpu().numpy(), ref.z), ("d1", g1, ref.d1), ("d2", g2, ref.d2),
                       ("d3", g3, ref.d3), ("d4", g4, ref.d4)):
        err = np.max(np.abs(a - b))
        say(f"  {name}: {err:.2e}")
        assert err <= tol, name


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_warm_start_resume_is_bitwise(dtype):
    S = need_gpu()
    H, W, K, M = 40, 52, 6, 2
    probs, _, _, c = problem_inputs(H, W, K, M, seed=4)
    x = torch.from_numpy(probs).to(device="cuda", dtype=dtype)
    full = S.Problem(K, H, W, M, c, 1.0, 1.0, 1.0, 12)
    ws = torch.empty(S.segsalsa_str_workspace_size(full, S._prec(dtype)), dtype=torch.uint8, device="cuda")
    z_full = torch.empty_like(x)
    S.segsalsa_str_solve(full, x, z_full, ws)
    first = S.Problem(K, H, W, M, c, 1.0, 1.0, 1.0, 5)
    rest = S.Problem(K, H, W, M, c, 1.0, 1.0, 1.0, 7, warm_start=True)
    ws2 = torch.empty_like(ws)
    z = torch.empty_like(x)
    S.segsalsa_str_solve(first, x, z, ws2)
    S.segsalsa_str_solve(rest, None, z, ws2)
    torch.cuda.synchronize()
    assert torch.equal(z, z_full)


def test_repeated_solves_are_bitwise_identical():
    S = need_gpu()
    probs, _, _, c = problem_inputs(97, 83, 9, 2, seed=5)
    z1, *_ = gpu_solve(S, probs, c, 2, 1.0, 1.5, 1.5, 20, torch.float32)
    z2, *_ = gpu_solve(S, probs, c, 2, 1.0, 1.5, 1.5, 20, torch.float32)
    assert torch.equal(z1, z2)


def test_labels_kernel():
    S = need_gpu()
    rng = np.random.default_rng(0)
    z = rng.standard_normal((7, 33, 29))
    z[3, 0, 0] = z[5, 0, 0] = 10.0     # a tie: the lower class wins
    for dtype in (torch.float32, torch.float64):
        zt = torch.from_numpy(z).to(device="cuda", dtype=dtype)
        lab = torch.empty(33, 29, dtype=torch.int32, device="cuda")
        S.segsalsa_str_labels(zt, lab)
        torch.cuda.synchronize()
        ref = np.argmax(zt.cpu().numpy(), axis=0)
        assert np.array_equal(lab.cpu().numpy(), ref)
        assert lab[0, 0].item() == 3


@pytest.mark.parametrize("bad,flag", [("negative", 2), ("zero", 4), ("nan", 1)])
def test_device_input_check_sets_flags(bad, flag):
    S = need_gpu()
    probs, _, _, c = problem_inputs(8, 9, 3, 1, seed=6)
    if bad == "negative":
        probs[1, 2, 3] = -0.5
    elif bad == "zero":
        probs[:, 4, 4] = 0.0
    else:
        probs[0, 1, 1] = np.nan
    _, _, _, st = gpu_solve(S, probs, c, 1, 1.0, 1.0, 1.0, 0, torch.float64, stats=True)
    assert st["flags"] & flag


def test_clean_input_has_no_flags():
    S = need_gpu()
    probs, _, _, c = problem_inputs(8, 9, 3, 1, seed=6)
    _, _, _, st = gpu_solve(S, probs, c, 1, 1.0, 1.0, 1.0, 3, torch.float64, stats=True)
    assert st["flags"] == 0 and st["rounds_done"] == 3


def test_stream_copy_moves_every_byte():
    """The streaming copy (the bench's reference for the prox kernel's streaming build) copies exactly:
    a size whose 16-byte words do not fill the four-deep unrolled loop, and one that does."""
    S = need_gpu()
    for n in (4 * 1000 + 4, 1 << 20):
        src = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device="cuda")
        dst = torch.zeros_like(src)
        say(f"case stream copy {n * 4} bytes")
        S.segsalsa_stream_copy(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
