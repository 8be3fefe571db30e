"""segsalsa_str_solve_noalloc (no workspace argument, the library's per-GPU scratch array)
against segsalsa_str_solve on the same inputs, through the C ABI: two calls in a row, the second
on a smaller problem, in both precisions; and its argument checks."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_common import need_gpu, problem_inputs, say

pytestmark = pytest.mark.gpu


def with_workspace(S, pr, x):
    ws = torch.empty(S.segsalsa_str_workspace_size(pr, S._prec(x.dtype)), dtype=torch.uint8, device="cuda")
    z = torch.empty_like(x)
    S.segsalsa_str_solve(pr, x, z, ws)
    torch.cuda.synchronize()
    return z


def no_alloc(S, pr, x):
    z = torch.full_like(x, float("nan"))
    s = pr.c_struct()
    st = S.lib().segsalsa_str_solve_noalloc(ctypes.byref(s), S._prec(x.dtype), ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(z.data_ptr()),
                                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, S.lib().segsalsa_last_error().decode()
    torch.cuda.synchronize()
    return z


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_noalloc_matches_solve_on_two_calls(dtype):
    S = need_gpu()
    # first a larger problem, then a smaller one: the second call must not see the first's state
    cases = [(96, 111, 9, 2, 12, 301), (23, 40, 5, 1, 9, 302)]
    for (H, W, K, M, iters, seed) in cases:
        probs, _, _, c = problem_inputs(H, W, K, M, seed)
        x = torch.from_numpy(probs).to(device="cuda", dtype=dtype)
        pr = S.Problem(K, H, W, M, c, 1.0, 0.9, 1.3, iters)
        need = S.segsalsa_str_workspace_size(pr, S._prec(dtype))
        assert need <= S.NOALLOC_SCRATCH_BYTES
        say(f"case noalloc {H}x{W} K={K} M={M} {iters} rounds {dtype} (workspace {need} bytes)")
        za = no_alloc(S, pr, x)
        zb = with_workspace(S, pr, x)
        err = float(torch.max(torch.abs(za - zb)).item())
        say(f"  max |z_noalloc - z_solve| = {err:.3e}")
        assert torch.equal(za, zb)


def test_noalloc_argument_errors():
    S = need_gpu()
    x = torch.rand(4, 16, 16, device="cuda", dtype=torch.float32) + 0.1
    z = torch.empty_like(x)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call(pr):
        s = pr.c_struct()
        return S.lib().segsalsa_str_solve_noalloc(ctypes.byref(s), 0, ctypes.c_void_p(x.data_ptr()),
                                                  ctypes.c_void_p(z.data_ptr()), stream)
    c = [1.0] * 9
    assert call(S.Problem(4, 16, 16, 1, c, 1.0, 1.0, 1.0, 3, use_graph=True)) == 1
    assert call(S.Problem(4, 16, 16, 1, c, 1.0, 1.0, 1.0, 3, residual_every=1)) == 1
    # a problem whose workspace exceeds the scratch array is refused before anything runs
    big = S.Problem(16, 1024, 1024, 2, [1.0] * 25, 1.0, 1.0, 1.0, 3)
    assert S.segsalsa_str_workspace_size(big, 0) > S.NOALLOC_SCRATCH_BYTES
    assert call(big) == 2
    assert b"no-allocation scratch" in S.lib().segsalsa_last_error()
