"""Reverse sweep (segsalsa_str_solve_ckpt + segsalsa_str_backward) on the GPU.

* Small images spanning several tiles: FP64 gradients (input, lambda, patch
  multipliers) equal the FP64 reference gradient (PyTorch CPU autograd of the
  oracle-equivalent rounds, itself pinned to finite differences of the numpy
  oracle) within 1e-9 relative to the largest entry, for p in {1, 2, inf},
  M in {0, 1, 2}, probabilities and logits, lambda = 0, and K up to 16 (one,
  two and four classes per wavefront in the reverse-sweep kernel); the FP32
  gradients within 1e-3 of the reference on the same inputs.
* The checkpoint interval changes nothing (bitwise); the checkpointed forward
  returns the same z as segsalsa_str_solve (bitwise); zero rounds.
* The 256x256, K = 8, 3x3 patch, 50-round workload: central finite
  differences of the GPU FP64 forward along random directions agree with the
  FP64 adjoint to 1e-5 relative; sum_k dL/dlogit_k = 0 per pixel; the FP32
  adjoint is reported against the FP64 one.
"""
import math

import numpy as np
import pytest
import torch

from gpu_common import need_gpu, say
import synth
from oracle import segsalsa_torch_ref as TR

pytestmark = pytest.mark.gpu


def gpu_grad(S, x, w, c, M, p, lam, mu, iters, logits, ck=10, dtype=torch.float64):
    """z and the gradients of <w, z> (w: cotangent of z) through the library."""
    K, H, W = x.shape
    xt = torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)
    wt = torch.as_tensor(np.ascontiguousarray(w)).to(device="cuda", dtype=dtype)
    pr = S.Problem(K, H, W, M, c, p, lam, mu, iters, input_is_logits=logits)
    ws = torch.empty(S.segsalsa_str_grad_workspace_size(pr, S._prec(dtype), ck), dtype=torch.uint8, device="cuda")
    z = torch.empty_like(xt)
    S.segsalsa_str_solve_ckpt(pr, ck, xt, z, ws)
    gi = torch.empty_like(xt)
    gl = torch.zeros(1, dtype=torch.float64, device="cuda")
    gw = torch.zeros(len(c), dtype=torch.float64, device="cuda")
    S.segsalsa_str_backward(pr, ck, xt, wt, gi, ws, gl, gw)
    torch.cuda.synchronize()
    return z, gi, float(gl.item()), gw.cpu().numpy()


def ref_grad(x, w, c, M, p, lam, mu, iters, logits):
    xt = torch.from_numpy(np.ascontiguousarray(x)).clone().requires_grad_(True)
    ct = torch.tensor(np.asarray(c, dtype=np.float64), requires_grad=True)
    lt = torch.tensor(float(lam), dtype=torch.float64, requires_grad=True)
    ph = TR.softmax_input(xt) if logits else TR.normalise_input(xt)
    z = TR.solve_torch(ph, ct, M, p, lt, mu, iters)
    loss = torch.sum(torch.from_numpy(w) * z)
    gx, gc, gl = torch.autograd.grad(loss, (xt, ct, lt), allow_unused=True, materialize_grads=True)
    return z.detach().numpy(), gx.numpy(), float(gl), gc.numpy()


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


# (H, W, K, M, p, lam, mu, iters, logits): sizes that span several tiles with ragged edges
CASES = [
    (40, 52, 5, 1, 1.0, 0.6, 1.3, 12, True),
    (37, 29, 4, 1, 2.0, 0.8, 1.1, 10, False),
    (33, 45, 6, 1, math.inf, 0.7, 1.5, 10, True),
    (29, 31, 3, 0, 1.0, 0.5, 1.0, 9, False),
    (26, 34, 4, 2, 1.0, 0.9, 1.7, 8, True),
    (31, 27, 5, 1, 1.0, 0.0, 1.2, 8, True),
    (20, 24, 11, 1, 1.0, 0.7, 1.4, 5, True),     # two (FP32) or four (FP64) classes per wavefront, last one padded
    (18, 22, 16, 2, math.inf, 0.9, 1.6, 4, False),  # four classes per wavefront (the paper's K and patch)
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}_k{c[2]}_m{c[3]}_p{c[4]}_l{c[5]}" for c in CASES])
def test_fp64_gradient_matches_reference(case):
    S = need_gpu()
    H, W, K, M, p, lam, mu, iters, logits = case
    probs, lg, _ = synth.make_image(H, W, K, 500 + H, 1.0, 1.5)
    x = lg if logits else probs
    c = synth.gaussian_patch_multipliers(M, 1.0)
    w = np.random.default_rng(H * W).standard_normal((K, H, W))
    say(f"case {case}")
    z, gi, gl, gw = gpu_grad(S, x, w, c, M, p, lam, mu, iters, logits)
    zr, gxr, glr, gwr = ref_grad(x, w, c, M, p, lam, mu, iters, logits)
    ez = float(np.max(np.abs(z.cpu().numpy() - zr)))
    ex, el, ew = rel(gi.cpu().numpy(), gxr), abs(gl - glr) / max(abs(glr), 1e-300), rel(gw, gwr)
    say(f"  z {ez:.1e}  grad_input {ex:.1e}  grad_lambda {el:.1e}  grad_weights {ew:.1e}")
    assert ez <= 1e-12
    assert ex <= 1e-9 and ew <= 1e-9
    assert el <= 1e-9 or (lam == 0.0 and abs(gl - glr) <= 1e-9 * max(1.0, abs(glr)))


FP32_CASES = [CASES[0], CASES[-2], CASES[-1]]


@pytest.mark.parametrize("case", FP32_CASES, ids=[f"{c[0]}x{c[1]}_k{c[2]}_m{c[3]}" for c in FP32_CASES])
def test_fp32_gradient_near_reference(case):
    S = need_gpu()
    H, W, K, M, p, lam, mu, iters, logits = case
    probs, lg, _ = synth.make_image(H, W, K, 500 + H, 1.0, 1.5)
    x32 = (lg if logits else probs).astype(np.float32).astype(np.float64)
    c = synth.gaussian_patch_multipliers(M, 1.0)
    w32 = np.random.default_rng(H * W).standard_normal((K, H, W)).astype(np.float32).astype(np.float64)
    c32 = np.asarray(c, dtype=np.float32).astype(np.float64)
    say(f"case {case} FP32")
    _, gi, gl, gw = gpu_grad(S, x32, w32, c32, M, p, lam, mu, iters, logits, dtype=torch.float32)
    _, gxr, glr, gwr = ref_grad(x32, w32, c32, M, p, lam, mu, iters, logits)
    ex, el, ew = rel(gi.double().cpu().numpy(), gxr), abs(gl - glr) / abs(glr), rel(gw, gwr)
    say(f"  FP32: grad_input {ex:.1e}  grad_lambda {el:.1e}  grad_weights {ew:.1e}")
    assert ex <= 1e-3 and el <= 1e-3 and ew <= 1e-3


def test_checkpoint_interval_and_forward_are_exact():
    S = need_gpu()
    H, W, K, M = 35, 41, 5, 1
    _, lg, _ = synth.make_image(H, W, K, 77, 1.0, 1.5)
    c = synth.gaussian_patch_multipliers(M, 1.0)
    w = np.random.default_rng(3).standard_normal((K, H, W))
    outs = [gpu_grad(S, lg, w, c, M, 1.0, 0.7, 1.3, 11, True, ck=ck) for ck in (1, 4, 11, 100)]
    for z, gi, gl, gw in outs[1:]:
        assert torch.equal(z, outs[0][0]) and torch.equal(gi, outs[0][1])
        assert gl == outs[0][2] and np.array_equal(gw, outs[0][3])
    x = torch.from_numpy(lg).cuda()
    pr = S.Problem(K, H, W, M, c, 1.0, 0.7, 1.3, 11, input_is_logits=True)
    ws = torch.empty(S.segsalsa_str_workspace_size(pr, S.SEGSALSA_FP64), dtype=torch.uint8, device="cuda")
    z = torch.empty_like(x)
    S.segsalsa_str_solve(pr, x, z, ws)
    torch.cuda.synchronize()
    assert torch.equal(z, outs[0][0])


def test_zero_rounds():
    S = need_gpu()
    H, W, K = 13, 17, 4
    probs, lg, _ = synth.make_image(H, W, K, 9, 1.0, 1.5)
    c = synth.gaussian_patch_multipliers(1, 1.0)
    w = np.random.default_rng(4).standard_normal((K, H, W))
    for x, logits in ((lg, True), (probs, False)):
        z, gi, gl, gw = gpu_grad(S, x, w, c, 1, 1.0, 0.7, 1.3, 0, logits)
        _, gxr, _, _ = ref_grad(x, w, c, 1, 1.0, 0.7, 1.3, 0, logits)
        assert rel(gi.cpu().numpy(), gxr) <= 1e-14
        assert gl == 0.0 and np.all(gw == 0.0)


def test_autograd_function_matches_direct_call():
    S = need_gpu()
    H, W, K, M = 24, 30, 4, 1
    _, lg, labels = synth.make_image(H, W, K, 12, 1.0, 1.5)
    c = synth.gaussian_patch_multipliers(M, 1.0)
    x = torch.from_numpy(lg).cuda().requires_grad_(True)
    lam = torch.tensor(0.6, dtype=torch.float64, device="cuda", requires_grad=True)
    wts = torch.tensor(c, dtype=torch.float64, device="cuda", requires_grad=True)
    z = S.SegSalsaSTR.apply(x, lam, wts, M, 1.0, 1.3, 9, True, 4)
    lab = torch.from_numpy(labels).long().cuda()
    loss = -torch.log(torch.gather(z, 0, lab[None])[0].clamp_min(1e-6)).mean()
    gx, glam, gw = torch.autograd.grad(loss, (x, lam, wts))
    # the same cotangent through the C-ABI directly
    zd = z.detach().clone().requires_grad_(True)
    ld = -torch.log(torch.gather(zd, 0, lab[None])[0].clamp_min(1e-6)).mean()
    (gzd,) = torch.autograd.grad(ld, zd)
    _, gi, gl, gwd = gpu_grad(S, lg, gzd.cpu().numpy(), c, M, 1.0, 0.6, 1.3, 9, True, ck=4)
    assert torch.equal(gx, gi) and float(glam) == gl and np.array_equal(gw.cpu().numpy(), gwd)


def ce_loss_gpu(S, pr, x, labels_t):
    ws = torch.empty(S.segsalsa_str_workspace_size(pr, S.SEGSALSA_FP64), dtype=torch.uint8, device="cuda")
    z = torch.empty_like(x)
    S.segsalsa_str_solve(pr, x, z, ws)
    zy = torch.gather(z, 0, labels_t[None])[0]
    return float(-torch.log(zy.clamp_min(1e-6)).mean().item())


def fullsize_adjoint(S, wl, d, dtype, gz=None, ck=10):
    lg = d["logits"]
    c = np.asarray(d["weights"])
    K, H, W = lg.shape
    lab = torch.from_numpy(d["labels"]).long().cuda()
    x = torch.from_numpy(lg).to(device="cuda", dtype=dtype)
    pr = S.Problem(K, H, W, wl.M, list(c), wl.schatten_p, wl.lam, wl.mu, wl.iters, input_is_logits=True)
    ws = torch.empty(S.segsalsa_str_grad_workspace_size(pr, S._prec(dtype), ck), dtype=torch.uint8, device="cuda")
    z = torch.empty_like(x)
    S.segsalsa_str_solve_ckpt(pr, ck, x, z, ws)
    if gz is None:
        zd = z.double().clone().requires_grad_(True)
        ld = -torch.log(torch.gather(zd, 0, lab[None])[0].clamp_min(1e-6)).mean()
        (gz,) = torch.autograd.grad(ld, zd)
    gi = torch.empty_like(x)
    gl = torch.zeros(1, dtype=torch.float64, device="cuda")
    gw = torch.zeros(len(c), dtype=torch.float64, device="cuda")
    S.segsalsa_str_backward(pr, ck, x, gz.to(dtype), gi, ws, gl, gw)
    torch.cuda.synchronize()
    return z, gz, gi.double().cpu().numpy(), float(gl.item()), gw.cpu().numpy()


def test_fullsize_few_rounds_against_reference():
    """256x256, K = 8, 3x3 patch (the full image and tile grid), 5 rounds: FP64 adjoint vs the reference."""
    S = need_gpu()
    wl = synth.WORKLOADS["diff_256x256_k8"]
    d = synth.make_workload(wl)
    short = synth.Workload(**{**wl.__dict__, "iters": 5})
    say(f"case {wl.name} at 5 rounds: FP64 adjoint vs the reference gradient")
    w = np.random.default_rng(21).standard_normal(d["logits"].shape)
    _, _, gi, gl, gw = fullsize_adjoint(S, short, d, torch.float64, gz=torch.from_numpy(w).cuda(), ck=2)
    _, gxr, glr, gwr = ref_grad(d["logits"], w, d["weights"], wl.M, wl.schatten_p, wl.lam, wl.mu, 5, True)
    ex, el, ew = rel(gi, gxr), abs(gl - glr) / abs(glr), rel(gw, gwr)
    say(f"  grad_input {ex:.1e}  grad_lambda {el:.1e}  grad_weights {ew:.1e}")
    assert ex <= 1e-9 and el <= 1e-9 and ew <= 1e-9


def test_fullsize_fd_and_invariants():
    """256x256, K = 8, 3x3 patch, 50 rounds: FP64 adjoint vs central differences of the GPU forward.

    The proximity maps have kinks (the clamp at 0, the singular-value
    thresholds), and after 50 rounds some iterates sit within ~1e-7 of one
    (active positivity constraints: min z < 0 by 1e-2).  A central difference
    with step h is exact to O(h^2) only while no iterate crosses a kink
    within +-h, so the step must stay below that distance: h = 1e-8 for every
    direction.  Its rounding error is about eps |L| / h ~ 1e-8 relative per
    evaluation (L ~ 1), amplified by the 50 rounds to at most ~1e-6.  The
    steps 1e-6 and 1e-7 are logged for comparison only.
    Directions: two random ones and one along the gradient's signs.
    """
    S = need_gpu()
    wl = synth.WORKLOADS["diff_256x256_k8"]
    d = synth.make_workload(wl)
    lg = d["logits"]
    c = np.asarray(d["weights"])
    K, H, W = lg.shape
    say(f"case {wl.name}: {wl.iters} rounds, FP64 adjoint vs finite differences")
    lab = torch.from_numpy(d["labels"]).long().cuda()
    x = torch.from_numpy(lg).cuda()

    def loss(xx, cc, ll):
        pr = S.Problem(K, H, W, wl.M, list(cc), wl.schatten_p, ll, wl.mu, wl.iters, input_is_logits=True)
        return ce_loss_gpu(S, pr, xx, lab)

    _, gz, gin, gl, gw = fullsize_adjoint(S, wl, d, torch.float64)
    # invariance: softmax ignores per-pixel constants
    inv = float(np.max(np.abs(gin.sum(axis=0)))) / float(np.max(np.abs(gin)))
    say(f"  max |sum_k dL/dlogit_k| / max |dL/dlogit| = {inv:.1e}")
    assert inv <= 1e-10
    rng = np.random.default_rng(11)
    FD_STEP = 1e-8

    def check(name, an, fplus_minus):
        out = None
        for h in (1e-6, 1e-7, FD_STEP):
            fp, fm = fplus_minus(h)
            fd = (fp - fm) / (2 * h)
            err = abs(an - fd) / abs(an)
            say(f"  {name}: h {h:.0e} adjoint {an:.10e} fd {fd:.10e} rel {err:.1e}")
            if h == FD_STEP:
                out = err
        return out

    worst = 0.0
    dirs = [rng.standard_normal(lg.shape), rng.standard_normal(lg.shape), np.sign(gin) * rng.random(lg.shape)]
    for t, dvec in enumerate(dirs):
        dt = torch.from_numpy(dvec).cuda()
        worst = max(worst, check(f"logits direction {t}", float(np.sum(gin * dvec)),
                                 lambda h: (loss(x + h * dt, c, wl.lam), loss(x - h * dt, c, wl.lam))))
    dc = rng.standard_normal(c.shape)
    worst = max(worst, check("weights", float(np.sum(gw * dc)),
                             lambda h: (loss(x, c + h * dc, wl.lam), loss(x, c - h * dc, wl.lam))))
    worst = max(worst, check("lambda", gl, lambda h: (loss(x, c, wl.lam + h), loss(x, c, wl.lam - h))))
    say(f"  worst relative difference at h = {FD_STEP:.0e}: {worst:.2e}")
    assert worst <= 1e-5
    # FP32 adjoint on the same cotangent against FP64.  After 50 rounds some iterates sit within
    # ~1e-7 of a kink, so FP32 rounding of the forward state (z differs by ~1e-6) moves a few of
    # them across it and changes the local derivative there: the max-abs difference of the input
    # gradient is dominated by those pixels, its L2 difference and the global sums (lambda,
    # weights) are not.
    z32, _, gi32, gl32, gw32 = fullsize_adjoint(S, wl, d, torch.float32, gz=gz)
    e_in, e_l, e_w = rel(gi32, gin), abs(gl32 - gl) / abs(gl), rel(gw32, gw)
    e_l2 = float(np.linalg.norm(gi32 - gin) / np.linalg.norm(gin))
    say(f"  FP32 vs FP64 adjoint: input max {e_in:.2e} L2 {e_l2:.2e} lambda {e_l:.2e} weights {e_w:.2e}")
    assert e_in <= 2.5e-2 and e_l2 <= 2e-3 and e_l <= 2.5e-4 and e_w <= 2.5e-4


def test_autograd_function_with_host_parameters():
    """SegSalsaSTR with lambda and the patch weights as CPU tensors: their gradients come back on
    the CPU (in their dtype) and equal those of device parameters."""
    S = need_gpu()
    H, W, K, M, iters = 20, 23, 4, 1, 6
    _, logits, _ = synth.make_image(H, W, K, 41, 1.0, 1.5)
    c = synth.gaussian_patch_multipliers(M, 1.0)
    wgt = torch.from_numpy(np.random.default_rng(42).standard_normal((K, H, W))).cuda()
    grads = {}
    for dev in ("cpu", "cuda"):
        x = torch.from_numpy(logits).cuda().requires_grad_(True)
        lam = torch.tensor(0.9, dtype=torch.float64, device=dev, requires_grad=True)
        cw = torch.tensor(np.asarray(c), dtype=torch.float32, device=dev, requires_grad=True)
        z = S.SegSalsaSTR.apply(x, lam, cw, M, 1.0, 1.2, iters, True, 3)
        torch.sum(wgt * z).backward()
        assert lam.grad.device.type == dev and cw.grad.device.type == dev and cw.grad.dtype == torch.float32
        grads[dev] = (x.grad.cpu(), lam.grad.cpu(), cw.grad.cpu())
    for a, b in zip(grads["cpu"], grads["cuda"]):
        assert torch.equal(a, b)
