"""FP64 reference gradient of the unrolled SegSALSA-STR rounds (PyTorch CPU autograd).

TEST INFRASTRUCTURE ONLY (same rules as segsalsa_ref: only the tests, the
smoke check and the benchmark's CPU baseline may import it).

The rounds of eqs. (12)-(14) written with differentiable PyTorch CPU ops in
FP64, so that autograd gives the gradient of a loss of z^N with respect to
the logits (or probabilities), lambda and the patch multipliers c_j.  The
steps are those of the numpy oracle (same readings); the Schatten proximity
operator is written through the 2x2 structure tensor with closed-form
eigenvalues and the eigenvector angle, so its a.e. derivative is finite at
repeated singular values.
"""
from __future__ import annotations

import math

import torch

__all__ = ["softmax_input", "normalise_input", "solve_torch", "schatten_prox_torch", "ce_loss"]


def patch_offsets(M):
    return [(dy, dx) for dy in range(-M, M + 1) for dx in range(-M, M + 1)]


def shift(w, dy, dx):
    """(S_s w)_i = w_{i+s}, periodic (Sec. 3)."""
    return torch.roll(w, shifts=(-dy, -dx), dims=(-2, -1))


def dh(z):
    return torch.roll(z, -1, dims=-1) - z


def dv(z):
    return torch.roll(z, -1, dims=-2) - z


def dh_adj(y):
    return torch.roll(y, 1, dims=-1) - y


def dv_adj(y):
    return torch.roll(y, 1, dims=-2) - y


def jac(z, c, M):
    """Patch-based Jacobian, eq. (4): list of (h, v) parts per offset, each [K][H][W]."""
    gh, gv = dh(z), dv(z)
    return [(c[j] * shift(gh, dy, dx), c[j] * shift(gv, dy, dx)) for j, (dy, dx) in enumerate(patch_offsets(M))]


def jac_adj(w, c, M):
    ah = 0.0
    av = 0.0
    for j, (dy, dx) in enumerate(patch_offsets(M)):
        ah = ah + c[j] * shift(w[j][0], -dy, -dx)
        av = av + c[j] * shift(w[j][1], -dy, -dx)
    return dh_adj(ah) + dv_adj(av)


def solve_gtg(rhs, c, H, W):
    """z-update, eq. (12): (3 + sum c^2 (D_h^T D_h + D_v^T D_v)) z = rhs by the 2-D DFT."""
    ky = torch.arange(H, dtype=torch.float64)[:, None]
    kx = torch.arange(W, dtype=torch.float64)[None, :]
    lap = 4 * torch.sin(math.pi * kx / W) ** 2 + 4 * torch.sin(math.pi * ky / H) ** 2
    sym = 3 + torch.sum(c * c) * lap
    return torch.fft.ifft2(torch.fft.fft2(rhs) / sym).real


def prox_data(v, p, mu):
    """g1 prox (eq. (10)): u = v + p / (mu t), t the positive root of mu t^2 - mu (p^T v) t - ||p||^2."""
    s = torch.sum(p * v, dim=0)
    q = torch.sum(p * p, dim=0)
    disc = torch.sqrt(s * s + 4 * q / mu)
    pos = s >= 0
    t = torch.where(pos, 0.5 * (s + disc), (2 * q / mu) / torch.where(pos, torch.ones_like(s), disc - s))
    return v + p / (mu * t)


def schatten_prox_torch(Y, tau, p):
    """Prox of tau ||.||_{S_p} per pixel on the (LK) x 2 blocks given as a list of (h, v) parts (Sec. 3/4)."""
    A = sum(torch.sum(yh * yh, dim=0) for yh, _ in Y)
    B = sum(torch.sum(yh * yv, dim=0) for yh, yv in Y)
    C = sum(torch.sum(yv * yv, dim=0) for _, yv in Y)
    hs, hd = 0.5 * (A + C), 0.5 * (A - C)
    R = torch.sqrt(hd * hd + B * B + 1e-300)
    lp = hs + R
    lm = torch.clamp(hs - R, min=0.0)
    sp = torch.sqrt(lp + 1e-300)
    sm = torch.sqrt(lm + 1e-300)
    zero = torch.zeros_like(sp)
    if p == 2.0:
        r = torch.sqrt(A + C + 1e-300)
        rho = torch.where(r > tau, 1 - tau / r, zero)
        return [(yh * rho, yv * rho) for yh, yv in Y]
    if p == 1.0:
        rp = torch.where(sp > tau, 1 - tau / sp, zero)
        rm = torch.where(sm > tau, 1 - tau / sm, zero)
    else:  # p = inf: sigma - projection on the l1 ball of radius tau
        th = 0.5 * (sp + sm - tau)
        inside = (sp + sm) <= tau
        caseb = (sp - sm) >= tau
        rp = torch.where(inside, zero, torch.where(caseb, 1 - tau / sp, th / sp))
        rm = torch.where(inside, zero, torch.where(caseb, torch.ones_like(sm), th / sm))
    ang = 0.5 * torch.atan2(2 * B, A - C)
    cs, sn = torch.cos(ang), torch.sin(ang)
    n11 = rp * cs * cs + rm * sn * sn
    n22 = rp * sn * sn + rm * cs * cs
    n12 = (rp - rm) * cs * sn
    return [(yh * n11 + yv * n12, yh * n12 + yv * n22) for yh, yv in Y]


def softmax_input(logits):
    return torch.softmax(logits, dim=0)


def normalise_input(probs):
    return probs / probs.sum(dim=0, keepdim=True)


def solve_torch(phat, c, M, p, lam, mu, iters):
    """z after `iters` rounds (u-update, d-update, z-update), differentiable in phat, c, lam."""
    K, H, W = phat.shape
    L = (2 * M + 1) ** 2
    z = phat
    d1 = torch.zeros_like(phat)
    d3 = torch.zeros_like(phat)
    d4 = torch.zeros_like(phat)
    d2 = [(torch.zeros_like(phat), torch.zeros_like(phat)) for _ in range(L)]
    tau = lam / mu
    for _ in range(iters):
        v1 = z - d1
        u1 = prox_data(v1, phat, mu)
        n1 = u1 - v1
        Jz = jac(z, c, M)
        Y = [(jh - e[0], jv - e[1]) for (jh, jv), e in zip(Jz, d2)]
        U2 = schatten_prox_torch(Y, tau, p)
        n2 = [(uh - yh, uv - yv) for (uh, uv), (yh, yv) in zip(U2, Y)]
        v3 = z - d3
        u3 = torch.clamp(v3, min=0.0)
        n3 = u3 - v3
        v4 = z - d4
        u4 = v4 - (v4.sum(dim=0, keepdim=True) - 1.0) / K
        n4 = u4 - v4
        a2 = [(uh + nh, uv + nv) for (uh, uv), (nh, nv) in zip(U2, n2)]
        rhs = (u1 + n1) + jac_adj(a2, c, M) + (u3 + n3) + (u4 + n4)
        z = solve_gtg(rhs, c, H, W)
        d1, d2, d3, d4 = n1, n2, n3, n4
    return z


def ce_loss(z, labels, floor=1e-6):
    """Cross-entropy of z against a label map: -(1/n) sum_i ln(max(z_{y_i, i}, floor))."""
    K, H, W = z.shape
    zy = torch.gather(z, 0, labels.long().view(1, H, W))[0]
    return -torch.mean(torch.log(torch.clamp(zy, min=floor)))
