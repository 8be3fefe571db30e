"""Independent pin code for the oracle's tests.

Nothing here imports the oracle.  Each helper computes a quantity the paper
fixes by a route other than the oracle's: explicit index arithmetic instead
of array rolls, dense matrices and least squares instead of FFT
diagonalisation, the literal three-step SALSA loop with an explicit u, the
SegSALSA vector-TV special case coded from its own definition, and a
primal-dual (Chambolle-Pock) solver for the same convex problem.
"""
from __future__ import annotations

import math

import numpy as np


def offsets(M):
    return [(dy, dx) for dy in range(-M, M + 1) for dx in range(-M, M + 1)]


def dense_jacobian(H, W, K, c, M):
    """Matrix of the patch-based Jacobian (eq. (4)) by explicit index arithmetic.

    Rows are ordered [L][2][K][H][W], columns [K][H][W].  Row (j, h, k, r, q)
    is c_j times the forward difference of class k taken at pixel
    (r + dy_j, q + dx_j), periodic, horizontal for h = 0 and vertical for h = 1.
    """
    offs = offsets(M)
    L = len(offs)
    n = H * W
    Jm = np.zeros((L * 2 * K * n, K * n))

    def col(k, r, q):
        return k * n + (r % H) * W + (q % W)

    row = 0
    for j, (dy, dx) in enumerate(offs):
        for h in range(2):
            for k in range(K):
                for r in range(H):
                    for q in range(W):
                        rr, qq = r + dy, q + dx
                        if h == 0:
                            Jm[row, col(k, rr, qq + 1)] += c[j]
                        else:
                            Jm[row, col(k, rr + 1, qq)] += c[j]
                        Jm[row, col(k, rr, qq)] -= c[j]
                        row += 1
    return Jm


def dense_G(H, W, K, c, M):
    """G = [I; J; I; I] stacked (eqs. (9), (11))."""
    I = np.eye(K * H * W)
    return np.vstack([I, dense_jacobian(H, W, K, c, M), I, I])


def data_prox_closed(v, p, mu):
    """argmin_u -ln(p^T u) + mu/2 ||u - v||^2 for one pixel (vectors of length K)."""
    s = float(p @ v)
    q = float(p @ p)
    t = (s + math.sqrt(s * s + 4.0 * q / mu)) / 2.0 if s >= 0 else \
        (2.0 * q / mu) / (math.sqrt(s * s + 4.0 * q / mu) - s)
    return v + p / (mu * t)


def shrink_sv(S, tau, pchoice):
    """Prox of tau ||.||_p on a vector of singular values (two entries)."""
    S = np.asarray(S, dtype=float)
    if pchoice not in (1, 2) and not math.isinf(pchoice):
        # general p: minimise 1/2 ||x - S||^2 + tau ||x||_p directly
        from scipy import optimize
        f = lambda x: 0.5 * np.sum((x - S) ** 2) + tau * np.sum(np.abs(x) ** pchoice) ** (1.0 / pchoice)
        best = None
        for x0 in (S, 0.5 * S, S * 0 + 1e-3):
            r = optimize.minimize(f, x0, method="Nelder-Mead",
                                  options=dict(xatol=1e-13, fatol=1e-16, maxiter=40000))
            if best is None or r.fun < best.fun:
                best = r
        return np.maximum(best.x, 0.0)
    if pchoice == 1:
        return np.maximum(S - tau, 0.0)
    if pchoice == 2:
        n = np.linalg.norm(S)
        return S * max(0.0, 1.0 - tau / n) if n > 0 else S * 0.0
    # p = inf: Moreau, l1-ball projection of two nonnegative numbers by bisection
    if S.sum() <= tau:
        return S * 0.0
    lo, hi = 0.0, float(S.max())
    for _ in range(200):
        th = 0.5 * (lo + hi)
        if np.maximum(S - th, 0).sum() > tau:
            lo = th
        else:
            hi = th
    th = 0.5 * (lo + hi)
    return S - np.maximum(S - th, 0.0)


def literal_salsa(phat, c, M, pchoice, lam, mu, n_zupdates, g4="affine"):
    """SALSA exactly as eqs. (12)-(14) print it, with u kept explicitly.

    z-update: least squares min ||G z - u - d|| on the dense G (eq. (12));
    u-update: prox of each g_j at H_j z^{k+1} - d_j^k (eq. (13), z^{k+1});
    d-update: d <- d - (G z - u) (eq. (14)).
    Initialisation z^0 = phat, u^0 = G z^0, d^0 = 0.  Returns z after
    `n_zupdates` z-updates.
    """
    K, H, W = phat.shape
    n = H * W
    L = (2 * M + 1) ** 2
    G = dense_G(H, W, K, c, M)
    z = phat.reshape(-1).copy()
    u = G @ z
    d = np.zeros_like(u)
    Kn = K * n
    p_pix = phat.reshape(K, n)
    for it in range(n_zupdates):
        z = np.linalg.lstsq(G, u + d, rcond=None)[0]
        if it == n_zupdates - 1:
            break
        Gz = G @ z
        v = Gz - d
        unew = np.empty_like(u)
        # g1: data term, per pixel
        v1 = v[:Kn].reshape(K, n)
        u1 = np.empty_like(v1)
        for i in range(n):
            u1[:, i] = data_prox_closed(v1[:, i], p_pix[:, i], mu)
        unew[:Kn] = u1.reshape(-1)
        # g2: Schatten prox of the (LK) x 2 block per pixel
        v2 = v[Kn:Kn + 2 * L * Kn].reshape(L, 2, K, n)
        u2 = np.empty_like(v2)
        for i in range(n):
            B = v2[:, :, :, i].transpose(0, 2, 1).reshape(L * K, 2)
            U, S, Vt = np.linalg.svd(B, full_matrices=False)
            Bn = U @ np.diag(shrink_sv(S, lam / mu, pchoice)) @ Vt
            u2[:, :, :, i] = Bn.reshape(L, K, 2).transpose(0, 2, 1)
        unew[Kn:Kn + 2 * L * Kn] = u2.reshape(-1)
        # g3: positive orthant
        off3 = Kn + 2 * L * Kn
        unew[off3:off3 + Kn] = np.maximum(v[off3:off3 + Kn], 0.0)
        # g4: 1^T xi = 1 per pixel
        v4 = v[off3 + Kn:].reshape(K, n)
        if g4 == "affine":
            unew[off3 + Kn:] = (v4 - (v4.sum(axis=0) - 1.0) / K).reshape(-1)
        else:  # probability simplex, threshold by bisection per pixel
            u4 = np.empty_like(v4)
            for i in range(n):
                u4[:, i] = simplex_proj_vec(v4[:, i])
            unew[off3 + Kn:] = u4.reshape(-1)
        u = unew
        d = d - (Gz - u)
    return z.reshape(K, H, W)


def vtv_salsa(phat, lam, mu, rounds):
    """SegSALSA with the vector-TV prior, coded from its own definition.

    Prior lam * sum_i ||grad z_i||_F with grad z_i the K x 2 matrix of forward
    periodic differences; splits (data, gradient, positivity, sum-to-one);
    the gradient prox is a group soft-threshold of the K x 2 block; the
    z-update solves (3 + D_h^T D_h + D_v^T D_v) z = rhs with the Laplacian's
    Fourier symbol.  Same initialisation and round order as the oracle.
    """
    K, H, W = phat.shape

    def gx(a):
        return a[:, :, np.r_[1:W, 0]] - a

    def gy(a):
        return a[:, np.r_[1:H, 0], :] - a

    def gxT(a):
        return a[:, :, np.r_[W - 1, 0:W - 1]] - a

    def gyT(a):
        return a[:, np.r_[H - 1, 0:H - 1], :] - a

    ky = np.arange(H)[:, None]
    kx = np.arange(W)[None, :]
    sym = 3.0 + (2.0 - 2.0 * np.cos(2 * np.pi * kx / W)) + (2.0 - 2.0 * np.cos(2 * np.pi * ky / H))
    z = phat.copy()
    d1 = np.zeros_like(z); d3 = np.zeros_like(z); d4 = np.zeros_like(z)
    dx_ = np.zeros_like(z); dy_ = np.zeros_like(z)
    tau = lam / mu
    for _ in range(rounds):
        v1 = z - d1
        u1 = np.empty_like(v1)
        for r in range(H):
            for q in range(W):
                u1[:, r, q] = data_prox_closed(v1[:, r, q], phat[:, r, q], mu)
        vx = gx(z) - dx_
        vy = gy(z) - dy_
        nrm = np.sqrt(np.sum(vx * vx + vy * vy, axis=0))
        fac = np.where(nrm > tau, 1.0 - tau / np.where(nrm > 0, nrm, 1.0), 0.0)
        ux, uy = vx * fac, vy * fac
        v3 = z - d3
        u3 = np.maximum(v3, 0.0)
        v4 = z - d4
        u4 = v4 - (v4.sum(axis=0) - 1.0) / K
        d1 = u1 - v1; dx_ = ux - vx; dy_ = uy - vy; d3 = u3 - v3; d4 = u4 - v4
        rhs = (u1 + d1) + gxT(ux + dx_) + gyT(uy + dy_) + (u3 + d3) + (u4 + d4)
        z = np.real(np.fft.ifft2(np.fft.fft2(rhs) / sym))
    return z


def simplex_proj_vec(v):
    """Projection of one vector onto the probability simplex by bisection on the threshold."""
    lo, hi = float(v.min()) - 1.0, float(v.max())
    for _ in range(200):
        th = 0.5 * (lo + hi)
        if np.maximum(v - th, 0).sum() > 1.0:
            lo = th
        else:
            hi = th
    return np.maximum(v - 0.5 * (lo + hi), 0.0)


def objective_dense(zvec, phat, Jm, K, n, L, lam, pchoice):
    """Objective of eq. (7) evaluated with the dense Jacobian and SVDs."""
    z = zvec.reshape(K, n)
    val = -np.sum(np.log(np.sum(phat.reshape(K, n) * z, axis=0)))
    Jz = (Jm @ zvec).reshape(L, 2, K, n)
    for i in range(n):
        B = Jz[:, :, :, i].transpose(0, 2, 1).reshape(L * K, 2)
        S = np.linalg.svd(B, compute_uv=False)
        if pchoice == 1:
            nrm = S.sum()
        elif pchoice == 2:
            nrm = np.linalg.norm(S)
        elif math.isinf(pchoice):
            nrm = S.max()
        else:   # general p >= 1: the l_p norm of the singular values, written out
            nrm = sum(float(x) ** pchoice for x in S) ** (1.0 / pchoice)
        val += lam * nrm
    return float(val)


def lq_ball_proj_2d(S, q, rad, grid=2049, refine=90):
    """Projection of nonnegative 2-vectors (rows of S) onto {y : y1^q + y2^q <= rad^q}, 1 < q < inf.

    Outside the ball the projection lies on its boundary, which in the first quadrant is
    y(t) = rad (cos(t)^(2/q), sin(t)^(2/q)), t in [0, pi/2].  The squared distance to y(t)
    is minimised on a dense grid of t, then refined by golden-section search inside the
    bracket around the best grid point.
    """
    S = np.asarray(S, dtype=float)
    out = S.copy()
    outside = np.sum(S ** q, axis=1) > rad ** q
    if not np.any(outside):
        return out
    w = S[outside]

    def dist(t):
        c = np.cos(t) ** (2.0 / q)
        s = np.sin(t) ** (2.0 / q)
        return (rad * c - w[:, :1]) ** 2 + (rad * s - w[:, 1:2]) ** 2

    ts = np.linspace(0.0, 0.5 * math.pi, grid)[None, :]
    i = np.argmin(dist(ts), axis=1)
    h = 0.5 * math.pi / (grid - 1)
    a = np.clip(ts[0, i] - h, 0.0, 0.5 * math.pi)[:, None]
    b = np.clip(ts[0, i] + h, 0.0, 0.5 * math.pi)[:, None]
    g = (math.sqrt(5.0) - 1.0) / 2.0
    for _ in range(refine):
        c1 = b - g * (b - a)
        c2 = a + g * (b - a)
        left = dist(c1) < dist(c2)
        b = np.where(left, c2, b)
        a = np.where(left, a, c1)
    t = 0.5 * (a + b)
    out[outside] = np.hstack([rad * np.cos(t) ** (2.0 / q), rad * np.sin(t) ** (2.0 / q)])
    return out


def pdhg(phat, c, M, pchoice, lam, iters):
    """Chambolle-Pock primal-dual solver for eq. (7).

    min_z  F(A z) + i_simplex(z),  A = [I; J] (dense J from index arithmetic),
    F(a, b) = sum_i -ln(p_i^T a_i) + lam sum_i ||b_i||_{S_p}.
    Dual prox of the Schatten part = projection of the singular values onto
    the dual-norm ball (S_inf, S_2, S_1 or, for general p, S_q ball of radius lam); dual prox of the
    data part by Moreau's identity with the closed-form primal prox.
    Returns (z, objective at z).
    """
    K, H, W = phat.shape
    n = H * W
    L = (2 * M + 1) ** 2
    Jm = dense_jacobian(H, W, K, c, M)
    A = np.vstack([np.eye(K * n), Jm])
    normA = np.linalg.norm(A, 2)
    tau_p = sig_d = 0.99 / normA
    z = phat.reshape(-1).copy()
    zbar = z.copy()
    y = np.zeros(A.shape[0])
    pp = phat.reshape(K, n)
    qq = np.sum(pp * pp, axis=0)
    for _ in range(iters):
        w = y + sig_d * (A @ zbar)
        # data part: prox_{sig f*}(w) = w - sig prox_{f/sig}(w/sig), vectorised over pixels
        wa = w[:K * n].reshape(K, n) / sig_d
        s = np.sum(pp * wa, axis=0)
        disc = np.sqrt(s * s + 4.0 * qq / sig_d)
        t = np.where(s >= 0, 0.5 * (s + disc), (2.0 * qq / sig_d) / np.where(s >= 0, 1.0, disc - s))
        ya = sig_d * wa - sig_d * (wa + pp / (sig_d * t))
        wb = w[K * n:].reshape(L, 2, K, n).transpose(3, 0, 2, 1).reshape(n, L * K, 2)
        U, S, Vt = np.linalg.svd(wb, full_matrices=False)
        if pchoice == 1:
            S2 = np.minimum(S, lam)
        elif pchoice == 2:
            nr = np.linalg.norm(S, axis=1, keepdims=True)
            S2 = S * np.minimum(1.0, lam / np.where(nr > 0, nr, 1.0))
        elif not math.isinf(pchoice):
            # general p: the dual norm ball is the l_q ball, 1/p + 1/q = 1
            S2 = lq_ball_proj_2d(S, pchoice / (pchoice - 1.0), lam)
        else:
            lo = np.zeros(n)
            hi = S.max(axis=1)
            for _b in range(100):
                th = 0.5 * (lo + hi)
                big = np.maximum(S - th[:, None], 0).sum(axis=1) > lam
                lo = np.where(big, th, lo)
                hi = np.where(big, hi, th)
            inside = S.sum(axis=1) <= lam
            S2 = np.where(inside[:, None], S, np.maximum(S - (0.5 * (lo + hi))[:, None], 0.0))
        yb = np.einsum("nij,nj,njk->nik", U, S2, Vt).reshape(n, L, K, 2).transpose(1, 3, 2, 0)
        y = np.concatenate([ya.reshape(-1), yb.reshape(-1)])
        zn = (z - tau_p * (A.T @ y)).reshape(K, n)
        lo = zn.min(axis=0) - 1.0
        hi = zn.max(axis=0)
        for _b in range(100):
            th = 0.5 * (lo + hi)
            big = np.maximum(zn - th, 0).sum(axis=0) > 1.0
            lo = np.where(big, th, lo)
            hi = np.where(big, hi, th)
        zn = np.maximum(zn - 0.5 * (lo + hi), 0.0).reshape(-1)
        zbar = 2 * zn - z
        z = zn
    return z.reshape(K, H, W), objective_dense(z, phat, Jm, K, n, L, lam, pchoice)


def _l1_theta(S, r):
    lo, hi = 0.0, float(S.max())
    for _ in range(200):
        th = 0.5 * (lo + hi)
        if np.maximum(S - th, 0).sum() > r:
            lo = th
        else:
            hi = th
    return 0.5 * (lo + hi)
