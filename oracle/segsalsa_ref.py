"""FP64 CPU oracle for the SegSALSA-STR iteration (arXiv 1504.07028).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  The product path (the HIP
library and its Python binding) never calls it and shares no code with it.

Plain, slow, FP64 numpy.  Every function cites the passage it follows.  The
method (Sec. 4 of the paper) is:

    minimise   sum_i -ln(p_i^T z_i) + lam * sum_i ||[J z]_i||_{S_p}        eq. (7)
    subject to z >= 0, 1_K^T z = 1_n

rewritten as sum_j g_j(H_j z) with H = (I, J, I, I) (eqs. (8)-(10)), split as
u = G z (eq. (11)) and solved by SALSA, eqs. (12)-(14).

Readings where the paper is silent or ambiguous (each one is also listed in
the design notes of the repository):

* initialisation (silent): z = p_i / 1^T p_i, d = 0, u = G z;
* eq. (13) prints z^k; ADMM uses the z just computed by eq. (12), z^{k+1};
* with that initialisation the first z-update returns z unchanged, so one
  "round" here is  u-update (13) -> d-update (14) -> z-update (12), and
  `iters = N` rounds give the paper's z^{N+1};
* g4 follows its definition in eq. (10), the indicator of {1_K^T xi = 1}: its
  proximity operator is the affine projection (the text calls it a simplex
  projection; positivity comes from g3);
* D_h, D_v are forward differences with periodic boundaries (the z-update is
  solved by cyclic convolutions);
* P_j shifts by the j-th offset s_j = (dy, dx) of the patch, row-major with dy
  outer, (P_j w)_i = c_j w_{i + s_j}; the multipliers c_j are inputs;
* the Schatten proximity operator is applied through the singular values of
  the (LK) x 2 block, obtained from the eigenvalues of the 2x2 structure
  tensor (Sec. 3); a singular value shrunk to 0 gets multiplier 0.

Arrays are class-planar: z, p are [K][H][W]; the J-split variables (u2, d2)
are [L][2][K][H][W] (offset, direction h/v, class, row, column).
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np

__all__ = [
    "patch_offsets", "shift", "diff_h", "diff_v", "diff_h_adj", "diff_v_adj",
    "jacobian", "jacobian_adj", "gtg_apply", "gtg_symbol", "solve_gtg",
    "prox_data", "prox_schatten", "prox_schatten_svd", "schatten_shrink",
    "project_l1_ball", "project_lq_ball", "prox_positive", "prox_sum_to_one",
    "State", "init_state", "salsa_round", "solve", "labels", "project_simplex",
    "objective", "schatten_norms", "Problem",
]


# ---------------------------------------------------------------------------
# Linear operators (Sec. 3, eq. (4); operator J of eq. (9))
# ---------------------------------------------------------------------------

def patch_offsets(M: int):
    """The L = (2M+1)^2 shifts of a (2M+1)x(2M+1) patch, row-major, dy outer (Sec. 3, eq. (4))."""
    return [(dy, dx) for dy in range(-M, M + 1) for dx in range(-M, M + 1)]


def shift(w: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """(S_s w)_i = w_{i+s} with periodic indices, s = (dy, dx) on the last two axes."""
    return np.roll(w, shift=(-dy, -dx), axis=(-2, -1))


def diff_h(z: np.ndarray) -> np.ndarray:
    """Horizontal forward difference, periodic: (D_h z)_{r,c} = z_{r,c+1} - z_{r,c} (Sec. 3)."""
    return np.roll(z, -1, axis=-1) - z


def diff_v(z: np.ndarray) -> np.ndarray:
    """Vertical forward difference, periodic: (D_v z)_{r,c} = z_{r+1,c} - z_{r,c} (Sec. 3)."""
    return np.roll(z, -1, axis=-2) - z


def diff_h_adj(y: np.ndarray) -> np.ndarray:
    """Adjoint of diff_h: (D_h^T y)_{r,c} = y_{r,c-1} - y_{r,c}."""
    return np.roll(y, 1, axis=-1) - y


def diff_v_adj(y: np.ndarray) -> np.ndarray:
    """Adjoint of diff_v: (D_v^T y)_{r,c} = y_{r-1,c} - y_{r,c}."""
    return np.roll(y, 1, axis=-2) - y


def jacobian(z: np.ndarray, c: np.ndarray, M: int) -> np.ndarray:
    """Patch-based Jacobian J z, eq. (4): rows (P_j D_h z)_i and (P_j D_v z)_i.

    Returns [L][2][K][H][W]; entry [j, 0] is c_j * shift(D_h z, s_j), entry
    [j, 1] is c_j * shift(D_v z, s_j).  J maps R^{K x n} to R^{2LK x n} (eq. (9)).
    """
    offs = patch_offsets(M)
    gh, gv = diff_h(z), diff_v(z)
    out = np.empty((len(offs), 2) + z.shape, dtype=np.float64)
    for j, (dy, dx) in enumerate(offs):
        out[j, 0] = c[j] * shift(gh, dy, dx)
        out[j, 1] = c[j] * shift(gv, dy, dx)
    return out


def jacobian_adj(w: np.ndarray, c: np.ndarray, M: int) -> np.ndarray:
    """Adjoint J^T w = sum_j c_j [D_h^T S_{-s_j} w[j,0] + D_v^T S_{-s_j} w[j,1]]."""
    offs = patch_offsets(M)
    acc_h = np.zeros(w.shape[2:], dtype=np.float64)
    acc_v = np.zeros(w.shape[2:], dtype=np.float64)
    for j, (dy, dx) in enumerate(offs):
        acc_h += c[j] * shift(w[j, 0], -dy, -dx)
        acc_v += c[j] * shift(w[j, 1], -dy, -dx)
    return diff_h_adj(acc_h) + diff_v_adj(acc_v)


def gtg_apply(z: np.ndarray, c: np.ndarray, M: int) -> np.ndarray:
    """G^T G z = (3 I + J^T J) z for G = (I, J, I, I) stacked (eqs. (9), (11))."""
    return 3.0 * z + jacobian_adj(jacobian(z, c, M), c, M)


def gtg_symbol(H: int, W: int, c: np.ndarray, M: int) -> np.ndarray:
    """Eigenvalues of the circulant operator G^T G on an H x W grid.

    G^T G is shift-invariant (periodic differences and shifts), hence
    diagonalised by the 2-D DFT; its eigenvalues are the DFT of its impulse
    response (the z-update is a set of cyclic convolutions, Sec. 4).
    """
    delta = np.zeros((1, H, W))
    delta[0, 0, 0] = 1.0
    resp = gtg_apply(delta, c, M)[0]
    return np.fft.fft2(resp).real


def _dft_matrix(n: int) -> np.ndarray:
    k = np.arange(n)
    return np.exp(-2j * math.pi * np.outer(k, k) / n)


def solve_gtg(rhs: np.ndarray, c: np.ndarray, M: int, method: str = "fft") -> np.ndarray:
    """z-update, eq. (12): solve G^T G z = rhs for every class image.

    method="fft"   : diagonalise by numpy's FFT (pocketfft);
    method="dft"   : same diagonalisation with explicit O(n^2) DFT matrices;
    method="dense" : assemble the n x n matrix of G^T G column by column and
                     solve it with LAPACK (tiny grids only).
    """
    K, H, W = rhs.shape
    if method == "dense":
        n = H * W
        A = np.empty((n, n))
        for col in range(n):
            e = np.zeros((1, H, W))
            e.reshape(-1)[col] = 1.0
            A[:, col] = gtg_apply(e, c, M).reshape(-1)
        sol = np.linalg.solve(A, rhs.reshape(K, n).T).T
        return sol.reshape(K, H, W)
    sym = gtg_symbol(H, W, c, M)
    if method == "fft":
        return np.fft.ifft2(np.fft.fft2(rhs, axes=(-2, -1)) / sym, axes=(-2, -1)).real
    if method == "dft":
        FH, FW = _dft_matrix(H), _dft_matrix(W)
        spec = np.einsum("ab,kbc,cd->kad", FH, rhs.astype(np.complex128), FW)
        spec = spec / sym
        out = np.einsum("ab,kbc,cd->kad", FH.conj(), spec, FW.conj()) / (H * W)
        return out.real
    raise ValueError(method)


# ---------------------------------------------------------------------------
# Proximity operators of g1..g4 (eq. (10); Sec. 4 "Solving the iterative
# decoupled problem")
# ---------------------------------------------------------------------------

def prox_data(v: np.ndarray, p: np.ndarray, mu: float) -> np.ndarray:
    """prox of g1/mu at v, g1(xi) = sum_i -ln(p_i^T xi_i) (eq. (10)).

    Minimiser u of -ln(p^T u) + mu/2 ||u - v||^2 per pixel.  Stationarity gives
    u = v + p / (mu t) with t = p^T u, and t is the positive root of
    mu t^2 - mu (p^T v) t - ||p||^2 = 0 (the closed-form polynomial root).
    """
    s = np.sum(p * v, axis=0)
    q = np.sum(p * p, axis=0)
    disc = np.sqrt(s * s + 4.0 * q / mu)
    # positive root, written without cancellation for either sign of s
    t = np.where(s >= 0.0, 0.5 * (s + disc), (2.0 * q / mu) / np.where(s >= 0.0, 1.0, disc - s))
    return v + p / (mu * t)


def project_l1_ball(v: np.ndarray, radius) -> np.ndarray:
    """Euclidean projection of each row of v (>= 0) onto {x : ||x||_1 <= radius} (sort-based)."""
    v = np.asarray(v, dtype=np.float64)
    radius = np.broadcast_to(np.asarray(radius, dtype=np.float64), v.shape[:-1])
    out = v.copy()
    inside = v.sum(axis=-1) <= radius
    u = -np.sort(-v, axis=-1)
    css = np.cumsum(u, axis=-1)
    idx = np.arange(1, v.shape[-1] + 1)
    cond = u - (css - radius[..., None]) / idx > 0
    rho = np.max(np.where(cond, idx, 0), axis=-1)
    rho = np.maximum(rho, 1)
    theta = (np.take_along_axis(css, (rho - 1)[..., None], axis=-1)[..., 0] - radius) / rho
    proj = np.maximum(v - theta[..., None], 0.0)
    return np.where(inside[..., None], out, proj)


def project_lq_ball(w: np.ndarray, q: float, iters: int = 100) -> np.ndarray:
    """Euclidean projection of each row of w (>= 0) onto the unit l_q ball, 1 < q < inf.

    Outside the ball the projection y satisfies the optimality conditions
    y_i - w_i + nu q y_i^{q-1} = 0 with sum_i y_i^q = 1 for some nu > 0.  For a
    given nu each y_i is the root of a function increasing on [0, w_i] (inner
    bisection), and sum_i y_i(nu)^q decreases in nu (outer bisection).
    """
    w = np.asarray(w, dtype=np.float64)
    inside = np.sum(w ** q, axis=-1) <= 1.0

    def y_of(nu):
        lo = np.zeros_like(w)
        hi = w.copy()
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            up = mid + nu[..., None] * q * mid ** (q - 1.0) > w
            hi = np.where(up, mid, hi)
            lo = np.where(up, lo, mid)
        return 0.5 * (lo + hi)

    nlo = np.zeros(w.shape[:-1])
    nhi = np.ones(w.shape[:-1])
    for _ in range(200):   # grow the upper end until sum y^q <= 1
        big = np.sum(y_of(nhi) ** q, axis=-1) > 1.0
        if not np.any(big & ~inside):
            break
        nhi = np.where(big, 2.0 * nhi, nhi)
    for _ in range(iters):
        mid = 0.5 * (nlo + nhi)
        big = np.sum(y_of(mid) ** q, axis=-1) > 1.0
        nlo = np.where(big, mid, nlo)
        nhi = np.where(big, nhi, mid)
    y = y_of(0.5 * (nlo + nhi))
    return np.where(inside[..., None], w, y)


def schatten_shrink(sig: np.ndarray, tau: float, p: float) -> np.ndarray:
    """Singular values of prox_{tau ||.||_{S_p}}: prox of tau ||.||_p on the singular values.

    p = 1: soft threshold (Sec. 4, the paper's choice); p = 2: group shrink of
    the vector; p = inf: sigma minus its projection on the l1 ball of radius tau;
    other p > 1 (the general Schatten norm of Sec. 3): sigma minus tau times the
    projection of sigma / tau on the unit l_q ball, 1/p + 1/q = 1 (Moreau
    decomposition; l_q is the dual norm of l_p).
    """
    sig = np.asarray(sig, dtype=np.float64)
    if p == 1.0:
        return np.maximum(sig - tau, 0.0)
    if p == 2.0:
        nrm = np.sqrt(np.sum(sig * sig, axis=-1, keepdims=True))
        fac = np.where(nrm > tau, 1.0 - tau / np.where(nrm > 0, nrm, 1.0), 0.0)
        return sig * fac
    if math.isinf(p):
        return sig - project_l1_ball(sig, tau)
    if p > 1.0:
        if tau <= 0.0:
            return sig.copy()
        q = p / (p - 1.0)
        return np.maximum(sig - tau * project_lq_ball(sig / tau, q), 0.0)
    raise ValueError("schatten p must be >= 1")


def _blocks(Y: np.ndarray) -> np.ndarray:
    """[L][2][K][H][W] -> per-pixel (LK) x 2 matrices, shape (n, LK, 2)."""
    L, _, K, H, W = Y.shape
    return Y.transpose(3, 4, 0, 2, 1).reshape(H * W, L * K, 2)


def _unblocks(B: np.ndarray, shape) -> np.ndarray:
    L, _, K, H, W = shape
    return B.reshape(H, W, L, K, 2).transpose(2, 4, 3, 0, 1)


def prox_schatten_svd(Y: np.ndarray, tau: float, p: float) -> np.ndarray:
    """prox of tau ||.||_{S_p} applied per pixel to the (LK)x2 block, by LAPACK SVD.

    The definition: shrink the singular values of [Y]_i and rebuild
    U diag(shrunk) V^T (Sec. 4, MPO of g2).
    """
    B = _blocks(Y)
    U, S, Vt = np.linalg.svd(B, full_matrices=False)
    Sh = schatten_shrink(S, tau, p)
    out = np.einsum("nij,nj,njk->nik", U, Sh, Vt)
    return _unblocks(out, Y.shape)


def prox_schatten(Y: np.ndarray, tau: float, p: float) -> np.ndarray:
    """prox of tau ||.||_{S_p} per pixel through the 2x2 structure tensor (Sec. 3, eq. (5)).

    The eigenvalues of [Y]_i^T [Y]_i are the squared singular values of [Y]_i
    and its eigenvectors are the right singular vectors V, so the proximal
    point is [Y]_i V diag(shrunk / sigma) V^T (multiplier 0 where the shrunk
    value is 0).  Eigen-decomposition by LAPACK (numpy.linalg.eigh).
    """
    L, _, K, H, W = Y.shape
    Yh = Y[:, 0].reshape(L * K, H * W)
    Yv = Y[:, 1].reshape(L * K, H * W)
    S = np.empty((H * W, 2, 2))
    S[:, 0, 0] = np.sum(Yh * Yh, axis=0)
    S[:, 0, 1] = S[:, 1, 0] = np.sum(Yh * Yv, axis=0)
    S[:, 1, 1] = np.sum(Yv * Yv, axis=0)
    lam, V = np.linalg.eigh(S)
    sig = np.sqrt(np.maximum(lam, 0.0))
    sh = schatten_shrink(sig, tau, p)
    rho = np.where(sh > 0.0, sh / np.where(sig > 0.0, sig, 1.0), 0.0)
    N = np.einsum("nij,nj,nkj->nik", V, rho, V)
    uh = Yh * N[:, 0, 0] + Yv * N[:, 1, 0]
    uv = Yh * N[:, 0, 1] + Yv * N[:, 1, 1]
    out = np.empty_like(Y)
    out[:, 0] = uh.reshape(L, K, H, W)
    out[:, 1] = uv.reshape(L, K, H, W)
    return out


def prox_positive(v: np.ndarray) -> np.ndarray:
    """prox of g3 = i_+ : projection onto the positive orthant (Sec. 4)."""
    return np.maximum(v, 0.0)


def prox_sum_to_one(v: np.ndarray) -> np.ndarray:
    """prox of g4 = i_1(1_K^T xi): projection onto {1_K^T xi_i = 1} per pixel (eq. (10))."""
    K = v.shape[0]
    return v - (np.sum(v, axis=0, keepdims=True) - 1.0) / K


# ---------------------------------------------------------------------------
# SALSA iteration (eqs. (12)-(14))
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    """Parameters of eq. (7) and of SALSA: multipliers c_j (L values), radius M, p, lambda, mu.

    g4 selects the reading of the fourth split (eq. (10) vs the text of Sec. 4):
    "affine" = projection onto {1^T xi = 1} (the definition), "simplex" = projection
    onto the probability simplex (the text's wording).
    """

    c: np.ndarray
    M: int
    p: float
    lam: float
    mu: float
    g4: str = "affine"


@dataclass
class State:
    """ADMM state: hidden field z and scaled multipliers d1..d4 (u is eliminated)."""

    z: np.ndarray
    d1: np.ndarray
    d2: np.ndarray
    d3: np.ndarray
    d4: np.ndarray

    def copy(self) -> "State":
        return State(self.z.copy(), self.d1.copy(), self.d2.copy(), self.d3.copy(), self.d4.copy())


def normalize_input(x: np.ndarray, is_logits: bool) -> np.ndarray:
    """Class probabilities p_i from the input: softmax of logits, or p_i / 1^T p_i."""
    x = np.asarray(x, dtype=np.float64)
    if is_logits:
        e = np.exp(x - x.max(axis=0, keepdims=True))
        return e / e.sum(axis=0, keepdims=True)
    s = x.sum(axis=0, keepdims=True)
    if np.any(~np.isfinite(x)) or np.any(x < 0) or np.any(s <= 0):
        raise ValueError("probabilities must be finite, >= 0 and have a positive sum per pixel")
    return x / s


def init_state(phat: np.ndarray, L: int) -> State:
    """Initial state: z = p_hat, all multipliers 0 (initialisation reading; u^0 = G z^0)."""
    K, H, W = phat.shape
    z = phat.copy()
    return State(z, np.zeros_like(z), np.zeros((L, 2, K, H, W)), np.zeros_like(z), np.zeros_like(z))


def salsa_round(st: State, phat: np.ndarray, pr: Problem, solve_method: str = "fft",
                prox2: str = "eigh", want_residuals: bool = False):
    """One round: u-update (eq. (13)), d-update (eq. (14)), z-update (eq. (12)).

    u_j = prox_{g_j/mu}(H_j z - d_j), d_j <- u_j - (H_j z - d_j), then
    z <- (G^T G)^{-1} G^T (u + d).  Returns the new state (and residuals if asked).
    """
    tau = pr.lam / pr.mu
    z = st.z
    v1 = z - st.d1
    u1 = prox_data(v1, phat, pr.mu)
    d1 = u1 - v1
    v2 = jacobian(z, pr.c, pr.M) - st.d2
    u2 = (prox_schatten if prox2 == "eigh" else prox_schatten_svd)(v2, tau, pr.p)
    d2 = u2 - v2
    v3 = z - st.d3
    u3 = prox_positive(v3)
    d3 = u3 - v3
    v4 = z - st.d4
    u4 = prox_sum_to_one(v4) if pr.g4 == "affine" else project_simplex(v4)
    d4 = u4 - v4
    rhs = (u1 + d1) + jacobian_adj(u2 + d2, pr.c, pr.M) + (u3 + d3) + (u4 + d4)
    znew = solve_gtg(rhs, pr.c, pr.M, method=solve_method)
    new = State(znew, d1, d2, d3, d4)
    if not want_residuals:
        return new
    # primal residual G z - u = d_old - d_new (eq. (14)); dual residual mu ||G (z_new - z)||
    rp2 = sum(float(np.sum((a - b) ** 2)) for a, b in
              ((d1, st.d1), (d2, st.d2), (d3, st.d3), (d4, st.d4)))
    dz = znew - z
    rd2 = float(np.sum(dz * gtg_apply(dz, pr.c, pr.M)))
    return new, math.sqrt(rp2), pr.mu * math.sqrt(max(rd2, 0.0))


def solve(x: np.ndarray, pr: Problem, iters: int, is_logits: bool = False, solve_method: str = "fft",
          prox2: str = "eigh", return_state: bool = False):
    """z after `iters` rounds from the initial state (the paper's z^{iters+1})."""
    phat = normalize_input(x, is_logits)
    st = init_state(phat, (2 * pr.M + 1) ** 2)
    for _ in range(iters):
        st = salsa_round(st, phat, pr, solve_method=solve_method, prox2=prox2)
    return (st, phat) if return_state else st.z


def labels(z: np.ndarray) -> np.ndarray:
    """Segmentation y_i = argmax_k z_ki, lowest k on ties (Fig. 1 readout)."""
    return np.argmax(z, axis=0).astype(np.int32)


def project_simplex(z: np.ndarray) -> np.ndarray:
    """Euclidean projection of each z_i onto the probability simplex (sort-based)."""
    K = z.shape[0]
    v = np.moveaxis(z, 0, -1)
    u = -np.sort(-v, axis=-1)
    css = np.cumsum(u, axis=-1)
    idx = np.arange(1, K + 1)
    cond = u - (css - 1.0) / idx > 0
    rho = np.max(np.where(cond, idx, 0), axis=-1)
    theta = (np.take_along_axis(css, (rho - 1)[..., None], axis=-1)[..., 0] - 1.0) / rho
    return np.moveaxis(np.maximum(v - theta[..., None], 0.0), -1, 0)


def schatten_norms(z: np.ndarray, pr: Problem) -> np.ndarray:
    """||[J z]_i||_{S_p} per pixel (eq. (6)), singular values by LAPACK SVD."""
    S = np.linalg.svd(_blocks(jacobian(z, pr.c, pr.M)), compute_uv=False)
    if pr.p == 1.0:
        return S.sum(axis=-1)
    if pr.p == 2.0:
        return np.sqrt(np.sum(S * S, axis=-1))
    if math.isinf(pr.p):
        return S.max(axis=-1)
    return np.sum(S ** pr.p, axis=-1) ** (1.0 / pr.p)


def objective(z: np.ndarray, phat: np.ndarray, pr: Problem, project: bool = True) -> float:
    """Objective of eq. (7) at z (by default at its projection onto the feasible set)."""
    zz = project_simplex(z) if project else z
    data = -np.sum(np.log(np.sum(phat * zz, axis=0)))
    return float(data + pr.lam * np.sum(schatten_norms(zz, pr)))
