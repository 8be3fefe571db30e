"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/segsalsa.h declares, and rejects invalid arguments
with the documented status before anything is enqueued."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "segsalsa.h")

OK, INVALID, UNSUPPORTED, WORKSPACE = 0, 1, 2, 3


@pytest.fixture(scope="module")
def S():
    from paper_1504_07028_amd import segsalsa
    if not os.path.exists(segsalsa.LIB_PATH):
        from paper_1504_07028_amd.build import build
        build()
    segsalsa.lib()
    return segsalsa


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(segsalsa_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(S):
    names = declared_functions()
    assert "segsalsa_str_solve" in names and len(names) >= 8
    lib = ctypes.CDLL(S.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def base_problem(S, **kw):
    args = dict(K=4, H=16, W=20, patch_radius=1, patch_weights=[1.0] * 9, schatten_p=1.0, lam=1.0, mu=1.0, iters=5)
    args.update(kw)
    return S.Problem(**args)


def status_of_size(S, pr, prec=0):
    n = ctypes.c_size_t(0)
    s = pr.c_struct()
    return S.lib().segsalsa_str_workspace_size(ctypes.byref(s), prec, ctypes.byref(n)), n.value


def test_workspace_size_grows_with_problem(S):
    st, small = status_of_size(S, base_problem(S))
    assert st == OK and small > 0
    st, big = status_of_size(S, base_problem(S, H=64, W=64))
    assert st == OK and big > small
    st, f64 = status_of_size(S, base_problem(S), prec=1)
    assert st == OK and f64 > small


@pytest.mark.parametrize("kw,code", [
    (dict(K=1), INVALID), (dict(K=65), UNSUPPORTED), (dict(H=0), INVALID), (dict(W=-3), INVALID),
    (dict(H=1, W=1), INVALID), (dict(H=5000), UNSUPPORTED), (dict(patch_radius=-1), INVALID),
    (dict(patch_radius=6, patch_weights=[1.0] * 169), UNSUPPORTED),
    (dict(patch_weights=[1.0] * 8 + [math.nan]), INVALID), (dict(schatten_p=1.5), OK), (dict(schatten_p=7.25), OK),
    (dict(schatten_p=math.nan), INVALID), (dict(schatten_p=0.5), INVALID), (dict(schatten_p=-math.inf), INVALID),
    (dict(lam=-1.0), INVALID),
    (dict(lam=math.inf), INVALID), (dict(mu=0.0), INVALID), (dict(mu=-2.0), INVALID), (dict(iters=-1), INVALID),
    (dict(tol=1e-3), INVALID), (dict(tol=-1.0), INVALID), (dict(residual_every=-1), INVALID),
])
def test_invalid_problems(S, kw, code):
    st, _ = status_of_size(S, base_problem(S, **kw))
    assert st == code
    assert (S.lib().segsalsa_last_error().decode() != "") == (code != OK)


def test_bad_precision_and_null_problem(S):
    n = ctypes.c_size_t(0)
    assert S.lib().segsalsa_str_workspace_size(None, 0, ctypes.byref(n)) == INVALID
    s = base_problem(S).c_struct()
    assert S.lib().segsalsa_str_workspace_size(ctypes.byref(s), 7, ctypes.byref(n)) == INVALID


def call_solve(S, pr, inp, z, ws, wsb, prec=0, stats=None):
    s = pr.c_struct()
    return S.lib().segsalsa_str_solve(ctypes.byref(s), prec, ctypes.c_void_p(inp), ctypes.c_void_p(z),
                                      ctypes.c_void_p(ws), wsb, stats, None)


def test_solve_argument_errors_before_launch(S):
    """Errors detected on the host; the fake device addresses are never dereferenced."""
    pr = base_problem(S)
    _, need = status_of_size(S, pr)
    fake_in, fake_z, fake_ws = 0x100000, 0x200000, 0x300000
    assert call_solve(S, pr, fake_in, None, fake_ws, need) == INVALID           # z_out NULL
    assert call_solve(S, pr, None, fake_z, fake_ws, need) == INVALID            # input NULL
    assert call_solve(S, pr, fake_in, fake_in, fake_ws, need) == INVALID        # aliasing
    assert call_solve(S, pr, fake_in + 2, fake_z, fake_ws, need) == INVALID     # misaligned
    assert call_solve(S, pr, fake_in, fake_z, None, need) == WORKSPACE          # no workspace
    assert call_solve(S, pr, fake_in, fake_z, fake_ws + 8, need) == WORKSPACE   # misaligned workspace
    assert call_solve(S, pr, fake_in, fake_z, fake_ws, need - 1) == WORKSPACE   # too small
    pr_res = base_problem(S, residual_every=5)
    assert call_solve(S, pr_res, fake_in, fake_z, fake_ws, need) == INVALID     # residuals need stats
    assert call_solve(S, base_problem(S, K=1), fake_in, fake_z, fake_ws, need) == INVALID


def test_labels_and_state_argument_errors(S):
    L = S.lib()
    assert L.segsalsa_str_labels(0, 4, 4, 0, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), None) == INVALID
    assert L.segsalsa_str_labels(3, 4, 4, 0, None, ctypes.c_void_p(0x2000), None) == INVALID
    pr = base_problem(S)
    s = pr.c_struct()
    _, need = status_of_size(S, pr)
    assert L.segsalsa_str_state_export(ctypes.byref(s), 0, None, need, None, None, None, None, None) == WORKSPACE
    assert L.segsalsa_str_state_import(ctypes.byref(s), 0, ctypes.c_void_p(0x300000), need, None, None, None, None,
                                       None, None) == INVALID


def test_status_strings(S):
    L = S.lib()
    assert L.segsalsa_status_string(0) == b"SEGSALSA_OK"
    assert L.segsalsa_status_string(3) == b"SEGSALSA_ERR_WORKSPACE"


def test_binding_rejects_host_tensors(S):
    import torch
    pr = base_problem(S)
    x = torch.zeros(4, 16, 20, dtype=torch.float32)
    with pytest.raises(TypeError):
        S.segsalsa_str_solve(pr, x, x.clone(), torch.zeros(10, dtype=torch.uint8))


def test_gpus_flag_rejected():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def grad_size(S, pr, ck, prec=1):
    n = ctypes.c_size_t(0)
    s = pr.c_struct()
    return S.lib().segsalsa_str_grad_workspace_size(ctypes.byref(s), prec, ck, ctypes.byref(n)), n.value


def test_grad_workspace_size_and_restrictions(S):
    st, base = grad_size(S, base_problem(S, iters=20), 10)
    assert st == OK and base > status_of_size(S, base_problem(S, iters=20), 1)[1]
    # states kept: ceil(20 / S) checkpoints + S - 1 segment slots: 20 (S = 1), 11 (S = 10), 8 (S = 5)
    assert grad_size(S, base_problem(S, iters=20), 1)[1] > base
    assert grad_size(S, base_problem(S, iters=20), 5)[1] < base
    assert grad_size(S, base_problem(S, iters=0), 10)[0] == OK
    assert grad_size(S, base_problem(S), -1)[0] == INVALID
    assert grad_size(S, base_problem(S, iters=20), 0) == grad_size(S, base_problem(S, iters=20), 1)   # auto: all
    assert grad_size(S, base_problem(S, residual_every=2), 5)[0] == UNSUPPORTED
    assert grad_size(S, base_problem(S, residual_every=2, tol=1e-3), 5)[0] == UNSUPPORTED
    assert grad_size(S, base_problem(S, warm_start=True), 5)[0] == UNSUPPORTED
    assert grad_size(S, base_problem(S, use_graph=True), 5)[0] == UNSUPPORTED
    assert grad_size(S, base_problem(S, K=1), 5)[0] == INVALID


def test_grad_argument_errors_before_launch(S):
    """Host-side checks of the differentiable entry points; fake addresses are never dereferenced."""
    L = S.lib()
    pr = base_problem(S)
    st, need = grad_size(S, pr, 2)
    assert st == OK
    s = pr.c_struct()
    V = ctypes.c_void_p
    fin, fz, fg, fgi, fws = 0x100000, 0x200000, 0x300000, 0x400000, 0x500000

    def ckpt(inp, z, ws, nbytes):
        return L.segsalsa_str_solve_ckpt(ctypes.byref(s), 1, 2, V(inp), V(z), V(ws), nbytes, None)

    def bwd(inp, gz, gi, gl, gw, ws, nbytes, ck=2):
        return L.segsalsa_str_backward(ctypes.byref(s), 1, ck, V(inp), V(gz), V(gi), V(gl), V(gw), V(ws), nbytes,
                                       None)

    assert ckpt(None, fz, fws, need) == INVALID
    assert ckpt(fin, None, fws, need) == INVALID
    assert ckpt(fin, fin, fws, need) == INVALID
    assert ckpt(fin + 4, fz, fws, need) == INVALID
    assert ckpt(fin, fz, fws, need - 1) == WORKSPACE
    assert ckpt(fin, fz, None, need) == WORKSPACE
    assert bwd(None, fg, fgi, None, None, fws, need) == INVALID
    assert bwd(fin, None, fgi, None, None, fws, need) == INVALID
    assert bwd(fin, fg, None, None, None, fws, need) == INVALID
    assert bwd(fin, fg, fg, None, None, fws, need) == INVALID          # grad_input aliases grad_z
    assert bwd(fin, fg, fgi, 0x600004, None, fws, need) == INVALID     # misaligned grad_lambda
    assert bwd(fin, fg, fgi, None, None, fws, need - 1) == WORKSPACE
    assert bwd(fin, fg, fgi, None, None, fws, need, ck=-1) == INVALID


def test_checkpoint_interval(S):
    """checkpoint_every = 0 keeps every state while they fit in 8 GiB, else the smallest interval that fits
    (ceil(N / S) checkpoints plus S - 1 recomputed states), else ceil(sqrt(N)); other values are clamped to
    [1, iters]."""
    pr = base_problem(S)
    assert S.segsalsa_str_grad_checkpoint_interval(pr, 1, 0) == 1
    assert S.segsalsa_str_grad_checkpoint_interval(pr, 1, 2) == 2
    assert S.segsalsa_str_grad_checkpoint_interval(pr, 1, 10 ** 6) == max(1, pr.iters)
    # 2048 x 2048, K = 16, 5x5 patch, FP32: one state is (4 + 2L) K n words = 54 * 16 * 4 Mi * 4 B = 13.5 GiB,
    # more than the budget even alone, so ceil(sqrt(500)) = 23
    big = S.Problem(16, 2048, 2048, 2, [0.2] * 25, 1.0, 1.0, 1.0, 500)
    assert S.segsalsa_str_grad_checkpoint_interval(big, 0, 0) == 23
    # 256 x 256, K = 8, 3x3, FP32, 50 rounds: 46 MB a state, all 51 fit
    mid = S.Problem(8, 256, 256, 1, [1.0 / 3] * 9, 1.0, 1.0, 1.0, 50)
    assert S.segsalsa_str_grad_checkpoint_interval(mid, 0, 0) == 1
    # 1024 x 1024, K = 16, 3x3, FP32, 200 rounds: 1.4 GiB a state; 8 GiB holds 5 of them, and
    # ceil(200 / S) + S - 1 <= 5 has no solution, so ceil(sqrt(200)) = 15
    lg = S.Problem(16, 1024, 1024, 1, [1.0 / 3] * 9, 1.0, 1.0, 1.0, 200)
    assert S.segsalsa_str_grad_checkpoint_interval(lg, 0, 0) == 15
    with pytest.raises(RuntimeError):
        S.segsalsa_str_grad_checkpoint_interval(pr, 1, -1)


def test_g4_simplex_flag(S):
    assert status_of_size(S, base_problem(S, g4_simplex=True))[0] == OK
    pr = base_problem(S)
    s = pr.c_struct()
    s.g4_simplex = 2
    n = ctypes.c_size_t(0)
    assert S.lib().segsalsa_str_workspace_size(ctypes.byref(s), 0, ctypes.byref(n)) == INVALID
    assert grad_size(S, base_problem(S, g4_simplex=True), 5)[0] == UNSUPPORTED
    assert grad_size(S, base_problem(S, schatten_p=3.0), 5)[0] == UNSUPPORTED


def test_shapes_beyond_one_workgroup_are_unsupported(S):
    """Large K with a large patch needs more registers than one workgroup holds (documented envelope)."""
    st, _ = status_of_size(S, base_problem(S, K=64, H=20, W=20, patch_radius=5, patch_weights=[1.0] * 121))
    assert st == UNSUPPORTED
    assert status_of_size(S, base_problem(S, K=64, H=20, W=20))[0] == OK            # FP32, 3x3
    assert status_of_size(S, base_problem(S, K=64, H=20, W=20), prec=1)[0] == UNSUPPORTED
    assert status_of_size(S, base_problem(S, K=32, H=20, W=20), prec=1)[0] == OK
    pw25 = dict(patch_radius=2, patch_weights=[1.0] * 25)
    assert status_of_size(S, base_problem(S, K=32, H=20, W=20, **pw25))[0] == OK
    assert status_of_size(S, base_problem(S, K=33, H=20, W=20, **pw25))[0] == UNSUPPORTED
    assert status_of_size(S, base_problem(S, K=16, H=20, W=20, **pw25), prec=1)[0] == OK
    assert status_of_size(S, base_problem(S, K=17, H=20, W=20, **pw25), prec=1)[0] == UNSUPPORTED


# ---------------------------------------------------------------------------
# Tuning table and cache (host side)
# ---------------------------------------------------------------------------

@pytest.fixture()
def clean_table(S):
    S.segsalsa_tuning_clear()
    yield S
    S.segsalsa_tuning_clear()
    if os.path.exists(S.DEFAULT_TUNING_CACHE):
        S.segsalsa_tuning_load(S.DEFAULT_TUNING_CACHE)


def test_tuning_set_get_and_workspace(clean_table):
    S = clean_table
    K, H, W, M = 4, 40, 60, 1
    plan, tuned = S.segsalsa_tuning_get(K, H, W, M, 0)
    assert not tuned and plan["tile_rows"] > 0 and plan["row_threads"] % 64 == 0
    st, before = status_of_size(S, base_problem(S, K=K, H=H, W=W))
    assert st == OK
    want = dict(tile_rows=4, tile_cols=20, classes_per_wave=2, prefetch=1, generic_fft=0, col_dft=0, rows_per_block=3,
                row_threads=128, cols_per_block=4, col_threads=192, us_per_round=12.5)
    S.segsalsa_tuning_set(K, H, W, M, 0, want)
    got, tuned = S.segsalsa_tuning_get(K, H, W, M, 0)
    assert tuned and got == want
    # the tile grid changed, so the workspace did too; FP64 of the same shape is untouched
    st, after = status_of_size(S, base_problem(S, K=K, H=H, W=W))
    assert st == OK and after != before
    assert not S.segsalsa_tuning_get(K, H, W, M, 1)[1]
    S.segsalsa_tuning_set(K, H, W, M, 0, None)
    assert not S.segsalsa_tuning_get(K, H, W, M, 0)[1]


@pytest.mark.parametrize("bad,code", [
    (dict(tile_rows=4), INVALID),                         # one side only
    (dict(classes_per_wave=3), INVALID),
    (dict(row_threads=100), INVALID),                     # not a multiple of 64
    (dict(col_threads=2048), INVALID),
    (dict(tile_rows=40, tile_cols=60, classes_per_wave=1), UNSUPPORTED),   # grown tile beyond LDS
    (dict(rows_per_block=40, row_threads=64), UNSUPPORTED),               # 40 x 60 elements > 16 per thread
    (dict(prefetch=2), INVALID),
    (dict(prefetch=1, classes_per_wave=1), UNSUPPORTED),                  # prefetching build: 2 classes per wave
    (dict(col_dft=2), INVALID),
    (dict(cols_per_block=64, col_threads=64), UNSUPPORTED),               # 64 columns x 2 chunks of 32 rows
    (dict(col_dft=1, cols_per_block=32, col_threads=64), UNSUPPORTED),    # the DFT pass: 32 x 40 elements > 16 each
])
def test_tuning_rejects_entries_that_do_not_fit(clean_table, bad, code):
    S = clean_table
    with pytest.raises(S.SegsalsaError) as e:
        S.segsalsa_tuning_set(16, 40, 60, 2, 0, bad)
    assert e.value.status == code
    assert not S.segsalsa_tuning_get(16, 40, 60, 2, 0)[1]


def test_tile_positions_beyond_256_are_encoded(clean_table):
    """A grown tile wider than 256 columns (fold-list positions above 255) is a valid tuned shape."""
    S = clean_table
    S.segsalsa_tuning_set(2, 8, 300, 0, 0, dict(tile_rows=2, tile_cols=300))
    got, tuned = S.segsalsa_tuning_get(2, 8, 300, 0, 0)
    assert tuned and got["tile_cols"] == 300


def test_tuning_cache_round_trip(clean_table, tmp_path):
    S = clean_table
    S.segsalsa_tuning_set(9, 61, 34, 2, 0, dict(tile_rows=8, tile_cols=17, classes_per_wave=1))
    S.segsalsa_tuning_set(16, 145, 145, 2, 1, dict(rows_per_block=2, row_threads=128, us_per_round=99.0))
    path = tmp_path / "cache.json"
    S.segsalsa_tuning_save(str(path))
    text = path.read_text()
    assert '"segsalsa-tuning-1"' in text and '"precision": "fp64"' in text
    S.segsalsa_tuning_clear()
    assert not S.segsalsa_tuning_get(9, 61, 34, 2, 0)[1]
    # one extra entry that does not fit is skipped, the others are read
    text = text.replace("\n  ]", ',\n    {"K": 16, "H": 40, "W": 60, "M": 2, "precision": "fp32", "tile_rows": 40, '
                                 '"tile_cols": 60, "classes_per_wave": 1, "rows_per_block": 0, "row_threads": 0, '
                                 '"cols_per_block": 0, "col_threads": 0}\n  ]')
    path.write_text(text)
    assert S.segsalsa_tuning_load(str(path)) == (2, 1)
    got, tuned = S.segsalsa_tuning_get(9, 61, 34, 2, 0)
    assert tuned and (got["tile_rows"], got["tile_cols"], got["classes_per_wave"]) == (8, 17, 1)
    got, tuned = S.segsalsa_tuning_get(16, 145, 145, 2, 1)
    assert tuned and got["rows_per_block"] == 2 and got["row_threads"] == 128 and got["us_per_round"] == 99.0
    with pytest.raises(S.SegsalsaError):
        S.segsalsa_tuning_load(str(tmp_path / "missing.json"))


def test_shipped_cache_is_read(S):
    """The cache shipped with the package loads without skipped entries, and its shapes plan as tuned."""
    if not os.path.exists(S.DEFAULT_TUNING_CACHE):
        pytest.skip("no tuning cache shipped")
    import json
    S.segsalsa_tuning_clear()
    loaded, skipped = S.segsalsa_tuning_load(S.DEFAULT_TUNING_CACHE)
    entries = json.load(open(S.DEFAULT_TUNING_CACHE))["entries"]
    assert loaded == len(entries) and skipped == 0
    for e in entries:
        got, tuned = S.segsalsa_tuning_get(e["K"], e["H"], e["W"], e["M"], 1 if e["precision"] == "fp64" else 0)
        assert tuned
        # fields the entry leaves at 0 (threads of the power-of-two FFT kernels) are filled in by the planner
        for f in S.TUNING_FIELDS[:-1]:
            assert e.get(f, 0) == 0 or got[f] == e[f], (e, f, got[f])


def test_autotune_argument_errors(S):
    pr = base_problem(S)
    s = pr.c_struct()
    n = ctypes.c_size_t(0)
    assert S.lib().segsalsa_str_autotune_workspace_size(ctypes.byref(s), 0, ctypes.byref(n)) == OK
    st, plain = status_of_size(S, pr)
    assert n.value >= plain
    t = S.segsalsa_tuning()
    dummy = ctypes.c_void_p(256)
    assert S.lib().segsalsa_str_autotune(ctypes.byref(s), 0, dummy, dummy, dummy, n.value, 5, ctypes.byref(t),
                                         None) == INVALID          # z_scratch aliases input
    assert S.lib().segsalsa_str_autotune(ctypes.byref(s), 0, dummy, ctypes.c_void_p(512), dummy, n.value, 0,
                                         ctypes.byref(t), None) == INVALID   # rounds out of range


def test_prefetch_entries_only_where_built(clean_table):
    S = clean_table
    S.segsalsa_tuning_set(16, 40, 60, 2, 0, dict(classes_per_wave=2, prefetch=1))
    got, tuned = S.segsalsa_tuning_get(16, 40, 60, 2, 0)
    assert tuned and got["prefetch"] == 1 and got["classes_per_wave"] == 2
    for prec, M in ((1, 2), (0, 3)):      # FP64, or a 7x7 patch: not built
        with pytest.raises(S.SegsalsaError) as e:
            S.segsalsa_tuning_set(16, 40, 60, M, prec, dict(classes_per_wave=2, prefetch=1))
        assert e.value.status == UNSUPPORTED


def test_fp32_column_pass_follows_the_weights(S):
    """The column recursions' FP32 rounding grows like eps / (1 - rho) at the largest rho (kx = 0), so
    FP32 solves whose weights put rho within 0.1 of 1 (Wsum above ~280) plan the DFT column pass; FP64
    keeps the recursions at any weights."""
    imgs, _ = S.image_table([(4, 96, 128)], [1.0], [1.0])
    for scale, prec, want in ((1.0, 0, 0), (250.0 ** 0.5, 0, 0), (300.0 ** 0.5, 0, 1), (100.0, 0, 1), (100.0, 1, 0)):
        params = S.BatchParams(1, [scale / 3] * 9, 1.0, 10)   # Wsum = scale ** 2
        (plan,) = S.segsalsa_str_batch_plans(imgs, params, prec)
        assert plan["col_dft"] == want, (scale, prec, plan)


def test_batch_plans_depend_on_transform_length_only(S):
    """In a batch of several images the FFT blocking is a function of the transform length, so images
    of one length share a launch: equal column lengths (211 and 227 both take Bluestein over 512
    points; 96 and 300 take the general kernels) and equal row kinds get equal thread counts."""
    shapes = [(4, 211, 300), (8, 227, 301), (9, 96, 227), (16, 300, 96)]   # (K, H, W)
    imgs, _ = S.image_table(shapes, [1.0] * 4, [1.0] * 4)
    params = S.BatchParams(1, [1.0 / 3] * 9, 1.0, 10)
    plans = S.segsalsa_str_batch_plans(imgs, params, 0)
    assert len(plans) == 4 and all(p["tile_rows"] > 0 and p["tile_cols"] > 0 for p in plans)
    assert plans[0]["col_threads"] == plans[1]["col_threads"] == 16 * 32      # 16 columns of 512 / 16 threads
    assert plans[2]["col_threads"] == plans[3]["col_threads"] == 512         # general kernels: 4096 elements / 8
    assert plans[0]["row_threads"] == plans[1]["row_threads"] == 256          # general rows: 2048 elements / 8
    assert plans[2]["row_threads"] == 8 * 32                                  # 227 -> Bluestein over 512
    # a single image of one of these shapes is planned on its own work instead
    single, _ = S.segsalsa_tuning_get(4, 211, 300, 1, 0)
    assert single["tile_rows"] == plans[0]["tile_rows"] and single["tile_cols"] == plans[0]["tile_cols"]


def test_planner_prefers_vector_fold_tiles(clean_table):
    """Among tile shapes of equal cost the planner takes one whose tile columns the vector fold handles
    (every tile column W / ntc wide, a multiple of 16 bytes of elements, at least 2M + 2): the 2048x2048
    workload, the 256x256 one and a 40x60 image, both precisions."""
    S = clean_table

    def vector_fold_fits(W, M, tile_cols, vec):
        ntc = -(-W // min(tile_cols, W))
        tc = -(-W // ntc)
        return W % ntc == 0 and tc % vec == 0 and tc >= 2 * M + 2

    for K, H, W, M in ((16, 2048, 2048, 2), (8, 256, 256, 1), (4, 40, 60, 1)):
        for prec, vec in ((0, 4), (1, 2)):
            plan, tuned = S.segsalsa_tuning_get(K, H, W, M, prec)
            assert not tuned and vector_fold_fits(W, M, plan["tile_cols"], vec), (K, H, W, M, prec, plan)


def test_stream_copy_rejects_bad_buffers_on_the_host(S):
    """The streaming copy checks its buffers before launching anything: NULL, misaligned, a size that is not
    a multiple of 16 bytes, or overlapping ranges give INVALID_ARG; zero bytes is a no-op."""
    lib = S.lib()
    assert lib.segsalsa_stream_copy(None, None, 0, None) == 0
    for src, dst, n in ((None, 4096, 64), (4096, None, 64), (4096 + 8, 1 << 20, 64), (4096, (1 << 20) + 4, 64),
                        (4096, 1 << 20, 60), (4096, 4096 + 32, 64)):
        assert lib.segsalsa_stream_copy(src, dst, n, None) == 1, (src, dst, n)   # INVALID_ARG
