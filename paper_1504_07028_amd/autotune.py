"""Measure launch shapes on the device and write the tuning cache.

For each image shape (K, H, W, patch radius) and precision, runs
segsalsa_str_autotune (the search itself is in the library: prox tile and
classes per wavefront by whole rounds, then the row and column FFT blocking
by the time of their passes) and saves the table as JSON.  The binding loads
the cache shipped with the package when the library is first loaded.

Usage:
  python -m paper_1504_07028_amd.autotune --shape 16,2048,2048,2 --shape 9,610,340,2 \\
      --precision fp32 --precision fp64 [--rounds 5] [--out PATH] [--fresh]

Timing does not depend on the input values for the plain method, so each
shape is tuned on positive random class probabilities.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import torch

from . import segsalsa as S


def tune_shapes(shapes, precisions, rounds=5, out=None, fresh=False, log=print):
    """Tune every (K, H, W, M) in `shapes` for every precision ("fp32"/"fp64"); returns {key: tuning}."""
    S.lib()
    if fresh:
        S.segsalsa_tuning_clear()
    elif out and os.path.exists(out):
        S.segsalsa_tuning_load(out)
    res = {}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    for (K, H, W, M) in shapes:
        for prec in precisions:
            dtype = torch.float32 if prec == "fp32" else torch.float64
            x = torch.rand((K, H, W), generator=gen, device="cuda", dtype=dtype) + 0.01
            pr = S.Problem(K, H, W, M, [1.0 / (2 * M + 1)] * (2 * M + 1) ** 2, 1.0, 1.5, 1.5, 1)
            ws = torch.empty(S.segsalsa_str_autotune_workspace_size(pr, S._prec(dtype)), dtype=torch.uint8,
                             device="cuda")
            z = torch.empty_like(x)
            t0 = time.perf_counter()
            best = S.segsalsa_str_autotune(pr, x, z, ws, rounds=rounds)
            torch.cuda.synchronize()
            res[(K, H, W, M, prec)] = best
            log(f"[autotune] K={K} H={H} W={W} M={M} {prec}: {best} ({time.perf_counter() - t0:.1f} s)")
            del ws, z, x
            torch.cuda.empty_cache()
    if out:
        os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
        S.segsalsa_tuning_save(out)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--shape", action="append", required=True, help="K,H,W,M (repeatable)")
    ap.add_argument("--precision", action="append", choices=("fp32", "fp64"))
    ap.add_argument("--rounds", type=int, default=5)
    ap.add_argument("--out", default=S.DEFAULT_TUNING_CACHE)
    ap.add_argument("--fresh", action="store_true", help="start from an empty table instead of the existing cache")
    a = ap.parse_args(argv)
    shapes = [tuple(int(v) for v in s.split(",")) for s in a.shape]
    if not torch.cuda.is_available():
        print("autotune needs a GPU", file=sys.stderr)
        return 2
    tune_shapes(shapes, a.precision or ["fp32"], a.rounds, a.out, a.fresh)
    return 0


if __name__ == "__main__":
    sys.exit(main())
