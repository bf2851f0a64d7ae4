"""The paper's measurement grid on this GPU: float64 operator throughput for the
nine cubic meshes N_E = 128 ... 32768 elements and 3 <= lx <= 8 (Sec. 4.4 and
Sec. 5), reported as Gflop/s with 12 lx + 18 flop per local node (the paper
states no flop formula; this counts 6 lx multiply-adds per node for the three
derivative passes, 6 lx for the transposed passes and 18 for the geometric
multiply), plus GB/s at 72 B per local node and unique GDOF/s.

The operator is element-local, so its throughput depends only on the element
count and lx: every point uses N_E elements of random symmetric positive
definite factors, h1 ~ U[0.5, 2] and u ~ N(0, 1).

With --tune every point first times each float64 kernel variant of the
operator on its own fields (sem_ax_tune_on: the column mapping, the same with
the other prefetch choice, the slice-pipelined column mapping, one thread per
node, one element per wave), as the paper's run-time autotuning does (Sec. 4),
and the timed run uses the fastest.

Usage: python -m paper_2506_20994_amd.sweep [--reps R] [--out FILE] [--lx 3,..] [--sizes ..] [--tune]
"""
import argparse
import json
import sys
import time

import numpy as np
import torch

import synth
from . import _binding as B

SIZES = [128, 256, 512, 1024, 2048, 4096, 8192, 16384, 32768]
LXS = [3, 4, 5, 6, 7, 8]


def _fields(ctx, nel, lx, seed=0):
    """Random operator inputs of nel elements (the operator is element-local, so
    the throughput does not depend on how the elements are connected)."""
    G, h1 = synth.random_spd_factors(nel, lx, seed)
    u = synth.local_normal(nel, lx, seed + 1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    _, _, dx, dxt = B.sem_gll(lx)
    D = [dev(dx)] * 3 + [dev(dxt)] * 3
    return dev(u), [dev(g) for g in G], dev(h1), D


def run(reps=50, lxs=LXS, sizes=SIZES, tune=False):
    ctx = B.sem_create()
    rows = []
    names = {B.SEM_AX_COLUMN: "column", B.SEM_AX_COLUMN_PF: "column_pf", B.SEM_AX_SLICE: "slice", B.SEM_AX_3D: "3d",
             B.SEM_AX_WAVE: "wave"}
    for lx in lxs:
        for nel in sizes:
            tuned = None
            u, G, h1, D = _fields(ctx, nel, lx)
            w = torch.empty_like(u)
            if tune:
                best, us = B.sem_ax_tune_on(ctx, w, u, *D, h1, *G, nel, lx, reps=20)
                tuned = {"variant": names[best],
                         "variant_us": {names[v]: round(t, 2) for v, t in enumerate(us) if t > 0}}
            for _ in range(5):
                B.sem_ax(ctx, w, u, *D, h1, *G, nel, lx)
            st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(st)
            for _ in range(reps):
                B.sem_ax(ctx, w, u, *D, h1, *G, nel, lx)
            e1.record(st)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / reps * 1e-3
            nl = nel * lx ** 3
            rows.append({"lx": lx, "nel": nel, "us": round(t * 1e6, 2),
                         "gflops": round((12 * lx + 18) * nl / t / 1e9, 1),
                         "gbs": round(72 * nl / t / 1e9, 1),
                         "gdofs": round(nel * (lx - 1) ** 3 / t / 1e9, 3)})
            if tuned:
                rows[-1].update(tuned)
            print(json.dumps(rows[-1]), flush=True)
        if tune:
            B.sem_ax_set_variant(ctx, lx, B.SEM_AX_DEFAULT)
    ctx.close()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=50)
    ap.add_argument("--out", default=None)
    ap.add_argument("--lx", default=None, help="comma-separated lx values (default 3..8)")
    ap.add_argument("--sizes", default=None, help="comma-separated element counts")
    ap.add_argument("--tune", action="store_true", help="time the kernel variants at every point, use the fastest")
    a = ap.parse_args()
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    lxs = [int(v) for v in a.lx.split(",")] if a.lx else LXS
    sizes = [int(v) for v in a.sizes.split(",")] if a.sizes else SIZES
    rows = run(a.reps, lxs, sizes, a.tune)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f, indent=1)
    print(f"[sweep] {len(rows)} points in {time.perf_counter() - t0:.1f} s", file=sys.stderr)


if __name__ == "__main__":
    main()
