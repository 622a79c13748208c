"""Profiling harness: one forward solve of a benchmark workload with a cap on
the seed iterations, for hardware-counter runs (rocprofv3 --pmc) whose
per-dispatch counts do not depend on how many iterations run.

    python -m paper_2506_11657_amd.profile_run --config graded64 --max-iter 2048

Prints one line per phase so that long profiler runs show progress.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="graded64", choices=["graded64", "plain16", "blocky128"])
    ap.add_argument("--max-iter", type=int, default=2048)
    ap.add_argument("--fields", action="store_true")
    args = ap.parse_args()
    import torch

    import tem_workloads as W
    from paper_2506_11657_amd import tem
    wl = {"graded64": W.cfg_graded64, "plain16": W.cfg_plain16, "blocky128": W.cfg_blocky128}[args.config]()
    xi, c, err = tem.poles(wl.t, wl.degree)
    print("poles: J=%d" % len(xi), flush=True)
    ctx = tem.Context.from_workload(wl)
    fields = None
    if args.fields:
        fields = torch.zeros((1, c.shape[1], ctx.n_storage), dtype=torch.float64, device="cuda")
    t0 = time.time()
    d, st = ctx.forward(wl.loops, wl.receivers, xi, c, fields=fields, max_iter=args.max_iter, allow_noconv=True)
    print("forward: %d iterations in %.2f s (%s)" % (st["iterations"], time.time() - t0, st["status"]), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
