"""Multi-table schedule benchmark: tune on one seed, evaluate on another.

    python -m paper_1908_05936_amd.bench_multi [--tune-seed 4] [--eval-seed 6] [--out FILE]
        [--config JSON]   (skip tuning, e.g. for a kernel trace of the measured runs only)

Prints one JSON line: the tuned configuration, then for the evaluation schedule the plan run, its
HIP-graph replay and the same operations as one-stream single-table calls (keys/s and speedup).
"""
from __future__ import annotations

import argparse
import json
import sys

import torch

from . import ct
from .multi import measure, tune
from .workloads import multi_table


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--tune-seed", type=int, default=4)
    ap.add_argument("--eval-seed", type=int, default=6)
    ap.add_argument("--cache", default=None)
    ap.add_argument("--config", default=None,
                    help='skip tuning and use this configuration, e.g. '
                         '\'{"lanes": 0, "merge": true, "chunk": -1, "provision": 1.5}\'')
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    dev = torch.device("cuda", 0)
    ct.lib()
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    if a.config:
        cfg = dict(json.loads(a.config), trials=0)
    else:
        log("[multi] generating tuning schedule")
        wt = multi_table(seed=a.tune_seed)
        cfg = tune(wt, dev, cache=a.cache, log=log)
        del wt
        torch.cuda.empty_cache()
    log(f"[multi] tuned: {cfg}")
    we = multi_table(seed=a.eval_seed)
    res = measure(we, dev, dict(lanes=cfg["lanes"], merge=cfg.get("merge", False),
                                chunk=cfg["chunk"], provision=cfg["provision"],
                                block=cfg.get("block", 256)))
    res["tuned_on_seed"] = a.tune_seed
    res["evaluated_on_seed"] = a.eval_seed
    res["tuning"] = cfg
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
