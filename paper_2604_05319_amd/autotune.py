"""Project autotuner: times candidate tile shapes and panel heights of the HODLR history
step on a workload and records the fastest in a JSON file that bench.py reads.

Knobs: the factor rows of one projection task (hnessi_set_tile_shape) and the panel height
P of the incremental TSVD merges.  Every candidate runs on the GPU through the library;
the choice is the candidate with the highest time steps per second over the timed sweep
(a full sweep for the single-object workload, a 1024-step prefix for the lattice).

    python -m paper_2604_05319_amd.autotune [--out FILE] [--workloads c2,c3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning.json")
PANELS = (8, 16)   # panel heights the handles accept (1..16)


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _time_sweep(P, cfg, arrs, nlvl, norb, panel, rows, n_end, nk=None):
    import torch
    P.set_tile_shape(norb, rows)
    try:
        if nk is None:
            H = P.Hodlr(cfg["nt"], nlvl, norb, k=cfg["k"], tol=cfg["tol"], panel=panel, max_rank=16)
        else:
            H = P.HodlrBatch(nk, cfg["nt"], nlvl, norb, k=cfg["k"], tol=cfg["tol"], panel=panel, max_rank=16)
    finally:
        P.set_tile_shape(norb, 0)
    IR, IL = arrs[4], arrs[5]
    H.sweep(0, min(256, n_end), *arrs[:4], cfg["h"], IR, IL)   # warm-up
    H.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H.sweep(0, n_end, *arrs[:4], cfg["h"], IR, IL)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    status = H.status()
    H.close()
    return n_end / dt, status


def tune(workload):
    import numpy as np
    import torch
    import paper_2604_05319_amd as P
    from kbe_inputs import make_config_inputs
    from kbe_inputs.packed import packed_torch
    cfg, G, S = make_config_inputs(workload)
    N, h, norb = cfg["nt"], cfg["h"], cfg["norb"]
    nlvl = int(round(np.log2(N // cfg["leaf"])))
    dev = torch.device("cuda:0")
    tot = N * (N + 1) // 2
    if workload == "c3":
        nk = len(G)
        arrs = []
        for src, kind in ((G, "ret"), (G, "les"), (S, "ret"), (S, "les")):
            a = torch.empty((nk * tot,), dtype=torch.complex128, device=dev)
            for o in range(nk):
                a[o * tot:(o + 1) * tot] = packed_torch(src[o], kind, N, h, dev).reshape(-1)
            arrs.append(a)
        n_end = 1024
    else:
        nk = None
        arrs = [packed_torch(G, "ret", N, h, dev), packed_torch(G, "les", N, h, dev),
                packed_torch(S, "ret", N, h, dev), packed_torch(S, "les", N, h, dev)]
        n_end = N
    arrs += [torch.empty_like(arrs[0]), torch.empty_like(arrs[0])]
    row_choices = (256, 512, 1024) if norb <= 4 else (128, 256)
    cands = []
    for panel in PANELS:
        for rows in row_choices:
            v, st = _time_sweep(P, cfg, arrs, nlvl, norb, panel, rows, n_end, nk)
            _log(f"{workload}: panel {panel}, projection rows {rows}: {v:.1f} steps/s (status {st})")
            if st == 0:
                cands.append(dict(panel=panel, proj_rows=rows, steps_per_s=round(v, 2)))
    del arrs
    torch.cuda.empty_cache()
    best = max(cands, key=lambda c: c["steps_per_s"])
    return dict(panel=best["panel"], proj_rows=best["proj_rows"], steps_per_s=best["steps_per_s"],
                timed_steps=n_end, objects=nk or 1, candidates=cands)


def load(path=DEFAULT_OUT):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--workloads", default="c2,c3")
    args = ap.parse_args()
    import torch
    out = load(args.out)
    for w in args.workloads.split(","):
        out[w] = tune(w)
        out[w]["device"] = torch.cuda.get_device_name(0)
        out[w]["date"] = time.strftime("%Y-%m-%d")
        _log(f"{w}: chosen {out[w]['panel']=} {out[w]['proj_rows']=}")
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    print(json.dumps({w: {k: out[w][k] for k in ('panel', 'proj_rows', 'steps_per_s')} for w in out}))


if __name__ == "__main__":
    main()
