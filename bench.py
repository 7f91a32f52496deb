"""Benchmark: staggered Dslash GB/s / GFLOP/s at 32^4 and mixed-vs-FP64 CG time to 1e-10.

One step = the whole hot path on the 32^4 workload (Haar SU(3) links, m = 0.01,
one Gaussian source, x0 = 0, stop at 1e-10 true relative residual):
  1. FP64 even-odd CG (FP64 links and vectors),
  2. mixed CG: FP32 12-real links, FP32 vectors, FP64 reliable update every 50,
  3. mixed CG: BF16 12-real links, FP32 vectors, FP64 iterative refinement (inner 0.1).
`value` is the FP64 Dslash bandwidth (algorithmic bytes / kernel time), measured
with HIP events around every FP64 Dslash launch inside the timed FP64 solves
(the library records them on its stream). Inputs are resident in HBM before the
timed region; link packing is done once per gauge field, outside it.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dslash GB/s & GFLOP/s at 32^4; mixed-vs-FP64 CG time to 1e-10 residual"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes_per_site(prec, recon):
    """Algorithmic HBM bytes per output site of one half-Dslash: 8 links read once,
    the input vector read once (perfect reuse of neighbours), the output written once."""
    import paper_1309_0551_amd as P
    return 8 * P.link_bytes_per_dir(prec, recon) + 2 * P.vec_bytes_per_site(prec)


def time_dslash(lat, Up, x, out, n=20, warm=5):
    import torch
    s = lat.stream
    for _ in range(warm):
        lat.dslash(Up, x, 1, out)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in evs:
        a.record(s)
        lat.dslash(Up, x, 1, out)
        b.record(s)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def cpu_baseline(L, U, chi, budget_s=15.0):
    import oracle
    oracle.dslash(L, U, chi, 1)  # warm (page in, thread pool)
    n, t0 = 0, time.perf_counter()
    while True:
        oracle.dslash(L, U, chi, 1)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 50:
            break
    return n, el


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, nargs=4, default=(32, 32, 32, 32))
    ap.add_argument("--mass", type=float, default=0.01)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharded design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import lgt_inputs as li
    import paper_1309_0551_amd as P

    L = tuple(args.L)
    V = int(np.prod(L))
    Vh = V // 2
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    U = li.links(L, "haar", 3001)
    b = li.vector(L, 3002)
    log(f"inputs generated in {time.perf_counter() - t0:.1f}s")

    lat = P.Lattice(L, device=0)
    Ut = torch.from_numpy(U).to(dev)
    bt = torch.from_numpy(b).to(dev)
    U64 = lat.pack_links(Ut, P.LGT_F64, P.LGT_R18)
    U32 = lat.pack_links(Ut, P.LGT_F32, P.LGT_R12)
    U16 = lat.pack_links(Ut, P.LGT_BF16, P.LGT_R12)
    del Ut
    torch.cuda.synchronize()

    # standalone Dslash, every format (context numbers; `value` comes from the solves)
    fmts = {"f64r18": U64, "f64r12": None, "f32r18": None, "f32r12": U32, "bf16r12": U16}
    dslash = {}
    for name, Up in fmts.items():
        if Up is None:
            prec = P.LGT_F64 if name.startswith("f64") else P.LGT_F32
            Up = lat.pack_links(torch.from_numpy(U).to(dev), prec, int(name[-2:]))
        vp = P.LGT_F64 if Up.prec == P.LGT_F64 else P.LGT_F32
        x = lat.pack_vec(bt, vp)
        out = lat.native_vec(vp)
        ms = statistics.median(time_dslash(lat, Up, x, out))
        by = alg_bytes_per_site(Up.prec, Up.recon) * Vh
        dslash[name] = {"us": round(ms * 1e3, 2), "GBps": round(by / (ms * 1e-3) / 1e9, 1),
                        "GFLOPs": round(P.DSLASH_FLOP_PER_SITE * Vh / (ms * 1e-3) / 1e9, 1),
                        "alg_bytes": by}
        log(f"dslash {name}: {dslash[name]}")

    def solves(timing):
        lat.set_timing(timing)
        out = {}
        x, r = lat.cg_solve(U64, bt, args.mass, tol=1e-10, scheme=P.LGT_CG_FP64)
        out["fp64"] = r
        x, r = lat.cg_solve(U64, bt, args.mass, tol=1e-10, scheme=P.LGT_CG_RELIABLE, U_lo=U32, ru_interval=50)
        out["f32r12_reliable"] = r
        x, r = lat.cg_solve(U64, bt, args.mass, tol=1e-10, scheme=P.LGT_CG_REFINE, U_lo=U16, inner_tol=0.1)
        out["bf16r12_refine"] = r
        return out

    for _ in range(args.warmup):
        solves(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    steps = []
    for _ in range(args.steps):
        steps.append(solves(True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    lat.set_timing(False)

    ms_hi = sum(s["fp64"].dslash_ms_hi for s in steps)
    n_hi = sum(s["fp64"].dslash_timed_hi for s in steps)
    avg_ms = ms_hi / max(n_hi, 1)
    by64 = alg_bytes_per_site(P.LGT_F64, P.LGT_R18) * Vh
    gbs = by64 / (avg_ms * 1e-3) / 1e9
    gflops = P.DSLASH_FLOP_PER_SITE * Vh / (avg_ms * 1e-3) / 1e9

    def summ(key):
        rs = [s[key] for s in steps]
        return {"seconds_median": round(statistics.median(r.seconds for r in rs), 4),
                "iters": rs[-1].iters, "updates": rs[-1].updates, "dslash_calls": rs[-1].dslash_calls,
                "true_rel_resid": rs[-1].true_rel_resid, "status": rs[-1].status,
                "dslash_us_avg": round(1e3 * sum(r.dslash_ms_lo + r.dslash_ms_hi for r in rs) /
                                       max(1, sum(r.dslash_timed_lo + r.dslash_timed_hi for r in rs)), 2)}

    cg = {k: summ(k) for k in ("fp64", "f32r12_reliable", "bf16r12_refine")}
    cg["speedup_f32_vs_fp64"] = round(cg["fp64"]["seconds_median"] / cg["f32r12_reliable"]["seconds_median"], 3)
    cg["speedup_bf16_vs_fp64"] = round(cg["fp64"]["seconds_median"] / cg["bf16r12_refine"]["seconds_median"], 3)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        n, el = cpu_baseline(L, U, b, args.cpu_budget)
        cpu = {"value": round(by64 * n / el / 1e9, 3), "unit": "GB/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"{n} FP64 D_oe applications of the oracle at {'x'.join(map(str, L))} "
                         f"({el:.1f} s), algorithmic bytes as for the GPU"}

    line = {
        "metric": METRIC, "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"staggered Dslash + even-odd CG, {'x'.join(map(str, L))} lattice, Haar SU(3) "
                               f"links, m={args.mass}, tol 1e-10; step = FP64 CG + FP32-12 reliable CG + "
                               f"BF16-12 refinement CG", "lattice": list(L), "mass": args.mass},
        "gflops": round(gflops, 1),
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_dslash<LinkF64R18, EPI_A|EPI_PLAIN> inside FP64 CG",
                     "alg_bytes_per_launch": by64, "avg_launch_us": round(avg_ms * 1e3, 2)},
        "cg": cg,
        "dslash_standalone": dslash,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    lat.close()


if __name__ == "__main__":
    main()
