"""Benchmark: staggered Dslash GB/s / GFLOP/s at 32^4 and mixed-vs-FP64 CG time to 1e-10.

Workload: 32^4 lattice, Haar-random SU(3) links, m = 0.01, one Gaussian source
on the even sites, x0 = 0, stop at 1e-10 true relative residual.

One step = the whole hot path:
  1. FP64 even-odd CG (FP64 links and vectors),
  2. mixed CG: FP32 12-real links, FP32 vectors, FP64 reliable update every 50,
  3. mixed CG: BF16 12-real links, FP32 vectors, FP64 iterative refinement
     (inner relative tolerance 0.1),
  4. batched CG: 24^3x48 with 16 right-hand sides, then 8^4, 12^4 and
     16^3x32 with 4 each in one call (Haar links, m = 0.02, FP32-12 with FP64
     reliable updates every 50; the multi-RHS Dslash variant the tuner picks
     for each lattice): both as kernel launches, the three lattices each on
     its own stream,
  5. S = phi^dag A^-1 phi and dS/dU at 16^3x32 (links exp(0.5 i H),
     m = 0.05) through the autograd function: FP64 CG forward, fermion-force
     kernel backward.
`value` is the FP64 Dslash bandwidth in algorithmic bytes (8 links + the
input vector read once + the output written once per site) over the kernel
time of the CG iteration's D_oe launch (whose epilogue also forms the
<p, A p> partials), measured with HIP events that the library records on the
launch's own dispatch packet in every 16th iteration of the timed FP64 solves.
The iteration's D_eo launch, which also applies the update of r, is reported
beside it with its own bytes. Inputs are resident in HBM before the timed
region; link packing is done once per gauge field, outside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dslash GB/s & GFLOP/s at 32^4; mixed-vs-FP64 CG time to 1e-10 residual"
HBM_PEAK_GBS = 8000.0
# Dslash kernel times come from HIP events around the Dslash pair of every
# TIMING_EVERY-th CG iteration: each event costs a few microseconds of stream
# time, so timing every launch would inflate the solve times it sits in.
TIMING_EVERY = 16
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dslash_f64r18_32x32x32x32_traffic.txt")
KERNEL_SOURCES = ["paper_1309_0551_amd/csrc/dslash.hip", "paper_1309_0551_amd/csrc/fields.hpp",
                  "paper_1309_0551_amd/csrc/geom.hpp", "paper_1309_0551_amd/csrc/reduce.hpp"]


# The paper's own measurements, quoted as context (Pentium 4 class hardware):
# seconds for 10^6 cache-warm calls of each routine, SSE2 vs optimised plain C
# (Table 2), and MILC ks_imp_dyn1 application seconds (Table 4).
PAPER_TABLE2 = {"mult_su3_mat_vec": (4.05, 7.13), "mult_adj_su3_mat_vec": (4.03, 5.68),
                "mult_su3_mat_vec_sum_4dir": (17.49, 30.01), "mult_adj_su3_mat_vec_4dir": (15.75, 25.0),
                "sub_four_su3_vecs": (2.33, 4.44), "su3_projector": (4.09, 16.14)}
PAPER_TABLE4 = {"4^4 serial FP64": {"plain": 220, "sse2_aligned": 135},
                "4^4 serial FP32": {"plain": 153, "sse_aligned": 89},
                "16^4 parallel FP64": {"plain": 17290, "sse2_unaligned": 16614},
                "16^4 parallel FP32": {"plain": 5367, "sse_unaligned": 4044}}


def paper_context():
    t4 = {k: {**v, "speedup": round(v["plain"] / min(x for n, x in v.items() if n != "plain"), 2)}
          for k, v in PAPER_TABLE4.items()}
    return {"hardware": "2.4 GHz Pentium 4, 8 KB L1D, 256 KB L2, 533 MHz bus, 2 GB RAM, gcc -O3 (Table 4); "
                        "routine timings gcc -O2, 10^6 cache-warm calls (Table 2)",
            "routine_speedup_sse2_table2": {k: round(b / a, 2) for k, (a, b) in PAPER_TABLE2.items()},
            "application_table4_s": t4,
            "single_over_double_plain_table4": {"4^4 serial": round(220 / 153, 2),
                                                "16^4 parallel": round(17290 / 5367, 2)},
            "note": "context only: other hardware, other quantities; the comparable figure here is "
                    "cg.speedup_f32_vs_fp64 (mixed precision over FP64 on one MI355X)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """Counted HBM bytes per FP64 Dslash launch from the committed counter summary,
    or None when the kernel sources changed since the counters were taken."""
    try:
        vals = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if "=" in line and not line.lstrip().startswith("#"):
                    k, v = line.split("=", 1)
                    vals[k.strip()] = v.strip()
        if vals.get("kernel_source_sha") != kernel_source_sha():
            return None
        return int(float(vals["bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def alg_bytes_per_site(prec, recon):
    """Algorithmic HBM bytes per output site of one half-Dslash: 8 links read once,
    the input vector read once (perfect reuse of neighbours), the output written once."""
    import paper_1309_0551_amd as P
    return 8 * P.link_bytes_per_dir(prec, recon) + 2 * P.vec_bytes_per_site(prec)


def event_times(lat, fn, n, warm):
    import torch
    for _ in range(warm):
        fn()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in evs:
        a.record(lat.stream)
        fn()
        b.record(lat.stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def probes(lat):
    """Measured streaming ceilings: read-only and copy of 1 GiB, median of 10."""
    import torch
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device=lat.device)
    dst = torch.empty_like(src)
    sink = torch.zeros(2, dtype=torch.float64, device=lat.device)
    rd = statistics.median(event_times(lat, lambda: lat.stream_read(src, sink), 10, 3))
    cp = statistics.median(event_times(lat, lambda: lat.stream_copy(src, dst), 10, 3))
    nb = n * 8
    del src, dst
    return {"read_GBps": round(nb / (rd * 1e-3) / 1e9, 1), "copy_GBps": round(2 * nb / (cp * 1e-3) / 1e9, 1),
            "bytes": nb}


def fd_check(lat, U, phi, mass, G, L, seed, ndir, eps=1e-6):
    """Central differences of the action along ndir random link directions.
    S~ = 2 Re <phi, x> - <x, A x> with x from the FP64 CG to 1e-12 (its error is
    quadratic in the residual) and A x from lgt_apply_normal; the difference of
    the two S~ is summed element by element so it keeps its own precision.
    Returns (seconds, largest |FD - <G, E>| relative to max(|<G, E>|, median))."""
    import lgt_inputs as li
    import numpy as np
    import paper_1309_0551_amd as P
    import torch
    mus, sites, Es = li.fd_directions(L, seed, ndir)

    def terms(Ut):
        Up = lat.pack_links(Ut, P.LGT_F64, P.LGT_R18)
        x, res = lat.cg_solve(Up, phi, mass, tol=1e-12)
        Ax = lat.unpack_vec(lat.apply_normal(Up, lat.pack_vec(x), mass)[0])
        return (2.0 * (phi[..., 0] * x[..., 0] + phi[..., 1] * x[..., 1])
                - (x[..., 0] * Ax[..., 0] + x[..., 1] * Ax[..., 1]))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    an, fd = [], []
    for mu, site, E in zip(mus, sites, Es):
        Et = torch.from_numpy(E).to(U.device)
        Up, Um = U.clone(), U.clone()
        Up[mu, site] += eps * Et
        Um[mu, site] -= eps * Et
        fd.append(float((terms(Up) - terms(Um)).sum()) / (2 * eps))
        an.append(float((G[mu, site] * Et).sum()))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    an, fd = np.array(an), np.array(fd)
    scale = np.maximum(np.abs(an), np.median(np.abs(an)))
    return el, float((np.abs(fd - an) / scale).max())


def small_configs(args):
    """The small workloads, timed after the steps: 4^4 (Haar, m = 0.1) and 16^4
    (exp(0.3 i H), m = 0.05). FP64 Dslash alone on both parities (mean of 100
    back-to-back launches between two events, after 10 warm-up launches), the
    FP64 CG (second of two solves), and the Dslash inside a third solve from
    events carried on its own dispatch packets."""
    import lgt_inputs as li
    import paper_1309_0551_amd as P
    import torch
    out, sols = {}, {}
    for key in ("c1_4x4x4x4", "c2_16x16x16x16"):
        cfg = li.CONFIGS[key]
        L = cfg["L"]
        with P.Lattice(L) as lat:
            dev = lat.device
            U = torch.from_numpy(li.links(L, cfg["kind"], cfg["link_seed"], cfg["c"] or 0.3)).to(dev)
            Up = lat.pack_links(U, P.LGT_F64, P.LGT_R18)
            if not args.no_tune:
                lat.tune_dslash(Up, report=False)
            b = torch.from_numpy(li.vector(L, cfg["src_seed"])).to(dev)
            xin = lat.pack_vec(b)
            y = torch.empty_like(xin)
            d = {}
            for par in (0, 1):
                for _ in range(10):
                    lat.dslash(Up, xin, par, y)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(lat.stream)
                for _ in range(100):
                    lat.dslash(Up, xin, par, y)
                e1.record(lat.stream)
                e1.synchronize()
                d["dslash_us_parity%d" % par] = round(e0.elapsed_time(e1) * 10.0, 2)
            x, r = lat.cg_solve(Up, b, cfg["mass"], tol=cfg["tol"])  # warm
            x, r = lat.cg_solve(Up, b, cfg["mass"], tol=cfg["tol"])
            lat.set_timing(1)
            _, rt = lat.cg_solve(Up, b, cfg["mass"], tol=cfg["tol"])
            lat.set_timing(False)
            d.update({"lattice": list(L), "mass": cfg["mass"], "cg_fp64_s": round(r.seconds, 5), "iters": r.iters,
                      "true_rel_resid": r.true_rel_resid,
                      "dslash_in_cg_us": round(1e3 * rt.dslash_ms_hi / max(rt.dslash_timed_hi, 1), 2),
                      "variant": "hops=%d streaming=%d workgroup=%d" % (
                          lat.dslash_variant(P.LGT_F64, P.LGT_R18) + (lat.dslash_workgroup(P.LGT_F64, P.LGT_R18),))})
            out[key[3:]] = d
            sols[key[3:]] = (L, U.cpu().numpy(), cfg["mass"], b.cpu().numpy(), x.cpu().numpy())
    return out, sols


def _timed(fn, budget_s):
    """Repeat fn until budget_s seconds have passed (at least once); (runs, seconds)."""
    n, t0 = 0, time.perf_counter()
    while True:
        fn()
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            return n, el


def cpu_leg(L, U, chi, mass, budget_s, gpu):
    """The oracle's side of the measurement, on the host cores after the GPU
    work: its FP64 Dslash and CG timed on bounded samples of the workloads
    (all threads and one thread), and the oracle's errors of the GPU results
    of this run (`gpu`: host copies of the 32^4 solutions, the Dslash output
    and the small-lattice solutions)."""
    import lgt_inputs as li
    import numpy as np
    import oracle
    nthreads = oracle.threads()
    Vh = int(np.prod(L)) // 2
    site_bytes = 1248
    oracle.dslash(L, U, chi, 1)  # warm: page in, start the thread pool
    n, el = _timed(lambda: oracle.dslash(L, U, chi, 1), budget_s)
    out = {"value": round(site_bytes * Vh * n / el / 1e9, 3), "unit": "GB/s", "cores": nthreads, "kind": "oracle",
           "sample": f"{n} FP64 D_oe applications of the C oracle (OpenMP, {nthreads} threads) at "
                     f"{'x'.join(map(str, L))} in {el:.1f} s; algorithmic bytes of a plain Dslash (1248 B/site)"}
    extra = {}
    oracle.set_threads(1)
    try:
        n1, el1 = _timed(lambda: oracle.dslash(L, U, chi, 1), budget_s / 4)
        extra["dslash_1thread_GBps"] = round(site_bytes * Vh * n1 / el1 / 1e9, 3)
        for key in ("c1_4x4x4x4", "c2_16x16x16x16"):
            cfg = li.CONFIGS[key]
            Lc = cfg["L"]
            Uc = li.links(Lc, cfg["kind"], cfg["link_seed"], cfg["c"] or 0.3)
            bc_ = li.vector(Lc, cfg["src_seed"])
            row = {}
            for label, th in (("all_threads", nthreads), ("1_thread", 1)):
                oracle.set_threads(th)
                t0 = time.perf_counter()
                st, _, it, rr = oracle.cg(Lc, Uc, cfg["mass"], bc_, tol=cfg["tol"])
                row[label + "_s"] = round(time.perf_counter() - t0, 4)
            row.update({"iters": it, "true_rel_resid": rr, "status": st})
            extra["cg_fp64_" + key[3:]] = row
        # 32^4: a bounded sample of the FP64 CG (the first 200 iterations), per iteration
        oracle.set_threads(nthreads)
        t0 = time.perf_counter()
        st, _, it, _ = oracle.cg(L, U, mass, chi, tol=1e-10, max_iter=200)
        per_it = (time.perf_counter() - t0) / max(it, 1)
        extra["cg_fp64_32x32x32x32_sample"] = {"iters_run": it, "s_per_iter": round(per_it, 5),
                                               "s_at_gpu_iters": round(per_it * gpu["fp64_iters"], 2),
                                               "threads": nthreads}
    finally:
        oracle.set_threads(nthreads)
    out["extra"] = extra
    # errors of this run's GPU results against the oracle (spec: per result)
    bn = float(np.linalg.norm(chi))
    errs = {}
    for key, x in gpu["x32"].items():
        r = chi - oracle.apply_A(L, U, mass, x)
        errs["cg_" + key] = {"oracle_true_rel_resid": float(np.linalg.norm(r) / bn),
                             "x_err_bound_rel": float(np.linalg.norm(r) / (4 * mass * mass) / np.linalg.norm(x))}
    for key in ("f32r12_reliable", "bf16r12_refine"):
        if key in gpu["x32"] and "fp64" in gpu["x32"]:
            d = gpu["x32"][key] - gpu["x32"]["fp64"]
            errs["cg_" + key]["rel_diff_vs_fp64_gpu"] = float(np.linalg.norm(d) / np.linalg.norm(gpu["x32"]["fp64"]))
    ref = oracle.dslash(L, U, gpu["dslash_in"], 1)
    d = gpu["dslash_out"] - ref
    errs["dslash_f64r18"] = {"rel": float(np.linalg.norm(d) / np.linalg.norm(ref)),
                             "max_abs_over_max_ref": float(np.abs(d).max() / np.abs(ref).max())}
    for key, (Lc, Uc, m, bc_, xg) in gpu["small"].items():
        st, xo, it, rr = oracle.cg(Lc, Uc, m, bc_, tol=1e-10)
        r = bc_ - oracle.apply_A(Lc, Uc, m, xg)
        errs["cg_fp64_" + key] = {"oracle_true_rel_resid": float(np.linalg.norm(r) / np.linalg.norm(bc_)),
                                  "x_rel_err_vs_oracle_solve": float(np.linalg.norm(xg - xo) / np.linalg.norm(xo)),
                                  "oracle_iters": it}
    return out, errs


PROBE_FMTS = {"f64r18": (0, 18), "f64r12": (0, 12), "f32r18": (1, 18), "f32r12": (1, 12), "bf16r12": (2, 12)}


def probe_dslash(L, fmt, launches, hops, streaming):
    """--probe: the one-link Dslash alone on a lattice of any size. Links are
    independent draws from a pool of 2^16 Haar matrices, gathered on the device
    (lattices of many GB take seconds); `launches` plain Dslash applications
    (output parity odd) after one warm-up, timed with events on their stream;
    prints the mean kernel time and the algorithmic bandwidth (8 links, the
    input once and the output once per output site). Run it under rocprofv3 to
    read the same launches' counters."""
    import math

    import torch

    import lgt_inputs as li
    import paper_1309_0551_amd as P
    dev = torch.device("cuda", 0)
    V = math.prod(L)
    prec, recon = PROBE_FMTS[fmt]
    vp = P.LGT_F64 if prec == P.LGT_F64 else P.LGT_F32
    pool = torch.from_numpy(li.to_real(li.haar_su3(1 << 16, li.rng(7)))).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(1)
    with P.Lattice(L) as lat:
        U = pool[torch.randint(0, pool.shape[0], (4 * V,), device=dev, generator=g)].reshape(4, V, 3, 3, 2)
        Up = lat.pack_links(U.contiguous(), prec, recon)
        del U, pool
        torch.cuda.empty_cache()
        if hops:
            lat.set_dslash_variant(prec, recon, hops, streaming)
        x = lat.pack_vec(torch.randn(lat.Vh, 3, 2, dtype=torch.float64, device=dev, generator=g), vp)
        y = torch.empty_like(x)
        lat.dslash(Up, x, 1, y)  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(lat.stream)
        for _ in range(launches):
            lat.dslash(Up, x, 1, y)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / launches
        h, st = lat.dslash_variant(prec, recon)
    alg = lat.Vh * alg_bytes_per_site(prec, recon)
    return {"probe": "dslash", "L": list(L), "fmt": fmt, "hops": h, "streaming": st, "launches": launches,
            "us_per_launch": round(us, 2), "alg_bytes_per_launch": alg, "alg_GBps": round(alg / us / 1e3, 1)}


def probe_dslash_mrhs(L, fmt, nrhs, launches):
    """--probe with --nrhs N > 1: the standalone multi-RHS Dslash on the same
    kind of links, every variant that applies (engine, groups of four lanes,
    LDS staging), each `launches` plain applications (output parity odd) after
    one warm-up, timed with events; algorithmic bytes per output site: 8 links
    and N input and N output vectors. Under rocprofv3 the kernel names tell the
    variants apart (k_dslash_mrhs4s: staged; template arguments R, groups,
    MFMA)."""
    import math

    import torch

    import lgt_inputs as li
    import paper_1309_0551_amd as P
    dev = torch.device("cuda", 0)
    V = math.prod(L)
    prec, recon = PROBE_FMTS[fmt]
    if prec == P.LGT_F64:
        raise SystemExit("--nrhs probes the FP32 / BF16 link formats")
    pool = torch.from_numpy(li.to_real(li.haar_su3(1 << 16, li.rng(7)))).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(1)
    out = {"probe": "dslash_mrhs", "L": list(L), "fmt": fmt, "nrhs": nrhs, "launches": launches, "variants": {}}
    with P.Lattice(L) as lat:
        U = pool[torch.randint(0, pool.shape[0], (4 * V,), device=dev, generator=g)].reshape(4, V, 3, 3, 2)
        Up = lat.pack_links(U.contiguous(), prec, recon)
        del U, pool
        torch.cuda.empty_cache()
        x = torch.randn((3, lat.Vh, nrhs, 2), dtype=torch.float32, device=dev, generator=g)
        y = torch.empty_like(x)
        alg = lat.Vh * (8 * P.link_bytes_per_dir(prec, recon) + 2 * nrhs * 24)
        out["alg_bytes_per_launch"] = alg
        for e, gr, st in P.Lattice.MRHS_VARIANTS:
            if e != P.LGT_MRHS_LANE and 4 * gr > nrhs:
                continue
            lat.set_mrhs_variant(prec, recon, nrhs, e, gr)
            lat.set_mrhs_staging(prec, recon, nrhs, bool(st))
            runs = lat.mrhs_variant(prec, recon, nrhs) + (int(lat.mrhs_staging(prec, recon, nrhs)),)
            if runs != (e, gr, st):
                continue  # does not apply on this lattice
            lat.dslash_mrhs(Up, x, 1, y)  # warm-up
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(lat.stream)
            for _ in range(launches):
                lat.dslash_mrhs(Up, x, 1, y)
            e1.record(lat.stream)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / launches
            name = {P.LGT_MRHS_LANE: "lane", P.LGT_MRHS_VALU4: "valu4", P.LGT_MRHS_MFMA: "mfma"}[e]
            name += "" if e == P.LGT_MRHS_LANE else f"_g{gr}" + ("_lds" if st else "")
            out["variants"][name] = {"us_per_launch": round(us, 2), "alg_GBps": round(alg / us / 1e3, 1)}
    return out


def probe_batch(launches):
    """--probe-batch: the 24^3x48 x16 batched solve of the benchmark step alone
    (same links, sources, mass and tolerance; FP32 x 12 inner CG with FP64
    reliable updates every 50; the multi-RHS variant the tuner picks), solved
    `launches` times after the tuner, then once more with the phase profile
    on. One problem of 5.3M (site, rhs) pairs: the library runs it as kernel
    launches, so a kernel trace of this probe covers the batched CG without a
    cooperative launch."""
    import torch

    import lgt_inputs as li
    import paper_1309_0551_amd as P
    dev = torch.device("cuda", 0)
    c4 = li.CONFIGS["c4_24x24x24x48"]
    out = {"probe": "batch", "L": list(c4["L"]), "nrhs": c4["nrhs"], "launches": launches, "seconds": []}
    with P.Lattice(c4["L"], device=0) as lb:
        Ub = torch.from_numpy(li.links(c4["L"], "haar", c4["link_seed"])).to(dev)
        bb = torch.from_numpy(li.vectors(c4["L"], c4["src_seed"], c4["nrhs"])).to(dev)
        uh, ul = lb.pack_links(Ub, P.LGT_F64, P.LGT_R18), lb.pack_links(Ub, P.LGT_F32, P.LGT_R12)
        del Ub
        lb.tune_dslash_mrhs(ul, c4["nrhs"], report=False)
        probs = [(lb, uh, ul, bb)]
        for _ in range(launches):
            _, res = P.cg_solve_batch(probs, c4["mass"], tol=c4["tol"], scheme=P.LGT_CG_RELIABLE, ru_interval=50)
            out["seconds"].append(round(res[0][0].seconds, 4))
        its = max(r.iters for r in res[0])
        out["iters"] = its
        out["us_per_iteration"] = round(1e6 * min(out["seconds"]) / its, 2)
        out["true_rel_resid_max"] = max(r.true_rel_resid for r in res[0])
        out["variant"] = list(lb.mrhs_variant(P.LGT_F32, P.LGT_R12, c4["nrhs"]))
        lb.set_timing(1)
        P.cg_solve_batch(probs, c4["mass"], tol=c4["tol"], scheme=P.LGT_CG_RELIABLE, ru_interval=50)
        lb.set_timing(0)
        prof = lb.batch_profile()
        pit = max(prof.pop("iters"), 1)
        out["form"] = "launched" if prof["wait1"] == 0.0 and prof["wait2"] == 0.0 else "persistent"
        out["phases_us_per_iter"] = {k: round(1e3 * v / pit, 2) for k, v in prof.items()}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, nargs=4, default=(32, 32, 32, 32))
    ap.add_argument("--mass", type=float, default=0.01)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in Dslash variants")
    ap.add_argument("--no-singles", action="store_true",
                    help="skip the one-time comparisons outside the timed steps (batched vs single solves, "
                         "BF16 links under reliable updates)")
    ap.add_argument("--no-hmc", action="store_true",
                    help="skip the HMC trajectory measurement after the timed steps")
    ap.add_argument("--no-routines", action="store_true",
                    help="skip the per-routine (Table 1) measurement after the timed steps")
    ap.add_argument("--no-improved", action="store_true",
                    help="skip the improved (fat + Naik) operator measurement after the timed steps")
    ap.add_argument("--no-batch", action="store_true",
                    help="leave the batched solves out of the step (short runs under hardware counters)")
    ap.add_argument("--probe", type=int, nargs=4, metavar="L",
                    help="instead of the benchmark: time the plain Dslash alone on this lattice and print one "
                         "JSON line (options --fmt, --launches, --hops, --streaming)")
    ap.add_argument("--probe-batch", action="store_true",
                    help="instead of the benchmark: the 24^3x48 x16 batched solve alone, --launches times, and "
                         "one JSON line")
    ap.add_argument("--fmt", default="f64r18", choices=sorted(PROBE_FMTS))
    ap.add_argument("--nrhs", type=int, default=1, choices=(1, 4, 8, 16),
                    help="with --probe: N > 1 probes the multi-RHS Dslash, every variant")
    ap.add_argument("--launches", type=int, default=12)
    ap.add_argument("--hops", type=int, default=0, choices=(0, 1, 2, 4, 8), help="0: the library's default")
    ap.add_argument("--streaming", type=int, default=1, choices=(0, 1))
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (its domain decomposition "
              "over several GPUs is a design only); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.probe_batch:
        print(json.dumps(probe_batch(args.launches)), flush=True)
        return
    if args.probe and args.nrhs > 1:
        print(json.dumps(probe_dslash_mrhs(tuple(args.probe), args.fmt, args.nrhs, args.launches)), flush=True)
        return
    if args.probe:
        print(json.dumps(probe_dslash(tuple(args.probe), args.fmt, args.launches, args.hops, args.streaming)),
              flush=True)
        return

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
    ceil = probes(lat)
    log(f"probes {ceil}")
    Ut = torch.from_numpy(U).to(dev)
    bt = torch.from_numpy(b).to(dev)
    formats = {"f64r18": (P.LGT_F64, P.LGT_R18), "f64r12": (P.LGT_F64, P.LGT_R12),
               "f32r18": (P.LGT_F32, P.LGT_R18), "f32r12": (P.LGT_F32, P.LGT_R12),
               "bf16r12": (P.LGT_BF16, P.LGT_R12)}
    packed = {k: lat.pack_links(Ut, *v) for k, v in formats.items()}
    del Ut
    torch.cuda.synchronize()

    # standalone Dslash per format (context; `value` comes from the solves)
    dslash = {}
    for name, Up in packed.items():
        tune = None if args.no_tune else lat.tune_dslash(Up)
        vp = P.LGT_F64 if Up.prec == P.LGT_F64 else P.LGT_F32
        x = lat.pack_vec(bt, vp)
        out = lat.native_vec(vp)
        ms = statistics.median(event_times(lat, lambda: lat.dslash(Up, x, 1, out), 20, 5))
        by = alg_bytes_per_site(Up.prec, Up.recon) * Vh
        dslash[name] = {"us": round(ms * 1e3, 2), "GBps": round(by / (ms * 1e-3) / 1e9, 1),
                        "GFLOPs": round(P.DSLASH_FLOP_PER_SITE * Vh / (ms * 1e-3) / 1e9, 1),
                        "alg_bytes": by, "variant": "hops=%d streaming=%d" % lat.dslash_variant(Up.prec, Up.recon),
                        "workgroup": lat.dslash_workgroup(Up.prec, Up.recon),
                        "tune_us": {"%d/%d/%d" % k: round(v, 2) for k, v in tune.items()} if tune else None}
        log(f"dslash {name}: {dslash[name]}")
        if name == "f64r18":
            dslash_f64_out = lat.unpack_vec(out).cpu().numpy()
    # the Dslash's own link-read pattern without vectors or arithmetic (streaming
    # FP64 x 18 links, parity 1): the achievable read rate of that pattern
    sink = torch.zeros(2, dtype=torch.float64, device=dev)
    lr_ms = statistics.median(event_times(lat, lambda: lat.stream_read_links(packed["f64r18"], 1, 1, sink), 20, 5))
    link_read = {"us": round(lr_ms * 1e3, 2), "bytes": 8 * 144 * Vh,
                 "GBps": round(8 * 144 * Vh / (lr_ms * 1e-3) / 1e9, 1)}
    log(f"link-read pattern: {link_read}")

    # ---- batching workload (row a8)
    c4, c4m = li.CONFIGS["c4_24x24x24x48"], li.CONFIGS["c4_mixed"]
    batch_lat = []

    def batch_problem(Lb, link_seed, src_seed, nrhs):
        lb = P.Lattice(Lb, device=0)
        Ub = torch.from_numpy(li.links(Lb, "haar", link_seed)).to(dev)
        bb = torch.from_numpy(li.vectors(Lb, src_seed, nrhs)).to(dev)
        uh, ul = lb.pack_links(Ub, P.LGT_F64, P.LGT_R18), lb.pack_links(Ub, P.LGT_F32, P.LGT_R12)
        batch_lat.append(lb)
        return (lb, uh, ul, bb)

    big = [batch_problem(c4["L"], c4["link_seed"], c4["src_seed"], c4["nrhs"])]
    mixed = [batch_problem(Lm, sd, sd + c4m["src_seed_offset"], c4m["nrhs"]) for Lm, sd in c4m["members"]]
    # autotuner: the multi-RHS tile shape of each batched lattice (its inner Dslash)
    def vname(e, g, st):
        base = {P.LGT_MRHS_LANE: "lane", P.LGT_MRHS_VALU4: "valu4", P.LGT_MRHS_MFMA: "mfma"}[e]
        return base if e == P.LGT_MRHS_LANE else f"{base}_g{g}" + ("_lds" if st else "")

    def chosen(lb, n):
        return vname(*lb.mrhs_variant(P.LGT_F32, P.LGT_R12, n), lb.mrhs_staging(P.LGT_F32, P.LGT_R12, n))
    # the standalone multi-RHS Dslash, every variant (the batched solver's
    # inner Dslash runs the chosen engine and groups, with its own staging)
    mrhs_tune = {}
    for lb, uh, ul, bb in big + mixed:
        n = int(bb.shape[0])
        key = f"{'x'.join(map(str, lb.L))}_f32r12_N{n}"
        if args.no_tune:
            mrhs_tune[key] = {"chosen": chosen(lb, n)}
            continue
        t = lb.tune_dslash_mrhs(ul, n)
        best = min(t.values())
        mrhs_tune[key] = {"chosen": chosen(lb, n), "us": {vname(*k): round(v, 2) for k, v in t.items()},
                          "alg_bytes": lb.Vh * (8 * 48 + 2 * n * 24),
                          "GBps_best": round(lb.Vh * (8 * 48 + 2 * n * 24) / (best * 1e-6) / 1e9, 1)}
        log(f"mrhs tune {key}: {mrhs_tune[key]}")
    torch.cuda.synchronize()
    # the tuner's times come from one buffer set launched back to back, whose
    # 12-real FP32 links (and part of the input) stay in the 256 MB Infinity
    # Cache between launches; the chosen variant on the large lattice again,
    # this time over three link and vector sets in turn (1.1 GB), which no
    # launch finds in that cache
    if not args.no_tune:
        lb, _, ul, bb = big[0]
        n = int(bb.shape[0])
        key = f"{'x'.join(map(str, lb.L))}_f32r12_N{n}"
        sets = []
        for k in range(3):
            Uk = ul if k == 0 else lb.pack_links(
                torch.from_numpy(li.links(lb.L, "haar", c4["link_seed"] + 7919 * k)).to(dev), P.LGT_F32, P.LGT_R12)
            xk = torch.from_numpy(li.vectors(lb.L, c4["src_seed"] + 7919 * k, n)).to(dev)
            xk = lb.pack_vec_mrhs(xk, P.LGT_F32)
            sets.append((Uk, xk, torch.empty_like(xk)))
        for k in range(30):  # warm
            Uk, xk, yk = sets[k % 3]
            lb.dslash_mrhs(Uk, xk, k & 1, yk)
        per = []
        for rep in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(lb.stream)
            for k in range(30):
                Uk, xk, yk = sets[k % 3]
                lb.dslash_mrhs(Uk, xk, k & 1, yk)
            e1.record(lb.stream)
            torch.cuda.synchronize()
            per.append(e0.elapsed_time(e1) * 1e3 / 30)
        us = statistics.median(per)
        ab = mrhs_tune[key]["alg_bytes"]
        mrhs_tune[key]["three_sets_in_turn"] = {"us": round(us, 2), "GBps": round(ab / (us * 1e-6) / 1e9, 1),
                                               "frac": round(ab / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"mrhs three sets in turn {key}: {mrhs_tune[key]['three_sets_in_turn']}")
        del sets
        torch.cuda.synchronize()

    def batched():
        out = {}
        for key, probs in (("24x24x24x48_x16", big), ("mixed_8x8x8x8_12x12x12x12_16x16x16x32_x4", mixed)):
            t0 = time.perf_counter()
            _, res = P.cg_solve_batch(probs, c4["mass"], tol=c4["tol"], scheme=P.LGT_CG_RELIABLE, ru_interval=50)
            out[key] = (time.perf_counter() - t0, res)
        return out

    # ---- differentiation workload (row a9)
    c5 = li.CONFIGS["c5_16x16x16x32"]
    flat = P.Lattice(c5["L"], device=0)
    Uf = torch.from_numpy(li.links(c5["L"], c5["kind"], c5["link_seed"], c5["c"])).to(dev)
    phi = torch.from_numpy(li.vector(c5["L"], c5["src_seed"])).to(dev)
    if not args.no_tune:  # the Dslash variants of this lattice (the action packs its own links)
        flat.tune_dslash(flat.pack_links(Uf, P.LGT_F64, P.LGT_R18), report=False)
        flat.tune_dslash(flat.pack_links(Uf, P.LGT_F32, P.LGT_R12), report=False)

    def action_and_force():
        U = Uf.clone().requires_grad_(True)
        t0 = time.perf_counter()
        S = P.PseudofermionAction.apply(U, phi, flat, c5["mass"])
        t1 = time.perf_counter()
        S.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return {"S": float(S.detach()), "forward_s": t1 - t0, "backward_s": t2 - t1, "grad_norm": float(U.grad.norm())}

    last_x = {}

    def solves():
        out = {}
        last_x["fp64"], out["fp64"] = lat.cg_solve(packed["f64r18"], bt, args.mass, tol=1e-10, scheme=P.LGT_CG_FP64)
        out["fp64_dslash_kinds"] = lat.cg_dslash_profile()  # host-side copy of the solve's own event times
        last_x["f32r12_reliable"], out["f32r12_reliable"] = lat.cg_solve(
            packed["f64r18"], bt, args.mass, tol=1e-10, scheme=P.LGT_CG_RELIABLE, U_lo=packed["f32r12"],
            ru_interval=50)
        last_x["bf16r12_refine"], out["bf16r12_refine"] = lat.cg_solve(
            packed["f64r18"], bt, args.mass, tol=1e-10, scheme=P.LGT_CG_REFINE, U_lo=packed["bf16r12"],
            inner_tol=0.1)
        if not args.no_batch:
            out["batch"] = batched()
        out["force"] = action_and_force()
        return out

    lat.set_timing(TIMING_EVERY)
    for _ in range(args.warmup):
        solves()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    steps = [solves() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    lat.set_timing(False)

    # The headline kernel: the FP64 CG's iteration D_oe (t = D_oe p; its epilogue
    # also reads p at the same cb for the <p, A p> partials), timed by events on
    # its own dispatch packets in every sampled iteration. Its bytes: the
    # Dslash's own 8 links + input once + output once = 1248 B per output site
    # (the value), 1296 with the epilogue's read of p. The iteration's D_eo also
    # carries the update r -= alpha (4m^2 p - D_eo t): its 8 links and input,
    # p and r read, r written (Ap is never stored) = 1248 + 96 = 1344 B per
    # site, reported beside it.
    def kind(k):
        ms = sum(s["fp64_dslash_kinds"][k]["ms"] * s["fp64_dslash_kinds"][k]["n"] for s in steps)
        n = sum(s["fp64_dslash_kinds"][k]["n"] for s in steps)
        return ms / max(n, 1), n
    avg_ms, n_hi = kind("iter_doe")
    deo_ms, n_deo = kind("iter_deo_update")
    base = alg_bytes_per_site(P.LGT_F64, P.LGT_R18)
    vb = P.vec_bytes_per_site(P.LGT_F64)
    doe_bytes, deo_bytes = base + vb, base + 2 * vb
    gbs_fused = doe_bytes * Vh / (avg_ms * 1e-3) / 1e9
    gbs = base * Vh / (avg_ms * 1e-3) / 1e9
    gflops = P.DSLASH_FLOP_PER_SITE * Vh / (avg_ms * 1e-3) / 1e9
    deo = {"bytes_per_site": deo_bytes, "avg_launch_us": round(deo_ms * 1e3, 2), "launches_timed": n_deo,
           "GBps": round(deo_bytes * Vh / (deo_ms * 1e-3) / 1e9, 1),
           "frac": round(deo_bytes * Vh / (deo_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    def summ(key):
        rs = [s[key] for s in steps]
        nlo, nhi = sum(r.dslash_timed_lo for r in rs), sum(r.dslash_timed_hi for r in rs)
        out = {"seconds_median": round(statistics.median(r.seconds for r in rs), 4),
               "iters": rs[-1].iters, "updates": rs[-1].updates, "dslash_calls": rs[-1].dslash_calls,
               "true_rel_resid": rs[-1].true_rel_resid, "status": rs[-1].status}
        # sampled kernel times: inner-precision Dslash and FP64 Dslash (CG or FP64 updates)
        if nlo:
            out["dslash_lo_us_avg"] = round(1e3 * sum(r.dslash_ms_lo for r in rs) / nlo, 2)
        if nhi:
            out["dslash_f64_us_avg"] = round(1e3 * sum(r.dslash_ms_hi for r in rs) / nhi, 2)
        return out

    cg = {k: summ(k) for k in ("fp64", "f32r12_reliable", "bf16r12_refine")}
    cg["speedup_f32_vs_fp64"] = round(cg["fp64"]["seconds_median"] / cg["f32r12_reliable"]["seconds_median"], 3)
    cg["speedup_bf16_vs_fp64"] = round(cg["fp64"]["seconds_median"] / cg["bf16r12_refine"]["seconds_median"], 3)
    if not args.no_singles:
        # FP64 with 12-real links (third row rebuilt in FP64): a third fewer link bytes (once, untimed)
        _, r = lat.cg_solve(packed["f64r12"], bt, args.mass, tol=1e-10, scheme=P.LGT_CG_FP64)
        cg["fp64_r12_untimed"] = {"seconds": round(r.seconds, 4), "iters": r.iters,
                                  "true_rel_resid": r.true_rel_resid, "status": r.status}
        log(f"fp64 with 12-real links: {cg['fp64_r12_untimed']}")
        # why BF16 links take refinement: the same reliable-update scheme as FP32 (once, untimed)
        _, r = lat.cg_solve(packed["f64r18"], bt, args.mass, tol=1e-10, scheme=P.LGT_CG_RELIABLE,
                            U_lo=packed["bf16r12"], ru_interval=50, max_iter=60000, raise_on_fail=False)
        cg["bf16r12_reliable_untimed"] = {"seconds": round(r.seconds, 4), "iters": r.iters, "updates": r.updates,
                                          "true_rel_resid": r.true_rel_resid, "status": r.status}
        log(f"bf16 reliable updates: {cg['bf16r12_reliable_untimed']}")

    # batching: wall time of each batched launch vs the same right-hand sides solved one by one
    # (the single solves run once, outside the timed steps)
    singles = {}
    for key, probs in (("24x24x24x48_x16", big), ("mixed_8x8x8x8_12x12x12x12_16x16x16x32_x4", mixed)):
        if args.no_batch:
            break
        if args.no_singles:
            singles[key] = None
            continue
        tot = 0.0
        for lb, uh, ul, bb in probs:
            for j in range(bb.shape[0]):
                _, r = lb.cg_solve(uh, bb[j].contiguous(), c4["mass"], tol=c4["tol"], scheme=P.LGT_CG_RELIABLE,
                                   U_lo=ul, ru_interval=50)
                tot += r.seconds
        singles[key] = tot
    batch = {}
    for key in singles:
        rs = [s["batch"][key] for s in steps]
        last = [r for per in rs[-1][1] for r in per]
        med = statistics.median(r[0] for r in rs)
        sg = singles[key]
        batch[key] = {"seconds_median": round(med, 4), "sum_of_single_solves_s": None if sg is None else round(sg, 4),
                      "speedup_vs_single_solves": None if sg is None else round(sg / med, 3),
                      "iters_max": max(r.iters for r in last), "updates_max": max(r.updates for r in last),
                      "true_rel_resid_max": max(r.true_rel_resid for r in last),
                      "status_all_ok": all(r.status == 0 for r in last)}
    # batched solver: phase profile of one more solve of each batch (workgroup
    # 0's clock inside the persistent launch; event-timed kernels of the
    # launched form, summed over its problems, with no barrier waits; with
    # timing on, its launches go out one by one instead of as graph replays),
    # and the roofline of an iteration: per even site and
    # right-hand side (FP32 x 12 inner links shared by the N right-hand sides),
    # step 1 reads r and p at the neighbours once (48 B) and writes t and p'
    # (48 B) plus 384/N B of links, step 2 reads t once, p', x and r (96 B) and
    # writes x and r (48 B) plus 384/N B of links; where p' = r + beta p runs as
    # a pass of its own (the launched form, and the persistent launch from 2^21
    # (site, rhs) pairs on) that pass reads r and p and writes p' (72 B) and
    # step 1 reads p' and writes t (48 B)
    for key, probs in (("24x24x24x48_x16", big), ("mixed_8x8x8x8_12x12x12x12_16x16x16x32_x4", mixed)):
        if args.no_batch:
            break
        lb0 = probs[0][0]
        lb0.set_timing(1)
        _, res = P.cg_solve_batch(probs, c4["mass"], tol=c4["tol"], scheme=P.LGT_CG_RELIABLE, ru_interval=50)
        lb0.set_timing(0)
        prof = lb0.batch_profile()
        its = max(prof.pop("iters"), 1)
        launched = prof["wait1"] == 0.0 and prof["wait2"] == 0.0
        two_pass = prof["step1_p"] > 0.0
        alg = sum(lb.Vh * (int(bb.shape[0]) * ((120 if two_pass else 96) + 144) + 2 * 384)
                  for lb, _, _, bb in probs)
        batch[key]["form"] = "launched" if launched else ("persistent, two-pass step 1" if two_pass else "persistent")
        # the whole iteration from the untimed solves (events around every
        # launch of the launched form slow the profiled one down)
        per_it_us = 1e6 * batch[key]["seconds_median"] / max(batch[key]["iters_max"], 1)
        # the FP64 updates are amortised over the iterations; the roofline is
        # that of the inner iteration (steps 1-3, their waits and scalar steps)
        inner_us = 1e3 * sum(v for k, v in prof.items() if k not in ("setup_and_final", "fp64_updates")) / its
        basis = "inner steps (kernels, waits, scalar steps)"
        if launched and len(probs) > 1:
            # the problems' kernels overlap in time: their summed times say
            # nothing of the iteration's; take the whole iteration instead
            inner_us = 1e6 * batch[key]["seconds_median"] / max(batch[key]["iters_max"], 1)
            basis = "whole iteration, wall clock (the problems run concurrently)"
        for k in ("step3_update", "wait3"):  # the update is part of step 2
            prof.pop(k, None)
        batch[key]["phases_us_per_iter"] = {k: round(1e3 * v / its, 2) for k, v in prof.items()}
        batch[key]["roofline_inner_iteration"] = {
            "bound": "hbm", "alg_bytes": alg, "us": round(inner_us, 2), "us_basis": basis,
            "achieved_GBps": round(alg / (inner_us * 1e-6) / 1e9, 1), "peak": HBM_PEAK_GBS,
            "frac": round(alg / (inner_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "whole_iteration_us": round(per_it_us, 2)}
        log(f"batch profile {key}: {batch[key]['phases_us_per_iter']} {batch[key]['roofline_inner_iteration']}")

    # the single-RHS CG per iteration at 32^4: Dslash pair, the vector kernels
    # and the rest (launch gaps, the reliable updates' other kernels), from one
    # more solve per scheme with every 16th iteration timed
    lat.set_timing(TIMING_EVERY)
    breakdown = {}
    for key, kw in (("fp64", dict(scheme=P.LGT_CG_FP64)),
                    ("f32r12_reliable", dict(scheme=P.LGT_CG_RELIABLE, U_lo=packed["f32r12"], ru_interval=50))):
        _, r = lat.cg_solve(packed["f64r18"], bt, args.mass, tol=1e-10, **kw)
        vk = lat.cg_profile()
        it = max(r.iters, 1)
        if key == "fp64":
            pair = 2e3 * r.dslash_ms_hi / max(r.dslash_timed_hi, 1)
            ru = (r.updates * pair) / it
        else:
            pair = 2e3 * r.dslash_ms_lo / max(r.dslash_timed_lo, 1)
            ru = (r.updates * 2e3 * r.dslash_ms_hi / max(r.dslash_timed_hi, 1)) / it
        vec = {k: round(1e3 * vk[k], 2) for k in ("xpay", "update", "beta_step", "alpha_step")}
        total = 1e6 * r.seconds / it
        breakdown[key] = {"total_us": round(total, 2), "dslash_pair_us": round(pair, 2), **{k + "_us": v for k, v in vec.items()},
                          "fp64_update_dslash_us_amortised": round(ru, 2),
                          "rest_us": round(total - pair - sum(vec.values()) - ru, 2), "iters": r.iters,
                          "host_waits": "none: the host enqueues 50 iterations ahead and polls the state one chunk behind"}
        log(f"cg breakdown {key}: {breakdown[key]}")
    lat.set_timing(0)
    cg["per_iteration_breakdown"] = breakdown

    # differentiation: whole S and dS/dU per step, and the force kernel alone
    fs = [s["force"] for s in steps]
    Upf = flat.pack_links(Uf, P.LGT_F64, P.LGT_R18)
    Xf, _ = flat.cg_solve(Upf, phi, c5["mass"], tol=1e-12)
    fk = statistics.median(event_times(flat, lambda: flat.force(Upf, Xf), 10, 3))
    Vf = int(np.prod(c5["L"]))
    force_bytes = (Vf // 2) * 96 + (Vf // 2) * alg_bytes_per_site(P.LGT_F64, P.LGT_R18) + 4 * Vf * 144 + Vf * 48
    force = {"lattice": list(c5["L"]), "S": fs[-1]["S"],
             "forward_s_median": round(statistics.median(f["forward_s"] for f in fs), 4),
             "backward_s_median": round(statistics.median(f["backward_s"] for f in fs), 4),
             # lgt_force = pack X + Y = D_oe X + outer-product kernel writing G (4 V x 144 B)
             "lgt_force_us": round(fk * 1e3, 2),
             "lgt_force_GBps": round(force_bytes / (fk * 1e-3) / 1e9, 1), "lgt_force_alg_bytes": force_bytes}
    # the same action with the mixed-precision forward solve (once, untimed)
    grads = {}
    for mixed in (False, True):
        Ug = Uf.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Sg = P.PseudofermionAction.apply(Ug, phi, flat, c5["mass"], 1e-12, 100000, mixed)
        torch.cuda.synchronize()
        grads[mixed] = (float(Sg), time.perf_counter() - t0)
        Sg.backward()
        grads[mixed] += (Ug.grad.detach().clone(),)
        del Ug
    force["mixed_forward"] = {"seconds": round(grads[True][1], 4), "fp64_seconds": round(grads[False][1], 4),
                              "S_rel_diff": abs(grads[True][0] - grads[False][0]) / abs(grads[False][0]),
                              "grad_rel_diff": float((grads[True][2] - grads[False][2]).norm()
                                                     / grads[False][2].norm())}
    # central finite differences over 64 random link directions (128 solves),
    # against dS/dU of the FP64 forward solve
    fd_s, fd_err = fd_check(flat, Uf, phi, c5["mass"], grads[False][2], c5["L"], c5["fd_seed"], 64)
    force["fd_64_directions"] = {"seconds": round(fd_s, 3), "max_rel_dev_from_grad": fd_err, "eps": 1e-6}
    del grads
    small, small_sols = small_configs(args)

    # improved (fat + Naik) operator at 32^4, measured after the timed steps:
    # standalone Dslash per format and link-load kind, FP64 vs FP32 reliable-update CG
    improved = None
    if not args.no_improved:
        ci = li.CONFIGS["imp_32x32x32x32"]
        Fi, Ni = li.improved_links(L, ci["link_seed"])
        bi = torch.from_numpy(li.vector(L, ci["src_seed"])).to(dev)
        Ft, Nt = torch.from_numpy(Fi).to(dev), torch.from_numpy(Ni).to(dev)
        del Fi, Ni
        imp_packed = {"f64r18": (lat.pack_links(Ft, P.LGT_F64, P.LGT_R18), lat.pack_links(Nt, P.LGT_F64, P.LGT_R18)),
                      "f32r18": (lat.pack_links(Ft, P.LGT_F32, P.LGT_R18), lat.pack_links(Nt, P.LGT_F32, P.LGT_R18))}
        del Ft, Nt
        improved = {"lattice": list(L), "flop_per_site": P.IMPROVED_FLOP_PER_SITE, "dslash": {}}
        for name, (Fp, Np) in imp_packed.items():
            prec = Fp.prec
            vb = P.vec_bytes_per_site(prec)
            by = (16 * P.link_bytes_per_dir(prec, P.LGT_R18) + 2 * vb) * Vh
            xi = lat.pack_vec(bi, prec)
            oi = lat.native_vec(prec)
            t = {}
            for streaming in (1, 0):
                lat.set_dslash_improved_variant(prec, streaming, 256)
                t[streaming] = statistics.median(event_times(lat, lambda: lat.dslash_improved(Fp, Np, xi, 1, oi), 20, 5))
            best = min(t, key=t.get)
            lat.set_dslash_improved_variant(prec, best, 256)
            ms = t[best]
            improved["dslash"][name] = {"us": round(ms * 1e3, 2), "GBps": round(by / (ms * 1e-3) / 1e9, 1),
                                        "GFLOPs": round(P.IMPROVED_FLOP_PER_SITE * Vh / (ms * 1e-3) / 1e9, 1),
                                        "alg_bytes": by, "streaming_links": best,
                                        "us_streaming_cached": [round(t[1] * 1e3, 2), round(t[0] * 1e3, 2)]}
            log(f"improved dslash {name}: {improved['dslash'][name]}")
        (F64p, N64p), (F32p, N32p) = imp_packed["f64r18"], imp_packed["f32r18"]
        lat.set_timing(TIMING_EVERY)
        cgs = {}
        for key, kw in (("fp64", dict(scheme=P.LGT_CG_FP64)),
                        ("f32r18_reliable", dict(scheme=P.LGT_CG_RELIABLE, F_lo=F32p, N_lo=N32p, ru_interval=50))):
            _, r = lat.cg_solve_improved(F64p, N64p, bi, ci["mass"], tol=ci["tol"], **kw)
            cgs[key] = {"seconds": round(r.seconds, 4), "iters": r.iters, "updates": r.updates,
                        "true_rel_resid": r.true_rel_resid, "status": r.status}
            if r.dslash_timed_hi:
                cgs[key]["dslash_f64_us_avg"] = round(1e3 * r.dslash_ms_hi / r.dslash_timed_hi, 2)
            if r.dslash_timed_lo:
                cgs[key]["dslash_lo_us_avg"] = round(1e3 * r.dslash_ms_lo / r.dslash_timed_lo, 2)
            log(f"improved cg {key}: {cgs[key]}")
        lat.set_timing(0)
        cgs["speedup_f32_vs_fp64"] = round(cgs["fp64"]["seconds"] / cgs["f32r18_reliable"]["seconds"], 3)
        improved["cg"] = cgs
        del imp_packed, F64p, N64p, F32p, N32p
        # link fattening of the headline Haar field with the asqtad weights:
        # median of 5 calls and the FP64 rate at the 20286 flop per link the
        # kernels execute (86 complex 3x3 products at 216 flop, 8 per complex
        # multiply-add, plus the weighted sums; summing every path separately
        # would take 40320), then the FP64 improved CG on the fattened fields
        Uh = torch.from_numpy(U).to(dev)
        Ff, Nf = lat.fatten_links(Uh)
        tf = statistics.median(event_times(lat, lambda: lat.fatten_links(Uh, F=Ff, N=Nf), 5, 1))
        fat_flop = 20286 * 4 * V
        # its chain rule (the improved force's last step), with F and N standing
        # in for dS/dF and dS/dN: 222 complex 3x3 products per link
        Gv = lat.fatten_links_vjp(Uh, Ff, Nf)
        tv = statistics.median(event_times(lat, lambda: lat.fatten_links_vjp(Uh, Ff, Nf, G=Gv), 5, 1))
        vjp_flop = 222 * 216 * 4 * V
        Ffp, Nfp = lat.pack_links(Ff, P.LGT_F64, P.LGT_R18), lat.pack_links(Nf, P.LGT_F64, P.LGT_R18)
        del Uh, Ff, Nf, Gv
        _, r = lat.cg_solve_improved(Ffp, Nfp, bi, ci["mass"], tol=ci["tol"])
        improved["fatten"] = {"ms": round(tf, 3), "flop_per_link": 20286, "path_sum_flop_per_link": 40320,
                              "GFLOPs": round(fat_flop / (tf * 1e-3) / 1e9, 1),
                              "frac_of_fp64_vector_peak": round(fat_flop / (tf * 1e-3) / 78.6e12, 4),
                              "vjp": {"ms": round(tv, 3), "products_per_link": 222,
                                      "GFLOPs": round(vjp_flop / (tv * 1e-3) / 1e9, 1),
                                      "frac_of_fp64_vector_peak": round(vjp_flop / (tv * 1e-3) / 78.6e12, 4)},
                              "cg_fp64_on_fattened_haar": {"seconds": round(r.seconds, 4), "iters": r.iters,
                                                           "true_rel_resid": r.true_rel_resid, "status": r.status}}
        log(f"fatten: {improved['fatten']}")
        del Ffp, Nfp

    # HMC trajectory around the solve (the paper's application-level comparison,
    # Table 4): FP64 CG vs FP32-12 reliable-update CG inside the same trajectory
    hmc_res = None
    if not args.no_hmc:
        ch = li.CONFIGS["hmc_16x16x16x16"]
        hl = P.Lattice(ch["L"], device=0)
        U0 = torch.from_numpy(li.links(ch["L"], ch["kind"], ch["link_seed"], ch["c"])).to(dev)
        Pm = li.momenta(ch["L"], ch["mom_seed"])
        P0 = torch.from_numpy(np.ascontiguousarray(np.stack([Pm.real, Pm.imag], -1))).to(dev)
        Re = torch.from_numpy(li.vector(ch["L"], ch["re_seed"])).to(dev)
        Ro = torch.from_numpy(li.vector(ch["L"], ch["ro_seed"])).to(dev)
        u = li.uniform(ch["u_seed"])
        kw = dict(beta=ch["beta"], mass=ch["mass"], eps=ch["eps"], nsteps=ch["nsteps"], u=u, tol=ch["tol"])
        if not args.no_tune:  # the trajectory packs F64 x 18 and F32 x 12 links of this lattice
            hl.tune_dslash(hl.pack_links(U0, P.LGT_F64, P.LGT_R18), report=False)
            hl.tune_dslash(hl.pack_links(U0, P.LGT_F32, P.LGT_R12), report=False)
        hl.hmc_trajectory(U0.clone(), P0.clone(), Re, Ro, **dict(kw, nsteps=1))  # allocate workspace
        hmc_res = {"lattice": list(ch["L"]), "beta": ch["beta"], "mass": ch["mass"], "eps": ch["eps"],
                   "nsteps": ch["nsteps"], "tol": ch["tol"]}
        for key, sch in (("fp64", P.LGT_CG_FP64), ("f32r12_reliable", P.LGT_CG_RELIABLE)):
            r = hl.hmc_trajectory(U0.clone(), P0.clone(), Re, Ro, scheme=sch, **kw)
            hmc_res[key] = {"seconds": round(r["seconds"], 4), "dH": r["dH"], "accepted": r["accepted"],
                            "cg_solves": r["cg_solves"], "cg_iters": r["cg_iters"]}
            log(f"hmc {key}: {hmc_res[key]}")
        hmc_res["speedup_f32_vs_fp64"] = round(hmc_res["fp64"]["seconds"] / hmc_res["f32r12_reliable"]["seconds"], 3)
        # the same trajectory with the improved operator (the application's
        # action): asqtad weights with the tadpole factor u0 = (mean plaquette / 3)^(1/4)
        # of the starting field, fattening and its chain rule at every step
        u0 = (hl.plaquette(U0) / (6 * li.volume(ch["L"])) / 3.0) ** 0.25
        w = P.asqtad_coeffs(u0)
        if not args.no_tune:  # the improved operator's own variants, on the fattened starting field
            F0, N0 = hl.fatten_links(U0, w)
            for prec in (P.LGT_F64, P.LGT_F32):
                hl.tune_dslash_improved(hl.pack_links(F0, prec, P.LGT_R18), hl.pack_links(N0, prec, P.LGT_R18))
            del F0, N0
        hl.hmc_trajectory_improved(U0.clone(), P0.clone(), Re, Ro, coeffs=w, **dict(kw, nsteps=1))
        imp = {"u0": round(u0, 6)}
        for key, sch in (("fp64", P.LGT_CG_FP64), ("f32r18_reliable", P.LGT_CG_RELIABLE)):
            r = hl.hmc_trajectory_improved(U0.clone(), P0.clone(), Re, Ro, coeffs=w, scheme=sch, **kw)
            imp[key] = {"seconds": round(r["seconds"], 4), "dH": r["dH"], "accepted": r["accepted"],
                        "cg_solves": r["cg_solves"], "cg_iters": r["cg_iters"]}
            log(f"hmc improved {key}: {imp[key]}")
        imp["speedup_f32_vs_fp64"] = round(imp["fp64"]["seconds"] / imp["f32r18_reliable"]["seconds"], 3)
        hmc_res["improved"] = imp
        hl.close()
        del U0, P0, Re, Ro

    # Table 1 routines one at a time (the paper times each routine on its own,
    # Table 2): n independent calls per launch, 20 launches back to back between
    # the events. "hbm": n = 2^24 calls, operands streamed from HBM; "cache":
    # operands of about 128 MB (n <= 2^20), which stay in the 256 MB Infinity
    # Cache from one launch to the next.
    routines = None
    if not args.no_routines:
        routines = {}
        gen = torch.Generator(device=dev)
        gen.manual_seed(7001)
        reps = 20
        for name, (rid, ka, kb, kc, fl) in P.ROUTINES.items():
            routines[name] = {"flop_per_call": fl}
            for prec, dt, eb in (("f64", torch.float64, 16), ("f32", torch.float32, 8)):
                per_call = (P.PLANES[ka] + P.PLANES[kb] + P.PLANES[kc]) * eb
                row = {}
                for label, n in (("hbm", 1 << 24), ("cache", min(1 << 20, (128 << 20) // per_call // 256 * 256))):
                    ra = torch.randn((P.PLANES[ka], n, 2), generator=gen, device=dev, dtype=dt)
                    rb = torch.randn((P.PLANES[kb], n, 2), generator=gen, device=dev, dtype=dt)
                    rc = torch.empty((P.PLANES[kc], n, 2), device=dev, dtype=dt)

                    def burst():
                        for _ in range(reps):
                            P.routine(lat, name, ra, rb, 0.5, out=rc)

                    ms = statistics.median(event_times(lat, burst, 5, 1)) / reps
                    row[label] = {"n": n, "ns_per_call": round(ms * 1e6 / n, 4),
                                  "GBps": round(per_call * n / (ms * 1e-3) / 1e9, 1),
                                  "GFLOPs": round(fl * n / (ms * 1e-3) / 1e9, 1)}
                    del ra, rb, rc
                routines[name][prec] = row
            log(f"routine {name}: {routines[name]}")
        torch.cuda.empty_cache()

    cpu, oracle_errors = None, None
    if not args.no_cpu_baseline:
        gpu_results = {"x32": {k: v.cpu().numpy() for k, v in last_x.items()}, "dslash_in": b,
                       "dslash_out": dslash_f64_out, "small": small_sols, "fp64_iters": cg["fp64"]["iters"]}
        cpu, oracle_errors = cpu_leg(L, U, b, args.mass, args.cpu_budget, gpu_results)
        log(f"cpu leg: {cpu}; oracle errors: {oracle_errors}")

    traffic = measured_traffic()
    line = {
        "metric": METRIC, "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"staggered Dslash in even-odd CG, {'x'.join(map(str, L))} lattice, Haar SU(3) "
                               f"links, m={args.mass}, tol 1e-10; step = FP64 CG + FP32-12 reliable-update CG "
                               f"+ BF16-12 refinement CG + batched CG (24^3x48 x16; 8^4, 12^4, 16^3x32 x4) "
                               f"+ S and dS/dU at 16^3x32", "lattice": list(L), "mass": args.mass},
        "gflops": round(gflops, 1),
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / (avg_ms * 1e-3) / 1e9, 1),
                     "traffic_bytes_per_launch": traffic,
                     "kernel": "k_dslash<LinkF64R18, EPI_PAP, *> inside the FP64 CG: the iteration's D_oe "
                               "(t = D_oe p with the <p, A p> partials)",
                     "alg_bytes_per_site": base, "alg_bytes_per_launch": base * Vh,
                     "avg_launch_us": round(avg_ms * 1e3, 2), "launches_timed": n_hi,
                     "with_epilogue_reads": {"bytes_per_site": doe_bytes, "GBps": round(gbs_fused, 1),
                                             "frac": round(gbs_fused / HBM_PEAK_GBS, 4)},
                     "deo_with_update": deo,
                     "measured_ceiling_GBps": {"read_1GiB_single_stream": ceil["read_GBps"],
                                               "copy_1GiB": ceil["copy_GBps"],
                                               "dslash_link_read_pattern": link_read["GBps"]},
                     "frac_of_link_read_pattern": round(gbs / link_read["GBps"], 4),
                     "link_read_pattern": link_read},
        "cg": cg,
        "batch": batch,
        "mrhs_tune": mrhs_tune,
        "improved": improved,
        "hmc": hmc_res,
        "routines": routines,
        "force": force,
        "dslash_standalone": dslash,
        "small_configs": small,
        "cpu_baseline": cpu,
        "oracle_errors": oracle_errors,
        "paper_context": paper_context(),
    }
    print(json.dumps(line), flush=True)
    lat.close()
    flat.close()
    for lb in batch_lat:
        lb.close()


if __name__ == "__main__":
    main()
