"""Time the one-link Dslash on a lattice of any size.

    python -m paper_1309_0551_amd.dslash_probe 64 64 64 64 --fmt f64r18 --launches 12

Packs a link field whose links are independent draws from a pool of 2^16
Haar matrices (built on the device, so lattices of many GB take seconds),
runs `--launches` plain Dslash applications (output parity odd) with the
chosen variant and prints the mean kernel time, measured with events on the
launches' own stream, and the algorithmic bandwidth: per output site 8 links,
the input vector once and the output vector once (1248 B for FP64 x 18 links).
Run it under rocprofv3 to read the same launches' counters.
"""
from __future__ import annotations

import argparse
import math

import torch

import lgt_inputs as li

from . import lgt as B

FMTS = {"f64r18": (B.LGT_F64, B.LGT_R18), "f64r12": (B.LGT_F64, B.LGT_R12), "f32r18": (B.LGT_F32, B.LGT_R18),
        "f32r12": (B.LGT_F32, B.LGT_R12), "bf16r12": (B.LGT_BF16, B.LGT_R12)}
LINK_BYTES = {"f64r18": 144, "f64r12": 96, "f32r18": 72, "f32r12": 48, "bf16r12": 24}


def main(argv=None) -> dict:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("L", type=int, nargs=4)
    ap.add_argument("--fmt", default="f64r18", choices=sorted(FMTS))
    ap.add_argument("--launches", type=int, default=12)
    ap.add_argument("--hops", type=int, default=8, choices=(1, 2, 4, 8))
    ap.add_argument("--streaming", type=int, default=1, choices=(0, 1))
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("dslash_probe needs a GPU")
    dev = torch.device("cuda", 0)
    L = tuple(a.L)
    V = math.prod(L)
    prec, recon = FMTS[a.fmt]
    vec_prec = B.LGT_F64 if prec == B.LGT_F64 else B.LGT_F32
    vec_bytes = 48 if vec_prec == B.LGT_F64 else 24
    pool = torch.from_numpy(li.to_real(li.haar_su3(1 << 16, li.rng(7)))).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(1)
    with B.Lattice(L) as lat:
        U = pool[torch.randint(0, pool.shape[0], (4 * V,), device=dev, generator=g)].reshape(4, V, 3, 3, 2)
        Up = lat.pack_links(U.contiguous(), prec, recon)
        del U
        torch.cuda.empty_cache()
        lat.set_dslash_variant(prec, recon, a.hops, a.streaming)
        x = lat.pack_vec(torch.randn(lat.Vh, 3, 2, dtype=torch.float64, device=dev, generator=g), vec_prec)
        y = torch.empty_like(x)
        lat.dslash(Up, x, 1, y)  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(a.launches):
            lat.dslash(Up, x, 1, y)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / a.launches
    alg = lat.Vh * (8 * LINK_BYTES[a.fmt] + 2 * vec_bytes)
    out = {"L": list(L), "fmt": a.fmt, "hops": a.hops, "streaming": a.streaming, "launches": a.launches,
           "us_per_launch": round(us, 2), "alg_bytes_per_launch": alg, "alg_GBps": round(alg / us / 1e3, 1)}
    print(out, flush=True)
    return out


if __name__ == "__main__":
    main()
