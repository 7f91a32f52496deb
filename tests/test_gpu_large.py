"""The largest lattice of the GPU tests: 64^4 (16.8M sites, 8.4M per parity).

Its FP64 18-real link field and the fermion-force gradient are 9.7 GB each,
so the plane bases of the packed links, of the canonical input and of the
gradient lie far beyond 4 GiB, and the CG runs with one alpha workgroup per
iteration (more than 3584 Dslash workgroups). The improved operator's
three-link hops are checked on the same field. Links are independent draws
from a pool of 2^16 Haar matrices (per-link QR would take minutes on the
host); every output is compared with the FP64 oracle over the whole lattice.

Tolerances as in the other parity tests: FP64 1e-12 (norm-wise and per
component), FP32 links 32 u32, BF16 links 8 u16; CG: the oracle's true
residual of the GPU's x.
"""
import numpy as np
import pytest

import lgt_inputs as li
import oracle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1309_0551_amd")

pytestmark = pytest.mark.gpu

L = (64, 64, 64, 64)
U32 = 2.0 ** -24
U16 = 2.0 ** -9


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda", 0)
    print("64^4 inputs", flush=True)
    U = li.links(L, "haar_pool", 6401)
    with P.Lattice(L) as lat:
        Ud = torch.from_numpy(U).to(dev)
        packs = {
            "f64r18": lat.pack_links(Ud, P.LGT_F64, P.LGT_R18),
            "f32r12": lat.pack_links(Ud, P.LGT_F32, P.LGT_R12),
            "bf16r12": lat.pack_links(Ud, P.LGT_BF16, P.LGT_R12),
        }
        del Ud
        torch.cuda.empty_cache()
        yield dev, lat, U, packs
        del packs
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fmt,tol", [("f64r18", 1e-12), ("f32r12", 32 * U32), ("bf16r12", 8 * U16)])
def test_dslash_64(big, fmt, tol):
    dev, lat, U, packs = big
    Up = packs[fmt]
    vec_prec = P.LGT_F64 if fmt == "f64r18" else P.LGT_F32
    for par in (0, 1):
        print("dslash 64^4", fmt, "parity", par, flush=True)
        chi = li.vector(L, 6410 + par)
        out = lat.unpack_vec(lat.dslash(Up, lat.pack_vec(torch.from_numpy(chi).to(dev), vec_prec), par),
                             vec_prec).cpu().numpy()
        ref = oracle.dslash(L, U, chi, par)
        assert _rel(out, ref) <= tol
        assert np.abs(out - ref).max() <= tol * np.abs(ref).max()


def test_improved_dslash_64(big):
    """The improved operator's 16 hops (one-link and three-link) at 64^4, with the
    9.7 GB link field serving as both its fat and its Naik field."""
    dev, lat, U, packs = big
    Up = packs["f64r18"]
    for par in (0, 1):
        print("improved dslash 64^4 parity", par, flush=True)
        chi = li.vector(L, 6440 + par)
        out = lat.unpack_vec(lat.dslash_improved(Up, Up, lat.pack_vec(torch.from_numpy(chi).to(dev)), par)).cpu().numpy()
        ref = oracle.dslash_imp(L, U, U, chi, par)
        assert _rel(out, ref) <= 1e-12
        assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


def test_force_64(big):
    """9.7 GB gradient: compared with the oracle in slices of the link field."""
    dev, lat, U, packs = big
    print("force 64^4", flush=True)
    X = li.vector(L, 6420)
    G = lat.force(packs["f64r18"], torch.from_numpy(X).to(dev), scale=1.0)
    Gr = oracle.force(L, U, X)
    num = den = 0.0
    gmax = dmax = 0.0
    step = 1 << 22
    for mu in range(4):
        for s0 in range(0, Gr.shape[1], step):
            g = G[mu, s0:s0 + step].cpu().numpy()
            r = Gr[mu, s0:s0 + step]
            d = g - r
            num += float(np.sum(d * d))
            den += float(np.sum(r * r))
            dmax = max(dmax, float(np.abs(d).max()))
            gmax = max(gmax, float(np.abs(r).max()))
    del G
    torch.cuda.empty_cache()
    assert (num / den) ** 0.5 <= 1e-12
    assert dmax <= 1e-12 * gmax


@pytest.mark.parametrize("scheme", ["fp64", "reliable_f32r12"])
def test_cg_64(big, scheme):
    dev, lat, U, packs = big
    print("cg 64^4", scheme, flush=True)
    b = li.vector(L, 6430)
    kw = dict(scheme=P.LGT_CG_FP64) if scheme == "fp64" else dict(scheme=P.LGT_CG_RELIABLE, U_lo=packs["f32r12"])
    x, res = lat.cg_solve(packs["f64r18"], torch.from_numpy(b).to(dev), 0.1, tol=1e-10, **kw)
    xh = x.cpu().numpy()
    r = b - oracle.apply_A(L, U, 0.1, xh)
    true = float(np.linalg.norm(r) / np.linalg.norm(b))
    assert true <= 1.05e-10
    assert true == pytest.approx(res.true_rel_resid, rel=1e-6)
