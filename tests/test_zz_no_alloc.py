"""lgt_force_noalloc, the force entry point that allocates nothing, through the
C ABI: two calls in a row (the second on a smaller lattice, so the shared
scratch array still holds the first call's larger vectors) each equal to
lgt_force bit for bit and to the oracle's force; a lattice beyond the scratch
limit is rejected on the host before anything runs."""
import ctypes as C

import numpy as np
import pytest

import lgt_inputs as li
import oracle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1309_0551_amd")
from paper_1309_0551_amd import lgt as B  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _force_noalloc(lat, Up, X, scale):
    G = torch.empty((4, lat.V, 3, 3, 2), dtype=torch.float64, device=lat.device)
    d = Up.desc()
    st = P.lib().lgt_force_noalloc(lat._ctx, C.byref(d), X.data_ptr(), float(scale), G.data_ptr())
    assert st == 0, P.lib().lgt_last_error().decode()
    return G


@pytest.mark.parametrize("order", ["large_then_small", "small_then_large"])
def test_force_noalloc_matches_force(dev, order):
    cases = [((8, 8, 8, 12), (1, 1, 1, -1), 701), ((6, 4, 6, 8), (1, 1, 1, 1), 711)]
    if order == "small_then_large":
        cases = cases[::-1]
    for L, bc, seed in cases:
        print("force_noalloc", L, bc, flush=True)
        U = li.links(L, "expih", seed, c=0.5)
        X = li.vector(L, seed + 1)
        with P.Lattice(L, bc) as lat:
            Up = lat.pack_links(torch.from_numpy(U).to(dev), P.LGT_F64, P.LGT_R18)
            Xt = torch.from_numpy(X).to(dev)
            got = _force_noalloc(lat, Up, Xt, 1.5)
            ref = lat.force(Up, Xt, scale=1.5)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (L, "noalloc differs from lgt_force")
        want = 1.5 * oracle.force(L, U, X, bc)
        g = got.cpu().numpy()
        assert np.linalg.norm(g - want) <= 1e-12 * np.linalg.norm(want)


def test_force_noalloc_rejects_beyond_the_limit(dev):
    # V/2 = 720896 > 699050: rejected before pointers are even looked at
    with P.Lattice((32, 32, 32, 44)) as lat:
        d = B._Links(None, P.LGT_F64, P.LGT_R18)
        d.ptr = 256
        st = P.lib().lgt_force_noalloc(lat._ctx, C.byref(d), None, 1.0, None)
        assert st == P.LgtError(-8, "").status
        assert "scratch" in P.lib().lgt_last_error().decode()
