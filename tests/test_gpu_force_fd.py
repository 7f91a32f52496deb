"""Differentiation form at full size: dS/dU from the fermion-force kernel (through
torch.autograd) against central finite differences of the GPU action and against
the oracle's gradient.

Workload: 16^3 x 32, links exp(0.5 i H), m = 0.05, phi Gaussian, 64 random link
directions (uniform (mu, site), Gaussian E in R^18 normalised), eps = 1e-6.

S(U +- eps E) is taken from the variational estimate
    S~ = 2 Re <phi, x> - <x, A x>,   x ~ A^-1 phi by the FP64 CG to 1e-12,
whose error -r^dag A^-1 r is quadratic in the residual (~1e-17 here). The
difference S~+ - S~- is summed from element-wise differences, so its rounding
error is relative to the difference itself rather than to S (~1e4): with eps =
1e-6 a difference of two separately summed S values would carry ~1e-5 of
rounding noise into each derivative.
"""
import numpy as np
import pytest

import lgt_inputs as li
import oracle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1309_0551_amd")

pytestmark = pytest.mark.gpu

L = (16, 16, 16, 32)
MASS = 0.05
EPS = 1e-6
NDIR = 64


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda", 0)
    U = li.links(L, "expih", 5001, c=0.5)
    phi = li.vector(L, 5002)
    lat = P.Lattice(L)
    yield dev, U, phi, lat
    lat.close()


def _pieces(lat, Ut, phit):
    """Per-element terms of S~ = 2 Re <phi, x> - <x, A x> for links Ut."""
    Up = lat.pack_links(Ut, P.LGT_F64, P.LGT_R18)
    x, res = lat.cg_solve(Up, phit, MASS, tol=1e-12)
    assert res.status == 0
    xn = lat.pack_vec(x)
    Dx = lat.unpack_vec(lat.dslash(Up, lat.dslash(Up, xn, P.LGT_ODD), P.LGT_EVEN))
    Ax = 4 * MASS * MASS * x - Dx
    # Re conj(a) b per complex element, a, b as [..., 2] real views
    t1 = 2.0 * (phit[..., 0] * x[..., 0] + phit[..., 1] * x[..., 1])
    t2 = x[..., 0] * Ax[..., 0] + x[..., 1] * Ax[..., 1]
    return t1 - t2, res


def test_force_central_differences_64_directions(setup):
    dev, U, phi, lat = setup
    Ut = torch.from_numpy(U).to(dev).requires_grad_(True)
    phit = torch.from_numpy(phi).to(dev)
    S = P.PseudofermionAction.apply(Ut, phit, lat, MASS, 1e-12)
    S.backward()
    G = Ut.grad.detach()
    mus, sites, Es = li.fd_directions(L, 5004, NDIR)
    an, fd = [], []
    base = Ut.detach()
    for mu, s, E in zip(mus, sites, Es):
        Et = torch.from_numpy(E).to(dev)
        Up, Um = base.clone(), base.clone()
        Up[mu, s] += EPS * Et
        Um[mu, s] -= EPS * Et
        tp, _ = _pieces(lat, Up, phit)
        tm, _ = _pieces(lat, Um, phit)
        fd.append(float((tp - tm).sum()) / (2 * EPS))
        an.append(float((G[mu, s] * Et).sum()))
    an, fd = np.array(an), np.array(fd)
    err = np.abs(fd - an)
    scale = np.maximum(np.abs(an), np.median(np.abs(an)))
    print(f"FD check: max |fd-an| = {err.max():.3e}, max rel = {(err / scale).max():.3e}, "
          f"median |an| = {np.median(np.abs(an)):.3e}", flush=True)
    # central-difference truncation O(eps^2) ~ 1e-12; CG error in S~ ~ 1e-17 / eps
    assert (err <= 1e-5 * scale).all(), (err / scale).max()


def test_force_matches_oracle_gradient(setup):
    dev, U, phi, lat = setup
    Ut = torch.from_numpy(U).to(dev).requires_grad_(True)
    S = P.PseudofermionAction.apply(Ut, torch.from_numpy(phi).to(dev), lat, MASS, 1e-12)
    S.backward()
    G = Ut.grad.cpu().numpy()
    st, Xo, it, rr = oracle.cg(L, U, MASS, phi, tol=1e-12)
    assert st == 0
    Go = oracle.force(L, U, Xo)
    So = oracle.cdot(phi, Xo).real
    # both X satisfy |X - X*| <= tol |phi| / (4 m^2); G is bilinear in X
    rel = np.linalg.norm(G - Go) / np.linalg.norm(Go)
    print(f"oracle gradient: rel {rel:.3e}; S gpu {S.item():.12e} oracle {So:.12e}", flush=True)
    assert rel <= 1e-7
    assert abs(S.item() - So) <= 1e-9 * abs(So)
