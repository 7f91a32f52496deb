"""The Table 1 routines on the GPU (one thread per call) against the oracle's
implementations of the same routines, which are pinned to numpy linear
algebra and, for the adjoint product, to Eqs (1.1)-(2.3)."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1309_0551_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lat():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with P.Lattice((4, 4, 4, 4)) as l:
        yield l


def _planes(z):
    """complex [n][P] -> real [P][n][2]"""
    return np.ascontiguousarray(np.stack([z.real.T, z.imag.T], axis=-1))


def _unplanes(x):
    return (x[..., 0] + 1j * x[..., 1]).T


def _oracle_call(name, a, b, s):
    """One call of the oracle's routine on operand rows a, b (complex, flat)."""
    kind_a, kind_b = P.ROUTINES[name][1], P.ROUTINES[name][2]
    shape = {"vec": (3,), "mat": (3, 3), "vec4": (4, 3), "mat4": (4, 3, 3)}
    A, B = a.reshape(shape[kind_a]), b.reshape(shape[kind_b])
    if name in ("scalar_mult_add_su3_matrix", "scalar_mult_add_su3_vector"):
        out = oracle.routine(name, A, B, scalar=s)
    else:
        out = oracle.routine(name, A, B)
    if isinstance(out, list):
        out = np.concatenate(out)
    return np.asarray(out).reshape(-1)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 777, 70000])
@pytest.mark.parametrize("name", sorted(P.ROUTINES))
def test_routine_vs_oracle(lat, name, n, prec):
    rid, ka, kb, kc, _ = P.ROUTINES[name]
    g = np.random.default_rng(rid * 1000 + n)
    za = g.standard_normal((n, P.PLANES[ka])) + 1j * g.standard_normal((n, P.PLANES[ka]))
    zb = g.standard_normal((n, P.PLANES[kb])) + 1j * g.standard_normal((n, P.PLANES[kb]))
    s = float(g.standard_normal())
    dt = torch.float64 if prec == "f64" else torch.float32
    if prec == "f32":  # the oracle sees the values the GPU sees
        za = za.astype(np.complex64).astype(np.complex128)
        zb = zb.astype(np.complex64).astype(np.complex128)
        s = float(np.float32(s))
    a = torch.from_numpy(_planes(za)).to(lat.device, dt)
    b = torch.from_numpy(_planes(zb)).to(lat.device, dt)
    c = P.routine(lat, name, a, b, s)
    got = _unplanes(c.cpu().double().numpy())
    assert got.shape == (n, P.PLANES[kc])
    idx = np.arange(n) if n <= 777 else np.concatenate([np.arange(8), g.choice(n, 300, replace=False), [n - 1]])
    tol = 1e-14 if prec == "f64" else 2e-6
    for i in idx:
        ref = _oracle_call(name, za[i], zb[i], s)
        scale = max(1.0, float(np.abs(ref).max()))
        assert np.abs(got[i] - ref).max() <= tol * 8 * scale, (name, prec, n, i)


def test_routine_in_place_and_errors(lat):
    n = 300
    g = np.random.default_rng(5)
    za = g.standard_normal((n, 3)) + 1j * g.standard_normal((n, 3))
    zb = g.standard_normal((n, 12)) + 1j * g.standard_normal((n, 12))
    a = torch.from_numpy(_planes(za)).to(lat.device)
    b = torch.from_numpy(_planes(zb)).to(lat.device)
    P.routine(lat, "sub_four_su3_vecs", a, b, out=a)  # c may be a
    got = _unplanes(a.cpu().numpy())
    np.testing.assert_allclose(got, za - zb.reshape(n, 4, 3).sum(1), rtol=1e-14, atol=1e-14)
    l = P.lib()
    assert l.lgt_routine(lat._ctx, 2, P.LGT_F64, n, a.data_ptr(), b.data_ptr(), a.data_ptr(), 0.0) == \
        -8
    assert l.lgt_routine(lat._ctx, 16, P.LGT_F64, n, a.data_ptr(), b.data_ptr(), a.data_ptr(), 0.0) == \
        -1
    assert l.lgt_routine(lat._ctx, 1, P.LGT_BF16, n, a.data_ptr(), b.data_ptr(), a.data_ptr(), 0.0) == \
        -1
    assert l.lgt_routine(lat._ctx, 1, P.LGT_F64, 0, None, None, None, 0.0) == 0
