"""GPU parity of the whole-block LDS path (order <= 64) against the CPU oracle.

Tolerance: the FP64 path must agree with the oracle to 1e-10 relative
Frobenius norm in svec space (an isometry, App. D.1).
"""
import numpy as np
import pytest

import oracle
from paper_2606_20519_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2606_20519_amd as P
    return P


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 16, 17, 25, 31, 32, 33, 36, 49, 63, 64])
def test_small_gue_parity(P, n):
    s = W.gue(n, 1001 + n)
    print(f"small gue n={n}", flush=True)
    y, info = P.project(dev(s), n, info=True)
    ref = oracle.project(s, n)
    assert rel(y.cpu().numpy(), ref) <= TOL
    lam = np.linalg.eigvalsh(oracle.unpack(s, n))
    assert info["status"] == 0
    assert info["n_pos"] == int((lam > 0).sum()) and info["n_neg"] == n - info["n_pos"]


@pytest.mark.parametrize("n", [16, 40, 64])
def test_small_constructed_and_sides(P, n):
    # mostly-positive and mostly-negative spectra exercise both reconstruction sides
    sx, u, lam = W.constructed(n, 1003 + n)
    for sign in (1.0, -1.0):
        lam_s = lam.copy()
        lam_s[: n // 4] = sign * np.abs(lam_s[: n // 4])
        x = (u * lam_s) @ u.conj().T
        s = W.upper_pack((x + x.conj().T) / 2)
        y = P.project(dev(s), n).cpu().numpy()
        assert rel(y, oracle.project(s, n)) <= TOL
        assert rel(y, oracle.constructed_projection(u, lam_s)) <= 1e-12


def test_small_clustered_and_wide_spectra(P):
    # repeated eigenvalues and exact zeros at an odd order, +-1 each of
    # multiplicity 32, and a spectrum over sixteen decades: against the
    # closed form and the oracle
    rng = np.random.default_rng(17)
    # (orders <= 32 run the one-barrier-per-step kernel, larger ones the other)
    cases = [(33, np.concatenate([np.repeat([-2.0, 0.0, 1.5], 10), [3.0, -4.0, 0.25]])),
             (64, np.repeat([-1.0, 1.0], 32)),
             (48, np.concatenate([np.logspace(-8, 8, 24), -np.logspace(-8, 8, 24)])),
             (25, np.concatenate([np.repeat([-2.0, 0.0, 1.5], 7), [3.0, -4.0, 0.25, 0.0]])),
             (16, np.repeat([-1.0, 1.0], 8)),
             (32, np.concatenate([np.logspace(-8, 8, 16), -np.logspace(-8, 8, 16)]))]
    for n, lam in cases:
        u = W.haar_unitary(n, rng)
        x = (u * lam) @ u.conj().T
        s = W.upper_pack((x + x.conj().T) / 2)
        y = P.project(dev(s), n).cpu().numpy()
        assert rel(y, oracle.constructed_projection(u, lam)) <= 1e-12, n
        assert rel(y, oracle.project(s, n)) <= TOL, n


def test_small_special_inputs(P):
    n = 12
    rng = np.random.default_rng(3)
    g = W.cn01(rng, (n, n))
    psd = oracle.pack(g @ g.conj().T)
    assert rel(P.project(dev(psd), n).cpu().numpy(), psd) <= TOL
    assert np.abs(P.project(dev(-psd), n).cpu().numpy()).max() <= 1e-12 * np.abs(psd).max()
    d = np.array([3.0, -1.0, 0.0, 2.5, -7.25, 1e-300, 4.0, -2.0, 0.5, 1.0, -1.0, 8.0])
    s = oracle.pack(np.diag(d).astype(complex))
    y = P.project(dev(s), n).cpu().numpy()
    assert np.array_equal(y, oracle.pack(np.diag(np.maximum(d, 0)).astype(complex)))
    z = np.zeros(n * n)
    assert np.array_equal(P.project(dev(z), n).cpu().numpy(), z)


@pytest.mark.parametrize("n", [20, 36])
def test_small_in_place_and_invariants(P, n):
    s = W.gue(n, 77)
    x = dev(s)
    y = P.project(x, n).cpu().numpy()
    P.project(x, n, out=x)
    assert np.array_equal(x.cpu().numpy(), y)
    # Moreau: Pi(X) - Pi(-X) = X
    ym = P.project(dev(-s), n).cpu().numpy()
    assert rel(y - ym, s) <= TOL
    # idempotence
    assert rel(P.project(dev(y), n).cpu().numpy(), y) <= TOL


def test_small_batched_choi_blocks(P):
    sizes = [25, 25, 36, 16, 64, 1, 49, 9]
    parts = [W.gue(m, 4000 + i) for i, m in enumerate(sizes)]
    x = np.concatenate(parts)
    y, infos = P.project_batched(dev(x), sizes, info=True)
    y = y.cpu().numpy()
    off = 0
    for m, s, inf in zip(sizes, parts, infos):
        assert rel(y[off:off + m * m], oracle.project(s, m)) <= TOL
        assert inf["status"] == 0
        off += m * m


def test_small_nonfinite_flagged(P):
    n = 8
    s = W.gue(n, 5)
    s[3] = np.nan
    _, info = P.project(dev(s), n, info=True)
    assert info["status"] == 4


@pytest.mark.parametrize("n", [16, 25, 40])
def test_small_saved_eigenpairs(P, n):
    import torch
    s = W.gue(n, 91)
    saved = torch.empty(P.saved_numel(n), dtype=torch.float64, device="cuda:0")
    P.project(dev(s), n, saved=saved)
    sv = saved.cpu().numpy()
    lam = sv[:n]
    v = sv[n:].view(np.complex128).reshape(n, n, order="F")
    m = oracle.unpack(s, n).conj()  # the kernels work on conj(X) = X^T
    assert np.all(np.diff(lam) >= 0)
    np.testing.assert_allclose(lam, np.linalg.eigvalsh(m), rtol=0, atol=1e-12 * np.abs(lam).max())
    assert np.linalg.norm(m @ v - v * lam) <= 1e-12 * np.linalg.norm(m)
    assert np.linalg.norm(v.conj().T @ v - np.eye(n)) <= 1e-12


@pytest.mark.parametrize("n", [16, 25, 64])
def test_small_deterministic(P, n):
    s = W.gue(n, 8)
    a = P.project(dev(s), n).cpu().numpy()
    b = P.project(dev(s), n).cpu().numpy()
    assert np.array_equal(a, b)
