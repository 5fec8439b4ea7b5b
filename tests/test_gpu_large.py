"""GPU parity of the large-block FP64 path (tridiagonalisation, divide and
conquer, back-transform, reconstruction) and of the Daleckii-Krein derivative
against the CPU oracle.  FP64 bar: 1e-10 relative Frobenius (svec space)."""
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


def saved_pair(P, s, n):
    import torch
    sv = torch.empty(P.saved_numel(n), dtype=torch.float64, device="cuda:0")
    y = P.project(dev(s), n, saved=sv)
    sv = sv.cpu().numpy()
    return y.cpu().numpy(), sv[:n], sv[n:].view(np.complex128).reshape(n, n, order="F")


@pytest.mark.parametrize("n", [65, 100, 129, 200])
def test_large_eigenpairs(P, n):
    s = W.gue(n, 2000 + n)
    print(f"large eigenpairs n={n}", flush=True)
    y, lam, v = saved_pair(P, s, n)
    m = oracle.unpack(s, n).conj()
    ref = np.linalg.eigvalsh(m)
    assert np.max(np.abs(lam - ref)) <= 1e-12 * np.abs(ref).max()
    assert np.linalg.norm(m @ v - v * lam) <= 1e-11 * np.linalg.norm(m)
    assert np.linalg.norm(v.conj().T @ v - np.eye(n)) <= 1e-11
    assert rel(y, oracle.project(s, n)) <= TOL


@pytest.mark.parametrize("n", [65, 97, 128, 130, 257])
def test_large_gue_parity(P, n):
    s = W.gue(n, 1001 + n)
    print(f"large gue n={n}", flush=True)
    y, info = P.project(dev(s), n, info=True)
    assert rel(y.cpu().numpy(), oracle.project(s, n)) <= TOL
    lam = np.linalg.eigvalsh(oracle.unpack(s, n))
    assert info["status"] == 0
    assert info["n_pos"] == int((lam > 0).sum()) and info["n_neg"] == n - info["n_pos"]


@pytest.mark.parametrize("n", [150])
def test_large_constructed_both_sides(P, n):
    sx, u, lam = W.constructed(n, 1003)
    for frac in (0.2, 0.8):
        lam_s = np.abs(lam).copy()
        lam_s[: int(frac * n)] *= -1.0
        x = (u * lam_s) @ u.conj().T
        s = W.upper_pack((x + x.conj().T) / 2)
        y = P.project(dev(s), n).cpu().numpy()
        assert rel(y, oracle.project(s, n)) <= TOL
        assert rel(y, oracle.constructed_projection(u, lam_s)) <= 1e-12


def test_large_degenerate_spectrum(P):
    n = 96
    u = W.haar_unitary(n, np.random.default_rng(1))
    lam = np.repeat([-1.0, 0.5, 2.0], 32)
    x = (u * lam) @ u.conj().T
    s = W.upper_pack((x + x.conj().T) / 2)
    y = P.project(dev(s), n).cpu().numpy()
    assert rel(y, oracle.constructed_projection(u, lam)) <= 1e-12
    assert rel(y, oracle.project(s, n)) <= TOL


def test_large_clustered_and_distinct_spectrum(P):
    # clusters (close-pair deflation by rotation: the sequential merge scan)
    # next to distinct eigenvalues (the parallel merge), n = 301
    n = 301
    rng = np.random.default_rng(11)
    u = W.haar_unitary(n, rng)
    lam = np.concatenate([np.repeat([-1.5, 0.75], 60), np.full(40, 1e-9), rng.uniform(-3.0, 3.0, n - 160)])
    x = (u * lam) @ u.conj().T
    s = W.upper_pack((x + x.conj().T) / 2)
    y = P.project(dev(s), n).cpu().numpy()
    assert rel(y, oracle.constructed_projection(u, lam)) <= 1e-12
    assert rel(y, oracle.project(s, n)) <= TOL


def test_large_special_inputs(P):
    n = 80
    d = np.linspace(-3.0, 5.0, n)
    s = oracle.pack(np.diag(d).astype(complex))
    y = P.project(dev(s), n).cpu().numpy()
    assert rel(y, oracle.pack(np.diag(np.maximum(d, 0)).astype(complex))) <= 1e-15
    z = np.zeros(n * n)
    assert np.abs(P.project(dev(z), n).cpu().numpy()).max() == 0.0
    g = W.cn01(np.random.default_rng(4), (n, n))
    psd = oracle.pack(g @ g.conj().T)
    assert rel(P.project(dev(psd), n).cpu().numpy(), psd) <= TOL
    assert np.abs(P.project(dev(-psd), n).cpu().numpy()).max() <= 1e-11 * np.abs(psd).max()


@pytest.mark.parametrize("n", [120, 121, 152, 153])
def test_large_tail_boundaries(P, n):
    # the last columns are reduced by one workgroup in LDS from the first
    # panel boundary p0 (a multiple of 32) with n - p0 <= 120: n = 120 has no
    # blocked panel, 121 and 153 the shortest tail (89), 152 the longest (120)
    s = W.gue(n, 3100 + n)
    print(f"large tail boundary n={n}", flush=True)
    y, lam, v = saved_pair(P, s, n)
    m = oracle.unpack(s, n).conj()
    ref = np.linalg.eigvalsh(m)
    assert np.max(np.abs(lam - ref)) <= 1e-12 * np.abs(ref).max()
    assert np.linalg.norm(m @ v - v * lam) <= 1e-11 * np.linalg.norm(m)
    assert np.linalg.norm(v.conj().T @ v - np.eye(n)) <= 1e-11
    assert rel(y, oracle.project(s, n)) <= TOL


@pytest.mark.parametrize("n,launches", [(100, 0), (120, 0), (121, 32), (200, 96)])
def test_tail_switch_launch_counts(P, n, launches):
    # per-column launches (HEMV and w step, counted by the timing hooks) run
    # up to the first panel boundary p0 with n - p0 <= 120; the rest is one
    # LDS launch
    from paper_2606_20519_amd import _lib
    import torch
    x = dev(W.gue(n, 77))
    for fam in (_lib.KF_HEMV, _lib.KF_WSTEP):
        _lib.timing_start(fam, 4 * n)
        P.project(x, n)
        torch.cuda.synchronize()
        ms, cnt, work = _lib.timing_stop()
        assert cnt == launches
        if fam == _lib.KF_HEMV:
            assert work == sum(8.0 * m * (m + 1) for m in range(n - 1, n - 1 - launches, -1))


def test_large_tail_structured_columns(P):
    # n = 152: blocked panels, then a tail of order 120 holding (a) a complex
    # tridiagonal stretch, where reflectors only rotate a phase (sigma = 0,
    # alpha complex), and (b) a zero column, where the reflector is the
    # identity (tau = 0)
    n = 152
    rng = np.random.default_rng(3152)
    a = W.cn01(rng, (n, n))
    a = (a + a.conj().T) / 2
    t0 = 90
    a[t0:, t0:] = 0.0
    for i in range(t0, n):
        a[i, i] = rng.standard_normal()
        if i + 1 < n:
            a[i + 1, i] = W.cn01(rng, ())
            a[i, i + 1] = np.conj(a[i + 1, i])
    a[:t0, t0:] = 0.0
    a[t0:, :t0] = 0.0
    z = 130
    a[z, :] = 0.0
    a[:, z] = 0.0
    s = oracle.pack(a)
    print("large tail structured n=152", flush=True)
    y, lam, v = saved_pair(P, s, n)
    m = oracle.unpack(s, n).conj()
    ref = np.linalg.eigvalsh(m)
    assert np.max(np.abs(lam - ref)) <= 1e-12 * np.abs(ref).max()
    assert np.linalg.norm(m @ v - v * lam) <= 1e-11 * np.linalg.norm(m)
    assert rel(y, oracle.project(s, n)) <= TOL


def test_large_invariants_in_place_determinism(P):
    n = 190
    s = W.gue(n, 33)
    x = dev(s)
    y1 = P.project(x, n).cpu().numpy()
    y2 = P.project(x, n).cpu().numpy()
    assert np.array_equal(y1, y2)
    ym = P.project(dev(-s), n).cpu().numpy()
    assert rel(y1 - ym, s) <= TOL                   # Moreau
    assert rel(P.project(dev(y1), n).cpu().numpy(), y1) <= TOL  # idempotent
    assert abs(y1 @ (y1 - s)) <= 1e-10 * (s @ s)    # <Pi, Pi - X> = 0
    P.project(x, n, out=x)
    assert np.array_equal(x.cpu().numpy(), y1)


def test_batched_mixed_sizes(P):
    sizes = [100, 25, 25, 16, 70, 49]
    parts = [W.gue(m, 5000 + i) for i, m in enumerate(sizes)]
    y, infos = P.project_batched(dev(np.concatenate(parts)), sizes, info=True)
    y = y.cpu().numpy()
    off = 0
    for m, s, inf in zip(sizes, parts, infos):
        assert rel(y[off:off + m * m], oracle.project(s, m)) <= TOL
        assert inf["status"] == 0
        off += m * m


@pytest.mark.parametrize("n", [16, 70, 130])
def test_vjp_parity(P, n):
    s, g = W.gue(n, 1005 + n), W.gue(n, 1006 + n)
    print(f"vjp n={n}", flush=True)
    ref = oracle.vjp(s, g, n)
    gx = P.vjp(dev(g), n, x=dev(s)).cpu().numpy()
    assert rel(gx, ref) <= TOL
    import torch
    sv = torch.empty(P.saved_numel(n), dtype=torch.float64, device="cuda:0")
    P.project(dev(s), n, saved=sv)
    gx2 = P.vjp(dev(g), n, saved=sv).cpu().numpy()
    assert rel(gx2, ref) <= TOL


def test_autograd_function(P):
    import torch
    n = 40
    s, g = W.gue(n, 71), W.gue(n, 72)
    x = dev(s).requires_grad_(True)
    y = P.PSDProject.apply(x, n)
    (y * dev(g)).sum().backward()
    assert rel(x.grad.cpu().numpy(), oracle.vjp(s, g, n)) <= TOL
    assert rel(y.detach().cpu().numpy(), oracle.project(s, n)) <= TOL


def test_vjp_finite_differences(P):
    n = 90
    s = W.gue(n, 81)
    rng = np.random.default_rng(82)
    h = 1e-6
    gbar = W.gue(n, 83)
    gx = P.vjp(dev(gbar), n, x=dev(s)).cpu().numpy()
    for _ in range(4):
        e = W.upper_pack(W.gue_matrix(n, rng))
        fd = (P.project(dev(s + h * e), n).cpu().numpy() - P.project(dev(s - h * e), n).cpu().numpy()) / (2 * h)
        assert abs(gbar @ fd - gx @ e) <= 1e-7 * np.linalg.norm(gbar) * np.linalg.norm(e)
