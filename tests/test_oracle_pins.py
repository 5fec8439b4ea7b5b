"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check is a value printed
or derived by hand from the definitions (golden files), a closed form, an
invariant of the Euclidean projection onto the PSD cone, a special case that
reduces to a library routine (LAPACK through NumPy), or a brute-force count.
"""
import os

import numpy as np
import pytest

from paper_2606_20519_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EPS = np.finfo(np.float64).eps


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *vals = line.split()
            out[k] = np.array([float(v) for v in vals])
    return out


def herm(n, rng):
    return W.gue_matrix(n, rng)


# --------------------------------------------------------------------------
# vec_R / mat_R  (App. D.1)
# --------------------------------------------------------------------------

def test_svec_golden_n2(orc):
    g = read_golden("svec_n2.txt")
    x = (g["matrix_re"] + 1j * g["matrix_im"]).reshape(2, 2)
    np.testing.assert_allclose(orc.pack(x), g["svec"], rtol=0, atol=4 * EPS)
    np.testing.assert_allclose(orc.unpack(g["svec"], 2), x, rtol=0, atol=8 * EPS)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 31])
def test_svec_offsets_bruteforce(orc, n):
    # Enumerate the upper triangle row by row: X_ii then (Re, Im) of X_ij.
    pos = 0
    for i in range(n):
        assert orc.row_offset(n, i) == pos
        pos += 1
        for j in range(i + 1, n):
            assert orc.offdiag_offset(n, i, j) == pos
            pos += 2
    assert pos == n * n


@pytest.mark.parametrize("n", [1, 2, 5, 17, 64])
def test_svec_isometry_and_roundtrip(orc, n):
    rng = np.random.default_rng(10 + n)
    x, y = herm(n, rng), herm(n, rng)
    sx, sy = orc.pack(x), orc.pack(y)
    # <svec X, svec Y> = tr[X^H Y]  (App. D.1)
    assert abs(sx @ sy - np.trace(x.conj().T @ y).real) <= 64 * EPS * np.linalg.norm(x) * np.linalg.norm(y)
    ux = orc.unpack(sx, n)
    np.testing.assert_allclose(ux, x, rtol=0, atol=4 * EPS * np.abs(x).max())
    assert np.array_equal(ux, ux.conj().T)  # Hermitian by construction
    np.testing.assert_allclose(orc.pack(orc.unpack(sx, n)), sx, rtol=0, atol=4 * EPS * np.abs(sx).max())
    # The input generator's independent packer agrees with the oracle's.
    np.testing.assert_allclose(W.upper_pack(x), sx, rtol=0, atol=0)


# --------------------------------------------------------------------------
# Jacobi eigendecomposition
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [0, 1])
def test_jacobi_n1(orc, mode):
    lam, v = orc.eigh(np.array([-2.5]), 1, mode)
    assert lam[0] == -2.5 and v[0, 0] == 1.0


@pytest.mark.parametrize("mode", [0, 1])
def test_jacobi_diagonal_needs_no_rotation(orc, mode):
    d = np.array([3.0, -1.0, 0.0, 2.5, -7.25, 1e-300])
    n = d.size
    s = orc.pack(np.diag(d).astype(complex))
    lam, v, st = orc.eigh(s, n, mode, return_stats=True)
    assert st["rotations"] == 0
    assert np.array_equal(np.sort(d), lam)


@pytest.mark.parametrize("mode", [0, 1])
def test_jacobi_2x2_closed_form(orc, mode):
    rng = np.random.default_rng(5)
    for _ in range(20):
        a, b = rng.standard_normal(2)
        c = complex(*rng.standard_normal(2))
        x = np.array([[a, c], [np.conj(c), b]])
        lam, v, st = orc.eigh(orc.pack(x), 2, mode, return_stats=True)
        m, r = (a + b) / 2, np.hypot((a - b) / 2, abs(c))
        np.testing.assert_allclose(lam, [m - r, m + r], rtol=0, atol=8 * EPS * (abs(m) + r))
        # a single rotation zeroes the pivot
        assert st["rotations"] == 1
        np.testing.assert_allclose(x @ v, v * lam, rtol=0, atol=16 * EPS * (abs(m) + r))


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n", [3, 8, 25, 64, 97])
def test_jacobi_residual_orthogonality_lapack(orc, n, mode):
    s = W.gue(n, 100 + n)
    x = orc.unpack(s, n)
    lam, v = orc.eigh(s, n, mode)
    nx = np.linalg.norm(x)
    assert np.linalg.norm(x @ v - v * lam) <= 8 * n * EPS * nx
    assert np.linalg.norm(v.conj().T @ v - np.eye(n)) <= 8 * n * EPS
    # eigenvalues agree with LAPACK (run as a library routine)
    ref = np.linalg.eigvalsh(x)
    assert np.max(np.abs(lam - ref)) <= 8 * n * EPS * np.abs(ref).max()


def test_jacobi_sweep_cap_reports_noconv(orc):
    import oracle
    s = W.gue(24, 3)
    with pytest.raises(oracle.OracleError):
        orc.eigh(s, 24, 0, max_sweeps=1)


# --------------------------------------------------------------------------
# Pi(X) = V diag(max(lam,0)) V^H  (App. D.2)
# --------------------------------------------------------------------------

def test_projection_golden_2x2(orc):
    g = read_golden("projection_2x2.txt")
    for c in ("case1", "case2"):
        np.testing.assert_allclose(orc.project(g[c + "_x"], 2), g[c + "_y"], rtol=0, atol=16 * EPS)


@pytest.mark.parametrize("mode", [0, 1])
def test_projection_diagonal_bitwise(orc, mode):
    d = np.array([3.0, -1.0, 0.0, 2.5, -7.25, 1e-300, -0.0])
    s = orc.pack(np.diag(d).astype(complex))
    y = orc.project(s, d.size, mode)
    assert np.array_equal(y, orc.pack(np.diag(np.maximum(d, 0.0)).astype(complex)))


def test_projection_2x2_closed_form(orc):
    rng = np.random.default_rng(7)
    for _ in range(50):
        a, b = rng.standard_normal(2)
        c = complex(*rng.standard_normal(2))
        x = np.array([[a, c], [np.conj(c), b]])
        m, r = (a + b) / 2, np.hypot((a - b) / 2, abs(c))
        lp, lm = m + r, m - r
        if lm >= 0:
            ref = x
        elif lp <= 0:
            ref = np.zeros_like(x)
        else:
            ref = lp * (x - lm * np.eye(2)) / (lp - lm)
        np.testing.assert_allclose(orc.project(orc.pack(x), 2), orc.pack(ref), rtol=0,
                                   atol=32 * EPS * (abs(m) + r))


@pytest.mark.parametrize("n", [5, 20, 48])
def test_projection_psd_nsd_rank1(orc, n):
    rng = np.random.default_rng(n)
    g = W.cn01(rng, (n, n))
    p = g @ g.conj().T  # PSD
    sp = orc.pack(p)
    assert rel(orc.project(sp, n), sp) <= 64 * n * EPS
    assert np.abs(orc.project(-sp, n)).max() <= 64 * n * EPS * np.abs(sp).max()
    v = W.cn01(rng, n)
    mu = 2.75
    r1 = mu * np.outer(v, v.conj())
    assert rel(orc.project(orc.pack(r1), n), orc.pack(r1)) <= 64 * n * EPS
    assert np.abs(orc.project(orc.pack(-r1), n)).max() <= 64 * n * EPS * np.abs(r1).max()


@pytest.mark.parametrize("n", [16, 41, 80])
def test_projection_constructed_spectrum(orc, n):
    sx, u, lam = W.constructed(n, 1003 + n)
    y = orc.project(sx, n)
    ref = orc.constructed_projection(u, lam)
    # ||Pi(X_fp64) - U Lam+ U^H|| <= ||X_fp64 - U Lam U^H|| by non-expansiveness
    assert rel(y, ref) <= 1e-13


@pytest.mark.parametrize("n", [10, 37, 64])
def test_projection_vs_lapack(orc, n):
    s = W.gue(n, 1001 + n)
    x = orc.unpack(s, n)
    w, u = np.linalg.eigh(x)
    ref = (u * np.maximum(w, 0)) @ u.conj().T
    assert rel(orc.project(s, n, 0), orc.pack(ref)) <= 1e-13
    assert rel(orc.project(s, n, 1), orc.pack(ref)) <= 1e-13


@pytest.mark.parametrize("n", [12, 50])
def test_projection_invariants(orc, n):
    rng = np.random.default_rng(77 + n)
    s = W.gue(n, 200 + n)
    x = orc.unpack(s, n)
    y = orc.project(s, n)
    p = orc.unpack(y, n)
    nx2 = np.linalg.norm(x, 2)
    tol = 64 * n * EPS * nx2
    assert np.linalg.eigvalsh(p).min() >= -tol           # Pi >= 0
    assert np.linalg.eigvalsh(p - x).min() >= -tol       # Pi - X >= 0
    assert abs(y @ (y - s)) <= 64 * n * EPS * np.linalg.norm(s) ** 2  # <Pi, Pi - X> = 0
    assert rel(orc.project(y, n), y) <= 64 * n * EPS     # idempotent
    # Moreau: Pi(X) - Pi(-X) = X  (App. D.1, Pi_{C*}(x) = x + Pi_C(-x), C = C*)
    assert rel(y - orc.project(-s, n), s) <= 64 * n * EPS
    # conjugation: Pi(conj X) = conj Pi(X)
    assert rel(orc.project(orc.pack(x.conj()), n), orc.pack(p.conj())) <= 64 * n * EPS
    # unitary equivariance
    u = W.haar_unitary(n, rng)
    assert rel(orc.project(orc.pack(u @ x @ u.conj().T), n), orc.pack(u @ p @ u.conj().T)) <= 1e-13
    # positive homogeneity, bitwise for powers of two
    assert np.array_equal(orc.project(8.0 * s, n), 8.0 * y)
    assert np.array_equal(orc.project(s / 1024.0, n), y / 1024.0)
    # non-expansive
    s2 = s + 0.3 * W.gue(n, 300 + n)
    assert np.linalg.norm(orc.project(s2, n) - y) <= np.linalg.norm(s2 - s) * (1 + 1e-12)


def test_projection_block_diagonal(orc):
    a, b = 9, 14
    xa = W.gue_matrix(a, np.random.default_rng(1))
    xb = W.gue_matrix(b, np.random.default_rng(2))
    x = np.zeros((a + b, a + b), complex)
    x[:a, :a], x[a:, a:] = xa, xb
    p = orc.unpack(orc.project(orc.pack(x), a + b), a + b)
    assert np.abs(p[:a, a:]).max() <= 1e-14
    assert rel(orc.pack(p[:a, :a]), orc.project(orc.pack(xa), a)) <= 1e-13
    assert rel(orc.pack(p[a:, a:]), orc.project(orc.pack(xb), b)) <= 1e-13


def test_modes_agree(orc):
    n = 70
    s = W.gue(n, 9)
    assert rel(orc.project(s, n, 0), orc.project(s, n, 1)) <= 1e-13


# --------------------------------------------------------------------------
# Daleckii-Krein derivative (back-propagation through Pi, App. E)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [4, 16, 30])
def test_vjp_finite_differences(orc, n):
    s = W.gue(n, 500 + n)
    rng = np.random.default_rng(600 + n)
    h = 1e-6
    for _ in range(3):
        e = orc.pack(herm(n, rng))
        fd = (orc.project(s + h * e, n) - orc.project(s - h * e, n)) / (2 * h)
        jv = orc.vjp(s, e, n)
        assert rel(jv, fd) <= 1e-7


def test_vjp_full_jacobian_small(orc):
    # all n^2 directions of a 6x6 problem against central differences
    n = 6
    s = W.gue(n, 42)
    h = 1e-6
    for k in range(n * n):
        e = np.zeros(n * n); e[k] = 1.0
        fd = (orc.project(s + h * e, n) - orc.project(s - h * e, n)) / (2 * h)
        assert np.linalg.norm(orc.vjp(s, e, n) - fd) <= 1e-7


@pytest.mark.parametrize("n", [7, 33])
def test_vjp_structure(orc, n):
    s = W.gue(n, 700 + n)
    y = orc.project(s, n)
    rng = np.random.default_rng(n)
    a, b = orc.pack(herm(n, rng)), orc.pack(herm(n, rng))
    tol = 64 * n * EPS
    # self-adjoint in svec space
    assert abs(a @ orc.vjp(s, b, n) - b @ orc.vjp(s, a, n)) <= tol * np.linalg.norm(a) * np.linalg.norm(b)
    # Euler identity for the 1-homogeneous Pi: DPi(X)[X] = Pi(X)
    assert rel(orc.vjp(s, s, n), y) <= tol
    # X > 0 => identity;  X < 0 => zero
    g = W.cn01(rng, (n, n))
    spd = orc.pack(g @ g.conj().T + 0.5 * np.eye(n))
    assert rel(orc.vjp(spd, a, n), a) <= tol
    assert np.abs(orc.vjp(-spd, a, n)).max() <= tol * np.abs(a).max()
    # 0 <= Gamma <= 1  =>  ||DPi[E]|| <= ||E||
    assert np.linalg.norm(orc.vjp(s, a, n)) <= np.linalg.norm(a) * (1 + tol)


def test_vjp_diagonal_input_is_hadamard(orc):
    d = np.array([2.0, -1.0, 0.5, -3.0, 4.0])
    n = d.size
    e = herm(n, np.random.default_rng(3))
    gam = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            a, b = d[i], d[j]
            if a > 0 and b > 0:
                gam[i, j] = 1.0
            elif a <= 0 and b <= 0:
                gam[i, j] = 0.0
            else:
                gam[i, j] = max(a, b) / (max(a, b) - min(a, b))
    ref = orc.pack(gam * e)
    got = orc.vjp(orc.pack(np.diag(d).astype(complex)), orc.pack(e), n)
    np.testing.assert_allclose(got, ref, rtol=0, atol=8 * EPS * np.abs(e).max())


def test_vjp_constructed_spectrum(orc):
    n = 24
    sx, u, lam = W.constructed(n, 1234, gap=1e-2)
    e = herm(n, np.random.default_rng(8))
    gam = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            a, b = lam[i], lam[j]
            if a > 0 and b > 0:
                gam[i, j] = 1.0
            elif a <= 0 and b <= 0:
                gam[i, j] = 0.0
            else:
                gam[i, j] = max(a, b) / (max(a, b) - min(a, b))
    ref = u @ (gam * (u.conj().T @ e @ u)) @ u.conj().T
    assert rel(orc.vjp(sx, orc.pack(e), n), orc.pack(ref)) <= 1e-12


def test_constructed_vjp_closed_form(orc):
    # the closed form used at full size (n = 4096), pinned here against the
    # hand-built divided-difference matrix, the Jacobi-based derivative and
    # central differences of the Jacobi projection, and the Euler identity
    n = 24
    sx, u, lam = W.constructed(n, 1234, gap=1e-2)
    e = herm(n, np.random.default_rng(8))
    gam = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            a, b = lam[i], lam[j]
            if a > 0 and b > 0:
                gam[i, j] = 1.0
            elif a <= 0 and b <= 0:
                gam[i, j] = 0.0
            else:
                gam[i, j] = max(a, b) / (max(a, b) - min(a, b))
    ref = orc.pack(u @ (gam * (u.conj().T @ e @ u)) @ u.conj().T)
    got = orc.constructed_vjp(u, lam, orc.pack(e))
    assert rel(got, ref) <= 1e-13
    assert rel(got, orc.vjp(sx, orc.pack(e), n)) <= 1e-12
    h = 1e-6
    fd = (orc.project(sx + h * orc.pack(e), n) - orc.project(sx - h * orc.pack(e), n)) / (2 * h)
    assert rel(got, fd) <= 1e-7
    assert rel(orc.constructed_vjp(u, lam, sx), orc.constructed_projection(u, lam)) <= 1e-13
    # opposite-sign pairs only: Gamma in (0, 1), and a pure sign flip of the
    # spectrum maps DPi to I - DPi (Moreau: Pi(X) - Pi(-X) = X)
    flip = orc.constructed_vjp(u, -lam, orc.pack(e))
    assert rel(got + flip, orc.pack(e)) <= 1e-13


# --------------------------------------------------------------------------
# Newton-Schulz reference (mixed form attribution)
# --------------------------------------------------------------------------

def test_ns_scalar_map_fixed_points_and_sign():
    import oracle
    t = np.array([-1.0, 1.0, 0.0])
    assert np.array_equal(oracle.ns_scalar_map(t, 10), t)
    x = np.array([-1.5, -0.3, -1e-3, 1e-3, 0.2, 1.7])
    s = oracle.ns_scalar_map(x, 40)
    np.testing.assert_allclose(s, np.sign(x), rtol=0, atol=1e-12)
    # one step is the cubic 1.5 t - 0.5 t^3 (hand value at t = 0.5: 0.6875)
    assert oracle.ns_scalar_map(np.array([0.5]), 1)[0] == 0.6875


@pytest.mark.parametrize("n", [12, 40])
def test_ns_matrix_matches_scalar_on_constructed_spectra(orc, n):
    import oracle
    sx, u, lam = W.constructed(n, 77 + n, gap=1e-3)
    alpha = 1.05
    for iters in (3, 12, 30):
        a = oracle.ns_matrix_projection(sx, n, alpha, iters)
        b = oracle.ns_constructed_projection(u, lam, alpha, iters)
        assert rel(a, b) <= 1e-12
    # converged iterations reproduce the exact projection
    exact = orc.constructed_projection(u, lam)
    assert rel(oracle.ns_constructed_projection(u, lam, alpha, 40), exact) <= 1e-13
    assert rel(oracle.ns_matrix_projection(sx, n, alpha, 40), orc.project(sx, n)) <= 1e-12


def test_ns_truncation_bounded_by_small_eigenvalues(orc):
    # Components with |lambda| below the resolved band contribute at most
    # |lambda| each to the truncated projection's error.
    import oracle
    n = 30
    sx, u, lam = W.constructed(n, 5, gap=1e-6)
    for iters in (5, 15, 25):
        s = oracle.ns_scalar_map(lam / 1.0, iters)
        err = np.linalg.norm(oracle.ns_constructed_projection(u, lam, 1.0, iters) - orc.constructed_projection(u, lam))
        bound = np.sqrt(np.sum((0.5 * lam * (s - np.sign(lam))) ** 2))
        assert abs(err - bound) <= 1e-12 * max(1.0, bound)
        assert bound <= np.sqrt(np.sum(lam[np.abs(s) < 1 - 1e-12] ** 2)) + 1e-15


def test_ns_schedule_equioscillation_and_start():
    # a_0 = 1; afterwards a_k = min(1.5, sqrt(3 / (1 + l + l^2))): below the
    # cap f(a l) = f(a) (f(t) = (3t - t^3)/2), and the new lower bound is the
    # smaller end value
    import oracle
    a = oracle.ns_schedule(1e-6, 1e-7)
    assert a[0] == 1.0
    f = lambda t: 0.5 * (3.0 * t - t ** 3)
    lk = f(1e-6)
    for ak in a[1:]:
        assert 1.0 <= ak <= 1.5
        if ak < 1.5:
            assert abs(f(ak * lk) - f(ak)) <= 1e-14  # f(sqrt 3) = 0: cancellation
        else:
            assert 1.5 <= np.sqrt(3.0 / (1.0 + lk + lk * lk))
        lk = min(f(ak * lk), f(ak))
    assert 1.0 - lk <= 1e-7
    # about half the unscaled steps for the same resolution
    t, k = 1e-6, 0
    while 1.0 - t > 1e-7:
        t, k = f(t), k + 1
    assert len(a) <= k // 2 + 2
    # explicit counts: the same prefix, then scalings tending to 1
    assert oracle.ns_schedule(1e-6, iters=3) == a[:3]
    long = oracle.ns_schedule(1e-6, iters=len(a) + 5)
    assert long[:len(a)] == a and abs(long[-1] - 1.0) <= 1e-12
    # uncapped (amax >= sqrt 3): the pure equal-end scaling, fewer steps
    un = oracle.ns_schedule(1e-6, 1e-7, amax=2.0)
    lk = f(1e-6)
    for ak in un[1:]:
        assert abs(f(ak * lk) - f(ak)) <= 1e-14  # f(sqrt 3) = 0: cancellation
        lk = min(f(ak * lk), f(ak))
    assert len(un) < len(a)


def test_ns_schedule_maps_interval_brute_force():
    # every magnitude in [l0, t*] ends within tol of 1 after the schedule and
    # never above 1 + 1e-15; t* in (1, sqrt 3) solves f(t*) = f(l0), i.e.
    # t*^2 + t* l0 + l0^2 = 3 (an alpha underestimated by up to t*)
    import oracle
    l0 = 1e-6
    a = oracle.ns_schedule(l0, 1e-7)
    tstar = 0.5 * (-l0 + np.sqrt(12.0 - 3.0 * l0 * l0))
    t = np.concatenate([np.geomspace(l0, 1.0, 200001), np.linspace(1.0, tstar * (1 - 1e-12), 20001)])
    s = oracle.ns_scalar_map(t, len(a), a)
    assert s.min() >= 1.0 - 1e-7 and s.max() <= 1.0 + 1e-15
    assert np.abs(oracle.ns_scalar_map(-t, len(a), a) + s).max() <= 1e-15  # odd map


def test_ns_scaled_matrix_matches_scalar(orc):
    # matrix products vs per-eigenvalue map (diagonal input and constructed U)
    import oracle
    a = oracle.ns_schedule(1e-6, iters=9)
    d = np.array([0.9, -0.5, 1e-3, -2e-4, 0.3, 1.0])
    n = len(d)
    sx = orc.pack(np.diag(d).astype(complex))
    got = orc.unpack(oracle.ns_matrix_projection(sx, n, 1.0, 9, a), n)
    want = 0.5 * (d + d * oracle.ns_scalar_map(d, 9, a))
    assert np.abs(np.diag(got).real - want).max() <= 1e-13 * np.abs(want).max()
    assert np.abs(got - np.diag(np.diag(got))).max() == 0.0
    sx, u, lam = W.constructed(24, 91, gap=1e-3)
    for k in (4, 11):
        ak = oracle.ns_schedule(1e-6, iters=k)
        assert rel(oracle.ns_matrix_projection(sx, 24, 1.05, k, ak),
                   oracle.ns_constructed_projection(u, lam, 1.05, k, ak)) <= 1e-12
    full = oracle.ns_schedule(1e-6, 1e-7)
    assert rel(oracle.ns_constructed_projection(u, lam, 1.05, len(full), full),
               orc.constructed_projection(u, lam)) <= 1e-7


def test_spectral_norm_pin(orc):
    import oracle
    sx, u, lam = W.constructed(20, 3)
    assert abs(oracle.spectral_norm(sx, 20) - np.abs(lam).max()) <= 1e-13
