"""GPU checks at the benchmark's full sizes, in the launch configurations
bench.py times.

* n = 625 warm-start iterates (FP64): element-wise against the oracle.
* n = 1296 and 2401 constructed spectra: against the closed form
  U diag(max(lambda, 0)) U^H (exact up to the rounding of X itself, since
  the projection is non-expansive), FP64 and both mixed forms.
* n = 4096 (FP64 and its derivative) on the GUE input: properties that hold
  at any size -- Moreau Pi(X) - Pi(-X) = X, idempotence, <Pi, Pi - X> = 0,
  Pi >= 0 and Pi - X >= 0 (Cholesky of each plus c n eps ||X||_2 I: these two
  rule out the negative-side projection X - Pi(X), which shares the others),
  the Euler identity DPi(X)[X] = Pi(X) and self-adjointness of DPi -- since
  the oracle cannot finish at this order.  Element-wise checks at n = 4096
  against the closed forms are in test_gpu_d8.py.
* one d = 5 cone (32 W blocks of order 625 and 256 Choi blocks) by one plan
  launch: the W blocks of instances 0 and 31 and every Choi block against the
  oracle, and the Moreau identity on every block.
* n = 4200, past 64 row blocks (the longest trailing loops): invariants.
* n = 4000 in BF16 (the 128x128-tile product with the split tail): against
  the closed form, within the BF16 band bound.

Mixed bars: tests/bars.py (band at 2 u ||X||_2 plus the first-order
eigenvector term; FP32 also a fixed 1e-5)."""
import numpy as np
import pytest

import oracle
from paper_2606_20519_amd import workloads as W

import bars

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
    P.set_ns_iterations(0, 1)
    return P


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_warm_sequence_625_against_oracle(P):
    n = 625
    xs = W.warm_sequence(n, 1002, 3)
    for i, s in enumerate(xs):
        y, info = P.project(dev(s), n, info=True)
        assert info["status"] == 0
        err = rel(y.cpu().numpy(), oracle.project(s, n))
        print(f"n=625 iterate {i}: rel err {err:.2e}", flush=True)
        assert err <= TOL


@pytest.mark.parametrize("n", [1296, 2401])
def test_constructed_full_size_all_modes(P, n):
    s, u, lam = W.constructed(n, 1003 if n == 1296 else 1004, gap=1e-6)
    exact = oracle.constructed_projection(u, lam)
    check_constructed_all_modes(P, s, lam, exact, n)


def check_constructed_all_modes(P, s, lam, exact, n, modes=("fp64", "mixed_fp32", "mixed_bf16")):
    nrm = np.linalg.norm(exact)
    for mode in modes:
        y, info = P.project(dev(s), n, mode, info=True)
        err = rel(y.cpu().numpy(), exact)
        assert info["status"] == 0
        npos = int((lam > 0).sum())
        if mode == "fp64":
            print(f"n={n} fp64: rel err vs closed form {err:.2e}", flush=True)
            assert info["n_pos"] == npos
            assert err <= TOL
            continue
        band = bars.band_norm(lam, mode)
        est = info["est_rel_err"]
        print(f"n={n} {mode}: rel err vs closed form {err:.2e} (band {band / nrm:.2e}, est {est:.2e})",
              flush=True)
        tau = bars.BAND_C * bars.unit_roundoff(mode) * np.abs(lam).max()
        # n_pos comes from tr sign(X); eigenvalues inside the band may be unresolved
        assert abs(info["n_pos"] - npos) <= int((np.abs(lam) < tau).sum())
        if mode == "mixed_fp32":
            assert err <= bars.FP32_REL_BAR
            assert err * nrm <= bars.mixed_bar_abs(lam, mode, nrm, est)
        else:
            # C3 spectra: half the eigenvalues below 1e-3, so the band term dominates
            assert err * nrm <= band + 1e-9 * nrm


def test_constructed_4000_mixed_bf16(P):
    # BF16 at an order past 3969: the 128x128-tile product with its split
    # tail (528 tiles, the last 16 in 16 k-parts) and a ragged last tile row
    # (npad = 4032); against the closed form, within the BF16 band bound
    n = 4000
    s, u, lam = W.constructed(n, 1008, gap=1e-6)
    exact = oracle.constructed_projection(u, lam)
    check_constructed_all_modes(P, s, lam, exact, n, modes=("mixed_bf16",))


def spectral_norm_upper(a, iters=30):
    """1.05 x a power-iteration estimate of ||A||_2 (Hermitian A, CPU)."""
    v = np.random.default_rng(0).standard_normal(a.shape[0]) + 0j
    lam = 0.0
    for _ in range(iters):
        w = a @ v
        lam = np.linalg.norm(w) / np.linalg.norm(v)
        v = w / np.linalg.norm(w)
    return 1.05 * lam


def psd_with_margin(a, delta):
    """A + delta I admits a Cholesky factorisation (LAPACK), i.e. lambda_min(A) > -delta."""
    b = a + delta * np.eye(a.shape[0])
    try:
        np.linalg.cholesky(b)
        return True
    except np.linalg.LinAlgError:
        return False


def check_psd_pair(s, y_np, n):
    """Pi >= 0 and Pi - X >= 0 up to 8 n eps ||X||_2 (backward-stable FP64:
    every eigenvalue of the computed Pi within c n eps ||X||_2 of the exact
    one); X - Pi(X), the projection onto the negative side, fails both."""
    xm = oracle.unpack(s, n)
    pm = oracle.unpack(y_np, n)
    delta = 8.0 * n * np.finfo(np.float64).eps * spectral_norm_upper(xm)
    assert psd_with_margin(pm, delta), "Pi(X) not PSD"
    assert psd_with_margin(pm - xm, delta), "Pi(X) - X not PSD"
    # the same check rejects the negative-side projection
    assert not psd_with_margin(xm - pm, delta)


def _invariants(P, s, n):
    import torch
    x = dev(s)
    y, info = P.project(x, n, info=True)
    ym = P.project(-x, n)
    yy = P.project(y, n)
    torch.cuda.synchronize()
    y_np, ym_np, yy_np = y.cpu().numpy(), ym.cpu().numpy(), yy.cpu().numpy()
    assert info["status"] == 0
    assert rel(y_np - ym_np, s) <= TOL                      # Moreau
    assert rel(yy_np, y_np) <= TOL                          # idempotent
    assert abs(y_np @ (y_np - s)) <= 1e-10 * (s @ s)        # <Pi, Pi - X> = 0
    check_psd_pair(s, y_np, n)                              # Pi >= 0, Pi - X >= 0
    return x, y, y_np


def test_order_4096_invariants_and_derivative(P):
    import torch
    n = 4096
    s = W.gue(n, 1005)
    x, y, y_np = _invariants(P, s, n)
    # derivative: Euler identity and self-adjointness (svec is an isometry)
    sv = torch.empty(P.saved_numel(n), dtype=torch.float64, device="cuda:0")
    P.project(x, n, saved=sv)
    dx = P.vjp(x, n, saved=sv).cpu().numpy()
    assert rel(dx, y_np) <= TOL
    a, b = W.gue(n, 1006), W.gue(n, 1007)
    da = P.vjp(dev(a), n, saved=sv).cpu().numpy()
    db = P.vjp(dev(b), n, saved=sv).cpu().numpy()
    lhs, rhs = a @ db, da @ b
    assert abs(lhs - rhs) <= 1e-10 * np.linalg.norm(a) * np.linalg.norm(b)


def test_order_4200_past_64_row_blocks(P):
    n = 4200
    _invariants(P, W.gue(n, 4200), n)


def test_cone_d5_full_plan(P):
    import torch
    x_np, sizes = W.cone(5, 32)
    x = dev(x_np)
    plan = P.Plan(sizes, "fp64")
    y = plan.execute(x)
    ym = plan.execute(-x)
    torch.cuda.synchronize()
    y, ym = y.cpu().numpy(), ym.cpu().numpy()
    off = 0
    checked = 0
    for b, m in enumerate(sizes):
        blk = slice(off, off + m * m)
        assert rel(y[blk] - ym[blk], x_np[blk]) <= TOL, b   # Moreau, every block
        inst = b // 9
        if m <= 64 or inst in (0, 31):
            assert rel(y[blk], oracle.project(x_np[blk], m)) <= TOL, b
            checked += 1
        off += m * m
    assert checked == 2 + 256
    plan.close()
