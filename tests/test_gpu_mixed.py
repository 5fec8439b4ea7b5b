"""GPU checks of the mixed-precision Newton-Schulz projection.

The mixed form approximates Pi; its error is stated against the FP64 oracle
for every case.  Bars (tests/bars.py derives them):
* FP32 iterations (+ FP64 correction): 3e-6 relative Frobenius at these
  orders (fixed bar 1e-5 at full size), and within the first-order estimate
  of the info record (error <= 2 est): the low-precision iterates compute
  sign(X + Delta) with ||Delta|| ~ K 2^-24 ||X||, whose eigenvector part no
  polynomial correction in S removes; it enters the assembled Pi as the
  commutator term est measures.
* BF16 iterations: the band bound sqrt(sum of lambda^2 over
  |lambda| < 2 u ||X||_2), u = 2^-8, plus the first-order term 2 est ||Pi||.
"""
FP32_TOL = 3e-6
import numpy as np
import pytest

import oracle
from paper_2606_20519_amd import workloads as W

import bars

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("mode,amp", [("mixed_fp32", 4.0), ("mixed_bf16", 2.0), ("mixed_bf16x3", 4.0)])
@pytest.mark.parametrize("iters", [1, 2, 5])
def test_ns_iterations_match_reference(P, mode, amp, iters):
    # No FP64 correction: the output is the Hermitian part of (X + X X_K)/2
    # with X_K from the low-precision scaled iterations; the oracle runs the
    # same recurrence (its own schedule of scalings) in FP64 with the same
    # alpha (reported in info["scale"]).  Bar: the K + 1 roundings to the low
    # precision (X_0 and each iterate) each perturb by at most u relative;
    # `amp` allows for their growth through the later steps.
    tol = amp * (iters + 1) * bars.unit_roundoff(mode)
    n = 96
    s = W.gue(n, 3500)
    P.set_ns_iterations(iters, 0)
    try:
        y, info = P.project(dev(s), n, mode=mode, info=True)
    finally:
        P.set_ns_iterations(0, 1)
    assert info["iters"] == iters
    ref = oracle.ns_matrix_projection(s, n, info["scale"], iters,
                                      oracle.ns_schedule(l0=bars.ns_l0(mode), iters=iters))
    err = rel(y.cpu().numpy(), ref)
    print(f"{mode} iters={iters}: rel err vs FP64 NS reference {err:.3e}", flush=True)
    assert err <= tol


@pytest.mark.parametrize("n", [100, 200])
def test_mixed_fp32_gue(P, n):
    s = W.gue(n, 3000 + n)
    print(f"mixed fp32 n={n}", flush=True)
    y, info = P.project(dev(s), n, mode="mixed_fp32", info=True)
    ref = oracle.project(s, n)
    err = rel(y.cpu().numpy(), ref)
    lam = np.linalg.eigvalsh(oracle.unpack(s, n))
    print(f"  rel err {err:.3e} est {info['est_rel_err']:.3e} scale {info['scale']:.4f} "
          f"|X|2 {np.abs(lam).max():.4f}", flush=True)
    assert info["status"] == 0
    assert err <= FP32_TOL
    nrm2 = np.abs(lam).max()
    assert nrm2 <= info["scale"] <= 1.25 * nrm2
    assert info["n_pos"] == int((lam > 0).sum())
    # first-order estimate ||[X, S]||_F / (4 ||Pi||_F): it bounds the error
    # (factor 2 for second order) and is of the same size (not 100x above)
    est = info["est_rel_err"]
    assert err <= 2.0 * est + 1e-12
    assert est <= 100.0 * err


@pytest.mark.parametrize("n", [100, 200])
def test_mixed_bf16_gue_within_band(P, n):
    s = W.gue(n, 3100 + n)
    print(f"mixed bf16 n={n}", flush=True)
    y, info = P.project(dev(s), n, mode="mixed_bf16", info=True)
    ref = oracle.project(s, n)
    lam = np.linalg.eigvalsh(oracle.unpack(s, n))
    band = bars.band_norm(lam, "mixed_bf16")
    err_abs = np.linalg.norm(y.cpu().numpy() - ref)
    nrm = np.linalg.norm(ref)
    print(f"  rel err {err_abs / nrm:.3e} band {band / nrm:.3e} est {info['est_rel_err']:.3e}", flush=True)
    assert info["status"] == 0
    assert err_abs <= bars.mixed_bar_abs(lam, "mixed_bf16", nrm, info["est_rel_err"])


@pytest.mark.parametrize("n", [100, 200, 333])
def test_mixed_bf16x3_gue(P, n):
    # split-BF16 products: the band at 2 u ||X||_2 with u = 2^-16, plus twice
    # the first-order estimate; and well inside the plain BF16 form's error
    s = W.gue(n, 3150 + n)
    print(f"mixed bf16x3 n={n}", flush=True)
    y, info = P.project(dev(s), n, mode="mixed_bf16x3", info=True)
    yb = P.project(dev(s), n, mode="mixed_bf16")
    ref = oracle.project(s, n)
    lam = np.linalg.eigvalsh(oracle.unpack(s, n))
    nrm = np.linalg.norm(ref)
    err_abs = np.linalg.norm(y.cpu().numpy() - ref)
    eb = rel(yb.cpu().numpy(), ref)
    print(f"  rel err {err_abs / nrm:.3e} (bf16 {eb:.3e}) est {info['est_rel_err']:.3e}", flush=True)
    assert info["status"] == 0 and info["n_pos"] == int((lam > 0).sum())
    assert err_abs <= bars.mixed_bar_abs(lam, "mixed_bf16x3", nrm, info["est_rel_err"])
    assert err_abs / nrm <= 0.05 * eb
    est = info["est_rel_err"]
    assert est <= 100.0 * err_abs / nrm


def test_mixed_bf16x3_batched_and_plan(P):
    sizes = [100, 25, 70, 100]
    parts = [W.gue(m, 3350 + i) for i, m in enumerate(sizes)]
    x = dev(np.concatenate(parts))
    y = P.project_batched(x, sizes, mode="mixed_bf16x3").cpu().numpy()
    plan = P.Plan(sizes, "mixed_bf16x3")
    yp = plan.execute(x).cpu().numpy()
    plan.close()
    off = 0
    for m, s in zip(sizes, parts):
        ref = oracle.project(s, m)
        got = y[off:off + m * m]
        if m <= 64:
            assert rel(got, ref) <= 1e-10      # the exact LDS kernel
        else:
            lam = np.linalg.eigvalsh(oracle.unpack(s, m))
            nrm = np.linalg.norm(ref)
            assert np.linalg.norm(got - ref) <= bars.mixed_bar_abs(lam, "mixed_bf16x3", nrm, 1e-5)
        single = P.project(dev(s), m, mode="mixed_bf16x3").cpu().numpy()
        assert np.array_equal(got, single)                     # grouping does not change a member
        assert np.array_equal(yp[off:off + m * m], single)     # nor does the graph
        off += m * m


def test_mixed_constructed_gap(P):
    n = 130
    sx, u, lam = W.constructed(n, 3200, gap=1e-3)
    exact = oracle.constructed_projection(u, lam)
    nrm = np.linalg.norm(exact)
    y32, i32 = P.project(dev(sx), n, mode="mixed_fp32", info=True)
    e32 = rel(y32.cpu().numpy(), exact)
    yx, ix = P.project(dev(sx), n, mode="mixed_bf16x3", info=True)
    ex = rel(yx.cpu().numpy(), exact)
    print(f"constructed gap 1e-3: bf16x3 {ex:.3e} (est {ix['est_rel_err']:.2e})", flush=True)
    assert ex * nrm <= bars.mixed_bar_abs(lam, "mixed_bf16x3", nrm, ix["est_rel_err"])
    yb, ib = P.project(dev(sx), n, mode="mixed_bf16", info=True)
    eb = rel(yb.cpu().numpy(), exact)
    band = bars.band_norm(lam, "mixed_bf16") / nrm
    print(f"constructed gap 1e-3: fp32 {e32:.3e} (est {i32['est_rel_err']:.2e})  bf16 {eb:.3e} "
          f"(band {band:.3e}, est {ib['est_rel_err']:.2e})", flush=True)
    assert e32 <= FP32_TOL
    assert e32 <= 2.0 * i32["est_rel_err"] + 1e-12
    assert eb * nrm <= bars.mixed_bar_abs(lam, "mixed_bf16", nrm, ib["est_rel_err"])


def test_mixed_batched_and_small_blocks_exact(P):
    sizes = [100, 25, 70]
    parts = [W.gue(m, 3300 + i) for i, m in enumerate(sizes)]
    y = P.project_batched(dev(np.concatenate(parts)), sizes, mode="mixed_fp32").cpu().numpy()
    off = 0
    for m, s in zip(sizes, parts):
        tol = 1e-10 if m <= 64 else FP32_TOL   # blocks <= 64 take the exact LDS kernel
        assert rel(y[off:off + m * m], oracle.project(s, m)) <= tol
        off += m * m


def test_mixed_autograd_uses_fp64_derivative(P):
    n = 80
    s, g = W.gue(n, 3400), W.gue(n, 3401)
    x = dev(s).requires_grad_(True)
    y = P.PSDProject.apply(x, n, "mixed_fp32")
    (y * dev(g)).sum().backward()
    assert rel(x.grad.cpu().numpy(), oracle.vjp(s, g, n)) <= 1e-10
