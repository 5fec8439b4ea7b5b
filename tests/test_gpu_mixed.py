"""GPU checks of the mixed-precision Newton-Schulz projection.

The mixed form approximates Pi; its error is stated against the FP64 oracle
for every case.  Bars (per case, see the assertions):
* FP32 iterations (+ FP64 corrections): 3e-6 relative Frobenius.  The
  low-precision iterates compute sign(X + Delta) with an effective
  perturbation ||Delta|| ~ 2^-24 ||X||; the eigenvector part of that error is
  left untouched by FP64 corrections S <- S(3I - S^2)/2 (they only move the
  eigenvalues of S to +-1), and it enters Pi = (X + XS)/2 as O(||Delta||).
  Observed: ~1e-6.
* BF16 iterations: within twice the band bound sqrt(sum of lambda^2 over
  |lambda| < 0.03 ||X||_2) plus 1e-9 relative -- components below the BF16
  resolution may be misclassified, each contributing at most |lambda|.
"""
FP32_TOL = 3e-6
import numpy as np
import pytest

import oracle
from paper_2606_20519_amd import workloads as W

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


@pytest.mark.parametrize("mode,tol", [("mixed_fp32", 1e-5), ("mixed_bf16", 5e-2)])
@pytest.mark.parametrize("iters", [1, 2, 5])
def test_ns_iterations_match_reference(P, mode, tol, iters):
    # No FP64 correction: the output is (X + X X_K)/2 with X_K from the
    # low-precision scaled iterations; the oracle runs the same recurrence
    # (its own schedule of scalings) in FP64 with the same alpha (reported in
    # info["scale"]).
    n = 96
    s = W.gue(n, 3500)
    P.set_ns_iterations(iters, 0)
    try:
        y, info = P.project(dev(s), n, mode=mode, info=True)
    finally:
        P.set_ns_iterations(0, 1)
    assert info["iters"] == iters
    ref = oracle.ns_matrix_projection(s, n, info["scale"], iters, oracle.ns_schedule(iters=iters))
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
    # ||I - S^2|| / sqrt(n) of the S entering the (one) FP64 correction: the
    # FP32 iterate's residual; the correction squares it
    assert info["est_rel_err"] <= 1e-5


@pytest.mark.parametrize("n", [100, 200])
def test_mixed_bf16_gue_within_band(P, n):
    s = W.gue(n, 3100 + n)
    print(f"mixed bf16 n={n}", flush=True)
    y, info = P.project(dev(s), n, mode="mixed_bf16", info=True)
    ref = oracle.project(s, n)
    lam = np.linalg.eigvalsh(oracle.unpack(s, n))
    nrm2 = np.abs(lam).max()
    band = np.sqrt(np.sum(lam[np.abs(lam) < 0.03 * nrm2] ** 2))
    err_abs = np.linalg.norm(y.cpu().numpy() - ref)
    print(f"  rel err {err_abs / np.linalg.norm(ref):.3e} band {band / np.linalg.norm(ref):.3e} "
          f"est {info['est_rel_err']:.3e}", flush=True)
    assert info["status"] == 0
    assert err_abs <= 2.0 * band + 1e-9 * np.linalg.norm(ref)


def test_mixed_constructed_gap(P):
    n = 130
    sx, u, lam = W.constructed(n, 3200, gap=1e-3)
    exact = oracle.constructed_projection(u, lam)
    y32 = P.project(dev(sx), n, mode="mixed_fp32").cpu().numpy()
    e32 = rel(y32, exact)
    yb = P.project(dev(sx), n, mode="mixed_bf16").cpu().numpy()
    eb = rel(yb, exact)
    band = np.sqrt(np.sum(lam[np.abs(lam) < 0.03] ** 2)) / np.linalg.norm(exact)
    print(f"constructed gap 1e-3: fp32 {e32:.3e}  bf16 {eb:.3e} (band {band:.3e})", flush=True)
    assert e32 <= FP32_TOL
    assert eb <= 2.0 * band + 1e-9


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
