"""Element-wise checks at the largest single-block order, n = d^4 = 4096 (d = 8),
in the configuration bench.py times, where the Jacobi oracle cannot finish:

* forward FP64 projection of a constructed spectrum X = U diag(lambda) U^H
  (U Haar, |lambda| log-uniform in [1e-6, 1], half negative) against the
  closed form U diag(max(lambda, 0)) U^H, element by element; FP32- and
  BF16-mixed forms against the same closed form within their derived bars
  (tests/bars.py);
* the Daleckii-Krein derivative at n = 4096, from x and from the saved
  eigen-pair, against the closed form U (Gamma o U^H G U) U^H on a
  constructed spectrum (|lambda| in [1e-3, 1]);
* central differences (h = 1e-6) on the leading 64 x 64 window: (i) the full
  gradient of <G, Pi(X_64)> over all 4096 svec coordinates of the window as a
  standalone order-64 problem, against the derivative; (ii) on the order-4096
  GUE input, 16 random unit Hermitian directions supported on the window,
  <G, (Pi(X + hE) - Pi(X - hE)) / 2h> against <DPi(X)[G], E>.
"""
import numpy as np
import pytest

import oracle
from paper_2606_20519_amd import workloads as W

import bars

pytestmark = pytest.mark.gpu
TOL = 1e-10
N = 4096


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


@pytest.fixture(scope="module")
def c3_4096():
    print("building the constructed n=4096 input (gap 1e-6)", flush=True)
    s, u, lam = W.constructed(N, 1009, gap=1e-6)
    return s, u, lam, oracle.constructed_projection(u, lam)


def test_d8_forward_fp64_constructed(P, c3_4096):
    s, u, lam, exact = c3_4096
    y, info = P.project(dev(s), N, "fp64", info=True)
    err = rel(y.cpu().numpy(), exact)
    print(f"n=4096 fp64 vs closed form: {err:.3e}", flush=True)
    assert info["status"] == 0
    assert info["n_pos"] == int((lam > 0).sum())
    assert err <= TOL


@pytest.mark.parametrize("mode", ["mixed_fp32", "mixed_bf16", "mixed_bf16x3"])
def test_d8_forward_mixed_constructed(P, c3_4096, mode):
    s, u, lam, exact = c3_4096
    nrm = np.linalg.norm(exact)
    y, info = P.project(dev(s), N, mode, info=True)
    err = rel(y.cpu().numpy(), exact)
    band = bars.band_norm(lam, mode)
    print(f"n=4096 {mode} vs closed form: {err:.3e} (band {band / nrm:.3e}, est {info['est_rel_err']:.3e})",
          flush=True)
    assert info["status"] == 0
    if mode == "mixed_fp32":
        assert err <= bars.FP32_REL_BAR
        assert err * nrm <= bars.mixed_bar_abs(lam, mode, nrm, info["est_rel_err"])
    elif mode == "mixed_bf16x3":
        assert err * nrm <= bars.mixed_bar_abs(lam, mode, nrm, info["est_rel_err"])
    else:
        assert err * nrm <= band + 1e-9 * nrm


def test_d8_vjp_constructed(P):
    import torch
    s, u, lam = W.constructed(N, 1010, gap=1e-3)
    g = W.cotangent(N, 1006)
    print("closed-form derivative at n=4096", flush=True)
    ref = oracle.constructed_vjp(u, lam, g)
    x, gd = dev(s), dev(g)
    gx = P.vjp(gd, N, x=x).cpu().numpy()
    e1 = rel(gx, ref)
    sv = torch.empty(P.saved_numel(N), dtype=torch.float64, device="cuda:0")
    y = P.project(x, N, saved=sv)
    gs = P.vjp(gd, N, saved=sv).cpu().numpy()
    e2 = rel(gs, ref)
    e3 = rel(y.cpu().numpy(), oracle.constructed_projection(u, lam))
    print(f"n=4096 vjp vs closed form: from x {e1:.3e}, from saved {e2:.3e}; forward {e3:.3e}", flush=True)
    assert e1 <= TOL and e2 <= TOL and e3 <= TOL


def _window_direction(rng, n, w=64):
    """svec of a unit-Frobenius Hermitian E supported on the leading w x w window."""
    e = np.zeros((n, n), dtype=np.complex128)
    a = W.gue_matrix(w, rng)
    e[:w, :w] = a / np.linalg.norm(a)
    return W.upper_pack(e)


def test_window64_full_gradient_fd(P):
    # Q16 (i): f(x) = <G64, Pi(X64)> for the leading 64 x 64 principal block of
    # the order-4096 input, differentiated along all 4096 svec coordinates
    # (central differences, h = 1e-6, 8192 order-64 projections in one batched
    # call), against the derivative DPi(X64)[G64] element by element
    import torch
    w = 64
    xm = oracle.unpack(W.gue(N, 1005), N)[:w, :w]
    gm = oracle.unpack(W.cotangent(N, 1006), N)[:w, :w]
    s, g = W.upper_pack(xm), W.upper_pack(gm)
    h = 1e-6
    eye = np.eye(w * w)
    batch = np.concatenate([np.concatenate([s + h * eye[k], s - h * eye[k]]) for k in range(w * w)])
    yb = P.project_batched(dev(batch), [w] * (2 * w * w)).cpu().numpy().reshape(w * w, 2, w * w)
    fd = ((yb[:, 0, :] - yb[:, 1, :]) @ g) / (2 * h)
    jv = P.vjp(dev(g), w, x=dev(s)).cpu().numpy()
    err = np.abs(fd - jv).max() / np.abs(jv).max()
    print(f"64x64 window: full gradient by central differences vs derivative: max rel {err:.3e}", flush=True)
    # rounding: |<G, dPi>| ~ 1e-15 ||G|| ||Pi|| per projection, over 2h
    assert err <= 1e-6
    assert rel(jv, oracle.vjp(s, g, w)) <= TOL
    torch.cuda.synchronize()


def test_d8_window_directions_fd(P):
    # Q16 (ii): 16 unit Hermitian directions on the leading 64 x 64 window of
    # the order-4096 GUE input, central differences with h = 1e-6
    import torch
    s, g = W.gue(N, 1005), W.cotangent(N, 1006)
    x, gd = dev(s), dev(g)
    sv = torch.empty(P.saved_numel(N), dtype=torch.float64, device="cuda:0")
    y0 = P.project(x, N, saved=sv)
    jg = P.vjp(gd, N, saved=sv)
    rng = np.random.default_rng(1011)
    h = 1e-6
    # rounding floor of the difference quotient: each projection is within
    # ~c n eps ||Pi||_F of the exact one, decorrelated between X +- hE
    pi_norm = float(torch.linalg.vector_norm(y0))
    g_norm = float(torch.linalg.vector_norm(gd))
    worst = 0.0
    for k in range(16):
        e = dev(_window_direction(rng, N))
        yp = P.project(x + h * e, N)
        ym = P.project(x - h * e, N)
        fd = float(torch.dot(gd, yp - ym)) / (2 * h)
        an = float(torch.dot(jg, e))
        noise = 2.0 * 1e-13 * pi_norm * g_norm / N / (2 * h)   # random-direction rounding, see below
        d = abs(fd - an)
        worst = max(worst, d / max(abs(an), 1e-300))
        print(f"  direction {k}: fd {fd:+.12e} derivative {an:+.12e} |diff| {d:.2e} "
              f"(rounding floor {noise:.1e})", flush=True)
        # the difference of two independent rounding errors of size
        # ~1e-13 ||Pi||_F, seen through G (a random direction in n^2
        # coordinates: a factor ||G|| / n), divided by 2h; plus O(h^2)
        assert d <= noise + 1e-7 * abs(an)
    print(f"n=4096 window FD: worst relative difference {worst:.3e}", flush=True)
