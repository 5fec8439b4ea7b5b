"""Warm-started FP64 projection (psd_project_warm): the eigen-pair of the
previous input refined by matrix products (Ogita-Aishima steps), the cold
FP64 path as the fallback.  Every result is held to the FP64 bar (1e-10
relative Frobenius) against the oracle or the closed form.

* the n = 625 warm sequence (successive inputs one 1e-3 step apart): a chain
  of warm calls, each from the pair the previous call left; sampled iterates
  against the oracle, every iterate against the cold GPU path; no fallback,
  at most five refinement steps;
* small and tile-ragged orders (1, 2, 16, 40, 65, 130, 257) along sequences of
  their own, against the oracle;
* a pair that is not close (another matrix's): the cold path runs
  (fallback = 1) and y and the saved pair are bitwise those of psd_project;
* a spectrum with repeated eigenvalues, from its own pair (converges at
  once, clusters kept whole) and one 1e-3 step on (either path), against
  the closed form / the oracle;
* in place: y == x and saved_out == saved_prev;
* the refined pair serves psd_project_vjp: against the oracle's derivative;
* a non-finite input: NaN output and PSD_ENONFINITE, through the cold path;
* host-side refusals: mixed workspace flags and overlapping buffers;
* two steps at the d = 6 order (three split-K slices on the lower products,
  one on the full ones) against the cold path."""
import numpy as np
import pytest

import oracle
from paper_2606_20519_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10
ENONFINITE = 4


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


def saved_buf(P, n):
    import torch
    return torch.empty(P.saved_numel(n), dtype=torch.float64, device="cuda:0")


def cold_with_saved(P, s, n):
    saved = saved_buf(P, n)
    y = P.project(dev(s), n, saved=saved)
    return y, saved


def test_warm_sequence_625(P):
    n = 625
    xs = W.warm_sequence(n, 1002, 12)
    y0, saved = cold_with_saved(P, xs[0], n)
    steps = []
    for k in range(1, len(xs)):
        print(f"warm n={n} iterate {k}", flush=True)
        y, info = P.project_warm(dev(xs[k]), n, saved, info=True)
        assert info["status"] == 0 and info["fallback"] == 0, info
        assert 1 <= info["iters"] <= 5
        steps.append(info["iters"])
        yc = P.project(dev(xs[k]), n)
        assert rel(y.cpu().numpy(), yc.cpu().numpy()) <= TOL
        if k in (1, 6, 11):
            err = rel(y.cpu().numpy(), oracle.project(xs[k], n))
            print(f"  vs oracle {err:.2e}, steps {info['iters']}, est {info['est_rel_err']:.1e}", flush=True)
            assert err <= TOL
    print("refinement steps per iterate:", steps, flush=True)


@pytest.mark.parametrize("n", [1, 2, 16, 40, 65, 130, 257])
def test_warm_sequence_small_and_ragged(P, n):
    xs = W.warm_sequence(n, 2000 + n, 4)
    _, saved = cold_with_saved(P, xs[0], n)
    for k in range(1, len(xs)):
        print(f"warm n={n} iterate {k}", flush=True)
        y, info = P.project_warm(dev(xs[k]), n, saved, info=True)
        assert info["status"] == 0 and info["fallback"] == 0, info
        assert rel(y.cpu().numpy(), oracle.project(xs[k], n)) <= TOL


@pytest.mark.parametrize("n", [40, 300])
def test_far_pair_falls_back_bitwise(P, n):
    s = W.gue(n, 3000 + n)
    _, other = cold_with_saved(P, W.gue(n, 3100 + n), n)
    print(f"far pair n={n}", flush=True)
    out = saved_buf(P, n)
    y, info = P.project_warm(dev(s), n, other, saved_out=out, info=True)
    assert info["status"] == 0 and info["fallback"] == 1, info
    yc, saved_c = cold_with_saved(P, s, n)
    assert np.array_equal(y.cpu().numpy(), yc.cpu().numpy())
    assert np.array_equal(out.cpu().numpy(), saved_c.cpu().numpy())


def repeated_spectrum(n, seed):
    rng = np.random.default_rng(seed)
    u = W.haar_unitary(n, rng)
    vals = np.array([-1.0, -0.25, 0.0, 0.5, 2.0])
    lam = np.sort(vals[rng.integers(0, len(vals), size=n)])
    x = (u * lam[None, :]) @ u.conj().T
    return W.upper_pack((x + x.conj().T) / 2.0), u, lam


@pytest.mark.parametrize("n", [48, 200])
def test_repeated_eigenvalues(P, n):
    s, u, lam = repeated_spectrum(n, 4000 + n)
    _, saved = cold_with_saved(P, s, n)
    print(f"repeated spectrum n={n}", flush=True)
    y, info = P.project_warm(dev(s), n, saved, saved_out=saved_buf(P, n), info=True)
    assert info["status"] == 0 and info["fallback"] == 0, info
    assert rel(y.cpu().numpy(), oracle.constructed_projection(u, lam)) <= TOL
    # one step on: the clusters split by ~1e-3; either path must be exact
    rng = np.random.default_rng(4100 + n)
    h = W.gue_matrix(n, rng)
    s2 = s + 1e-3 * W.upper_pack(h)
    y2, info2 = P.project_warm(dev(s2), n, saved, info=True)
    print(f"  one step on: fallback {info2['fallback']}, steps {info2['iters']}", flush=True)
    assert info2["status"] == 0
    assert rel(y2.cpu().numpy(), oracle.project(s2, n)) <= TOL


def test_in_place(P):
    n = 150
    xs = W.warm_sequence(n, 5000, 3)
    _, saved = cold_with_saved(P, xs[0], n)
    for k in (1, 2):
        x = dev(xs[k])
        y, info = P.project_warm(x, n, saved, saved_out=saved, out=x, info=True)
        assert y.data_ptr() == x.data_ptr()
        assert info["fallback"] == 0
        assert rel(y.cpu().numpy(), oracle.project(xs[k], n)) <= TOL


@pytest.mark.parametrize("n", [30, 120])
def test_refined_pair_serves_the_derivative(P, n):
    xs = W.warm_sequence(n, 6000 + n, 2)
    _, saved = cold_with_saved(P, xs[0], n)
    out = saved_buf(P, n)
    P.project_warm(dev(xs[1]), n, saved, saved_out=out)
    gy = W.cotangent(n, 6100 + n)
    gx = P.vjp(dev(gy), n, saved=out)
    assert rel(gx.cpu().numpy(), oracle.vjp(xs[1], gy, n)) <= TOL


@pytest.mark.parametrize("n", [20, 100])
def test_nonfinite_input(P, n):
    xs = W.warm_sequence(n, 7000 + n, 2)
    _, saved = cold_with_saved(P, xs[0], n)
    s = xs[1].copy()
    s[3] = np.nan
    y, info = P.project_warm(dev(s), n, saved, saved_out=saved_buf(P, n), info=True)
    assert info["status"] == ENONFINITE
    assert np.isnan(y.cpu().numpy()).all()


def test_host_refusals(P):
    import ctypes
    from paper_2606_20519_amd import _lib
    L = _lib.lib()
    out = ctypes.c_size_t(0)
    n = _lib.int_array([100])
    assert L.psd_workspace_size(1, n, 0, _lib.PSD_FLAG_WARM, ctypes.byref(out)) == 0 and out.value > 0
    assert L.psd_workspace_size(1, n, 1, _lib.PSD_FLAG_WARM, ctypes.byref(out)) == 1
    assert L.psd_workspace_size(2, _lib.int_array([100, 100]), 0, _lib.PSD_FLAG_WARM, ctypes.byref(out)) == 1
    x = dev(W.gue(100, 8000))
    sv = saved_buf(P, 100)
    with pytest.raises(_lib.PsdError):
        P.project_warm(x, 100, sv, saved_out=sv, out=sv[: 100 * 100])   # y inside the saved pair


@pytest.mark.parametrize("n", [1296])
def test_warm_step_full_size_d6(P, n):
    """d = 6 order (three split-K slices on the lower products, one on the
    full ones): two 1e-3 steps of the sequence,
    against the cold GPU path (itself held to the oracle at this order by
    the closed-form tests)."""
    xs = W.warm_sequence(n, 9000 + n, 3)
    _, saved = cold_with_saved(P, xs[0], n)
    for k in (1, 2):
        print(f"warm n={n} iterate {k}", flush=True)
        y, info = P.project_warm(dev(xs[k]), n, saved, info=True)
        assert info["status"] == 0 and info["fallback"] == 0, info
        yc = P.project(dev(xs[k]), n)
        assert rel(y.cpu().numpy(), yc.cpu().numpy()) <= TOL
