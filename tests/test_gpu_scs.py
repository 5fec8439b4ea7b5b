"""The GPU SCS solver (psd_scs_solve) against the SCS oracle (oracle/scs.py)
and against optimality certificates that share nothing with either:

* iterate by iterate at d = 2 and d = 3 (eps = 0, k iterations): x, y, s,
  tau and kappa equal the oracle's after k steps (the oracle solves M z = a
  by the general reduced system and projects by Jacobi; the GPU by the
  closed-form affine step and its own eigensolver), FP64 rounding only;
* full solves: the iteration count and the objective of the oracle at d = 2;
  at d = 3..5 a certificate on the CPU from the trace-and-replace projector
  and LAPACK eigenvalues (s, y PSD, s in the process subspace with
  tr s = d^2, y + G orthogonal to the traceless process subspace, value and
  dual bound equal); the post-processed W is PSD and in the subspace;
* with type-I Anderson acceleration (memory 10): the iterates equal the
  oracle's for the first iterations at d = 2, the full solve reaches the
  oracle's value, and a d = 4 solve needs fewer iterations than without;
* closed-form optima (G = an allowed Pauli string: 1; a forbidden element:
  0; G = 1: d^2 with c = 0), warm start at the solution, the low-precision
  start (mixed_iters), a non-finite objective;
* at d = 8 (order 4096), a few iterations: tau > 0, s PSD and the reported
  residuals equal a recomputation from the returned x, y, s.
"""
import numpy as np
import pytest

import oracle
from oracle import affine as AF
from oracle import scs
from paper_2606_20519_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2606_20519_amd as P
    return P


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    return t.cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


_PROBS = {}


def gyni(d, seed=7):
    key = (d, seed)
    if key not in _PROBS:
        g = W.upper_pack(W.gyni_objective(d, seed))
        _PROBS[key] = (g, scs.problem(g, d) if d <= 3 else None)
    return _PROBS[key]


@pytest.mark.parametrize("d, k, warm", [(2, 1, False), (2, 3, False), (2, 40, False), (3, 1, False),
                                        (3, 12, False), (2, 40, True), (3, 40, True)])
def test_iterates_match_oracle(P, d, k, warm):
    """warm: the FP64 cone steps after the first by psd_project_warm (the
    oracle projects every step by Jacobi from scratch); early steps move too
    far and fall back to the cold path, later ones are refined."""
    g, prob = gyni(d)
    print(f"SCS iterates d={d} k={k} warm cone steps {warm}", flush=True)
    sv = scs.Solver(prob)
    sv.start()
    for _ in range(k):
        sv.step()
    tau, kappa = sv.ut, sv.vk
    if tau > 0:
        x, y, s, _, _ = sv.iterate_state()
    else:        # tau = 0 (the first step from the cold start): the raw u_x, u_y, v_s
        x, y, s = sv.u[: sv.nx], sv.u[sv.nx:], sv.v[sv.nx:]
    print(f"  oracle tau {tau:.6e} kappa {kappa:.6e}", flush=True)
    r = P.scs_solve(dev(g), d, eps=0.0, max_iters=k, post=False, warm_proj=warm)
    assert r["status"] == 5 and r["iters"] == k      # PSD_ENOCONV: eps = 0 runs max_iters
    if warm:
        print(f"  warm cone steps: {r['warm_refined']} refined, {r['warm_fallbacks']} fell back", flush=True)
        assert r["warm_refined"] + r["warm_fallbacks"] > 0
        if d == 2:
            assert r["warm_refined"] > 0
    assert abs(r["tau"] - tau) <= 1e-12 * max(1.0, abs(tau))
    assert abs(r["kappa"] - kappa) <= 1e-12 * max(1.0, abs(kappa))
    ex, ey, es = rel(host(r["x"]), x), rel(host(r["y"]), y), rel(host(r["s"]), s)
    print(f"  rel err x {ex:.2e} y {ey:.2e} s {es:.2e}", flush=True)
    assert ex <= 1e-10 and ey <= 1e-10 and es <= 1e-10
    assert abs(r["sigma"] - sv.sigma) <= 1e-14 * sv.sigma


@pytest.mark.parametrize("k", [2, 5, 12])
def test_anderson_iterates_match_oracle(P, k):
    d = 2
    g, prob = gyni(d)
    ref = scs.solve(g, d, eps=0.0, max_iters=k, prob=prob, anderson=10)
    r = P.scs_solve(dev(g), d, eps=0.0, max_iters=k, post=False, anderson=10)
    print(f"AA iterates k={k}: oracle tau {ref['tau']:.12e} accepted/rejected {ref['aa']}; GPU tau {r['tau']:.12e} "
          f"{r['aa_accepted']}/{r['aa_rejected']}", flush=True)
    assert (r["aa_accepted"], r["aa_rejected"]) == ref["aa"]
    assert abs(r["tau"] - ref["tau"]) <= 1e-10 * max(1.0, abs(ref["tau"]))
    for key in ("x", "y", "s"):
        e = rel(host(r[key]), ref[key])
        print(f"  {key}: {e:.2e}", flush=True)
        assert e <= 1e-9


def test_anderson_full_solve(P):
    g, prob = gyni(2)
    ref = scs.solve(g, 2, eps=1e-5, prob=prob, anderson=10)
    r = P.scs_solve(dev(g), 2, eps=1e-5, anderson=10)
    plain = P.scs_solve(dev(g), 2, eps=1e-5, post=False)
    print(f"d=2 AA: oracle {ref['iters']} iterations {ref['res']['pobj']:.10f}; GPU {r['iters']} "
          f"{r['pobj']:.10f} ({r['aa_accepted']} accepted, {r['aa_rejected']} rejected); plain {plain['iters']}",
          flush=True)
    assert r["status"] == 0
    # the accelerated trajectory is sensitive to rounding: the same solution, a similar count
    assert abs(r["pobj"] - ref["res"]["pobj"]) < 1e-4
    assert r["iters"] <= 1.5 * ref["iters"] + 10 and r["iters"] < plain["iters"]
    gmat = oracle.unpack(g, 16)
    _certificate(2, r, gmat, 1e-4)


def test_full_solve_matches_oracle_d2(P):
    g, prob = gyni(2)
    ref = scs.solve(g, 2, eps=1e-5, prob=prob)
    r = P.scs_solve(dev(g), 2, eps=1e-5)
    print(f"d=2: oracle {ref['iters']} iterations {ref['res']['pobj']:.10f}; GPU {r['iters']} {r['pobj']:.10f}",
          flush=True)
    assert r["status"] == 0
    assert abs(r["iters"] - ref["iters"]) <= 1
    assert abs(r["pobj"] - ref["res"]["pobj"]) < 1e-8
    assert abs(r["dobj"] - ref["res"]["dobj"]) < 1e-8


def _certificate(d, r, gmat, tol):
    n = d ** 4
    s = oracle.unpack(host(r["s"]), n)
    y = oracle.unpack(host(r["y"]), n)
    assert np.linalg.eigvalsh(s)[0] >= -1e-10
    assert np.linalg.eigvalsh(y)[0] >= -1e-10
    np.testing.assert_allclose(AF.p_proc(s, d), s, atol=tol)
    assert abs(np.trace(s).real - d * d) < tol * n
    z = y + gmat
    np.testing.assert_allclose(AF.p_proc(z, d) - np.trace(z) / n * np.eye(n), 0, atol=tol)
    value = np.trace(s @ gmat).real
    bound = np.trace(z).real / d ** 2
    assert np.trace(gmat).real / d ** 2 <= value + tol and value <= bound + tol
    assert abs(value - bound) < 10 * tol
    w = oracle.unpack(host(r["w"]), n)
    assert np.linalg.eigvalsh(w)[0] >= -1e-12
    np.testing.assert_allclose(AF.p_proc(w, d), w, atol=1e-11)
    assert abs(np.trace(w).real - d * d) < 1e-10
    return value, bound


@pytest.mark.parametrize("d, aa", [(3, 0), (4, 0), (5, 0), (4, 10), (5, 10)])
def test_certificate(P, d, aa):
    g, _ = gyni(d)
    gmat = oracle.unpack(g, d ** 4)
    eps = 1e-6 if d < 5 else 1e-5
    r = P.scs_solve(dev(g), d, eps=eps, max_iters=10000, anderson=aa)
    print(f"d={d} anderson={aa}: {r['iters']} iterations ({r['aa_accepted']}/{r['aa_rejected']}), "
          f"value {r['pobj']:.9f} bound {r['dobj']:.9f} "
          f"res {r['res_pri']:.1e} {r['res_dual']:.1e} {r['gap']:.1e} post lam {r['post_lambda']:.1e}", flush=True)
    assert r["status"] == 0 and r["proj_status"] == 0
    _certificate(d, r, gmat, 10 * eps)


@pytest.mark.parametrize("d, aa", [(3, 0), (4, 0), (5, 5)])
def test_warm_cone_steps(P, d, aa):
    """warm_proj: every FP64 cone step after the first refines the eigen-pair
    the previous one left (psd_project_warm); the solve reaches the same
    certificate, in about as many iterations as the cold solve (the
    projections agree to rounding)."""
    g, _ = gyni(d)
    gmat = oracle.unpack(g, d ** 4)
    eps = 1e-6 if d < 5 else 1e-5
    cold = P.scs_solve(dev(g), d, eps=eps, max_iters=10000, anderson=aa)
    r = P.scs_solve(dev(g), d, eps=eps, max_iters=10000, anderson=aa, warm_proj=True)
    print(f"d={d} anderson={aa}: cold {cold['iters']} iterations, warm cone steps {r['iters']} "
          f"({r['warm_refined']} refined, {r['warm_fallbacks']} cold fallbacks), value {r['pobj']:.9f} "
          f"(cold {cold['pobj']:.9f})", flush=True)
    assert r["status"] == 0 and r["proj_status"] == 0
    assert r["warm_refined"] + r["warm_fallbacks"] <= r["iters"] - 1
    assert r["warm_refined"] > 0
    assert abs(r["iters"] - cold["iters"]) <= max(3, cold["iters"] // 50)
    _certificate(d, r, gmat, 10 * eps)


@pytest.mark.parametrize("d, which, value", [(2, 0, 1.0), (2, 86, 1.0), (2, "forbidden", 0.0),
                                             (2, "identity", 4.0), (3, "identity", 9.0),
                                             (3, "forbidden", 0.0)])
def test_closed_form_optima(P, d, which, value):
    sig = AF.gellmann(d)
    if which == "identity":
        g = np.eye(d ** 4)
    elif which == "forbidden":
        g = AF.basis_element(sig, (0, 1, 0, 0))
    else:
        g = AF.basis_element(sig, AF.allowed_indices(d)[which])
    r = P.scs_solve(dev(oracle.pack(g)), d, eps=1e-9, max_iters=20000)
    print(f"closed form d={d} {which}: {r['iters']} iterations, {r['pobj']:.12f}", flush=True)
    assert r["status"] == 0
    assert abs(r["pobj"] - value) < 1e-7 and abs(r["dobj"] - value) < 1e-7


def test_warm_start_and_mixed_start(P):
    d = 4
    g, _ = gyni(d)
    gd = dev(g)
    ref = P.scs_solve(gd, d, eps=1e-6, max_iters=20000)
    assert ref["status"] == 0
    warm = P.scs_solve(gd, d, eps=1e-6, warm=(ref["x"], ref["y"], ref["s"]))
    print(f"d=4 cold {ref['iters']} iterations; warm {warm['iters']}", flush=True)
    assert warm["status"] == 0 and warm["iters"] <= 2
    for mode in ("mixed_fp32", "mixed_bf16", "mixed_bf16x3"):
        mx = P.scs_solve(gd, d, eps=1e-6, max_iters=20000, mixed_iters=60, mixed_mode=mode)
        print(f"d=4 {mode} for 60 iterations: {mx['iters']} iterations, value {mx['pobj']:.9f} "
              f"(FP64 {ref['pobj']:.9f})", flush=True)
        assert mx["status"] == 0 and mx["switch_iter"] == 0
        assert abs(mx["pobj"] - ref["pobj"]) < 1e-5
    # the residual-based switch: mixed cone steps until the iterate is within
    # 10x the tolerance, then FP64 to the end
    sw = P.scs_solve(gd, d, eps=1e-6, max_iters=20000, mixed_iters=20000, mixed_mode="mixed_bf16x3",
                     mixed_switch=10.0)
    print(f"d=4 BF16x3 until 10x the tolerance: switched after {sw['switch_iter']}, {sw['iters']} iterations, "
          f"value {sw['pobj']:.9f}", flush=True)
    assert sw["status"] == 0 and 0 < sw["switch_iter"] < sw["iters"]
    assert abs(sw["pobj"] - ref["pobj"]) < 1e-5


def test_nonfinite_objective(P):
    g, _ = gyni(2)
    g = g.copy()
    g[5] = np.nan
    r = P.scs_solve(dev(g), 2, eps=1e-5)
    assert r["status"] == 4      # PSD_ENONFINITE


def test_d8_iterations(P):
    import torch
    d, n = 8, 4096
    g = W.upper_pack(W.gyni_objective(d, 11))
    gd = dev(g)
    print("d=8: 6 iterations", flush=True)
    r = P.scs_solve(gd, d, eps=0.0, max_iters=6)
    assert r["status"] == 5 and r["iters"] == 6 and r["tau"] > 0
    x, y, s = r["x"], r["y"], r["s"]
    # s = v_s / tau is PSD by construction (Moreau): Pi(s) = s
    ps = P.project(s, n)
    assert float(torch.linalg.vector_norm(ps - s)) <= 1e-10 * float(torch.linalg.vector_norm(s))
    # the reported residuals recomputed from x, y, s
    b = torch.zeros(n * n, dtype=torch.float64, device="cuda:0")
    b[torch.tensor([i * (2 * n - i) for i in range(n)], device="cuda:0")] = 1.0 / d ** 2
    ax = P.constraint_apply(x, d)
    c = P.constraint_adjoint(gd, d)
    aty = P.constraint_adjoint(y, d)
    res_pri = float((ax + s - b).abs().max())
    res_dual = float((aty + c).abs().max())
    gap = abs(float(c @ x) + float(b @ y))
    print(f"d=8 residuals: reported {r['res_pri']:.6e} {r['res_dual']:.6e} {r['gap']:.6e}; "
          f"recomputed {res_pri:.6e} {res_dual:.6e} {gap:.6e}", flush=True)
    assert abs(res_pri - r["res_pri"]) <= 1e-9 * max(res_pri, 1e-300) + 1e-14
    assert abs(res_dual - r["res_dual"]) <= 1e-9 * max(res_dual, 1e-300) + 1e-14
    assert abs(gap - r["gap"]) <= 1e-8 * max(abs(float(c @ x)), 1e-300)
    w = r["w"]
    pw = P.project(w, n)
    assert float(torch.linalg.vector_norm(pw - w)) <= 1e-10 * float(torch.linalg.vector_norm(w))


@pytest.mark.parametrize("d, anderson, mixed", [(3, 0, None), (4, 5, None), (3, 0, "mixed_bf16x3"),
                                               (3, 5, "mixed_fp32")])
def test_batched_equals_single_solves(P, d, anderson, mixed):
    # instances of a batch advance in lockstep, their cone steps in one
    # batched projection: each equals its own single solve bit for bit; an
    # instance with a non-finite objective stops at setup without touching
    # the others
    import torch
    gs = [W.upper_pack(W.gyni_objective(d, seed)) for seed in (7, 8, 9)]
    bad = gs[1].copy()
    bad[3] = np.nan
    batch = np.stack([gs[0], bad, gs[2]])
    # (a low-precision start, a fixed number of cone steps, is per instance
    # too: the batched projection's groups match single calls in every mode)
    kw = dict(mixed_iters=40, mixed_mode=mixed) if mixed else {}
    outs = P.scs_solve_batched(dev(batch), d, eps=1e-6, max_iters=5000, anderson=anderson, **kw)
    assert outs[1]["status"] == 4
    for b in (0, 2):
        one = P.scs_solve(dev(gs[b]), d, eps=1e-6, max_iters=5000, anderson=anderson, **kw)
        print(f"d={d} batch member {b}: {outs[b]['iters']} iterations (single {one['iters']}), "
              f"value {outs[b]['pobj']:.10f}", flush=True)
        assert outs[b]["status"] == 0 and one["status"] == 0
        for key in ("iters", "pobj", "dobj", "res_pri", "res_dual", "gap", "tau", "kappa", "aa_accepted",
                    "aa_rejected", "post_lambda"):
            assert outs[b][key] == one[key], key
        for key in ("x", "y", "s", "w"):
            assert torch.equal(outs[b][key], one[key]), key
