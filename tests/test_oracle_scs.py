"""Pins of the SCS oracle (oracle/scs.py) against what the paper and the
mathematics fix, not against its own formulas:

* the Sherman-Morrison form of the affine projection equals a dense solve of
  (1 + Q) u = a with Q written out as the skew-symmetric block matrix of the
  homogeneous self-dual embedding (App. D.1), and M^-1 solves M z = a;
* closed-form optima at d = 2: for G = F_mu an allowed Pauli-string basis
  element the value is 1 (Hoelder: tr[W F] <= ||F||_op tr W = (1/4)(4),
  reached by W = (1 + P)/4); a forbidden element gives 0 (tr[W F] = 0 on the
  process subspace); G = 1 gives tr W = d^2 = 4 (c = 0, the degenerate
  objective);
* on a random GYNI instance solved to eps = 1e-9, an optimality certificate
  built with the trace-and-replace projector and LAPACK eigenvalues, which
  share nothing with the iteration: s and y PSD, s in the process subspace
  with tr s = d^2, y + G orthogonal to the traceless process subspace, the
  game value between the trivial process's tr G / d^2 and the dual bound,
  and primal and dual values equal;
* the embedding's invariants at every iterate: the slack block of v is PSD
  (Moreau: v_s = Pi(-(u~ - v)_s)), tau, kappa >= 0, v_x = 0;
* the optimum does not depend on the partial normalisation or on the
  over-relaxation; a warm start at the solution stops at once;
* post-processing leaves a PSD process matrix with lambda_min = 0 exactly
  when the input had a negative eigenvalue;
* Anderson acceleration: the accelerated solve reaches the same certified
  optimum, and with memory 1 the step is the secant step written out by
  hand (gamma = s^T f / s^T y).
"""
import numpy as np
import pytest

import oracle
from oracle import affine as AF
from oracle import scs
from paper_2606_20519_amd import workloads as W


@pytest.fixture(scope="module")
def gyni2():
    g = W.upper_pack(W.gyni_objective(2, 7))
    prob = scs.problem(g, 2)
    return g, prob


def test_sherman_morrison_is_the_dense_solve(gyni2):
    _, prob = gyni2
    sv = scs.Solver(prob)
    a, nx, ny = prob["A"], sv.nx, sv.ny
    c, b = sv.cs, prob["b"]
    q = np.zeros((nx + ny + 1, nx + ny + 1))
    q[:nx, nx:nx + ny] = a.T
    q[:nx, -1] = c
    q[nx:nx + ny, :nx] = -a
    q[nx:nx + ny, -1] = b
    q[-1, :nx] = -c
    q[-1, nx:nx + ny] = -b
    assert np.allclose(q, -q.T)
    rng = np.random.default_rng(3)
    rhs = rng.standard_normal(nx + ny + 1)
    ref = np.linalg.solve(np.eye(nx + ny + 1) + q, rhs)
    u_xy, u_tau = sv.affine(rhs[:-1], rhs[-1])
    np.testing.assert_allclose(u_xy, ref[:-1], atol=1e-12)
    assert abs(u_tau - ref[-1]) < 1e-12
    # M^-1 alone
    m = np.block([[np.eye(nx), a.T], [-a, np.eye(ny)]])
    z = sv.m_inverse(rhs[:-1])
    np.testing.assert_allclose(m @ z, rhs[:-1], atol=1e-12)


@pytest.mark.parametrize("which, value", [(0, 1.0), (40, 1.0), (86, 1.0), ("forbidden", 0.0), ("identity", 4.0)])
def test_closed_form_optima(which, value):
    sig = AF.gellmann(2)
    idx = AF.allowed_indices(2)
    if which == "identity":
        g = np.eye(16)
    elif which == "forbidden":
        g = AF.basis_element(sig, (0, 1, 0, 0))      # transformation-like A_o alone
        assert (0, 1, 0, 0) not in idx
    else:
        g = AF.basis_element(sig, idx[which])
        # a Pauli string over 4: eigenvalues +-1/4
        np.testing.assert_allclose(np.abs(np.linalg.eigvalsh(g)), 0.25, atol=1e-15)
    r = scs.solve(oracle.pack(g), 2, eps=1e-9, max_iters=20000)
    assert r["converged"]
    assert abs(r["res"]["pobj"] - value) < 1e-7
    assert abs(r["res"]["dobj"] - value) < 1e-7


def _psd_min(s, n):
    return float(np.linalg.eigvalsh(oracle.unpack(s, n))[0])


def test_certificate_gyni(gyni2):
    g, prob = gyni2
    d, n = 2, 16
    r = scs.solve(g, d, eps=1e-9, prob=prob, max_iters=20000)
    assert r["converged"]
    smat, ymat, gmat = oracle.unpack(r["s"], n), oracle.unpack(r["y"], n), prob["G"]
    tol = 1e-7
    assert _psd_min(r["s"], n) >= -1e-12                    # s in the cone
    assert _psd_min(r["y"], n) >= -1e-12                    # y in the dual cone
    np.testing.assert_allclose(AF.p_proc(smat, d), smat, atol=tol)   # process subspace
    assert abs(np.trace(smat).real - d * d) < tol                      # tr W = d_Ao d_Bo
    z = ymat + gmat                                          # dual feasibility
    np.testing.assert_allclose(AF.p_proc(z, d) - np.trace(z) / n * np.eye(n), 0, atol=tol)
    value = np.trace(smat @ gmat).real
    bound = np.trace(z).real / d ** 2
    trivial = np.trace(gmat).real / d ** 2
    assert trivial <= value + tol and value <= bound + tol and bound <= 1.0
    assert abs(value - bound) < 1e-7
    assert abs(r["res"]["pobj"] - value) < 1e-7 and abs(r["res"]["dobj"] - bound) < 1e-7


def test_iterate_invariants(gyni2):
    _, prob = gyni2
    sv = scs.Solver(prob)
    sv.start()
    for k in range(60):
        sv.step()
        assert sv.ut >= 0 and sv.vk >= 0
        assert np.all(sv.v[: sv.nx] == 0)
        assert _psd_min(sv.v[sv.nx:], 16) >= -1e-13 * max(1.0, np.abs(sv.v).max())
        assert _psd_min(sv.u[sv.nx:], 16) >= -1e-13 * max(1.0, np.abs(sv.u).max())


def test_normalisation_relaxation_warm_start(gyni2):
    g, prob = gyni2
    ref = scs.solve(g, 2, eps=1e-9, prob=prob, max_iters=20000)
    for kw in ({"normalize": False}, {"alpha": 1.0}):
        r = scs.solve(g, 2, eps=1e-9, prob=prob, max_iters=40000, **kw)
        assert r["converged"]
        assert abs(r["res"]["pobj"] - ref["res"]["pobj"]) < 1e-7
    warm = scs.solve(g, 2, eps=1e-7, prob=prob, warm=(ref["x"], ref["y"], ref["s"]))
    assert warm["converged"] and warm["iters"] <= 2


def test_postprocess_restores_psd(gyni2):
    g, prob = gyni2
    r = scs.solve(g, 2, eps=1e-3, prob=prob)
    w = scs.process_matrix(prob, r["x"])
    lmin = _psd_min(w, 16)
    rng = np.random.default_rng(4)
    if lmin >= 0:       # push it out of the cone along an allowed direction
        w = w + 0.5 * (prob["A"] @ rng.standard_normal(prob["A"].shape[1]))
    lmin = _psd_min(w, 16)
    assert lmin < 0
    w2, lam = scs.postprocess(w, 16, prob["gamma"])
    assert 0 < lam < 1
    assert abs(_psd_min(w2, 16)) < 1e-14
    m2 = oracle.unpack(w2, 16)
    np.testing.assert_allclose(AF.p_proc(m2, 2), m2, atol=1e-13)
    assert abs(np.trace(m2).real - 4.0) < 1e-13


def test_anderson_same_optimum(gyni2):
    g, prob = gyni2
    ref = scs.solve(g, 2, eps=1e-9, prob=prob, max_iters=20000)
    acc = scs.solve(g, 2, eps=1e-9, prob=prob, max_iters=20000, anderson=5)
    assert acc["converged"]
    assert abs(acc["res"]["pobj"] - ref["res"]["pobj"]) < 1e-7
    assert abs(acc["res"]["dobj"] - ref["res"]["dobj"]) < 1e-7
    assert acc["aa"][0] > 0


def test_anderson_memory_one_is_the_secant_step():
    # with one stored pair (s, y) the type-I system is the scalar
    # (s^T y + lam) gamma = s^T f; the next input g - (s - y) gamma
    rng = np.random.default_rng(9)
    aa = scs.Anderson(1)
    q0, g0 = rng.standard_normal(7), rng.standard_normal(7)
    assert np.array_equal(aa.next_input(q0, g0), g0)          # no pair yet: the plain step
    q1, g1 = g0, rng.standard_normal(7)
    out = aa.next_input(q1, g1)
    s, y, f = q1 - q0, (q1 - g1) - (q0 - g0), q1 - g1
    lam = scs.AA_REG * np.linalg.norm(s) * np.linalg.norm(y)
    gam = (s @ f) / (s @ y + lam)
    np.testing.assert_allclose(out, g1 - (s - y) * gam, rtol=1e-13, atol=1e-13)
