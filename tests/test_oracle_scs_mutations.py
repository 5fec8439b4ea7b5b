"""Planted mistakes in the SCS oracle must be caught by its pins.

Each case copies ``oracle/scs.py``, plants one plausible mistake (a wrong
sign, a dropped or misplaced term, a wrong constant), loads the copy as a
fresh module and runs a compact battery of the pins of test_oracle_scs.py
against it: the Sherman-Morrison step against a dense solve of (1 + Q) u = a,
the embedding's invariants along the iterates, a closed-form optimum at
d = 2, an optimality certificate from the
trace-and-replace projector, post-processing, and the Anderson step.  The
battery must fail for every mutant (and pass for the unmodified source).
"""
import os
import types

import numpy as np
import pytest

import oracle
from oracle import affine as AF
from paper_2606_20519_amd import workloads as W

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "scs.py")

MUTANTS = {
    "sherman_morrison_sign": ("u_xy = w - self.mh * (self.h @ w) / (1.0 + self.eta)",
                              "u_xy = w + self.mh * (self.h @ w) / (1.0 + self.eta)"),
    "sherman_morrison_denominator": ("(self.h @ w) / (1.0 + self.eta)", "(self.h @ w) / self.eta"),
    "tau_row_sign": ("u_tau = a_tau + self.cs @ u_xy", "u_tau = a_tau - self.cs @ u_xy"),
    "m_inverse_sign": ("zy = ay + a @ zx", "zy = ay - a @ zx"),
    "relaxation_on_v": ("r_xy = self.alpha * ut_xy + (1.0 - self.alpha) * self.u",
                        "r_xy = self.alpha * ut_xy + (1.0 - self.alpha) * self.v"),
    "dual_update_sign": ("self.v = u_new - q_xy", "self.v = q_xy - u_new"),
    "tau_not_clamped": ("return out, max(w_tau, 0.0)", "return out, w_tau"),
    "gamma_dtot": ("gamma = 1.0 / d ** 2", "gamma = 1.0 / d ** 4"),
    "c_sign": ('"c": -bmu,', '"c": bmu,'),
    "dual_residual_sign": ('du = aty + p["c"]', 'du = aty - p["c"]'),
    "postprocess_lambda": ("lam = -lmin / (gamma - lmin)", "lam = -lmin / gamma"),
    "anderson_sign": ("return g - (S - Y) @ gam", "return g + (S - Y) @ gam"),
    "anderson_normal_equations": ("S.T @ Y + lam * np.eye(S.shape[1]), S.T @ f",
                                  "Y.T @ Y + lam * np.eye(S.shape[1]), S.T @ f"),
}


def load(text: str):
    mod = types.ModuleType("scs_mutant")
    exec(compile(text, "scs_mutant.py", "exec"), mod.__dict__)
    return mod


def battery(M):
    """Raises (AssertionError or another error) if any pin fails."""
    d, n = 2, 16
    g = W.upper_pack(W.gyni_objective(2, 7))
    prob = M.problem(g, d)
    # (1) Sherman-Morrison step = dense solve of (1 + Q) u = a
    sv = M.Solver(prob)
    a, nx, ny = prob["A"], sv.nx, sv.ny
    q = np.zeros((nx + ny + 1, nx + ny + 1))
    q[:nx, nx:nx + ny], q[:nx, -1] = a.T, sv.cs
    q[nx:nx + ny, :nx], q[nx:nx + ny, -1] = -a, prob["b"]
    q[-1, :nx], q[-1, nx:nx + ny] = -sv.cs, -prob["b"]
    rhs = np.random.default_rng(3).standard_normal(nx + ny + 1)
    ref = np.linalg.solve(np.eye(nx + ny + 1) + q, rhs)
    u_xy, u_tau = sv.affine(rhs[:-1], rhs[-1])
    assert np.allclose(u_xy, ref[:-1], atol=1e-12) and abs(u_tau - ref[-1]) < 1e-12
    # (2) the embedding's invariants along the iterates: tau, kappa >= 0, v_s PSD
    sv.start()
    for _ in range(30):
        sv.step()
        assert sv.ut >= 0 and sv.vk >= 0
        assert np.linalg.eigvalsh(oracle.unpack(sv.v[nx:], n))[0] >= -1e-12 * max(1.0, np.abs(sv.v).max())
    # (3) closed-form optimum: an allowed Pauli string has value 1
    f = AF.basis_element(AF.gellmann(2), AF.allowed_indices(2)[40])
    r = M.solve(oracle.pack(f), d, eps=1e-8, max_iters=4000)
    assert r["converged"] and abs(r["res"]["pobj"] - 1.0) < 1e-6
    # (4) certificate on the GYNI instance
    r = M.solve(g, d, eps=1e-8, prob=prob, max_iters=8000)
    assert r["converged"]
    smat, ymat, gmat = oracle.unpack(r["s"], n), oracle.unpack(r["y"], n), oracle.unpack(g, n)
    assert np.linalg.eigvalsh(smat)[0] >= -1e-10 and np.linalg.eigvalsh(ymat)[0] >= -1e-10
    assert np.allclose(AF.p_proc(smat, d), smat, atol=1e-6)
    assert abs(np.trace(smat).real - 4.0) < 1e-6
    z = ymat + gmat
    assert np.allclose(AF.p_proc(z, d) - np.trace(z) / n * np.eye(n), 0, atol=1e-6)
    value, bound = np.trace(smat @ gmat).real, np.trace(z).real / 4
    assert abs(value - bound) < 1e-6 and abs(r["res"]["pobj"] - value) < 1e-6
    # (5) post-processing: lambda_min = 0 after mixing
    w = M.process_matrix(prob, r["x"]) + 0.5 * (prob["A"] @ np.random.default_rng(4).standard_normal(nx))
    w2, lam = M.postprocess(w, n, prob["gamma"])
    assert 0 < lam < 1 and abs(np.linalg.eigvalsh(oracle.unpack(w2, n))[0]) < 1e-13
    # (6) Anderson: the same certified optimum; memory one is the secant step
    ra = M.solve(g, d, eps=1e-8, prob=prob, max_iters=8000, anderson=5)
    assert ra["converged"] and abs(ra["res"]["pobj"] - value) < 1e-6
    aa = M.Anderson(1)
    rng = np.random.default_rng(9)
    q0, g0 = rng.standard_normal(7), rng.standard_normal(7)
    aa.next_input(q0, g0)
    g1 = rng.standard_normal(7)
    out = aa.next_input(g0, g1)
    s_, y_, f_ = g0 - q0, (g0 - g1) - (q0 - g0), g0 - g1
    gam = (s_ @ f_) / (s_ @ y_ + M.AA_REG * np.linalg.norm(s_) * np.linalg.norm(y_))
    assert np.allclose(out, g1 - (s_ - y_) * gam, atol=1e-13)


def test_unmodified_source_passes():
    battery(load(open(SRC).read()))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, name
    mutant = load(text.replace(old, new))
    with np.errstate(all="ignore"):
        with pytest.raises(Exception):
            battery(mutant)
