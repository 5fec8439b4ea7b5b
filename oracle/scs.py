"""CPU FP64 oracle of the paper's SCS iteration for the process-matrix SDP --
TEST INFRASTRUCTURE ONLY (imported by tests, never by the GPU library).

The problem (App. D, eq. scs_canonical_form with the correspondence of eq.
constraint_map_def): maximise tr[W G] over process matrices
W = gamma 1 + sum_mu w_mu F_mu >= 0 (eq. sparse_process_sdp), written for SCS
as

    min c^T x  s.t.  A x + s = b,  s in H_+^{d_tot},

with x = (w_mu), A x = -sum_mu x_mu F_mu, b = gamma 1, c = -(b_mu),
b_mu = tr[G F_mu], gamma = tr W / d_tot = 1/d^2 (tr W = d_Ao d_Bo = d^2,
d_tot = d^4), and the dropped constant b_0 = gamma tr G.  The game value of
x is b_0 - c^T x; weak duality bounds it by b_0 + b^T y for every dual
feasible y.

Everything below is the plain definition with explicit matrices:

* ``problem`` -- A as the dense matrix of columns -vec_R(F_mu) (Kronecker
  products of the Gell-Mann matrices), b, c from the traces tr[G F_mu].
* ``Solver.m_inverse`` -- z = M^-1 a for M = [[1, A^T], [-A, 1]] by the reduced
  system (1 + A^T A) z_x = a_x - A^T a_y, z_y = a_y + A z_x (eq.
  projection_system), with 1 + A^T A formed and inverted by a library routine
  -- the general form, not the A^T A = 1 shortcut that the GPU path takes.
* ``Solver.affine`` -- u~ = (1 + Q)^-1 a by the Sherman-Morrison form of App. D.1
  ("Solving the affine projection"): u~_xy = (1 - (M^-1 h) h^T /
  (1 + h^T M^-1 h)) (M^-1 a_xy - a_tau M^-1 h), u~_tau = a_tau + c^T u~_x +
  b^T u~_y, with h = (c, b).
* ``Solver.cone_input`` / ``cone_step`` -- the iteration of eq. final_iterates: u~ = (1 + Q)^-1 (u + v),
  u = Pi_C(u~ - v), v = v - u~ + u, with C = R^n x H_+ x R_+; over-relaxation
  replaces u~ in the last two updates by alpha u~ + (1 - alpha) u (alpha = 1
  is the printed iteration).
* ``Solver.residuals`` -- the termination test of App. D.1 ("Convergence criteria")
  on x = u_x/tau, s = v_s/tau, y = u_y/tau, with eps_abs = eps_rel = eps.
* ``solve`` -- cold start u = v = (0, 0, 1) or a warm start u = (x, y, 1),
  v = (0, s, 0); partial normalisation (App. D.2): c is scaled by
  sigma = ||b|| / ||c|| inside the iteration, so that the two norms agree,
  and the residuals are reported for the unscaled problem (y = u_y /
  (sigma tau)); projections in FP64 by the Jacobi oracle.
* ``Anderson`` -- type-I Anderson acceleration (the paper keeps SCS's;
  App. D.2).  The iterate is fixed by the cone step's input q = u~_r - v
  alone (u = Pi_C(q), v = u - q by Moreau), so the iteration is the
  fixed-point map q -> G(q) (project q, then the affine step), of dimension
  n_x + n_y + 1, and the acceleration acts on q: with the last m differences
  s_i = q_{i+1} - q_i and y_i = f_{i+1} - f_i of the inputs and of the
  residuals f = q - G(q), gamma solves (S^T Y + lam 1) gamma = S^T f_k,
  lam = 1e-8 ||S||_F ||Y||_F, and the next input is G(q_k) - (S - Y) gamma.
  Safeguard: when the residual at an accelerated input exceeds twice the
  previous one, the plain G(q_{k-1}) it replaced is projected instead and
  the memory is cleared; a step with max |gamma| > 1e10 or a singular
  system is not taken.  (Type-I Anderson with these safeguards after Zhang, O'Donoghue
  and Boyd, SIAM J. Optim. 2020; the constants are this solver's reading.)
* ``postprocess`` -- W' = (1 - lam) W + lam gamma 1 with the smallest
  lam in [0, 1] that makes W' PSD (App. "Sparse SDP formulation for process
  matrices and post-processing").
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle import affine as AF


def problem(g_svec, d: int) -> dict:
    """Data (A, b, c, b_0, gamma) of the process-matrix SDP for the objective
    G (svec of a d^4 x d^4 Hermitian matrix)."""
    n = d ** 4
    gmat = oracle.unpack(np.asarray(g_svec, dtype=np.float64), n)
    sig = AF.gellmann(d)
    idx = AF.allowed_indices(d)
    cols = []
    bmu = np.empty(len(idx))
    for k, mu in enumerate(idx):
        f = AF.basis_element(sig, mu)
        cols.append(-oracle.pack(f))
        bmu[k] = np.real(np.trace(gmat @ f))
    gamma = 1.0 / d ** 2
    return {
        "d": d, "n": n,
        "A": np.column_stack(cols),
        "b": oracle.pack(gamma * np.eye(n)),
        "c": -bmu,
        "gamma": gamma,
        "b0": gamma * float(np.real(np.trace(gmat))),
        "G": gmat,
    }


class Solver:
    """State and fixed factors of one SCS run (see the module docstring)."""

    def __init__(self, prob: dict, alpha: float = 1.5, normalize: bool = True):
        self.p = prob
        a = prob["A"]
        self.nx, self.ny = a.shape[1], a.shape[0]
        c, b = prob["c"], prob["b"]
        nc = np.linalg.norm(c)
        self.sigma = (np.linalg.norm(b) / nc) if (normalize and nc > 0) else 1.0
        self.cs = self.sigma * c                      # the iteration's c
        self.alpha = alpha
        self.kinv = np.linalg.inv(np.eye(self.nx) + a.T @ a)
        self.h = np.concatenate([self.cs, b])
        self.mh = self.m_inverse(self.h)
        self.eta = float(self.h @ self.mh)

    def m_inverse(self, a_xy: np.ndarray) -> np.ndarray:
        a = self.p["A"]
        ax, ay = a_xy[: self.nx], a_xy[self.nx:]
        zx = self.kinv @ (ax - a.T @ ay)
        zy = ay + a @ zx
        return np.concatenate([zx, zy])

    def affine(self, a_xy: np.ndarray, a_tau: float):
        w = self.m_inverse(a_xy) - a_tau * self.mh
        u_xy = w - self.mh * (self.h @ w) / (1.0 + self.eta)
        u_tau = a_tau + self.cs @ u_xy[: self.nx] + self.p["b"] @ u_xy[self.nx:]
        return u_xy, float(u_tau)

    def cone(self, w_xy: np.ndarray, w_tau: float):
        """Pi_C on R^n x H_+ x R_+."""
        out = w_xy.copy()
        out[self.nx:] = oracle.project(w_xy[self.nx:], self.p["n"])
        return out, max(w_tau, 0.0)

    def start(self, warm=None):
        """u = v = (0, 0, 1) cold; u = (x, sigma y, 1), v = (0, s, 0) warm."""
        self.u = np.zeros(self.nx + self.ny)
        self.v = np.zeros(self.nx + self.ny)
        if warm is None:
            self.ut, self.vk = 1.0, 1.0
        else:
            x, y, s = warm
            self.u[: self.nx] = x
            self.u[self.nx:] = self.sigma * np.asarray(y)
            self.v[self.nx:] = s
            self.ut, self.vk = 1.0, 0.0

    def cone_input(self):
        """q = u~_r - v with u~ = (1 + Q)^-1 (u + v): the point the next cone
        step projects (x, y and tau parts)."""
        ut_xy, ut_tau = self.affine(self.u + self.v, self.ut + self.vk)
        r_xy = self.alpha * ut_xy + (1.0 - self.alpha) * self.u
        r_tau = self.alpha * ut_tau + (1.0 - self.alpha) * self.ut
        return r_xy - self.v, r_tau - self.vk

    def cone_step(self, q_xy: np.ndarray, q_tau: float):
        """u = Pi_C(q), v = v - u~_r + u = u - q (Moreau: v in C*)."""
        u_new, t_new = self.cone(q_xy, q_tau)
        self.v = u_new - q_xy
        self.v[: self.nx] = 0.0          # x is free: v_x = 0 exactly
        self.vk = t_new - q_tau
        self.u, self.ut = u_new, t_new

    def step(self):
        self.cone_step(*self.cone_input())

    def iterate_state(self):
        """(x, y, s, tau, kappa) of the current iterate, unscaled."""
        tau = self.ut
        x = self.u[: self.nx] / tau
        y = self.u[self.nx:] / (self.sigma * tau)
        s = self.v[self.nx:] / tau
        return x, y, s, tau, self.vk

    def residuals(self, eps: float) -> dict:
        p = self.p
        if not self.ut > 0.0:          # tau = 0: no primal-dual pair to test
            inf = float("inf")
            return {"res_pri": inf, "res_dual": inf, "gap": inf, "converged": False,
                    "pobj": float("nan"), "dobj": float("nan"), "tau": self.ut, "kappa": self.vk}
        x, y, s, tau, kappa = self.iterate_state()
        ax = p["A"] @ x
        aty = p["A"].T @ y
        pr = ax + s - p["b"]
        du = aty + p["c"]
        cx, by = float(p["c"] @ x), float(p["b"] @ y)
        g = cx + by
        inf = lambda v: float(np.max(np.abs(v))) if v.size else 0.0
        out = {
            "res_pri": inf(pr), "res_dual": inf(du), "gap": abs(g),
            "bound_pri": eps + eps * max(inf(ax), inf(s), inf(p["b"])),
            "bound_dual": eps + eps * max(inf(aty), inf(p["c"])),
            "bound_gap": eps + eps * max(abs(cx), abs(by)),
            "pobj": p["b0"] - cx, "dobj": p["b0"] + by, "tau": tau, "kappa": kappa,
        }
        out["converged"] = (tau > 0 and out["res_pri"] <= out["bound_pri"]
                            and out["res_dual"] <= out["bound_dual"]
                            and out["gap"] <= out["bound_gap"])
        return out


AA_REG = 1e-8
AA_MAX_WEIGHT = 1e10
AA_SAFEGUARD = 2.0


class Anderson:
    """Type-I Anderson acceleration of q -> G(q) with memory m (module
    docstring)."""

    def __init__(self, m: int):
        self.m = m
        self.accepted = self.rejected = 0
        self.reset()

    def reset(self):
        self.S, self.Y = [], []
        self.prev = None          # (q_k, f_k) of the last input
        self.g_save = None        # the plain G(q_{k-1}) behind an accelerated input
        self.nf_save = None       # ||f_{k-1}|| at that step

    def next_input(self, qk: np.ndarray, g: np.ndarray) -> np.ndarray:
        """Given the input q_k just projected and G(q_k), the next input."""
        f = qk - g
        nf = float(np.linalg.norm(f))
        if self.g_save is not None:           # q_k was accelerated: safeguard
            back, limit = self.g_save, self.nf_save
            self.g_save = None
            if not nf <= AA_SAFEGUARD * limit:
                self.reset()
                self.rejected += 1
                return back
        if self.prev is not None:
            self.S.append(qk - self.prev[0])
            self.Y.append(f - self.prev[1])
            if len(self.S) > self.m:
                self.S.pop(0)
                self.Y.pop(0)
        self.prev = (qk, f)
        if not self.S:
            return g
        S, Y = np.column_stack(self.S), np.column_stack(self.Y)
        lam = AA_REG * np.linalg.norm(S) * np.linalg.norm(Y)
        try:
            gam = np.linalg.solve(S.T @ Y + lam * np.eye(S.shape[1]), S.T @ f)
        except np.linalg.LinAlgError:
            return g
        if not np.all(np.isfinite(gam)) or np.max(np.abs(gam)) > AA_MAX_WEIGHT:
            return g
        self.g_save, self.nf_save = g, nf
        self.accepted += 1
        return g - (S - Y) @ gam


def solve(g_svec, d: int, eps: float = 1e-5, alpha: float = 1.5, max_iters: int = 5000,
          normalize: bool = True, warm=None, prob=None, anderson: int = 0) -> dict:
    """Run the iteration until the termination test holds (checked after
    every iteration) or `max_iters` iterations; eps = 0 runs exactly
    max_iters.  anderson = m > 0 accelerates the cone-step inputs.  Returns
    the unscaled (x, y, s), tau, kappa, the iteration count, the last
    residuals and the history of (res_pri, res_dual, gap)."""
    prob = prob if prob is not None else problem(g_svec, d)
    sv = Solver(prob, alpha=alpha, normalize=normalize)
    sv.start(warm)
    aa = Anderson(anderson) if anderson > 0 else None
    hist = []
    res = {"converged": False}
    it = 0
    q_xy, q_tau = sv.cone_input()
    for it in range(1, max_iters + 1):
        sv.cone_step(q_xy, q_tau)
        res = sv.residuals(eps)
        hist.append((res["res_pri"], res["res_dual"], res["gap"]))
        if eps > 0 and res["converged"]:
            break
        if it == max_iters:
            break
        g_xy, g_tau = sv.cone_input()
        if aa:
            nxt = aa.next_input(np.append(q_xy, q_tau), np.append(g_xy, g_tau))
            g_xy, g_tau = nxt[:-1], float(nxt[-1])
        q_xy, q_tau = g_xy, g_tau
    x, y, s, tau, kappa = sv.iterate_state()
    return {"x": x, "y": y, "s": s, "tau": tau, "kappa": kappa, "iters": it,
            "converged": bool(res["converged"]), "res": res, "history": hist,
            "sigma": sv.sigma, "prob": prob,
            "aa": (aa.accepted, aa.rejected) if aa else None}


def process_matrix(prob: dict, x) -> np.ndarray:
    """W = b - A x = gamma 1 + sum_mu x_mu F_mu (svec)."""
    return prob["b"] - prob["A"] @ np.asarray(x)


def postprocess(w_svec, n: int, gamma: float):
    """W' = (1 - lam) W + lam gamma 1, lam the smallest value in [0, 1] with
    W' PSD: lam = 0 if lambda_min(W) >= 0, else
    -lambda_min / (gamma - lambda_min).  Returns (svec W', lam)."""
    lmin = float(oracle.eigh(w_svec, n)[0][0])
    if lmin >= 0.0:
        return np.array(w_svec, dtype=np.float64), 0.0
    lam = -lmin / (gamma - lmin)
    w = oracle.unpack(w_svec, n)
    return oracle.pack((1.0 - lam) * w + lam * gamma * np.eye(n)), lam
