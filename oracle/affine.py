"""CPU FP64 oracle of the affine step of the paper's SCS iteration for the
bipartite process-matrix SDP -- TEST INFRASTRUCTURE ONLY (imported by tests,
never by the GPU library).

Everything here is the plain definition, written with explicit matrices:

* ``gellmann(d)`` -- the orthonormal Hermitian local basis of App. A
  (eq. gellmann_basis): sigma_0 = 1/sqrt(d), the diagonal elements
  sqrt(1/((l+1)(l+2))) (sum_{j<=l} |j><j| - (l+1)|l+1><l+1|), l = 0..d-2, the
  symmetric (|j><k| + |k><j|)/sqrt2 and the antisymmetric
  -i(|j><k| - |k><j|)/sqrt2 off-diagonal elements, j < k in lexicographic
  order.
* ``allowed_indices(d)`` -- the multi-indices mu = (alpha_1, beta_1,
  alpha_2, beta_2) of F_mu = sigma_a1 (x) sigma_b1 (x) sigma_a2 (x) sigma_b2 on
  A_i (x) A_o (x) B_i (x) B_o kept by the process constraints
  (App. "Sparse basis for the process-matrix subspace"): every party in the
  transformation-like sector (beta >= 1) needs a party in the effect-like
  sector (alpha >= 1, beta = 0); the all-identity index is excluded (the
  trace normalisation fixes it).  Lexicographic order of mu.
* ``constraint_apply`` / ``constraint_adjoint`` -- A x = -sum_mu x_mu F_mu and
  (A^T Z)_mu = -tr[F_mu Z] (App. D.1, eq. constraint_map_def), with F_mu
  formed by Kronecker products.
* ``affine_step`` -- z_x = (a_x - A^T a_y)/2, z_y = a_y + A z_x, the closed
  form of the affine projection when A^T A = I (App. D.2).
* ``p_proc`` -- the projector onto the process-matrix subspace by
  trace-and-replace maps (App. "Projector-based SDP formulation", eq.
  projector_definition), independent of the Gell-Mann basis: the pin
  A A^T y = P_proc(y) - tr(y)/d_tot 1 of App. D.1 ties the two together.

Matrices travel as the library's svec (``oracle.pack`` / ``oracle.unpack``).
"""
from __future__ import annotations

import itertools

import numpy as np


def gellmann(d: int) -> list:
    """Local basis sigma_alpha, alpha = 0..d^2-1, in the order above."""
    out = [np.eye(d, dtype=np.complex128) / np.sqrt(d)]
    for l in range(d - 1):
        m = np.zeros((d, d), dtype=np.complex128)
        for j in range(l + 1):
            m[j, j] = 1.0
        m[l + 1, l + 1] = -(l + 1)
        out.append(m * np.sqrt(1.0 / ((l + 1) * (l + 2))))
    pairs = [(j, k) for j in range(d) for k in range(j + 1, d)]
    for j, k in pairs:
        m = np.zeros((d, d), dtype=np.complex128)
        m[j, k] = m[k, j] = 1.0 / np.sqrt(2.0)
        out.append(m)
    for j, k in pairs:
        m = np.zeros((d, d), dtype=np.complex128)
        m[j, k] = -1j / np.sqrt(2.0)
        m[k, j] = 1j / np.sqrt(2.0)
        out.append(m)
    return out


def sector(alpha: int, beta: int) -> str:
    """Sector of one party's local index pair: baseline, effect-like or
    transformation-like."""
    if beta >= 1:
        return "T"
    return "E" if alpha >= 1 else "B"


def allowed_indices(d: int) -> list:
    """Allowed traceless multi-indices (alpha_1, beta_1, alpha_2, beta_2),
    lexicographic."""
    D = d * d
    out = []
    for mu in itertools.product(range(D), repeat=4):
        s1, s2 = sector(mu[0], mu[1]), sector(mu[2], mu[3])
        has_t = "T" in (s1, s2)
        has_e = "E" in (s1, s2)
        if has_t and not has_e:
            continue              # forbidden
        if s1 == "B" and s2 == "B":
            continue              # the identity: fixed by the trace
        out.append(mu)
    return out


def basis_element(sig: list, mu) -> np.ndarray:
    """F_mu = sigma_a1 (x) sigma_b1 (x) sigma_a2 (x) sigma_b2."""
    f = sig[mu[0]]
    for a in mu[1:]:
        f = np.kron(f, sig[a])
    return f


def constraint_apply(x, d: int) -> np.ndarray:
    """A x = -sum_mu x_mu F_mu as a dense d^4 x d^4 matrix."""
    sig = gellmann(d)
    idx = allowed_indices(d)
    n = d ** 4
    y = np.zeros((n, n), dtype=np.complex128)
    for xm, mu in zip(np.asarray(x, dtype=np.float64), idx):
        y -= xm * basis_element(sig, mu)
    return y


def constraint_adjoint(z, d: int) -> np.ndarray:
    """(A^T Z)_mu = -tr[F_mu Z] (real for Hermitian Z)."""
    sig = gellmann(d)
    z = np.asarray(z, dtype=np.complex128)
    out = np.empty(len(allowed_indices(d)))
    for i, mu in enumerate(allowed_indices(d)):
        out[i] = -np.real(np.sum(basis_element(sig, mu).T * z))   # tr[F Z] = sum_ab F_ba Z_ab
    return out


def affine_step(ax, ay_mat, d: int):
    """(z_x, z_y) = ((a_x - A^T a_y)/2, a_y + A z_x) (App. D.2), z_y dense."""
    zx = 0.5 * (np.asarray(ax, dtype=np.float64) - constraint_adjoint(ay_mat, d))
    zy = np.asarray(ay_mat, dtype=np.complex128) + constraint_apply(zx, d)
    return zx, zy


def trace_replace(m: np.ndarray, d: int, systems) -> np.ndarray:
    """_X M = 1_X/d_X (x) tr_X M for the listed subsystems X of
    A_i (x) A_o (x) B_i (x) B_o (indices 0..3), every one of dimension d."""
    t = np.asarray(m, dtype=np.complex128).reshape([d] * 8)  # rows a0..a3, columns b0..b3
    for s in systems:
        tr = np.trace(t, axis1=s, axis2=4 + s)                 # removes both axes of s
        tr = np.expand_dims(np.expand_dims(tr, s), 4 + s)
        eye = np.eye(d).reshape([d if k in (s, 4 + s) else 1 for k in range(8)])
        t = tr * eye / d
    return t.reshape(d ** 4, d ** 4)


AI, AO, BI, BO = 0, 1, 2, 3


def p_proc(m: np.ndarray, d: int) -> np.ndarray:
    """P_proc[M] = _AoM + _BoM - _AoBoM - _AiAoM - _BiBoM + _AoBiBoM + _AiAoBoM."""
    tr = lambda *s: trace_replace(m, d, s)
    return (tr(AO) + tr(BO) - tr(AO, BO) - tr(AI, AO) - tr(BI, BO) + tr(AO, BI, BO) + tr(AI, AO, BO))


def count_allowed(d: int) -> int:
    """|I| = d^8 - (1 + d^2 (d^2 - 1))^2: the paper's count of allowed
    multi-indices for two parties, without the identity."""
    return d ** 8 - (1 + d * d * (d * d - 1)) ** 2
