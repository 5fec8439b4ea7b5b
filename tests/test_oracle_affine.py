"""Pins of the affine-step oracle (oracle/affine.py) against what the paper
and the mathematics fix, independently of its own Gell-Mann construction:

* the local basis is orthonormal, Hermitian and traceless apart from
  sigma_0 (so that A^T A = I, App. D.1);
* the allowed multi-indices number d^8 - (1 + d^2(d^2-1))^2 (the paper's
  count for two parties, identity excluded): 87 for qubits;
* A A^T y = P_proc(y) - tr(y)/d_tot 1 (App. D.1), with P_proc built from
  partial traces (trace-and-replace maps, eq. projector_definition) -- a
  formula that shares nothing with the Gell-Mann tensors;
* P_proc is an idempotent, self-adjoint projector whose image satisfies the
  three process constraints, and it fixes the trivial process 1/d^2;
* (z_x, z_y) solves the affine system [[1, A^T], [-A, 1]] z = a
  (eq. main_system_affine), which needs A^T A = I.
"""
import numpy as np
import pytest

import oracle
from oracle import affine as AF

EPS = np.finfo(np.float64).eps


def rand_herm(n, rng):
    g = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2)
    return (g + g.conj().T) / 2


@pytest.mark.parametrize("d", [2, 3, 4])
def test_gellmann_orthonormal(d):
    sig = AF.gellmann(d)
    assert len(sig) == d * d
    gram = np.array([[np.trace(a.conj().T @ b) for b in sig] for a in sig])
    np.testing.assert_allclose(gram, np.eye(d * d), atol=1e-14)
    for k, s in enumerate(sig):
        np.testing.assert_allclose(s, s.conj().T, atol=0)
        if k:
            assert abs(np.trace(s)) < 1e-14


@pytest.mark.parametrize("d", [2, 3])
def test_allowed_count(d):
    D = d * d
    n = len(AF.allowed_indices(d))
    assert n == AF.count_allowed(d) == (D - 1) * (2 * D * D - D + 1)
    if d == 2:
        assert n == 87


@pytest.mark.parametrize("d", [2, 3])
def test_constraint_map_isometry_and_projector(d):
    rng = np.random.default_rng(10 + d)
    nx = AF.count_allowed(d)
    x = rng.standard_normal(nx)
    # A^T A = I
    np.testing.assert_allclose(AF.constraint_adjoint(AF.constraint_apply(x, d), d), x, atol=1e-12)
    # A A^T y = P_proc(y) - tr(y)/d_tot 1 (trace-and-replace form)
    y = rand_herm(d ** 4, rng)
    lhs = AF.constraint_apply(AF.constraint_adjoint(y, d), d)
    rhs = AF.p_proc(y, d) - np.trace(y) / d ** 4 * np.eye(d ** 4)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("d", [2, 3])
def test_p_proc_is_the_process_projector(d):
    rng = np.random.default_rng(20 + d)
    m = rand_herm(d ** 4, rng)
    p = AF.p_proc(m, d)
    np.testing.assert_allclose(AF.p_proc(p, d), p, atol=1e-12)                # idempotent
    m2 = rand_herm(d ** 4, rng)
    assert abs(np.trace(AF.p_proc(m2, d) @ m) - np.trace(m2 @ p)) < 1e-10   # self-adjoint
    tr = lambda *s: AF.trace_replace(p, d, s)
    np.testing.assert_allclose(tr(AF.AI, AF.AO), tr(AF.AI, AF.AO, AF.BO), atol=1e-12)
    np.testing.assert_allclose(tr(AF.BI, AF.BO), tr(AF.AO, AF.BI, AF.BO), atol=1e-12)
    np.testing.assert_allclose(p, tr(AF.AO) + tr(AF.BO) - tr(AF.AO, AF.BO), atol=1e-12)
    w = np.eye(d ** 4) / d ** 2                                             # trivial process
    np.testing.assert_allclose(AF.p_proc(w, d), w, atol=1e-14)
    assert abs(np.trace(w) - d * d) < 1e-12                                 # tr W = d_Ao d_Bo


@pytest.mark.parametrize("d", [2, 3])
def test_affine_step_solves_the_system(d):
    rng = np.random.default_rng(30 + d)
    ax = rng.standard_normal(AF.count_allowed(d))
    ay = rand_herm(d ** 4, rng)
    zx, zy = AF.affine_step(ax, ay, d)
    np.testing.assert_allclose(zx + AF.constraint_adjoint(zy, d), ax, atol=1e-12)
    np.testing.assert_allclose(-AF.constraint_apply(zx, d) + zy, ay, atol=1e-12)


def test_trace_replace_definition():
    # _X M = 1_X/d (x) tr_X M on a product operator: replaces that factor by
    # its trace times the maximally mixed state
    d = 2
    rng = np.random.default_rng(5)
    f = [rand_herm(d, rng) for _ in range(4)]
    m = np.kron(np.kron(f[0], f[1]), np.kron(f[2], f[3]))
    g = list(f)
    g[1] = np.trace(f[1]) * np.eye(d) / d
    ref = np.kron(np.kron(g[0], g[1]), np.kron(g[2], g[3]))
    np.testing.assert_allclose(AF.trace_replace(m, d, (AF.AO,)), ref, atol=1e-14)


def test_gellmann_qubit_is_pauli():
    # d = 2: (1, sigma_z, sigma_x, sigma_y) / sqrt2 in the paper's order
    # (identity, diagonal, symmetric, antisymmetric), written out by hand
    s = 1 / np.sqrt(2)
    pauli = [np.array([[1, 0], [0, 1]]), np.array([[1, 0], [0, -1]]),
             np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]])]
    for got, want in zip(AF.gellmann(2), pauli):
        np.testing.assert_allclose(got, s * want, atol=1e-15)
