"""The reading behind the warm-started projection, checked on the CPU with
plain matrix products (no GPU code): one refinement step of the eigen-pair,
as the device kernels form it from the lower triangles of S = X^H A X and
G = X^H X (E_ii = (1 - G_ii)/2; E_ij = (S_ij - lambda_j G_ij)/(lambda_j -
lambda_i) for the lower entry and, from the conjugates of the same two
values, E_ji; pairs closer than 2^-40 max|lambda| kept whole), squares the
error of a nearby basis, and X diag(max(lambda, 0)) X^H with the step's
Rayleigh quotients reaches the oracle's projection."""
import numpy as np

import oracle
from paper_2606_20519_amd import workloads as W


def step(a, x):
    s = x.conj().T @ (a @ x)
    g = x.conj().T @ x
    lam = s.diagonal().real / g.diagonal().real
    tau = 2.0 ** -40 * np.abs(lam).max()
    n = len(a)
    e = np.zeros_like(a)
    for j in range(n):
        e[j, j] = 0.5 * (1.0 - g[j, j].real)
        for i in range(j + 1, n):
            d = lam[j] - lam[i]
            if abs(d) > tau:
                e[i, j] = (s[i, j] - lam[j] * g[i, j]) / d
                e[j, i] = (np.conj(s[i, j]) - lam[i] * np.conj(g[i, j])) / (-d)
            else:
                e[i, j] = -0.5 * g[i, j]
                e[j, i] = -0.5 * np.conj(g[i, j])
    off = np.abs(e - np.diag(e.diagonal())).max()
    return x + x @ e, lam, off


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_refinement_squares_the_error_and_reaches_the_projection():
    n = 40
    xs = W.warm_sequence(n, 4242, 2)
    a0, a1 = oracle.unpack(xs[0], n), oracle.unpack(xs[1], n)
    _, v0 = np.linalg.eigh(a0)
    exact = oracle.unpack(oracle.project(xs[1], n), n)
    x, offs = v0, []
    for _ in range(5):
        x, lam, off = step(a1, x)
        offs.append(off)
        if off <= 1e-7:
            break
    # quadratic: each step's rotation at most a modest multiple of the square of the last
    for p, q in zip(offs, offs[1:]):
        assert q <= 10.0 * p * p + 1e-14, offs
    assert offs[-1] <= 1e-7 and len(offs) <= 5, offs
    pi = (x * np.maximum(lam, 0.0)) @ x.conj().T
    assert rel(pi, exact) <= 1e-12


def test_repeated_eigenvalues_stay_exact_from_their_own_basis():
    n = 24
    rng = np.random.default_rng(77)
    u = W.haar_unitary(n, rng)
    lam = np.repeat([-1.0, 0.5, 2.0], n // 3)
    a = (u * lam[None, :]) @ u.conj().T
    a = (a + a.conj().T) / 2.0
    x, lt, off = step(a, u)
    assert off <= 1e-12
    pi = (x * np.maximum(lt, 0.0)) @ x.conj().T
    exact = oracle.constructed_projection(u, lam)
    assert rel(oracle.pack(pi), exact) <= 1e-12
