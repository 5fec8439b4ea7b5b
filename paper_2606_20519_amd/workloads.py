"""Seeded synthetic inputs for the PSD-cone projection (host-side NumPy).

This module is the only code shared by the GPU path's tests/benchmark and the
CPU oracle.  It draws random numbers and lays them out in the svec encoding;
it contains none of the projection's arithmetic.

svec encoding (App. D.1, vec_R): diagonal X_ii, then sqrt(2) Re X_ij and
sqrt(2) Im X_ij for i<j, ordered row by row over the upper triangle with
Re/Im interleaved; row i starts at offset i(2n-i); a block has n*n reals.

The paper's workloads are GYNI process matrices W (n = d^4) and instrument
Choi blocks (m = d^2) inside SCS iterates; neither its SDP instances nor its
iterates are available, so these seeded constructions stand in for them:

* ``gue(n, seed)``: X = (G + G^H)/2 with G iid circular CN(0,1) (Re, Im each
  N(0, 1/2)); about half the spectrum is negative.
* ``warm_sequence(n, seed, count)``: X_0 as above and
  X_{k+1} = X_k + 1e-3 (H_k + H_k^H)/2 -- slowly moving SCS-like iterates.
* ``constructed(n, seed, gap)``: X = U diag(lam) U^H, U Haar (QR of a CN(0,1)
  matrix with R's diagonal phases absorbed), floor(n/2) negative eigenvalues,
  magnitudes 10^(-log10(1/gap) t), t ~ U[0,1], each sign group's extreme
  magnitudes pinned to exactly gap and 1.
* ``cone(d, instance, seed)``: one SCS cone = W (d^4) + 8 Choi blocks (d^2).
* ``random_instrument`` / ``gyni_objective(d, seed)``: the objective
  G = 1/4 sum_{x,y} C^A_{a=y|x} (x) C^B_{b=x|y} of the GYNI game (two
  inputs and outputs per party, win iff a = y and b = x) for a pair of random
  feasible two-outcome instruments (random Kraus operators normalised to a
  trace-preserving sum) -- the paper's "randomly generated feasible pair of
  instruments" of its wall-clock table.
"""
from __future__ import annotations

import numpy as np

SQRT2 = np.sqrt(2.0)


def upper_pack(a: np.ndarray) -> np.ndarray:
    """Hermitian (n, n) complex -> svec (float64, n*n), reading the upper
    triangle.  Vectorised layout builder for inputs only."""
    n = a.shape[0]
    out = np.empty(n * n, dtype=np.float64)
    pos = 0
    for i in range(n):
        out[pos] = a[i, i].real
        row = a[i, i + 1:]
        seg = out[pos + 1: pos + 1 + 2 * row.size]
        seg[0::2] = SQRT2 * row.real
        seg[1::2] = SQRT2 * row.imag
        pos += 1 + 2 * row.size
    return out


def cn01(rng: np.random.Generator, shape) -> np.ndarray:
    """iid circular complex normal CN(0,1): Re, Im ~ N(0, 1/2)."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / SQRT2


def gue_matrix(n: int, rng: np.random.Generator) -> np.ndarray:
    g = cn01(rng, (n, n))
    return (g + g.conj().T) / 2.0


def gue(n: int, seed: int) -> np.ndarray:
    """svec of X = (G + G^H)/2, G iid CN(0,1)."""
    return upper_pack(gue_matrix(n, np.random.default_rng(seed)))


def warm_sequence(n: int, seed: int, count: int = 50, step: float = 1e-3):
    """List of `count` svec iterates X_0..X_{count-1} (one RNG stream)."""
    rng = np.random.default_rng(seed)
    x = gue_matrix(n, rng)
    out = [upper_pack(x)]
    for _ in range(count - 1):
        h = cn01(rng, (n, n))
        x = x + step * (h + h.conj().T) / 2.0
        out.append(upper_pack(x))
    return out


def haar_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    z = cn01(rng, (n, n))
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def constructed_spectrum(n: int, rng: np.random.Generator, gap: float = 1e-6) -> np.ndarray:
    nneg = n // 2
    npos = n - nneg
    decades = -np.log10(gap)

    def group(k):
        if k == 0:
            return np.empty(0)
        mag = 10.0 ** (-decades * rng.uniform(0.0, 1.0, size=k))
        if k >= 1:
            mag[np.argmin(mag)] = gap
        if k >= 2:
            mag[np.argmax(mag)] = 1.0
        return mag

    lam = np.concatenate([-group(nneg), group(npos)])
    return lam


def constructed(n: int, seed: int, gap: float = 1e-6):
    """(svec X, U, lam) with X = U diag(lam) U^H (spectrum in
    [-1,-gap] u [gap, 1])."""
    rng = np.random.default_rng(seed)
    u = haar_unitary(n, rng)
    lam = constructed_spectrum(n, rng, gap)
    x = (u * lam[None, :]) @ u.conj().T
    x = (x + x.conj().T) / 2.0
    return upper_pack(x), u, lam


def cotangent(n: int, seed: int) -> np.ndarray:
    """svec of a random Hermitian cotangent (K + K^H)/2."""
    return gue(n, seed)


CHOI_LABELS = ("A0|0", "A1|0", "A0|1", "A1|1", "B0|0", "B1|0", "B0|1", "B1|1")


def cone_sizes(d: int, instances: int = 32):
    """Block sizes of a batched cone: per instance W (d^4) then 8 Choi (d^2)."""
    return [d ** 4] + [d ** 2] * 8 if instances == 1 else ([d ** 4] + [d ** 2] * 8) * instances


def cone(d: int, instances: int = 32, seed_base: int = 4000):
    """Concatenated svec of `instances` x [W (d^4) + 8 Choi (d^2)], each block
    (G + G^H)/2; instance i uses seed seed_base + 100 d + i."""
    parts = []
    for i in range(instances):
        rng = np.random.default_rng(seed_base + 100 * d + i)
        parts.append(upper_pack(gue_matrix(d ** 4, rng)))
        for _ in range(8):
            parts.append(upper_pack(gue_matrix(d ** 2, rng)))
    return np.concatenate(parts), cone_sizes(d, instances)


def random_instrument(d: int, rng: np.random.Generator, outcomes: int = 2, kraus: int = 2):
    """Choi operators C_a (a < outcomes) on A_i (x) A_o (input factor first) of
    a random quantum instrument d -> d: random complex Gaussian Kraus
    operators K_{a,k}, normalised so that sum_{a,k} K^H K = 1 (trace
    preserving), C_a = sum_k |K_{a,k}>><<K_{a,k}| with |K>> = sum_i |i> (x) K|i>."""
    ks = [[cn01(rng, (d, d)) for _ in range(kraus)] for _ in range(outcomes)]
    s = sum(k.conj().T @ k for row in ks for k in row)
    w, v = np.linalg.eigh(s)
    inv_sqrt = (v * (1.0 / np.sqrt(w))) @ v.conj().T
    out = []
    for row in ks:
        c = np.zeros((d * d, d * d), dtype=np.complex128)
        for k in row:
            kk = k @ inv_sqrt
            vec = np.zeros(d * d, dtype=np.complex128)
            for i in range(d):
                vec[i * d:(i + 1) * d] = kk[:, i]     # |i> (x) K|i>
            c += np.outer(vec, vec.conj())
        out.append(c)
    return out


def gyni_objective(d: int, seed: int) -> np.ndarray:
    """G = 1/4 sum_{x,y} C^A_{a=y|x} (x) C^B_{b=x|y} of the GYNI game for a
    seeded random instrument pair (two inputs, two outcomes per party), on
    A_i (x) A_o (x) B_i (x) B_o; max tr[G W] over process matrices W is the
    winning probability with these instruments."""
    rng = np.random.default_rng(seed)
    ca = [random_instrument(d, rng) for _ in range(2)]   # ca[x][a]
    cb = [random_instrument(d, rng) for _ in range(2)]   # cb[y][b]
    g = np.zeros((d ** 4, d ** 4), dtype=np.complex128)
    for x in range(2):
        for y in range(2):
            g += np.kron(ca[x][y], cb[y][x])
    return g / 4.0
