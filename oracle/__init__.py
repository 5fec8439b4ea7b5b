"""CPU FP64 oracle for the PSD-cone projection -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  It shares no code with the GPU
library in ``paper_2606_20519_amd`` and never imports it.

Contents (each function cites the passage it follows):

* ``unpack`` / ``pack`` -- the paper's real encoding vec_R / mat_R of a
  Hermitian matrix (App. D.1): diagonal entries, then sqrt(2) Re X_ij and
  sqrt(2) Im X_ij for i<j.  Ordering (open in the paper): row-major over the
  upper triangle, Re/Im interleaved; row i starts at offset i(2n-i).
* ``eigh`` -- cyclic complex Jacobi eigendecomposition (C, ``psd_oracle.c``).
* ``project`` -- Pi(X) = V diag(max(lam,0)) V^H, the Euclidean projection onto
  the PSD cone (App. D.1, Pi_S), implemented as in App. D.2: eigendecompose,
  set the negative eigenvalues to zero.  Reconstruction in long double.
* ``vjp`` -- Daleckii-Krein derivative DPi(X)[G] = V (Gamma o V^H G V) V^H,
  which is what back-propagation through the projection needs (App. E).
* ``constructed_projection`` -- the closed form U diag(max(lam,0)) U^H for an
  input built as U diag(lam) U^H (matmul as a library step).
* ``constructed_vjp`` -- the closed form U (Gamma o U^H G U) U^H of the
  derivative for such an input (App. E; Daleckii-Krein divided differences).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "psd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile ``psd_oracle.c`` (or a variant source) into a shared library
    with gcc + OpenMP."""
    if force or not os.path.exists(out):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
               "-o", out + ".tmp", src, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return out


class OracleError(RuntimeError):
    pass


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _check(st: int, what: str):
    if st != 0:
        raise OracleError(f"{what} failed with status {st}")


class Oracle:
    """ctypes front end of one compiled oracle library."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_long)
        lib.or_unpack.argtypes = [ctypes.c_int, dp, dp]
        lib.or_pack.argtypes = [ctypes.c_int, dp, dp]
        lib.or_eigh_svec.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_int, ip, lp]
        lib.or_project.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ip, dp, dp]
        lib.or_reconstruct.argtypes = [ctypes.c_int, dp, dp, dp]
        lib.or_vjp.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int]
        lib.or_svec_row_offset.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.or_svec_row_offset.restype = ctypes.c_long
        lib.or_svec_offdiag_offset.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.or_svec_offdiag_offset.restype = ctypes.c_long
        lib.or_num_threads.restype = ctypes.c_int
        self.lib = lib
        self.path = path

    def row_offset(self, n: int, i: int) -> int:
        return int(self.lib.or_svec_row_offset(n, i))

    def offdiag_offset(self, n: int, i: int, j: int) -> int:
        return int(self.lib.or_svec_offdiag_offset(n, i, j))

    def unpack(self, s, n: int) -> np.ndarray:
        """mat_R: svec (n*n reals) -> Hermitian complex128 (n, n)."""
        s = _f64(s)
        assert s.size == n * n
        a = np.empty((n, n), dtype=np.complex128)
        _check(self.lib.or_unpack(n, _dp(s), _dp(a.view(np.float64))), "unpack")
        return a

    def pack(self, a) -> np.ndarray:
        """vec_R: Hermitian (n, n) -> svec (upper triangle read)."""
        a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
        n = a.shape[0]
        s = np.empty(n * n, dtype=np.float64)
        _check(self.lib.or_pack(n, _dp(a.view(np.float64)), _dp(s)), "pack")
        return s

    def eigh(self, s, n: int, mode: int = 1, max_sweeps: int = 0, return_stats: bool = False):
        """Jacobi eigendecomposition of mat_R(s).  Returns (lam, V) with lam
        ascending and V[:, k] the eigenvector of lam[k].

        mode 0: row-cyclic serial sweeps; mode 1: round-robin parallel sweeps.
        """
        s = _f64(s)
        lam = np.empty(n, dtype=np.float64)
        v = np.empty((n, n), dtype=np.complex128)
        sw = ctypes.c_int(0)
        rot = ctypes.c_long(0)
        st = self.lib.or_eigh_svec(n, _dp(s), _dp(lam), _dp(v.view(np.float64)), mode,
                                   max_sweeps, ctypes.byref(sw), ctypes.byref(rot))
        _check(st, "eigh")
        order = np.argsort(lam, kind="stable")
        lam, v = lam[order], v[:, order]
        if return_stats:
            return lam, v, {"sweeps": sw.value, "rotations": rot.value}
        return lam, v

    def project(self, s, n: int, mode: int = 1) -> np.ndarray:
        """svec(Pi(mat_R(s))): eigendecompose, clamp negative eigenvalues to
        0, reconstruct (App. D.2)."""
        s = _f64(s)
        y = np.empty(n * n, dtype=np.float64)
        sw = ctypes.c_int(0)
        _check(self.lib.or_project(n, _dp(s), _dp(y), mode, ctypes.byref(sw), None, None), "project")
        return y

    def reconstruct(self, lam, v) -> np.ndarray:
        """svec(V diag(max(lam,0)) V^H) with long-double accumulation."""
        lam = _f64(lam)
        v = np.ascontiguousarray(np.asarray(v, dtype=np.complex128))
        n = lam.size
        y = np.empty(n * n, dtype=np.float64)
        _check(self.lib.or_reconstruct(n, _dp(lam), _dp(v.view(np.float64)), _dp(y)), "reconstruct")
        return y

    def vjp(self, s, gy, n: int, mode: int = 1) -> np.ndarray:
        """svec(DPi(X)[mat_R(gy)]) by the Daleckii-Krein formula; equal to the
        vector-Jacobian product since DPi(X) is self-adjoint in svec space."""
        s, gy = _f64(s), _f64(gy)
        gx = np.empty(n * n, dtype=np.float64)
        _check(self.lib.or_vjp(n, _dp(s), _dp(gy), _dp(gx), mode), "vjp")
        return gx

    def constructed_projection(self, u, lam) -> np.ndarray:
        """Closed form for X = U diag(lam) U^H with U unitary:
        Pi(X) = U diag(max(lam,0)) U^H, returned as svec."""
        u = np.asarray(u, dtype=np.complex128)
        lp = np.maximum(np.asarray(lam, dtype=np.float64), 0.0)
        p = (u * lp[None, :]) @ u.conj().T
        return self.pack(p)

    def constructed_vjp(self, u, lam, gy) -> np.ndarray:
        """Closed form of the Daleckii-Krein derivative (App. E needs the
        derivative of Pi) for X = U diag(lam) U^H with U unitary:
        DPi(X)[G] = U (Gamma o (U^H G U)) U^H, G = mat_R(gy), with the divided
        differences of f(t) = max(t, 0),
            Gamma_ij = (f(lam_i) - f(lam_j)) / (lam_i - lam_j)  for opposite signs,
                       1 if both are > 0, 0 if both are <= 0,
        returned as svec (matmul as the library step)."""
        u = np.asarray(u, dtype=np.complex128)
        lam = np.asarray(lam, dtype=np.float64)
        n = lam.size
        g = self.unpack(gy, n)
        pos = lam > 0.0
        f = np.maximum(lam, 0.0)
        den = lam[:, None] - lam[None, :]
        mixed = pos[:, None] != pos[None, :]
        gam = np.where(pos[:, None] & pos[None, :], 1.0, 0.0)
        gam[mixed] = (f[:, None] - f[None, :])[mixed] / den[mixed]
        m = u.conj().T @ g @ u
        return self.pack(u @ (gam * m) @ u.conj().T)

    def num_threads(self) -> int:
        return int(self.lib.or_num_threads())


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _default = Oracle(_LIB)
    return _default


def svec_len(n: int) -> int:
    return n * n


def row_offset(n, i): return default().row_offset(n, i)
def offdiag_offset(n, i, j): return default().offdiag_offset(n, i, j)
def unpack(s, n): return default().unpack(s, n)
def pack(a): return default().pack(a)
def eigh(s, n, mode=1, max_sweeps=0, return_stats=False): return default().eigh(s, n, mode, max_sweeps, return_stats)
def project(s, n, mode=1): return default().project(s, n, mode)
def reconstruct(lam, v): return default().reconstruct(lam, v)
def vjp(s, gy, n, mode=1): return default().vjp(s, gy, n, mode)
def constructed_projection(u, lam): return default().constructed_projection(u, lam)
def constructed_vjp(u, lam, gy): return default().constructed_vjp(u, lam, gy)


def num_threads() -> int:
    return default().num_threads()


# ---------------------------------------------------------------------------
# Newton-Schulz reference for the mixed-precision form (attribution of error)
# ---------------------------------------------------------------------------
#
# The paper's outlook (Sec. V, "Approximate semidefinite-cone projections")
# proposes replacing the eigendecomposition by a matrix polynomial that
# approximates the eigenvalue threshold with matrix-matrix products only.
# The simplest such polynomial is the Newton-Schulz iteration for the matrix
# sign function, X_{k+1} = 1/2 X_k (3I - X_k^2), started from X_0 = X/alpha
# with alpha >= ||X||_2 (it converges to sign(X) for spectra inside
# (-sqrt3, sqrt3)); the projection then follows from Pi(X) = (X + X sign X)/2
# since max(t, 0) = (t + t sgn t)/2.  These functions are the plain FP64
# version of that recurrence (NumPy matmul as the only library step), used to
# attribute the GPU mixed form's error to truncation versus rounding.

def ns_schedule(l0: float = 1e-6, tol: float = 1e-7, iters: int = None, amax: float = 1.5) -> list:
    """Per-step scalings a_k of the scaled Newton-Schulz iteration
    X_{k+1} = (a_k / 2) X_k (3I - a_k^2 X_k^2) (Chen and Chow, 2014), with
    the scaling capped at `amax`.

    The first step is unscaled (a_0 = 1): it maps any spectrum inside
    (-sqrt 3, sqrt 3) into [-1, 1].  After it, with [l_k, 1] the bound on the
    eigenvalue magnitudes (l_1 = f(l0), f(t) = (3t - t^3)/2), the uncapped
    choice sqrt(3 / (1 + l_k + l_k^2)) gives f(a t) equal values at both ends
    of the interval; the cap keeps the top of the spectrum from being pushed
    far down (f(sqrt 3) = 0), which in low precision costs accuracy when those
    components grow back.  With a_k = min(amax, that value) the new bound is
    l_{k+1} = min(f(a_k l_k), f(a_k)).  Without `iters` the schedule stops
    once 1 - l_k <= tol; with it, exactly `iters` scalings are returned (a_k
    tends to 1 as l_k tends to 1)."""
    def f(t):
        return 0.5 * (3.0 * t - t ** 3)
    a = [1.0]
    lk = f(l0)
    while (len(a) < iters) if iters is not None else (1.0 - lk > tol):
        ak = min(amax, float(np.sqrt(3.0 / (1.0 + lk + lk * lk))))
        a.append(ak)
        lk = min(f(ak * lk), f(ak))
    return a[:iters] if iters is not None else a


def ns_scalar_map(t, iters: int, coeffs=None):
    """The scalar recurrence t <- 1.5 t - 0.5 t^3 applied `iters` times
    (elementwise, float64); with `coeffs` (a_k, k < iters) the scaled step
    t <- (3 a_k t - a_k^3 t^3) / 2."""
    t = np.asarray(t, dtype=np.float64).copy()
    for k in range(iters):
        a = 1.0 if coeffs is None else coeffs[k]
        t = 0.5 * (3.0 * a * t - (a * t) ** 3)
    return t


def ns_constructed_projection(u, lam, alpha: float, iters: int, coeffs=None) -> np.ndarray:
    """Exact-arithmetic Newton-Schulz projection of X = U diag(lam) U^H after
    `iters` steps: U diag((lam + lam p(lam/alpha))/2) U^H as svec, where p is
    the iterated scalar map.  Only per-eigenvalue arithmetic."""
    lam = np.asarray(lam, dtype=np.float64)
    s = ns_scalar_map(lam / alpha, iters, coeffs)
    f = 0.5 * (lam + lam * s)
    u = np.asarray(u, dtype=np.complex128)
    return default().pack((u * f[None, :]) @ u.conj().T)


def ns_matrix_projection(x_svec, n: int, alpha: float, iters: int, coeffs=None) -> np.ndarray:
    """FP64 Newton-Schulz projection by matrix products: X_0 = X/alpha,
    X_{k+1} = (a_k/2) X_k (3I - a_k^2 X_k^2) for `iters` steps (a_k = 1
    without `coeffs`), then (X + X X_K)/2, whose Hermitian part is returned
    as svec."""
    x = default().unpack(x_svec, n)
    xk = x / alpha
    eye = np.eye(n)
    for k in range(iters):
        a = 1.0 if coeffs is None else coeffs[k]
        xk = (0.5 * a) * xk @ (3.0 * eye - (a * a) * (xk @ xk))
    p = 0.5 * (x + x @ xk)
    return default().pack(0.5 * (p + p.conj().T))


def spectral_norm(x_svec, n: int) -> float:
    """||mat(x)||_2 from LAPACK eigenvalues (library routine)."""
    w = np.linalg.eigvalsh(default().unpack(x_svec, n))
    return float(np.abs(w).max()) if n else 0.0
