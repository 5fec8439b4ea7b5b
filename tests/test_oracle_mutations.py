"""Planted mistakes in the oracle must be caught by its pins.

Each case copies ``oracle/psd_oracle.c``, plants one plausible mistake (a
dropped term, a wrong sign or index, a transposed operand), compiles the copy
on the CPU and runs a compact battery of the pins from test_oracle_pins.py
against it.  The battery must fail for every mutant.
"""
import os
import tempfile

import numpy as np
import pytest

import oracle
from paper_2606_20519_amd import workloads as W

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "psd_oracle.c")

MUTANTS = {
    "rotation_diag_sign": ("aqq + g->t * g->r", "aqq - g->t * g->r"),
    "phase_not_conjugated": ("g->ph = conj(apq) / r", "g->ph = apq / r"),
    "row_rotation_phase": ("hqp = -g->s * conj(g->ph)", "hqp = -g->s * g->ph"),
    "tau_sign": ("double tau = (aqq - app)", "double tau = (app - aqq)"),
    "unpack_lower_not_conjugate": ("a[(long)j * n + i] = re - im * I", "a[(long)j * n + i] = re + im * I"),
    "pack_dropped_sqrt2": ("s[o + 1] = M_SQRT2 * cimag", "s[o + 1] = cimag"),
    "unpack_dropped_sqrt2": ("im = s[o + 1] / M_SQRT2", "im = s[o + 1]"),
    "no_clamp": ("if (!(lam[k] > 0.0)) continue;", "if (lam[k] != lam[k]) continue;"),
    "clamp_wrong_side": ("if (!(lam[k] > 0.0)) continue;", "if (lam[k] > 0.0) continue;"),
    "reconstruct_im_sign": ("im += (long double)lam[k] * (ai * br - ar * bi)",
                            "im += (long double)lam[k] * (ai * br + ar * bi)"),
    "gamma_numerator": ("return pa ? a / (a - b)", "return pa ? b / (a - b)"),
    "gamma_both_negative": ("if (!pa && !pb) return 0.0;", "if (!pa && !pb) return 1.0;"),
    "vjp_transposed_operand": ("conj(v[(long)k * n + i]) * t[(long)k * n + j]",
                               "conj(v[(long)i * n + k]) * t[(long)k * n + j]"),
    "vjp_missing_conj": ("m[(long)i * n + k] * conj(v[(long)j * n + k])",
                         "m[(long)i * n + k] * v[(long)j * n + k]"),
    "rotation_v_skipped": ("or_rot_cols(a, n, &g[k], 0, n); or_rot_cols(v, n, &g[k], 0, n);",
                           "or_rot_cols(a, n, &g[k], 0, n);"),
}


def battery(o: oracle.Oracle):
    """Raises AssertionError (or OracleError) if any pin fails."""
    eps = np.finfo(float).eps
    # golden 2x2 (projection_2x2.txt, case 2) and vec_R of a known matrix
    y = o.project(np.array([0.0, 0.0, np.sqrt(2.0), 0.0]), 2)
    assert np.allclose(y, [0.5, 0.0, np.sqrt(0.5), 0.5], atol=1e-14)
    x2 = np.array([[1, 2 + 3j], [2 - 3j, 4]])
    assert np.allclose(o.pack(x2), [1, 2 * np.sqrt(2), 3 * np.sqrt(2), 4], atol=1e-14)
    assert np.allclose(o.unpack(o.pack(x2), 2), x2, atol=1e-14)
    for mode in (0, 1):
        n = 10
        s = W.gue(n, 31)
        x = W.gue_matrix(n, np.random.default_rng(31))
        assert np.allclose(W.upper_pack(x), s)
        w, u = np.linalg.eigh(x)
        ref = W.upper_pack((u * np.maximum(w, 0)) @ u.conj().T)
        got = o.project(s, n, mode)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
        lam, v = o.eigh(s, n, mode)
        assert np.linalg.norm(x @ v - v * lam) <= 1e-12 * np.linalg.norm(x)
    # DK derivative: central differences and the diagonal (Hadamard) case
    n = 5
    s = W.gue(n, 32)
    e = W.gue(n, 33)
    h = 1e-6
    fd = (o.project(s + h * e, n) - o.project(s - h * e, n)) / (2 * h)
    assert np.linalg.norm(o.vjp(s, e, n) - fd) <= 1e-7 * np.linalg.norm(fd)
    d = np.array([2.0, -1.0, 0.5, -3.0, 4.0])
    gd = o.vjp(o.pack(np.diag(d).astype(complex)), e, n)
    ed = o.unpack(e, n)
    gam = np.array([[1.0 if a > 0 and b > 0 else 0.0 if a <= 0 and b <= 0 else max(a, b) / (max(a, b) - min(a, b))
                     for b in d] for a in d])
    assert np.allclose(gd, W.upper_pack(gam * ed), atol=8 * eps * np.abs(ed).max() * 4)


def test_battery_passes_on_the_real_oracle(orc):
    battery(orc)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    with tempfile.TemporaryDirectory() as td:
        path_c = os.path.join(td, f"mut_{name}.c")
        with open(path_c, "w") as f:
            f.write(src.replace(old, new, 1))
        lib = oracle.build(force=True, src=path_c, out=os.path.join(td, f"libmut_{name}.so"))
        mut = oracle.Oracle(lib)
        with pytest.raises((AssertionError, oracle.OracleError)):
            battery(mut)
