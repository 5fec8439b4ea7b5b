"""Planted mistakes in the affine-step oracle must be caught by its pins.

Each case copies ``oracle/affine.py``, plants one plausible mistake (a wrong
normalisation, sign, transposition or selection rule), loads the copy as a
fresh module and runs a compact battery of the pins of
test_oracle_affine.py: the orthonormal Hermitian basis and the Pauli
matrices at d = 2, the paper's index count, A^T A = I and
A A^T = P_proc - tr/d_tot with P_proc from partial traces, P_proc a
projector fixing the trivial process, and the affine system.  The battery
must fail for every mutant (and pass for the unmodified source).
"""
import os
import types

import numpy as np
import pytest

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "affine.py")

MUTANTS = {
    "diagonal_normalisation": ("np.sqrt(1.0 / ((l + 1) * (l + 2)))", "np.sqrt(1.0 / (l + 1))"),
    "antisymmetric_sign": ("m[j, k] = -1j / np.sqrt(2.0)", "m[j, k] = 1j / np.sqrt(2.0)"),
    "forbidden_rule": ("if has_t and not has_e:", "if has_t and has_e:"),
    "identity_kept": ("continue              # the identity", "pass                  # the identity"),
    "apply_sign": ("y -= xm * basis_element(sig, mu)", "y += xm * basis_element(sig, mu)"),
    "adjoint_not_transposed": ("basis_element(sig, mu).T * z", "basis_element(sig, mu) * z"),
    "affine_half_dropped": ("zx = 0.5 * (np.asarray", "zx = (np.asarray"),
    "p_proc_term_sign": ("- tr(AI, AO) - tr(BI, BO)", "+ tr(AI, AO) - tr(BI, BO)"),
    "trace_replace_unnormalised": ("t = tr * eye / d", "t = tr * eye"),
}


def load(text: str):
    mod = types.ModuleType("affine_mutant")
    exec(compile(text, "affine_mutant.py", "exec"), mod.__dict__)
    return mod


def herm(n, rng):
    g = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2)
    return (g + g.conj().T) / 2


def battery(M):
    for d in (2, 3):
        sig = M.gellmann(d)
        gram = np.array([[np.trace(a.conj().T @ b) for b in sig] for a in sig])
        assert np.allclose(gram, np.eye(d * d), atol=1e-14)
        assert all(np.allclose(s, s.conj().T) for s in sig)
    s = 1 / np.sqrt(2)
    pauli = [np.eye(2), np.diag([1, -1]), np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]])]
    assert all(np.allclose(g, s * p, atol=1e-15) for g, p in zip(M.gellmann(2), pauli))
    d = 2
    D = d * d
    assert len(M.allowed_indices(d)) == (D - 1) * (2 * D * D - D + 1) == 87
    rng = np.random.default_rng(12)
    x = rng.standard_normal(87)
    assert np.allclose(M.constraint_adjoint(M.constraint_apply(x, d), d), x, atol=1e-12)
    y = herm(16, rng)
    lhs = M.constraint_apply(M.constraint_adjoint(y, d), d)
    assert np.allclose(lhs, M.p_proc(y, d) - np.trace(y) / 16 * np.eye(16), atol=1e-12)
    p = M.p_proc(herm(16, rng), d)
    assert np.allclose(M.p_proc(p, d), p, atol=1e-12)
    w = np.eye(16) / 4
    assert np.allclose(M.p_proc(w, d), w, atol=1e-14)
    ax, ay = rng.standard_normal(87), herm(16, rng)
    zx, zy = M.affine_step(ax, ay, d)
    assert np.allclose(zx + M.constraint_adjoint(zy, d), ax, atol=1e-12)
    assert np.allclose(-M.constraint_apply(zx, d) + zy, ay, atol=1e-12)


def test_unmodified_source_passes():
    battery(load(open(SRC).read()))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, name
    with pytest.raises(Exception):
        battery(load(text.replace(old, new)))
