"""GPU parity of the SCS affine step for bipartite process matrices
(psd_constraint_apply / psd_constraint_adjoint / psd_affine_step) against the
oracle (oracle/affine.py):

* d = 2, 3: element by element against the oracle's explicit Kronecker
  construction of A x = -sum x_mu F_mu, A^T Z = -tr[F_mu Z] and
  z = ((a_x - A^T a_y)/2, a_y + A z_x);
* d = 4 .. 8 (d = 8: y of order 4096): A^T A x = x, A A^T y against the
  oracle's trace-and-replace projector P_proc(y) - tr(y)/d_tot 1 element by
  element, and the residual of the affine system [[1, A^T], [-A, 1]] z = a;
* in place (zx = ax, zy = ay) equal to out of place, bit for bit.
FP64 throughout: bars 1e-12 relative (a handful of roundings per entry)."""
import numpy as np
import pytest

import oracle
from oracle import affine as AF

pytestmark = pytest.mark.gpu
TOL = 1e-12


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2606_20519_amd as P
    return P


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def rand_herm(n, rng):
    g = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2)
    return (g + g.conj().T) / 2


@pytest.mark.parametrize("d", [2, 3])
def test_affine_against_explicit_oracle(P, d):
    rng = np.random.default_rng(40 + d)
    nx, ny = P.affine_dims(d)
    assert nx == AF.count_allowed(d) and ny == d ** 8
    x = rng.standard_normal(nx)
    y = rand_herm(d ** 4, rng)
    ys = oracle.pack(y)
    ga = P.constraint_apply(dev(x), d).cpu().numpy()
    assert rel(ga, oracle.pack(AF.constraint_apply(x, d))) <= TOL
    gt = P.constraint_adjoint(dev(ys), d).cpu().numpy()
    assert rel(gt, AF.constraint_adjoint(y, d)) <= TOL
    ax = rng.standard_normal(nx)
    zx, zy = P.affine_step(dev(ax), dev(ys), d)
    rx, ry = AF.affine_step(ax, y, d)
    assert rel(zx.cpu().numpy(), rx) <= TOL
    assert rel(zy.cpu().numpy(), oracle.pack(ry)) <= TOL
    print(f"d={d}: A, A^T and the affine step match the explicit construction", flush=True)


@pytest.mark.parametrize("d", [4, 5, 6, 7, 8])
def test_affine_identities_full_size(P, d):
    import torch
    rng = np.random.default_rng(50 + d)
    nx, ny = P.affine_dims(d)
    n = d ** 4
    x = dev(rng.standard_normal(nx))
    # A^T A = I
    back = P.constraint_adjoint(P.constraint_apply(x, d), d)
    e1 = float(torch.linalg.vector_norm(back - x) / torch.linalg.vector_norm(x))
    # A A^T y = P_proc(y) - tr(y)/d_tot 1, P_proc from partial traces
    y = rand_herm(n, rng)
    ys = oracle.pack(y)
    got = P.constraint_apply(P.constraint_adjoint(dev(ys), d), d).cpu().numpy()
    ref = oracle.pack(AF.p_proc(y, d) - np.trace(y) / n * np.eye(n))
    e2 = rel(got, ref)
    # the affine system [[1, A^T], [-A, 1]] z = a, and in place == out of place
    ax = dev(rng.standard_normal(nx))
    ay = dev(ys)
    zx, zy = P.affine_step(ax, ay, d)
    r1 = zx + P.constraint_adjoint(zy, d) - ax
    r2 = zy - P.constraint_apply(zx, d) - ay
    e3 = float(torch.linalg.vector_norm(r1) / torch.linalg.vector_norm(ax))
    e4 = float(torch.linalg.vector_norm(r2) / torch.linalg.vector_norm(ay))
    ix, iy = ax.clone(), ay.clone()
    P.affine_step(ix, iy, d, zx=ix, zy=iy)
    torch.cuda.synchronize()
    print(f"d={d}: A^T A {e1:.1e}, A A^T vs P_proc {e2:.1e}, system residuals {e3:.1e} {e4:.1e}", flush=True)
    assert e1 <= TOL and e2 <= TOL and e3 <= TOL and e4 <= TOL
    assert torch.equal(ix, zx) and torch.equal(iy, zy)
