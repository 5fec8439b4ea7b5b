"""Batched SCS cones by one plan launch at d = 5..8: per instance one W block
(n = d^4) and 8 instrument Choi blocks (m = d^2), 32 instances.

The W blocks of instances 0 and 31 are replaced by constructed spectra
X = U diag(lambda) U^H (U Haar, |lambda| log-uniform in [1e-3, 1], half
negative) and checked element by element against the closed form
U diag(max(lambda, 0)) U^H; every Choi block is checked against the oracle
(blocks of order <= 64 take the exact LDS kernel in every mode); the Moreau
identity Pi(X) - Pi(-X) = X is checked on every block.  FP64 at 1e-10;
FP32-mixed within tests/bars.py's bars; BF16-mixed (d = 5) within its band
plus first-order bar, using the per-block error estimate of the info records.
"""
import numpy as np
import pytest

import oracle
from paper_2606_20519_amd import workloads as W

import bars

pytestmark = pytest.mark.gpu
TOL = 1e-10
CHECKED = (0, 31)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2606_20519_amd as P
    P.set_ns_iterations(0, 1)
    return P


_cones = {}


def cone_with_constructed(d):
    """(svec of the cone, sizes, {instance: (u, lam)}) -- cached per d."""
    if d not in _cones:
        print(f"building the d={d} cone", flush=True)
        x, sizes = W.cone(d, 32)
        n = d ** 4
        per = n * n + 8 * d ** 4
        known = {}
        for inst in CHECKED:
            s, u, lam = W.constructed(n, 5000 + 100 * d + inst, gap=1e-3)
            x[inst * per: inst * per + n * n] = s
            known[inst] = (u, lam)
        _cones.clear()
        _cones[d] = (x, sizes, known)
    return _cones[d]


def run_cone(P, d, mode):
    import torch
    x_np, sizes, known = cone_with_constructed(d)
    nb = len(sizes)
    x = torch.from_numpy(x_np).to("cuda:0")
    plan = P.Plan(sizes, mode)
    infos = torch.zeros(P.INFO_WORDS * nb, dtype=torch.int32, device="cuda:0")
    y = plan.execute(x, infos=infos)
    ym = plan.execute(-x)
    torch.cuda.synchronize()
    recs = P.info_records(infos, nb)
    y, ym = y.cpu().numpy(), ym.cpu().numpy()
    plan.close()
    del x
    torch.cuda.empty_cache()
    off = 0
    worst = {"closed": 0.0, "choi": 0.0, "moreau": 0.0}
    for b, m in enumerate(sizes):
        blk = slice(off, off + m * m)
        inst = b // 9
        assert recs[b]["status"] == 0, b
        mo = rel(y[blk] - ym[blk], x_np[blk])
        worst["moreau"] = max(worst["moreau"], mo)
        if m <= 64:
            e = rel(y[blk], oracle.project(x_np[blk], m))
            worst["choi"] = max(worst["choi"], e)
            assert e <= TOL, b
            assert mo <= TOL, b
        elif mode == "fp64":
            assert mo <= TOL, b
        elif mode == "mixed_fp32":
            # each side within the FP32 bar of its projection (||Pi|| <= ||X||)
            assert mo <= 2.0 * bars.FP32_REL_BAR, b
        else:
            # each side within band + 2 est ||Pi|| (the same estimate for both)
            lam_b = np.linalg.eigvalsh(oracle.unpack(x_np[blk], m))
            est = recs[b]["est_rel_err"]
            bar = 2.0 * (bars.band_norm(lam_b, mode) + 2.0 * est * np.linalg.norm(y[blk]))
            assert mo * np.linalg.norm(x_np[blk]) <= bar, (b, mo, est)
        if m > 64 and inst in known:
            u, lam = known[inst]
            exact = oracle.constructed_projection(u, lam)
            e = rel(y[blk], exact)
            worst["closed"] = max(worst["closed"], e)
            if mode == "fp64":
                assert e <= TOL, b
            else:
                nrm = np.linalg.norm(exact)
                est = recs[b]["est_rel_err"]
                assert e * nrm <= bars.mixed_bar_abs(lam, mode, nrm, est), (b, e, est)
                if mode == "mixed_fp32":
                    assert e <= bars.FP32_REL_BAR, b
        off += m * m
    print(f"d={d} {mode}: worst closed-form {worst['closed']:.2e}, Choi {worst['choi']:.2e}, "
          f"Moreau {worst['moreau']:.2e}", flush=True)


@pytest.mark.parametrize("d,mode", [(6, "fp64"), (6, "mixed_fp32"), (7, "fp64"), (7, "mixed_fp32"),
                                    (8, "fp64"), (8, "mixed_fp32")])
def test_cone_plan(P, d, mode):
    run_cone(P, d, mode)


def test_cone_d5_bf16(P):
    run_cone(P, 5, "mixed_bf16")
