"""Lockstep groups of the FP64 large-block path: the same-order blocks of one
batched call (the W blocks of a cone) go through every kernel launch of the
path together, one workspace slot per member.  A member computes exactly what
a single-block call computes, so every member is compared bitwise with the
single-block result, and against the oracle (1e-10 relative Frobenius)."""
import numpy as np
import pytest

import oracle
from paper_2606_20519_amd import workloads as W

import bars

pytestmark = pytest.mark.gpu
TOL = 1e-10


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2606_20519_amd as P
    return P


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def check_against_single(P, parts, sizes, oracle_every=1):
    y, infos = P.project_batched(dev(np.concatenate(parts)), sizes, info=True)
    y = y.cpu().numpy()
    off = 0
    for i, (m, s, inf) in enumerate(zip(sizes, parts, infos)):
        single, sinf = P.project(dev(s), m, info=True)
        got = y[off:off + m * m]
        assert np.array_equal(got, single.cpu().numpy()), (i, m)
        assert (inf["status"], inf["n_pos"], inf["n_neg"]) == (sinf["status"], sinf["n_pos"], sinf["n_neg"]), i
        assert inf["status"] == 0
        if i % oracle_every == 0:
            assert rel(got, oracle.project(s, m)) <= TOL, (i, m)
        off += m * m


def test_group_members_equal_single_blocks(P):
    # groups {100 x 3}, {70 x 2}, {130}; the order-20 block takes the LDS kernel
    sizes = [100, 70, 100, 130, 100, 70, 20]
    parts = [W.gue(m, 7000 + i) for i, m in enumerate(sizes)]
    check_against_single(P, parts, sizes)


def test_group_members_select_different_sides(P):
    # X and -X pick opposite sides (k+ <= k- vs k+ > k-) inside one group
    n = 96
    s, _, _ = W.constructed(n, 71, gap=1e-6)
    t = W.gue(n, 72)
    parts = [s, -s, t, -t]
    check_against_single(P, parts, [n] * 4)


def test_group_cap_splits_into_chunks(P):
    # 130 blocks of one order: a group of 128 and one of 2
    sizes = [65] * 130
    parts = [W.gue(65, 7100 + i) for i in range(130)]
    check_against_single(P, parts, sizes, oracle_every=13)


def test_cone_blocks_grouped(P):
    # a d = 3 cone: 4 instances x (W of order 81 + 8 Choi blocks of order 9)
    x, sizes = W.cone(3, 4)
    off, parts = 0, []
    for m in sizes:
        parts.append(x[off:off + m * m])
        off += m * m
    check_against_single(P, parts, sizes, oracle_every=9)


@pytest.mark.parametrize("mode,tol", [("mixed_fp32", 3e-6), ("mixed_bf16", None)])
def test_mixed_group_members_equal_single_blocks(P, mode, tol):
    # the Newton-Schulz form grouped the same way: bitwise equal to single
    # calls; error against the exact projection within the mixed bars
    sizes = [96, 96, 80, 96]
    parts = [W.constructed(m, 7200 + i, gap=1e-6)[0] for i, m in enumerate(sizes)]
    y, infos = P.project_batched(dev(np.concatenate(parts)), sizes, mode, info=True)
    y = y.cpu().numpy()
    off = 0
    for i, (m, s, inf) in enumerate(zip(sizes, parts, infos)):
        single, sinf = P.project(dev(s), m, mode, info=True)
        got = y[off:off + m * m]
        assert np.array_equal(got, single.cpu().numpy()), (i, m)
        assert inf == sinf, i
        assert inf["status"] == 0
        if tol is not None:
            assert rel(got, oracle.project(s, m)) <= tol, (i, m)
        off += m * m


def test_mixed_bf16_group_many_members(P):
    # 32 blocks of order 400 in BF16 in one group (the 64x64-tile product, as
    # for a single block of this order): against the closed form, and the
    # first members bitwise against single calls
    n, count = 400, 32
    cons = [W.constructed(n, 7300 + i, gap=1e-3) for i in range(count)]
    y, infos = P.project_batched(dev(np.concatenate([c[0] for c in cons])), [n] * count, "mixed_bf16", info=True)
    y = y.cpu().numpy()
    for i, ((s, u, lam), inf) in enumerate(zip(cons, infos)):
        exact = oracle.constructed_projection(u, lam)
        got = y[i * n * n:(i + 1) * n * n]
        err = np.linalg.norm(got - exact)
        bar = bars.mixed_bar_abs(lam, "mixed_bf16", np.linalg.norm(exact), inf["est_rel_err"])
        assert inf["status"] == 0, i
        assert err <= bar, (i, err, bar)
        if i < 2:
            assert np.array_equal(got, P.project(dev(s), n, "mixed_bf16").cpu().numpy()), i


@pytest.mark.parametrize("mode", ["mixed_bf16", "mixed_bf16x3"])
def test_mixed_bf16_group_large_orders(P, mode):
    # orders on the 128x128-tile product: two members of order 4000 (split
    # tail, ragged last tile row) and one of 2100, each bitwise equal to its
    # single-block call (the tile form depends on the order only)
    sizes = [4000, 2100, 4000]
    parts = [W.gue(m, 7400 + i) for i, m in enumerate(sizes)]
    y, infos = P.project_batched(dev(np.concatenate(parts)), sizes, mode, info=True)
    y = y.cpu().numpy()
    off = 0
    for i, (m, s, inf) in enumerate(zip(sizes, parts, infos)):
        single, sinf = P.project(dev(s), m, mode, info=True)
        assert np.array_equal(y[off:off + m * m], single.cpu().numpy()), (i, m)
        assert inf == sinf, i
        assert inf["status"] == 0
        off += m * m


def test_mixed_bf16x3_large_order_closed_form(P):
    # the split 128x128-tile product at order 2100 (ragged last tile row)
    # against the closed form, within the split form's band bar
    n = 2100
    s, u, lam = W.constructed(n, 7450, gap=1e-6)
    exact = oracle.constructed_projection(u, lam)
    y, inf = P.project(dev(s), n, "mixed_bf16x3", info=True)
    err = np.linalg.norm(y.cpu().numpy() - exact)
    nrm = np.linalg.norm(exact)
    print(f"bf16x3 n=2100: rel err {err / nrm:.3e} est {inf['est_rel_err']:.3e}", flush=True)
    assert inf["status"] == 0
    assert err <= bars.mixed_bar_abs(lam, "mixed_bf16x3", nrm, inf["est_rel_err"])
