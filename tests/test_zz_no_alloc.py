"""psd_project_noalloc (the entry point for callers that cannot allocate)
against psd_project, through the C ABI: two calls in a row on the shared
device scratch, the second with a smaller order, in FP64 (bitwise equal to
psd_project with a caller workspace, and within 1e-10 of the oracle) and in
the mixed modes (bitwise equal as well: the same kernels on the same data);
orders beyond the scratch are rejected before anything runs."""
import numpy as np
import pytest

import oracle
from paper_2606_20519_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("mode,sizes", [("fp64", (700, 300)), ("mixed_bf16", (600, 130)),
                                        ("mixed_fp32", (640, 90))])
def test_noalloc_matches_workspace_entry_point(P, mode, sizes):
    import torch
    for n in sizes:
        s = W.gue(n, 9400 + n)
        x = dev(s)
        print(f"noalloc {mode} n={n}", flush=True)
        y0, i0 = P.project_noalloc(x, n, mode, info=True)
        y1, i1 = P.project(x, n, mode, info=True)
        torch.cuda.synchronize()
        a, b = y0.cpu().numpy(), y1.cpu().numpy()
        assert i0["status"] == 0 and i1["status"] == 0
        assert np.array_equal(a, b), (mode, n)
        assert i0 == i1
        if mode == "fp64":
            assert rel(a, oracle.project(s, n)) <= 1e-10


def test_noalloc_in_place_and_small(P):
    n = 500
    s = W.gue(n, 9500)
    x = dev(s)
    P.project_noalloc(x, n, out=x)
    assert rel(x.cpu().numpy(), oracle.project(s, n)) <= 1e-10
    m = 40
    s = W.gue(m, 9501)
    assert rel(P.project_noalloc(dev(s), m).cpu().numpy(), oracle.project(s, m)) <= 1e-10


def test_noalloc_rejects_orders_beyond_scratch(P):
    from paper_2606_20519_amd import PsdError
    for mode, n in (("fp64", 832), ("mixed_bf16", 769), ("mixed_fp32", 705)):
        x = dev(np.zeros(n * n))
        with pytest.raises(PsdError) as ei:
            P.project_noalloc(x, n, mode)
        assert ei.value.status == 2   # PSD_EWORKSPACE
