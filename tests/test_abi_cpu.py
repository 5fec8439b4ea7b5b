"""Host-side checks of the C ABI: the library loads, exports every symbol
include/psdproj.h declares, and rejects bad arguments before touching the
device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2606_20519_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2606_20519_amd import build
        build.build()
    return _lib


def header_functions():
    src = open(os.path.join(ROOT, "include", "psdproj.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(psd_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    names = header_functions()
    assert set(names) == set(L.EXPORTS), names
    lib = L.lib()
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(L):
    lib = L.lib()
    for st in range(8):
        assert lib.psd_status_string(st)
    assert lib.psd_version().startswith(b"psdproj")


def test_workspace_size_validation(L):
    lib = L.lib()
    out = ctypes.c_size_t(0)
    n = L.int_array([16])
    assert lib.psd_workspace_size(1, n, 0, 0, ctypes.byref(out)) == 0 and out.value > 0
    assert lib.psd_workspace_size(0, n, 0, 0, ctypes.byref(out)) == 1
    assert lib.psd_workspace_size(1, L.int_array([0]), 0, 0, ctypes.byref(out)) == 1
    assert lib.psd_workspace_size(1, n, 9, 0, ctypes.byref(out)) == 1
    assert lib.psd_workspace_size(1, None, 0, 0, ctypes.byref(out)) == 1
    # monotone in n for the large path
    sizes = []
    for k in (65, 100, 625, 1296):
        assert lib.psd_workspace_size(1, L.int_array([k]), 0, 0, ctypes.byref(out)) == 0
        sizes.append(out.value)
    assert sizes == sorted(sizes)


def test_workspace_size_lockstep_groups(L):
    """Batched calls run same-order blocks in lockstep groups of at most 128,
    one workspace slot per member, in every mode."""
    lib = L.lib()
    out = ctypes.c_size_t(0)
    for mode in (0, 1, 2, 3):
        assert lib.psd_workspace_size(1, L.int_array([256]), mode, 0, ctypes.byref(out)) == 0
        one = out.value
        assert lib.psd_workspace_size(32, L.int_array([256] * 32), mode, 0, ctypes.byref(out)) == 0
        assert out.value > 16 * one
        assert lib.psd_workspace_size(128, L.int_array([256] * 128), mode, 0, ctypes.byref(out)) == 0
        assert out.value > 64 * one
        g128 = out.value
        assert lib.psd_workspace_size(140, L.int_array([256] * 140), mode, 0, ctypes.byref(out)) == 0
        assert out.value < g128 + 4096  # groups of at most 128 share the slots


def test_saved_size(L):
    assert L.saved_size(1) == 8 * (1 + 2)
    assert L.saved_size(16) == 8 * (16 + 2 * 256)
    assert L.saved_size(0) == 0


def test_project_rejects_bad_arguments_on_host(L):
    lib = L.lib()
    fake = ctypes.c_void_p(0x10000)   # never dereferenced: validation fails first
    fake2 = ctypes.c_void_p(0x10000 + 8 * 256)
    ws = ctypes.c_void_p(0x100000)
    # n < 1, null pointers, bad mode
    assert lib.psd_project(0, fake, fake2, 0, ws, 1 << 20, None, None, None) == 1
    assert lib.psd_project(16, None, fake2, 0, ws, 1 << 20, None, None, None) == 1
    assert lib.psd_project(16, fake, None, 0, ws, 1 << 20, None, None, None) == 1
    assert lib.psd_project(16, fake, fake2, 5, ws, 1 << 20, None, None, None) == 1
    # misaligned pointer
    assert lib.psd_project(16, ctypes.c_void_p(0x10004), fake2, 0, ws, 1 << 20, None, None, None) == 1
    # partial overlap of x and y
    assert lib.psd_project(16, fake, ctypes.c_void_p(0x10000 + 8), 0, ws, 1 << 20, None, None, None) == 1
    # workspace too small
    assert lib.psd_project(16, fake, fake2, 0, ws, 0, None, None, None) == 2
    # batched: bad sizes
    assert lib.psd_project_batched(2, L.int_array([4, 0]), fake, fake2, 0, ws, 1 << 20, None, None) == 1
    assert lib.psd_project_batched(0, L.int_array([4]), fake, fake2, 0, ws, 1 << 20, None, None) == 1
    # vjp: needs x or saved
    assert lib.psd_project_vjp(16, None, None, fake, fake2, 0, ws, 1 << 20, None) == 1
    assert lib.psd_project_vjp(0, fake, None, fake, fake2, 0, ws, 1 << 20, None) == 1


def test_setters_validate_on_host(L):
    lib = L.lib()
    assert lib.psd_set_mixed_fallback(-1.0) == 1
    assert lib.psd_set_mixed_fallback(float("nan")) == 1
    assert lib.psd_set_mixed_fallback(1e-3) == 0
    assert lib.psd_set_mixed_fallback(0.0) == 0
    assert lib.psd_set_ns_iterations(-1, 1) == 1
    assert lib.psd_set_ns_iterations(0, 9) == 1
    assert lib.psd_set_ns_iterations(0, 1) == 0
    assert lib.psd_set_ns_iterations(0, -2) == 1
    assert lib.psd_set_ns_iterations(0, -1) == 0      # automatic corrections


def test_affine_host_validation(L):
    lib = L.lib()
    nx, ny = ctypes.c_int64(0), ctypes.c_int64(0)
    for d in range(2, 9):
        assert lib.psd_affine_dims(d, ctypes.byref(nx), ctypes.byref(ny)) == 0
        D = d * d
        assert nx.value == d ** 8 - (1 + D * (D - 1)) ** 2 and ny.value == d ** 8
    # Table II's m column: the number of free parameters x of the process matrix
    table2_m = {2: 87, 3: 1232, 4: 7455, 5: 29424, 6: 89495, 7: 228192, 8: 512127}
    for d, m in table2_m.items():
        assert lib.psd_affine_dims(d, ctypes.byref(nx), ctypes.byref(ny)) == 0 and nx.value == m, d
    assert lib.psd_affine_dims(1, ctypes.byref(nx), ctypes.byref(ny)) == 1
    assert lib.psd_affine_dims(9, ctypes.byref(nx), ctypes.byref(ny)) == 1
    out = ctypes.c_size_t(0)
    assert lib.psd_affine_workspace_size(8, ctypes.byref(out)) == 0 and out.value == 2 * 16 * 8 ** 8
    fake = ctypes.c_void_p(0x10000)
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40
    # workspace too small, bad d, misaligned workspace, overlapping outputs
    assert lib.psd_constraint_apply(2, fake, fake, ws, 0, None) == 2
    assert lib.psd_constraint_apply(9, fake, fake, ws, big, None) == 1
    assert lib.psd_constraint_adjoint(2, fake, fake, ctypes.c_void_p(0x100008), big, None) == 1
    ax, ay = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000)
    assert lib.psd_affine_step(2, ax, ay, ctypes.c_void_p(0x20008), ctypes.c_void_p(0x40000), ws, big, None) == 1


def test_scs_settings_validation():
    import ctypes
    from paper_2606_20519_amd import _lib
    L = _lib.lib()

    def st(**kw):
        base = dict(d=4, max_iters=10, check_every=1, mixed_iters=0, mixed_mode=2, normalize=1, warm_start=0,
                    anderson=0, eps=1e-5, alpha=1.5, mixed_switch=0.0)
        base.update(kw)
        return _lib.ScsSettings(**base)

    out = ctypes.c_size_t(0)
    assert L.psd_scs_workspace_size(ctypes.byref(st()), ctypes.byref(out)) == 0 and out.value > 0
    plain = out.value
    assert L.psd_scs_workspace_size(ctypes.byref(st(anderson=10)), ctypes.byref(out)) == 0
    nx, ny = _lib.affine_dims(4)
    assert out.value >= plain + 24 * 8 * (nx + ny + 1)       # 2m + 4 vectors of the cone input
    one = ctypes.c_size_t(0)
    assert L.psd_scs_workspace_size_batched(ctypes.byref(st()), 1, ctypes.byref(one)) == 0 and one.value == plain
    assert L.psd_scs_workspace_size_batched(ctypes.byref(st()), 8, ctypes.byref(out)) == 0
    assert out.value > plain + 7 * 8 * (2 * ny)               # every instance's cone-step blocks
    assert L.psd_scs_workspace_size_batched(ctypes.byref(st()), 0, ctypes.byref(out)) == 1
    assert L.psd_scs_workspace_size_batched(ctypes.byref(st()), 65535, ctypes.byref(out)) == 0  # the bound
    assert L.psd_scs_workspace_size_batched(ctypes.byref(st()), 65536, ctypes.byref(out)) == 1  # beyond it
    assert ctypes.sizeof(_lib.ScsSettings) == 64 and ctypes.sizeof(_lib.ScsInfo) == 112
    assert L.psd_scs_workspace_size_batched(ctypes.byref(st(warm_proj=1)), 1, ctypes.byref(out)) == 0
    assert out.value >= plain + _lib.saved_size(256)        # the warm cone steps' eigen-pair
    assert L.psd_scs_workspace_size_batched(ctypes.byref(st(warm_proj=1)), 2, ctypes.byref(out)) == 1
    for bad in (dict(warm_proj=2), dict(warm_proj=-1), dict(d=1), dict(d=9), dict(max_iters=0), dict(check_every=0), dict(alpha=2.0), dict(alpha=0.0),
                dict(eps=-1.0), dict(eps=float("nan")), dict(mixed_iters=5, mixed_mode=0), dict(anderson=17),
                dict(anderson=-1), dict(mixed_switch=-1.0), dict(mixed_switch=float("inf")),
                dict(normalize=2), dict(mixed_iters=-1)):
        assert L.psd_scs_workspace_size(ctypes.byref(st(**bad)), ctypes.byref(out)) == 1, bad
    info = _lib.ScsInfo()
    # host-side rejections enqueue nothing
    assert L.psd_scs_solve(ctypes.byref(st(d=9)), None, None, None, None, None, None, 0, None,
                           ctypes.byref(info)) == 1
    assert L.psd_scs_solve(ctypes.byref(st()), ctypes.c_void_p(256), ctypes.c_void_p(1 << 40),
                           ctypes.c_void_p(2 << 40), ctypes.c_void_p(3 << 40), None, ctypes.c_void_p(4 << 40),
                           16, None, ctypes.byref(info)) == 2          # workspace too small


def test_warm_rejects_bad_arguments_on_host(L):
    lib = L.lib()
    x = ctypes.c_void_p(0x10000)
    y = ctypes.c_void_p(0x10000 + 8 * 256)
    sp, so = ctypes.c_void_p(0x200000), ctypes.c_void_p(0x400000)
    ws = ctypes.c_void_p(0x1000000)
    big = 1 << 34
    assert lib.psd_project_warm(0, x, y, sp, so, ws, big, None, None) == 1
    assert lib.psd_project_warm(16, x, y, None, so, ws, big, None, None) == 1
    assert lib.psd_project_warm(16, x, y, sp, None, ws, big, None, None) == 1
    assert lib.psd_project_warm(16, x, y, sp, ctypes.c_void_p(0x200000 + 8), ws, big, None, None) == 1
    assert lib.psd_project_warm(16, x, ctypes.c_void_p(0x200000), sp, so, ws, big, None, None) == 1
    assert lib.psd_project_warm(16, x, y, ctypes.c_void_p(0x200004), so, ws, big, None, None) == 1
    assert lib.psd_project_warm(16, x, y, sp, so, ws, 0, None, None) == 2      # workspace too small
    out = ctypes.c_size_t(0)
    assert lib.psd_workspace_size(1, L.int_array([100]), 0, L.PSD_FLAG_WARM, ctypes.byref(out)) == 0
    warm = out.value
    assert lib.psd_workspace_size(1, L.int_array([100]), 0, L.PSD_FLAG_SAVE, ctypes.byref(out)) == 0
    assert warm >= out.value                      # the cold fallback fits in it too
    assert lib.psd_workspace_size(1, L.int_array([100]), 2, L.PSD_FLAG_WARM, ctypes.byref(out)) == 1
    assert lib.psd_workspace_size(2, L.int_array([9, 9]), 0, L.PSD_FLAG_WARM, ctypes.byref(out)) == 1


def test_header_is_plain_c(tmp_path):
    """include/psdproj.h compiles as strict C99 and as C++11 (a C ABI with no
    HIP or C++ types in its declarations)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if not gcc:
        import pytest
        pytest.skip("gcc not found")
    src = tmp_path / "use.c"
    src.write_text('#include "psdproj.h"\n'
                   "int main(void) { size_t b; int n = 16; return (int)psd_workspace_size(1, &n, PSD_FP64_EIG, 0, &b); }\n")
    inc = "-I" + os.path.join(ROOT, "include")
    for cmd in ([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only", inc, str(src)],
                ["g++", "-std=c++11", "-Wall", "-Werror", "-fsyntax-only", "-x", "c++", inc, str(src)]):
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def test_warm_workspace_layout(L):
    """psd_project_warm's workspace: five n x n complex matrices (the input,
    two bases, A X, the correction) and the split-K partials of the
    products (8 + 8 slices at n = 625, 3 + 3 at 1296, one each from 2048 on:
    about 512 workgroups, at most one round of them), and never less than
    the cold path with the saved pair needs."""
    out = ctypes.c_size_t(0)
    lib = L.lib()
    for n, mats in ((625, 21), (1296, 11), (4096, 7)):
        assert lib.psd_workspace_size(1, L.int_array([n]), 0, L.PSD_FLAG_WARM, ctypes.byref(out)) == 0
        warm = out.value
        assert mats * 16 * n * n <= warm <= mats * 16 * n * n + (1 << 20), (n, warm)
        assert lib.psd_workspace_size(1, L.int_array([n]), 0, L.PSD_FLAG_SAVE, ctypes.byref(out)) == 0
        assert warm >= out.value
