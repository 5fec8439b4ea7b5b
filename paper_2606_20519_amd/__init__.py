"""MI355X (gfx950) projection onto the complex Hermitian PSD cone.

Python binding of libpsdproj.so (include/psdproj.h).  PyTorch supplies device
memory and the stream; every step of the projection runs in the library's
HIP kernels.  Inputs and outputs are float64 device tensors in the svec
encoding (App. D.1 vec_R): per row i of the upper triangle, X_ii followed by
sqrt(2) Re X_ij, sqrt(2) Im X_ij for j > i; a block of order n has n*n reals.

    project(x, n, mode="fp64")            -> svec(Pi(mat(x)))
    project_batched(x, sizes, mode)       -> blocks projected independently
    vjp(gy, n, x=None, saved=None)        -> svec(DPi(X)[mat(gy)])
    PSDProject.apply(x, n, mode)          -> differentiable projection
    scs_solve(g, d, eps=1e-5, ...)        -> SCS solve of the process-matrix SDP
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import MODES, PSD_FLAG_SAVE, PSD_FLAG_WARM, PsdError, PsdInfo, check  # noqa: F401

__all__ = ["project", "project_batched", "vjp", "PSDProject", "Plan", "workspace", "set_ns_iterations",
           "set_mixed_fallback", "project_noalloc", "affine_dims", "constraint_apply", "constraint_adjoint",
           "affine_step", "scs_solve", "scs_solve_batched",
           "PsdError", "MODES"]

_ws_cache: dict = {}
INFO_WORDS = ctypes.sizeof(PsdInfo) // 4


def set_ns_iterations(iters: int = 0, corrections: int = -1):
    """Newton-Schulz steps (0: automatic, the scaled schedule's 21) and FP64
    correction steps of the mixed modes (-1: automatic, 1 for BF16 and 0 for
    FP32 and split BF16)."""
    _lib.set_ns_iterations(iters, corrections)


def set_mixed_fallback(max_rel_err: float = 0.0):
    """FP64 re-run of a mixed-mode `project` whose error estimate exceeds
    `max_rel_err` (0 disables it; the call then synchronises its stream)."""
    _lib.set_mixed_fallback(max_rel_err)


def _mode(mode) -> int:
    if isinstance(mode, str):
        return MODES[mode]
    return int(mode)


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def workspace(sizes, mode, device, flags: int = 0) -> torch.Tensor:
    """A cached device workspace large enough for `sizes` in `mode`."""
    nbytes = _lib.workspace_size(list(sizes), _mode(mode), flags)
    key = (str(device), torch.cuda.current_stream(device).cuda_stream)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = ws
    return ws


def _check_vec(x: torch.Tensor, numel: int, what: str):
    if not x.is_cuda or x.dtype != torch.float64:
        raise TypeError(f"{what} must be a float64 HIP tensor")
    if x.numel() != numel or not x.is_contiguous():
        raise ValueError(f"{what} must be contiguous with {numel} elements")


def project(x: torch.Tensor, n: int, mode="fp64", out: torch.Tensor = None, info: bool = False,
            saved: torch.Tensor = None):
    """svec(Pi(mat(x))) for one block of order n.  With info=True also
    returns the device record (status, n_pos, n_neg, ...) as a dict (this
    synchronises).  `saved` (float64, psd_saved_size(n)/8 elements) receives
    the eigen-pair for a later vjp."""
    _check_vec(x, n * n, "x")
    y = torch.empty_like(x) if out is None else out
    _check_vec(y, n * n, "out")
    m = _mode(mode)
    ws = workspace([n], m, x.device, PSD_FLAG_SAVE if saved is not None else 0)
    inf_t = torch.zeros(INFO_WORDS, dtype=torch.int32, device=x.device) if info else None
    st = _lib.lib().psd_project(n, _ptr(x), _ptr(y), m, _ptr(ws), ws.numel(), ctypes.c_void_p(_stream_ptr(x.device)),
                                _ptr(inf_t), _ptr(saved))
    check(st, "psd_project")
    if info:
        return y, _info_dict(inf_t)
    return y


def project_warm(x: torch.Tensor, n: int, saved_prev: torch.Tensor, saved_out: torch.Tensor = None,
                 out: torch.Tensor = None, info: bool = False):
    """svec(Pi(mat(x))) in FP64 through psd_project_warm: the eigen-pair in
    `saved_prev` (from project(..., saved=) or an earlier call) is refined
    for x, and the refined pair goes to `saved_out` (default: saved_prev,
    updated in place).  Falls back to the cold path when the pair is not
    close (info["fallback"] == 1).  Synchronises the current stream."""
    _check_vec(x, n * n, "x")
    nsv = _lib.saved_size(n) // 8
    _check_vec(saved_prev, nsv, "saved_prev")
    so = saved_prev if saved_out is None else saved_out
    _check_vec(so, nsv, "saved_out")
    y = torch.empty_like(x) if out is None else out
    _check_vec(y, n * n, "out")
    ws = workspace([n], MODES["fp64"], x.device, PSD_FLAG_WARM)
    inf_t = torch.zeros(INFO_WORDS, dtype=torch.int32, device=x.device) if info else None
    st = _lib.lib().psd_project_warm(n, _ptr(x), _ptr(y), _ptr(saved_prev), _ptr(so), _ptr(ws), ws.numel(),
                                     ctypes.c_void_p(_stream_ptr(x.device)), _ptr(inf_t))
    check(st, "psd_project_warm")
    if info:
        return y, _info_dict(inf_t)
    return y


def project_noalloc(x: torch.Tensor, n: int, mode="fp64", out: torch.Tensor = None, info: bool = False):
    """svec(Pi(mat(x))) through psd_project_noalloc: the library's fixed
    device scratch instead of a workspace (orders up to 831 in FP64, 768 in
    BF16-mixed, 704 in FP32-mixed)."""
    _check_vec(x, n * n, "x")
    y = torch.empty_like(x) if out is None else out
    _check_vec(y, n * n, "out")
    inf_t = torch.zeros(INFO_WORDS, dtype=torch.int32, device=x.device) if info else None
    st = _lib.lib().psd_project_noalloc(n, _ptr(x), _ptr(y), _mode(mode), ctypes.c_void_p(_stream_ptr(x.device)),
                                        _ptr(inf_t))
    check(st, "psd_project_noalloc")
    if info:
        return y, _info_dict(inf_t)
    return y


def _info_dict(t: torch.Tensor) -> dict:
    raw = t.cpu().numpy().tobytes()
    rec = PsdInfo.from_buffer_copy(raw[:ctypes.sizeof(PsdInfo)])
    return {f: getattr(rec, f) for f, _ in PsdInfo._fields_}


def info_records(t: torch.Tensor, count: int) -> list:
    """The first `count` psd_info records of an int32 tensor (device or host)
    as dicts (synchronises)."""
    raw = t.cpu().numpy().tobytes()
    k = ctypes.sizeof(PsdInfo)
    recs = [PsdInfo.from_buffer_copy(raw[i * k:(i + 1) * k]) for i in range(count)]
    return [{f: getattr(r, f) for f, _ in PsdInfo._fields_} for r in recs]


def project_batched(x: torch.Tensor, sizes, mode="fp64", out: torch.Tensor = None, info: bool = False):
    """Projects consecutive svec blocks of orders `sizes` independently."""
    sizes = [int(s) for s in sizes]
    total = sum(s * s for s in sizes)
    _check_vec(x, total, "x")
    y = torch.empty_like(x) if out is None else out
    _check_vec(y, total, "out")
    m = _mode(mode)
    ws = workspace(sizes, m, x.device)
    inf_t = torch.zeros(INFO_WORDS * len(sizes), dtype=torch.int32, device=x.device) if info else None
    st = _lib.lib().psd_project_batched(len(sizes), _lib.int_array(sizes), _ptr(x), _ptr(y), m, _ptr(ws),
                                        ws.numel(), ctypes.c_void_p(_stream_ptr(x.device)), _ptr(inf_t))
    check(st, "psd_project_batched")
    if info:
        return y, info_records(inf_t, len(sizes))
    return y


def saved_numel(n: int) -> int:
    return _lib.saved_size(n) // 8


def vjp(gy: torch.Tensor, n: int, x: torch.Tensor = None, saved: torch.Tensor = None, mode="fp64",
        out: torch.Tensor = None):
    """svec(DPi(X)[mat(gy)]) (Daleckii-Krein); DPi is self-adjoint, so this is
    the vector-Jacobian product.  Pass x or the `saved` eigen-pair."""
    _check_vec(gy, n * n, "gy")
    if x is None and saved is None:
        raise ValueError("vjp needs x or saved")
    gx = torch.empty_like(gy) if out is None else out
    m = _mode(mode)
    ws = workspace([n], m, gy.device, PSD_FLAG_SAVE)
    st = _lib.lib().psd_project_vjp(n, _ptr(x), _ptr(saved), _ptr(gy), _ptr(gx), m, _ptr(ws), ws.numel(),
                                    ctypes.c_void_p(_stream_ptr(gy.device)))
    check(st, "psd_project_vjp")
    return gx


_aff_ws: dict = {}


def _affine_ws(d: int, device) -> torch.Tensor:
    nbytes = _lib.affine_workspace_size(d)
    key = (str(device), d)
    ws = _aff_ws.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _aff_ws[key] = ws
    return ws


def affine_dims(d: int):
    """(nx, ny) of the bipartite process-matrix SDP at local dimension d."""
    return _lib.affine_dims(d)


def constraint_apply(x: torch.Tensor, d: int, out: torch.Tensor = None) -> torch.Tensor:
    """svec(A x), A x = -sum_mu x_mu F_mu (App. D.1)."""
    nx, ny = _lib.affine_dims(d)
    _check_vec(x, nx, "x")
    y = torch.empty(ny, dtype=torch.float64, device=x.device) if out is None else out
    _check_vec(y, ny, "out")
    ws = _affine_ws(d, x.device)
    check(_lib.lib().psd_constraint_apply(d, _ptr(x), _ptr(y), _ptr(ws), ws.numel(),
                                          ctypes.c_void_p(_stream_ptr(x.device))), "psd_constraint_apply")
    return y


def constraint_adjoint(y: torch.Tensor, d: int, out: torch.Tensor = None) -> torch.Tensor:
    """A^T mat(y), (A^T Z)_mu = -tr[F_mu Z] (App. D.1)."""
    nx, ny = _lib.affine_dims(d)
    _check_vec(y, ny, "y")
    x = torch.empty(nx, dtype=torch.float64, device=y.device) if out is None else out
    _check_vec(x, nx, "out")
    ws = _affine_ws(d, y.device)
    check(_lib.lib().psd_constraint_adjoint(d, _ptr(y), _ptr(x), _ptr(ws), ws.numel(),
                                            ctypes.c_void_p(_stream_ptr(y.device))), "psd_constraint_adjoint")
    return x


def affine_step(ax: torch.Tensor, ay: torch.Tensor, d: int, zx: torch.Tensor = None, zy: torch.Tensor = None):
    """(z_x, z_y) = ((a_x - A^T a_y)/2, a_y + A z_x): the affine projection of
    the SCS iteration (App. D.2)."""
    nx, ny = _lib.affine_dims(d)
    _check_vec(ax, nx, "ax")
    _check_vec(ay, ny, "ay")
    zx = torch.empty_like(ax) if zx is None else zx
    zy = torch.empty_like(ay) if zy is None else zy
    _check_vec(zx, nx, "zx")
    _check_vec(zy, ny, "zy")
    ws = _affine_ws(d, ay.device)
    check(_lib.lib().psd_affine_step(d, _ptr(ax), _ptr(ay), _ptr(zx), _ptr(zy), _ptr(ws), ws.numel(),
                                     ctypes.c_void_p(_stream_ptr(ay.device))), "psd_affine_step")
    return zx, zy


def scs_solve(g: torch.Tensor, d: int, eps: float = 1e-5, alpha: float = 1.5, max_iters: int = 5000,
              check_every: int = 1, normalize: bool = True, mixed_iters: int = 0, mixed_mode="mixed_fp32",
              warm=None, post: bool = True, anderson: int = 0, mixed_switch: float = 0.0,
              ws: torch.Tensor = None, warm_proj: bool = False) -> dict:
    """Solve max tr[W G] over process matrices by the SCS iteration on the
    GPU (App. D; psd_scs_solve).  g: svec of G (d^8 float64 on the device).
    warm: optional (x, y, s) start.  anderson: memory of the type-I
    Anderson acceleration (0: off).  mixed_iters / mixed_mode: cone steps in
    a mixed mode first; mixed_switch > 0 moves to FP64 as soon as the
    residuals are within that factor of the tolerance.  warm_proj: the FP64
    cone steps after the first by psd_project_warm from the previous step's
    eigen-pair (counts in warm_refined / warm_fallbacks).  Returns the unscaled
    x, y, s, the post-processed process matrix w (if `post`), and the info
    record as a dict (status, iters, pobj, dobj, residuals, tau, kappa,
    sigma, ...)."""
    out = scs_solve_batched(g.reshape(1, -1), d, eps=eps, alpha=alpha, max_iters=max_iters,
                            check_every=check_every, normalize=normalize, mixed_iters=mixed_iters,
                            mixed_mode=mixed_mode, warm=None if warm is None else tuple(t.reshape(1, -1) for t in warm),
                            post=post, anderson=anderson, mixed_switch=mixed_switch, ws=ws, _single=True,
                            warm_proj=warm_proj)
    return out[0]


def scs_solve_batched(g: torch.Tensor, d: int, eps: float = 1e-5, alpha: float = 1.5, max_iters: int = 5000,
                      check_every: int = 1, normalize: bool = True, mixed_iters: int = 0, mixed_mode="mixed_fp32",
                      warm=None, post: bool = True, anderson: int = 0, mixed_switch: float = 0.0,
                      ws: torch.Tensor = None, _single: bool = False, warm_proj: bool = False) -> list:
    """A batch of independent solves in lockstep (psd_scs_solve_batched):
    g is (B, d^8); warm an optional (x, y, s) of shapes (B, n_x), (B, d^8),
    (B, d^8).  Returns one dict per instance, as scs_solve."""
    nx, ny = _lib.affine_dims(d)
    if g.dim() != 2 or g.shape[1] != ny:
        raise ValueError(f"g must be (B, {ny})")
    B = g.shape[0]
    _check_vec(g.reshape(-1), B * ny, "g")
    st = _lib.ScsSettings(d=d, max_iters=max_iters, check_every=check_every, mixed_iters=mixed_iters,
                          mixed_mode=_mode(mixed_mode), normalize=int(bool(normalize)),
                          warm_start=int(warm is not None), anderson=anderson, eps=eps, alpha=alpha,
                          mixed_switch=mixed_switch, warm_proj=int(bool(warm_proj)))
    nbytes = _lib.scs_workspace_size(st, B)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=g.device)
    if warm is not None:
        x, y, s = (t.contiguous().clone() for t in warm)
        _check_vec(x.reshape(-1), B * nx, "warm x")
        _check_vec(y.reshape(-1), B * ny, "warm y")
        _check_vec(s.reshape(-1), B * ny, "warm s")
    else:
        x = torch.empty(B, nx, dtype=torch.float64, device=g.device)
        y = torch.empty(B, ny, dtype=torch.float64, device=g.device)
        s = torch.empty(B, ny, dtype=torch.float64, device=g.device)
    w = torch.empty(B, ny, dtype=torch.float64, device=g.device) if post else None
    infos = (_lib.ScsInfo * B)()
    fn = _lib.lib().psd_scs_solve if _single else None
    if _single:
        st_ = fn(ctypes.byref(st), _ptr(g), _ptr(x), _ptr(y), _ptr(s), _ptr(w), _ptr(ws), ws.numel(),
                 ctypes.c_void_p(_stream_ptr(g.device)), infos)
        check(st_, "psd_scs_solve")
    else:
        check(_lib.lib().psd_scs_solve_batched(ctypes.byref(st), B, _ptr(g), _ptr(x), _ptr(y), _ptr(s), _ptr(w),
                                               _ptr(ws), ws.numel(), ctypes.c_void_p(_stream_ptr(g.device)), infos),
              "psd_scs_solve_batched")
    out = []
    for b in range(B):
        rec = {f: getattr(infos[b], f) for f, _ in _lib.ScsInfo._fields_}
        rec.update(x=x[b], y=y[b], s=s[b], w=None if w is None else w[b])
        out.append(rec)
    return out


class PSDProject(torch.autograd.Function):
    """y = svec(Pi(mat(x))) with backward gx = svec(DPi(X)[mat(gy)]).

    fp64: the forward saves the eigen-pair and the backward reuses it.
    Mixed modes: the forward is the Newton-Schulz form (no eigenvectors), so
    it saves x and the backward recomputes the FP64 eigen-pair."""

    @staticmethod
    def forward(ctx, x, n, mode="fp64"):
        xd = x.detach().contiguous()
        ctx.n = n
        ctx.mode = mode
        if _mode(mode) == MODES["fp64"]:
            saved = torch.empty(saved_numel(n), dtype=torch.float64, device=x.device)
            y = project(xd, n, mode, saved=saved)
            ctx.save_for_backward(saved)
            ctx.from_x = False
        else:
            y = project(xd, n, mode)
            ctx.save_for_backward(xd)
            ctx.from_x = True
        return y

    @staticmethod
    def backward(ctx, gy):
        (t,) = ctx.saved_tensors
        if ctx.from_x:
            gx = vjp(gy.contiguous(), ctx.n, x=t, mode=ctx.mode)
        else:
            gx = vjp(gy.contiguous(), ctx.n, saved=t, mode=ctx.mode)
        return gx, None, None


class Plan:
    """All blocks of one cone projected by a single graph launch
    (psd_plan_* in the C ABI).  Typical use: create once per cone layout,
    then `execute(x, out=y)` every SCS iteration with the same buffers."""

    def __init__(self, sizes, mode="fp64", concurrency: int = 0, device="cuda:0"):
        self.sizes = [int(s) for s in sizes]
        self.mode = _mode(mode)
        self.device = torch.device(device)
        h = ctypes.c_void_p(0)
        check(_lib.lib().psd_plan_create(len(self.sizes), _lib.int_array(self.sizes), self.mode, concurrency,
                                          ctypes.byref(h)), "psd_plan_create")
        self._h = h
        self.total = sum(s * s for s in self.sizes)
        self._ws = None

    @property
    def concurrency(self) -> int:
        return int(_lib.lib().psd_plan_concurrency(self._h))

    @property
    def group_size(self) -> int:
        """Members of the largest lockstep group (same-order blocks sharing
        every launch)."""
        return int(_lib.lib().psd_plan_group_size(self._h))

    @property
    def ns_tile_threshold(self) -> int:
        """Padded order from which the plan's BF16 Newton-Schulz products use
        128x128 tiles (2048 by default; 1024 if the autotuner chose it)."""
        return int(_lib.lib().psd_plan_ns_tile_threshold(self._h))

    def workspace(self, concurrency: int = 0) -> torch.Tensor:
        nb = ctypes.c_size_t(0)
        check(_lib.lib().psd_plan_workspace_size(self._h, concurrency, ctypes.byref(nb)), "psd_plan_workspace_size")
        if self._ws is None or self._ws.numel() < nb.value:
            self._ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def execute(self, x: torch.Tensor, out: torch.Tensor = None, infos: torch.Tensor = None) -> torch.Tensor:
        _check_vec(x, self.total, "x")
        y = torch.empty_like(x) if out is None else out
        _check_vec(y, self.total, "out")
        ws = self.workspace()
        st = _lib.lib().psd_plan_execute(self._h, _ptr(x), _ptr(y), _ptr(ws), ws.numel(),
                                         ctypes.c_void_p(_stream_ptr(x.device)), _ptr(infos))
        check(st, "psd_plan_execute")
        return y

    def tune(self, x: torch.Tensor, out: torch.Tensor, reps: int = 3, max_concurrency: int = 32) -> int:
        ws = self.workspace(max_concurrency)
        best = ctypes.c_int32(0)
        st = _lib.lib().psd_plan_tune(self._h, _ptr(x), _ptr(out), _ptr(ws), ws.numel(),
                                      ctypes.c_void_p(_stream_ptr(x.device)), reps, ctypes.byref(best))
        check(st, "psd_plan_tune")
        return int(best.value)

    def close(self):
        if self._h is not None and self._h.value:
            _lib.lib().psd_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
