"""ctypes binding of libs3ttv.so (the C ABI declared in include/s3ttv.h and s3ttv_cnn.h).

Argument marshalling only: every step of the solver runs in the HIP kernels of the library.
torch is used for device memory and the current stream. Loading fails loudly when the
library has not been built — there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libs3ttv.so")

OK, NOT_CONVERGED, EINVAL, EUNSUPPORTED, EWORKSPACE, EHIP, ENONFINITE = 0, 1, -1, -2, -3, -4, -5
K_PRIMAL, K_L1, K_GRAD, K_GRAM, K_EIG, K_APPLY, K_ZSUM, K_DUAL, K_FINAL, K_BLOCK = range(10)
GRAM_FP32, GRAM_BF16, GRAM_FP16 = 0, 1, 2
REG_S3TTV, REG_STV, REG_SSTV, REG_HSSTV, REG_SSST = 0, 1, 2, 3, 4
REGULARIZERS = {"s3ttv": REG_S3TTV, "stv": REG_STV, "sstv": REG_SSTV, "hsstv": REG_HSSTV,
                "ssst": REG_SSST}
KERNEL_NAMES = ["primal", "l1", "grad", "gram", "eig", "apply", "zsum", "dual", "final", "block"]
N_KERNEL_CLASSES = len(KERNEL_NAMES)
OP_GRAD, OP_GRAD_ADJ, OP_CLIP, OP_DUAL_BLOCKS, OP_L1 = range(5)

EXPORTS = ["s3ttv_workspace_bytes", "s3ttv_solve", "s3ttv_solve_from", "s3ttv_solve_continue",
           "s3ttv_strerror", "s3ttv_op_workspace_bytes",
           "s3ttv_op_grad", "s3ttv_op_grad_adj", "s3ttv_op_spectral_clip",
           "s3ttv_op_dual_blocks", "s3ttv_op_l1_project", "s3ttv_op_l1_project_noalloc",
           "s3ttv_batch_workspace_bytes",
           "s3ttv_solve_batched", "s3ttv_cnn_param_count", "s3ttv_cnn_workspace_bytes",
           "s3ttv_cnn_forward", "s3ttv_cnn_grad", "s3ttv_cnn_train_step"]


class Shape(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32),
                ("k1", ctypes.c_int32), ("k2", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("mu_min", ctypes.c_double), ("mu_max", ctypes.c_double),
                ("gamma_u", ctypes.c_double), ("gamma_s", ctypes.c_double),
                ("gamma_t", ctypes.c_double), ("gamma_Y", ctypes.c_double),
                ("gamma_y2", ctypes.c_double), ("gamma_y3", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("rel_tol", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("timing_mask", ctypes.c_int32),
                ("eig_max_steps", ctypes.c_int32), ("gram_precision", ctypes.c_int32),
                ("regularizer", ctypes.c_int32), ("omega", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_change", ctypes.c_double), ("l1_s", ctypes.c_double),
                ("l1_t", ctypes.c_double), ("fid", ctypes.c_double), ("dv_t", ctypes.c_double),
                ("eig_max_sweeps", ctypes.c_int32), ("eig_avg_sweeps", ctypes.c_float),
                ("eig_avg_steps", ctypes.c_float), ("eig_max_steps", ctypes.c_int32),
                ("eig_fallback_blocks", ctypes.c_int64),
                ("ms", ctypes.c_float),
                ("kernel_ms", ctypes.c_float * 10), ("kernel_calls", ctypes.c_int32 * 10),
                ("tile_a", ctypes.c_int32), ("tile_b", ctypes.c_int32), ("status", ctypes.c_int32),
                ("eig_blocks", ctypes.c_int64)]


class CnnShape(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32),
                ("nb", ctypes.c_int32)]


class S3TTVError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {strerror(code)} (code {code})")
        self.code = code


_lib = None


def lib():
    """Load libs3ttv.so (raises if it is missing: build it with paper_2404_03313_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; run `python -m paper_2404_03313_amd.build` "
                               "(the solver has no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.s3ttv_workspace_bytes.argtypes = [ctypes.POINTER(Shape), ctypes.POINTER(Params),
                                            ctypes.POINTER(sz)]
        L.s3ttv_solve.argtypes = [ctypes.POINTER(Shape), ctypes.POINTER(Params), vp, vp, vp, vp, vp,
                                  vp, sz, vp, ctypes.POINTER(Stats)]
        L.s3ttv_solve_from.argtypes = [ctypes.POINTER(Shape), ctypes.POINTER(Params), vp, vp, vp,
                                       vp, vp, vp, vp, vp, sz, vp, ctypes.POINTER(Stats)]
        L.s3ttv_solve_continue.argtypes = [ctypes.POINTER(Shape), ctypes.POINTER(Params), vp, vp,
                                           vp, vp, vp, sz, vp, ctypes.POINTER(Stats)]
        L.s3ttv_strerror.argtypes = [ctypes.c_int32]
        L.s3ttv_strerror.restype = ctypes.c_char_p
        L.s3ttv_op_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.POINTER(Shape),
                                               ctypes.c_int64, ctypes.POINTER(sz)]
        L.s3ttv_op_grad.argtypes = [ctypes.POINTER(Shape), vp, vp, vp, vp, sz, vp]
        L.s3ttv_op_grad_adj.argtypes = [ctypes.POINTER(Shape), vp, vp, vp, vp, sz, vp]
        L.s3ttv_op_spectral_clip.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp,
                                             vp, sz, vp]
        L.s3ttv_op_dual_blocks.argtypes = [ctypes.POINTER(Shape), ctypes.c_double, vp, vp, vp, vp,
                                           vp, vp, sz, vp]
        L.s3ttv_op_l1_project.argtypes = [ctypes.c_int64, vp, ctypes.c_double, vp,
                                          ctypes.POINTER(ctypes.c_double), vp, sz, vp]
        L.s3ttv_op_l1_project_noalloc.argtypes = [ctypes.c_int64, vp, ctypes.c_double, vp,
                                                  ctypes.POINTER(ctypes.c_double), vp]
        L.s3ttv_batch_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.POINTER(Shape),
                                                  ctypes.POINTER(Params), ctypes.POINTER(sz)]
        L.s3ttv_solve_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(Shape),
                                          ctypes.POINTER(Params), ctypes.POINTER(vp),
                                          ctypes.POINTER(vp), ctypes.POINTER(vp),
                                          ctypes.POINTER(vp), ctypes.POINTER(vp), vp, sz, vp,
                                          ctypes.POINTER(Stats)]
        cs = ctypes.POINTER(CnnShape)
        dp = ctypes.POINTER(ctypes.c_double)
        L.s3ttv_cnn_param_count.argtypes = []
        L.s3ttv_cnn_workspace_bytes.argtypes = [cs, ctypes.c_int32, ctypes.POINTER(sz)]
        L.s3ttv_cnn_forward.argtypes = [cs, vp, vp, vp, vp, sz, vp]
        L.s3ttv_cnn_grad.argtypes = [cs, vp, vp, vp, vp, dp, vp, sz, vp]
        L.s3ttv_cnn_train_step.argtypes = [cs, vp, vp, vp, ctypes.c_int32, ctypes.c_float, vp, vp,
                                           dp, vp, sz, vp]
        for name in EXPORTS:
            if name == "s3ttv_cnn_param_count":
                L.s3ttv_cnn_param_count.restype = ctypes.c_int64
            elif name != "s3ttv_strerror":
                getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().s3ttv_strerror(int(code)).decode()


def _check(code: int, where: str, allow=(OK,)) -> int:
    if code not in allow:
        raise S3TTVError(code, where)
    return code


# ---------------------------------------------------------------- torch helpers

def _torch():
    import torch
    return torch


def _dev_ptr(x, name: str):
    torch = _torch()
    if x is None:
        return None
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if x.dtype != torch.float32 or not x.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    return ctypes.c_void_p(x.data_ptr())


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def default_gammas(k1: int, k2: int) -> dict:
    """Lemma-2 step sizes of the stacked operator (the library's defaults)."""
    K = k1 * k2
    return dict(gamma_u=1.0 / (8 * K + 1), gamma_s=1.0, gamma_t=1.0 / 3, gamma_Y=0.25,
                gamma_y2=0.5, gamma_y3=1.0 / 3)


def make_params(eps, alpha, beta, max_iter, mu_min=0.0, mu_max=1.0, gammas: Optional[dict] = None,
                rel_tol=0.0, check_every=16, timing_mask=0, eig_max_steps=0,
                gram_precision=0, regularizer=REG_S3TTV, omega=0.0) -> Params:
    """regularizer: REG_* value or one of "s3ttv", "stv", "sstv", "hsstv"."""
    if isinstance(regularizer, str):
        regularizer = REGULARIZERS[regularizer]
    g = gammas or {}
    return Params(eps, alpha, beta, mu_min, mu_max, g.get("gamma_u", 0.0), g.get("gamma_s", 0.0),
                  g.get("gamma_t", 0.0), g.get("gamma_Y", 0.0), g.get("gamma_y2", 0.0),
                  g.get("gamma_y3", 0.0), int(max_iter), float(rel_tol), int(check_every),
                  int(timing_mask), int(eig_max_steps), int(gram_precision), int(regularizer),
                  float(omega))


def _reg_params(regularizer) -> Params:
    """Parameters carrying only a regulariser (what the workspace queries read)."""
    if isinstance(regularizer, str):
        regularizer = REGULARIZERS[regularizer]
    p = Params()
    p.regularizer = int(regularizer)
    return p


def workspace_bytes(n1, n2, n3, k1, k2, regularizer=REG_S3TTV) -> int:
    sz = ctypes.c_size_t()
    sh = Shape(n1, n2, n3, k1, k2)
    prm = _reg_params(regularizer)
    _check(lib().s3ttv_workspace_bytes(ctypes.byref(sh), ctypes.byref(prm), ctypes.byref(sz)),
           "s3ttv_workspace_bytes")
    return sz.value


class Solver:
    """Holds a workspace for one shape and runs s3ttv_solve on torch tensors."""

    def __init__(self, n1, n2, n3, k1, k2, device="cuda", regularizer=REG_S3TTV):
        self.shape = Shape(n1, n2, n3, k1, k2)
        self.dims = (n1, n2, n3)
        self.device = device
        self.ws = _workspace(workspace_bytes(n1, n2, n3, k1, k2, regularizer), device)

    def _fit(self, params: Params):
        """Grows the workspace when params' regulariser needs more (SSST's blocks have three
        columns per band); a larger workspace holds no state, so it suits a new solve only."""
        sh = self.shape
        need = workspace_bytes(sh.n1, sh.n2, sh.n3, sh.k1, sh.k2, params.regularizer)
        if self.ws.numel() < need:
            self.ws = _workspace(need, self.device)

    def solve(self, v, params: Params, u0=None, out=None, s0=None, t0=None):
        """s3ttv_solve, or s3ttv_solve_from when s0 or t0 is given."""
        torch = _torch()
        if tuple(v.shape) != self.dims:
            raise ValueError(f"v has shape {tuple(v.shape)}, expected {self.dims}")
        if out is None:
            out = tuple(torch.empty_like(v) for _ in range(3))
        u, s, t = out
        self._fit(params)
        st = Stats()
        ws = (ctypes.c_void_p(self.ws.data_ptr()), ctypes.c_size_t(self.ws.numel()), _stream(),
              ctypes.byref(st))
        if s0 is None and t0 is None:
            name = "s3ttv_solve"
            rc = lib().s3ttv_solve(ctypes.byref(self.shape), ctypes.byref(params),
                                   _dev_ptr(v, "v"), _dev_ptr(u0, "u0"), _dev_ptr(u, "u"),
                                   _dev_ptr(s, "s"), _dev_ptr(t, "t"), *ws)
        else:
            name = "s3ttv_solve_from"
            rc = lib().s3ttv_solve_from(ctypes.byref(self.shape), ctypes.byref(params),
                                        _dev_ptr(v, "v"), _dev_ptr(u0, "u0"), _dev_ptr(s0, "s0"),
                                        _dev_ptr(t0, "t0"), _dev_ptr(u, "u"), _dev_ptr(s, "s"),
                                        _dev_ptr(t, "t"), *ws)
        _check(rc, name, allow=(OK, NOT_CONVERGED))
        return u, s, t, _stats_dict(st, rc)

    def resume(self, v, params: Params, out=None):
        """s3ttv_solve_continue: params.max_iter more iterations from the iterate an earlier
        solve (or resume) of this Solver left in its workspace (same v)."""
        torch = _torch()
        if tuple(v.shape) != self.dims:
            raise ValueError(f"v has shape {tuple(v.shape)}, expected {self.dims}")
        if out is None:
            out = tuple(torch.empty_like(v) for _ in range(3))
        u, s, t = out
        st = Stats()
        rc = lib().s3ttv_solve_continue(ctypes.byref(self.shape), ctypes.byref(params),
                                        _dev_ptr(v, "v"), _dev_ptr(u, "u"), _dev_ptr(s, "s"),
                                        _dev_ptr(t, "t"), ctypes.c_void_p(self.ws.data_ptr()),
                                        ctypes.c_size_t(self.ws.numel()), _stream(),
                                        ctypes.byref(st))
        _check(rc, "s3ttv_solve_continue", allow=(OK, NOT_CONVERGED))
        return u, s, t, _stats_dict(st, rc)


def _stats_dict(st: Stats, rc: int) -> dict:
    return dict(iters=st.iters, converged=bool(st.converged), rel_change=st.rel_change,
                l1_s=st.l1_s, l1_t=st.l1_t, fid=st.fid, dv_t=st.dv_t,
                eig_max_sweeps=st.eig_max_sweeps, eig_avg_sweeps=st.eig_avg_sweeps,
                eig_avg_steps=st.eig_avg_steps, eig_max_steps=st.eig_max_steps,
                eig_fallback_blocks=st.eig_fallback_blocks, eig_blocks=st.eig_blocks, ms=st.ms,
                kernel_ms={KERNEL_NAMES[i]: st.kernel_ms[i] for i in range(N_KERNEL_CLASSES)},
                kernel_calls={KERNEL_NAMES[i]: st.kernel_calls[i]
                              for i in range(N_KERNEL_CLASSES)},
                tile=(st.tile_a, st.tile_b), status=st.status, code=rc)


def batch_workspace_bytes(shapes, params=None) -> int:
    """shapes: list of (n1, n2, n3, k1, k2); params: list of Params (their regularisers size
    the regions) or None (S3TTV)."""
    arr = (Shape * len(shapes))(*[Shape(*sh) for sh in shapes])
    prm = (Params * len(shapes))(*params) if params is not None else None
    sz = ctypes.c_size_t()
    _check(lib().s3ttv_batch_workspace_bytes(len(shapes), arr, prm, ctypes.byref(sz)),
           "s3ttv_batch_workspace_bytes")
    return sz.value


def solve_batched(problems, workspace=None):
    """Solves several problems in one batched call (s3ttv_solve_batched).

    problems: list of dicts with keys v (device cube), k1, k2, params (Params), optional u0.
    Returns ([(u, s, t, stats)], overall code). workspace: optional reusable uint8 tensor."""
    torch = _torch()
    n = len(problems)
    shapes = [(*p["v"].shape, p["k1"], p["k2"]) for p in problems]
    sh = (Shape * n)(*[Shape(*x) for x in shapes])
    prm = (Params * n)(*[p["params"] for p in problems])
    need = batch_workspace_bytes(shapes, [p["params"] for p in problems])
    dev = problems[0]["v"].device
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, dev)
    outs = [tuple(torch.empty_like(p["v"]) for _ in range(3)) for p in problems]
    vp = ctypes.c_void_p
    ptrs = lambda xs, nm: (vp * n)(*[_dev_ptr(x, nm) for x in xs])
    v = ptrs([p["v"] for p in problems], "v")
    u0 = ptrs([p.get("u0") for p in problems], "u0")
    u = ptrs([o[0] for o in outs], "u")
    s = ptrs([o[1] for o in outs], "s")
    t = ptrs([o[2] for o in outs], "t")
    st = (Stats * n)()
    rc = lib().s3ttv_solve_batched(n, sh, prm, v, u0, u, s, t, vp(workspace.data_ptr()),
                                   ctypes.c_size_t(workspace.numel()), _stream(), st)
    _check(rc, "s3ttv_solve_batched", allow=(OK, NOT_CONVERGED))
    return [(o[0], o[1], o[2], _stats_dict(st[i], st[i].status)) for i, o in enumerate(outs)], rc


def solve(v, k1, k2, eps, alpha, beta, max_iter, u0=None, s0=None, t0=None, **kw):
    """One-shot solve of Prob. (18) by Alg. 1 on the GPU; returns (u, s, t, stats)."""
    n1, n2, n3 = v.shape
    params = make_params(eps, alpha, beta, max_iter, **kw)
    sv = Solver(n1, n2, n3, k1, k2, device=v.device, regularizer=params.regularizer)
    return sv.solve(v, params, u0=u0, s0=s0, t0=t0)


# ---------------------------------------------------------------- operator entry points

def _op_ws(op, shape: Optional[Shape], n: int, device):
    sz = ctypes.c_size_t()
    _check(lib().s3ttv_op_workspace_bytes(op, ctypes.byref(shape) if shape else None, int(n),
                                          ctypes.byref(sz)), "s3ttv_op_workspace_bytes")
    return _workspace(sz.value, device)


def op_grad(u, k1=1, k2=1):
    torch = _torch()
    n1, n2, n3 = u.shape
    sh = Shape(n1, n2, n3, k1, k2)
    ws = _op_ws(OP_GRAD, sh, 0, u.device)
    gv, gh = torch.empty_like(u), torch.empty_like(u)
    _check(lib().s3ttv_op_grad(ctypes.byref(sh), _dev_ptr(u, "u"), _dev_ptr(gv, "gv"),
                               _dev_ptr(gh, "gh"), ctypes.c_void_p(ws.data_ptr()),
                               ctypes.c_size_t(ws.numel()), _stream()), "s3ttv_op_grad")
    return gv, gh


def op_grad_adj(zv, zh, k1=1, k2=1):
    torch = _torch()
    n1, n2, n3 = zv.shape
    sh = Shape(n1, n2, n3, k1, k2)
    ws = _op_ws(OP_GRAD_ADJ, sh, 0, zv.device)
    w = torch.empty_like(zv)
    _check(lib().s3ttv_op_grad_adj(ctypes.byref(sh), _dev_ptr(zv, "zv"), _dev_ptr(zh, "zh"),
                                   _dev_ptr(w, "w"), ctypes.c_void_p(ws.data_ptr()),
                                   ctypes.c_size_t(ws.numel()), _stream()), "s3ttv_op_grad_adj")
    return w


def op_spectral_clip(Y):
    """Y: (nblk, K, ncols) float32 CUDA tensor -> projection onto the unit spectral ball."""
    torch = _torch()
    nblk, K, ncols = Y.shape
    sh = Shape(1, 1, ncols, K, 1)  # CLIP: k1 = K rows, n3 = ncols
    ws = _op_ws(OP_CLIP, sh, nblk, Y.device)
    out = torch.empty_like(Y)
    _check(lib().s3ttv_op_spectral_clip(nblk, K, ncols, _dev_ptr(Y, "Y"), _dev_ptr(out, "out"),
                                        ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                        _stream()), "s3ttv_op_spectral_clip")
    return out


def op_dual_blocks(up, Y, k1, k2, gamma_Y=0.25):
    """Alg. 1 steps 9-10 on all blocks + overlap-add. up: (N1,N2,N3); Y: (N1*N2, K, 2*N3)."""
    torch = _torch()
    n1, n2, n3 = up.shape
    sh = Shape(n1, n2, n3, k1, k2)
    ws = _op_ws(OP_DUAL_BLOCKS, sh, 0, up.device)
    yout = torch.empty_like(Y)
    zv, zh = torch.empty_like(up), torch.empty_like(up)
    _check(lib().s3ttv_op_dual_blocks(ctypes.byref(sh), float(gamma_Y), _dev_ptr(up, "up"),
                                      _dev_ptr(Y, "Y"), _dev_ptr(yout, "yout"), _dev_ptr(zv, "zv"),
                                      _dev_ptr(zh, "zh"), ctypes.c_void_p(ws.data_ptr()),
                                      ctypes.c_size_t(ws.numel()), _stream()),
           "s3ttv_op_dual_blocks")
    return yout, zv, zh


def op_l1_project(x, radius):
    torch = _torch()
    ws = _op_ws(OP_L1, None, x.numel(), x.device)
    out = torch.empty_like(x)
    tau = ctypes.c_double()
    _check(lib().s3ttv_op_l1_project(x.numel(), _dev_ptr(x, "x"), float(radius),
                                     _dev_ptr(out, "out"), ctypes.byref(tau),
                                     ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                     _stream()), "s3ttv_op_l1_project")
    return out, tau.value


def op_l1_project_noalloc(x, radius, out=None):
    """s3ttv_op_l1_project_noalloc: the same projection with the library's static scratch
    (no workspace; x.numel() <= 2^24)."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(x)
    tau = ctypes.c_double()
    _check(lib().s3ttv_op_l1_project_noalloc(x.numel(), _dev_ptr(x, "x"), float(radius),
                                             _dev_ptr(out, "out"), ctypes.byref(tau), _stream()),
           "s3ttv_op_l1_project_noalloc")
    return out, tau.value


# ---------------------------------------------------------------- learned initial estimate

def cnn_param_count() -> int:
    return int(lib().s3ttv_cnn_param_count())


def _cnn_shape(v) -> CnnShape:
    """v: one (n1, n2, n3) volume or a stack (nb, n1, n2, n3)."""
    if v.dim() == 3:
        return CnnShape(*v.shape, 1)
    if v.dim() == 4:
        nb, n1, n2, n3 = v.shape
        return CnnShape(n1, n2, n3, nb)
    raise ValueError(f"expected a (n1, n2, n3) or (nb, n1, n2, n3) tensor, got {tuple(v.shape)}")


def cnn_workspace_bytes(v_shape, training: bool) -> int:
    """v_shape: (n1, n2, n3) or (nb, n1, n2, n3)."""
    d = tuple(int(x) for x in v_shape)
    sh = CnnShape(*d, 1) if len(d) == 3 else CnnShape(d[1], d[2], d[3], d[0])
    sz = ctypes.c_size_t()
    _check(lib().s3ttv_cnn_workspace_bytes(ctypes.byref(sh), int(bool(training)), ctypes.byref(sz)),
           "s3ttv_cnn_workspace_bytes")
    return sz.value


def _cnn_ws(v, training, workspace):
    need = cnn_workspace_bytes(v.shape, training)
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, v.device)
    return workspace


def cnn_forward(params, v, out=None, workspace=None):
    """u0 = v + f(v) (s3ttv_cnn_forward). params: float32 device vector."""
    torch = _torch()
    sh = _cnn_shape(v)
    ws = _cnn_ws(v, False, workspace)
    u0 = torch.empty_like(v) if out is None else out
    _check(lib().s3ttv_cnn_forward(ctypes.byref(sh), _dev_ptr(params, "params"), _dev_ptr(v, "v"),
                                   _dev_ptr(u0, "u0"), ctypes.c_void_p(ws.data_ptr()),
                                   ctypes.c_size_t(ws.numel()), _stream()), "s3ttv_cnn_forward")
    return u0


def cnn_grad(params, v, target, workspace=None):
    """(loss, gradient) of mean((v + f(v) - target)^2) (s3ttv_cnn_grad)."""
    torch = _torch()
    sh = _cnn_shape(v)
    ws = _cnn_ws(v, True, workspace)
    grad = torch.empty_like(params)
    loss = ctypes.c_double()
    _check(lib().s3ttv_cnn_grad(ctypes.byref(sh), _dev_ptr(params, "params"), _dev_ptr(v, "v"),
                                _dev_ptr(target, "target"), _dev_ptr(grad, "grad"),
                                ctypes.byref(loss), ctypes.c_void_p(ws.data_ptr()),
                                ctypes.c_size_t(ws.numel()), _stream()), "s3ttv_cnn_grad")
    return loss.value, grad


def cnn_train_step(params, adam_m, adam_v, step, lr, v, target, workspace=None):
    """One Adam step in place on params (s3ttv_cnn_train_step); returns the loss before it."""
    sh = _cnn_shape(v)
    ws = _cnn_ws(v, True, workspace)
    loss = ctypes.c_double()
    _check(lib().s3ttv_cnn_train_step(ctypes.byref(sh), _dev_ptr(params, "params"),
                                      _dev_ptr(adam_m, "adam_m"), _dev_ptr(adam_v, "adam_v"),
                                      int(step), float(lr), _dev_ptr(v, "v"),
                                      _dev_ptr(target, "target"), ctypes.byref(loss),
                                      ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                      _stream()), "s3ttv_cnn_train_step")
    return loss.value
