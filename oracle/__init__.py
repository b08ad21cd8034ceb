"""FP64 CPU oracle for S3TTV / P-PDS (arXiv 2404.03313) — TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package. It wraps ``s3ttv_oracle.c`` (plain C + OpenMP, float64) through
ctypes and shares no code with the GPU library. Arrays are C-contiguous float64 cubes of
shape (N1, N2, N3) = (rows, columns, bands).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "s3ttv_oracle.c")
_LIB = os.path.join(_HERE, "libs3ttv_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (IEEE double, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        for name in ("ora_dv", "ora_dv_t", "ora_dh", "ora_dh_t", "ora_ds", "ora_ds_t"):
            f = getattr(L, name)
            f.argtypes = [ctypes.c_int] * 3 + [_dp, _dp]
            f.restype = None
        L.ora_blocks_extract.argtypes = [ctypes.c_int] * 5 + [_dp, _dp, _dp]
        L.ora_blocks_scatter.argtypes = [ctypes.c_int] * 5 + [_dp, _dp, _dp]
        L.ora_blocks_extract3.argtypes = [ctypes.c_int] * 5 + [_dp, _dp, _dp, _dp]
        L.ora_blocks_scatter3.argtypes = [ctypes.c_int] * 5 + [_dp, _dp, _dp, _dp]
        L.ora_struct_tensor.argtypes = [ctypes.c_int] * 5 + [_dp, _dp]
        L.ora_struct_tensor_adj.argtypes = [ctypes.c_int] * 5 + [_dp, _dp]
        L.ora_svd_rows.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp]
        L.ora_svd_rows.restype = ctypes.c_int
        L.ora_prox_nuclear.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.ora_prox_nuclear.restype = ctypes.c_int
        L.ora_dual_nuclear.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.ora_dual_nuclear.restype = ctypes.c_int
        L.ora_proj_box.argtypes = [ctypes.c_int64, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.ora_proj_l2.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_double, _dp]
        L.ora_proj_l1.argtypes = [ctypes.c_int64, _dp, ctypes.c_double, _dp]
        L.ora_proj_l1.restype = ctypes.c_double
        L.ora_s3ttv.argtypes = [ctypes.c_int] * 5 + [_dp]
        L.ora_s3ttv.restype = ctypes.c_double
        L.ora_solve.argtypes = [_ip, _dp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                _dp, _dp, _dp, _dp, _dp]
        L.ora_solve.restype = ctypes.c_int
        L.ora_set_threads.argtypes = [ctypes.c_int]
        L.ora_get_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    lib().ora_set_threads(int(n))


def get_threads() -> int:
    return int(lib().ora_get_threads())


def _unary(name: str, x: np.ndarray) -> np.ndarray:
    x = _f64(x)
    y = np.empty_like(x)
    getattr(lib(), name)(*x.shape, _p(x), _p(y))
    return y


def dv(x):
    return _unary("ora_dv", x)


def dv_t(x):
    return _unary("ora_dv_t", x)


def dh(x):
    return _unary("ora_dh", x)


def dh_t(x):
    return _unary("ora_dh_t", x)


def ds(x):
    return _unary("ora_ds", x)


def ds_t(x):
    return _unary("ora_ds_t", x)


def blocks_extract(gv, gh, k1: int, k2: int) -> np.ndarray:
    """P applied to the two-component field (gv, gh): returns (N1*N2, k1*k2, 2*N3)."""
    gv, gh = _f64(gv), _f64(gh)
    n1, n2, n3 = gv.shape
    T = np.empty((n1 * n2, k1 * k2, 2 * n3))
    lib().ora_blocks_extract(n1, n2, n3, k1, k2, _p(gv), _p(gh), _p(T))
    return T


def blocks_scatter(Y, shape, k1: int, k2: int):
    """P^T: sum of the blocks back onto the two-component field; returns (zv, zh)."""
    Y = _f64(Y)
    n1, n2, n3 = shape
    zv = np.empty(shape)
    zh = np.empty(shape)
    lib().ora_blocks_scatter(n1, n2, n3, k1, k2, _p(Y), _p(zv), _p(zh))
    return zv, zh


def blocks_extract3(gv, gh, gs, k1: int, k2: int) -> np.ndarray:
    """P applied to a three-component field (gv, gh, gs), column 3b + comp: returns
    (N1*N2, k1*k2, 3*N3)."""
    gv, gh, gs = _f64(gv), _f64(gh), _f64(gs)
    n1, n2, n3 = gv.shape
    T = np.empty((n1 * n2, k1 * k2, 3 * n3))
    lib().ora_blocks_extract3(n1, n2, n3, k1, k2, _p(gv), _p(gh), _p(gs), _p(T))
    return T


def blocks_scatter3(Y, shape, k1: int, k2: int):
    """Adjoint of blocks_extract3; returns (zv, zh, zs)."""
    Y = _f64(Y)
    n1, n2, n3 = shape
    z = [np.empty(shape) for _ in range(3)]
    lib().ora_blocks_scatter3(n1, n2, n3, k1, k2, _p(Y), *(_p(x) for x in z))
    return tuple(z)


def struct_tensor(u, k1: int, k2: int) -> np.ndarray:
    """T_l = P_l D D_s u for all l (eq. rewrite_Lu): (N1*N2, k1*k2, 2*N3)."""
    u = _f64(u)
    n1, n2, n3 = u.shape
    T = np.empty((n1 * n2, k1 * k2, 2 * n3))
    lib().ora_struct_tensor(n1, n2, n3, k1, k2, _p(u), _p(T))
    return T


def struct_tensor_adj(Y, shape, k1: int, k2: int) -> np.ndarray:
    Y = _f64(Y)
    n1, n2, n3 = shape
    w = np.empty(shape)
    lib().ora_struct_tensor_adj(n1, n2, n3, k1, k2, _p(Y), _p(w))
    return w


def svd_rows(A):
    """Hand-written one-sided Jacobi SVD of A (m x n, m <= n): (sig, U, Vt, sweeps)."""
    A = _f64(A)
    m, n = A.shape
    assert m <= n
    sig = np.empty(m)
    U = np.empty((m, m))
    Vt = np.empty((m, n))
    sw = lib().ora_svd_rows(m, n, _p(A), _p(sig), _p(U), _p(Vt))
    return sig, U, Vt, sw


def prox_nuclear(A, lam: float) -> np.ndarray:
    A = _f64(A)
    out = np.empty_like(A)
    sw = lib().ora_prox_nuclear(A.shape[0], A.shape[1], float(lam), _p(A), _p(out))
    if sw < 0:
        raise RuntimeError("oracle Jacobi SVD did not converge")
    return out


def dual_nuclear(Yp, gamma: float) -> np.ndarray:
    """Alg. 1 step 10 on one block: Y' - g prox_{||.||_*/g}(Y'/g)."""
    Yp = _f64(Yp)
    out = np.empty_like(Yp)
    sw = lib().ora_dual_nuclear(Yp.shape[0], Yp.shape[1], float(gamma), _p(Yp), _p(out))
    if sw < 0:
        raise RuntimeError("oracle Jacobi SVD did not converge")
    return out


def proj_box(x, lo: float, hi: float) -> np.ndarray:
    x = _f64(x)
    out = np.empty_like(x)
    lib().ora_proj_box(x.size, _p(x), float(lo), float(hi), _p(out))
    return out


def proj_l2(x, v, eps: float) -> np.ndarray:
    x, v = _f64(x), _f64(v)
    out = np.empty_like(x)
    lib().ora_proj_l2(x.size, _p(x), _p(v), float(eps), _p(out))
    return out


def proj_l1(x, alpha: float):
    """Returns (projection, tau)."""
    x = _f64(x)
    out = np.empty_like(x)
    tau = lib().ora_proj_l1(x.size, _p(x), float(alpha), _p(out))
    return out, float(tau)


def s3ttv(u, k1: int, k2: int) -> float:
    u = _f64(u)
    return float(lib().ora_s3ttv(*u.shape, k1, k2, _p(u)))


REGULARIZERS = {"s3ttv": 0, "stv": 1, "sstv": 2, "hsstv": 3, "ssst": 4}
BLOCK_COMPONENTS = {"s3ttv": 2, "stv": 2, "ssst": 3}


def default_gammas(k1: int, k2: int, regularizer: str = "s3ttv", omega: float = 0.05) -> dict:
    """Lemma-2 step sizes for the stacked operator. S3TTV: column sums 8K+1, 1, 3; row sums 4,
    2, 3. STV (blocks of D u): 4K+1 and block rows 2. SSTV (||D D_s u||_1): 9 and rows 4.
    HSSTV (+ omega ||D u||_1): 9 + 4 omega; its second field steps with 1/(2 omega).
    SSST (blocks of (D_v u, D_h u, D_s u)): 6K+1 and block rows 2."""
    K = k1 * k2
    g_u = {"s3ttv": 1.0 / (8 * K + 1), "stv": 1.0 / (4 * K + 1), "sstv": 1.0 / 9,
           "hsstv": 1.0 / (9 + 4 * omega), "ssst": 1.0 / (6 * K + 1)}[regularizer]
    return dict(gamma_u=g_u, gamma_s=1.0, gamma_t=1.0 / 3,
                gamma_Y=0.5 if regularizer in ("stv", "ssst") else 0.25, gamma_y2=0.5,
                gamma_y3=1.0 / 3)


def solve(v, k1: int, k2: int, eps: float, alpha: float, beta: float, max_iter: int,
          mu_min: float = 0.0, mu_max: float = 1.0, gammas: Optional[dict] = None,
          rel_tol: float = 0.0, u0=None, trace: bool = False, duals: bool = False,
          s0=None, t0=None, regularizer: str = "s3ttv", omega: float = 0.05) -> dict:
    """Alg. 1 in float64. Returns dict(u, s, t, stats[, trace][, Y or Z, y2, y3]).
    u0, s0, t0: optional initial values (zero when None); the duals start at zero.
    regularizer: "s3ttv" (Prob. (18)), or the compared P-PDS-applicable terms "stv",
    "sstv", "hsstv" (weight omega), "ssst" in its place (Sec. IV-A). Y (S3TTV, STV, SSST): the
    block duals (N1*N2, K, c*N3), c = 2 (3 for SSST, column 3b + comp). Z (SSTV, HSSTV): the
    dual fields (z1v, z1h, z2v, z2h) stacked, shape (4, N1, N2, N3)."""
    reg = REGULARIZERS[regularizer]
    v = _f64(v)
    n1, n2, n3 = v.shape
    g = gammas or {}
    prm = np.array([eps, alpha, beta, mu_min, mu_max,
                    g.get("gamma_u", 0.0), g.get("gamma_s", 0.0), g.get("gamma_t", 0.0),
                    g.get("gamma_Y", 0.0), g.get("gamma_y2", 0.0), g.get("gamma_y3", 0.0),
                    rel_tol, reg, omega], dtype=np.float64)
    dims = (ctypes.c_int * 5)(n1, n2, n3, k1, k2)
    u = np.empty_like(v)
    s = np.empty_like(v)
    t = np.empty_like(v)
    st = np.zeros(8)
    tr = np.zeros(max_iter) if trace else None
    blk = regularizer in BLOCK_COMPONENTS
    Y = (np.empty((n1 * n2, k1 * k2, BLOCK_COMPONENTS[regularizer] * n3)) if duals and blk
         else None)
    Z = np.empty((4,) + v.shape) if duals and not blk else None
    y2 = np.empty_like(v) if duals else None
    y3 = np.empty_like(v) if duals else None
    u0a = _f64(u0) if u0 is not None else None
    s0a = _f64(s0) if s0 is not None else None
    t0a = _f64(t0) if t0 is not None else None
    rc = lib().ora_solve(dims, _p(prm), int(max_iter), _p(v), _p(u0a), _p(s0a), _p(t0a), _p(u),
                         _p(s), _p(t), _p(st), _p(tr), _p(Y), _p(Z), _p(y2), _p(y3))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    out = dict(u=u, s=s, t=t, stats=dict(iters=int(st[0]), rel_change=st[1],
                                         converged=bool(st[2]), dv_t_norm=st[3],
                                         fid_excess=st[4], l1_s_excess=st[5],
                                         l1_t_excess=st[6], worst_sweeps=int(st[7])))
    if trace:
        out["trace"] = tr[:out["stats"]["iters"]]
    if duals:
        out.update(y2=y2, y3=y3)
        out.update(Y=Y) if blk else out.update(Z=Z)
    return out
