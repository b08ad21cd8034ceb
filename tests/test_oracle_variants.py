"""Pins for the oracle's regulariser variants on the P-PDS skeleton of Alg. 1 (Sec. IV-A puts
the terms of the compared P-PDS-applicable methods in place of S3TTV in Prob. (18)):
  STV   sum_l ||P_l D u||_*          (blocks of first-order spatial differences)
  SSTV  ||D D_s u||_1
  HSSTV ||D D_s u||_1 + omega ||D u||_1
  SSST  sum_l ||P_l [D_v u, D_h u, D_s u]||_*   (blocks of first-order spatial and spectral
        differences, three columns per band)
Each is pinned by Lemma 2 on the dense stacked operator (the default steps are its reciprocal
column / row sums and satisfy the condition of Thm. 1), by convex duality (the primal-dual
gap closes at the P-PDS limit, with LAPACK singular values for the nuclear norms), by shift
equivariance, and HSSTV by its omega -> 0 limit. CPU only."""
import numpy as np
import pytest

import oracle
from paper_2404_03313_amd import synth

OMEGA = 0.05


def _tiny(seed=5, shape=(6, 6, 4)):
    cfg = synth.HSIConfig(*shape, endmembers=3, cells=4, sigma=0.05, p_sp=0.05, p_stripe=0.25,
                          seed=seed)
    return synth.make_hsi(cfg)


def _reg_ops(reg, shape, k1, k2):
    """Linear maps u -> dual-side vectors of the regulariser, one per dual variable."""
    dvds = lambda u: np.concatenate([oracle.dv(oracle.ds(u)).ravel(), oracle.dh(oracle.ds(u)).ravel()])
    dd = lambda u: np.concatenate([oracle.dv(u).ravel(), oracle.dh(u).ravel()])
    if reg == "stv":
        return [lambda u: oracle.blocks_extract(oracle.dv(u), oracle.dh(u), k1, k2).ravel()]
    if reg == "ssst":
        return [lambda u: oracle.blocks_extract3(oracle.dv(u), oracle.dh(u), oracle.ds(u), k1,
                                                 k2).ravel()]
    if reg == "sstv":
        return [dvds]
    return [dvds, lambda u: OMEGA * dd(u)]


@pytest.mark.parametrize("reg", ["stv", "sstv", "hsstv", "ssst"])
def test_lemma2_steps_of_each_variant(reg):
    shape, (k1, k2) = (3, 4, 3), (2, 2)
    n = int(np.prod(shape))
    I = np.eye(n)
    blocks = [np.stack([op(e.reshape(shape)) for e in I], axis=1) for op in _reg_ops(reg, shape, k1, k2)]
    A_y2t = np.stack([oracle.dv(e.reshape(shape)).ravel() for e in I], axis=1)
    Z = np.zeros
    rows = [[B, Z((B.shape[0], n)), Z((B.shape[0], n))] for B in blocks]
    rows += [[Z((n, n)), Z((n, n)), A_y2t], [I, I, I]]
    A = np.block(rows)
    col = np.abs(A).sum(axis=0)
    row = np.abs(A).sum(axis=1)
    g = oracle.default_gammas(k1, k2, reg, OMEGA)
    np.testing.assert_allclose(col[:n], 1.0 / g["gamma_u"], rtol=1e-14)
    np.testing.assert_allclose(col[n:2 * n], 1.0 / g["gamma_s"])
    np.testing.assert_allclose(col[2 * n:], 1.0 / g["gamma_t"])
    steps = [g["gamma_Y"]] + ([1.0 / (2 * OMEGA)] if reg == "hsstv" else [])
    off = 0
    G2 = []
    for B, gam in zip(blocks, steps):
        np.testing.assert_allclose(row[off:off + B.shape[0]], 1.0 / gam, rtol=1e-14)
        G2.append(np.full(B.shape[0], gam))
        off += B.shape[0]
    np.testing.assert_allclose(row[off:off + n], 1.0 / g["gamma_y2"])
    np.testing.assert_allclose(row[off + n:], 1.0 / g["gamma_y3"])
    G2 = np.concatenate(G2 + [np.full(n, g["gamma_y2"]), np.full(n, g["gamma_y3"])])
    G1 = np.concatenate([np.full(n, g["gamma_u"]), np.full(n, g["gamma_s"]), np.full(n, g["gamma_t"])])
    M = np.sqrt(G2)[:, None] * A * np.sqrt(G1)[None, :]
    assert np.linalg.norm(M, 2) ** 2 <= 1 + 1e-12


def _primal_and_adjoint(reg, r, shape, k1, k2):
    u = r["u"]
    if reg == "ssst":
        T = oracle.blocks_extract3(oracle.dv(u), oracle.dh(u), oracle.ds(u), k1, k2)
        primal = np.linalg.svd(T, compute_uv=False).sum()
        Y = r["Y"]
        assert np.linalg.norm(Y, 2, axis=(1, 2)).max() <= 1 + 1e-12
        zv, zh, zs = oracle.blocks_scatter3(Y, shape, k1, k2)
        return primal, oracle.dv_t(zv) + oracle.dh_t(zh) + oracle.ds_t(zs)
    if reg == "stv":
        T = oracle.blocks_extract(oracle.dv(u), oracle.dh(u), k1, k2)
        primal = np.linalg.svd(T, compute_uv=False).sum()
        Y = r["Y"]
        assert np.linalg.norm(Y, 2, axis=(1, 2)).max() <= 1 + 1e-12
        zv, zh = oracle.blocks_scatter(Y, shape, k1, k2)
        return primal, oracle.dv_t(zv) + oracle.dh_t(zh)
    Zd = r["Z"]
    assert np.abs(Zd).max() <= 1.0
    g = oracle.ds(u)
    primal = np.abs(oracle.dv(g)).sum() + np.abs(oracle.dh(g)).sum()
    adj = oracle.ds_t(oracle.dv_t(Zd[0]) + oracle.dh_t(Zd[1]))
    if reg == "hsstv":
        primal += OMEGA * (np.abs(oracle.dv(u)).sum() + np.abs(oracle.dh(u)).sum())
        adj = adj + OMEGA * (oracle.dv_t(Zd[2]) + oracle.dh_t(Zd[3]))
    return primal, adj


@pytest.mark.parametrize("reg", ["stv", "sstv", "hsstv", "ssst"])
def test_variant_duality_gap_closes(reg):
    """Weak duality for the variant of Prob. (19): the regulariser value at u is at least the
    dual value at any dual-feasible point, and both meet at the P-PDS limit (Thm. 1)."""
    d = _tiny()
    k1 = k2 = 2
    rad = d["radii"]
    v = d["v64"]
    gaps = []
    for iters in (3000, 10000):
        r = oracle.solve(v, k1, k2, max_iter=iters, duals=True, regularizer=reg, omega=OMEGA, **rad)
        primal, adj = _primal_and_adjoint(reg, r, v.shape, k1, k2)
        y2, y3 = r["y2"], r["y3"]
        z = adj + y3
        dual = (np.minimum(0.0 * z, 1.0 * z).sum() - rad["alpha"] * np.abs(y3).max()
                - rad["beta"] * np.abs(oracle.dv_t(y2) + y3).max()
                - np.vdot(y3, v) - rad["eps"] * np.linalg.norm(y3))
        gaps.append((primal - dual) / max(1.0, abs(primal)))
    res_dv = np.linalg.norm(oracle.dv(r["t"]))
    res_fid = np.linalg.norm(r["u"] + r["s"] + r["t"] - v) - rad["eps"]
    assert gaps[1] > -1e-9
    assert abs(gaps[1]) < abs(gaps[0])
    assert abs(gaps[1]) < 1e-5, gaps
    assert res_dv < 1e-4 and abs(res_fid) < 1e-4


@pytest.mark.parametrize("reg", ["stv", "sstv", "hsstv", "ssst"])
def test_variant_shift_equivariance(reg):
    d = _tiny(seed=3, shape=(8, 8, 6))
    kw = dict(k1=2, k2=3, max_iter=15, regularizer=reg, omega=OMEGA, **d["radii"])
    base = oracle.solve(d["v64"], **kw)
    for tr in [lambda a: np.roll(a, 3, axis=0), lambda a: np.roll(a, -2, axis=1),
               lambda a: np.roll(a, 1, axis=2)]:
        r = oracle.solve(np.ascontiguousarray(tr(d["v64"])), **kw)
        for key in ("u", "s", "t"):
            np.testing.assert_allclose(r[key], tr(base[key]), atol=1e-11)


def test_three_component_blocks_geometry():
    """P for three components: a unit impulse of component c at pixel (i, j), band b appears in
    exactly the K windows anchored at (i - a, j - c'), in row a k2 + c' and column 3b + c; the
    scatter is its adjoint; a field (0, 0, g(b)) constant over the image gives blocks of K equal
    rows, each of spectral norm sqrt(K) ||g||."""
    shape, (k1, k2) = (5, 4, 3), (2, 3)
    n1, n2, n3 = shape
    K = k1 * k2
    for comp in range(3):
        f = [np.zeros(shape) for _ in range(3)]
        f[comp][3, 1, 2] = 1.0
        T = oracle.blocks_extract3(*f, k1, k2)
        hits = np.argwhere(T != 0)
        assert len(hits) == K
        for l, r, c in hits:
            p, q = divmod(l, n2)
            a, cc = divmod(r, k2)
            assert ((p + a) % n1, (q + cc) % n2) == (3, 1) and c == 3 * 2 + comp
    rng = np.random.default_rng(7)
    f = [rng.normal(size=shape) for _ in range(3)]
    Y = rng.normal(size=(n1 * n2, K, 3 * n3))
    lhs = np.vdot(oracle.blocks_extract3(*f, k1, k2), Y)
    rhs = sum(np.vdot(a, b) for a, b in zip(f, oracle.blocks_scatter3(Y, shape, k1, k2)))
    assert abs(lhs - rhs) < 1e-10
    g = rng.normal(size=n3)
    T = oracle.blocks_extract3(np.zeros(shape), np.zeros(shape), np.broadcast_to(g, shape), k1, k2)
    np.testing.assert_allclose(np.linalg.norm(T, 2, axis=(1, 2)), np.sqrt(K) * np.linalg.norm(g),
                               rtol=1e-13)


def test_hsstv_tends_to_sstv():
    """omega -> 0 removes the first-order term: HSSTV with a negligible weight runs SSTV."""
    d = _tiny()
    g = oracle.default_gammas(2, 2, "sstv")
    a = oracle.solve(d["v64"], 2, 2, max_iter=200, gammas=g, regularizer="sstv", **d["radii"])
    b = oracle.solve(d["v64"], 2, 2, max_iter=200, gammas=g, regularizer="hsstv", omega=1e-12,
                     **d["radii"])
    for key in ("u", "s", "t"):
        np.testing.assert_allclose(b[key], a[key], atol=1e-9)
    c = oracle.solve(d["v64"], 2, 2, max_iter=200, gammas=g, regularizer="hsstv", omega=0.5,
                     **d["radii"])
    assert np.abs(c["u"] - a["u"]).max() > 1e-4


def test_rejects_bad_variant_arguments():
    d = _tiny()
    with pytest.raises(ValueError):
        oracle.solve(d["v64"], 2, 2, max_iter=5, regularizer="hsstv", omega=0.0, **d["radii"])
