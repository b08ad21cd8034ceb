"""Benchmark: P-PDS iterations/s of the S3TTV solver on one MI355X.

A step is one full iteration of Alg. 1 (primal step, both l1-ball projections, gradient
field, block Gram / eigen-solve / spectral clip / overlap-add, dual steps, scalar
reductions) on a seeded synthetic 256 x 256 x 128 hyperspectral cube with block 4 x 4. The
timed steps continue a solve from zero after a pre-roll (200 iterations by default) and the
warm-up steps, so they are iterations of the phase in which the blocks clip (from zero no
block clips during the first ~30 iterations; a solve to rel-tol 1e-4 takes ~625).

Prints one JSON line. Besides the throughput it reports
  - roofline: the dominant kernel (the fused block pass: Gram, eigen-solve, clip and
    overlap-add of every dual block) timed live with HIP events inside the timed solve,
    against the algorithmic bytes of steps 9-10 (every dual block read and written once) and
    the 8 TB/s HBM peak; the bytes the pass moves by design are reported beside them;
  - gram_mfma: the Gram products' flop rate over the block-pass time against the MFMA peak
    of their input precision, and the matrix-pipe busy fraction from the counter summary;
  - time_to_rel_tol: wall time and iterations of a solve stopped by the paper's rule with
    tolerance 1e-4;
  - cpu_baseline: the FP64 oracle timed on this host on a bounded sample (the first three
    iterations of the same workload).
Other workloads (--workload): c4, the uneven batch of 24 images in one batched call; c5, the
learned initial estimate (training on solver-generated pairs, then a 512 x 512 x 191 scene
solved from zero and from the network's estimate); paper10, the paper's experimental shape
(100 x 100 x 198, 10 x 10 windows, stop rule 1e-5) with the paper's running time as context.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "P-PDS iters/sec + time-to-rel-tol 1e-4, 256×256×128 HSI, vs plain FP32 on one GPU"


def block_pass_algorithmic_bytes(n1: int, n2: int, n3: int, k1: int, k2: int) -> int:
    """Bytes the block pass (Alg. 1 steps 9-10) must move per launch: read and write every dual
    block Y_l, K x 2 n3 floats, i.e. 16 K n3 bytes per block, L = n1 n2 blocks. The gradient
    field, the overlap-add field and the kept eigenbases are this implementation's own
    traffic and are not counted."""
    L = n1 * n2
    K = k1 * k2
    return 16 * K * n3 * L


def block_pass_design_bytes(n1: int, n2: int, n3: int, k1: int, k2: int) -> int:
    """Bytes the fused block pass as designed moves per launch: the dual blocks read and
    written, the gradient field read (2 floats per voxel), the overlap-add field written
    (2 floats per voxel) and the stored 16 x 16 eigenbasis of every block read and written."""
    L = n1 * n2
    K = k1 * k2
    return 4 * L * (2 * K * 2 * n3 + 2 * n3 + 2 * n3 + 2 * 256)


def gram_flops(n1: int, n2: int, n3: int, k1: int, k2: int) -> int:
    """Flops of the block Gram products Y' Y'^T of one block pass: K x K outputs of length
    2 n3, two flops per product term, L = n1 n2 blocks."""
    K = k1 * k2
    return 2 * K * K * 2 * n3 * n1 * n2


MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}


def measured_counter(name: str, kernel: str):
    """A per-launch figure of `kernel` from the committed rocprofv3 counter summaries (lines
    `<name> <kernel> value=... source=... sha256_16=...`), or None when the kernel source has
    changed since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for line in fh:
                parts = line.split()
                if len(parts) < 4 or parts[0] != name or parts[1] != kernel:
                    continue
                kv = dict(p.split("=", 1) for p in parts[2:] if "=" in p)
                src = os.path.join(ROOT, kv.get("source", ""))
                if not os.path.isfile(src):
                    continue
                with open(src, "rb") as fs:
                    digest = hashlib.sha256(fs.read()).hexdigest()[:16]
                if digest == kv.get("sha256_16"):
                    return float(kv["value"]), os.path.relpath(path, ROOT)
    return None


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel source has changed since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_bytes_*.md"))):
        with open(path) as fh:
            for line in fh:
                parts = line.split()
                if len(parts) < 5 or parts[0] != "traffic" or parts[1] != kernel:
                    continue
                kv = dict(p.split("=", 1) for p in parts[2:] if "=" in p)
                src = os.path.join(ROOT, kv.get("source", ""))
                if not os.path.isfile(src):
                    continue
                with open(src, "rb") as fs:
                    digest = hashlib.sha256(fs.read()).hexdigest()[:16]
                if digest == kv.get("sha256_16"):
                    return int(kv["bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None


def iteration_algorithmic_bytes(n1: int, n2: int, n3: int, k1: int, k2: int) -> int:
    """(44 + 16K) bytes per voxel: u, s, t, y2, y3 read+written, v read, Y read+written."""
    N = n1 * n2 * n3
    return (44 + 16 * k1 * k2) * N


def cpu_baseline(d, k1, k2, iters: int, label: str = "256x256x128",
                 regularizer: str = "s3ttv") -> dict:
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    oracle.solve(d["v64"], k1, k2, max_iter=iters, regularizer=regularizer, **d["radii"])
    dt = time.perf_counter() - t0
    return {"value": iters / dt, "unit": "iters/s", "cores": oracle.get_threads(), "kind": "oracle",
            "sample": f"{iters} iteration(s) of the same {label} workload, FP64, "
                      f"{dt:.1f} s wall"}


FP32_VECTOR_PEAK_TFLOPS = 157.3
# The paper's running times of its own method on its three scenes (MATLAB on an Intel Core
# i9-13900 with an RTX 4090, averaged over its noise cases; Sec. IV, running-time table).
# Context only: another machine, real data, several noise cases.
PAPER_SECONDS_100x100x198 = 1.37e4
PAPER_SCENES = {"100x100x198": ("paper10", PAPER_SECONDS_100x100x198),
                "120x120x98": ("paper10_120x120x98", 2.05e4),
                "100x100x128": ("paper10_100x100x128", 1.74e4)}
# The same table's rows for the compared regularisers this library runs on the P-PDS
# skeleton (HSSTV in its l1 form, the paper's HSSTV1; STV and SSST with 10 x 10 blocks).
PAPER_SECONDS_COMPARED = {
    "sstv": {"100x100x198": 1.92e2, "120x120x98": 2.39e2, "100x100x128": 2.47e2},
    "hsstv": {"100x100x198": 2.03e2, "120x120x98": 2.05e2, "100x100x128": 1.81e2},
    "stv": {"100x100x198": 1.82e4, "120x120x98": 1.83e4, "100x100x128": 9.66e3},
    "ssst": {"100x100x198": 6.95e4, "120x120x98": 1.47e4, "100x100x128": 9.01e4},
}


def big_block_dense_flops(n3: int, K: int, nblk: int, eig_blocks: float,
                          sim_steps: float = 0.0) -> float:
    """FP32 flops of the dense products of one launch of the large-block pass: the symmetric
    Gram (K (K + 1) / 2 dot products of length 2 n3) of every block and, for the blocks that
    needed the eigen-solve, V^T G V and the Newton-Schulz step (four K x K x K products), the
    clip M Y' (a K x K x 2 n3 product) and, per simultaneous rotation step (`sim_steps` per
    such block on average), at least four K x K x K products (K^T K, V J and two for the
    rotated A). The cyclic Jacobi rotations, extra Newton-Schulz steps and the forming of M
    are not counted, so the figure is a lower bound on the work done."""
    c = 2 * n3
    return nblk * K * (K + 1) * c + eig_blocks * (8 * K ** 3 + 2 * K * K * c
                                                  + 8 * K ** 3 * sim_steps)


def bench_paper_shape(nt, synth, torch, args) -> int:
    """The paper's experimental shape: a 100 x 100 x 198 scene with 10 x 10 windows (K = 100),
    throughput over iterations that continue a solve from zero after a pre-roll (as the default
    workload: the clipping phase) and the time to the paper's stop rule (1e-5) from zero."""
    wname, paper_seconds = PAPER_SCENES[args.scene]
    reg = args.regularizer
    if reg != "s3ttv":
        paper_seconds = PAPER_SECONDS_COMPARED[reg][args.scene]
    l1_reg = reg in ("sstv", "hsstv")
    w = synth.WORKLOADS[wname]
    cfg = w["cfg"]
    k1, k2 = w["k"]
    n1, n2, n3 = cfg.n1, cfg.n2, cfg.n3
    print(f"[bench] generating {n1}x{n2}x{n3} workload, block {k1}x{k2}", file=sys.stderr,
          flush=True)
    d = synth.make_hsi(cfg)
    dev = torch.device("cuda:0")
    v = torch.from_numpy(d["v"]).to(dev)
    rad = d["radii"]
    solver = nt.Solver(n1, n2, n3, k1, k2, device=dev)
    first = args.preroll + max(args.warmup, 1)
    print(f"[bench] pre-roll {first} iterations from zero ({reg})", file=sys.stderr, flush=True)
    solver.solve(v, nt.make_params(max_iter=first, regularizer=reg, **rad))
    torch.cuda.synchronize()
    steps = args.paper_steps
    print(f"[bench] timed {steps} iterations (iterations {first + 1}-{first + steps})",
          file=sys.stderr, flush=True)
    cls = nt.K_DUAL if l1_reg else nt.K_BLOCK
    params = nt.make_params(max_iter=steps, timing_mask=1 << cls, regularizer=reg, **rad)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, st = solver.resume(v, params)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    name = nt.KERNEL_NAMES[cls]
    calls = st["kernel_calls"][name]
    if calls < 1:
        print(f"bench.py: the timed kernel ({name}) did not run", file=sys.stderr)
        return 3
    block_ms = st["kernel_ms"][name] / calls
    K = k1 * k2
    if l1_reg:
        # no block pass: the dual sweep is the largest pass (as in the default workload)
        dbytes = n1 * n2 * n3 * (52 + 16 * (2 if reg == "hsstv" else 1))
        achieved = dbytes / (block_ms * 1e-3) / 1e9
        roofline = {"kernel": "k_dual_grad", "bound": "hbm", "achieved": achieved,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "traffic": None, "avg_launch_ms": block_ms, "launches_timed": calls,
                    "algorithmic_bytes_per_launch": dbytes}
    else:
        flops = big_block_dense_flops(n3, K, n1 * n2, st["eig_blocks"] / calls,
                                      st["eig_avg_sweeps"])
        achieved = flops / (block_ms * 1e-3) / 1e12
        # the dense products run on v_mfma_f32_16x16x4_f32, whose peak is the FP32 one; the
        # matrix pipe's busy fraction comes from the committed counter summary of the S3TTV run
        busy = measured_counter("mfma_busy_frac", "k_big_block") if reg == "s3ttv" else None
        # HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary of this scene
        traffic = (measured_traffic("k_big_block")
                   if reg == "s3ttv" and args.scene == "100x100x198" else None)
        roofline = {"kernel": "k_big_block", "bound": "mfma", "achieved": achieved,
                    "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                    "traffic": traffic[0] if traffic else None,
                    "traffic_source": traffic[1] if traffic else None,
                    "avg_launch_ms": block_ms, "launches_timed": calls,
                    "dense_flops_per_launch": flops,
                    "launch_mfma_busy_frac": busy[0] if busy else None,
                    "busy_source": busy[1] if busy else None}
    out = {
        "metric": f"P-PDS iters/sec + time to the stop rule 1e-5, {n1}x{n2}x{n3} HSI, block 10x10",
        "value": steps / wall,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{reg.upper()} P-PDS, synthetic HSI {n1}x{n2}x{n3}, block "
                               f"{k1}x{k2} (K = {K}), sigma {cfg.sigma}, salt-and-pepper "
                               f"{cfg.p_sp}, stripes {cfg.p_stripe} (offsets in +-{cfg.stripe_amp})",
                   "n1": n1, "n2": n2, "n3": n3, "k1": k1, "k2": k2, "seed": cfg.seed,
                   "regularizer": reg},
        "roofline": roofline,
        "timed_iterations": [first + 1, first + steps],
        "eig_blocks_per_launch": st["eig_blocks"] / calls,
        "eig_sim_steps_per_solved_block": st["eig_avg_sweeps"],
        "eig_avg_sweeps_per_solved_block": st["eig_avg_steps"],
        "eig_max_sweeps": st["eig_max_sweeps"],
        "eig_uncertified_blocks": st["eig_fallback_blocks"],
    }
    if not args.skip_tol:
        tol = w["rel_tol"]
        print(f"[bench] time to the stop rule {tol} (cap {args.tol_cap})", file=sys.stderr,
              flush=True)
        p2 = nt.make_params(max_iter=args.tol_cap, rel_tol=tol, check_every=32, regularizer=reg,
                            **rad)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, st2 = solver.solve(v, p2)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        out["time_to_rel_tol"] = {"tol": tol, "seconds": secs, "iters": st2["iters"],
                                  "converged": st2["converged"],
                                  "uncertified_blocks": st2["eig_fallback_blocks"]}
        out["paper_context"] = {"seconds": paper_seconds,
                                "what": f"the paper's implementation of {reg.upper()} on its "
                                        f"{n1}x{n2}x{n3} scene (CPU + RTX 4090), averaged over "
                                        "noise cases",
                                "ratio_paper_over_this": paper_seconds / secs}
    if not args.skip_cpu:
        print("[bench] CPU oracle baseline (2 iterations)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(d, k1, k2, 2, label=f"{n1}x{n2}x{n3}, block 10x10",
                                           regularizer=reg)
    print(json.dumps(out), flush=True)
    return 0


def bench_batched(nt, synth, torch, prec) -> int:
    """The uneven batch: 24 images solved to rel-tol 1e-4 in one batched call, against the
    same 24 solved one after another with s3ttv_solve; results must be identical."""
    import numpy as np
    dev = torch.device("cuda:0")
    cfgs = synth.batch_configs()
    probs = []
    for i, cfg in enumerate(cfgs):
        print(f"[bench] image {i}: {cfg.n1}x{cfg.n2}x{cfg.n3}", file=sys.stderr, flush=True)
        d = synth.make_hsi(cfg)
        prm = nt.make_params(max_iter=20000, rel_tol=1e-4, check_every=32, gram_precision=prec,
                             **d["radii"])
        probs.append(dict(v=torch.from_numpy(d["v"]).to(dev), k1=4, k2=4, params=prm))
    ws = nt._workspace(nt.batch_workspace_bytes([(*p["v"].shape, 4, 4) for p in probs]), dev)
    print("[bench] batched warm-up (tile tuning)", file=sys.stderr, flush=True)
    warm = [dict(p, params=nt.make_params(max_iter=2, **{k: getattr(p["params"], k) for k in
                                                        ("eps", "alpha", "beta")}))
            for p in probs]
    nt.solve_batched(warm, workspace=ws)
    torch.cuda.synchronize()
    print("[bench] batched solve", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    res, rc = nt.solve_batched(probs, workspace=ws)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    print("[bench] sequential solves", file=sys.stderr, flush=True)
    seq = []
    t0 = time.perf_counter()
    for p in probs:
        n1, n2, n3 = p["v"].shape
        seq.append(nt.Solver(n1, n2, n3, 4, 4, device=dev).solve(p["v"], p["params"]))
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    same = all(np.array_equal(a.cpu().numpy(), b.cpu().numpy())
               for r, q in zip(res, seq) for a, b in zip(r[:3], q[:3]))
    iters = [r[3]["iters"] for r in res]
    voxels = sum(int(np.prod(p["v"].shape)) for p in probs)
    out = {
        "metric": "batched S3TTV solve to rel-tol 1e-4, 24 uneven synthetic HSIs, one GPU",
        "value": t_batch, "unit": "s", "n_gpus": 1, "steps": sum(iters), "warmup": 1,
        "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == nt.GRAM_FP32 else "f32 (reduced-precision Gram inputs)",
        "data": "synthetic",
        "config": {"workload": "24 images, N1,N2 ~ U{64..307}, N3 ~ U{32..191}, block 4x4, "
                               "noise rates from {0.05, 0.1}, seed 4",
                   "voxels": voxels, "images": len(probs)},
        "sequential_s": t_seq, "speedup_vs_sequential": t_seq / t_batch,
        "identical_to_standalone": same, "converged": sum(r[3]["converged"] for r in res),
        "iterations_min_max": [min(iters), max(iters)],
        "tiles": sorted({tuple(r[3]["tile"]) for r in res}),
    }
    print(json.dumps(out), flush=True)
    return 0 if same else 4


def bench_warm_start(nt, synth, torch, args) -> int:
    """The learned initial estimate: the network is trained on the GPU on seeded 64^3 scenes
    whose targets the batched solver computes (rel-tol 1e-5), then the 512 x 512 x 191 scene
    is solved to rel-tol 1e-4 from zero and from the network's estimate. A tighter solve of
    the same scene (rel-tol 1e-6) is the yardstick for both results."""
    import numpy as np
    from paper_2404_03313_amd import warmstart as ws
    dev = torch.device("cuda:0")

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    V, U, pair_iters = ws.make_pairs(synth.cnn_train_configs(count=args.pairs), rel_tol=1e-5,
                                     max_iter=3000, log=log)
    t_pairs = time.perf_counter() - t0
    ident = float(((V - U) ** 2).mean())
    tr = ws.Trainer(synth.cnn_init(0), device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = tr.train(V, U, steps=args.train_steps, batch=8, lr=1e-3, log=log, log_every=250)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del V, U
    torch.cuda.empty_cache()

    w = synth.WORKLOADS["c5"]
    cfg, (k1, k2), tol = w["cfg"], w["k"], w["rel_tol"]
    log(f"scene {cfg.n1}x{cfg.n2}x{cfg.n3}")
    d = synth.make_hsi(cfg)
    v = torch.from_numpy(d["v"]).to(dev)
    sv = nt.Solver(cfg.n1, cfg.n2, cfg.n3, k1, k2, device=dev)
    sv.solve(v, nt.make_params(max_iter=2, **d["radii"]))   # first-launch set-up, untimed
    log("cold and warm solves")
    r = ws.solve_cold_warm(v, d["radii"], tr.params, k=(k1, k2), rel_tol=tol,
                           max_iter=args.tol_cap, solver=sv)
    log("observation as the start (u0 = v)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    triv = sv.solve(v, nt.make_params(max_iter=args.tol_cap, rel_tol=tol, **d["radii"]), u0=v)
    torch.cuda.synchronize()
    t_triv = time.perf_counter() - t0
    triv = tuple(x.clone() for x in triv[:3]) + (triv[3],)
    log("reference solve (rel-tol 1e-6)")
    ref = sv.solve(v, nt.make_params(max_iter=args.ref_iters, rel_tol=1e-6, check_every=64,
                                     **d["radii"]))
    uref = ref[0].clone()

    def dist(a, b):
        return float((a - b).norm() / b.norm())

    early = {}
    for name, u0 in (("cold", None), ("warm", r["u0"]), ("u0=v", v)):
        ue = sv.solve(v, nt.make_params(max_iter=100, **d["radii"]), u0=u0)[0]
        early[name] = dist(ue, uref)

    # iterations the warm start needs to be as close to the reference as the cold result:
    # first doubling budget that gets there, refined by bisection (P-PDS iterates do not
    # approach the solution monotonically, so this is the first such budget on that grid)
    log("iterations of the warm start to the cold result's accuracy")
    target = dist(r["cold"][0], uref)

    def warm_at(k):
        return dist(sv.solve(v, nt.make_params(max_iter=k, **d["radii"]), u0=r["u0"])[0], uref)

    hi = 50
    while hi < 4 * r["cold"][3]["iters"] and warm_at(hi) > target:
        hi *= 2
    lo = hi // 2
    for _ in range(4):
        mid = (lo + hi) // 2
        if mid <= lo:
            break
        if warm_at(mid) <= target:
            hi = mid
        else:
            lo = mid
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nt.cnn_forward(tr.params, v)
    sv.solve(v, nt.make_params(max_iter=hi, **d["radii"]), u0=r["u0"])
    torch.cuda.synchronize()
    t_match = time.perf_counter() - t0

    cold, warm = r["cold"], r["warm"]
    keys = ("fid", "l1_s", "l1_t", "dv_t")
    out = {
        "metric": "P-PDS time to rel-tol 1e-4, 512×512×191 HSI, learned warm start vs zero start",
        "value": r["t_warm"], "unit": "s", "n_gpus": 1, "steps": warm[3]["iters"], "warmup": 1,
        "ms_per_step": 1e3 * r["t_warm"] / max(warm[3]["iters"], 1), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (network: bf16 weights)",
        "data": "synthetic",
        "config": {"workload": f"S3TTV P-PDS, synthetic HSI {cfg.n1}x{cfg.n2}x{cfg.n3}, "
                               f"sigma {cfg.sigma}, salt-and-pepper {cfg.p_sp}, stripes "
                               f"{cfg.p_stripe}, block {k1}x{k2}, rel-tol {tol}, seed {cfg.seed}"},
        "cold": {"s": r["t_cold"], "iters": cold[3]["iters"],
                 "converged": cold[3]["converged"], **{k: cold[3][k] for k in keys}},
        "warm": {"s": r["t_warm"], "iters": warm[3]["iters"], "network_ms": 1e3 * r["t_net"],
                 "converged": warm[3]["converged"], **{k: warm[3][k] for k in keys}},
        "u0_is_v": {"s": t_triv, "iters": triv[3]["iters"], "converged": triv[3]["converged"],
                    **{k: triv[3][k] for k in keys}},
        "warm_to_cold_accuracy": {"target_rel_l2": target, "iters": hi, "s": t_match,
                                  "speedup_time": r["t_cold"] / t_match,
                                  "speedup_iters": cold[3]["iters"] / hi},
        "speedup_time": r["t_cold"] / r["t_warm"],
        "speedup_iters": cold[3]["iters"] / max(warm[3]["iters"], 1),
        "warm_start_result": (
            "gain: the learned start needs fewer iterations to the stop rule than the zero start"
            if warm[3]["iters"] < cold[3]["iters"] else
            "regression: the learned start needs at least as many iterations to the stop rule "
            "as the zero start"),
        "rel_l2_warm_vs_cold": dist(warm[0], cold[0]),
        "reference": {"rel_tol": 1e-6, "iters": ref[3]["iters"], "converged": ref[3]["converged"],
                      "rel_l2_cold": dist(cold[0], uref), "rel_l2_warm": dist(warm[0], uref),
                      "rel_l2_u0_is_v": dist(triv[0], uref),
                      "rel_l2_estimate": dist(r["u0"], uref), "rel_l2_observation": dist(v, uref),
                      "rel_l2_after_100_iterations": early},
        "training": {"pairs": args.pairs, "pair_shape": [64, 64, 64], "pair_rel_tol": 1e-5,
                     "pair_iters_mean": float(np.mean(pair_iters)), "pair_s": t_pairs,
                     "steps": args.train_steps, "batch": 8, "train_s": t_train,
                     "ms_per_step": 1e3 * t_train / max(args.train_steps, 1),
                     "loss_identity": ident, "loss_final": float(np.mean(losses[-100:]))},
    }
    print(json.dumps(out), flush=True)
    return 0


CNN_FLOP_PER_VOXEL = 2 * 27 * (32 + 3 * 32 * 32 + 32)   # forward: 1->32, 3 x 32->32, 32->1


def bench_cnn(nt, synth, torch, args) -> int:
    """Network kernels alone: Adam steps at batch 8 x 64^3 and the forward pass over the
    512 x 512 x 191 scene, timed with events on the stream the kernels run on."""
    import numpy as np
    dev = torch.device("cuda:0")
    rng = np.random.Generator(np.random.PCG64(7))
    v = torch.from_numpy(rng.uniform(0, 1, size=(8, 64, 64, 64)).astype(np.float32)).to(dev)
    tgt = (v + 0.05 * torch.randn(v.shape, generator=torch.Generator(device=dev).manual_seed(8),
                                  device=dev)).contiguous()
    params = torch.from_numpy(synth.cnn_init(0)).to(dev)
    m, v2 = torch.zeros_like(params), torch.zeros_like(params)
    ws = nt._workspace(nt.cnn_workspace_bytes(v.shape, True), dev)
    for k in range(1, args.warmup + 1):
        nt.cnn_train_step(params, m, v2, k, 1e-3, v, tgt, workspace=ws)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for k in range(args.warmup + 1, args.warmup + args.steps + 1):
        nt.cnn_train_step(params, m, v2, k, 1e-3, v, tgt, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / args.steps
    cfg = synth.WORKLOADS["c5"]["cfg"]
    big = torch.from_numpy(rng.uniform(0, 1, size=(cfg.n1, cfg.n2, cfg.n3)).astype(np.float32)).to(dev)
    wsb = nt._workspace(nt.cnn_workspace_bytes(big.shape, False), dev)
    out = torch.empty_like(big)
    nt.cnn_forward(params, big, out=out, workspace=wsb)
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        e0.record()
        nt.cnn_forward(params, big, out=out, workspace=wsb)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    fwd_ms = min(times)
    nvox = big.numel()
    achieved = CNN_FLOP_PER_VOXEL * nvox / (fwd_ms * 1e-3) / 1e12
    res = {
        "metric": "initial-estimate network: Adam step (batch 8 x 64^3) and forward (512x512x191)",
        "value": 1e3 / step_ms, "unit": "train steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (fp32 sums)", "data": "synthetic",
        "config": {"workload": "CNN 1-32-32-32-32-1, 3x3x3, train batch 8 x 64^3, forward "
                               f"{cfg.n1}x{cfg.n2}x{cfg.n3}"},
        "forward_ms": fwd_ms,
        "roofline": {"kernel": "whole forward pass (dominated by k_cnn_conv32<0>)",
                     "bound": "mfma", "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": achieved / 2500.0, "traffic": None,
                     "flop_per_voxel": CNN_FLOP_PER_VOXEL},
    }
    print(json.dumps(res), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--skip-tol", action="store_true", help="skip the time-to-tolerance solve")
    ap.add_argument("--skip-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tol-cap", type=int, default=20000)
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--workload", choices=["c2", "c4", "c5", "cnn", "paper10"], default="c2",
                    help="c2: the single 256x256x128 image (default); c4: the uneven batch of 24; "
                         "c5: learned initial estimate vs zero start on 512x512x191; cnn: the "
                         "network kernels alone; paper10: the paper's 100x100x198 shape with "
                         "10x10 windows")
    ap.add_argument("--paper-steps", type=int, default=100,
                    help="paper10: timed iterations (continuing a solve after the pre-roll)")
    ap.add_argument("--scene", choices=sorted(PAPER_SCENES), default="100x100x198",
                    help="paper10: the shape of one of the paper's scenes")
    ap.add_argument("--regularizer", choices=["s3ttv", "stv", "sstv", "hsstv", "ssst"],
                    default="s3ttv",
                    help="c2, paper10: term minimised on the P-PDS skeleton (S3TTV is the paper's)")
    ap.add_argument("--pairs", type=int, default=2000, help="c5: training pairs (64^3 scenes)")
    ap.add_argument("--train-steps", type=int, default=2500, help="c5: Adam steps (batch 8)")
    ap.add_argument("--ref-iters", type=int, default=10000,
                    help="c5: iteration cap of the rel-tol 1e-6 reference solve")
    ap.add_argument("--gram-precision", choices=["fp32", "bf16", "fp16"], default="fp32",
                    help="input precision of the block Gram products (accumulation stays FP32)")
    ap.add_argument("--preroll", type=int, default=200,
                    help="c2: iterations from zero run before the warm-up and timed ones (the "
                         "timed iterations continue that solve)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}); the solver is a "
              "single-GPU library", file=sys.stderr)
        return 2

    import numpy as np  # noqa: F401
    import torch

    from paper_2404_03313_amd import native as nt
    from paper_2404_03313_amd import synth

    prec = {"fp32": nt.GRAM_FP32, "bf16": nt.GRAM_BF16, "fp16": nt.GRAM_FP16}[args.gram_precision]
    if args.workload == "c4":
        return bench_batched(nt, synth, torch, prec)
    if args.workload == "c5":
        return bench_warm_start(nt, synth, torch, args)
    if args.workload == "cnn":
        return bench_cnn(nt, synth, torch, args)
    if args.workload == "paper10":
        return bench_paper_shape(nt, synth, torch, args)
    w = synth.WORKLOADS["c2"]
    cfg = w["cfg"]
    k1, k2 = w["k"]
    n1, n2, n3 = cfg.n1, cfg.n2, cfg.n3
    print(f"[bench] generating {n1}x{n2}x{n3} workload", file=sys.stderr, flush=True)
    d = synth.make_hsi(cfg)
    dev = torch.device("cuda:0")
    v = torch.from_numpy(d["v"]).to(dev)
    solver = nt.Solver(n1, n2, n3, k1, k2, device=dev)
    rad = d["radii"]

    reg = args.regularizer
    l1_reg = reg in ("sstv", "hsstv")
    # The timed iterations continue a solve from zero after `preroll` iterations (plus the
    # warm-up ones), so that they are iterations of the clipping phase that makes up almost
    # all of a solve to tolerance (from zero no block clips for the first ~30 iterations).
    first = args.preroll + max(args.warmup, 1)
    print(f"[bench] pre-roll {args.preroll} + warmup {args.warmup} iterations from zero",
          file=sys.stderr, flush=True)
    solver.solve(v, nt.make_params(max_iter=first, gram_precision=prec, regularizer=reg, **rad))
    torch.cuda.synchronize()

    print(f"[bench] timed {args.steps} iterations (iterations {first + 1}-{first + args.steps})",
          file=sys.stderr, flush=True)
    # blocks of at most 16 rows and 24 column tiles take the fused block pass; more columns
    # (SSST's three components at N3 > 128) the separate Gram / eigen / apply kernels
    comps = 3 if reg == "ssst" else 2
    bq = 32 if comps == 3 else 16
    fused = k1 * k2 <= 16 and comps * ((n3 + bq - 1) // bq * bq) <= 384
    if l1_reg:
        classes = [nt.K_DUAL]
    elif fused:
        classes = [nt.K_BLOCK]
    else:
        classes = [nt.K_GRAM, nt.K_EIG, nt.K_APPLY]
    cls = classes[0]
    params = nt.make_params(max_iter=args.steps, timing_mask=sum(1 << c for c in classes),
                            gram_precision=prec, regularizer=reg, **rad)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, s, t, st = solver.resume(v, params)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = args.steps / wall
    name = nt.KERNEL_NAMES[cls]
    block_calls = st["kernel_calls"][name]
    if block_calls < 1:
        print(f"bench.py: the timed kernel ({name}) did not run", file=sys.stderr)
        return 3
    # average time of the pass per iteration (the separate route: its three kernels together)
    block_ms = sum(st["kernel_ms"][nt.KERNEL_NAMES[c]] for c in classes) / block_calls
    design_bytes = None
    if l1_reg:
        # the dual sweep is the largest pass of the l1 variants: 36 B read and 16 B written per
        # voxel for the vector duals and s, t, plus the l1 dual field(s) read and written
        kname = "k_dual_grad"
        block_bytes = n1 * n2 * n3 * (52 + 16 * (2 if reg == "hsstv" else 1))
    else:
        kname = "k_block_fused" if fused else "k_gram + k_eig + k_apply"
        # steps 9-10 read and write every block once: K x comps N3 floats
        block_bytes = block_pass_algorithmic_bytes(n1, n2, n3, k1, k2) * comps // 2
        design_bytes = block_pass_design_bytes(n1, n2, n3, k1, k2) if comps == 2 and fused else None
    achieved = block_bytes / (block_ms * 1e-3) / 1e9

    traffic = measured_traffic(kname) if reg == "s3ttv" and fused else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.gram_precision == "fp32" else f"f32 ({args.gram_precision} Gram inputs)",
        "data": "synthetic",
        "config": {"workload": f"{reg.upper()} P-PDS, synthetic HSI {n1}x{n2}x{n3}, block {k1}x{k2}, "
                               f"sigma {cfg.sigma}, salt-and-pepper {cfg.p_sp}, stripes {cfg.p_stripe}",
                   "n1": n1, "n2": n2, "n3": n3, "k1": k1, "k2": k2, "seed": cfg.seed,
                   "gram_precision": args.gram_precision, "regularizer": reg},
        "loop_ms_per_step": st["ms"] / args.steps,
        "iteration_algorithmic_bytes": (None if l1_reg
                                        else iteration_algorithmic_bytes(n1, n2, n3, k1, k2)),
        "roofline": {"kernel": kname, "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic[0] if traffic else None, "avg_launch_ms": block_ms,
                     "launches_timed": block_calls,
                     "algorithmic_bytes_per_launch": block_bytes,
                     "design_bytes_per_launch": design_bytes,
                     "traffic_source": traffic[1] if traffic else None},
        "timed_iterations": [first + 1, first + args.steps],
        "eig_max_sweeps": st["eig_max_sweeps"],
        "eig_avg_sweeps": st["eig_avg_sweeps"],
        "eig_avg_steps": st["eig_avg_steps"],
        "eig_max_steps": st["eig_max_steps"],
        "eig_fallback_blocks": st["eig_fallback_blocks"],
    }
    if not l1_reg:
        # MFMA use of the Gram stage: the Gram flops of a launch over the whole block-pass time
        # (the stage shares the launch with the eigen-solve, the clip and the overlap-add, so
        # this is a lower bound of the stage's own rate), and the matrix-pipe busy fraction of
        # the whole launch from the committed counter summary while the source is unchanged
        gf = gram_flops(n1, n2, n3, k1, k2) * comps // 2
        busy = measured_counter("mfma_busy_frac", kname) if reg == "s3ttv" and fused else None
        peak = MFMA_PEAK_TFLOPS[args.gram_precision]
        out["gram_mfma"] = {"flops_per_launch": gf, "achieved_tflops": gf / (block_ms * 1e-3) / 1e12,
                            "peak_tflops": peak,
                            "frac": gf / (block_ms * 1e-3) / 1e12 / peak,
                            "launch_mfma_busy_frac": busy[0] if busy else None,
                            "busy_source": busy[1] if busy else None}

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        dst.copy_(src)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        out["copy_probe"] = {"bytes_each_way": src.numel() * 4, "ms": ms,
                             "GBps_read_plus_write": 2 * src.numel() * 4 / (ms * 1e-3) / 1e9}
        del src, dst

    if not args.skip_tol:
        print(f"[bench] time to rel-tol 1e-4 (cap {args.tol_cap})", file=sys.stderr, flush=True)
        p2 = nt.make_params(max_iter=args.tol_cap, rel_tol=1e-4, check_every=32,
                            gram_precision=prec, regularizer=reg, **rad)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, st2 = solver.solve(v, p2)
        torch.cuda.synchronize()
        out["time_to_rel_tol"] = {"tol": 1e-4, "seconds": time.perf_counter() - t0,
                                  "iters": st2["iters"], "converged": st2["converged"]}

    if not args.skip_cpu:
        print(f"[bench] CPU oracle baseline ({args.cpu_iters} iteration(s))", file=sys.stderr,
              flush=True)
        out["cpu_baseline"] = cpu_baseline(d, k1, k2, args.cpu_iters)

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
