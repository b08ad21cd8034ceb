"""The defaults of the oracle, the synthetic workloads and the bench against the values the
paper prints (fixture: tests/golden/paper_settings.json, each group with its citation).
CPU only."""
import json
import os
from fractions import Fraction

import oracle
from paper_2404_03313_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    with open(os.path.join(HERE, "golden", "paper_settings.json")) as fh:
        return json.load(fh)


def test_default_step_sizes_are_the_printed_ones():
    """eq. stepsize_denoising: gamma_s = 1, gamma_t = 1/3, gamma_Y = 1/4, gamma_y2 = 1/2,
    gamma_y3 = 1/3 exactly; gamma_u is printed as 1/(8L+1) and taken as 1/(8K+1) with K the
    block rows (the Lemma-2 column sum of the stacked operator), which is the printed value
    when L = K and a larger admissible step otherwise."""
    g = _golden()["step_sizes"]
    for k1, k2 in [(10, 10), (4, 4), (3, 2)]:
        d = oracle.default_gammas(k1, k2)
        for name in ("gamma_s", "gamma_t", "gamma_Y", "gamma_y2", "gamma_y3"):
            num, den = g[name]
            assert Fraction(d[name]).limit_denominator(1000) == Fraction(num, den), name
        K = k1 * k2
        assert d["gamma_u"] == 1.0 / (8 * K + 1)
        assert g["gamma_u"] == "1/(8L+1)"


def test_experiment_settings():
    """Sec. IV-A: 10 x 10 blocks, rho = 0.95 in eq. RadiusSet, stop rule 1e-5 and the HSSTV
    weight 0.05 are the defaults of the paper-shaped workload, the generator and the oracle."""
    e = _golden()["experiments"]
    w = synth.WORKLOADS["paper10"]
    assert list(w["k"]) == e["block"]
    assert w["rel_tol"] == e["stop_tol"]
    cfg = w["cfg"]
    assert [cfg.n1, cfg.n2, cfg.n3] == e["jasper_ridge_shape"]
    assert synth.HSIConfig(4, 4, 4).rho == e["rho"]
    d_default = oracle.default_gammas(2, 2, "hsstv")
    d_given = oracle.default_gammas(2, 2, "hsstv", e["hsstv_omega"])
    assert d_default == d_given


def test_bench_context_is_the_printed_running_time():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(HERE, "..", "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    t = _golden()["running_time_s3ttv_seconds"]
    assert bench.PAPER_SECONDS_100x100x198 == t["jasper_ridge"]
    assert bench.PAPER_SCENES["120x120x98"][1] == t["pavia_university"]
    assert bench.PAPER_SCENES["100x100x128"][1] == t["beltsville"]
    c = _golden()["running_time_compared_seconds"]
    scene = {"100x100x198": "jasper_ridge", "120x120x98": "pavia_university",
             "100x100x128": "beltsville"}
    for reg, key in (("sstv", "sstv"), ("hsstv", "hsstv1"), ("stv", "stv")):
        for shape, name in scene.items():
            assert bench.PAPER_SECONDS_COMPARED[reg][shape] == c[key][name], (reg, shape)
    for name, (wname, _) in bench.PAPER_SCENES.items():
        cfg = synth.WORKLOADS[wname]["cfg"]
        assert f"{cfg.n1}x{cfg.n2}x{cfg.n3}" == name
        assert list(synth.WORKLOADS[wname]["k"]) == _golden()["experiments"]["block"]
