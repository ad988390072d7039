"""Host-side logic of bench.py: the one-GPU guard and the algorithmic flop
count of the condensation the roofline line is priced with."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_condense_flops_24cubed():
    sys.path.insert(0, ROOT)
    import bench
    cfg = dict(dim=3, p=2, m=3)
    n_u, n_b = 1715, 1470
    lu = 2.0 / 3.0 * n_u ** 3
    schur = 2.0 * n_u ** 2 * n_b + 2.0 * n_b ** 2 * n_u
    # formation: 2 d n_s^2 (p+1)^(2d) per (node, element) pair and twice that per trace row
    form = 2 * 3 * 25 * 3 ** 6 * 343 * 27 + 4 * 3 * 25 * 3 ** 6 * (n_b / 5) * 27
    f = bench.condense_flops(cfg, n_u, n_b)
    assert f == pytest.approx(lu + schur + form, rel=1e-12)
    # 2.22e10 per macro, 1.135e13 for the 512 macros of the workload
    assert f == pytest.approx(2.217e10, rel=2e-3)
    assert 512 * f == pytest.approx(1.135e13, rel=2e-3)


def test_condense_flops_48cubed_headline():
    """The headline workload (48^3, 4^3-element macros, p = 2): n_u = 3645,
    n_b = 2430 per macro, 1.52e11 flop per macro, 2.62e14 per condensation of
    the 1728 macros."""
    sys.path.insert(0, ROOT)
    import bench
    cfg = dict(dim=3, p=2, m=4)
    n_u, n_b = 5 * 9 ** 3, 5 * 6 * 9 ** 2
    assert (n_u, n_b) == (3645, 2430)
    f = bench.condense_flops(cfg, n_u, n_b)
    assert f == pytest.approx(1.52e11, rel=5e-3)
    assert 1728 * f == pytest.approx(2.62e14, rel=5e-3)


def test_cpu_baseline_leg_on_the_small_2d_workload():
    """The oracle leg of the bench (host only): phases present, positive,
    scaled to the mesh, and the sampled condensed block returned for the
    error against the GPU."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2402_11361_amd import inputs
    cfg = dict(inputs.CONFIGS["shear16_m4_p2"])
    out, blocks = bench.cpu_baseline(cfg, dict(outer_its=10, applies=60), n_sample=1)
    assert out["kind"] == "oracle" and out["value"] > 0 and out["cores"] >= 1
    for k in ("condense", "backsolve", "apply", "krylov_vectors"):
        assert out["phases_ms"][k] >= 0
    assert out["linearisation_not_a_fair_baseline"]["ms_per_macro"] > 0
    A, b = blocks[0]
    assert A.shape == (b.size, b.size) and abs(A).max() > 0
