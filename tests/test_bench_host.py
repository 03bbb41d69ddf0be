"""Host-side logic of bench.py (no GPU): the roofline's slot model, the match between the committed
HBM counter summaries and the kernel source they were taken on, and the one-GPU guard."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_min_slots_model():
    # C2: dim subtractions + dim FMAs for r^2 + 4 for the quarter-rate root + 1 - eta, max, t^2,
    # t^4, 4 eta + 1, product (6) + dim accumulating FMAs.
    assert bench.min_slots(2, "c2", "fp64") == 2 + 2 + 4 + 6 + 2 + 1
    assert bench.min_slots(3, "c2", "fp64") == 3 + 3 + 4 + 6 + 3 + 1
    assert bench.min_slots(2, "c2", "mixed") == bench.min_slots(2, "c2", "fp64") + 1
    order = [bench.min_slots(3, b, "fp64") for b in ("c0", "c2", "c4", "c6")]
    assert order == sorted(order)
    # The peak in pairs/s is the lane-slot rate over the slots per pair.
    assert bench.VALU_LANE_OPS == pytest.approx(256 * 64 * 2.4e9)
    assert bench.VALU_LANE_OPS / bench.min_slots(2, "c2", "fp64") / 1e9 == pytest.approx(2313.035, rel=1e-6)


@pytest.mark.parametrize("workload,precision", [("cfg1", "fp64"), ("cfg1", "mixed"), ("cfg2", "fp64")])
def test_committed_traffic_matches_current_kernel(workload, precision):
    """The committed counter summaries were taken on the kernel source as it stands, so the bench
    reports their traffic, which lies within a factor 1.5 of the launch's algorithmic bytes
    (prefix rows x (dim + 1) x 8 + 4 read, all stored rows x dim x 8 written, the rest 4 B read)."""
    path = os.path.join(ROOT, "profiles", f"traffic_volume_ksum_{workload}_{precision}.txt")
    text = open(path).read()
    assert f"ksum_source_sha256_16: {bench.kernel_source_hash()}" in text
    dim, n_red, n_rows = {"cfg1": (2, 244584, 400384), "cfg2": (3, 2542809, 4002304)}[workload]
    algo = n_red * ((dim + 1) * 8 + 4) + (n_rows - n_red) * 4 + n_rows * dim * 8
    t = bench.measured_traffic(workload, precision)
    assert t is not None and algo / 1.5 < t < algo * 1.5


def test_traffic_dropped_for_another_kernel_source(tmp_path, monkeypatch):
    """A change to the code of the kernel-sum device sources (not to their comments) drops the
    traffic."""
    csrc = tmp_path / "paper_2107_13887_amd" / "csrc"
    csrc.mkdir(parents=True)
    shutil.copytree(os.path.join(ROOT, "profiles"), tmp_path / "profiles")
    for name in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2107_13887_amd", "csrc", name), csrc / name)
    src = open(os.path.join(ROOT, "paper_2107_13887_amd", "csrc", "ksum.hip")).read()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))

    (csrc / "ksum.hip").write_text("// another comment\n/* and a block\n comment */\n" + src + "\n\n")
    assert bench.measured_traffic("cfg1", "fp64") is not None

    (csrc / "ksum.hip").write_text(src.replace("__launch_bounds__(BLOCK)", "__launch_bounds__(BLOCK, 2)", 1))
    assert bench.measured_traffic("cfg1", "fp64") is None
    assert bench.measured_traffic("no_such_workload", "fp64") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_in_support_pair_count_is_exact():
    """The headline's work count: pairs of a reduced volume point (d < D_l) and a control of the
    same level within its support radius (||x - x_c|| < R_l), equal to a brute-force count."""
    import numpy as np

    import synth

    w = synth.random_workload(3, 3, 200, 5000, [1.0, 0.4], 1e-6)
    rng = np.random.default_rng(0)
    xc = rng.uniform(-1, 1, (3, 50))
    off, R, D = [0, 20, 50], [1.0, 0.4], [1.2, 0.8]
    total, per = bench.in_support_pairs(w, R, D, off, xc)
    want = []
    for l in range(2):
        pts = w.xv[:, w.dwall < D[l]]
        d = np.sqrt(((pts[:, :, None] - xc[:, None, off[l]:off[l + 1]]) ** 2).sum(0))
        want.append(int((d < R[l]).sum()))
    assert per == want and total == sum(want)
    # a control exactly one radius away from a point is outside the support (phi = 0 there)
    w.xv[:, 0] = xc[:, 0] + np.array([R[0], 0.0, 0.0])
    w.dwall[0] = 0.0
    pts = w.xv[:, w.dwall < D[0]]
    d = np.sqrt(((pts[:, :, None] - xc[:, None, :20]) ** 2).sum(0))
    assert bench.in_support_pairs(w, R, D, off, xc)[1][0] == int((d < R[0]).sum())
