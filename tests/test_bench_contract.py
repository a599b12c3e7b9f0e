"""Host-side checks of the benchmark script (no GPU): the single-GPU guard, the
algorithmic byte counts behind the roofline, and that the committed counter
profile still matches the dslash sources it was taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_device_call():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    out = json.loads(p.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_algorithmic_dslash_bytes():
    V = 16 ** 3 * 32
    # every spinor read and written once (96 B FP32 per site-RHS each way), every link once (4 x 72 B)
    assert bench.dslash_bytes(V, 48, 1) == V * (2 * 96 * 48 + 4 * 9 * 8)
    assert bench.dslash_bytes(V, 48, 1) == 1245708288
    assert bench.dslash_bytes(V, 10, 0) == V * (2 * 192 * 10 + 4 * 9 * 16)
    # FP16S: 12 half2 values plus one float scale per site-RHS, half links
    assert bench.dslash_bytes(V, 12, 2) == V * (2 * (12 * 4 + 4) * 12 + 4 * 9 * 4)


def test_counter_profile_traffic_is_reported_only_for_the_profiled_kernel():
    """The roofline's measured traffic comes from the committed FETCH_SIZE /
    WRITE_SIZE profile of the 64-RHS smoother dslash at 32^4, and only while the
    dslash sources hash to the value recorded with the counters."""
    if not os.path.exists(bench.PROFILE):
        assert bench.measured_traffic() is None
        return
    with open(bench.PROFILE) as f:
        rec = json.load(f)
    assert rec["algorithmic_bytes_per_launch"] == bench.dslash_bytes(32 ** 4, 64, 1)
    t = bench.measured_traffic()
    if rec["kernel_source_sha256"] == bench.kernel_source_hash():
        assert t is not None and t >= 0.9 * rec["algorithmic_bytes_per_launch"]
    else:
        assert t is None


def test_tuned_masses_load():
    for ens in ("aniso_xi3.5_eps0.2", "iso_xi1_eps0.25"):
        m0 = bench.tuned_m0(ens)
        assert -0.5 < m0 < 0.5
        # the benchmark masses sit between the small-lattice critical mass and m_c + 0.01
        assert m0 - 0.01 < bench.LIGHT_M0[ens] < m0
