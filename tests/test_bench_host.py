"""Host-side pieces of bench.py (no GPU): the one-GPU refusal, the step-kernel name
parser the counter summary relies on, and the copy-calibrated traffic arithmetic."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


@pytest.mark.parametrize("name,kind", [
    ("void pfk::(anonymous namespace)::k_explicit2d_seam<float, 1, 3, false>(float const*)", ("seam", 3)),
    ("void pfk::(anonymous namespace)::k_explicit2d<float, 1, 4, 2, false, false>(float const*)",
     ("halo", 2)),
    ("void pfk::(anonymous namespace)::k_explicit2d<float, 0, 8, 1, true, false>(float const*)", ("halo", 1)),
    ("void pfk::(anonymous namespace)::k_jvp2d<float, 0, true>(float const*)", None),
    ("__amd_rocclr_copyBuffer", None),
])
def test_step_kernel_names(name, kind):
    assert bench._step_kernel(name) == kind


def _counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_summarize_counters_scales_by_the_copy(tmp_path, monkeypatch, capsys):
    """The step kernel's FETCH_SIZE/WRITE_SIZE (KiB per dispatch, averaged over
    dispatches) are each scaled by true bytes / counter reading of a copy of known
    size; the kernel fusing the most steps is the one summarised."""
    seam = "void pfk::(anonymous namespace)::k_explicit2d_seam<float, 1, 3, false>(float const*)"
    single = "void pfk::(anonymous namespace)::k_explicit2d<float, 1, 4, 1, false, false>(float const*)"
    copy = "k_stream_copy(float4 const*)"
    step, cp = tmp_path / "step", tmp_path / "copy"
    _counters(str(step / "fetch"), [(seam, "FETCH_SIZE", 100.0), (seam, "FETCH_SIZE", 300.0),
                                    (single, "FETCH_SIZE", 9999.0)])
    _counters(str(step / "write"), [(seam, "WRITE_SIZE", 50.0), (single, "WRITE_SIZE", 7777.0)])
    mib = 4  # the copy moved 4 MiB each way; its counters read 5/8 and all of it
    _counters(str(cp / "fetch"), [(copy, "FETCH_SIZE", mib * 1024 * 0.625)])
    _counters(str(cp / "write"), [(copy, "WRITE_SIZE", mib * 1024)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "_traffic_path", lambda n, ks: str(out))
    bench.summarize_counters(str(step), str(cp), mib, n=64)
    rec = json.load(open(out))
    assert rec["kernel"] == seam and rec["ks"] == 3 and rec["n"] == 64
    assert rec["copy_fetch_scale"] == pytest.approx(1.6) and rec["copy_write_scale"] == pytest.approx(1.0)
    assert rec["bytes_per_launch"] == pytest.approx(200.0 * 1024 * 1.6 + 50.0 * 1024)
    assert rec["algorithmic_bytes_per_launch"] == bench.BYTES_PER_NODE_STEP * 64 * 64
    assert rec["kernel_src_sha256_16"] == bench.kernel_hash()
    assert json.loads(capsys.readouterr().out.strip()) == rec
