"""Host logic of bench.py that needs no GPU: the HBM-traffic figure is the
counted total per factorization over the run's own launches and is withheld
once the kernel source differs from the one counted, and more than one GPU
is refused before anything touches a device."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.fixture
def counted_source(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_bytes(b"// a kernel source\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC", {"id": (1.0e9, "kernel.hip", digest)})
    return src


def test_traffic_per_launch_divides_the_factorization_total(counted_source):
    assert bench.traffic_for("id", 1000) == pytest.approx(1.0e6)
    assert bench.traffic_for("id", 2000) == pytest.approx(5.0e5)


def test_traffic_is_withheld_when_unmeasured_or_changed(counted_source):
    assert bench.traffic_for("gemm64", 1000) is None
    assert bench.traffic_for("id", 0) is None
    counted_source.write_bytes(b"// the kernel, edited since the counters were taken\n")
    assert bench.traffic_for("id", 1000) is None


def test_recorded_traffic_names_an_existing_source():
    for cls, (nbytes, src, digest) in bench.TRAFFIC.items():
        assert nbytes > 0 and len(digest) == 16
        assert os.path.exists(os.path.join(ROOT, src)), src


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("name", sorted(bench.NEXT_WORKLOADS))
def test_workload_options_are_valid_on_both_sides(name):
    """Each --workload entry: its options make a valid hssmf_opts (the
    library's own check runs in hssmf_factor; here the binding accepts every
    key) and the oracle's Options accept the keys the CPU baseline passes."""
    from oracle import mf
    from paper_1502_07405_amd import hssmf as H
    w = bench.NEXT_WORKLOADS[name]
    o = H.default_opts(**w["opts"])
    assert o.rel_tol == w["opts"]["rel_tol"]
    keys = ("min_sep_hss", "leaf_size", "rel_tol", "d0", "dd", "p", "power_q", "srrqr_f")
    mf.Options(**{k: v for k, v in w["opts"].items() if k in keys})
    assert w["kind"] in ("convdiff", "poisson", "helmholtz")
