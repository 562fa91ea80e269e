"""CPU checks of bench.py's host logic: the one-GPU rule, and that HBM
traffic is reported only for the configuration the counters were taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.fixture
def digest_matches(monkeypatch):
    monkeypatch.setattr(bench, "kernel_sources_digest", lambda: bench.MEASURED_TRAFFIC["sources_sha256"])


def test_traffic_of_the_measured_configuration(digest_matches):
    m = bench.MEASURED_TRAFFIC
    for (prec, name), (fetch, write) in m["kib"].items():
        got = bench.measured_traffic(name, m["skin"], m["replicas"], prec, m["block"][prec])
        assert got == pytest.approx(1024.0 * (fetch * m["fetch_factor"] + write * m["write_factor"]))


@pytest.mark.parametrize("change", ["skin", "replicas", "block", "kernel"])
def test_no_traffic_for_another_configuration(digest_matches, change):
    m = bench.MEASURED_TRAFFIC
    args = dict(name="pass2", skin=m["skin"], replicas=m["replicas"], precision="mixed",
                block=m["block"]["mixed"])
    if change == "skin":
        args["skin"] = m["skin"] + 0.4
    elif change == "replicas":
        args["replicas"] = m["replicas"] // 2
    elif change == "block":
        args["block"] = 64 if m["block"]["mixed"] != 64 else 256
    else:
        args["name"] = "gather"  # a kernel the counters were not recorded for
    assert bench.measured_traffic(**args) is None


def test_no_traffic_once_the_kernel_sources_change(monkeypatch):
    m = bench.MEASURED_TRAFFIC
    monkeypatch.setattr(bench, "kernel_sources_digest", lambda: "0" * 64)
    assert bench.measured_traffic("pass2", m["skin"], m["replicas"], "mixed", m["block"]["mixed"]) is None


def test_digest_covers_the_kernels_and_the_block_placement(tmp_path, monkeypatch):
    """The digest hashes the kernel sources and the host file that places
    blocks on the XCDs: a change to any of them changes it."""
    src = os.path.join(ROOT, "paper_2103_10449_amd", "csrc")
    dst = tmp_path / "paper_2103_10449_amd" / "csrc"
    dst.mkdir(parents=True)
    files = ("swfe_kernels.hip", "swfe_internal.h", "swfe_api.hip")
    for f in files:
        (dst / f).write_bytes(open(os.path.join(src, f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.kernel_sources_digest()
    assert d0 == bench.kernel_sources_digest() and len(d0) == 64
    for f in files:
        orig = (dst / f).read_bytes()
        (dst / f).write_bytes(orig + b"\n")
        assert bench.kernel_sources_digest() != d0, f
        (dst / f).write_bytes(orig)
    assert bench.kernel_sources_digest() == d0


def test_kernel_flops_count_each_unique_term_once():
    pairs, atoms = 1000, 90
    assert bench.kernel_flops("pass1", atoms, pairs) == pairs / 2 * bench.C_PAIR + pairs * bench.C_MOM
    assert bench.kernel_flops("pass2", atoms, pairs) == pairs * bench.C_D3 + atoms * bench.C_ATOM2
    assert bench.kernel_flops("integrate", atoms, pairs) is None


def test_step_algorithmic_bytes_by_hand():
    # 10 atoms (4 Frenkel-Ladd), 30 ordered pairs, 80 list entries, 5 atoms
    # rebuilt per step, 2 tiles, FP32 moments
    a = bench.step_algorithmic_bytes(10, 4, 30, 80, 5, 2, 36)
    assert a["integrate"] == 10 * 180 + 4 * 24
    assert a["pass1"] == 10 * (24 + 4 + 36 + 4 + 24) + 2 * 80 + 2 * 30
    assert a["pass2"] == 10 * (24 + 36 + 4 + 4 + 96 + 24) + 4 * 24 + 2 * 30
    assert a["rebuild"] == pytest.approx(5 * (384 + 2 * 8.0))
    assert a["finalize"] == 2 * 2 * 26 * 8


def test_step_traffic_needs_every_step_kernel(digest_matches):
    m = bench.MEASURED_TRAFFIC
    run = dict(block=m["block"]["mixed"], n_atoms=10, pairs=30, list_entries=80, rebuilt_atoms_per_step=5,
               n_tiles=2)
    got = bench.step_traffic(run, m["skin"], m["replicas"], "mixed", 4, 36)
    have_all = all(("mixed", k) in m["kib"] for k in bench.STEP_KERNELS)
    if not have_all:
        assert got is None
    else:
        assert got["counter_bytes"] == pytest.approx(
            sum(bench.measured_traffic(k, m["skin"], m["replicas"], "mixed", run["block"])
                for k in bench.STEP_KERNELS))
        assert got["ratio"] == pytest.approx(got["counter_bytes"] / got["algorithmic_bytes"])


def test_step_traffic_against_the_one_pass_budget(digest_matches):
    m = bench.MEASURED_TRAFFIC
    run = dict(block=m["block"]["mixed"], n_atoms=10, pairs=30, list_entries=80, rebuilt_atoms_per_step=5,
               n_tiles=2)
    got = bench.step_traffic(run, m["skin"], m["replicas"], "mixed", 4, 36)
    if got is not None:
        assert got["one_pass_bytes"] == 10 * 156 + 4 * 24
        assert got["ratio_one_pass"] == pytest.approx(got["counter_bytes"] / got["one_pass_bytes"])
