"""CPU checks of the benchmark's host logic: the one-GPU refusal, the
algorithmic work per replica-step behind the roofline figure, and the rule
that HBM traffic is reported only for the kernel source the counters were
taken on."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from pamd_inputs import systems as S  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_peptide_work_per_replica_step():
    """25 flops per nonbonded pair, 21 per bond, 70 per angle, 110 per
    dihedral, 18 per atom: the 75-atom peptide has 2569 pairs (75 * 74 / 2
    minus 74 bonds and 132 angles of a tree), so 95,949 flops."""
    sysd = S.c2_system()
    flops, pairs = bench.algorithmic_flops_per_replica_step(sysd)
    assert (len(sysd.bonds), len(sysd.angles), len(sysd.dihedrals)) == (74, 132, 178)
    assert pairs == 75 * 74 // 2 - 74 - 132 == 2569
    assert flops == 25 * 2569 + 21 * 74 + 70 * 132 + 110 * 178 + 18 * 75 == 95949


def test_traffic_only_for_the_profiled_source(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1806_06016_amd", "csrc", "md_kernel.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "match.txt").write_text(f"# comment\nkernel_source_sha256_prefix = {sha}\n"
                                    "fetch_bytes_per_launch = 100\nwrite_bytes_per_launch = 23\n")
    (prof / "stale.txt").write_text("kernel_source_sha256_prefix = 0000000000000000\n"
                                    "fetch_bytes_per_launch = 100\nwrite_bytes_per_launch = 23\n")
    fake_root = tmp_path
    csrc = fake_root / "paper_1806_06016_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "md_kernel.hip").write_bytes(open(src, "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(fake_root))
    assert bench.measured_traffic("match.txt") == 123
    assert bench.measured_traffic("stale.txt") is None
    assert bench.measured_traffic("missing.txt") is None


@pytest.mark.parametrize("name", ["k_md_traffic.txt", "k_md_wide_traffic.txt"])
def test_committed_traffic_summaries_are_current(name):
    """The committed counter summaries belong to the committed kernel source
    (otherwise the bench would report traffic null)."""
    assert bench.measured_traffic(name) is not None


def test_cpu_baseline_fields():
    """The oracle baseline on the host: the bench line's cpu_baseline object
    (all host threads, and one core in a child process) on a short sample."""
    one = bench.cpu_baseline_one_core(0.3)
    assert one["cores"] == 1 and one["value"] > 0 and "one thread" in one["sample"]
    r, steps, el = bench._oracle_sample(16, 0.3)
    assert r > 0 and steps >= 20 and el > 0
