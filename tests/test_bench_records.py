"""bench.py's lookup of stored HBM traffic (the traffic-record lines of the
committed rocprofv3 summaries): a record counts only for the kernel source it
was taken on and for launches of the same plan, so a record left behind by a
change of the kernels or of the pass planner reads as null, not as a figure
of other launches."""
import hashlib

import bench


def make_tree(tmp_path, src=b"// kernels\n"):
    (tmp_path / "paper_2108_06831_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "paper_2108_06831_amd" / "csrc" / "kernels.hip").write_bytes(src)
    (tmp_path / "profiles").mkdir()
    sha = hashlib.sha256(src).hexdigest()[:16]
    (tmp_path / "profiles" / "k.md").write_text(
        "# summary\n\n"
        f"traffic-record: config=3 precision=c64 kernel=sweep kernels_hip_sha256={sha} "
        "bytes_per_launch=1000 alg_bytes_per_launch=990.0 fetch_scale=2.0 write_scale=1.0\n")
    return sha


def test_record_is_used_for_the_same_kernels_and_plan(tmp_path, monkeypatch):
    make_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.stored_traffic(3, "c64", "sweep", 990.0) == 1000.0
    assert bench.stored_traffic(3, "c64", "sweep", 990.0 * (1 + 1e-7)) == 1000.0


def test_record_of_other_launches_or_sources_is_ignored(tmp_path, monkeypatch):
    make_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.stored_traffic(3, "c64", "sweep", 1200.0) is None   # another plan's launches
    assert bench.stored_traffic(4, "c64", "sweep", 990.0) is None    # another workload
    assert bench.stored_traffic(3, "bf16x3", "sweep", 990.0) is None
    assert bench.stored_traffic(3, "c64", "adjoint", 990.0) is None
    (tmp_path / "paper_2108_06831_amd" / "csrc" / "kernels.hip").write_bytes(b"// changed\n")
    assert bench.stored_traffic(3, "c64", "sweep", 990.0) is None    # kernels changed since


def test_committed_records_name_their_plan():
    """Every committed record carries the algorithmic bytes per launch it was
    taken on, or the lookup could never use it."""
    import glob
    import os
    n = 0
    for f in glob.glob(os.path.join(bench.ROOT, "profiles", "*.md")):
        for line in open(f):
            if line.startswith("traffic-record:"):
                kv = dict(x.split("=", 1) for x in line.split()[1:])
                assert float(kv["alg_bytes_per_launch"]) > 0 and float(kv["bytes_per_launch"]) > 0
                n += 1
    assert n >= 3
