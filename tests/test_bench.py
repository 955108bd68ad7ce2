"""Host logic of bench.py (no GPU): the recorded HBM traffic is reported only
while every source it was measured on is unchanged, more than one GPU is
refused with a message, and the CPU-baseline leg times the oracle on a
bounded sample."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_traffic_record_follows_the_sources(tmp_path, monkeypatch):
    """A record counts while its sources hash to the recorded value and stops
    counting once any of them changes."""
    import hashlib

    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    key = next(iter(rec))
    kernel, workload = key.split("/")
    h = hashlib.sha256()
    for f in rec[key]["sources"]:
        os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
        shutil.copy(os.path.join(ROOT, f), tmp_path / f)
        h.update(open(tmp_path / f, "rb").read())
    rec[key]["sources_sha256"] = h.hexdigest()  # as recorded when the counters were taken on these sources
    os.makedirs(tmp_path / "profiles")
    json.dump(rec, open(tmp_path / "profiles" / "traffic.json", "w"))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    want = rec[key]["fetch_bytes"] + rec[key]["write_bytes"]
    assert bench.measured_traffic(kernel, workload) == pytest.approx(want)
    assert bench.measured_traffic(kernel, "no-such-workload") is None
    with open(tmp_path / rec[key]["sources"][-1], "a") as fh:
        fh.write("\n// changed\n")
    assert bench.measured_traffic(kernel, workload) is None


def test_record_traffic_scales_each_counter_by_the_calibration_copy(tmp_path, monkeypatch):
    """A record holds the kernel's FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
    scaled by the ratio of the calibration copy's size to what the counter read
    for that copy: the last matching dispatch for one launch, or the mean times
    the launches of a sequence; with the closure and digest of its sources."""
    import shutil as sh

    src = "paper_2505_18508_amd/csrc/sweep_batch.hip"
    for f in bench.source_closure(src):
        os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
        sh.copy(os.path.join(ROOT, f), tmp_path / f)
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    kib = bench.CALIBRATION_COPY_BYTES / 1024

    def run(name, counter, copy_kib, values):
        d = tmp_path / name
        os.makedirs(d)
        rows = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
        rows.append("1,__amd_rocclr_copyBuffer,%s,%r" % (counter, copy_kib))
        for i, v in enumerate(values):  # two instances of the counter per dispatch
            rows.append('%d,"void k_x<2>(Args)",%s,%r' % (i + 2, counter, v / 2))
            rows.append('%d,"void k_x<2>(Args)",%s,%r' % (i + 2, counter, v / 2))
        rows.append('9,"void k_other(int)",%s,1000.0' % counter)
        (d / "run_counter_collection.csv").write_text("\n".join(rows) + "\n")
        return str(d)

    fetch = run("f", "FETCH_SIZE", kib / 2, [100.0, 300.0])  # the copy reads half its bytes: x2
    write = run("w", "WRITE_SIZE", kib, [50.0, 70.0])
    rec = bench.record_traffic("k_x/w1", src, "k_x<2>", fetch, write, "profiles/x.md")
    assert rec["fetch_bytes"] == pytest.approx(300.0 * 1024 * 2)
    assert rec["write_bytes"] == pytest.approx(70.0 * 1024)
    assert rec["sources"] == bench.source_closure(src) and "include/ising.h" in rec["sources"]
    assert bench.measured_traffic("k_x", "w1") == pytest.approx((600.0 + 70.0) * 1024)
    rec = bench.record_traffic("k_x/w2", src, "k_x<2>", fetch, write, "profiles/x.md", per_sequence=10)
    assert rec["fetch_bytes"] == pytest.approx(200.0 * 10 * 1024 * 2)
    assert rec["write_bytes"] == pytest.approx(60.0 * 10 * 1024)
    assert set(json.load(open(bench.traffic_path()))) == {"k_x/w1", "k_x/w2"}


def test_traffic_record_lists_every_included_source():
    """The record's sources are the kernel file and the transitive closure of
    its quoted includes, so no header the kernel is built from can change
    unnoticed."""
    import re

    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for key, r in rec.items():
        todo, seen = [r["sources"][0]], set()
        while todo:
            f = todo.pop()
            if f in seen:
                continue
            seen.add(f)
            text = open(os.path.join(ROOT, f)).read()
            for inc in re.findall(r'^#include "([^"]+)"', text, re.M):
                path = os.path.normpath(os.path.join(os.path.dirname(f), inc))
                if not os.path.exists(os.path.join(ROOT, path)):
                    path = os.path.normpath(os.path.join("include", inc))
                todo.append(path)
        assert set(r["sources"]) == seen, key


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=300, cwd=ROOT)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


def test_cpu_baseline_times_the_oracle():
    wl = dict(bench.WORKLOADS["torus100x100"], dims=[8, 8], R=3, S=40)
    res, done = bench.cpu_baseline(0.0, wl, task_s=10.0)
    assert res["kind"] == "oracle" and res["unit"] == "attempts/s" and res["value"] > 0
    assert res["cores"] == min(os.cpu_count() or 1, 16)
    assert "full 40-sweep schedule" in res["sample"]
    assert sorted(r for r, _ in done) == list(range(min(3, res["cores"])))
    assert all(s.shape == (64,) and set(s.tolist()) <= {-1, 1} for _, s in done)
    # the oracle's replicas are the same trajectories as a run of all of them
    import oracle

    w = oracle.random_weights(wl["weight_seed"], 2 * 64)
    ref, _ = oracle.run(wl["dims"], w, wl["seed"], 3, 40, schedule=oracle.SCHED_GEOMETRIC, beta0=wl["beta0"],
                        beta1=wl["beta1"])
    assert bench.with_parity(res, done, ref)["parity_with_gpu"] is True


def test_cpu_baseline_windows_large_lattices_and_samples_the_batch():
    """A lattice too large for one replica's whole schedule within half the
    budget runs the first sweeps (no parity claim); 3-D lattices take ndim n
    edges; the batch samples its largest instance."""
    wl = dict(bench.WORKLOADS["torus64x64x64"], dims=[4, 4, 6], R=2, S=30)
    res, done = bench.cpu_baseline(0.0, wl, task_s=96 * 10 / 1e8)  # one task's time covers 10 sweeps of 96 sites
    assert "sweeps [0, 10) of the 30-sweep schedule" in res["sample"] and done is None
    assert bench.with_parity(res, done, None)["parity_with_gpu"] is None
    b = bench.cpu_workload("batch4tori")
    assert b["dims"] == [100, 200] and b["S"] == 20000 and b["R"] == 4096 and "100x200 instance" in b["sample_of"]
    assert bench.cpu_workload("torus100x100") is bench.WORKLOADS["torus100x100"]


def test_ttt_leg_configuration_and_model():
    """The time-to-target leg's network loads without unpickling, is a
    16-64-64-1 network of the relative label, and its schedule gives 19
    rankings per trial."""
    import numpy as np

    from paper_2505_18508_amd import learn

    W = bench.TTT
    with np.load(os.path.join(ROOT, W["model"]), allow_pickle=False) as z:
        assert z["params"].shape == (5313,) and z["mean"].shape == (16,) and z["std"].shape == (16,)
        assert learn.LABELS[int(z["label"])] == "relative"
        assert np.isfinite(z["params"]).all()
    assert len(learn.checkpoints(W["S"], W["window"])) == 19
    assert W["dims"] == bench.WORKLOADS[bench.DEFAULT_WORKLOAD]["dims"]
    assert W["weight_seed"] == bench.WORKLOADS[bench.DEFAULT_WORKLOAD]["weight_seed"]


def test_ttt_workload_seeds():
    """--ttt-seeds swaps the run seeds and the workload's name, nothing else."""
    W = bench.ttt_workload([201, 202, 203, 204, 205])
    assert W["seeds"] == (201, 202, 203, 204, 205)
    assert W["name"].endswith("run seeds 201, 202, 203, 204, 205")
    assert {k: v for k, v in W.items() if k not in ("seeds", "name")} == \
        {k: v for k, v in bench.TTT.items() if k not in ("seeds", "name")}
    assert bench.ttt_workload() is bench.TTT
    with pytest.raises(ValueError):
        bench.ttt_workload([])
