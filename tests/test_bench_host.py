"""Host logic of bench.py (no GPU): the one-GPU contract, the rocprofv3 counter summary and its
scaling by the copy calibration, and the gating of measured traffic on the kernel sources."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _db(path, copies_kib, kernels):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, grid_size integer, "
                "value real)")
    rows = [(i, "__amd_rocclr_copyBuffer", 131072, v) for i, v in enumerate(copies_kib)]
    rows += [(len(rows) + i, name, 1024, v) for i, (name, v) in enumerate(kernels)]
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()


def test_counter_summary_is_scaled_by_the_copy_calibration(tmp_path):
    # FETCH_SIZE reading half of each 1 GiB copy (factor 2), WRITE_SIZE all of it (factor 1)
    fetch, write = str(tmp_path / "fetch.db"), str(tmp_path / "write.db")
    flux = "void gks::k_flux_chunked<true, false>(gks::DevMesh, ...)"
    recon = "void gks::k_reconstruct<double, false, 0>(gks::DevMesh, ...)"
    _db(fetch, [524288.0] * 3, [(flux, 1000.0), (flux, 3000.0), (recon, 10.0), ("other_kernel(", 5.0)])
    _db(write, [1048576.0] * 3, [(flux, 100.0), (flux, 300.0), (recon, 1.0)])
    d = bench.counters_from(fetch, write)
    assert d["fetch_factor"] == pytest.approx(2.0)
    assert d["write_factor"] == pytest.approx(1.0)
    assert d["kernel_source_sha256"] == bench.kernel_source_hash()
    assert set(d["kernels"]) == {"flux", "reconstruct"}
    assert d["kernels"]["flux"]["read_bytes"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert d["kernels"]["flux"]["write_bytes"] == pytest.approx(200.0 * 1024)
    assert d["kernels"]["reconstruct"]["read_bytes"] == pytest.approx(10.0 * 1024 * 2.0)


def test_measured_traffic_only_for_the_sources_it_was_measured_on(tmp_path, monkeypatch):
    kernels = {"flux": {"read_bytes": 3.0, "write_bytes": 1.0}}
    good = tmp_path / "good.json"
    good.write_text(json.dumps({"kernel_source_sha256": bench.kernel_source_hash(), "kernels": kernels}))
    stale = tmp_path / "stale.json"
    stale.write_text(json.dumps({"kernel_source_sha256": "0" * 64, "kernels": kernels}))
    monkeypatch.setattr(bench, "COUNTERS_JSON", str(good))
    assert bench.measured_traffic() == {"flux": 4.0}
    monkeypatch.setattr(bench, "COUNTERS_JSON", str(stale))
    assert bench.measured_traffic() == {}
    monkeypatch.setattr(bench, "COUNTERS_JSON", str(tmp_path / "missing.json"))
    assert bench.measured_traffic() == {}


def test_committed_counter_summary_names_every_timed_kernel():
    with open(bench.COUNTERS_JSON) as fh:
        d = json.load(fh)
    assert {"reconstruct", "flux", "stage1", "stage2", "timestep"} <= set(d["kernels"])
    assert 1.5 < d["fetch_factor"] < 2.5 and 0.5 < d["write_factor"] < 1.5


def test_algorithmic_bytes_scale_with_the_mesh_and_the_precision():
    class H:
        pass

    h = H()
    h.n, h.n_faces, h.n_stencil, h.n_subcoef = 1000, 2300, 16000, 33000
    h.n_cellfaces = 2 * h.n_faces
    b64, b32 = bench.algorithmic_bytes(h, 8), bench.algorithmic_bytes(h, 4)
    for k in ("reconstruct", "flux", "stage1", "stage2"):
        assert b32[k] < b64[k], k
    h2 = H()
    h2.n, h2.n_faces, h2.n_stencil, h2.n_subcoef, h2.n_cellfaces = (2 * h.n, 2 * h.n_faces, 2 * h.n_stencil,
                                                                    2 * h.n_subcoef, 2 * h.n_cellfaces)
    b2 = bench.algorithmic_bytes(h2, 8)
    for k, v in b64.items():
        assert b2[k] == 2 * v, k


def test_flops_count_lanes_and_fma_twice():
    c = {"SQ_INSTS_VALU_FMA_F64": 10.0, "SQ_INSTS_VALU_MUL_F64": 3.0, "SQ_INSTS_VALU_ADD_F64": 2.0,
         "SQ_INSTS_VALU_FMA_F32": 1.0}
    assert bench.flops(c, 64) == 64 * (2 * 10 + 3 + 2)
    assert bench.flops(c, 32) == 64 * 2


def test_valu_summary_from_a_counter_database(tmp_path):
    db = str(tmp_path / "valu.db")
    con = sqlite3.connect(db)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
                "value real)")
    flux = "void gks::k_flux_chunked<true, false>(gks::DevMesh, ...)"
    con.executemany("insert into counters_collection values (?, ?, ?, ?)",
                    [(1, flux, "SQ_INSTS_VALU", 100.0), (1, flux, "SQ_INSTS_VALU_FMA_F64", 40.0),
                     (2, flux, "SQ_INSTS_VALU", 300.0), (2, flux, "SQ_INSTS_VALU_FMA_F64", 60.0),
                     (3, "other(", "SQ_INSTS_VALU", 7.0)])
    con.commit()
    con.close()
    d = bench.valu_from([db])
    assert d["kernel_source_sha256"] == bench.kernel_source_hash()
    assert d["kernels"] == {"flux": {"SQ_INSTS_VALU": 200.0, "SQ_INSTS_VALU_FMA_F64": 50.0}}


def test_committed_valu_summary_has_the_flux_counts():
    with open(bench.VALU_JSON) as fh:
        d = json.load(fh)
    f = d["kernels"]["flux"]
    assert f["SQ_INSTS_VALU_FMA_F64"] > 0 and f["SQ_INSTS_VALU"] > f["SQ_INSTS_VALU_FMA_F64"]
