"""Host logic of bench.py's roofline fields (no GPU): kernel-name keys, the
kernels of a profile class, the dispatch-weighted HBM traffic per launch,
and the kernel-trace summary written from a rocprofv3 database."""

import json
import os
import sqlite3

import bench


def test_kernel_key_strips_return_type_namespace_and_arguments():
    assert bench.kernel_key("void ocm::k_tiescan_tile<int, true>(ocm::SweepArgs, int const*)") == \
        "k_tiescan_tile<int, true>"
    assert bench.kernel_key("ocm::k_conn_claim(int, int, int const*)") == "k_conn_claim"
    assert bench.kernel_key("k_val_round") == "k_val_round"


def test_class_kernels_match_base_and_instantiation():
    table = {"k_sweep_tile<int, true>": 1, "k_tiescan_tile<int, true>": 2,
             "k_tiescan_tile<int, false>": 3, "k_conn_claim": 4, "k_round_claim": 5}
    assert sorted(bench.class_kernels(table, "sweep")) == [1, 2]
    assert bench.class_kernels(table, "tiescan") == [3]
    assert bench.class_kernels(table, "conn_claim") == [4]   # not the device-loop kernel
    assert bench.class_kernels(table, "no_such_class") == []


def test_traffic_per_launch_is_the_dispatch_weighted_calibrated_average():
    pmc = {"calibration": {"fetch_factor": 2.0, "write_factor": 1.0},
           "kernels": {"k_sweep_tile<int, true>": {"dispatches": 1, "fetch_kib": 100.0,
                                                   "write_kib": 10.0},
                       "k_tiescan_tile<int, true>": {"dispatches": 3, "fetch_kib": 200.0,
                                                     "write_kib": 20.0}}}
    got = bench.traffic_per_launch(pmc, "sweep")
    want = 1024.0 * (1 * (100 * 2 + 10) + 3 * (200 * 2 + 20)) / 4
    assert abs(got - want) < 1e-6
    assert bench.traffic_per_launch(pmc, "conn_claim") is None
    assert bench.traffic_per_launch(None, "sweep") is None


def test_trace_summary_round_trip(tmp_path, monkeypatch):
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(str(db))
    con.execute("create table kernels (name text, start integer, end integer)")
    rows = [("void ocm::k_conn_claim(int)", 0, 50_000), ("void ocm::k_conn_claim(int)", 100_000, 160_000),
            ("void ocm::k_round_claim(int)", 200_000, 210_000)]
    con.executemany("insert into kernels values (?, ?, ?)", rows)
    con.commit()
    con.close()
    out = tmp_path / "profiles" / "w_kernel_trace.md"
    bench.summarize_trace(str(db), str(out), "w", "cmd", "note")
    text = out.read_text()
    d = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    assert d["source_sha256"] == bench.source_digest()
    assert d["kernels"]["k_conn_claim"] == {"calls": 2, "total_ns": 110_000}
    # the average the roofline reports beside its own: only the class's kernel
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    trace = bench.load_trace("w")
    assert trace is not None
    assert abs(bench.trace_avg_us(trace, "conn_claim") - 55.0) < 1e-9
    assert bench.trace_avg_us(trace, "values") is None


def test_stale_counter_files_are_not_used(tmp_path, monkeypatch):
    os.makedirs(tmp_path / "profiles")
    blob = {"workload": "w", "source_sha256": "0" * 64, "calibration": {}, "kernels": {}}
    (tmp_path / "profiles" / "pmc_w.md").write_text("x\n```json\n" + json.dumps(blob) + "\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_pmc("w") is None
