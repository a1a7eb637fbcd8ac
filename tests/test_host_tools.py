"""Host-side tools (no GPU): the trace/counter summariser, the bench's
accounting and traffic lookup, and the warm start's validation helpers."""
import math
import os
import sqlite3

import pytest

import bench
from paper_2206_13164_amd import inputs as I
from paper_2206_13164_amd import profsum as P
from paper_2206_13164_amd import warmstart as W


def fake_trace(path):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start int, end int, duration int, grid_x int, "
                "workgroup_x int, vgpr_count int, lds_size int, scratch_size int)")
    rows = [
        ("void nrxx::(anonymous namespace)::k_a<8, 2, 2>(int)", 50, 90, 40, 256, 128, 96, 100, 0),
        ("void nrxx::(anonymous namespace)::k_a<8, 2, 2>(int)", 100, 160, 60, 256, 128, 96, 100, 0),
        ("void nrxx::(anonymous namespace)::k_b(int)", 140, 200, 60, 64, 64, 8, 0, 0),
        ("void nrxx::(anonymous namespace)::k_b(int)", 300, 320, 20, 64, 64, 8, 0, 0),  # outside
    ]
    con.executemany("insert into kernels values (?,?,?,?,?,?,?,?,?)", rows)
    con.execute("create table pmc_events (name text, dispatch_id int, counter_name text, "
                "counter_value real, start int, end int)")
    ev = [("void k_a<8>(int)", 1, "SQ_WAVES", 10.0, 50, 90), ("void k_a<8>(int)", 1, "SQ_WAVES", 6.0, 50, 90),
          ("void k_a<8>(int)", 2, "SQ_WAVES", 20.0, 100, 160), ("void k_a<8>(int)", 3, "SQ_WAVES", 99.0, 300, 320)]
    con.executemany("insert into pmc_events values (?,?,?,?,?,?)", ev)
    con.commit()
    con.close()


def test_profsum_keeps_the_timed_window_and_merges_overlaps(tmp_path):
    db = str(tmp_path / "t.db")
    fake_trace(db)
    w0, w1 = P.window("[bench] timed window monotonic_ns 40 250 boottime_ns 1 2\n")
    assert (w0, w1) == (40, 250)
    per, busy = P.summarise(db, w0, w1)
    assert per["k_a<8, 2, 2>"]["calls"] == 2 and per["k_a<8, 2, 2>"]["ns"] == 100
    assert per["k_b"]["calls"] == 1
    # union of [50, 90], [100, 160], [140, 200]
    assert busy == 40 + 100
    with pytest.raises(SystemExit):
        P.window("no window here")


def test_profsum_counters_sum_instances_and_average_dispatches(tmp_path):
    db = str(tmp_path / "t.db")
    fake_trace(db)
    res = P.counters(db)
    n, mean = res["k_a<8>"]["SQ_WAVES"]
    assert n == 3 and mean == pytest.approx((16.0 + 20.0 + 99.0) / 3)
    n, mean = P.counters(db, 40, 250)["k_a<8>"]["SQ_WAVES"]
    assert n == 2 and mean == pytest.approx(18.0)


def test_cycle_accounting_counts_cells_and_the_dependency_chain():
    s = I.spec(None, nx=64, ny=32, M=5, levels=3, s1=2, s2=2, s3=4)
    a = bench.cycle_accounting(s)
    cells = 4 * 4 * 64 * 32 + 4 * 4 * 32 * 16 + 4 * 4 * 16 * 8
    assert a["cells"] == cells
    assert a["chain"] == 16 * (95 + 47) + 16 * 23
    f, b = bench.per_update_cost(5, 2, coarse=False)
    assert f == 2 * 9 * 3 * math.comb(9, 4) + 80 * 56 and b == 2 * 59 * 8


def test_sweep_traffic_is_used_only_for_the_profiled_kernel_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.sweep_traffic("w") is None
    table = ("| kernel | dispatches | FETCH_SIZE KiB per dispatch | WRITE_SIZE KiB per dispatch | "
             "HBM bytes per launch |\n|---|---:|---:|---:|---:|\n"
             "| `k_wsweep<8, 2, 2>` | 16 | 1 | 1 | 3072 |\n")
    path = os.path.join(str(tmp_path), "sweep_traffic_w.md")
    with open(path, "w") as fh:
        fh.write(table + "- kernel_source_sha256: `deadbeef`\n")
    assert bench.sweep_traffic("w") is None  # another source
    with open(path, "w") as fh:
        fh.write(table + f"- kernel_source_sha256: `{bench.kernel_source_hash()}`\n")
    assert bench.sweep_traffic("w") == {"k_wsweep<8, 2, 2>": 3072.0}


def test_sweep_kernel_names_follow_the_tuning():
    t = dict(M=8, order=2, kernel=1, team_width=4, split=1)
    assert bench.sweep_kernel_name(t) == "k_wsweep<8, 2, 2>"
    assert bench.sweep_kernel_name(dict(t, M=5)) == "k_wsweep<5, 2, 4>"
    assert bench.sweep_kernel_name(dict(t, M=3, kernel=0, team_width=1, split=1)) == \
        "k_bsweep<double, 3, 2, 1, true>"


def test_warm_start_gate_and_validation_draws():
    rows = [dict(Kn=0.5, maxwellian=100, learned=104), dict(Kn=0.02, maxwellian=40, learned=31),
            dict(Kn=0.04, maxwellian=22, learned=22), dict(Kn=0.03, maxwellian=22, learned=19)]
    assert W.choose_gate(rows) == 0.04
    assert W.choose_gate([dict(Kn=0.1, maxwellian=10, learned=9)]) is None
    v = W.validation_draws(3)
    train = I.cavity_draws(2003, I.SEED_TRAIN, sides=(W.FIELD_GRID,), levels=W.TRAIN_LEVELS,
                           tol=W.TRAIN_TOL)[2000:]
    for a, b in zip(v, train):  # the training stream's draws 2000.. at 256^2, M = 5
        assert a["Kn"] == b["Kn"] and a["wall_u"] == b["wall_u"]
        assert (a["nx"], a["ny"], a["M"], a["levels"], a["tol"]) == (256, 256, 5, 6, 1e-8)


def test_profsum_selects_a_labelled_window():
    text = ("[bench] timed window monotonic_ns 1 2 boottime_ns 3 4\n"
            "[bench] heated256_shakhov_m8_kn005_fp64 window monotonic_ns 10 20\n"
            "[bench] heated256_shakhov_m8_kn005_fp32_blocks window monotonic_ns 30 40\n")
    assert P.window(text) == (1, 2)
    assert P.window(text, "heated256_shakhov_m8_kn005_fp64") == (10, 20)
    assert P.window(text, "heated256_shakhov_m8_kn005_fp32_blocks") == (30, 40)
    with pytest.raises(SystemExit):
        P.window(text, "heated256_shakhov_m8_kn02_fp64")
