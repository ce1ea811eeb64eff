"""The rocprofv3 summaries behind the committed profiles, on small
synthetic files in both of rocprofv3's formats (CSV and its SQLite
database): kernel statistics, per-dispatch counter means over the last N
dispatches, last-N durations, and the copy calibration factor."""
import csv
import sqlite3

import pytest

from paper_cs_0105004_amd import profiling as P

STEP = "void tr::k_step<false>(tr::DevScen const*, int, int4 const*, int)"
COPY = "void at::native::copy_kernel(float*)"


def test_short_names():
    assert P.short_name(STEP) == "k_step<false>"
    assert P.short_name("k_back<true>") == "k_back<true>"


def write_csv(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_kernel_stats_from_csv_and_db(tmp_path):
    c = tmp_path / "run_kernel_stats.csv"
    write_csv(c, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage",
                  "MinNs", "MaxNs"],
              [[STEP, 3, 36000, 12000, 99.0, 11000, 13000]])
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, duration integer)")
    con.executemany("insert into kernels values (?, ?)",
                    [(STEP, 11000), (STEP, 12000), (STEP, 13000)])
    con.commit()
    con.close()
    a, b = P.kernel_stats(str(c)), P.kernel_stats(str(db))
    for st in (a, b):
        s = st["k_step<false>"]
        assert s["calls"] == 3 and s["avg_ns"] == 12000.0
        assert s["total_ns"] == 36000.0
        assert (s["min_ns"], s["max_ns"]) == (11000.0, 13000.0)


def counter_rows():
    # dispatch ids out of order; the last two dispatches of k_step read 30, 40
    return [(STEP, "FETCH_SIZE", 5, 30.0), (STEP, "FETCH_SIZE", 2, 10.0),
            (STEP, "FETCH_SIZE", 9, 40.0), (STEP, "FETCH_SIZE", 3, 20.0),
            (STEP, "WRITE_SIZE", 2, 7.0), (COPY, "FETCH_SIZE", 1, 524288.0)]


@pytest.mark.parametrize("fmt", ["csv", "db"])
def test_counter_means_over_the_last_dispatches(tmp_path, fmt):
    rows = counter_rows()
    if fmt == "csv":
        path = tmp_path / "run_counter_collection.csv"
        write_csv(path, ["Dispatch_Id", "Kernel_Name", "Counter_Name",
                         "Counter_Value"],
                  [[d, k, c, v] for k, c, d, v in rows])
    else:
        path = tmp_path / "run_results.db"
        con = sqlite3.connect(path)
        con.execute("create table counters_collection (kernel_name text,"
                    " counter_name text, dispatch_id integer, value real)")
        con.executemany("insert into counters_collection values (?, ?, ?, ?)",
                        rows)
        con.commit()
        con.close()
    allc = P.counters(str(path))
    assert allc["k_step<false>"]["FETCH_SIZE"] == (4, 25.0)
    assert allc["k_step<false>"]["WRITE_SIZE"] == (1, 7.0)
    last = P.counters(str(path), last=2)
    assert last["k_step<false>"]["FETCH_SIZE"] == (2, 35.0)


def test_last_durations_and_copy_factor(tmp_path, capsys):
    trace = tmp_path / "run_kernel_trace.csv"
    write_csv(trace, ["Dispatch_Id", "Kernel_Name", "Start_Timestamp",
                      "End_Timestamp"],
              [[1, STEP, 0, 100], [4, STEP, 500, 530], [3, STEP, 200, 220],
               [2, COPY, 100, 150]])
    got = P.last_durations(str(trace), 2)
    assert got["k_step<false>"] == (2, 25.0)  # dispatches 3 and 4
    cc = tmp_path / "run_counter_collection.csv"
    write_csv(cc, ["Dispatch_Id", "Kernel_Name", "Counter_Name",
                   "Counter_Value"],
              [[1, COPY, "FETCH_SIZE", 524288.0]])
    assert P.main(["copy", str(cc), str(1 << 30)]) == 0
    out = capsys.readouterr().out
    assert "factor 2.0000" in out  # a 1 GiB copy read as 512 MiB
