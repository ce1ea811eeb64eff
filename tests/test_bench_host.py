"""Host-side helpers of bench.py: the kernel-source digest ignores comments,
kernel kinds map to their families, the all-cores oracle rate counts
exactly the updates of the scenarios it ran, the roofline object prices
the algorithmic bytes per launch against the launch time and reports
measured traffic only where it was measured, and more than one GPU is
refused."""
import os
import sys

import oracle
from paper_cs_0105004_amd import scenarios as S

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_code_only_ignores_comments_and_blank_lines():
    a = "int f(int x) {\n  return x + 1;\n}\n"
    b = ("// helper\nint f(int x) {  // one more\n\n  /* the sum\n"
         "     of two */\n  return x + 1;   \n}\n")
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(a.replace("1", "2"))


def test_digests_cover_every_family():
    d = {f: bench.kernel_digest(f) for f in bench.KERNEL_SOURCES}
    assert len(set(d.values())) == len(d)
    assert all(len(v) == 16 for v in d.values())
    assert bench.family_of(["front", "back"]) == "front_back"
    assert bench.family_of(["step"]) == "step"
    assert bench.family_of(["ring"]) == "ring"


def test_all_cores_oracle_counts_every_update():
    scens = [S.portland_like(scale=0.01, T=120, depart_max=60, seed=s)
             for s in (1, 2, 3)]
    r = bench.oracle_all_cores(scens, budget_s=60.0, max_workers=3)
    want = 0
    for sc in scens:
        o = oracle.OracleSim(sc)
        o.step(sc.T)
        want += o.stats()["veh_updates"]
    assert r["cores"] == min(3, bench.host_info()["usable_cores"])
    if r["cores"] == 3:
        assert r["vehicle_updates"] == want
    assert r["value"] > 0 and r["kind"] == "oracle"
    assert {"cpu_model", "nproc", "usable_cores"} <= set(r["host"])


def test_more_than_one_gpu_is_refused():
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=root,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_split_between_the_kernels():
    st = {"c_occ": 1000, "veh_updates": 70, "crossings": 5, "exits": 2,
          "insertions": 3}
    step = 2 * 1000 + 8 * 70 + 16 * 7 + 8 * 3
    assert bench.algorithmic_bytes("step", st) == step
    assert (bench.algorithmic_bytes("front", st) +
            bench.algorithmic_bytes("back", st)) == step
    assert bench.algorithmic_bytes("ring", st) == 2 * 1000 + 8 * 70


def test_roofline_from_event_time_and_traffic_validity(monkeypatch):
    st = {"c_occ": 4_000_000, "veh_updates": 100_000, "crossings": 3_000,
          "exits": 500, "insertions": 600}
    kt = {"front": (0, 0.0), "back": (0, 0.0), "ring": (0, 0.0),
          "step": (100, 1.3)}
    table = {bench.kernel_digest("step"): {"portland": [
        {"window": (1800, 100), "tiles": (0, 0), "bytes_per_launch": 7.5e6}]}}
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", table)
    r = bench.roofline_from(kt, [st, st], region_ms=1.2, workload="portland",
                            window=(1800, 100))
    per_launch = bench.algorithmic_bytes("step", {k: 2 * v for k, v in st.items()}) / 100
    assert r["algorithmic_bytes_per_launch"] == per_launch
    assert r["avg_launch_us"] == 12.0  # the region's time per launch
    assert r["achieved"] == per_launch / 12e-6 / 1e9
    assert r["frac"] == r["achieved"] / 8000.0 and r["bound"] == "hbm"
    # traffic only for the workload, window and tiles it was measured on
    assert r["traffic"] == 7.5e6 and "window" in r["traffic_note"]
    for kw in ({"window": (1800, 20)}, {"window": (1750, 100)},
               {"window": (1800, 100), "tiles": (8, 1024)},
               {"window": None}):
        got = bench.roofline_from(kt, [st], region_ms=1.2,
                                  workload="portland", **kw)
        assert got["traffic"] is None and got["traffic_note"].startswith("null")
    # and only while the kernel sources are the ones it was measured on
    monkeypatch.setattr(bench, "kernel_digest", lambda fam="step": "0" * 16)
    assert bench.roofline_from(kt, [st], region_ms=1.2, workload="portland",
                               window=(1800, 100))["traffic"] is None


def test_roofline_prices_the_two_kernels_together():
    st = {"c_occ": 10_000, "veh_updates": 900, "crossings": 40, "exits": 4,
          "insertions": 9}
    kt = {"front": (50, 2.0), "back": (50, 1.5), "ring": (0, 0.0),
          "step": (0, 0.0)}
    r = bench.roofline_from(kt, [st], region_ms=5.0)
    assert r["kernel"] == "k_front + k_back"
    assert r["algorithmic_bytes_per_launch"] == bench.algorithmic_bytes("step", st) / 50
    assert r["avg_launch_us"] == 100.0
    # without an event time of the region: the dominant kernel alone
    r = bench.roofline_from(kt, [st])
    assert r["kernel"] == "k_front" and r["avg_launch_us"] == 40.0
    assert r["algorithmic_bytes_per_launch"] == bench.algorithmic_bytes("front", st) / 50


def test_cpu_window_times_the_window_after_its_own_advance():
    sc = S.portland_like(scale=0.01, T=200, depart_max=100, seed=4)
    base, end = bench.cpu_window(sc, 120, 20, budget_s=0.05, max_reps=3)
    o = oracle.OracleSim(sc)
    o.step(140)
    assert end == o.stats()  # counters from t = 0 to the window's end
    assert base["kind"] == "oracle" and base["cores"] == 1
    assert base["value"] > 0 and "steps 120..139" in base["sample"]
