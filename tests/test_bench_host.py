"""Host-side helpers of bench.py: the kernel-source digest ignores comments,
kernel kinds map to their families, and the all-cores oracle rate counts
exactly the updates of the scenarios it ran."""
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
