"""The oracle's pins against planted mistakes in the oracle.

Each mutant below is the oracle with one plausible slip: a strict
comparison made non-strict, a dropped term, an off-by-one, a swapped order.
It is compiled on its own (the oracle's library is left alone) and run
over the hand-worked cases of tests/golden/; at least one case must
notice.  This is what makes the cases pins rather than a copy of the
oracle's behaviour: a mistake at any of these places would change an
outcome that was worked out by hand.  A second set of mutants (the ring,
the draws, signals, exit times, parking) is run against all of the
oracle's pins."""
import os
import subprocess

import pytest

import oracle
from hand_cases import BOUNDARIES, build, check, load_cases

ORACLE_DIR = os.path.dirname(os.path.abspath(oracle.__file__))
SRC = os.path.join(ORACLE_DIR, "transims_oracle.c")

MUTANTS = [
    ("incentive_non_strict",  # ahead(own) < min(v+1, vmax) read as <=
     "if (own >= want) return -1;", "if (own > want) return -1;"),
    ("incentive_wants_v",  # min(v+1, vmax) read as min(v, vmax)
     "int32_t want = v + 1 < vmax ? v + 1 : vmax;",
     "int32_t want = v < vmax ? v : vmax;"),
    ("side_gap_not_strict",  # ahead(m) > ahead(own) read as >=
     "if (a <= own) continue;", "if (a < own) continue;"),
    ("gap_behind_short_by_one",
     "if (behind(s, l, m, x) < vmax) continue;",
     "if (behind(s, l, m, x) < vmax - 1) continue;"),
    ("side_cell_not_checked",
     "if (*cell(s, l, m, x) >= 0) continue;", "if (0) continue;"),
    ("ties_go_right",
     "int32_t sides[2] = {k - 1, k + 1};", "int32_t sides[2] = {k + 1, k - 1};"),
    ("side_gap_capped_at_vmax_plus_1",
     "for (int32_t c = x + 1; c < s->len[l] && n < s->p.vmax; ++c) {",
     "for (int32_t c = x + 1; c < s->len[l] && n <= s->p.vmax; ++c) {"),
    ("link_start_blocks_the_gap_behind",
     "    if (c >= 0 && *cell(s, l, m, c) >= 0) break;",
     "    if (c < 0 || *cell(s, l, m, c) >= 0) break;"),
    ("conflict_not_resolved",
     "if (j >= 0 && s->dec[j] == m) s->dec[i] = -1;", "if (0) s->dec[i] = -1;"),
    ("desperation_non_strict",
     "behind(s, l, m, x) >= need) return m;",
     "behind(s, l, m, x) > need) return m;"),
    ("desperation_distance_off_by_one",
     "int32_t need = (s->len[l] - 1 - x) / s->p.lc_desp;",
     "int32_t need = (s->len[l] - x) / s->p.lc_desp;"),
    ("desperation_cell_not_checked",
     "if (*cell(s, l, m, x) < 0 && behind(s, l, m, x) >= need) return m;",
     "if (behind(s, l, m, x) >= need) return m;"),
    ("winner_extra_off_by_one",
     "s->extra[i] = s->rear_x[tq] < vmax ? s->rear_x[tq] : vmax;",
     "s->extra[i] = s->rear_x[tq] + 1 < vmax ? s->rear_x[tq] + 1 : vmax;"),
    ("node_key_lane_before_rank",
     "int32_t key = s->rank[l] * 8 + k;", "int32_t key = k * 8 + s->rank[l];"),
    ("candidate_range_includes_vmax",  # len-1-x < vmax read as <=
     "if (i < 0 || s->len[l] - 1 - s->x[i] >= vmax) continue;",
     "if (i < 0 || s->len[l] - 1 - s->x[i] > vmax) continue;"),
    ("loser_keeps_room",  # every candidate, not only the winner, gets extra
     "} else if (key == s->best[tq]) {", "} else {"),
    ("trip_end_without_extra",
     "s->extra[i] = vmax;\n          continue;", "continue;"),
    ("gap_counts_the_vehicle_ahead",
     "gap = c - x - 1;", "gap = c - x;"),
    ("parking_highest_lane_first",
     "for (int32_t k = 0; k < s->lanes[l]; ++k) {\n      int32_t* c = cell(s, l, k, 0);",
     "for (int32_t k = s->lanes[l] - 1; k >= 0; --k) {\n      int32_t* c = cell(s, l, k, 0);"),
    ("parking_one_step_late",
     "if (s->depart[i] > t) continue;", "if (s->depart[i] >= t) continue;"),
    ("crossing_lands_one_cell_short",
     "      x -= s->len[l];\n", "      x -= s->len[l] + 1;\n"),
]


@pytest.fixture(scope="module")
def cases():
    return load_cases() + load_cases(BOUNDARIES)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_each_planted_mistake_fails_a_hand_case(name, old, new, cases,
                                                tmp_path, monkeypatch):
    with open(SRC) as f:
        src = f.read()
    assert src.count(old) == 1, f"{name}: the oracle no longer reads {old!r}"
    c_file, so = tmp_path / "mutant.c", tmp_path / "mutant.so"
    c_file.write_text(src.replace(old, new))
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared",
                           "-I", ORACLE_DIR, "-o", str(so), str(c_file)])
    monkeypatch.setattr(oracle, "_lib", oracle.bind(str(so)))
    noticed = []
    for case in cases:
        o = oracle.OracleSim(build(case))
        try:
            o.step(case["steps"])
            check(case, o.state(), o.stats())
        except (AssertionError, oracle.OracleError):
            noticed.append(case["name"])
        finally:
            o.close()
    assert noticed, f"no hand-worked case notices {name}"


# Slips elsewhere in the oracle (the ring, the draws, signals, exit times,
# parking, the state hash, the step counters): each mutant must make the rest of the oracle's pins fail.  They
# run in a child process that loads the mutant through TRANSIMS_ORACLE_LIB.
RING = "    s->nx[i] = (x + v3) % L;"
WIDE_MUTANTS = [
    ("philox_nine_rounds", "for (int r = 0; r < 10; ++r)", "for (int r = 0; r < 9; ++r)"),
    ("philox_key_bumped_before_round_one", "if (r > 0) {", "if (r >= 0) {"),
    ("philox_words_crossed", "T n0 = hi1 ^ x1 ^ k0;", "T n0 = hi1 ^ x3 ^ k0;"),
    ("draw_key_halves_swapped",
     "uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};",
     "uint32_t key[2] = {(uint32_t)(seed >> 32), (uint32_t)seed};"),
    ("ring_slowdown_uses_lane_change_draw",
     "(uint64_t)draw(s->p.seed, i, t, 1u) < s->p.slow_thr) v3 = v2 - 1;\n"
     "    s->nv[i] = v3;\n" + RING,
     "(uint64_t)draw(s->p.seed, i, t, 0u) < s->p.slow_thr) v3 = v2 - 1;\n"
     "    s->nv[i] = v3;\n" + RING),
    ("ring_slowdown_at_rest",
     "if (v2 > 0 && (uint64_t)draw(s->p.seed, i, t, 1u) < s->p.slow_thr) v3 = v2 - 1;\n"
     "    s->nv[i] = v3;\n" + RING,
     "if (v2 >= 0 && (uint64_t)draw(s->p.seed, i, t, 1u) < s->p.slow_thr) v3 = v2 - 1;\n"
     "    s->nv[i] = v3;\n" + RING),
    ("ring_free_gap_one_short", "int32_t gap = lim;\n", "int32_t gap = lim - 1;\n"),
    ("ring_gap_counts_the_vehicle_ahead", "gap = d - 1;", "gap = d;"),
    ("signal_red_one_step_long",
     "% s->sig_cycle[j]) < s->sig_red[j];", "% s->sig_cycle[j]) <= s->sig_red[j];"),
    ("signal_offset_subtracted", "(int64_t)t + s->sig_off[j]", "(int64_t)t - s->sig_off[j]"),
    ("red_light_ignored", "if (is_red(s, l, s->t)) continue;", "if (0) continue;"),
    ("exit_time_one_late", "s->exit_t[s->route_off[i] + s->rptr[i]] = t;",
     "s->exit_t[s->route_off[i] + s->rptr[i]] = t + 1;"),
    ("lane_change_uses_the_slowdown_draw",
     "draw(s->p.seed, i, t, 0u) >= s->p.lc_thr",
     "draw(s->p.seed, i, t, 1u) >= s->p.lc_thr"),
    ("hash_ignores_route_pointer",
     "return orc_mix64(h ^ (uint64_t)(uint32_t)rptr);", "return orc_mix64(h);"),
    ("hash_ignores_speed",
     "((uint64_t)(uint32_t)v << 8) |", "((uint64_t)0 << 8) |"),
    ("hash_ignores_link",
     "((uint64_t)(uint32_t)link << 32);", "((uint64_t)0 << 32);"),
    ("hash_xor_not_sum",
     "      h += vehicle_hash(i, st, cur_link(s, i),",
     "      h ^= vehicle_hash(i, st, cur_link(s, i),"),
    ("c_occ_counts_empty_lanes",
     "      if (s->lead_id[q] >= 0) s->st.c_occ += s->len[l];\n"
     "      else s->rear_x[q] = s->len[l];",
     "      s->st.c_occ += s->len[l];\n"
     "      if (s->lead_id[q] < 0) s->rear_x[q] = s->len[l];"),
    ("crossing_not_counted", "s->st.crossings++;", ";"),
    ("insertion_not_counted", "s->st.insertions++;", ";"),
    ("lane_change_counted_twice", "s->st.lane_changes++;", "s->st.lane_changes += 2;"),
    ("exit_not_counted", "s->st.exits++;", ";"),
    ("winner_room_from_the_front_vehicle",
     "if (s->rear_x[q] < 0 || s->x[i] < s->rear_x[q]) s->rear_x[q] = s->x[i];",
     "if (s->rear_x[q] < 0 || s->x[i] > s->rear_x[q]) s->rear_x[q] = s->x[i];"),
    ("parking_queue_by_id_only",
     "  if (g_depart[i] != g_depart[j]) return g_depart[i] < g_depart[j] ? -1 : 1;\n",
     ""),
    ("parking_into_an_occupied_cell",
     "      if (*c >= 0) continue;\n      *c = i;\n      s->status[i] = ORC_ACTIVE;",
     "      *c = i;\n      s->status[i] = ORC_ACTIVE;"),
]

PIN_FILES = ["test_oracle_hash.py", "test_oracle_counters.py",
             "test_oracle_philox.py",
             "test_oracle_ring.py", "test_oracle_network.py",
             "test_oracle_signals.py"]


@pytest.mark.parametrize("name,old,new", WIDE_MUTANTS,
                         ids=[m[0] for m in WIDE_MUTANTS])
def test_each_planted_mistake_fails_a_pin(name, old, new, tmp_path):
    import sys
    with open(SRC) as f:
        src = f.read()
    assert src.count(old) == 1, f"{name}: the oracle no longer reads {old!r}"
    c_file, so = tmp_path / "mutant.c", tmp_path / "mutant.so"
    c_file.write_text(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                           "-I", ORACLE_DIR, "-o", str(so), str(c_file)])
    here = os.path.dirname(os.path.abspath(__file__))
    env = dict(os.environ, TRANSIMS_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q",
                        "-p", "no:cacheprovider", "-m", "not gpu"] +
                       [os.path.join(here, f) for f in PIN_FILES],
                       cwd=os.path.dirname(here), env=env,
                       capture_output=True, text=True, timeout=600)
    # 1: a pin failed; < 0: a pin failed or the mutant corrupted memory and
    # the child died of it (either way the mistake was noticed)
    assert r.returncode == 1 or r.returncode < 0, \
        f"no pin notices {name} (exit {r.returncode}):\n{r.stdout[-2000:]}"
