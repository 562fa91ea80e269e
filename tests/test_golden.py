"""The paper's printed phase-boundary values (tests/golden/paper_phase_points.json):
every entry carries its citation, and the values are consistent with the
phase diagram they describe: both melting lines fall from their starting
points to the triple point (T_tp < T_m(15 GPa) < T_m(0 GPa)), and the
cd/beta-tin line falls in pressure from 400 K to the triple point
(P_tp < P_coex(400 K))."""
import json
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_phase_points.json")


def test_entries_are_cited():
    data = json.load(open(GOLDEN))
    for key, entry in data.items():
        if key == "description":
            continue
        assert "section" in entry["cite"], key


def test_values_describe_one_phase_diagram():
    d = json.load(open(GOLDEN))
    T0, T15 = d["melting_point_cd_0GPa"]["value"], d["melting_point_beta_tin_15GPa"]["value"]
    Tt, Pt = d["triple_point"]["T"], d["triple_point"]["P"]
    Pc = d["coexistence_pressure_cd_beta_tin_400K"]["value"]
    assert 400.0 < Tt < T15 < T0
    assert 0.0 < Pt < 15.0 and Pt < Pc
