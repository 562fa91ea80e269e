"""The paper's printed phase-boundary values (tests/golden/paper_phase_points.json):
every entry carries its citation, and the values are consistent with the
phase diagram they describe (the triple point lies between the cd/liquid
melting point at 0 GPa and the beta-tin/liquid one at 15 GPa, and below the
cd/beta-tin coexistence pressure at 400 K, since that line has dP/dT < 0)."""
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
    assert T15 < Tt + 200 and Tt < T0 and Tt > 400.0
    assert 0.0 < Pt < 15.0 and Pt < Pc
