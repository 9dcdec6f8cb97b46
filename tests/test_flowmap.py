"""Host logic of the flow-state map (paper_2211_05009_amd/flowmap.py) and the
Table 3 fixture."""
import json
import os

from paper_2211_05009_amd import flowmap as FM

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_tables.json")


def test_observing_points_of_sec_3_3():
    assert FM.observing_point(0.4) == (0.5, 0.2)
    assert FM.observing_point(0.5) == FM.observing_point(0.6) == (0.5, 0.3)
    for ar in (0.7, 0.8, 1.0, 1.2, 1.5, 2.0):
        assert FM.observing_point(ar) == (0.5, 0.5)


def test_fig17_grid():
    assert FM.FIG17_RE == (4000.0, 4500.0, 5000.0, 5500.0, 6000.0, 6500.0, 7000.0, 7500.0,
                           8000.0)
    assert len(FM.FIG17_AR) == 17 and FM.FIG17_AR[0] == 0.4 and FM.FIG17_AR[-1] == 2.0
    assert all(abs(b - a - 0.1) < 1e-12 for a, b in zip(FM.FIG17_AR, FM.FIG17_AR[1:]))


def test_table3_fixture():
    t3 = json.load(open(GOLDEN))["table3"]
    assert t3["re"] == [4000, 4500, 5000, 5500, 6000, 6500, 7000, 7500, 8000]
    rows = {k: v for k, v in t3.items() if k not in ("note", "re")}
    assert len(rows) == 11 and all(len(v) == 9 for v in rows.values())
    assert rows["0.6"][6] == 22.13 and rows["1.2"][4] == 31.16 and rows["0.4"][8] == 13.14


def test_config_cli_usage():
    """The per-workload runner rejects unknown configurations without
    touching the device."""
    from paper_2211_05009_amd import configs
    assert configs.main([]) == 2 and configs.main(["9"]) == 2 and configs.main(["x"]) == 2
    assert sorted(configs.RUNS) == [1, 2, 3, 4, 5]
