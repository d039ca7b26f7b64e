"""Host logic of the autotuner: class keys, representatives, the table."""
from paper_1301_1714_amd import autotune


def test_class_keys_and_representatives():
    assert autotune.system_class(1024, 0.25) == "n10_phi0"
    assert autotune.system_class(1500, 0.35) == "n11_phi1"
    assert autotune.system_class(262144, 0.5) == "n18_phi2"
    rep = autotune.representative("n12_phi1")
    assert rep["n"] == 4096 and 0.3 < rep["phi"] < 0.42
    assert autotune.system_class(rep["n"], rep["phi"]) == "n12_phi1"


def test_table_lookup_and_roundtrip(tmp_path):
    t = autotune.Table({"n10_phi0": {"factor": 1.5, "tile": 8}, "n12_phi2": {"factor": 1.0, "tile": 0, "divisor": 2}})
    assert t.factor(1000, 0.21) == 1.5 and t.tile(1000, 0.21) == 8
    assert t.divisor(1000, 0.21) == 1  # an entry without a divisor: the paper's 27 cells
    assert t.divisor(4000, 0.5) == 2
    assert t.factor(5000, 0.21) == 1.0  # unknown class: the minimum cell, direct detection
    assert t.tile(5000, 0.21) == 0 and t.divisor(5000, 0.21) == 1
    p = str(tmp_path / "a.json")
    t.save(p)
    assert autotune.Table.load(p).entries == t.entries
    assert autotune.Table.load(str(tmp_path / "missing.json")).entries == {}
