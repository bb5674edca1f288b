"""Autotuner selection logic and signatures (no device)."""
from paper_1906_08148_amd import autotune


def test_choose_picks_fastest_and_breaks_ties_by_smaller_leaf():
    times = {(32, 0): 3.0, (32, 1): 2.0, (64, 0): 1.0, (64, 1): 1.0, (128, 0): 5.0}
    best, table = autotune.choose(list(times), lambda l, t: times[(l, t)])
    assert best == (64, 0)
    assert len(table) == len(times)
    assert {(r["leaf"], r["tile"]) for r in table} == set(times)


def test_signature_buckets():
    a = autotune.signature("3d", 32768, 1.0, 1e-6, 1, 1)
    b = autotune.signature("3d", 30000, 0.9, 2e-6, 1, 1)
    c = autotune.signature("3d", 65536, 1.0, 1e-6, 1, 1)
    assert a == b and a != c
    assert autotune.signature("1d", 2048, 0.5, 0.0, 0, 0)[3] == -999
