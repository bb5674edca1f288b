"""Autotuner selection logic and signatures (no device)."""
from paper_1906_08148_amd import autotune


def test_candidates_add_quads_from_leaf_64():
    c = autotune.candidates((32, 64, 128), (0, 1))
    assert c == [(32, 0, 0), (32, 1, 0), (64, 0, 0), (64, 1, 0), (128, 0, 0), (128, 1, 0), (64, 1, 1), (128, 1, 1)]
    assert autotune.candidates((16, 32), (0,)) == [(16, 0, 0), (32, 0, 0)]
    assert autotune.candidates((64,), (0,), quads=False) == [(64, 0, 0)]


def test_choose_picks_fastest_and_breaks_ties_by_smaller_leaf():
    times = {(32, 0, 0): 3.0, (32, 1, 0): 2.0, (64, 0, 0): 1.0, (64, 1, 0): 1.0, (128, 0, 0): 5.0,
             (64, 1, 1): 1.0}
    best, table = autotune.choose(list(times), lambda l, t, q: (times[(l, t, q)], 0.0))
    assert best == (64, 0, 0)
    assert len(table) == len(times)
    assert {(r["leaf"], r["tile"], r["quad"]) for r in table} == set(times)
    assert all(r["admissible"] for r in table)
    # quads win when they are faster
    times[(64, 1, 1)] = 0.5
    assert autotune.choose(list(times), lambda l, t, q: (times[(l, t, q)], 0.0))[0] == (64, 1, 1)


def test_choose_rejects_candidates_over_the_error_budget():
    """The fastest candidate breaks the budget: the fastest admissible one
    wins; an error exactly on the budget is admissible."""
    meas = {(32, 0, 0): (3.0, 1e-7), (64, 0, 0): (1.0, 5e-5), (64, 1, 0): (1.5, 1e-5), (128, 0, 0): (0.5, 2e-3),
            (256, 0, 0): (2.0, 1e-6)}
    best, table = autotune.choose(list(meas), lambda l, t, q: meas[(l, t, q)], budget=1e-5)
    assert best == (64, 1, 0)
    rej = {(r["leaf"], r["tile"], r["quad"]) for r in table if not r["admissible"]}
    assert rej == {(64, 0, 0), (128, 0, 0)}
    # a tighter budget moves the choice; none admissible gives None
    assert autotune.choose(list(meas), lambda l, t, q: meas[(l, t, q)], budget=1e-6)[0] == (256, 0, 0)
    best, table = autotune.choose(list(meas), lambda l, t, q: meas[(l, t, q)], budget=1e-9)
    assert best is None and not any(r["admissible"] for r in table)
    # an unknown error never meets a budget
    assert autotune.choose([(64, 0, 0)], lambda l, t, q: (1.0, None), budget=1.0)[0] is None


def test_signature_buckets():
    a = autotune.signature("3d", 32768, 1.0, 1e-6, 1, 1)
    b = autotune.signature("3d", 30000, 0.9, 2e-6, 1, 1)
    c = autotune.signature("3d", 65536, 1.0, 1e-6, 1, 1)
    assert a == b and a != c
    assert autotune.signature("1d", 2048, 0.5, 0.0, 0, 0)[3] == -999
