"""Selection logic of the sweep autotuner (no GPU: measurements injected)."""
import json

import pytest

from paper_1910_10863_amd import autotune as at


def _fake(table):
    calls = []

    def measure(leaf, p):
        calls.append((leaf, p))
        return table[(leaf, p)]
    return measure, calls


def test_picks_cheapest_accurate_candidate():
    # err falls with p; larger leaves cost more setup but apply faster
    table = {}
    for leaf, (ts, ta0) in {16: (1.0, 0.30), 32: (1.5, 0.20), 64: (3.0, 0.18)}.items():
        for p in at.P_CANDIDATES:
            table[(leaf, p)] = (10.0 ** (-p / 2.0), ts, ta0 + 0.002 * p)
    measure, calls = _fake(table)
    ch = at.autotune({"g": 1}, 4.0, [0.0, 0.1], target_err=1e-10, measure=measure, iters=30)
    # p = 20 is the first order with 10^-10; cost 1.5 + 30 * 0.24 = 8.7 at leaf 32 is the least
    assert (ch.leaf_max, ch.p) == (32, 20)
    # at every leaf size the orders stop at the first accurate one
    assert (16, 24) not in calls and (32, 24) not in calls and (64, 24) not in calls
    assert all(t.ok == (t.err <= 1e-10) for t in ch.trials)


def test_raises_when_nothing_is_accurate():
    measure, _ = _fake({(l, p): (1.0, 1.0, 1.0) for l in at.LEAF_CANDIDATES for p in at.P_CANDIDATES})
    with pytest.raises(RuntimeError):
        at.autotune({"g": 2}, 4.0, [0.0], measure=measure)


def test_cache_round_trip(tmp_path):
    table = {(l, p): (1e-12, 1.0 + l / 100.0, 0.1) for l in at.LEAF_CANDIDATES for p in at.P_CANDIDATES}
    measure, calls = _fake(table)
    path = str(tmp_path / "tune.json")
    ch = at.autotune({"g": 3}, 2.0, [0.0], cache=path, measure=measure)
    assert (ch.leaf_max, ch.p) == (16, 12)
    n = len(calls)
    ch2 = at.autotune({"g": 3}, 2.0, [0.0], cache=path, measure=measure)
    assert len(calls) == n and (ch2.leaf_max, ch2.p) == (16, 12)
    assert len(json.load(open(path))) == 1


def test_tie_prefers_larger_p():
    ts = [at.Trial(32, 16, 1e-11, 1.0, 0.1, 4.0, True), at.Trial(32, 20, 1e-13, 1.0, 0.1, 4.0, True)]
    assert at.select(ts).p == 20


def test_frequency_bands_get_their_own_order():
    """The truncation error grows with k (Theorems 1-2; Sec. 4 closes with p
    growing with frequency): with an error model err = (k/32)^p each band is
    tuned at its largest frequency and the higher bands get larger p."""
    def factory(ka):
        def measure(leaf, p):
            return ((ka / 32.0) ** p, 1.0, 0.1 + 0.001 * p + 0.01 * leaf / 16)
        return measure
    kas = [0.2 + 0.25 * i for i in range(32)]
    bands = at.autotune_bands({"g": 4}, kas, [0.0], n_bands=4, target_err=1e-10, measure_factory=factory)
    assert [len(b) for b, _ in bands] == [8, 8, 8, 8]
    assert sorted(sum((b for b, _ in bands), [])) == sorted(kas)
    ps = [ch.p for _, ch in bands]
    assert ps == sorted(ps) and ps[0] < ps[-1]
    for band, ch in bands:
        assert (max(band) / 32.0) ** ch.p <= 1e-10
