"""The autotuner's search (successive halving) finds the minimum of a
noiseless cost and keeps halving until one candidate is left."""
from paper_2605_27323_amd import autotune


def test_successive_halving_picks_minimum():
    cands = [{"a": a, "b": b} for a in range(7) for b in range(5)]
    calls = []

    def measure(c, reps):
        calls.append(reps)
        return (c["a"] - 4) ** 2 + 0.5 * abs(c["b"] - 1) + 1.0

    best, hist = autotune.successive_halving(cands, measure)
    assert best == {"a": 4, "b": 1}
    assert len(hist) == 5 and max(calls) == 16  # 35 -> 17 -> 8 -> 4 -> 2 -> 1


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "cache.json")
    autotune._store(p, "k", {"block": 128})
    assert autotune._load(p)["k"] == {"block": 128}
