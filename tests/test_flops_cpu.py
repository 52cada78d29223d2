"""Algorithmic work accounting and autotune bucketing (CPU)."""
import numpy as np

from paper_2503_18356_amd import flops, inputs


def test_multiplication_chains():
    # Shortest addition chains: q^1..q^6 need 0, 1, 2, 2, 3, 3 multiplies.
    assert list(flops.CHAIN[1:7]) == [0, 1, 2, 2, 3, 3]


def test_rhs_and_step_flops():
    n = np.array([[1, 6], [3, 2]], np.uint8)  # 2 edges x 2 sets
    f = flops.rhs_flops_per_set(4, n)
    assert list(f) == [(6 + 0) + (6 + 2) + 12, (6 + 3) + (6 + 1) + 12]
    s = flops.step_flops_per_set(4, n)
    assert list(s) == [6 * f[0] + 56 * 4, 6 * f[1] + 56 * 4]
    steps = np.array([10, 20, 5, 5])  # 2 sets x 2 ICs
    assert flops.credited(4, n, 2, steps) == s[0] * 30 + s[1] * 10


def test_algorithmic_bytes():
    b = flops.algorithmic_bytes(10, 25, 100, 10, 4)
    assert b == 100 * ((20 + 50) * 4 + 25) + 10 * 40 + 1000 * (40 + 17)


def test_autotune_bucket_rounds_up():
    from paper_2503_18356_amd.autotune import bucket
    t = inputs.erdos_renyi(10, 25, 1002)
    b = bucket(t)
    assert b.startswith("N16_E32_D")


def test_refine_batch_keeps_only_switches_that_pay():
    # refine_batch with a synthetic batch time: switching group A saves 5 %,
    # group B costs 3 %, group C saves 0.4 % (below the 1 % margin).
    from paper_2503_18356_amd.autotune import Autotuner
    default = [(0, 0)] * 6
    tuned = [(4, 2), (4, 2), (16, 1), (16, 1), (8, 4), (8, 4)]
    effect = {0: -0.05, 2: 0.03, 4: -0.004}
    calls = []

    def run(knobs):
        calls.append(list(knobs))
        t = 1.0
        for first, d in effect.items():
            if knobs[first] != (0, 0):
                t *= 1.0 + d
        return t

    knobs, log = Autotuner.refine_batch(run, default, tuned, [[0, 1], [2, 3], [4, 5]])
    assert knobs == [(4, 2), (4, 2), (0, 0), (0, 0), (0, 0), (0, 0)]
    assert [r["kept"] for r in log] == [True, True, False, False]
    # One untimed call and two timed ones per trial: the start and three groups.
    assert len(calls) == 4 * 3
    # A group whose tuned knobs equal the current ones is not tried again.
    knobs2, log2 = Autotuner.refine_batch(run, default, default, [[0, 1]])
    assert knobs2 == default and len(log2) == 1


def test_autotune_cache_that_cannot_be_read_is_dropped(tmp_path):
    # A cut-short or hand-edited cache file starts an empty cache (measured
    # again on use) instead of failing; a readable one is kept.
    import json
    from paper_2503_18356_amd.autotune import Autotuner
    bad = tmp_path / "cut.json"
    bad.write_text('{"gfx950|fp32|N16_E32_D4": {"lanes": 4,')
    assert Autotuner(str(bad)).cache == {}
    wrong = tmp_path / "list.json"
    wrong.write_text("[1, 2]")
    assert Autotuner(str(wrong)).cache == {}
    good = tmp_path / "good.json"
    entry = {"k": {"lanes": 4, "refill_min": 2, "solves_per_s": 1.0}}
    good.write_text(json.dumps(entry))
    assert Autotuner(str(good)).cache == entry
