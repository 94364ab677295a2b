"""Host logic of the work-partition autotuner (no GPU): the coordinate
descent, the validity rule, the shape-class key and the JSON cache."""
import itertools

from paper_1910_02371_amd import autotune as AT


def test_descent_finds_separable_minimum():
    # separable cost with a known best setting; every evaluated candidate
    # must be valid, and no setting is evaluated twice
    best = {"chunk": 512, "gram_piece": 8192, "gram_light": 1024, "gram_waves": 2,
            "solve_wgs": 8}
    seen = []

    def cost(t):
        seen.append(tuple(sorted(t.items())))
        return 10.0 + sum(0.0 if t[k] == best[k] else 1.0 + AT.KNOBS[k].index(t[k])
                          for k in t)

    start = {"chunk": 1024, "gram_piece": 4096, "gram_light": 512, "gram_waves": 4,
             "solve_wgs": 0}
    got, t, trials = AT.coordinate_descent(start, cost)
    assert got == best and t == 10.0
    assert all(AT.valid(dict(s)) for s in seen)
    assert len(seen) == len(set(seen))
    assert len(trials) == len(seen)


def test_descent_keeps_start_without_gain_and_respects_validity():
    start = {"chunk": 1024, "gram_piece": 2048, "gram_light": 512, "gram_waves": 4,
             "solve_wgs": 0}
    got, _, trials = AT.coordinate_descent(start, lambda t: 5.0)
    assert got == start
    # gram_light 1024 > gram_piece 2048 is fine; gram_piece 2048 with light
    # 1024 valid; an invalid pair is never tried
    for t, _ in trials:
        assert t["gram_light"] <= t["gram_piece"]
    # a 0.5% gain is below min_gain (1%) and does not move the setting
    got, _, _ = AT.coordinate_descent(start, lambda t: 5.0 if t == start else 4.98)
    assert got == start


def test_shape_key_and_cache(tmp_path):
    k1 = AT.shape_key((480189, 17770, 2182), 100_000_000, 64, "f32")
    k2 = AT.shape_key((480189, 17770, 2182), 100_000_000, 64, "f32")
    # log2 of 1e8 nonzeros and of the mean degrees 208, 5627, 45830
    assert k1 == k2 == "f32_R64_m27_d8_d12_d15"
    assert AT.shape_key((480189, 17770, 2182), 100_000_000, 64, "bf16") != k1
    p = str(tmp_path / "sub" / "tuning.json")
    assert AT.load_cache(p) == {}
    AT.save_cache(p, {k1: {"tuning": {"chunk": 512}, "ms": 1.0}})
    assert AT.load_cache(p)[k1]["tuning"]["chunk"] == 512


def test_knob_values_are_accepted_by_the_library_rules():
    # the C ABI accepts chunk 512/1024/2048, gram_piece 1024..65536,
    # gram_waves 2/4/8, 0 <= gram_light <= gram_piece and solve_wgs 0..64
    for c, p, l, w, sw in itertools.product(*AT.KNOBS.values()):
        assert c in (512, 1024, 2048) and 1024 <= p <= 65536 and w in (2, 4, 8)
        assert 0 <= sw <= 64
        assert 0 <= l
