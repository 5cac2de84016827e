"""Host logic of the coordinate search behind the autotuner, on a synthetic
cost function whose optimum is known."""
from paper_1912_08453_amd import autotune


def _setup(cost):
    state = {}

    def set_value(k, v):
        state[k] = v

    def timer():
        return cost(state)

    return state, set_value, timer


def test_separable_cost_reaches_the_optimum_in_one_pass():
    target = {"a": 3, "b": 16, "c": 0}
    cost = lambda s: sum(abs(s[k] - target[k]) for k in target) + 1.0
    state, set_value, timer = _setup(cost)
    space = {"a": [1, 2, 3, 4], "b": [4, 16, 64], "c": [0, 1]}
    best, table = autotune.coordinate_search(set_value, timer, {"a": 1, "b": 64, "c": 1}, space)
    assert best == target and state == target
    # start + every candidate that differs from the value held when tried
    assert table[0][0] == "start" and len(table) == 1 + 3 + 2 + 1


def test_ties_keep_the_current_value_and_settings_are_left_applied():
    state, set_value, timer = _setup(lambda s: 5.0)
    best, _ = autotune.coordinate_search(set_value, timer, {"x": 2}, {"x": [1, 2, 3]})
    assert best == {"x": 2} and state == {"x": 2}


def test_coupled_cost_improves_with_a_second_pass():
    # the best b depends on a: one pass from a bad start stops short
    cost = lambda s: (s["a"] - 2) ** 2 + (s["b"] - s["a"]) ** 2 + 1.0
    space = {"b": [0, 1, 2], "a": [0, 1, 2]}
    _, set_value, timer = _setup(cost)
    one, _ = autotune.coordinate_search(set_value, timer, {"a": 0, "b": 0}, space)
    state, set_value, timer = _setup(cost)
    two, _ = autotune.coordinate_search(set_value, timer, {"a": 0, "b": 0}, space, passes=3)
    assert one == {"a": 1, "b": 0} and cost(two) < cost(one)


class _BinCtx:
    """Stand-in for a context that, like the library, refuses a lower bin
    bound above the upper one and the reverse."""

    def __init__(self, small, mid):
        self.p = {"lcc_bin_small": small, "lcc_bin_mid": mid}

    def get_param(self, k):
        return self.p[k]

    def set_param(self, k, v):
        if k == "lcc_bin_small" and not 0 <= v <= self.p["lcc_bin_mid"]:
            raise ValueError(k)
        if k == "lcc_bin_mid" and not self.p["lcc_bin_small"] <= v <= 4096:
            raise ValueError(k)
        self.p[k] = v


def test_stored_settings_are_applied_in_an_order_the_bounds_accept(tmp_path, monkeypatch):
    import json
    path = tmp_path / "tuned.json"
    path.write_text(json.dumps({"w": {"settings": {"lcc_bin_small": 300, "lcc_bin_mid": 500}},
                                "v": {"settings": {"lcc_bin_small": 2, "lcc_bin_mid": 6}}}))
    monkeypatch.setattr(autotune, "TUNED_PATH", str(path))
    assert autotune.load_tuned("w", str(path)) == {"lcc_bin_small": 300, "lcc_bin_mid": 500}
    assert autotune.load_tuned("missing", str(path)) == {}
    ctx = _BinCtx(8, 64)
    monkeypatch.setattr(autotune, "load_tuned", lambda w: json.loads(path.read_text())[w]["settings"])
    autotune.apply_tuned(ctx, "w")   # the upper bound has to move first
    assert ctx.p == {"lcc_bin_small": 300, "lcc_bin_mid": 500}
    autotune.apply_tuned(ctx, "v")   # the lower bound has to move first
    assert ctx.p == {"lcc_bin_small": 2, "lcc_bin_mid": 6}


def test_shipped_settings_name_known_parameters():
    from paper_1912_08453_amd import pm
    s = autotune.load_tuned("theta8-s26")
    assert s and set(s) <= set(pm.PM.TUNING)
