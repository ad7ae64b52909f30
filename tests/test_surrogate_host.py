"""Host-side checks of the surrogate network's bookkeeping (no GPU)."""
from types import SimpleNamespace

from paper_1904_03618_amd import surrogate as S


def _net(shape):
    c1, c2, c3, c4 = S.WIDTHS
    spec = [("e1a", S.CIN, c1), ("e1b", c1, c1), ("e2a", c1, c2), ("e2b", c2, c2), ("e3a", c2, c3),
            ("e3b", c3, c3), ("e4a", c3, c4), ("e4b", c4, c4), ("d3a", c4 + c3, c3), ("d3b", c3, c3),
            ("d2a", c3 + c2, c2), ("d2b", c2, c2), ("d1a", c2 + c1, c1), ("d1b", c1, c1)]
    layers = [SimpleNamespace(name=n, ci=ci, co=co, k=3) for n, ci, co in spec]
    layers.append(SimpleNamespace(name="head", ci=c1, co=S.NF, k=1))
    return SimpleNamespace(shape=shape, layers=layers)


def test_flop_count_by_hand():
    """The 128 x 128 x 512 box, counted layer by layer: 27-tap convolutions at
    the four levels (positions P0 / 8^l), the first layer on its 4 real input
    channels, and the 1x1x1 head."""
    P0 = 512 * 128 * 128
    conv = [(0, 4, 16), (0, 16, 16), (1, 16, 32), (1, 32, 32), (2, 32, 64), (2, 64, 64), (3, 64, 128),
            (3, 128, 128), (2, 192, 64), (2, 64, 64), (1, 96, 32), (1, 32, 32), (0, 48, 16), (0, 16, 16)]
    fwd = sum(2 * (P0 >> 3 * l) * 27 * ci * co for l, ci, co in conv) + 2 * P0 * 16 * 4
    first = 2 * P0 * 27 * 4 * 16
    got_fwd, got_train = S.flops(_net((1, 512, 128, 128)))
    assert got_fwd == fwd
    # training: forward + weight gradients of every layer + data gradients of all but the first
    assert got_train == 3 * fwd - first
    assert abs(fwd / 1e9 - 1110.0) < 0.1


def test_selection_key_prefers_bounded_drift_then_jumps():
    """The validation key of the surrogate pipeline, on hand-made run
    summaries: a candidate counts as within the gate only if every validation
    case keeps its largest jump and its end within 1 l.u.; among those the
    fewest jumps of any case decide (so a trust that is safe on both cases but
    takes fewer jumps loses to one that is safe and takes more), and among the
    rest the worst final error decides before the jumps."""
    from paper_1904_03618_amd import surrogate_rt as R

    def run(jumps, largest, final):
        return dict(jumps=jumps, max_jump_error=largest, final_front_error=final)

    safe23 = [run(23, 0.51, 0.41), run(23, 0.43, 0.37)]
    safe31 = [run(31, 0.90, 0.95), run(32, 0.99, 0.97)]
    one_side = [run(32, 0.91, 0.92), run(33, 3.22, 3.23)]     # fine on one amplitude only
    drift_small = [run(31, 1.35, 1.33), run(31, 1.73, 1.75)]
    drift_large = [run(33, 4.96, 5.04), run(33, 3.40, 3.45)]
    nan_end = [run(33, 0.5, float("nan")), run(33, 0.5, 0.5)]
    keys = {name: R.score(v) for name, v in dict(safe23=safe23, safe31=safe31, one_side=one_side,
                                                 drift_small=drift_small, drift_large=drift_large,
                                                 nan_end=nan_end).items()}
    order = sorted(keys, key=keys.get, reverse=True)
    assert order == ["safe31", "safe23", "drift_small", "one_side", "drift_large", "nan_end"]
    # the unsafe candidates all rank below every safe one
    assert all(keys[s] > keys[u] for s in ("safe23", "safe31") for u in ("one_side", "drift_small", "nan_end"))
