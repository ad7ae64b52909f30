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
