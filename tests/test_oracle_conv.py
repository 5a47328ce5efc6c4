"""Pins of the convolution oracle (the implicit-GEMM extension's result).

* pure-loop brute force on tiny cases (padding, stride, dilation);
* a 1 x 1 filter with stride 1 and no padding is the GEMM of the pixels by the
  channels (checked against the GEMM oracle);
* a delta filter copies (shifted) input channels;
* torch's float64 CPU convolution (an independent library routine: the
  oracle itself contracts tap by tap with matrix products);
* integer inputs give integer outputs equal to the loops'.
"""
import itertools

import numpy as np
import pytest

from oracle import conv as OC
from oracle import gemm as og


def _rand(shape, seed, integer=False):
    g = np.random.default_rng(seed)
    return g.integers(-2, 3, shape).astype(np.float64) if integer else g.standard_normal(shape)


@pytest.mark.parametrize("pad,stride,dil", [((0, 0), (1, 1), (1, 1)), ((1, 1), (1, 1), (1, 1)), ((1, 0), (2, 1), (1, 1)),
                                           ((2, 1), (1, 2), (2, 1)), ((0, 2), (3, 2), (1, 2))])
def test_brute_force_tiny(pad, stride, dil):
    x = _rand((2, 5, 6, 3), 1)
    w = _rand((4, 3, 2, 3), 2)
    assert np.allclose(OC.conv2d_f64(x, w, pad, stride, dil), OC.conv2d_loops(x, w, pad, stride, dil),
                       rtol=1e-13, atol=1e-13)


def test_one_by_one_is_the_gemm():
    x = _rand((2, 7, 5, 16), 3)
    w = _rand((9, 1, 1, 16), 4)
    y = OC.conv2d_f64(x, w)
    ref = og.gemm_f64(x.reshape(-1, 16), w.reshape(9, 16).T.copy())
    assert np.allclose(y.reshape(-1, 9), ref, rtol=1e-13, atol=1e-13)


def test_delta_filter_shifts_channels():
    x = _rand((1, 6, 7, 4), 5)
    w = np.zeros((4, 3, 3, 4))
    for k in range(4):
        w[k, 2, 0, (k + 1) % 4] = 1.0        # tap (r, s) = (2, 0), channel k + 1 -> k
    y = OC.conv2d_f64(x, w, pad=(1, 1))
    # y[p, q, k] = x[p + 1, q - 1, k + 1] where inside the image, else 0
    for p, q, k in itertools.product(range(6), range(7), range(4)):
        h, ww = p + 1, q - 1
        want = x[0, h, ww, (k + 1) % 4] if 0 <= h < 6 and 0 <= ww < 7 else 0.0
        assert y[0, p, q, k] == want


def test_torch_conv2d_f64():
    torch = pytest.importorskip("torch")
    for (N, H, W, C, K, R, S), pad, stride, dil in [((2, 9, 11, 8, 5, 3, 3), (1, 1), (1, 1), (1, 1)),
                                                    ((1, 12, 7, 16, 4, 5, 3), (2, 0), (2, 1), (1, 2)),
                                                    ((3, 6, 6, 4, 6, 1, 1), (0, 0), (2, 2), (1, 1))]:
        x = _rand((N, H, W, C), N + H)
        w = _rand((K, R, S, C), K + R)
        ref = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2), torch.from_numpy(w).permute(0, 3, 1, 2),
                                         stride=stride, padding=pad, dilation=dil).permute(0, 2, 3, 1).numpy()
        assert np.allclose(OC.conv2d_f64(x, w, pad, stride, dil), ref, rtol=1e-12, atol=1e-12)


def test_integer_exact_and_alpha_beta():
    x = _rand((1, 5, 5, 3), 7, integer=True)
    w = _rand((2, 3, 3, 3), 8, integer=True)
    y0 = _rand((1, 5, 5, 2), 9, integer=True)
    got = OC.conv2d_f64(x, w, (1, 1), alpha=2.0, beta=-1.0, y=y0)
    want = 2.0 * OC.conv2d_loops(x, w, (1, 1)) - y0
    assert np.array_equal(got, want)


def test_planted_mistake_is_caught():
    """A flipped filter (convolution instead of correlation) differs from the loops."""
    x = _rand((1, 6, 6, 2), 10)
    w = _rand((3, 3, 3, 2), 11)
    flipped = w[:, ::-1, ::-1, :]
    assert not np.allclose(OC.conv2d_f64(x, flipped, (1, 1)), OC.conv2d_loops(x, w, (1, 1)))
