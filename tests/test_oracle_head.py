"""Pins of the Gaussian-primary-head and Y-PSNR oracle (oracle/head.py)
against values the definitions fix independently: constructed activations
with exact closed forms, the covariance the Cholesky factor must reproduce,
the geometry of the reference grid, finite differences of the forward, and
the BT.601 luma of known colours."""
import math

import numpy as np
import pytest

from oracle import head as Hd


def _raw(n, seed, spread=2.0):
    rng = np.random.default_rng(seed)
    return (rng.normal(0, spread, n), rng.normal(0, spread, (n, 3)),
            rng.normal(0, spread, (n, 2)), rng.normal(0, spread, n),
            rng.normal(0, 0.5, (n, 2)))


@pytest.mark.parametrize("H,W,g", [(1, 1, 1), (3, 5, 1), (4, 3, 4), (2, 7, 3), (5, 5, 2)])
def test_reference_grid_geometry(H, W, g):
    P = Hd.reference_positions(H, W, g)
    assert P.shape == (g * g * H * W, 2)
    # row-major: x runs fastest, spacing 1/g on both axes
    xs = P[: g * W, 0]
    assert np.allclose(np.diff(xs), 1.0 / g, rtol=0, atol=1e-15)
    assert np.allclose(P[:: g * W, 1][1:] - P[:: g * W, 1][:-1], 1.0 / g, rtol=0, atol=1e-15)
    # symmetric about the image centre, half a cell inside the image edges
    assert np.allclose(P.mean(axis=0), [(W - 1) / 2, (H - 1) / 2], atol=1e-12)
    assert np.allclose(P.min(axis=0), [0.5 / g - 0.5] * 2, atol=1e-15)
    assert np.allclose(P.max(axis=0), [W - 0.5 - 0.5 / g, H - 0.5 - 0.5 / g], atol=1e-12)
    # g^2 points in every LR pixel [j - 1/2, j + 1/2)
    pix = np.floor(P + 0.5).astype(int)
    counts = np.zeros((H, W), int)
    np.add.at(counts, (pix[:, 1], pix[:, 0]), 1)
    assert (counts == g * g).all()
    if g == 1:  # the LR pixel centres themselves
        assert np.array_equal(P, np.stack(np.meshgrid(np.arange(W), np.arange(H)), -1)
                              .reshape(-1, 2).astype(float))


def test_head_forward_closed_forms():
    """sigmoid(0) = 1/2, sigmoid(ln 3) = 3/4, tanh(0) = 0, tanh(ln 2) = 3/5
    (so sqrt(1 - rho^2) = 4/5): exact values the formulas must produce."""
    ln2, ln3 = math.log(2.0), math.log(3.0)
    raw_op = np.array([0.0, ln3, -ln3])
    raw_col = np.array([[0.0, ln3, -ln3]] * 3)
    raw_sig = np.array([[0.0, 0.0], [ln3, ln3], [ln3, -ln3]])
    raw_rho = np.array([0.0, ln2, -ln2])
    off = np.array([[0.25, -0.5], [0.0, 0.0], [-1.0, 2.0]])
    ref = np.array([[1.0, 2.0], [3.5, 0.5], [0.0, 0.0]])
    mean, chol, color, alpha = Hd.head_forward(raw_op, raw_col, raw_sig, raw_rho, off, ref)
    np.testing.assert_allclose(alpha, [0.5, 0.75, 0.25], rtol=1e-15)
    np.testing.assert_allclose(color, [[0.5, 0.75, 0.25]] * 3, rtol=1e-15)
    np.testing.assert_allclose(mean, [[1.25, 1.5], [3.5, 0.5], [-1.0, 2.0]], rtol=0, atol=0)
    # (sigma_x, sigma_y, rho) = (1/2, 1/2, 0), (3/4, 3/4, 3/5), (3/4, 1/4, -3/5)
    np.testing.assert_allclose(chol, [[0.5, 0.0, 0.5],
                                      [0.75, 0.6 * 0.75, 0.8 * 0.75],
                                      [0.75, -0.6 * 0.25, 0.8 * 0.25]], rtol=1e-14, atol=1e-16)


def test_head_cholesky_reproduces_the_covariance():
    raw = _raw(500, 1, spread=3.0)
    mean, chol, color, alpha = Hd.head_forward(*raw, np.zeros((500, 2)))
    sx = 1 / (1 + np.exp(-raw[2][:, 0]))
    sy = 1 / (1 + np.exp(-raw[2][:, 1]))
    rho = np.tanh(raw[3])
    l11, l21, l22 = chol.T
    assert (l11 > 0).all() and (l22 > 0).all()
    np.testing.assert_allclose(l11 * l11, sx * sx, rtol=1e-14)
    np.testing.assert_allclose(l11 * l21, rho * sx * sy, rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(l21 * l21 + l22 * l22, sy * sy, rtol=1e-13)
    # determinant sigma_x^2 sigma_y^2 (1 - rho^2) of Eq. 2's normaliser
    np.testing.assert_allclose((l11 * l22) ** 2, (sx * sy) ** 2 * (1 - rho ** 2), rtol=1e-12)


def test_head_backward_against_central_differences():
    n = 64
    raw = _raw(n, 2)
    ref = Hd.reference_positions(4, 4, 2)
    rng = np.random.default_rng(3)
    W = [rng.normal(size=s) for s in [(n, 2), (n, 3), (n, 3), (n,)]]

    def f(ro, rc, rs, rr, off):
        outs = Hd.head_forward(ro, rc, rs, rr, off, ref)
        return sum(float((w * o).sum()) for w, o in zip(W, outs))

    grads = Hd.head_backward(raw[0], raw[1], raw[2], raw[3], *W)
    for k in range(5):
        g = grads[k]
        base = [np.array(a, np.float64) for a in raw]
        fd = np.zeros_like(g)
        it = np.nditer(g, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            h = 1e-6 * max(1.0, abs(base[k][idx]))
            up = [a.copy() for a in base]
            dn = [a.copy() for a in base]
            up[k][idx] += h
            dn[k][idx] -= h
            fd[idx] = (f(*up) - f(*dn)) / (2 * h)
        np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_head_backward_planted_mistakes_fail():
    """The finite-difference pin notices a dropped sqrt(1 - rho^2) factor in
    d sigma_y or a dropped (1 - rho^2) in d rho."""
    n = 16
    raw = _raw(n, 4)
    rng = np.random.default_rng(5)
    W = [rng.normal(size=s) for s in [(n, 2), (n, 3), (n, 3), (n,)]]
    g = Hd.head_backward(raw[0], raw[1], raw[2], raw[3], *W)
    v = raw[3]
    rho = np.tanh(v)
    sy = 1 / (1 + np.exp(-raw[2][:, 1]))
    wrong_rho = g[3] / (1 - rho * rho)
    wrong_sy = (W[1][:, 1] * rho + W[1][:, 2]) * sy * (1 - sy)
    h = 1e-6
    ref = np.zeros((n, 2))
    fd_rho = []
    fd_sy = []
    for i in range(n):
        def f(dv=0.0, du=0.0):
            rs = raw[2].copy()
            rs[i, 1] += du
            rr = raw[3].copy()
            rr[i] += dv
            outs = Hd.head_forward(raw[0], raw[1], rs, rr, raw[4], ref)
            return sum(float((w * o).sum()) for w, o in zip(W, outs))
        fd_rho.append((f(dv=h) - f(dv=-h)) / (2 * h))
        fd_sy.append((f(du=h) - f(du=-h)) / (2 * h))
    assert np.allclose(g[3], fd_rho, rtol=1e-6, atol=1e-9)
    assert not np.allclose(wrong_rho, fd_rho, rtol=1e-3)
    assert np.allclose(g[2][:, 1], fd_sy, rtol=1e-6, atol=1e-9)
    assert not np.allclose(wrong_sy, fd_sy, rtol=1e-3)


def test_luma_of_known_colours():
    """BT.601 studio range: black 16/255, white 235/255, grey v (16 + 219 v)/255,
    the primaries their own coefficients."""
    def img(r, g, b):
        return np.array([r, g, b], np.float64).reshape(3, 1, 1) * np.ones((3, 2, 2))
    assert np.allclose(Hd.rgb_to_y(img(0, 0, 0)), 16 / 255, rtol=0, atol=1e-15)
    assert np.allclose(Hd.rgb_to_y(img(1, 1, 1)), 235 / 255, rtol=0, atol=1e-15)
    for v in (0.1, 0.5, 0.9):
        assert np.allclose(Hd.rgb_to_y(img(v, v, v)), (16 + 219 * v) / 255, atol=1e-15)
    assert np.allclose(Hd.rgb_to_y(img(1, 0, 0)), (16 + 65.481) / 255, atol=1e-15)
    assert np.allclose(Hd.rgb_to_y(img(0, 1, 0)), (16 + 128.553) / 255, atol=1e-15)
    assert np.allclose(Hd.rgb_to_y(img(0, 0, 1)), (16 + 24.966) / 255, atol=1e-15)


def test_psnr_y_closed_forms():
    rng = np.random.default_rng(6)
    ref = rng.uniform(0, 1, (3, 20, 30))
    # the same shift delta in every channel moves Y by 219 delta / 255
    for delta in (1e-3, 0.01, 0.2):
        p, sse, n = Hd.psnr_y(ref + delta, ref)
        assert n == 600
        assert p == pytest.approx(-20 * math.log10(219 * delta / 255), abs=1e-9)
    # blue alone moves Y by 24.966 delta / 255
    test = ref.copy()
    test[2] += 0.05
    assert Hd.psnr_y(test, ref)[0] == pytest.approx(-20 * math.log10(24.966 * 0.05 / 255),
                                                    abs=1e-9)
    # a change confined to the border vanishes under the crop
    test = ref.copy()
    test[:, :2, :] += 0.3
    test[:, :, -2:] -= 0.1
    assert Hd.psnr_y(test, ref, crop=2)[0] == math.inf
    assert Hd.psnr_y(test, ref, crop=2)[2] == 16 * 26
    assert Hd.psnr_y(test, ref, crop=1)[0] < 40
    assert Hd.psnr_y(ref, ref)[0] == math.inf
