"""Pins of the completion-network oracle against closed forms, brute force and finite
differences (not against its own formulas)."""
import numpy as np
import pytest

from oracle import completion as OC


def _rng(seed=0):
    return np.random.default_rng(seed)


def _brute_conv(x, W, b, dil=(1, 1)):
    """Seven nested loops over the definition, on tiny grids."""
    B, H, Wd, Ci = x.shape
    Co = W.shape[1]
    y = np.zeros((B, H, Wd, Co))
    for bb in range(B):
        for h in range(H):
            for w in range(Wd):
                for o in range(Co):
                    s = b[o]
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            hh, ww = h + dy * dil[0], w + dx * dil[1]
                            if 0 <= hh < H and 0 <= ww < Wd:
                                t = 3 * (dy + 1) + (dx + 1)
                                for c in range(Ci):
                                    s += W[t, o, c] * x[bb, hh, ww, c]
                    y[bb, h, w, o] = s
    return y


@pytest.mark.parametrize("dil", [(1, 1), (2, 3), (1, 4)])
def test_conv_matches_brute_force(dil):
    r = _rng(1)
    x = r.standard_normal((2, 5, 9, 2))
    W = r.standard_normal((9, 3, 2))
    b = r.standard_normal(3)
    np.testing.assert_allclose(OC.conv3x3(x, W, b, dil), _brute_conv(x, W, b, dil), rtol=0, atol=1e-12)


def test_dilated_delta_kernel_is_a_long_shift():
    r = _rng(9)
    x = r.standard_normal((1, 6, 11, 1))
    W = np.zeros((9, 1, 1))
    W[3 * 2 + 0] = 1.0                       # dy = +1, dx = -1
    y = OC.conv3x3(x, W, np.zeros(1), (2, 3))
    ref = np.zeros_like(x)
    ref[0, :4, 3:, 0] = x[0, 2:, :8, 0]      # y[h][w] = x[h + 2][w - 3]
    np.testing.assert_array_equal(y, ref)


@pytest.mark.parametrize("dy,dx", [(0, 0), (-1, 0), (1, 1), (0, -1), (1, -1)])
def test_delta_kernel_is_a_shift(dy, dx):
    r = _rng(2)
    x = r.standard_normal((1, 4, 6, 2))
    W = np.zeros((9, 2, 2))
    t = 3 * (dy + 1) + (dx + 1)
    W[t] = np.eye(2)
    y = OC.conv3x3(x, W, np.zeros(2))
    ref = np.zeros_like(x)
    for h in range(4):
        for w in range(6):
            if 0 <= h + dy < 4 and 0 <= w + dx < 6:
                ref[0, h, w] = x[0, h + dy, w + dx]
    np.testing.assert_array_equal(y, ref)


def test_conv_is_linear_in_input_and_weights():
    r = _rng(3)
    x1, x2 = r.standard_normal((2, 1, 3, 4, 3))
    W1, W2 = r.standard_normal((2, 9, 2, 3))
    z = np.zeros(2)
    np.testing.assert_allclose(OC.conv3x3(2 * x1 - 3 * x2, W1, z),
                               2 * OC.conv3x3(x1, W1, z) - 3 * OC.conv3x3(x2, W1, z), atol=1e-12)
    np.testing.assert_allclose(OC.conv3x3(x1, W1 + W2, z), OC.conv3x3(x1, W1, z) + OC.conv3x3(x1, W2, z),
                               atol=1e-12)


def _params(r, widths):
    return [(r.standard_normal((9, co, ci)) * np.sqrt(2.0 / (9 * ci)), 0.1 * r.standard_normal(co))
            for ci, co in zip(widths[:-1], widths[1:])]


@pytest.mark.parametrize("dils", [None, [(1, 2), (2, 1), (1, 3)]])
def test_network_gradients_match_finite_differences(dils):
    r = _rng(4)
    params = _params(r, [3, 4, 4, 2])
    x = r.standard_normal((2, 4, 7, 3))
    tgt = r.standard_normal((2, 4, 7, 2))
    obs = (r.random((2, 4, 7)) < 0.3).astype(float)

    def loss_of(ps, xx):
        out, _ = OC.forward(xx, ps, dils)
        return OC.masked_mse(out, tgt, obs)[0]

    out, acts = OC.forward(x, params, dils)
    _, gout = OC.masked_mse(out, tgt, obs)
    grads = OC.backward(params, acts, gout, dils)
    h = 1e-6
    for l in range(len(params)):
        for which in (0, 1):
            arr = params[l][which]
            for _ in range(4):
                idx = tuple(int(r.integers(0, n)) for n in arr.shape)
                ps_p = [(W.copy(), b.copy()) for W, b in params]
                ps_m = [(W.copy(), b.copy()) for W, b in params]
                ps_p[l][which][idx] += h
                ps_m[l][which][idx] -= h
                fd = (loss_of(ps_p, x) - loss_of(ps_m, x)) / (2 * h)
                assert abs(fd - grads[l][which][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, which, idx)
    # the input gradient (through every layer) by the conv backward
    d0 = (dils or [(1, 1)])[0]
    gx, _, _ = OC.conv3x3_backward(x, params[0][0], np.ones((2, 4, 7, 4)), d0)
    for _ in range(4):
        idx = tuple(int(r.integers(0, n)) for n in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (OC.conv3x3(xp, *params[0], d0).sum() - OC.conv3x3(xm, *params[0], d0).sum()) / (2 * h)
        assert abs(fd - gx[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_masked_mse_ignores_observed_pairs():
    r = _rng(5)
    out = r.standard_normal((1, 2, 3, 2))
    tgt = out.copy()
    obs = np.array([[[1, 0, 1], [0, 0, 1]]], float)
    tgt[0, 0, 0] += 5.0          # observed: no effect
    loss, g = OC.masked_mse(out, tgt, obs)
    assert loss == 0.0 and not g.any()
    tgt[0, 1, 1, 0] += 2.0       # unobserved: (2^2) / (2 * 3 unobserved positions)
    loss, g = OC.masked_mse(out, tgt, obs)
    assert loss == pytest.approx(4.0 / 6.0)
    assert g[0, 1, 1, 0] == pytest.approx(2 * -2.0 / 6.0)


def test_adam_first_step_moves_by_the_learning_rate():
    r = _rng(6)
    p = r.standard_normal(50)
    g = r.standard_normal(50)
    g[:5] = 0.0
    p1, m, v = OC.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, eps=0.0 + 1e-30)
    # bias-corrected first moments: m_hat = g, v_hat = g^2, so the step is lr * sign(g)
    np.testing.assert_allclose(p1[5:], p[5:] - 1e-3 * np.sign(g[5:]), rtol=0, atol=1e-15)
    np.testing.assert_array_equal(p1[:5], p[:5])
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_prepare_and_merge_round_trip():
    r = _rng(7)
    grid = r.standard_normal((5, 12)) + 1j * r.standard_normal((5, 12))
    cols = [0, 3, 4, 11]
    inp, tgt, obs, scale = OC.prepare(grid, cols)
    vals = grid[:, cols]
    assert scale == pytest.approx(np.sqrt(np.mean(np.abs(vals) ** 2)))
    assert obs[:, cols].all() and obs.sum() == 5 * 4
    np.testing.assert_allclose(inp[..., 0] * scale, np.where(obs > 0, grid.real, 0.0), atol=1e-14)
    np.testing.assert_array_equal(inp[..., 2], obs)
    # a network that outputs the target reproduces the full grid
    np.testing.assert_allclose(OC.merge(grid, tgt, obs, scale), grid, atol=1e-14)
    # unobserved predictions are rescaled; observed pairs are kept
    out = np.zeros_like(tgt)
    m = OC.merge(grid, out, obs, scale)
    np.testing.assert_array_equal(m[:, cols], grid[:, cols])
    assert not m[:, [1, 2, 5]].any()
