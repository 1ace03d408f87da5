"""Pins of the first-order baseline oracle: the gradient it assembles against central
finite differences of the loss, gradient descent and Adam against their closed forms,
the rotation update as a descent direction, and the parameter limits."""
import numpy as np
import pytest

from oracle import first_order as F
from oracle import oracle as O
from tests.test_oracle_pins import GROUPS, fd_grad, loss_value, rel_err, smooth_opts, tiny_cam, tiny_scene

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.fixture(scope="module")
def setup():
    g = tiny_scene(5, K=4, seed=21)
    cam = tiny_cam()
    tgt = O.render(tiny_scene(5, K=4, seed=22), cam, O.opts(smooth=1)).img
    o = smooth_opts(0.2)
    fr = O.render(g, cam, o)
    _, dL, hd = O.loss(fr.img, tgt, 0.2)
    S = O.sum_blocks([O.blocks(g, fr, dL, hd)])
    return g, cam, tgt, o, S


def test_gradient_matches_finite_differences(setup):
    g, cam, tgt, o, S = setup
    g = g.copy()
    G = F.gradient(S, 1, g.K)
    for k in range(g.n):
        assert rel_err(G[k, 0:3], fd_grad(g, cam, tgt, o, "p", k)) < 1e-6
        assert rel_err(G[k, 3:6], fd_grad(g, cam, tgt, o, "w", k)) < 1e-6
        assert rel_err(G[k, 6:9], fd_grad(g, cam, tgt, o, "s", k)) < 1e-6
        assert rel_err(G[k, 9:10], fd_grad(g, cam, tgt, o, "o", k)) < 1e-6
        # every SH coefficient of every channel (the view-direction basis is only in the oracle)
        fd = np.zeros(3 * g.K)
        for ch in range(3):
            for i in range(g.K):
                h = 1e-6
                x0 = g.sh[ch, i, k]
                g.sh[ch, i, k] = x0 + h
                lp = loss_value(g, cam, tgt, o)
                g.sh[ch, i, k] = x0 - h
                lm = loss_value(g, cam, tgt, o)
                g.sh[ch, i, k] = x0
                fd[ch * g.K + i] = (lp - lm) / (2 * h)
        assert rel_err(G[k, 10:], fd) < 1e-6, k


def test_gradient_descent_moves_by_minus_lr_gradient(setup):
    g, cam, tgt, o, S = setup
    lr = [1e-3, 1e-3, 1e-4, 1e-2, 1e-3]
    new = F.step(g, S, 1, lr, adam=False, mask=1 | 4 | 8 | 16)
    G = F.gradient(S, 1, g.K)
    assert np.allclose(new.pos - g.pos, -lr[0] * G[:, 0:3].T, rtol=0, atol=1e-15)
    assert np.allclose(new.scale - g.scale, -lr[2] * G[:, 6:9].T, rtol=0, atol=1e-15)
    assert np.allclose(new.opac - g.opac, -lr[3] * G[:, 9], rtol=0, atol=1e-15)
    assert np.allclose((new.sh - g.sh).transpose(2, 0, 1).reshape(g.n, -1), -lr[4] * G[:, 10:], rtol=0, atol=1e-15)
    assert np.array_equal(new.rot, np.asarray(g.rot, np.float64))


def test_adam_first_and_constant_gradient_steps_are_sign_steps(setup):
    """With m and v started at zero, bias correction makes the first step -lr g / (|g| + eps);
    with the gradient held fixed every later step is the same."""
    g, cam, tgt, o, S = setup
    K = g.K
    lr = [1e-3, 1e-3, 1e-4, 1e-2, 1e-3]
    state = (np.zeros((g.n, F.n_features(K))), np.zeros((g.n, F.n_features(K))))
    G = F.gradient(S, 1, K)
    want = -lr[0] * G[:, 0:3] / (np.abs(G[:, 0:3]) + 1e-15)
    cur = g
    for t in range(1, 4):
        new = F.step(cur, S, 1, lr, adam=True, state=state, t=t, mask=1)
        assert np.allclose((new.pos - cur.pos).T, want, rtol=1e-12, atol=1e-18), t
        cur = new
    assert np.allclose(state[0][:, 0:3], (1 - 0.9 ** 3) * G[:, 0:3], rtol=1e-12)
    assert np.allclose(state[1][:, 0:3], (1 - 0.999 ** 3) * G[:, 0:3] ** 2, rtol=1e-12)
    assert np.all(state[0][:, 3:] == 0.0)  # groups outside the mask keep their moments


def test_rotation_step_is_a_descent_direction(setup):
    """For a small step the loss changes by -lr |g_omega|^2 to first order (sign and axis
    convention of the exponential map)."""
    g, cam, tgt, o, S = setup
    G = F.gradient(S, 1, g.K)
    lr = 1e-3 / np.max(np.abs(G[:, 3:6]))
    for k in range(g.n):
        S1 = S.copy()
        S1[:, 38] = 0.0
        S1[k, 38] = S[k, 38]  # move kernel k only
        new = F.step(g, S1, 1, [0, lr, 0, 0, 0], adam=False, mask=2)
        assert np.allclose(np.linalg.norm(new.rot, axis=0), 1.0)
        dl = loss_value(new, cam, tgt, o) - loss_value(g, cam, tgt, o)
        pred = -lr * np.dot(G[k, 3:6], G[k, 3:6])
        assert dl == pytest.approx(pred, rel=1e-2), k


def test_limits_and_unseen_kernels(setup):
    g, cam, tgt, o, S = setup
    S1 = S.copy()
    S1[0, 38] = 0.0  # kernel 0 not seen by the primary view
    big = [0.0, 0.0, 1e9, 1e9, 0.0]
    new = F.step(g, S1, 1, big, adam=False, mask=4 | 8, scale_floor=0.1, opac_eps=1e-6)
    assert np.array_equal(new.scale[:, 0], np.asarray(g.scale[:, 0], np.float64))
    assert new.opac[0] == g.opac[0]
    G = F.gradient(S, 1, g.K)
    for k in range(1, g.n):
        for a in range(3):
            if G[k, 6 + a] > 0:
                assert new.scale[a, k] == pytest.approx(0.1 * g.scale[a, k], rel=1e-15)
        assert 1e-6 <= new.opac[k] <= 1 - 1e-6
        assert new.opac[k] in (1e-6, 1 - 1e-6)
