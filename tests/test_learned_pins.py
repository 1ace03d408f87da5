"""Pins of the learned step-scale oracle (no GPU): gradients against finite
differences, Adam against its closed form, features of hand-built blocks, labels
of constructed steps."""
import numpy as np

from oracle import learned as L
from oracle import oracle as O
from synth.mlp_init import init_params, random_features
from synth.scenes import make_config


def _data(n=64, seed=3):
    rng = np.random.default_rng(seed)
    F = random_features(n, seed).astype(np.float64)
    lab = rng.uniform(0.0, 1.5, (n, 5))
    msk = (rng.random((n, 5)) < 0.7).astype(np.float64)
    return F, lab, msk


def test_param_count():
    assert L.N_PARAMS == 32 * 17 + 32 + 5 * 32 + 5 == 741 and init_params().size == 741


def test_loss_gradient_matches_central_differences():
    F, lab, msk = _data()
    p = init_params(5).astype(np.float64) + 0.3 * np.random.default_rng(0).standard_normal(L.N_PARAMS)
    _, g = L.loss_grad(p, F, lab, msk)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (L.loss_grad(p + e, F, lab, msk)[0] - L.loss_grad(p - e, F, lab, msk)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-6 * np.max(np.abs(g))


def test_loss_value_is_masked_mean_square():
    F, lab, msk = _data()
    p = init_params(2).astype(np.float64)
    a = L.forward(p, F)
    want = float(((a - lab) ** 2 * msk).sum() / msk.sum())
    assert abs(L.loss_grad(p, F, lab, msk)[0] - want) <= 1e-14 * want


def test_output_range_and_zero_network():
    F, _, _ = _data()
    a = L.forward(init_params(1), F * 50.0)
    assert np.all(a > 0.0) and np.all(a < 1.5)
    assert np.allclose(L.forward(np.zeros(L.N_PARAMS), F), 0.75)


def test_adam_closed_form_with_constant_gradient():
    # with a constant gradient the bias-corrected moments are g and g^2 at every step:
    # each update is -lr g / (|g| + eps)
    rng = np.random.default_rng(4)
    g = rng.standard_normal(L.N_PARAMS)
    p = rng.standard_normal(L.N_PARAMS)
    m = np.zeros(L.N_PARAMS)
    v = np.zeros(L.N_PARAMS)
    p0 = p.copy()
    for t in range(1, 6):
        p, m, v = L.adam(p, m, v, t, g, lr=1e-2)
        assert np.allclose(p, p0 - t * 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_training_reduces_loss():
    F, _, msk = _data(256)
    target = L.forward(init_params(9).astype(np.float64) * 2.0, F)
    p = init_params(0).astype(np.float64)
    m = np.zeros(L.N_PARAMS)
    v = np.zeros(L.N_PARAMS)
    l0 = L.loss_grad(p, F, target, msk)[0]
    for t in range(1, 301):
        _, gr = L.loss_grad(p, F, target, msk)
        p, m, v = L.adam(p, m, v, t, gr, lr=1e-2)
    assert L.loss_grad(p, F, target, msk)[0] < 0.2 * l0


def test_labels_of_scaled_and_orthogonal_steps():
    K = 16
    rng = np.random.default_rng(2)
    prim = rng.standard_normal((6, 11 + 3 * K))
    dec = np.zeros((6, 5), np.int32)
    dec[5, :] = -2
    c = np.array([0.2, 0.9, 1.0, 1.3, 2.5, 0.5])
    lab, msk = L.labels(prim, prim * c[:, None], dec, K)
    assert np.allclose(lab[:5], np.minimum(c[:5], 1.5)[:, None])
    assert np.all(msk[:5] == 1) and np.all(msk[5] == 0) and np.all(lab[5] == 0)
    # a full-rule step orthogonal to the primary one keeps none of it
    aug = np.zeros_like(prim)
    aug[:, 0], aug[:, 1] = -prim[:, 1], prim[:, 0]
    prim2 = prim.copy()
    prim2[:, 2] = 0.0
    lab2, _ = L.labels(prim2, aug, dec, K)
    assert np.allclose(lab2[:5, 0], 0.0, atol=1e-15)


def test_features_of_isotropic_blocks():
    # isotropic position and rotation Hessians reduce to the same scalar in any basis
    cfg = make_config("c1", n=40, width=120, height=90, n_views=3)
    g, cam = cfg.init, cfg.cams[0]
    o = O.opts(npix_primary=120 * 90)
    n, V = g.n, 1
    S = np.zeros((n, 40 + 10 * V))
    a, h = 3.0e-3, -2.0e-5
    S[:, 3:12] = (a * np.eye(3)).ravel()
    S[:, 15:24] = (h * np.eye(3)).ravel()
    S[:, 0:3] = [4e-4, 0.0, 0.0]
    S[:, 36], S[:, 37], S[:, 38] = 1e-3, 2e-3, 5.0
    S[:, 42:45] = [1e-4, 2e-4, 3e-4]
    F, ok = L.features(g, cam, o, S, V)
    Lg = lambda x: np.log10(x + 1e-30) / 10.0
    assert np.allclose(F[:, 0], Lg(a)) and np.allclose(F[:, 1], Lg(a)) and np.all(F[:, 2] == 1.0)
    assert np.allclose(F[:, 3], Lg(abs(h))) and np.all(F[:, 4] == -1.0)
    assert np.allclose(F[:, 9], Lg(6e-4)) and np.allclose(F[:, 10], Lg(5.0))
    assert np.allclose(F[:, 15], Lg(np.asarray(g.opac, np.float64)))
    # |U^T g_p| is the part of g_p orthogonal to the view axis
    r = np.asarray(g.pos, np.float64).T - cam.center
    r /= np.linalg.norm(r, axis=1, keepdims=True)
    gp = np.array([4e-4, 0.0, 0.0])
    gperp = np.linalg.norm(gp - (r @ gp)[:, None] * r, axis=1)
    assert np.allclose(F[:, 11], Lg(gperp))
    # opacity: H_sigma + h_B with the closed-form barrier
    sig = np.asarray(g.opac, np.float64)
    al = 1e-2 / (3.0 * 120 * 90)
    assert np.allclose(F[:, 8], Lg(np.abs(2e-3 + al * (1 / sig ** 2 + 1 / (1 - sig) ** 2))))
    assert np.all(ok == 1)
    # the cached neighbouring-view residual enters as feature 16 (0 without a cache)
    assert np.all(F[:, 16] == -3.0)
    resid = np.linspace(1e-3, 10.0, n)
    F2, _ = L.features(g, cam, o, S, V, resid=resid)
    assert np.allclose(F2[:, 16], Lg(resid)) and np.array_equal(F2[:, :16], F[:, :16])
    # a feature out of [-3, 3] marks the kernel out of range (code 2); unseen kernels are 0
    F3, ok3 = L.features(g, cam, o, S, V, resid=np.full(n, 1e40))
    assert np.all(ok3 == 2) and np.all(F3[:, 16] == 3.0)
    S[:, 38] = 0.0
    _, ok0 = L.features(g, cam, o, S, V)
    assert np.all(ok0 == 0)


def test_neighbour_residual_of_constructed_views():
    # three view slots: the residual is the secondaries' colour-gradient norms over the primary's
    n, V = 5, 3
    S = np.zeros((n, 40 + 10 * V))
    S[:, 38] = [1.0, 1.0, 1.0, 0.0, 1.0]  # kernel 3: not seen by the primary
    g0 = np.array([[3.0, 4.0, 0.0]] * n)  # |gamma_0| = 5
    S[:, 39:42] = g0
    S[:, 39 + 9] = S[:, 38]
    S[:, 49:52] = [[0.0, 0.0, 2.0]] * n  # view 1: |gamma| = 2
    S[:, 49 + 9] = [1.0, 0.0, 1.0, 1.0, 0.0]
    S[:, 59:62] = [[1.0, 2.0, 2.0]] * n  # view 2: |gamma| = 3
    S[:, 59 + 9] = [1.0, 0.0, 0.0, 1.0, 0.0]
    prev = np.full(n, 7.0)
    r = L.neighbour_residual(S, V, prev)
    assert np.allclose(r, [(2 + 3) / 5, 7.0, 2 / 5, 7.0, 7.0], rtol=1e-14)
