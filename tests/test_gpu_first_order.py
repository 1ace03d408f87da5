"""GPU parity of the first-order baseline (gradient descent and Adam on the gradients of the
sweep's blocks) against the oracle on the oracle's own blocks, rounded to the library's
float32 storage."""
import numpy as np
import pytest

from oracle import first_order as F
from oracle import oracle as O
from synth.scenes import make_config
from tests.parity import summed_to_gpu_blocks

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LR = [2e-3, 5e-3, 1e-4, 1e-2, 2e-3]


@pytest.fixture(scope="module")
def gsn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_13975_amd import gsn as G
    return G


@pytest.fixture(scope="module")
def ctx(gsn):
    c = gsn.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def case():
    cfg = make_config("c1", n=4000, width=200, height=150, n_views=10)
    tg = [O.render(cfg.gt, c, O.opts()).img.astype(np.float32) for c in cfg.cams]
    knn = O.camera_knn(cfg.cams, cfg.init, 3)
    res = O.sweep(cfg.init, cfg.cams, tg, 3, knn, O.opts(lambda_ssim=0.2))
    return cfg, res["summed"].astype(np.float32).astype(np.float64)


def _close(dg, want, start, seen, det=None):
    """Per attribute: |got - want| <= 4 float32 ulps of the value + 1e-4 of the largest change,
    on the entries marked in det (all if None)."""
    got = dg.to_host()
    for a in ("pos", "rot", "scale", "opac", "sh"):
        x = np.asarray(getattr(got, a), np.float64)
        y = np.asarray(getattr(want, a), np.float64)
        d = np.max(np.abs(y - np.asarray(getattr(start, a), np.float64)))
        assert d > 0, a
        bound = 4 * np.finfo(np.float32).eps * np.abs(y) + 1e-4 * d
        ok = np.abs(x - y) <= bound
        if det is not None:
            ok |= ~det[a]
        assert np.all(ok), (a, float(np.max(np.abs(x - y) / bound)))
        assert np.array_equal(x[..., ~seen], y[..., ~seen]), a


def _determined(G, K, n):
    """Entries whose gradient is at least 1e-3 of its group's largest: Adam moves every entry by
    about lr whatever its size, so an entry whose gradient is the cancelled remainder of larger
    terms (float32 sums are exact only to a fraction of those) has no determined Adam step."""
    A = np.abs(G)
    big = lambda sl: A[:, sl] >= 1e-3 * A[:, sl].max()  # noqa: E731
    rot = np.all(big(slice(3, 6)), axis=1)
    return {"pos": big(slice(0, 3)).T, "rot": np.repeat(rot[None], 4, 0), "scale": big(slice(6, 9)).T,
            "opac": big(slice(9, 10))[:, 0], "sh": big(slice(10, 10 + 3 * K)).reshape(n, 3, K).transpose(1, 2, 0)}


@pytest.mark.parametrize("adam", [False, True])
def test_first_order_steps_match_oracle(gsn, ctx, case, adam):
    cfg, S32 = case
    g = cfg.init
    V, K = 4, (g.sh_degree + 1) ** 2
    seen = S32[:, 38] > 0
    assert seen.sum() > 1000
    dg = gsn.DeviceGaussians.from_host(g)
    b = gsn.Blocks(g.n, V, ctx.device)
    b.view().copy_(torch.tensor(summed_to_gpu_blocks(S32, V), dtype=torch.float32, device=ctx.device))
    so = gsn.solve_opts(cfg.cams[3].width * cfg.cams[3].height)
    nf = F.n_features(K)
    state = torch.zeros(2, nf, g.n, device=ctx.device) if adam else None
    ms = (np.zeros((g.n, nf)), np.zeros((g.n, nf)))
    # plain descent: learning rates that move each group's largest entry by about LR
    G = np.abs(F.gradient(S32, V, K))
    gmax = [G[:, sl].max() for sl in (slice(0, 3), slice(3, 6), slice(6, 9), slice(9, 10), slice(10, None))]
    lr = LR if adam else [x / m for x, m in zip(LR, gmax)]
    det = _determined(F.gradient(S32, V, K), K, g.n) if adam else None
    if adam:
        for a, m in det.items():
            assert m[..., seen].mean() > 0.3, a
    want = g
    for t in range(1, 4):
        # the same (oracle) gradients every step; both sides carry their own state forward
        ctx.first_order_step(dg, b, so, lr, adam=adam, step=t, state=state)
        want = F.step(want, S32, V, lr, adam=adam, state=ms, t=t, eps=1e-15,
                      scale_floor=so.scale_floor, opac_eps=so.opac_eps)
        torch.cuda.synchronize()
        _close(dg, want, g, seen, det)
    if adam:
        # moments of the determined entries (their gradients are exact to float rounding)
        m = state.cpu().numpy()
        A = np.abs(F.gradient(S32, V, K))
        big = np.zeros_like(A, bool)
        for sl in (slice(0, 3), slice(3, 6), slice(6, 9), slice(9, 10), slice(10, None)):
            big[:, sl] = A[:, sl] >= 1e-3 * A[:, sl].max()
        big &= seen[:, None]
        for i in range(2):
            got, want_m = m[i].T[big], ms[i][big]
            assert np.all(np.abs(got - want_m) <= 1e-4 * np.abs(want_m)), i
        assert np.all(m[:, :, ~seen] == 0.0)


def test_first_order_group_mask_and_errors(gsn, ctx, case):
    cfg, S32 = case
    g = cfg.init
    dg = gsn.DeviceGaussians.from_host(g)
    b = gsn.Blocks(g.n, 4, ctx.device)
    b.view().copy_(torch.tensor(summed_to_gpu_blocks(S32, 4), dtype=torch.float32, device=ctx.device))
    so = gsn.solve_opts(200 * 150)
    ctx.first_order_step(dg, b, so, [0.1] * 5, adam=False, group_mask=8)
    got = dg.to_host()
    for a in ("pos", "rot", "scale", "sh"):
        assert np.array_equal(np.asarray(getattr(got, a)), np.asarray(getattr(g, a))), a
    assert not np.array_equal(got.opac, g.opac)
    with pytest.raises(gsn.GsnError):
        ctx.first_order_step(dg, b, so, [0.1] * 5, adam=True, step=1, state=None)
    with pytest.raises(gsn.GsnError):
        ctx.first_order_step(dg, b, so, [-1.0] * 5, adam=False)
