"""GPU parity of the learned step scale: features, labels, network inference and
Adam training against the FP64 oracle on the same inputs (the oracle's own
blocks and steps, rounded to the library's float32 storage), the scaled apply,
and a short run of the learned form."""
import numpy as np
import pytest

from oracle import learned as L
from oracle import oracle as O
from synth.mlp_init import init_params, random_features
from synth.scenes import make_config
from tests.parity import rel_inf, summed_to_gpu_blocks

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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
def sweep_case():
    cfg = make_config("c1", n=4000, width=200, height=150, n_views=8)
    tg = [O.render(cfg.gt, c, O.opts()).img.astype(np.float32) for c in cfg.cams]
    t = 3
    knn = O.camera_knn(cfg.cams, cfg.init, 3)
    res = O.sweep(cfg.init, cfg.cams, tg, t, knn, O.opts(lambda_ssim=0.2))
    return cfg, t, res


def _gpu_blocks(gsn, S, V, device):
    b = gsn.Blocks(S.shape[0], V, device)
    b.view().copy_(torch.tensor(summed_to_gpu_blocks(S, V), dtype=torch.float32, device=device))
    return b


def test_features_parity(gsn, ctx, sweep_case):
    cfg, t, res = sweep_case
    g, cam, o = cfg.init, cfg.cams[t], res["opts"]
    S1 = O.sum_blocks(res["per_view"][:1]).astype(np.float32).astype(np.float64)
    dg = gsn.DeviceGaussians.from_host(g)
    b = _gpu_blocks(gsn, S1, 1, ctx.device)
    n = g.n
    feat = torch.zeros(17, n, device=ctx.device)
    ok = torch.zeros(n, dtype=torch.uint8, device=ctx.device)
    so = gsn.solve_opts(cam.width * cam.height)
    # the cached residual of a full-rule sweep (all four views), by the library and by the oracle
    V = len(res["per_view"])
    Sfull = O.sum_blocks(res["per_view"]).astype(np.float32).astype(np.float64)
    prev = np.random.default_rng(1).uniform(0.0, 2.0, n).astype(np.float32)
    r_want = L.neighbour_residual(Sfull, V, prev.astype(np.float64))
    r_dev = torch.tensor(prev, device=ctx.device)
    ctx.neighbour_residual(_gpu_blocks(gsn, Sfull, V, ctx.device), r_dev)
    r_got = r_dev.cpu().numpy().astype(np.float64)
    upd = r_want != prev
    assert upd.sum() > 500
    assert np.array_equal(r_got[~upd], prev[~upd].astype(np.float64))
    assert np.max(np.abs(r_got[upd] - r_want[upd]) / np.maximum(r_want[upd], 1e-30)) < 1e-5
    want, ok_want = L.features(g, cam, o, S1, 1, resid=r_got)
    ctx.step_features(dg, gsn.camera(cam), b, so, feat, ok, resid=r_dev)
    got = feat.cpu().numpy().T.astype(np.float64)
    okg = ok.cpu().numpy()
    vis = S1[:, 38] > 0
    assert vis.sum() > 1000
    # magnitudes: 1e-5 in feature units is a relative error of 2.3e-4 in the summarised quantity
    for col in (0, 3, 5, 8, 9, 10, 11, 12, 13, 14, 15, 16):
        assert np.max(np.abs(got[vis, col] - want[vis, col])) < 1e-5, col
    # smaller eigenvalues and signs where the smaller eigenvalue is determined at float precision
    for lo, hi, sg in ((1, 0, 2), (6, 5, 7)):
        det = vis & (want[:, lo] > want[:, hi] - 0.5)  # |lambda_lo| > 1e-5 |lambda_hi|
        assert det.sum() > 0.5 * vis.sum()
        assert np.max(np.abs(got[det, lo] - want[det, lo])) < 1e-5, lo
        assert np.array_equal(got[det, sg], want[det, sg])
    well = vis & (want[:, 3] > -2.9)
    assert np.array_equal(got[well, 4], want[well, 4])
    assert np.array_equal(okg[~vis], ok_want[~vis]) and np.all(okg[~vis] == 0)
    assert np.mean(okg[vis] == ok_want[vis]) > 0.999


def _upload_steps(gsn, steps, dec, sh_degree, device):
    st = gsn.Steps(steps.shape[0], sh_degree, device)
    sv, fv = st.view()
    sv.copy_(torch.tensor(steps.T.astype(np.float32), device=device))
    fv.copy_(torch.tensor(dec.T.astype(np.int32), device=device))
    return st


def test_labels_parity(gsn, ctx, sweep_case):
    cfg, t, res = sweep_case
    g, cam, o = cfg.init, cfg.cams[t], res["opts"]
    K = (g.sh_degree + 1) ** 2
    S1 = O.sum_blocks(res["per_view"][:1])
    prim, dec_p = O.solve(g, cam, o, S1, 1)
    aug = res["steps"]
    p32 = prim.astype(np.float32).astype(np.float64)
    a32 = aug.astype(np.float32).astype(np.float64)
    want, mw = L.labels(p32, a32, dec_p, K)
    sp = _upload_steps(gsn, p32, dec_p, g.sh_degree, ctx.device)
    sa = _upload_steps(gsn, a32, res["dec"], g.sh_degree, ctx.device)
    lab = torch.zeros(5, g.n, device=ctx.device)
    msk = torch.zeros(5, g.n, device=ctx.device)
    ctx.step_labels(sp, sa, lab, msk)
    got, mg = lab.cpu().numpy().T, msk.cpu().numpy().T
    assert mw.sum() > 1000
    assert np.array_equal(mg, mw)
    assert np.max(np.abs(got - want)[mw > 0]) < 1e-5
    # with feature status codes: kernels out of range are not labelled; the error sums against the
    # network's scales accumulate in fixed order
    rng = np.random.default_rng(9)
    ok = np.where(dec_p[:, 0] >= -1, 1, 0).astype(np.uint8)
    ok[rng.random(g.n) < 0.1] = 2
    alpha = rng.uniform(0.0, 1.5, (g.n, 5)).astype(np.float32)
    want2, mw2 = L.labels(p32, a32, dec_p, K, ok=ok)
    e_want = L.label_error(alpha.astype(np.float64), want2, mw2)
    err = torch.tensor([0.5, 2.0], dtype=torch.float64, device=ctx.device)
    ctx.step_labels(sp, sa, lab, msk, ok=torch.tensor(ok, device=ctx.device),
                    alpha=torch.tensor(alpha.T.copy(), device=ctx.device), err=err)
    got2, mg2 = lab.cpu().numpy().T, msk.cpu().numpy().T
    assert np.array_equal(mg2, mw2) and mw2.sum() < mw.sum()
    assert np.max(np.abs(got2 - want2)[mw2 > 0]) < 1e-5
    e = err.cpu().numpy()
    assert e[1] == 2.0 + e_want[1]
    assert abs(e[0] - 0.5 - e_want[0]) < 1e-5 * e_want[1]


def test_mlp_infer_parity(gsn, ctx):
    n = 5000
    F = random_features(n, 11)
    p = init_params(3) * 3.0
    mlp = gsn.MLP(p, ctx.device)
    ctx.mlp_reset(mlp)
    ok = np.ones(n, np.uint8)
    ok[::7] = 0
    ok[3::11] = 2
    alpha = torch.zeros(5, n, device=ctx.device)
    oor = torch.zeros(1, dtype=torch.int32, device=ctx.device)
    ctx.mlp_infer(mlp, torch.tensor(F.T.copy(), device=ctx.device), torch.tensor(ok, device=ctx.device), alpha,
                  oor)
    got = alpha.cpu().numpy().T
    # the library infers with fp16 weights: the oracle takes the same rounded weights
    want = L.forward(p.astype(np.float16).astype(np.float64), F.astype(np.float64))
    assert np.max(np.abs(got[ok == 1] - want[ok == 1])) < 1e-5
    assert np.all(got[ok != 1] == 0.0)
    assert int(oor.cpu()[0]) == int((ok == 2).sum())


def test_mlp_train_steps_parity(gsn, ctx):
    n = 5000
    rng = np.random.default_rng(8)
    F = random_features(n, 12)
    lab = rng.uniform(0.0, 1.5, (n, 5)).astype(np.float32)
    msk = (rng.random((n, 5)) < 0.6).astype(np.float32)
    p0 = init_params(4)
    mlp = gsn.MLP(p0, ctx.device)
    ctx.mlp_reset(mlp)
    dF = torch.tensor(F.T.copy(), device=ctx.device)
    dl = torch.tensor(lab.T.copy(), device=ctx.device)
    dm = torch.tensor(msk.T.copy(), device=ctx.device)
    loss = torch.zeros(1, dtype=torch.float64, device=ctx.device)
    grad = torch.zeros(gsn.GSN_MLP_PARAMS, device=ctx.device)
    p = p0.astype(np.float64)
    m = np.zeros(L.N_PARAMS)
    v = np.zeros(L.N_PARAMS)
    lr = 1e-2
    for step in range(1, 4):
        # the oracle continues from the library's float32 state, so each step is compared alone
        pg = mlp.params.cpu().numpy().astype(np.float64)
        mg = mlp.m.cpu().numpy().astype(np.float64)
        vg = mlp.v.cpu().numpy().astype(np.float64)
        lw, gw = L.loss_grad(pg, F, lab, msk)
        pw, _, _ = L.adam(pg, mg, vg, step, gw, lr=lr)
        ctx.mlp_train_step(mlp, dF, dl, dm, lr=lr, loss=loss, grad=grad)
        torch.cuda.synchronize()
        assert mlp.step == step
        assert abs(float(loss.cpu()[0]) - lw) <= 1e-5 * lw
        assert rel_inf(grad.cpu().numpy(), gw) < 1e-4
        # where |g| is not tiny each Adam step moves a weight by about lr; allow 1% of that
        pn = mlp.params.cpu().numpy().astype(np.float64)
        big = np.abs(gw) > 1e-3 * np.max(np.abs(gw))
        assert np.max(np.abs(pn - pw)[big]) < 1e-2 * lr
        assert np.max(np.abs(pn - pw)) < 2.0 * lr
    h = mlp.half.cpu().numpy().astype(np.float64)
    assert np.array_equal(h, mlp.params.cpu().numpy().astype(np.float16).astype(np.float64))


def test_scaled_apply_parity(gsn, ctx, sweep_case):
    cfg, t, res = sweep_case
    g, o = cfg.init, res["opts"]
    st32 = res["steps"].astype(np.float32)
    scale = np.random.default_rng(5).uniform(0.0, 1.5, (g.n, 5)).astype(np.float32)
    dg = gsn.DeviceGaussians.from_host(g)
    st = _upload_steps(gsn, st32.astype(np.float64), res["dec"], g.sh_degree, ctx.device)
    so = gsn.solve_opts(cfg.cams[t].width * cfg.cams[t].height)
    ctx.apply_step(dg, st, so, 31, scale=torch.tensor(scale.T.copy(), device=ctx.device))
    new_g = dg.to_host()
    new_o = O.apply(g, st32.astype(np.float64), res["dec"], o, 31, scale=scale.astype(np.float64))
    for a in ("pos", "rot", "scale", "opac", "sh"):
        assert np.allclose(getattr(new_g, a), getattr(new_o, a), rtol=2e-6, atol=2e-6), a


def test_learned_form_runs(gsn, ctx):
    from paper_2501_13975_amd.train import LocalNewtonTrainer
    cfg = make_config("c1", n=3000, width=160, height=120, n_views=6)
    tg = [torch.tensor(O.render(cfg.gt, c, O.opts()).img.astype(np.float32), device=ctx.device) for c in cfg.cams]
    dg = gsn.DeviceGaussians.from_host(cfg.init)
    tr = LocalNewtonTrainer(dg, cfg.cams, tg, 3)
    tr.enable_learned(init_params(0), every=2, lr=1e-2)
    for i in range(6):
        tr.sweep_learned(i % len(cfg.cams), i)
    torch.cuda.synchronize()
    a = tr.alpha[:, :dg.n].cpu().numpy()
    assert np.all(np.isfinite(a)) and np.all(a >= 0.0) and np.all(a <= 1.5)
    assert tr.mlp.step == 3
    e = tr.learned_error()
    assert e is not None and np.isfinite(e)
    for x in (dg.pos, dg.rot, dg.scale, dg.opac, dg.sh):
        assert torch.isfinite(x).all()
    tr.close()


def test_out_of_range_features_bring_the_full_rule_two_sweeps_later(gsn, ctx):
    """The fallback of the learned form: a learned sweep whose inference counts kernels with features
    out of the trained range (forced here by adding to the library's count after the real inference)
    makes the learned sweep two after it run the full rule (it trains the network), and only that one."""
    from paper_2501_13975_amd.train import LocalNewtonTrainer
    cfg = make_config("c1", n=3000, width=160, height=120, n_views=6)
    tg = [torch.tensor(O.render(cfg.gt, c, O.opts()).img.astype(np.float32), device=ctx.device) for c in cfg.cams]
    dg = gsn.DeviceGaussians.from_host(cfg.init)
    tr = LocalNewtonTrainer(dg, cfg.cams, tg, 3)
    tr.enable_learned(init_params(0), every=100, lr=1e-2)
    infer = tr.ctx.mlp_infer
    forced = {"sweep": None, "i": 0}

    def mlp_infer(*args, **kw):
        infer(*args, **kw)
        if forced["i"] == forced["sweep"]:
            tr.out_of_range.add_(1)  # on the device, after the library's count

    tr.ctx.mlp_infer = mlp_infer
    steps = []
    for i in range(1, 8):  # sweep 0 would be a scheduled full-rule sweep
        forced["i"] = i
        forced["sweep"] = 2
        tr.sweep_learned(i % len(cfg.cams), i)
        steps.append(tr.mlp.step)
    # the network trains only on full-rule sweeps: the one at i = 4, two after the counted i = 2
    assert steps == [0, 0, 0, 1, 1, 1, 1], steps
    assert tr.fallback_sweeps == 1
    tr.close()


def test_trained_network_predicts_the_overshoot_rule(gsn, ctx):
    """What the network gains over the method without it: trained on (features, alpha_eff) rows that
    plain full-rule sweeps log, it predicts the scale the overshoot rule applies to the primary-only
    step on held-out views better than the primary-only step itself (alpha = 1) and better than the
    best constant (the logged mean label of each group)."""
    from paper_2501_13975_amd.train import LocalNewtonTrainer, pretrain
    cfg = make_config("c1", n=6000, width=200, height=150, n_views=12)
    tg = [torch.tensor(O.render(cfg.gt, c, O.opts()).img.astype(np.float32), device=ctx.device) for c in cfg.cams]
    dg = gsn.DeviceGaussians.from_host(cfg.init)
    tr = LocalNewtonTrainer(dg, cfg.cams, tg, 3, solve_kw={"step_frac": 0.3})
    train_log, held = [], []
    for i, t in enumerate(range(8)):
        tr.log_sweep(t, train_log, seed=i)
    for t in range(8, 12):
        tr.log_sweep(t, held, seed=100 + t)
    mlp = gsn.MLP(init_params(0), ctx.device)
    ctx.mlp_reset(mlp)
    curve = pretrain(ctx, mlp, train_log, epochs=40, batch=4096, lr=1e-2)
    print(f"\n[gain] pretraining loss per epoch: first {curve[0]:.4f} last {curve[-1]:.4f}", flush=True)
    assert curve[-1] < curve[0]
    F = torch.cat([x[0] for x in held], 1).contiguous()
    Lb = torch.cat([x[1] for x in held], 1).cpu().numpy()
    M = torch.cat([x[2] for x in held], 1).cpu().numpy()
    m = F.shape[1]
    assert m > 1000
    alpha = torch.zeros(5, m, device=ctx.device)
    ctx.mlp_infer(mlp, F, torch.ones(m, dtype=torch.uint8, device=ctx.device), alpha)
    a = alpha.cpu().numpy()
    Lt = torch.cat([x[1] for x in train_log], 1).cpu().numpy()
    Mt = torch.cat([x[2] for x in train_log], 1).cpu().numpy()
    mean = (Lt * Mt).sum(1) / Mt.sum(1)
    err = lambda pred: float((np.abs(pred - Lb) * M).sum() / M.sum())  # noqa: E731
    e_mlp, e_one, e_mean = err(a), err(np.ones_like(Lb)), err(np.broadcast_to(mean[:, None], Lb.shape))
    print(f"[gain] held-out mean |alpha - alpha_eff|: network {e_mlp:.4f}, alpha=1 {e_one:.4f}, "
          f"mean label {e_mean:.4f} ({int(M.sum())} entries)", flush=True)
    assert e_mlp < e_one and e_mlp < e_mean
    tr.close()
