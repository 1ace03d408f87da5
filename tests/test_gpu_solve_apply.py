"""GPU tests of gsn_solve_apply: the solve with the update fused into its launch leaves the same
steps, decisions, parameters and opacity-bound count, bit for bit, as gsn_local_newton_solve
followed by gsn_apply_step, in the plain and the mixed form, for every group and for subsets."""
import numpy as np
import pytest

from oracle import oracle as O
from synth.scenes import make_config

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_13975_amd import gsn as G
    return G


@pytest.fixture(scope="module")
def trainer(gsn):
    from paper_2501_13975_amd.train import LocalNewtonTrainer
    cfg = make_config("c1", n=5000, width=200, height=150, n_views=8)
    tg = [O.render(cfg.gt, c, O.opts()).img.astype(np.float32) for c in cfg.cams]
    dg = gsn.DeviceGaussians.from_host(cfg.init)
    tr = LocalNewtonTrainer(dg, cfg.cams, [torch.tensor(x, device="cuda") for x in tg], 3, 0.2)
    yield tr
    tr.close()


def _params(g):
    return [x.clone() for x in (g.pos, g.rot, g.scale, g.opac, g.sh)]


def _restore(g, ps):
    for dst, src in zip((g.pos, g.rot, g.scale, g.opac, g.sh), ps):
        dst.copy_(src)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("mask", [31, 12, 1, 16])
def test_fused_update_equals_solve_then_apply(gsn, trainer, precision, mask):
    tr = trainer
    for t in (1, 5):
        print(f"\n[solve_apply] precision={precision} mask={mask} t={t}", flush=True)
        tr.accumulate(t)
        so = tr.solve_opts(t)
        so.precision = precision
        so.step_frac = 1.0  # whole steps, so that the bounds and clamps bind for some kernels
        p0 = _params(tr.g)
        tr.ctx.profile_enable(True)
        tr.ctx.local_newton_solve(tr.g, tr.ccams[t], tr.blocks, so, tr.steps)
        tr.ctx.apply_step(tr.g, tr.steps, so, mask)
        _, c_ref = tr.ctx.profile_read()
        torch.cuda.synchronize()
        s_ref, f_ref = [x.clone() for x in tr.steps.view()]
        p_ref = _params(tr.g)
        _restore(tr.g, p0)
        tr.steps.data.fill_(float("nan"))
        tr.ctx.profile_enable(True)  # counters back to zero
        tr.ctx.solve_apply(tr.g, tr.ccams[t], tr.blocks, so, tr.steps, mask)
        _, c_fused = tr.ctx.profile_read()
        tr.ctx.profile_enable(False)
        torch.cuda.synchronize()
        s_f, f_f = tr.steps.view()
        assert torch.equal(s_f, s_ref) and torch.equal(f_f, f_ref)
        for a, b in zip(_params(tr.g), p_ref):
            assert torch.equal(a, b)
        assert any(not torch.equal(a, b) for a, b in zip(p_ref, p0))  # the update did move something
        for key in ("opacity_bound", "solved", "clamped_colour", "escalated_position"):
            assert c_fused[key] == c_ref[key], key
        _restore(tr.g, p0)
    st, stats, msg = tr.ctx.sync_status()
    assert st == 0 and not any(stats.values()), (st, stats, msg)


def test_solve_apply_rejects_unknown_groups(gsn, trainer):
    tr = trainer
    so = tr.solve_opts(0)
    with pytest.raises(gsn.GsnError):
        tr.ctx.solve_apply(tr.g, tr.ccams[0], tr.blocks, so, tr.steps, 32)
