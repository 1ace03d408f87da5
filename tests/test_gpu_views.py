"""GPU tests of gsn_accumulate_views: the views of a sweep rendered and accumulated with their work
overlapped on the library's streams give blocks and losses identical bit for bit to the same
renders and accumulations issued one after another (primary first, then the secondaries), with
growing and reserved frames, with more views than streams, for the secondaries alone after the
primary, and with the profiler on (views in sequence on the context's stream)."""
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
def case():
    cfg = make_config("c1", n=4000, width=200, height=150, n_views=10)
    tg = [O.render(cfg.gt, c, O.opts()).img.astype(np.float32) for c in cfg.cams]
    return cfg, tg


def _trainer(gsn, cfg, tg, nsec, reserve):
    from paper_2501_13975_amd.train import LocalNewtonTrainer
    dg = gsn.DeviceGaussians.from_host(cfg.init)
    tr = LocalNewtonTrainer(dg, cfg.cams, [torch.tensor(x, device="cuda") for x in tg], nsec, 0.2)
    if reserve:
        tr.reserve_frames()
    return tr


def _views(tr, t):
    return ([tr.ccams[t]] + [tr.chalf[j] for j in tr.knn[t]],
            [tr.targets[t]] + [tr.half_targets[j] for j in tr.knn[t]])


def _sequential(tr, t):
    tr.ctx.blocks_zero(tr.blocks)
    tr.loss.zero_()
    cams, tgts = _views(tr, t)
    for slot, (cam, tgt) in enumerate(zip(cams, tgts)):
        tr.ctx.render(tr.g, cam, tr.ro, tr.frames[slot])
        tr.ctx.accumulate_hessian(tr.g, tr.frames[slot], tgt, tr.lo, slot, tr.blocks, tr.loss[slot])
    torch.cuda.synchronize()
    return tr.blocks.view().clone(), tr.loss.clone()


@pytest.mark.parametrize("nsec,reserve", [(3, False), (3, True), (8, True)])
def test_overlapped_views_equal_sequential_calls(gsn, case, nsec, reserve):
    cfg, tg = case
    tr = _trainer(gsn, cfg, tg, nsec, reserve)
    for t in (0, 4, 7):
        print(f"\n[views] |N_t|={nsec} reserved={reserve} t={t}", flush=True)
        b_seq, l_seq = _sequential(tr, t)
        tr.loss.zero_()
        tr.accumulate(t)  # gsn_accumulate_views over the primary and its secondaries
        torch.cuda.synchronize()
        assert torch.equal(tr.blocks.view(), b_seq)
        assert torch.equal(tr.loss, l_seq)
        # the secondaries alone, after the primary accumulated on its own
        tr.ctx.blocks_zero(tr.blocks)
        tr.loss.zero_()
        cams, tgts = _views(tr, t)
        tr.ctx.render(tr.g, cams[0], tr.ro, tr.frames[0])
        tr.ctx.accumulate_hessian(tr.g, tr.frames[0], tgts[0], tr.lo, 0, tr.blocks, tr.loss[0])
        tr.ctx.accumulate_views(tr.g, cams[1:], tr.frames[1:len(cams)], tgts[1:], tr.ro, tr.lo, tr.blocks,
                                tr.loss[1:], first_slot=1)
        torch.cuda.synchronize()
        assert torch.equal(tr.blocks.view(), b_seq)
        assert torch.equal(tr.loss, l_seq)
    st, stats, msg = tr.ctx.sync_status()
    assert st == 0 and not any(stats.values()), (st, stats, msg)
    tr.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_held_shares_give_the_primary_system_then_the_sweep(gsn, case, precision):
    """Views accumulated with their shares of the summed rows held in the frames: after the primary's
    share the solve on the primary's slot alone equals the solve of the blocks of the primary alone,
    and after the secondaries' shares the blocks equal those of the sequential calls."""
    cfg, tg = case
    tr = _trainer(gsn, cfg, tg, 3, True)
    for t in (2, 6):
        print(f"\n[held shares] precision={precision} t={t}", flush=True)
        b_seq, l_seq = _sequential(tr, t)
        so = tr.solve_opts(t)
        so.precision = precision
        sp = tr._primary_only(so)
        cams, tgts = _views(tr, t)
        # the primary alone, its blocks and primary-only step
        tr.ctx.blocks_zero(tr.blocks)
        tr.ctx.render(tr.g, cams[0], tr.ro, tr.frames[0])
        tr.ctx.accumulate_hessian(tr.g, tr.frames[0], tgts[0], tr.lo, 0, tr.blocks, tr.loss[0])
        tr.ctx.local_newton_solve(tr.g, cams[0], tr.blocks, so, tr.steps)
        torch.cuda.synchronize()
        s_prim, f_prim = [x.clone() for x in tr.steps.view()]
        # every view, shares held; the primary's added, solved on slot 0 alone
        tr.loss.zero_()
        tr._accumulate_held(t)
        tr.ctx.add_view_shares(tr.blocks, tr.frames[:1])
        tr.ctx.local_newton_solve(tr.g, cams[0], tr.blocks, sp, tr.steps)
        torch.cuda.synchronize()
        assert torch.equal(tr.steps.view()[0], s_prim)
        assert torch.equal(tr.steps.view()[1], f_prim)
        tr.ctx.add_view_shares(tr.blocks, tr.frames[1:len(cams)])
        torch.cuda.synchronize()
        assert torch.equal(tr.blocks.view(), b_seq)
        assert torch.equal(tr.loss, l_seq)
    with pytest.raises(gsn.GsnError):  # more frames than the entry takes
        tr.ctx.add_view_shares(tr.blocks, [tr.frames[0]] * 10)
    st, stats, msg = tr.ctx.sync_status()
    assert st == 0 and not any(stats.values()), (st, stats, msg)
    tr.close()


def test_profiled_views_run_in_sequence_with_equal_results(gsn, case):
    cfg, tg = case
    tr = _trainer(gsn, cfg, tg, 3, True)
    b_seq, l_seq = _sequential(tr, 5)
    tr.ctx.profile_enable(True)
    tr.loss.zero_()
    tr.accumulate(5)
    stages, _ = tr.ctx.profile_read()
    tr.ctx.profile_enable(False)
    assert torch.equal(tr.blocks.view(), b_seq) and torch.equal(tr.loss, l_seq)
    assert stages["raster_bwd"][1] == 4 and stages["chain"][1] == 4  # one timed stage per view
    tr.close()


def test_views_argument_errors(gsn, case):
    cfg, tg = case
    tr = _trainer(gsn, cfg, tg, 3, True)
    cams, tgts = _views(tr, 1)
    with pytest.raises(gsn.GsnError):  # one frame given twice
        tr.ctx.accumulate_views(tr.g, cams[:2], [tr.frames[0], tr.frames[0]], tgts[:2], tr.ro, tr.lo, tr.blocks)
    with pytest.raises(gsn.GsnError):  # slots past the blocks' views
        tr.ctx.accumulate_views(tr.g, cams, tr.frames[:4], tgts, tr.ro, tr.lo, tr.blocks, first_slot=1)
    tr.close()
