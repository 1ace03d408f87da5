"""GPU parity of the batched solve (several scenes in one persistent launch), its
HIP-graph replay and its launch-shape autotuner: identical to per-scene solves,
which match the FP64 oracle on the same (float32-rounded) blocks."""
import numpy as np
import pytest

from oracle import oracle as O
from synth.scenes import make_config
from tests.parity import STEP_GROUPS, rel_inf, summed_to_gpu_blocks

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
def scenes(gsn, ctx):
    """Three scenes of different sizes, SH degrees and view counts with oracle blocks."""
    out = []
    for name, kw, V in (("c1", dict(n=3000, width=160, height=120, n_views=6), 4),
                        ("c1", dict(n=1200, width=128, height=96, n_views=4), 2),
                        ("c0", {}, 1)):
        cfg = make_config(name, **kw)
        tg = [O.render(cfg.gt, c, O.opts()).img.astype(np.float32) for c in cfg.cams]
        knn = O.camera_knn(cfg.cams, cfg.init, V - 1) if V > 1 else None
        res = O.sweep(cfg.init, cfg.cams, tg, 0, knn, O.opts(lambda_ssim=0.2))
        S32 = res["summed"].astype(np.float32).astype(np.float64)
        g = cfg.init
        dg = gsn.DeviceGaussians.from_host(g)
        b = gsn.Blocks(g.n, V, ctx.device)
        b.view().copy_(torch.tensor(summed_to_gpu_blocks(S32, V), dtype=torch.float32, device=ctx.device))
        cam = cfg.cams[0]
        so = gsn.solve_opts(cam.width * cam.height)
        out.append(dict(cfg=cfg, g=g, dg=dg, blocks=b, cam=cam, ccam=gsn.camera(cam), so=so, V=V, S32=S32,
                        opts=res["opts"]))
    return out


def _solve_each(gsn, ctx, scenes):
    ref = []
    for sc in scenes:
        st = gsn.Steps(sc["g"].n, sc["g"].sh_degree, ctx.device)
        ctx.local_newton_solve(sc["dg"], sc["ccam"], sc["blocks"], sc["so"], st)
        ref.append(st)
    torch.cuda.synchronize()
    return [(s.view()[0].cpu().numpy().copy(), s.view()[1].cpu().numpy().copy()) for s in ref]


def _items(gsn, ctx, scenes):
    steps = [gsn.Steps(sc["g"].n, sc["g"].sh_degree, ctx.device) for sc in scenes]
    items = [(sc["dg"], sc["ccam"], sc["blocks"], sc["so"], st) for sc, st in zip(scenes, steps)]
    return items, steps


def _same(a, b):
    (sa, fa), (sb, fb) = a, b
    assert np.array_equal(fa, fb)
    assert np.max(np.abs(sa - sb)) <= 1e-6 * max(np.max(np.abs(sa)), 1e-30)


def test_batched_equals_per_scene_and_oracle(gsn, ctx, scenes):
    ref = _solve_each(gsn, ctx, scenes)
    items, steps = _items(gsn, ctx, scenes)
    ctx.solve_batched(items)
    torch.cuda.synchronize()
    for sc, r, st in zip(scenes, ref, steps):
        got = (st.view()[0].cpu().numpy(), st.view()[1].cpu().numpy())
        _same(got, r)
        want, dec = O.solve(sc["g"], sc["cam"], sc["opts"], sc["S32"], sc["V"])
        vis = dec[:, 0] != -2
        same = np.all(got[1][:4].T == dec[:, :4], axis=1) & vis
        assert same[vis].mean() > 0.999
        K = (sc["g"].sh_degree + 1) ** 2
        for name, sl in list(STEP_GROUPS.items()) + [("colour", slice(11, 11 + 3 * K))]:
            assert rel_inf(got[0][sl].T[same], want[same, sl]) < 1e-5, name


def test_graph_replays_match_eager(gsn, ctx, scenes):
    ref = _solve_each(gsn, ctx, scenes)
    items, steps = _items(gsn, ctx, scenes)
    graph = ctx.solve_graph(items)
    for _ in range(3):
        for st in steps:  # eager work between replays
            st.data.fill_(-7.0)
            st.flags.fill_(99)
        graph.launch()
        torch.cuda.synchronize()
        for r, st in zip(ref, steps):
            _same((st.view()[0].cpu().numpy(), st.view()[1].cpu().numpy()), r)
    graph.close()


def test_autotuner_picks_a_candidate_and_keeps_results(gsn, ctx, scenes):
    ref = _solve_each(gsn, ctx, scenes)
    items, steps = _items(gsn, ctx, scenes)
    block, grid = ctx.solve_tune(items)
    assert block in (64, 128, 256) and grid > 0
    for st in steps:
        st.data.fill_(0.0)
    ctx.solve_batched(items)
    torch.cuda.synchronize()
    for r, st in zip(ref, steps):
        _same((st.view()[0].cpu().numpy(), st.view()[1].cpu().numpy()), r)


def test_batched_rejects_bad_input(gsn, ctx, scenes):
    with pytest.raises(gsn.GsnError):
        ctx.solve_batched([])
    sc = scenes[0]
    bad = gsn.Steps(sc["g"].n + 1, sc["g"].sh_degree, ctx.device)
    with pytest.raises(gsn.GsnError):
        ctx.solve_batched([(sc["dg"], sc["ccam"], sc["blocks"], sc["so"], bad)])
