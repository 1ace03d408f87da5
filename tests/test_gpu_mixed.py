"""The mixed-precision form of the solve: the BF16 matrix-core colour Gram matrices
against B B^T in double on the same directions (checks the instruction's lane
layout), and the mixed solve's error against the FP64 oracle on the oracle's own
blocks (reported, and bounded where the step is determined)."""
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


@pytest.mark.parametrize("sh_degree,V", [(3, 4), (3, 2), (1, 3), (0, 1)])
def test_sh_gram_matches_double(gsn, ctx, sh_degree, V):
    rng = np.random.default_rng(10 + V)
    n = 1000 + 13  # several waves of 16 kernels and a ragged tail
    K = (sh_degree + 1) ** 2
    rows = np.zeros((31 + 10 * V, n), np.float32)
    dirs = rng.standard_normal((V, n, 3))
    dirs /= np.linalg.norm(dirs, axis=2, keepdims=True)
    cover = rng.random((V, n)) < 0.7
    for v in range(V):
        rows[30 + 10 * v + 6:30 + 10 * v + 9] = dirs[v].T
        rows[30 + 10 * v + 9] = np.where(cover[v], rng.uniform(0.1, 2.0, n), 0.0)
    b = gsn.Blocks(n, V, ctx.device)
    b.view().copy_(torch.tensor(rows, device=ctx.device))
    out = torch.zeros(10, n, device=ctx.device)
    ctx.sh_gram(b, sh_degree, out)
    got = out.cpu().numpy()
    for k in range(n):
        act = [v for v in range(V) if cover[v, k]]
        Bm = np.zeros((4, K))
        for i, v in enumerate(act):
            Bm[i] = O.sh_basis(K, rows[30 + 10 * v + 6:30 + 10 * v + 9, k].astype(np.float64))
        G = Bm @ Bm.T
        idx = 0
        for i in range(4):
            for j in range(i, 4):
                assert abs(got[idx, k] - G[i, j]) <= 1e-4 * max(1.0, abs(G[i, j])), (k, i, j, got[idx, k], G[i, j])
                idx += 1


def test_mixed_solve_error_against_oracle(gsn, ctx):
    cfg = make_config("c1", n=4000, width=200, height=150, n_views=8)
    tg = [O.render(cfg.gt, c, O.opts()).img.astype(np.float32) for c in cfg.cams]
    g, t = cfg.init, 3
    knn = O.camera_knn(cfg.cams, g, 3)
    res = O.sweep(g, cfg.cams, tg, t, knn, O.opts(lambda_ssim=0.2))
    S32 = res["summed"].astype(np.float32).astype(np.float64)
    want, dec = O.solve(g, cfg.cams[t], res["opts"], S32, 4)
    dg = gsn.DeviceGaussians.from_host(g)
    b = gsn.Blocks(g.n, 4, ctx.device)
    b.view().copy_(torch.tensor(summed_to_gpu_blocks(S32, 4), dtype=torch.float32, device=ctx.device))
    st = gsn.Steps(g.n, g.sh_degree, ctx.device)
    cam = cfg.cams[t]
    so = gsn.solve_opts(cam.width * cam.height, precision=1)
    ctx.profile_enable(True)
    ctx.local_newton_solve(dg, gsn.camera(cam), b, so, st)
    _, counts = ctx.profile_read()
    ctx.profile_enable(False)
    got, fl = (x.cpu().numpy() for x in st.view())
    vis = dec[:, 0] != -2
    same = np.all(fl[:4].T == dec[:, :4], axis=1) & vis
    errs = {"decision_agreement": float(same[vis].mean()), "fp64_resolves": counts["fp64_solves"]}
    K = 16
    for name, sl in STEP_GROUPS.items():
        errs[name] = rel_inf(got[sl].T[same], want[same, sl])
    col = slice(11, 11 + 3 * K)
    d = np.abs(got[col].T - want[:, col]).max(1)
    scale = np.abs(want[:, col]).max(1)
    rel = d[vis & (scale > 0)] / scale[vis & (scale > 0)]
    errs["colour_rel_p50"] = float(np.percentile(rel, 50))
    errs["colour_rel_p99"] = float(np.percentile(rel, 99))
    errs["colour_rel_max"] = float(rel.max())
    print("\n[mixed solve vs FP64 oracle] " + " ".join(f"{k}={v:.3g}" for k, v in errs.items()), flush=True)
    assert errs["decision_agreement"] > 0.99
    for name in STEP_GROUPS:
        assert errs[name] < 1e-4, (name, errs[name])
    assert errs["colour_rel_p50"] < 1e-4 and errs["colour_rel_p99"] < 1e-3
