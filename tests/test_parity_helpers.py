"""Host-side checks of the layout conversions and frame helpers the GPU parity tests rely on."""
import numpy as np

from synth.scenes import make_config
from tests.parity import (gpu_blocks_to_summed, oracle_frames, summed_to_gpu_blocks, sym_from_packed,
                          zstats_to_frame)
from oracle import oracle as O


def test_block_layout_round_trip():
    rng = np.random.default_rng(0)
    n, V = 7, 4
    S = rng.standard_normal((n, 40 + 10 * V))
    for off in (3, 15, 27):  # the three 3x3 blocks are symmetric
        M = S[:, off:off + 9].reshape(n, 3, 3)
        S[:, off:off + 9] = (M + M.transpose(0, 2, 1)).reshape(n, 9)
    assert np.array_equal(gpu_blocks_to_summed(summed_to_gpu_blocks(S, V), V), S)


def test_packed_order():
    p = np.arange(6, dtype=float)[:, None]
    H = sym_from_packed(p, 3)[0]
    assert H[0, 0] == 0 and H[0, 1] == 1 and H[0, 2] == 2 and H[1, 1] == 3 and H[1, 2] == 4 and H[2, 2] == 5


def test_oracle_frames_are_eigenvectors():
    cfg = make_config("c1", n=300, width=160, height=120, n_views=4)
    cam = cfg.cams[0]
    out, ok = O.project64(cfg.init, cam, kappa=0.3)
    c, s = oracle_frames(cfg.init, cam)
    for k in np.nonzero(ok)[0]:
        S = np.array([[out[k, 2], out[k, 3]], [out[k, 3], out[k, 4]]])
        w, V = np.linalg.eigh(S)
        e1 = np.array([c[k], s[k]])
        assert abs(abs(e1 @ V[:, 1]) - 1.0) < 1e-9
        assert abs(e1 @ S @ e1 - w[1]) <= 1e-9 * w[1]


def test_zstats_frame_rotation_is_orthogonal_change_of_variables():
    # a quadratic form in (pi, Q) keeps its value when both the point and the statistics are rotated
    rng = np.random.default_rng(1)
    n = 5
    Z = np.zeros((n, 91))
    Z[:, :9] = rng.standard_normal((n, 9))
    H = rng.standard_normal((n, 9, 9))
    Z[:, 9:90] = (H + H.transpose(0, 2, 1)).reshape(n, 81)
    th = rng.uniform(0, 2 * np.pi, n)
    c, s = np.cos(th), np.sin(th)
    Zf = zstats_to_frame(Z, c, s)
    for k in range(n):
        V = np.array([[c[k], -s[k]], [s[k], c[k]]])
        dpf = rng.standard_normal(2)
        dQf = rng.standard_normal((2, 2))
        dQf = dQf + dQf.T
        dp = V @ dpf
        dQ = V @ dQf @ V.T
        x = np.concatenate([dp, [dQ[0, 0], dQ[0, 1], dQ[1, 1]], rng.standard_normal(4)])
        xf = np.concatenate([dpf, [dQf[0, 0], dQf[0, 1], dQf[1, 1]], x[5:]])
        g, Hm = Z[k, :9], Z[k, 9:90].reshape(9, 9)
        gf, Hf = Zf[k, :9], Zf[k, 9:90].reshape(9, 9)
        assert np.isclose(g @ x, gf @ xf) and np.isclose(x @ Hm @ x, xf @ Hf @ xf)


def test_ssim_reach_is_the_two_window_radius_square():
    from tests.parity import ssim_reach
    mask = np.ones((40, 50), bool)
    mask[20, 3] = False
    reach = ssim_reach(mask)
    ys, xs = np.nonzero(reach)
    assert (ys.min(), ys.max(), xs.min(), xs.max()) == (10, 30, 0, 13)
    assert reach.sum() == 21 * 14
    assert not ssim_reach(np.ones((8, 8), bool)).any()


def test_kernels_in_reach_takes_each_tile_prefix_to_its_deepest_pixel():
    from types import SimpleNamespace

    from tests.parity import kernels_in_reach
    # two 16x16 tiles side by side; tile 0 lists kernels 5, 3, 7, tile 1 lists 1, 2
    fr = SimpleNamespace(cam=SimpleNamespace(width=32, height=16), tile_start=np.array([0, 3, 5]),
                         ids=np.array([5, 3, 7, 1, 2]), ncontrib=np.zeros((16, 32), np.int64))
    fr.ncontrib[4, 2] = 1  # last composited entry of that pixel: index 0 of tile 0's list
    fr.ncontrib[9, 20] = 2
    reach = np.zeros((16, 32), bool)
    reach[4, 2] = True
    got = kernels_in_reach(fr, reach, 8)
    # up to and including the entry after the last composited one (the stopping entry)
    assert np.array_equal(np.nonzero(got)[0], [3, 5])
    reach[9, 20] = True
    assert np.array_equal(np.nonzero(kernels_in_reach(fr, reach, 8))[0], [1, 2, 3, 5])
