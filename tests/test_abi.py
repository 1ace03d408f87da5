"""The C-ABI library loads and exports every entry point include/gsn.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsn.h")
LIB = os.path.join(ROOT, "paper_2501_13975_amd", "libgsn.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsn_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_step():
    names = declared_functions()
    for required in ("gsn_render", "gsn_accumulate_hessian", "gsn_local_newton_solve", "gsn_apply_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libgsn.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_helpers_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("libgsn.so not built")
    lib = ctypes.CDLL(LIB)
    lib.gsn_blocks_floats.restype = ctypes.c_int64
    lib.gsn_steps_floats.restype = ctypes.c_int64
    assert lib.gsn_blocks_floats(1000, 4) == (30 + 40 + 1) * 1000
    assert lib.gsn_steps_floats(10, 3) == (11 + 48) * 10
    assert lib.gsn_steps_floats(10, 4) == 0


def test_camera_knn_matches_oracle():
    """Host-side KNN of the library against the oracle's (Sec. 4.1)."""
    if not os.path.exists(LIB):
        pytest.skip("libgsn.so not built")
    import numpy as np
    from oracle import oracle as O
    from synth.scenes import make_config
    from paper_2501_13975_amd import gsn
    cfg = make_config("c1", n=300, width=16, height=16, n_views=50)
    cen = np.stack([c.center for c in cfg.cams])
    sc = np.asarray(cfg.gt.pos, np.float64).mean(1)
    assert np.array_equal(gsn.camera_knn(cen, sc, 3), O.knn(cen, sc, 3))
    with pytest.raises(gsn.GsnError):
        gsn.camera_knn(cen, sc, 50)


def test_half_resolution_camera_matches_oracle():
    """The library's secondary-target camera (Sec. 4.3) equals the oracle's, bit for bit."""
    if not os.path.exists(LIB):
        pytest.skip("libgsn.so not built")
    import numpy as np
    from oracle import oracle as O
    from synth.scenes import make_config
    from paper_2501_13975_amd import gsn
    for cfg in (make_config("c1", n=10, n_views=5), make_config("c2", n=10, n_views=5), make_config("c0", n=10)):
        for c in cfg.cams:
            h = gsn.camera_half(gsn.camera(c))
            o = O.half_camera(c)
            got = [h.fx, h.fy, h.cx, h.cy, h.width, h.height, h.znear]
            want = [np.float32(o.fx), np.float32(o.fy), np.float32(o.cx), np.float32(o.cy), o.width, o.height,
                    np.float32(o.znear)]
            assert got == [float(x) if isinstance(x, np.float32) else x for x in want]
            assert list(h.R) == [float(x) for x in np.asarray(o.R, np.float32).ravel()]
    c = gsn.camera(make_config("c0", n=10).cams[0])
    c.width = 1
    with pytest.raises(gsn.GsnError):
        gsn.camera_half(c)


def _enum_values(prefix):
    src = open(HEADER).read()
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(" + prefix + r"[A-Z0-9_]+)\s*=\s*(\d+)", src)}


def test_binding_counter_names_follow_the_header():
    """The binding's names of the profile counters and of the status counters match the header's enums."""
    from paper_2501_13975_amd import gsn
    counts = _enum_values("GSN_COUNT_")
    assert len(gsn.Context.COUNTERS) == counts["GSN_COUNT_N"]
    assert gsn.Context.COUNTERS[counts["GSN_COUNT_BWD_STAGED"]] == "bwd_staged"
    assert gsn.Context.COUNTERS[counts["GSN_COUNT_SOLVE_ESCALATED"]] == "escalated_position"
    assert gsn.Context.COUNTERS[counts["GSN_COUNT_SOLVE_FALLBACK"] + 3] == "fallback_opacity"
    assert gsn.Context.COUNTERS[counts["GSN_COUNT_SOLVE_CLAMPED"] + 3] == "clamped_colour"
    assert gsn.Context.COUNTERS[counts["GSN_COUNT_SOLVED"]] == "solved"
    assert gsn.Context.COUNTERS[counts["GSN_COUNT_OPAC_BOUND"]] == "opacity_bound"
    stats = _enum_values("GSN_STAT_")
    assert len(gsn.STATS) == stats["GSN_STAT_N"]
    assert gsn.STATS[stats["GSN_STAT_PAIRS_NEEDED"]] == "pairs_needed"
    stages = _enum_values("GSN_STAGE_")
    assert len(gsn.Context.STAGES) == stages["GSN_STAGE_COUNT"]


# every option and handle struct of include/gsn.h against the binding's ctypes mirror
_STRUCTS = {
    "gsn_gaussians": "CGaussians", "gsn_camera": "CCamera", "gsn_render_opts": "CRenderOpts",
    "gsn_loss_opts": "CLossOpts", "gsn_solve_opts": "CSolveOpts", "gsn_blocks": "CBlocks", "gsn_steps": "CSteps",
    "gsn_first_order_opts": "CFirstOrderOpts", "gsn_solve_item": "CSolveItem", "gsn_mlp": "CMlp",
    "gsn_adam_opts": "CAdamOpts",
}


def _c_layouts(tmp_path):
    """sizeof and the offset of every field of each struct, from a host C program built with gcc."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    src = open(HEADER).read()
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gsn.h"', "int main(void) {"]
    for cname in _STRUCTS:
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + r"\s*;", src)
        assert body, cname
        text = re.sub(r"/\*.*?\*/", "", body.group(1), flags=re.S)
        fields = []
        for decl in text.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            m = re.match(r"(.*?)\s*([A-Za-z_][A-Za-z0-9_]*)\s*(\[[^\]]*\])?\s*$", decl.split(",")[0])
            assert m, decl
            fields.append(m.group(2))
            for extra in decl.split(",")[1:]:
                fields.append(re.sub(r"[\s*]|\[.*\]", "", extra))
        lines.append(f'printf("{cname} %zu", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf(" {f}=%zu", offsetof({cname}, {f}));')
        lines.append('printf("\\n");')
    lines.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(c), "-o", str(exe)])
    out = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        parts = line.split()
        out[parts[0]] = (int(parts[1]), {k: int(v) for k, v in (p.split("=") for p in parts[2:])})
    return out


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors in gsn.py have the size and field offsets of the header's structs (checked
    on the host with gcc), so that no option is marshalled into the wrong field."""
    from paper_2501_13975_amd import gsn
    layouts = _c_layouts(tmp_path)
    for cname, pyname in _STRUCTS.items():
        size, offs = layouts[cname]
        cls = getattr(gsn, pyname)
        assert ctypes.sizeof(cls) == size, (cname, ctypes.sizeof(cls), size)
        py = {name: getattr(cls, name).offset for name, _ in cls._fields_}
        assert list(py) == list(offs), (cname, list(py), list(offs))
        assert py == offs, (cname, py, offs)
