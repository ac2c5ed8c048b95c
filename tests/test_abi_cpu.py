"""CPU-side checks of the C-ABI library: it loads, exports every function
include/swgs.h declares, and its host-only entry points behave.  No GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2409_07759_amd import swgs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_function():
    names = swgs.header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(swgs._lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_function():
    names = swgs.header_functions()
    assert sorted(n for n in names) == sorted(swgs._sigs)


def test_version():
    assert swgs.swgs_version() == 1


def test_record_bytes():
    assert swgs.swgs_record_bytes(0, 0) == 32
    assert swgs.swgs_record_bytes(40000, 0) == 32 + 40000 * (16 + 4 * 14)
    assert swgs.swgs_record_bytes(10, 3) == 32 + 10 * (16 + 4 * 59)
    assert swgs.swgs_record_bytes(10, 4) == 0


def test_step_cfg_defaults():
    c = swgs.step_cfg()
    assert c.struct_size == ctypes.sizeof(swgs.SwgsStepCfg)
    assert c.noise_lr == 5e4 and c.lambda_opacity == pytest.approx(2e-2) and c.lambda_scale == pytest.approx(1e-2)
    assert c.beta1 == pytest.approx(0.9) and c.eps == pytest.approx(1e-15) and c.reloc_n_max == 32
    assert c.noise_k == 100.0 and c.noise_t0 == pytest.approx(0.005)


def test_struct_sizes_match_the_header():
    # swgs_view: 4 int32 + 16 doubles + 4 floats
    assert ctypes.sizeof(swgs.SwgsView) == 16 + 16 * 8 + 16
    assert ctypes.sizeof(swgs.SwgsPool) == 8 + 16 + 7 * 8
    assert ctypes.sizeof(swgs.SwgsPlanOpts) == 8 + 16 + 8


def test_struct_layouts_match_a_c_compiler(tmp_path):
    """sizeof / offsetof of every ABI struct as gcc sees the header equal the
    ctypes mirrors the binding uses."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    structs = {"swgs_pool": swgs.SwgsPool, "swgs_view": swgs.SwgsView, "swgs_plan_opts": swgs.SwgsPlanOpts,
               "swgs_step_cfg": swgs.SwgsStepCfg, "swgs_server_opts": swgs.SwgsServerOpts,
               "swgs_request": swgs.SwgsRequest, "swgs_serve_stats": swgs.SwgsServeStats,
               "swgs_player_opts": swgs.SwgsPlayerOpts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "swgs.h"', "int main(void) {"]
    for cname, ct in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in ct._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {" ".join(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, ct in structs.items():
        assert got[f"{cname} size"] == ctypes.sizeof(ct), cname
        for fname, _ in ct._fields_:
            assert got[f"{cname} {fname}"] == getattr(ct, fname).offset, (cname, fname)


def test_buffer_enum_matches_the_header():
    txt = open(os.path.join(ROOT, "include", "swgs.h")).read()
    block = txt[txt.index("SWGS_BUF_ACTIVE_LIST = 0"):txt.index("SWGS_BUF_COUNT_")]
    names = re.findall(r"(SWGS_BUF_[A-Z_]+)", block)
    for i, n in enumerate(names):
        assert getattr(swgs, n) == i, n


def test_no_cpu_fallback_in_the_product_path():
    """The package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2409_07759_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f


def test_trainer_view_sampling_is_philox_mapped():
    """The trainer's view of iteration i: floor(x0 n / 2^32), x0 the first
    word of Philox4x32-10 at counter (i_lo, i_hi, 0, 'SAMP') keyed by the
    seed -- against the oracle's Philox (pinned by the published
    known-answer vectors); uniform over the views."""
    import oracle as O
    from paper_2409_07759_amd import swgs
    for seed in (0, 11, 0x1234_5678_9ABC_DEF0):
        for n in (1, 6, 180):
            for i in list(range(50)) + [2 ** 32 + 3, 2 ** 40 + 17]:
                x = O.philox4x32_10([i & 0xFFFFFFFF, i >> 32, 0, 0x504D4153],
                                    [seed & 0xFFFFFFFF, seed >> 32])
                assert swgs.trainer_view(seed, i, n) == (int(x[0]) * n) >> 32, (seed, n, i)
    counts = np.bincount([swgs.trainer_view(5, i, 8) for i in range(8000)], minlength=8)
    chi2 = float(((counts - 1000) ** 2 / 1000).sum())
    assert chi2 < 24.3      # 7 degrees of freedom, p = 0.001
