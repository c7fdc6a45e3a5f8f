"""The C-ABI library loads, exports every symbol include/*.h declare, and its
host-only logic (argument checks, mapping constants, level count) is right.
No kernel is launched here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from workloads import Window, random_params, random_windows

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ask():
    from paper_2206_02255_amd import ask
    return ask


def declared_functions():
    names = set()
    for h in ("ask.h", "ask3d.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(ask3?_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported(ask):
    names = declared_functions()
    assert len(names) >= 9 and "ask3_dwell_subdiv" in names
    for n in names:
        assert hasattr(ask.lib, n), n
        assert n in ask.SIGNATURES, n


def test_status_strings(ask):
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert ask.status_str(s)


def test_mapping_equals_oracle_bit_for_bit(ask, ref):
    for w in random_windows(1, 50) + [Window(-1.5, 0.5, -1.0, 1.0, 16384, 16384, 2048)]:
        assert ask.ask_mapping(ask.window(w)) == ref.mapping(w)


def test_validation(ask):
    good = ask.window(Window(-1.5, 0.5, -1.0, 1.0, 64, 48, 100))
    assert ask.ask_validate(good) == 0
    assert ask.ask_validate(good, ask.params(4, 2, 8)) == 0
    for g, r, B in [(0, 2, 8), (49, 2, 8), (4, 1, 8), (4, 1025, 8), (4, 2, 0)]:
        assert ask.ask_validate(good, ask.params(g, r, B)) == ask.EINVAL
    assert ask.ask_validate(good, ask.params(4, 2, 8, form=7)) == ask.EINVAL
    for band in (0, 64, 1000, 1 << 24, ask.BAND_NONE):
        assert ask.ask_validate(good, ask.params(4, 2, 8, "persistent", band)) == 0
    for band in (1, 63, (1 << 24) + 1):
        assert ask.ask_validate(good, ask.params(4, 2, 8, "persistent", band)) == ask.EINVAL
    for w in [Window(0.5, -1.5, -1, 1, 8, 8, 10), Window(-1, 1, -1, 1, 0, 8, 10),
              Window(-1, 1, -1, 1, 8, 8, 0), Window(-1, float("inf"), -1, 1, 8, 8, 10),
              Window(-1, 1, -1, 1, 8, 65537, 10), Window(-1, 1, -1, 1, 8, 8, 2**31)]:
        assert ask.ask_validate(ask.window(w)) == ask.EINVAL
    bad = ask.window(Window(-1, 1, -1, 1, 8, 8, 10))
    bad.set = 2
    assert ask.ask_validate(bad) == ask.EINVAL
    # wave tiles: both 0, or a power-of-two width 4..64 holding exactly 64 pixels
    for tile in ((0, 0), (4, 16), (8, 8), (16, 4), (32, 2), (64, 1)):
        assert ask.ask_validate(good, ask.params(4, 2, 8, "levels", 0, tile)) == 0, tile
    for tile in ((0, 4), (16, 0), (2, 32), (128, 1), (12, 5), (16, 8), (8, 4), (1, 64)):
        assert ask.ask_validate(good, ask.params(4, 2, 8, "levels", 0, tile)) == ask.EINVAL, tile


def test_level_count_bounds_the_oracle_depth(ask, ref):
    # The host fixes the number of level kernels from (W, H, g, r, B) alone;
    # it must never be below the depth the subdivision actually reaches.
    for i, w in enumerate(random_windows(7, 20, max_side=80, max_dwell=150)):
        for p in random_params(200 + i, w, 4):
            n = ask.ask_level_count(ask.window(w), ask.params(p.g, p.r, p.B))
            _, st = ref.subdiv(w, p.g, p.r, p.B)
            assert st["levels"] <= n
    # the paper's window: the boundary crosses every level down to B
    w = Window(-1.5, 0.5, -1.0, 1.0, 1024, 1024, 512)
    n = ask.ask_level_count(ask.window(w), ask.params(4, 2, 32))
    _, st = ref.subdiv(w, 4, 2, 32)
    assert n == st["levels"] == 4


def test_create_without_device_reports_device_error(ask):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(ask.AskError) as e:
        ask.ask_create(0)
    assert e.value.status == ask.EDEVICE


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding have the header's sizes and field
    offsets (compiled with the host C compiler from include/ask.h)."""
    import ctypes
    import subprocess

    from paper_2206_02255_amd import ask
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    fields = {"ask_window": [f for f, _ in ask.ask_window._fields_],
              "ask_params": [f for f, _ in ask.ask_params._fields_],
              "ask_stats": [f for f, _ in ask.ask_stats._fields_],
              "ask_server_cfg": [f for f, _ in ask.ask_server_cfg._fields_],
              "ask_volume": [f for f, _ in ask.ask_volume._fields_],
              "ask3_params": [f for f, _ in ask.ask3_params._fields_],
              "ask3_stats": [f for f, _ in ask.ask3_stats._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ask.h"', '#include "ask3d.h"',
             'int main(void) {']
    for s, fs in fields.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (s, s))
        for f in fs:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (s, f, s, f))
    lines.append('return 0; }')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for s, fs in fields.items():
        cls = getattr(ask, s)
        assert int(got[s]) == ctypes.sizeof(cls), s
        for f in fs:
            assert int(got["%s.%s" % (s, f)]) == getattr(cls, f).offset, (s, f)


def test_volume_validation(ask):
    from workloads import Volume
    good = ask.volume(Volume(-1, 1, -1, 1, -1, 1, 40, 30, 20, 100))
    assert ask.ask3_validate(good) == 0
    assert ask.ask3_validate(good, ask.params3(4, 2, 4)) == 0
    assert ask.ask3_validate(good, ask.params3(4, 2, 4, "morton")) == 0
    for g, r, B, c in [(0, 2, 4, 0), (1025, 2, 4, 0), (4, 1, 4, 0), (4, 17, 4, 0), (4, 2, 0, 0),
                       (4, 2, 4, 2)]:
        assert ask.ask3_validate(good, ask.params3(g, r, B, c)) == ask.EINVAL, (g, r, B, c)
    for v in [Volume(1, -1, -1, 1, -1, 1, 8, 8, 8, 10), Volume(-1, 1, -1, 1, -1, 1, 8, 0, 8, 10),
              Volume(-1, 1, -1, 1, -1, 1, 8, 8, 8, 0), Volume(-1, 1, -1, 1, -1, 1, 8, 8, 65537, 10),
              Volume(-1, 1, -1, 1, -1, 1, 4096, 4096, 256, 10),
              Volume(-1, 1, -1, 1, -1, 1, 8, 8, 8, 10, c=(float("nan"), 0.0))]:
        assert ask.ask3_validate(ask.volume(v)) == ask.EINVAL, v
    # the deepest and the widest grids valid sizes reach stay within the 32 levels
    # and the 2^21 cells per axis a Morton scalar can name: a level whose sides
    # still exceed B has G < n, so the next grid has G < n r <= 2^20
    for g, r in ((1, 2), (1024, 16), (1000, 16)):
        assert ask.ask3_validate(ask.volume(Volume(-1, 1, -1, 1, -1, 1, 65536, 8, 8, 10)),
                                 ask.params3(g, r, 1, "morton")) == 0


def test_volume_workspace_bytes(ask):
    from workloads import Volume
    v = Volume(-1, 1, -1, 1, -1, 1, 40, 30, 20, 100)
    V = 40 * 30 * 20
    for g, r, B in [(4, 2, 4), (8, 3, 1), (1, 2, 100), (64, 2, 2)]:
        cap = min(V, max(min(g, 40) * min(g, 30) * min(g, 20), r ** 3 * (V // (B + 1))))
        cap = (cap + 31) // 32 * 32
        # a 36 KiB control block (counters, and per level eight claim
        # counters on 128-byte lines) and two tables of 8-byte entries
        assert ask.ask3_workspace_bytes(ask.volume(v), ask.params3(g, r, B)) == 36864 + 16 * cap
