"""The autotuner cache shipped with the package (tune_gfx950.json): the layout
the library's reader expects (a JSON object, one entry per line of the form
"arch|dtype|precision|NXxNYxNZ|kind": [vx, ty, kz, wpb, ms]) and, per entry, a
tile shape the kernels accept for that grid and kind: vx in {1, 2, 4} with
vx times the element size at most 16 bytes and dividing nx; ty in {1, 2, 4,
8} (at most 2 for the batched kernels, 1 for the Smagorinsky kernel); kz >= 1;
1 <= wpb <= 4; a positive time.  The benchmark's hill has entries for its
dense pass and for its Smagorinsky kernel."""
import json
import os
import re

import pytest

CACHE = os.path.join(os.path.dirname(__file__), "..", "paper_2006_03343_amd", "tune_gfx950.json")
LINE = re.compile(r'^"(gfx\d+)\|(f32|f64)\|(plain|mixed)\|(\d+)x(\d+)x(\d+)\|(plain|batch|sgs)": '
                  r'\[(\d+), (\d+), (\d+), (\d+), ([0-9.]+)\],?$')


def _entries():
    lines = open(CACHE).read().splitlines()
    assert lines[0] == "{" and lines[-1] == "}"
    out = []
    for ln in lines[1:-1]:
        m = LINE.match(ln)
        assert m, f"unreadable cache line: {ln!r}"
        out.append(m.groups())
    return out


def test_layout_and_json_agree():
    entries = _entries()
    as_json = json.load(open(CACHE))
    assert len(entries) == len(as_json) > 0
    for e in entries:
        key = "|".join(e[:3]) + f"|{e[3]}x{e[4]}x{e[5]}|{e[6]}"
        assert as_json[key] == [int(e[7]), int(e[8]), int(e[9]), int(e[10]), float(e[11])]


@pytest.mark.parametrize("entry", _entries(), ids=lambda e: "|".join(e[:7]))
def test_tile_is_valid(entry):
    arch, dtype, prec, nx, ny, nz, kind, vx, ty, kz, wpb, ms = entry
    nx, vx, ty, kz, wpb, ms = int(nx), int(vx), int(ty), int(kz), int(wpb), float(ms)
    size = 8 if dtype == "f64" else 4
    assert arch == "gfx950"
    assert not (dtype == "f64" and prec == "mixed")
    assert vx in (1, 2, 4) and vx * size <= 16 and nx % vx == 0
    assert ty in (1, 2, 4, 8)
    if kind == "batch":
        assert ty <= 2
    if kind == "sgs":
        assert ty == 1
    assert kz >= 1 and 1 <= wpb <= 4 and ms > 0.0


def test_benchmark_hill_is_covered():
    keys = {"|".join(e[:3]) + f"|{e[3]}x{e[4]}x{e[5]}|{e[6]}" for e in _entries()}
    assert "gfx950|f32|mixed|512x256x256|plain" in keys
    assert "gfx950|f32|mixed|512x256x256|sgs" in keys
    assert "gfx950|f64|plain|512x256x256|plain" in keys
