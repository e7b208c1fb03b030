"""The enumeration's tuning file (dsd_tune_load), host side only: a flat
JSON object of "arch/hH/cC": cap pairs loads; anything else is refused with
DSD_EINVAL and leaves the caps as they were; NULL restores the built-in
caps.  (The file only sets launch grids; results never depend on them, which
tests/test_gpu_tune.py checks on the GPU.)"""
from __future__ import annotations

import pytest

from paper_1906_00341_amd import dsd


def test_good_and_empty_files(tmp_path):
    p = tmp_path / "t.json"
    p.write_text('{\n  "gfx950/h4/c0": 2048,\n  "gfx950/h4/c2": 1024\n}\n')
    dsd.tune_load(str(p))
    p.write_text("{}")
    dsd.tune_load(str(p))
    dsd.tune_load(None)


@pytest.mark.parametrize("text", ['{"gfx950/h4/c0": -1}', '{"gfx950/h4/c0": 0}', '{"a": 1,}', '["a", 1]',
                                  '{"gfx950/h4/c0": 99999999999}', '{"a" 1}', '', '{"a": 1.5}'])
def test_malformed_files(tmp_path, text):
    p = tmp_path / "bad.json"
    p.write_text(text)
    with pytest.raises(dsd.DsdError) as e:
        dsd.tune_load(str(p))
    assert e.value.status == -1
    dsd.tune_load(None)


def test_missing_file(tmp_path):
    with pytest.raises(dsd.DsdError) as e:
        dsd.tune_load(str(tmp_path / "none.json"))
    assert e.value.status == -1
