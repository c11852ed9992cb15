"""The autotuner's cache file, through the C ABI on the host (no GPU).

fif_tune_cache_store / fif_tune_cache_lookup: round trip, several device
keys and lengths, replacement, and corruption -- lines that do not parse or
whose choice is not a valid plan of their length are ignored, a store keeps
only valid lines, invalid choices are refused.
"""
from __future__ import annotations

import os

import pytest

import paper_1802_01359_amd as fif
from paper_1802_01359_amd import _binding

pytestmark = pytest.mark.skipif(not os.path.exists(_binding.LIB_PATH), reason="libfif.so not built")

C65536 = {"N": 65536, "N1": 256, "N2": 256, "TC": 16, "TR": 8, "rad1": [4, 8, 8], "rad2": [8, 8, 4],
          "us": 812.5, "us_default": 850.25}
C20736 = {"N": 20736, "N1": 144, "N2": 144, "TC": 4, "TR": 2, "rad1": [8, 2, 3, 3],
          "rad2": [3, 3, 8, 2], "us": 100.0, "us_default": 120.0}


def test_round_trip(tmp_path):
    path = str(tmp_path / "tune.txt")
    assert fif.tune_cache_lookup(path, "gfx950/hip1", 65536) is None        # no file yet
    fif.tune_cache_store(path, "gfx950/hip1", C65536)
    got = fif.tune_cache_lookup(path, "gfx950/hip1", 65536)
    assert got == C65536
    assert fif.tune_cache_lookup(path, "gfx950/hip2", 65536) is None        # other runtime version
    assert fif.tune_cache_lookup(path, "gfx950/hip1", 131072) is None       # other length


def test_several_entries_and_replacement(tmp_path):
    path = str(tmp_path / "tune.txt")
    fif.tune_cache_store(path, "gfx950/hip1", C65536)
    fif.tune_cache_store(path, "gfx950/hip1", C20736)
    fif.tune_cache_store(path, "gfx942/hip1", dict(C65536, TC=8))
    newer = dict(C65536, TR=16, rad1=[8, 8, 4], us=700.0)
    fif.tune_cache_store(path, "gfx950/hip1", newer)
    assert fif.tune_cache_lookup(path, "gfx950/hip1", 65536) == newer
    assert fif.tune_cache_lookup(path, "gfx950/hip1", 20736) == C20736
    assert fif.tune_cache_lookup(path, "gfx942/hip1", 65536)["TC"] == 8
    lines = open(path).read().splitlines()
    assert len(lines) == 3 and all(l.startswith("FIFTUNE1 ") for l in lines)


@pytest.mark.parametrize("bad", [
    "garbage",
    "FIFTUNE1 gfx950/hip1 65536 256 256 16",                                # truncated
    "FIFTUNE1 gfx950/hip1 65536 128 256 16 8 4.8.8 8.8.4 1.0 2.0",          # N1 N2 != N
    "FIFTUNE1 gfx950/hip1 65536 256 256 16 8 4.8.8 6.8.4 1.0 2.0",          # no radix 6
    "FIFTUNE1 gfx950/hip1 65536 256 256 12 8 4.8.8 8.8.4 1.0 2.0",          # TC does not divide N1
    "FIFTUNE1 gfx950/hip1 65536 256 256 64 8 4.8.8 8.8.4 1.0 2.0",          # pass-1 tile > 8192 elements
    "FIFTUNE1 gfx950/hip1 65536 256 256 16 8 4.8.8 8.8.4 1.0 2.0 extra",    # trailing field
    "FIFTUNE2 gfx950/hip1 65536 256 256 16 8 4.8.8 8.8.4 1.0 2.0",          # other format
    "FIFTUNE1 gfx950/hip1 65536 256 256 16 8 4.8.8 8.8.x 1.0 2.0",          # radix text
])
def test_corrupt_lines_are_ignored(tmp_path, bad):
    path = str(tmp_path / "tune.txt")
    fif.tune_cache_store(path, "gfx950/hip1", C65536)
    good = open(path).read()
    with open(path, "w") as f:
        f.write(bad + "\n" + good + bad[: len(bad) // 2] + "\n")
    assert fif.tune_cache_lookup(path, "gfx950/hip1", 65536) == C65536
    # a corrupt line naming the entry's own length does not shadow it
    with open(path, "w") as f:
        f.write(good + bad + "\n")
    assert fif.tune_cache_lookup(path, "gfx950/hip1", 65536) == C65536
    # the next store drops the corrupt lines
    fif.tune_cache_store(path, "gfx950/hip1", C20736)
    lines = open(path).read().splitlines()
    assert bad not in lines and len(lines) == 2


def test_only_corrupt_entries_means_not_found(tmp_path):
    path = str(tmp_path / "tune.txt")
    with open(path, "w") as f:
        f.write("FIFTUNE1 gfx950/hip1 65536 128 256 16 8 4.8.8 8.8.4 1.0 2.0\n\x00\xff\n")
    assert fif.tune_cache_lookup(path, "gfx950/hip1", 65536) is None


@pytest.mark.parametrize("field,value", [("N1", 128), ("TC", 12), ("rad1", [4, 4, 4]), ("rad2", [6, 8, 4])])
def test_store_refuses_invalid_choices(tmp_path, field, value):
    path = str(tmp_path / "tune.txt")
    with pytest.raises(fif.FifError) as e:
        fif.tune_cache_store(path, "gfx950/hip1", dict(C65536, **{field: value}))
    assert e.value.status == _binding.FIF_ERR_INVALID_ARG
    assert not os.path.exists(path)


def test_single_pass_choice(tmp_path):
    path = str(tmp_path / "tune.txt")
    c = {"N": 6000, "N1": 1, "N2": 6000, "TC": 1, "TR": 1, "rad1": [8, 2, 3, 5, 5, 5], "rad2": [],
         "us": 0.0, "us_default": 0.0}
    fif.tune_cache_store(path, "k", c)
    assert fif.tune_cache_lookup(path, "k", 6000) == c
