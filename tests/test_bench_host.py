"""Host-side pieces of bench.py (no GPU): the workload definitions and the
algorithmic byte counts its roofline divides by."""
from __future__ import annotations

import numpy as np
import pytest

import bench


def test_headline_workload_shape():
    w = bench.workload("chirps")
    assert w["workload"] == "chirps-1024x65536"
    assert len(w["lengths"]) == 1024 and set(w["lengths"]) == {65536}
    assert (w["delta"], w["max_imfs"], w["io"]) == (1e-3, 12, "f32")


def test_variants_are_library_and_oracle_options():
    for name, (lib, ora) in bench.VARIANTS.items():
        assert lib and ora, name
    assert bench.VARIANTS["abs"] == ({"stop_mode": 1}, {"stop": "abs"})


@pytest.mark.parametrize("kind,factor", [("scan", 1.0), ("pass1_step", 2.0)])
def test_algorithmic_bytes_count_active_spectra(kind, factor):
    # three four-step signals of 65536 samples with 3, 1 and 2 IMFs over 3 steps:
    # the step kernels touch 3 + 1 + 2 = 6 half spectra of 32769 complex doubles
    lengths = [65536, 65536, 65536]
    n_imfs = np.array([3, 1, 2])
    got = bench.algorithmic_bytes(kind, lengths, n_imfs, 3, 4)
    assert got == pytest.approx(factor * 6 * 32769 * 16)


def test_algorithmic_bytes_pass2_writes_every_imf_row():
    got = bench.algorithmic_bytes("pass2_step", [65536, 16384], np.array([2, 5]), 5, 4)
    assert got == pytest.approx(5 * (65536 + 16384) * 4)


def test_algorithmic_bytes_select_the_kernels_signals():
    # a 4096-sample signal takes the one-pass kernel, not the four-step ones
    assert bench.algorithmic_bytes("pass1_step", [4096], np.array([2]), 2, 4) == 0.0
    assert bench.algorithmic_bytes("single_step", [4096], np.array([2]), 2, 4) == pytest.approx(
        2 * 2 * 2049 * 16 + 2 * 4096 * 4)
