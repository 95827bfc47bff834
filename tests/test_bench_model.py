"""The benchmark's algorithmic byte model against the closed forms it is
built from (CPU only): the five convolution passes move about 27 s bytes per
physical mesh point (1.83 GB at 256^3 FP32), and the particle kernels move
the per-particle bytes of their records."""

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_convolution_bytes_per_point():
    n = (256, 256, 256)
    pts = 256 ** 3
    for s in (4, 8):
        b = bench.conv_bytes(n, s)
        assert 26.5 * s * pts < b < 28.5 * s * pts
    assert bench.conv_bytes(n, 4) == pytest.approx(1.829e9, rel=1e-3)


def test_particle_kernel_bytes():
    n, npart, s = (256, 256, 256), 100_000_000, 4
    m = lambda k: bench.algorithmic_bytes(n, npart, s, k)
    assert m("bbox") == m("bin_count") == 3 * s * npart
    assert m("bin_scatter") == (6 * s + 4) * npart             # positions in, records and permutation out
    assert m("unsort") == (6 * s + 4) * npart
    assert m("deposit") == 3 * s * npart + s * 256 ** 3
    assert m("geometry") == s * 256 ** 3                        # the zero fill
    assert set(bench.KERNEL_SYMBOL) <= set(["bbox", "geometry", "bin_count", "bin_scan", "bin_scatter", "deposit",
                                            "fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv",
                                            "gradient", "gather", "unsort"])


def test_method_bytes_of_the_step():
    """The method's bytes per step: the path's byte model (mesh fit, deposit
    with one binning read and write, five convolution passes, gather), with
    no share for this design's permutation, count pass or unsort re-reads."""
    n, npart, s = (256, 256, 256), 100_000_000, 4
    mb = lambda k: bench.method_bytes(n, npart, s, k)
    part = 3 * s * npart
    assert mb("bin_count") == 0
    assert mb("bin_scatter") == 2 * part
    assert mb("gather") + mb("unsort") == 2 * part + s * 258 ** 3
    names = ("bbox", "geometry", "bin_count", "bin_scan", "bin_scatter", "deposit", "fft_x_fwd", "fft_y_fwd",
             "fft_z_conv", "fft_y_inv", "fft_x_inv", "gather", "unsort")
    total = sum(mb(k) for k in names)
    model = part + s * 256 ** 3 + (part + s * 256 ** 3 + 2 * part) + bench.conv_bytes(n, s) + \
        (2 * part + s * 258 ** 3)
    assert total == model
    assert all(mb(k) <= bench.algorithmic_bytes(n, npart, s, k) for k in names)


def test_tile_order_step_bytes():
    """The tile-ordered step: the scatter writes the binned positions into the
    caller's arrays and no permutation, the gather reads them and writes the
    field (no unsort follows)."""
    n, npart, s = (256, 256, 256), 100_000_000, 4
    mesh_ext = s * 258 ** 3
    assert bench.algorithmic_bytes(n, npart, s, "bin_scatter", True) == 6 * s * npart
    assert bench.algorithmic_bytes(n, npart, s, "bin_scatter") == 6 * s * npart + 4 * npart
    assert bench.algorithmic_bytes(n, npart, s, "gather", True) == 6 * s * npart + mesh_ext
    assert bench.method_bytes(n, npart, s, "gather", True) == 6 * s * npart + mesh_ext
    assert bench.method_bytes(n, npart, s, "gather", True) == (
        bench.method_bytes(n, npart, s, "gather") + bench.method_bytes(n, npart, s, "unsort"))
