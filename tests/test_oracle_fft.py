"""Pins of the FFT oracle (oracle/fft_oracle.py) against what the definition
of the discrete Fourier transform and its theorems fix: the literal sum on
tiny arrays, numpy's FFT (an independent library routine), transforms of
deltas and constants, the shift theorem, Parseval's identity, inversion,
Hermitian symmetry of real inputs, and the sampled single-output sum."""

import cmath
import itertools

import numpy as np
import pytest

from oracle import fft_oracle as fo


def literal_dft3(x, inverse=False):
    """The triple sum with one complex exponential per term (pure Python)."""
    nz, ny, nx = x.shape
    s = 1.0 if inverse else -1.0
    out = np.zeros(x.shape, dtype=np.complex128)
    for kz, ky, kx in itertools.product(range(nz), range(ny), range(nx)):
        acc = 0j
        for z, y, xx in itertools.product(range(nz), range(ny), range(nx)):
            acc += x[z, y, xx] * cmath.exp(s * 2j * cmath.pi * (kx * xx / nx + ky * y / ny + kz * z / nz))
        out[kz, ky, kx] = acc
    return out


def rnd(shape, seed, complex_=True):
    g = np.random.default_rng(seed)
    a = g.standard_normal(shape)
    return a + 1j * g.standard_normal(shape) if complex_ else a


@pytest.mark.parametrize("shape", [(3, 2, 4), (1, 6, 1), (2, 3, 3), (4, 1, 9)])
@pytest.mark.parametrize("inverse", [False, True])
def test_matches_literal_sum(shape, inverse):
    x = rnd(shape, sum(shape))
    np.testing.assert_allclose(fo.dft3(x, inverse), literal_dft3(x, inverse), rtol=0, atol=1e-12)


@pytest.mark.parametrize("shape", [(8, 12, 6), (27, 4, 16), (1, 1, 64), (5, 9, 2)])
def test_matches_numpy_fft(shape):
    x = rnd((2,) + shape, 3)
    np.testing.assert_allclose(fo.dft3(x), np.fft.fftn(x, axes=(-3, -2, -1)), rtol=0, atol=1e-11)
    N = np.prod(shape)
    np.testing.assert_allclose(fo.dft3(x, inverse=True), N * np.fft.ifftn(x, axes=(-3, -2, -1)), rtol=0, atol=1e-11)


def test_delta_and_constant():
    shape = (4, 6, 9)
    d = np.zeros(shape)
    d[0, 0, 0] = 1.0
    np.testing.assert_allclose(fo.dft3(d), np.ones(shape), atol=1e-14)
    c = np.ones(shape)
    X = fo.dft3(c)
    ref = np.zeros(shape, dtype=complex)
    ref[0, 0, 0] = np.prod(shape)
    np.testing.assert_allclose(X, ref, atol=1e-12)


def test_shift_theorem_fixes_sign_and_axes():
    shape = (6, 4, 8)
    x = rnd(shape, 5)
    X = fo.dft3(x)
    sz, sy, sx = 1, 3, 2
    Xs = fo.dft3(np.roll(x, (sz, sy, sx), axis=(0, 1, 2)))
    kz, ky, kx = np.meshgrid(np.arange(6), np.arange(4), np.arange(8), indexing="ij")
    phase = np.exp(-2j * np.pi * (kx * sx / 8 + ky * sy / 4 + kz * sz / 6))
    np.testing.assert_allclose(Xs, X * phase, atol=1e-12)


def test_parseval_and_inversion():
    shape = (9, 8, 12)
    x = rnd(shape, 6)
    X = fo.dft3(x)
    N = np.prod(shape)
    assert abs(np.sum(abs(X) ** 2) - N * np.sum(abs(x) ** 2)) <= 1e-10 * N * np.sum(abs(x) ** 2)
    np.testing.assert_allclose(fo.dft3(X, inverse=True), N * x, atol=1e-10)


@pytest.mark.parametrize("shape", [(4, 6, 8), (3, 3, 9), (2, 1, 1), (1, 4, 2)])
def test_real_to_complex_and_back(shape):
    x = rnd(shape, 7, complex_=False)
    nx = shape[-1]
    H = fo.rdft3(x)
    full = fo.dft3(x)
    np.testing.assert_allclose(H, full[..., : nx // 2 + 1], atol=1e-12)
    # Hermitian symmetry of a real input's spectrum
    idx = tuple(np.negative(np.indices(shape)) % np.array(shape)[:, None, None, None])
    np.testing.assert_allclose(full, np.conj(full[idx]), atol=1e-12)
    np.testing.assert_allclose(fo.irdft3(H, nx), np.prod(shape) * x, atol=1e-11)
    np.testing.assert_allclose(H, np.fft.rfftn(x), atol=1e-11)


def test_sampled_output_equals_full_transform():
    x = rnd((6, 8, 12), 8)
    X = fo.dft3(x)
    for k in [(0, 0, 0), (5, 7, 11), (3, 2, 6), (1, 4, 9)]:
        assert abs(fo.dft3_at(x, k) - X[k]) <= 1e-12
        assert abs(fo.dft3_at(x, k, inverse=True) - fo.dft3(x, inverse=True)[k]) <= 1e-12
