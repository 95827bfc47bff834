"""Oracle of the raw 3-D FFT entry points -- test infrastructure only.

Only tests/, the smoke check and the benchmark's CPU leg import this module;
the library never does.

The operation is the discrete Fourier transform of the FFT usage example of
the paper's DKS section (the transform its Poisson solver applies to the
doubled grid, section "FFT Based Particle-Mesh Solver"): for an array
x[batch][nz][ny][nx],

    X[kz, ky, kx] = sum_{z, y, x} x[z, y, x] exp(s 2 pi i (kx x / nx + ky y / ny + kz z / nz)),

s = -1 forward, +1 inverse, with no normalisation.  The sum is separable, so
the definition is written out as one DFT matrix per axis (entries
exp(s 2 pi i ((j k) mod n) / n), built in FP64 from the exact integer phase)
applied by a matrix product along that axis.  Everything is complex128.

Real-to-complex: the forward transform of a real array keeps kx in
[0, nx/2].  Complex-to-real (a reading where a half spectrum is not the
transform of a real array): inverse transforms along z and y of the half
spectrum, then each x row is completed to X[nx - k] = conj X[k] and inverse
transformed, keeping the real part.
"""

import numpy as np


def dft_matrix(n, inverse=False):
    """M[k, j] = exp(s 2 pi i ((j k) mod n) / n)."""
    j = np.arange(n)
    phase = np.outer(j, j) % n
    s = 1.0 if inverse else -1.0
    return np.exp(s * 2j * np.pi * phase / n)


def dft_axis(x, axis, inverse=False):
    """The 1-D DFT of every line of x along `axis`."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[axis]
    M = dft_matrix(n, inverse)
    return np.moveaxis(np.tensordot(M, np.moveaxis(x, axis, 0), axes=(1, 0)), 0, axis)


def dft3(x, inverse=False):
    """DFT over the last three axes (z, y, x) of x [..., nz, ny, nx]."""
    out = np.asarray(x, dtype=np.complex128)
    for axis in (-1, -2, -3):
        out = dft_axis(out, axis, inverse)
    return out


def rdft3(x):
    """Forward real-to-complex: the kx <= nx/2 half of dft3 of a real array."""
    x = np.asarray(x, dtype=np.float64)
    nx = x.shape[-1]
    return dft3(x)[..., : nx // 2 + 1]


def irdft3(X, nx):
    """Complex-to-real inverse of a half spectrum [..., nz, ny, nx//2 + 1]."""
    Y = dft_axis(dft_axis(X, -3, inverse=True), -2, inverse=True)
    full = np.zeros(Y.shape[:-1] + (nx,), dtype=np.complex128)
    h = nx // 2 + 1
    full[..., :h] = Y
    for k in range(1, h):
        if nx - k > k:
            full[..., nx - k] = np.conj(Y[..., k])
    return dft_axis(full, -1, inverse=True).real


def dft3_at(x, k, inverse=False):
    """One output X[kz, ky, kx] of dft3 of a single array x [nz, ny, nx], by
    the sum over all inputs (used to sample outputs of large transforms)."""
    x = np.asarray(x, dtype=np.complex128)
    nz, ny, nx = x.shape
    kz, ky, kx = k
    s = 1.0 if inverse else -1.0
    wx = np.exp(s * 2j * np.pi * ((np.arange(nx) * kx) % nx) / nx)
    wy = np.exp(s * 2j * np.pi * ((np.arange(ny) * ky) % ny) / ny)
    wz = np.exp(s * 2j * np.pi * ((np.arange(nz) * kz) % nz) / nz)
    return complex(((x @ wx) @ wy) @ wz)
