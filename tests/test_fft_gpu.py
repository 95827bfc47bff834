"""Parity of the raw 3-D FFT entry points with the FP64 DFT oracle, through
the C ABI.

Tolerance (relative L2 over the whole output): 1e-12 for FP64 and 1e-5 for
FP32.  The rounding error of a radix-2/3/4/8 FFT grows like the unit
roundoff times the number of passes (at most 27 radix-2 levels here):
about 2e-6 in FP32 and 4e-15 in FP64 at the largest size.  The 512 x 512 x
256 transform is checked on sampled outputs (each by the full sum over the
inputs) and by inversion."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fft_oracle as fo  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}
CDT = {"f32": torch.complex64, "f64": torch.complex128}
RDT = {"f32": torch.float32, "f64": torch.float64}


def dks():
    from paper_1509_07685_amd import dks as mod
    return mod


def rel_l2(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def crand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


C2C_CASES = [
    ((1, 1, 1), 1),
    ((8, 1, 1), 3),
    ((4096, 1, 1), 2),        # longest row; FP64 tile without padding
    ((1, 64, 1), 2),          # y only
    ((1, 1, 81), 1),          # z only, radix 3
    ((12, 18, 1), 2),
    ((27, 16, 24), 2),        # radix-3 rows, ragged column tiles
    ((72, 48, 36), 1),        # several column tiles with a ragged tail
    ((512, 8, 6), 1),         # compile-time 512 row plan
    ((128, 256, 64), 1),      # compile-time row, y and z plans
    ((6, 4096, 2), 1),        # longest column pencils (narrow tiles)
]


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n,batch", C2C_CASES)
def test_c2c_forward_inverse(n, batch, dt):
    nx, ny, nz = n
    x = crand((batch, nz, ny, nx), 11 + nx + ny + nz)
    plan = dks().FFTPlan(n, batch, "c2c", dt)
    xd = torch.from_numpy(x).to(CDT[dt]).cuda()
    X = plan.forward(xd)
    xi = plan.inverse(xd)
    torch.cuda.synchronize()
    xq = xd.cpu().numpy().astype(np.complex128)   # the values the device saw
    assert rel_l2(X.cpu().numpy(), fo.dft3(xq)) <= TOL[dt]
    assert rel_l2(xi.cpu().numpy(), fo.dft3(xq, inverse=True)) <= TOL[dt]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_c2c_in_place_equals_out_of_place(dt):
    n, batch = (48, 36, 32), 2
    x = crand((batch, n[2], n[1], n[0]), 12)
    plan = dks().FFTPlan(n, batch, "c2c", dt)
    xd = torch.from_numpy(x).to(CDT[dt]).cuda()
    ref = plan.forward(xd)
    buf = xd.clone()
    plan.forward(buf, out=buf)
    back = buf.clone()
    plan.inverse(back, out=back)
    torch.cuda.synchronize()
    assert torch.equal(buf, ref)
    N = n[0] * n[1] * n[2]
    assert rel_l2(back.cpu().numpy() / N, xd.cpu().numpy()) <= TOL[dt]


R2C_CASES = [((8, 1, 1), 1), ((1, 4, 4), 2), ((9, 4, 6), 2), ((64, 32, 48), 2), ((512, 4, 4), 1),
             ((36, 27, 1), 3), ((256, 64, 128), 1)]


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n,batch", R2C_CASES)
def test_r2c_and_c2r(n, batch, dt):
    nx, ny, nz = n
    x = np.random.default_rng(13 + nx).standard_normal((batch, nz, ny, nx))
    plan = dks().FFTPlan(n, batch, "r2c", dt)
    xd = torch.from_numpy(x).to(RDT[dt]).cuda()
    H = plan.forward(xd)
    xq = xd.cpu().numpy().astype(np.float64)
    Href = fo.rdft3(xq)
    Hin = H.clone()
    y = plan.inverse(H)
    torch.cuda.synchronize()
    assert rel_l2(H.cpu().numpy(), Href) <= TOL[dt]
    assert torch.equal(H, Hin)                  # the inverse leaves its input alone
    Hq = H.cpu().numpy().astype(np.complex128)
    assert rel_l2(y.cpu().numpy(), fo.irdft3(Hq, nx)) <= TOL[dt]
    assert rel_l2(y.cpu().numpy() / (nx * ny * nz), xq) <= TOL[dt]


def test_c2r_of_a_general_half_spectrum_follows_the_stated_order():
    """A half spectrum that is not the transform of a real array: z and y
    inverse transforms first, then each x row completed and inverted."""
    n, batch, dt = (12, 6, 8), 1, "f64"
    H = crand((batch, n[2], n[1], n[0] // 2 + 1), 14)
    plan = dks().FFTPlan(n, batch, "r2c", dt)
    y = plan.inverse(torch.from_numpy(H).cuda())
    torch.cuda.synchronize()
    assert rel_l2(y.cpu().numpy(), fo.irdft3(H, n[0])) <= TOL[dt]


def test_full_size_512x512x256_f32_sampled_and_inverted():
    """The paper's largest FFT size, FP32, in place: sampled outputs against
    the full sum, and inverse(forward(x)) = N x."""
    n = (512, 512, 256)
    g = np.random.default_rng(15)
    x = (g.standard_normal((n[2], n[1], n[0])) + 1j * g.standard_normal((n[2], n[1], n[0]))).astype(np.complex64)
    plan = dks().FFTPlan(n, 1, "c2c", "f32")
    buf = torch.from_numpy(x).cuda().unsqueeze(0).contiguous()
    plan.forward(buf, out=buf)
    torch.cuda.synchronize()
    X = buf.cpu().numpy()[0]
    xq = x.astype(np.complex128)
    ks = [(0, 0, 0), (255, 511, 511), (128, 256, 256), (1, 2, 3)]
    ks += [tuple(int(v) for v in (g.integers(256), g.integers(512), g.integers(512))) for _ in range(4)]
    scale = np.sqrt(np.mean(np.abs(X) ** 2))
    for k in ks:
        ref = fo.dft3_at(xq, k)
        assert abs(X[k] - ref) <= TOL["f32"] * scale, k
    plan.inverse(buf, out=buf)
    torch.cuda.synchronize()
    N = n[0] * n[1] * n[2]
    assert rel_l2(buf.cpu().numpy()[0] / N, x) <= TOL["f32"]
