"""Pins of the FP64 CPU oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: a closed form, an independent
numerical quadrature, a multipole expansion derived from the mean-value
property of 1/r, the literal O(M^2) sum of the paper's brute-force
convolution equation, conservation laws and exactness properties of CIC and
central differences, and analytic potentials of charge distributions.
"""

import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import poisson_oracle as orc
from paper_1509_07685_amd import workloads as wl

K = 1.0 / (4.0 * math.pi * 8.8541878128e-12)


# --------------------------------------------------------------------------
# Integrated Green's function
# --------------------------------------------------------------------------

def cube_self_integral():
    """Integral of 1/r over the unit cube centred at 0 (classical closed form).

    The integral over [0,1]^3 is (3/2) ln((sqrt3+1)/(sqrt3-1)) - pi/4; by
    symmetry and the degree-2 homogeneity of the integral, the centred unit
    cube gives 8 * (1/2)^2 times that.
    """
    s3 = math.sqrt(3.0)
    i1 = 1.5 * math.log((s3 + 1.0) / (s3 - 1.0)) - math.pi / 4.0
    return 2.0 * i1


@pytest.mark.parametrize("h", [1.0, 1e-4, 3.7])
def test_igf_centre_cell_closed_form(h):
    g = orc.igf_octant((2, 2, 2), (h, h, h))
    assert g[0, 0, 0] / (h * h) == pytest.approx(cube_self_integral(), rel=1e-14)
    assert cube_self_integral() == pytest.approx(2.3800773639795535, rel=1e-15)


def _quad_cell(a, b, c, h):
    hx, hy, hz = h
    f = lambda z, y, x: 1.0 / math.sqrt(x * x + y * y + z * z)
    val, err = integrate.tplquad(
        f, (a - 0.5) * hx, (a + 0.5) * hx,
        (b - 0.5) * hy, (b + 0.5) * hy,
        (c - 0.5) * hz, (c + 0.5) * hz, epsabs=0.0, epsrel=1e-13)
    return val


@pytest.mark.parametrize("offset,h", [
    ((1, 0, 0), (1.0, 1.0, 1.0)),
    ((0, 1, 0), (1.0, 1.0, 1.0)),
    ((2, 1, 0), (1.0, 1.0, 1.0)),
    ((3, 2, 1), (1.0, 1.0, 1.0)),
    ((1, 0, 0), (5e-5, 5e-5, 2e-4)),
    ((0, 0, 1), (5e-5, 5e-5, 2e-4)),
    ((4, 7, 2), (5e-5, 5e-5, 2e-4)),
    ((2, 0, 3), (1.0, 2.0, 0.5)),
])
def test_igf_matches_numerical_quadrature(offset, h):
    a, b, c = offset
    n = (a + 1, b + 1, c + 1)
    g = orc.igf_octant(n, h)[c, b, a]
    assert g == pytest.approx(_quad_cell(a, b, c, h), rel=1e-10)
    assert orc.igf_at(a, b, c, h) == pytest.approx(g, rel=1e-15)


def test_igf_anisotropic_centre_cell_quadrature():
    # Octant symmetry: 8 x integral over [0,hx/2]x[0,hy/2]x[0,hz/2] (corner singularity)
    h = (1.0, 2.0, 0.5)
    f = lambda z, y, x: 1.0 / math.sqrt(x * x + y * y + z * z)
    val, _ = integrate.tplquad(f, 0.0, 0.5 * h[0], 0.0, 0.5 * h[1], 0.0, 0.5 * h[2],
                               epsabs=0.0, epsrel=1e-11)
    g = orc.igf_octant((1, 1, 1), h)[0, 0, 0]
    assert g == pytest.approx(8.0 * val, rel=1e-8)


def _mp_closed_form(a, b, c, h):
    """The antiderivative's third difference evaluated with 40 significant digits."""
    import mpmath as mp
    mp.mp.dps = 40

    def F(x, y, z):
        r = mp.sqrt(x * x + y * y + z * z)
        return (y * z * mp.log(x + r) + x * z * mp.log(y + r) + x * y * mp.log(z + r)
                - x * x / 2 * mp.atan(y * z / (x * r)) - y * y / 2 * mp.atan(x * z / (y * r))
                - z * z / 2 * mp.atan(x * y / (z * r)))
    hm = [mp.mpf(v) for v in h]
    t = mp.mpf(0)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                t += (-1) ** (3 - dx - dy - dz) * F((a - mp.mpf(0.5) + dx) * hm[0],
                                                      (b - mp.mpf(0.5) + dy) * hm[1],
                                                      (c - mp.mpf(0.5) + dz) * hm[2])
    return t


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (5e-5, 5e-5, 2e-4), (1.3e-4, 0.7e-4, 2.1e-4), (2.0, 0.5, 0.5)])
def test_igf_reaches_fp64_accuracy_at_all_offsets(h):
    """The closed form evaluated in 40-digit arithmetic is the exact integral
    (it agrees with independent quadrature above); the oracle's FP64 value must
    be that number correctly rounded (within one unit in the last place) from
    the centre cell out to 256 cells and beyond, for cubic and 4:1 cells."""
    offsets = [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 1, 0), (4, 0, 0), (8, 3, 1), (16, 16, 16),
               (32, 5, 9), (64, 64, 64), (128, 0, 0), (128, 128, 256), (256, 256, 256),
               (3, 40, 7), (200, 1, 90), (0, 256, 1), (512, 511, 3), (1000, 0, 0)]
    for off in offsets:
        exact = float(_mp_closed_form(*off, h))
        got = float(orc.igf_at(*off, h))
        assert abs(got - exact) <= 2.3e-16 * abs(exact), off


def test_igf_octant_equals_pointwise_values():
    """The lattice form of the octant and the per-offset form take the same
    corner sums: identical values, anisotropic cells, offsets up to n."""
    n, h = (20, 13, 9), (1.3e-4, 0.7e-4, 2.1e-4)
    g = orc.igf_octant(n, h)
    c, b, a = np.meshgrid(np.arange(n[2] + 1), np.arange(n[1] + 1), np.arange(n[0] + 1), indexing="ij")
    np.testing.assert_array_equal(g, orc.igf_at(a, b, c, h))


@pytest.mark.parametrize("R", [8, 16])
@pytest.mark.parametrize("direction", [(1, 0, 0), (0, 1, 0), (1, 1, 0), (1, 1, 1), (2, 1, 0)])
def test_igf_far_field_multipole(R, direction):
    """Cube average of 1/r: the h^2 term vanishes (1/r is harmonic) and the
    h^4 term is -(h^4/2880) sum_d d^4/dx_d^4 (1/r), which gives
    G/(V/R) - 1 = -(h^4/960) (35 sum x_d^4/R^4 - 21)/R^4 + O((h/R)^6)."""
    h = 1.0
    d = np.array(direction, dtype=float)
    d = d / np.linalg.norm(d)
    off = np.rint(d * R).astype(int)
    Rv = float(np.linalg.norm(off))
    g = orc.igf_at(*off, (h, h, h))
    measured = g / (h ** 3 / Rv) - 1.0
    s4 = float(np.sum(off.astype(float) ** 4)) / Rv ** 4
    predicted = -(h ** 4 / 960.0) * (35.0 * s4 - 21.0) / Rv ** 4
    assert abs(measured - predicted) < 3.0 * (h / Rv) ** 6


def test_igf_symmetry_and_homogeneity():
    n = (6, 5, 7)
    h = (1.3e-4, 0.7e-4, 2.1e-4)
    g = orc.igf_octant(n, h)
    lam = 3.0
    g2 = orc.igf_octant(n, tuple(lam * x for x in h))
    np.testing.assert_allclose(g2, lam * lam * g, rtol=1e-12)
    # even in each axis: evaluating at negative offsets gives the same value
    a, b, c = np.meshgrid(np.arange(7), np.arange(6), np.arange(8), indexing="ij")
    neg = orc.igf_at(-a, -b, -c, h)
    np.testing.assert_allclose(neg.transpose(2, 1, 0), g, rtol=1e-12)
    # cubic cells: permutation symmetric
    gc = orc.igf_octant((5, 5, 5), (1.0, 1.0, 1.0))
    np.testing.assert_allclose(gc, gc.transpose(1, 0, 2), rtol=1e-13)
    np.testing.assert_allclose(gc, gc.transpose(2, 1, 0), rtol=1e-13)
    # monotone decreasing along an axis
    assert np.all(np.diff(gc[0, 0, :]) < 0)


def test_doubled_kernel_spectrum_is_real():
    n = (8, 6, 12)
    K = orc.doubled_kernel(n, (1.0, 1.5, 0.8))
    spec = np.fft.fftn(K)
    assert np.max(np.abs(spec.imag)) <= 1e-13 * np.max(np.abs(spec.real))


# --------------------------------------------------------------------------
# Convolution: FFT form vs the literal sum of the brute-force equation
# --------------------------------------------------------------------------

def _rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("n,h", [
    ((8, 8, 8), (1e-4, 1e-4, 1e-4)),
    ((12, 12, 12), (1e-4, 1e-4, 1e-4)),   # doubled grid 24: radix 3
    ((6, 8, 10), (5e-5, 5e-5, 2e-4)),     # anisotropic cells, non-cubic mesh
    ((9, 4, 3), (1.0, 2.0, 3.0)),         # odd sizes
])
def test_fft_convolution_equals_direct_sum(n, h):
    g = np.random.default_rng(11)
    rho = g.standard_normal((n[2], n[1], n[0]))
    phi_fft = orc.potential_fft(rho, h)
    phi_dir = orc.potential_direct(rho, h)
    # whole extended box [-1, n]^3, ghost layer included
    assert _rel_l2(phi_fft, phi_dir) <= 1e-14
    assert np.max(np.abs(phi_fft - phi_dir)) <= 1e-13 * np.max(np.abs(phi_dir))


def test_potential_at_matches_fft():
    n = (10, 7, 6)
    h = (1e-4, 2e-4, 1.5e-4)
    rho = np.random.default_rng(3).random((n[2], n[1], n[0]))
    phi = orc.potential_fft(rho, h)
    targets = [(0, 0, 0), (-1, 3, 9), (5, 6, 10), (2, -1, 4)]
    vals = orc.potential_at(rho, h, targets)
    for (k, j, i), v in zip(targets, vals):
        assert v == pytest.approx(phi[k + 1, j + 1, i + 1], rel=1e-13)


def test_point_charge_matches_multipole_far_field():
    n = (33, 33, 33)
    h = 2e-4
    rho = np.zeros((33, 33, 33))
    q = 1e-12
    rho[16, 16, 16] = q / h ** 3
    phi = orc.potential_fft(rho, (h, h, h))
    # self term: the centre-cell integral
    assert phi[17, 17, 17] == pytest.approx(K * q / h * cube_self_integral(), rel=1e-13)
    for R in (4, 8, 16):
        ratio = phi[17, 17, 17 + R] * R * h / (K * q)
        predicted = 1.0 - (1.0 / 960.0) * (35.0 - 21.0) / R ** 4
        assert ratio == pytest.approx(predicted, abs=3.0 / R ** 6)


def gaussian_potential(r, sigma, Q):
    r = np.maximum(r, 1e-30)
    return K * Q * special.erf(r / (math.sqrt(2.0) * sigma)) / r


def test_gaussian_density_second_order_convergence():
    """rho = Q N(0, sigma^2 I) sampled on a +-5 sigma mesh; phi vs the erf law."""
    sigma, Q = 1e-3, 1e-9
    errs = []
    for n in (16, 32, 64):
        h = 10.0 * sigma / (n - 1)
        c = (np.arange(n) - 0.5 * (n - 1)) * h
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        r = np.sqrt(X * X + Y * Y + Z * Z)
        rho = Q * np.exp(-0.5 * (r / sigma) ** 2) / ((2 * math.pi) ** 1.5 * sigma ** 3)
        phi = orc.potential_fft(rho, (h, h, h))[1:-1, 1:-1, 1:-1]
        errs.append(_rel_l2(phi, gaussian_potential(r, sigma, Q)))
    assert errs[0] < 6e-3
    for a, b in zip(errs, errs[1:]):
        assert a / b == pytest.approx(4.0, abs=0.3)


# --------------------------------------------------------------------------
# CIC deposit and gather
# --------------------------------------------------------------------------

def _random_particles(num, n, h, origin, seed, margin=0.0):
    g = np.random.default_rng(seed)
    pos = []
    for d in range(3):
        lo = origin[d] + margin * h[d]
        hi = origin[d] + (n[d] - 1 - margin) * h[d]
        pos.append(g.uniform(lo, hi, num))
    return pos


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_deposit_conserves_charge_and_dipole(dtype):
    n = (9, 7, 11)
    h = (1e-4, 2e-4, 1.5e-4)
    origin = orc.centred_origin(n, h)
    x, y, z = (np.asarray(c).astype(dtype) for c in _random_particles(5000, n, h, origin, 5))
    q = 2e-15
    Q, n_out = orc.deposit_cic(x, y, z, q, n, h, origin, dtype)
    assert n_out == 0
    assert Q.sum() == pytest.approx(q * 5000, rel=1e-13)
    # CIC reproduces the first moment exactly (its weights interpolate
    # linearly), and the weights come from the FP64 cell coordinate of the
    # input positions, so the deposited dipole is that of the positions as
    # given (FP32 inputs included: no FP32 rounding of s enters the weights)
    nodes = [origin[d] + np.arange(n[d]) * h[d] for d in range(3)]
    for d, axis, pos in ((0, 2, x), (1, 1, y), (2, 0, z)):
        shape = [1, 1, 1]
        shape[axis] = n[d]
        moment = float((Q * nodes[d].reshape(shape)).sum())
        want = q * float(np.sum(pos.astype(np.float64)))
        assert moment == pytest.approx(want, rel=1e-12, abs=1e-13 * q * 5000 * h[d])


def test_deposit_node_and_edges():
    n = (5, 5, 5)
    h = (1.0, 1.0, 1.0)
    origin = (0.0, 0.0, 0.0)
    # exactly on node (2, 3, 1); exactly on the last node; just outside each face
    x = np.array([2.0, 4.0, -1e-9, 4.0 + 1e-9, 1.0])
    y = np.array([3.0, 4.0, 1.0, 1.0, 0.5])
    z = np.array([1.0, 4.0, 1.0, 1.0, 2.5])
    Q, n_out = orc.deposit_cic(x, y, z, 1.0, n, h, origin)
    assert n_out == 2
    assert Q[1, 3, 2] == pytest.approx(1.0)
    assert Q[4, 4, 4] == pytest.approx(1.0)
    # (1, 0.5, 2.5): four nodes with 1/4 each
    for (k, j) in ((2, 0), (2, 1), (3, 0), (3, 1)):
        assert Q[k, j, 1] == pytest.approx(0.25)
    assert Q.sum() == pytest.approx(3.0)


def test_deposit_pure_python_loop_small():
    """Independent per-particle loop (scalar arithmetic, no numpy indexing tricks)."""
    n = (4, 5, 6)
    h = (0.5, 0.25, 1.0)
    origin = (-0.7, 0.1, 2.0)
    xs, ys, zs = _random_particles(40, n, h, origin, 9, margin=-0.3)  # some outside
    Q, n_out = orc.deposit_cic(xs, ys, zs, 1.0, n, h, origin)
    ref = np.zeros((n[2], n[1], n[0]))
    outside = 0
    for p in range(40):
        pos = (xs[p], ys[p], zs[p])
        s = [(pos[d] - origin[d]) * (1.0 / h[d]) for d in range(3)]
        if any(s[d] < 0 or s[d] > n[d] - 1 for d in range(3)):
            outside += 1
            continue
        i = [min(int(math.floor(s[d])), n[d] - 2) for d in range(3)]
        f = [s[d] - i[d] for d in range(3)]
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    w = ((f[0] if cx else 1 - f[0]) * (f[1] if cy else 1 - f[1])
                         * (f[2] if cz else 1 - f[2]))
                    ref[i[2] + cz, i[1] + cy, i[0] + cx] += w
    assert n_out == outside and outside > 0
    np.testing.assert_allclose(Q, ref, rtol=1e-13, atol=1e-15)


def _round_f32(v):
    """Nearest binary32 value of the rational v (ties to even), by exact
    rational arithmetic (no floating point on the way)."""
    from fractions import Fraction
    v = Fraction(v)
    if v == 0:
        return Fraction(0)
    sign = -1 if v < 0 else 1
    a = abs(v)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    scale = Fraction(2) ** (e - 23)           # 24-bit significand (normal range)
    m = a / scale
    lo = m.numerator // m.denominator
    rem = m - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    return sign * lo * scale


def test_float32_cell_decision_uses_float32_arithmetic():
    """The in/out decision and the cell of an FP32 particle come from
    s = (x - x0) * (1/h) with two correctly rounded binary32 operations
    (x0 and 1/h rounded to binary32 from FP64), emulated here by exact
    rational arithmetic.  FP32 positions next to the mesh end and to interior
    nodes are scanned; some of them are decided differently by exact
    arithmetic, and the oracle must follow the binary32 result for all."""
    from fractions import Fraction
    n, h, origin = (4, 4, 4), (0.1, 0.1, 0.1), (0.0, 0.0, 0.0)
    inv32 = _round_f32(Fraction(1.0 / 0.1))
    cands = []
    for centre in (np.float32(0.3), np.float32(0.2), np.float32(0.1)):
        v = centre
        for _ in range(8):
            v = np.nextafter(v, np.float32(-1))
        for _ in range(17):
            cands.append(v)
            v = np.nextafter(v, np.float32(1))
    x = np.array(cands, dtype=np.float32)
    yz = np.full(x.size, 0.15, dtype=np.float32)
    s_dec, s_exact = orc.cell_coordinates(x, origin[0], h[0], np.float32)
    differs = 0
    for k, xv in enumerate(x):
        s32 = _round_f32(_round_f32(Fraction(float(xv)) - 0) * inv32)
        assert Fraction(float(s_dec[k])) == s32
        ex = Fraction(float(xv)) / Fraction(0.1)
        inside32, inside_ex = 0 <= s32 <= 3, 0 <= ex <= 3
        cell32 = min(int(s32), 2) if inside32 else None
        cell_ex = min(int(ex), 2) if inside_ex else None
        differs += (inside32 != inside_ex) or (cell32 != cell_ex)
        assert s_exact[k] == pytest.approx(float(ex), rel=2e-16)
    assert differs > 0
    inside, idx, frac = orc.cic_stencil(x, yz, yz, n, h, origin, np.float32)
    for k in range(x.size):
        s32 = Fraction(float(s_dec[k]))
        assert bool(inside[k]) == (0 <= s32 <= 3)
        if inside[k]:
            assert idx[0][k] == min(int(s32), 2)
            assert frac[0][k] == pytest.approx(float(s_exact[k]) - idx[0][k], abs=1e-15)
    Q, n_out = orc.deposit_cic(x, yz, yz, 1.0, n, h, origin, np.float32)
    assert n_out == int((~inside).sum())
    assert Q.sum() == pytest.approx(float(inside.sum()), rel=1e-14)


def test_gradient_exact_for_quadratic():
    n = (6, 7, 8)
    h = (0.3, 0.2, 0.5)
    i = np.arange(-1, n[0] + 1) * h[0]
    j = np.arange(-1, n[1] + 1) * h[1]
    k = np.arange(-1, n[2] + 1) * h[2]
    Z, Y, X = np.meshgrid(k, j, i, indexing="ij")
    phi = 1.5 + 2.0 * X - 3.0 * Y + 0.5 * Z + 0.7 * X * X - 0.2 * Y * Z + 0.3 * Z * Z
    E = orc.gradient(phi, h)
    core = (slice(1, -1),) * 3
    np.testing.assert_allclose(E[0], -(2.0 + 1.4 * X[core]), rtol=1e-12)
    np.testing.assert_allclose(E[1], -(-3.0 - 0.2 * Z[core]), rtol=1e-12)
    np.testing.assert_allclose(E[2], -(0.5 - 0.2 * Y[core] + 0.6 * Z[core]), rtol=1e-12)


def test_gather_reproduces_trilinear_field():
    n = (6, 5, 7)
    h = (0.5, 0.25, 1.0)
    origin = (1.0, -2.0, 0.5)
    nodes = [origin[d] + np.arange(n[d]) * h[d] for d in range(3)]
    Z, Y, X = np.meshgrid(nodes[2], nodes[1], nodes[0], indexing="ij")
    f = lambda x, y, z: (0.3 + 1.1 * x - 0.4 * y + 2.0 * z + 0.5 * x * y - 0.25 * y * z
                         + 0.125 * x * y * z)
    E = np.stack([f(X, Y, Z), 2.0 * f(X, Y, Z), -f(X, Y, Z)])
    x, y, z = _random_particles(300, n, h, origin, 4)
    out = orc.gather_cic(E, x, y, z, n, h, origin)
    want = f(np.asarray(x), np.asarray(y), np.asarray(z))
    np.testing.assert_allclose(out[0], want, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out[1], 2.0 * want, rtol=1e-12, atol=1e-12)
    # particles outside receive zero
    out2 = orc.gather_cic(E, np.array([origin[0] - 0.1]), np.array([0.0]), np.array([1.0]),
                          n, h, origin)
    assert np.all(out2 == 0.0)


def test_fitted_mesh_leaves_margin():
    x, y, z = wl.gaussian_bunch(20000, (1e-3, 2e-3, 0.5e-3), 7)
    n = (16, 24, 20)
    hc, origin = orc.fit_mesh(x, y, z, n)
    for c, o, nd in zip((x, y, z), origin, n):
        s = (c - o) / hc
        assert s.min() >= 1.0 - 1e-12 and s.max() <= nd - 2 + 1e-12
    # the binding axis spans exactly n-3 cells
    ext = [c.max() - c.min() for c in (x, y, z)]
    assert max(e / (nd - 3) for e, nd in zip(ext, n)) == pytest.approx(hc, rel=1e-15)


# --------------------------------------------------------------------------
# Whole path against analytic fields
# --------------------------------------------------------------------------

def test_uniform_sphere_particles_analytic():
    R, Q = 2.5e-3, 1e-9
    num = 400_000
    x, y, z = wl.uniform_ball(num, R, 2)
    n = (48, 48, 48)
    out = orc.solve_particles(x, y, z, Q / num, n)
    assert out["n_outside"] == 0
    h = out["h"][0]
    o = out["origin"]
    c = [o[d] + np.arange(n[d]) * h for d in range(3)]
    Zg, Yg, Xg = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    r = np.sqrt(Xg ** 2 + Yg ** 2 + Zg ** 2)
    rho0 = Q / (4.0 / 3.0 * math.pi * R ** 3)
    eps0 = 8.8541878128e-12
    ana = np.where(r < R, rho0 * (3 * R * R - r * r) / (6 * eps0), K * Q / np.maximum(r, 1e-30))
    phi = out["phi_ext"][1:-1, 1:-1, 1:-1]
    assert _rel_l2(phi, ana) < 3e-3
    # field at the particles inside 0.8 R: E = rho r / (3 eps0)
    rp = np.sqrt(x ** 2 + y ** 2 + z ** 2)
    sel = rp < 0.8 * R
    Er = (out["E"][0] * x + out["E"][1] * y + out["E"][2] * z)[sel] / rp[sel]
    assert _rel_l2(Er, rho0 * rp[sel] / (3 * eps0)) < 3e-2


def test_gaussian_particles_field_analytic():
    """Fitted mesh over a Gaussian bunch: phi and E at the particles approach the
    erf laws, and the E error falls as the mesh is refined (CIC is second order)."""
    sigma, Q, num = 1e-3, 1e-9, 200_000
    x, y, z = wl.gaussian_bunch(num, (sigma, sigma, sigma), 12)
    rp = np.sqrt(x ** 2 + y ** 2 + z ** 2)
    a = rp / (math.sqrt(2) * sigma)
    Er_ana = K * Q * (special.erf(a) / rp ** 2
                      - math.sqrt(2 / math.pi) * np.exp(-a * a) / (sigma * rp))
    errs = []
    for n in (32, 64):
        out = orc.solve_particles(x, y, z, Q / num, (n, n, n))
        h = out["h"][0]
        o = out["origin"]
        c = [o[d] + np.arange(n) * h for d in range(3)]
        Zg, Yg, Xg = np.meshgrid(c[2], c[1], c[0], indexing="ij")
        r = np.sqrt(Xg ** 2 + Yg ** 2 + Zg ** 2)
        phi = out["phi_ext"][1:-1, 1:-1, 1:-1]
        assert _rel_l2(phi, gaussian_potential(r, sigma, Q)) < 1e-2
        Er = (out["E"][0] * x + out["E"][1] * y + out["E"][2] * z) / rp
        errs.append(_rel_l2(Er, Er_ana))
    assert errs[0] < 6e-2
    assert errs[1] < 0.5 * errs[0]


def test_small_config_literal_reading_excludes_particles():
    cfg = wl.SMALL_GAUSSIAN
    x, y, z = wl.particles_for(cfg)
    out = orc.solve_particles(x, y, z, cfg.charge_per_particle, cfg.n, cfg.h)
    frac_in = 1.0 - out["n_outside"] / cfg.num_particles
    # +-1.55 sigma per axis: erf(1.55/sqrt2)^3 ~ 0.68 of the bunch is on the mesh
    assert frac_in == pytest.approx(special.erf(15.5e-4 / (math.sqrt(2) * 1e-3)) ** 3, abs=0.01)
    assert out["Q"].sum() == pytest.approx(cfg.charge_per_particle * (cfg.num_particles - out["n_outside"]),
                                          rel=1e-12)
    assert np.all(out["E"][:, (np.abs(x) > 15.5e-4)] == 0.0)


# --------------------------------------------------------------------------
# Assignment schemes (NGP, TSC beside CIC) and the point kernel
# --------------------------------------------------------------------------

def _unit_mesh_particles(num, n, seed, margin=1.5):
    g = np.random.default_rng(seed)
    pts = [g.uniform(margin, n[d] - 1 - margin, num) for d in range(3)]
    return pts


def test_generic_cic_equals_dedicated_cic():
    n, h = (12, 10, 9), (1.0, 1.0, 1.0)
    x, y, z = _unit_mesh_particles(500, n, 3, margin=0.0)
    origin = (0.0, 0.0, 0.0)
    Q1, o1 = orc.deposit(x, y, z, 1e-12, n, h, origin, scheme="cic")
    Q2, o2 = orc.deposit_cic(x, y, z, 1e-12, n, h, origin)
    assert o1 == o2 == 0
    assert np.allclose(Q1, Q2, rtol=0, atol=1e-27)
    E = np.random.default_rng(4).standard_normal((3, n[2], n[1], n[0]))
    assert np.allclose(orc.gather(E, x, y, z, n, h, origin, scheme="cic"),
                       orc.gather_cic(E, x, y, z, n, h, origin), rtol=0, atol=1e-13)


def test_tsc_weights_partition_unity_first_and_second_moment():
    """TSC weights: sum 1, zero first moment, second moment exactly 1/4 about
    the particle (a dropped term, a wrong sign or a shifted offset breaks one)."""
    n, h = (16, 16, 16), (1.0, 1.0, 1.0)
    x, y, z = _unit_mesh_particles(2000, n, 5)
    inside, base, weights = orc.stencil(x, y, z, n, h, (0.0, 0.0, 0.0), np.float64, "tsc")
    assert inside.all()
    s = (x, y, z)
    for d in range(3):
        w = weights[d]
        assert len(w) == 3
        assert np.allclose(w[0] + w[1] + w[2], 1.0, atol=1e-15)
        first = sum(w[k] * (base[d] + k - s[d]) for k in range(3))
        second = sum(w[k] * (base[d] + k - s[d]) ** 2 for k in range(3))
        assert np.allclose(first, 0.0, atol=1e-13)
        assert np.allclose(second, 0.25, atol=1e-13)
        assert np.all(np.abs(base[d] + 1 - s[d]) <= 0.5)          # centre is the nearest node


def test_tsc_particle_on_a_node_and_ngp_nearest_node():
    n, h = (8, 8, 8), (1.0, 1.0, 1.0)
    Q, out = orc.deposit([3.0], [4.0], [5.0], 1.0, n, h, (0.0, 0.0, 0.0), scheme="tsc")
    assert out == 0
    w1 = np.array([0.125, 0.75, 0.125])
    expect = np.zeros((8, 8, 8))
    expect[4:7, 3:6, 2:5] = w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
    assert np.allclose(Q, expect, atol=1e-16)
    # NGP by brute force: each particle's whole charge at round-half-up(s)
    g = np.random.default_rng(8)
    px, py, pz = (g.uniform(0, 7, 40) for _ in range(3))
    px[0] = 2.5                                           # a tie goes up
    Q, out = orc.deposit(px, py, pz, 1.0, n, h, (0.0, 0.0, 0.0), scheme="ngp")
    ref = np.zeros((8, 8, 8))
    for a, b, c in zip(px, py, pz):
        ref[int(math.floor(c + 0.5)), int(math.floor(b + 0.5)), int(math.floor(a + 0.5))] += 1.0
    assert out == 0 and np.array_equal(Q, ref)
    assert Q[int(math.floor(pz[0] + 0.5)), int(math.floor(py[0] + 0.5)), 3] >= 1.0


def test_tsc_inside_rule_and_charge_conservation():
    n, h = (10, 10, 10), (1.0, 1.0, 1.0)
    g = np.random.default_rng(9)
    x, y, z = (g.uniform(-0.3, 9.3, 3000) for _ in range(3))
    for scheme in orc.SCHEMES:
        Q, out = orc.deposit(x, y, z, 2.0, n, h, (0.0, 0.0, 0.0), scheme=scheme)
        inside, base, w = orc.stencil(x, y, z, n, h, (0.0, 0.0, 0.0), np.float64, scheme)
        assert out == int((~inside).sum())
        assert math.isclose(Q.sum(), 2.0 * inside.sum(), rel_tol=1e-13)
        if scheme == "tsc":
            near = [np.floor(c + 0.5) for c in (x, y, z)]
            ok = np.ones(x.size, bool)
            for d in range(3):
                ok &= (near[d] >= 1) & (near[d] <= 8) & ((x, y, z)[d] >= 0) & ((x, y, z)[d] <= 9)
            assert np.array_equal(inside, ok)


def test_gather_reproduces_linear_field_cic_tsc_and_constant_ngp():
    n, h = (12, 11, 10), (1e-3, 2e-3, 1.5e-3)
    origin = orc.centred_origin(n, h)
    g = np.random.default_rng(10)
    x = origin[0] + g.uniform(1.5, n[0] - 2.5, 300) * h[0]
    y = origin[1] + g.uniform(1.5, n[1] - 2.5, 300) * h[1]
    z = origin[2] + g.uniform(1.5, n[2] - 2.5, 300) * h[2]
    kk, jj, ii = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    xn, yn, zn = origin[0] + ii * h[0], origin[1] + jj * h[1], origin[2] + kk * h[2]
    E = np.stack([3.0 * xn - 2.0 * yn + 1.0, 0.5 * zn + 4.0, -xn + yn + zn])
    exact = np.stack([3.0 * x - 2.0 * y + 1.0, 0.5 * z + 4.0, -x + y + z])
    for scheme in ("cic", "tsc"):
        got = orc.gather(E, x, y, z, n, h, origin, scheme=scheme)
        assert np.allclose(got, exact, rtol=1e-12, atol=1e-12)
    const = np.ones((3,) + xn.shape) * np.array([1.0, -2.0, 0.5])[:, None, None, None]
    got = orc.gather(const, x, y, z, n, h, origin, scheme="ngp")
    assert np.allclose(got, np.array([1.0, -2.0, 0.5])[:, None], atol=1e-15)


@pytest.mark.parametrize("R", [8, 16])
def test_point_kernel_against_integrated_far_field(R):
    """V/R differs from the cell integral by the cube's quadrupole-free
    multipole term: G_int / (V / R) - 1 = -(h^4 / 960)(35 sum x^4 / R^4 - 21) / R^4."""
    h = (1.0, 1.0, 1.0)
    Kp = orc.point_kernel_octant((R, 1, 1), h)
    Gi = orc.igf_octant((R, 1, 1), h)
    assert Kp[0, 0, 0] == Gi[0, 0, 0]
    predicted = -(1.0 / 960.0) * (35.0 - 21.0) / R ** 4
    assert math.isclose(Gi[0, 0, R] / Kp[0, 0, R] - 1.0, predicted, rel_tol=2e-2)


def test_point_kernel_convolution_direct_sum_and_point_charge():
    n, h = (8, 8, 8), (1e-4, 1e-4, 1e-4)
    rho = np.random.default_rng(11).standard_normal((8, 8, 8))
    a = orc.potential_direct(rho, h, green="point")
    b = orc.potential_fft(rho, h, green="point")
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-14
    # one charge exactly on a node: phi = q / (4 pi eps0 r) exactly at every other node
    q = 1e-12
    Q, _ = orc.deposit([0.0], [0.0], [0.0], q, n, h, (-3e-4, -4e-4, -2e-4), scheme="ngp")
    phi = orc.potential_fft(Q / (h[0] * h[1] * h[2]), h, green="point")
    kk, jj, ii = np.meshgrid(np.arange(-1, 9), np.arange(-1, 9), np.arange(-1, 9), indexing="ij")
    r = np.sqrt(((ii - 3) * h[0]) ** 2 + ((jj - 4) * h[1]) ** 2 + ((kk - 2) * h[2]) ** 2)
    mask = r > 0
    assert np.allclose(phi[mask], orc.COULOMB_K * q / r[mask], rtol=1e-12)
