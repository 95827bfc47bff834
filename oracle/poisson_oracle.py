"""FP64 CPU oracle for the Hockney free-space particle-mesh Poisson solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code, constants or tables with the
HIP library.

What it computes (paper section "FFT Based Particle-Mesh Solver", subsection
"FFT-based Convolutions"; the open-boundary doubled grid of the same section):

  1. Charge assignment of particles to mesh nodes (the "NGP, CIC, TSI"
     interpolation box of the OPAL/IPPL structure figure): CIC by default,
     nearest grid point and the triangular-shaped cloud as variants (read as
     the second-order, 27-node scheme).
  2. The integrated Green's function (IGF): the free-space kernel 1/r of the
     equation following the convolution solution, integrated over one mesh
     cell.  At every offset it is the alternating sum of a closed-form
     antiderivative over the cell corners, evaluated in 113-bit arithmetic
     (oracle/igf_quad.c, built with gcc) so that the sum's cancellation, which
     would cost FP64 up to 9 digits at 256 cells, leaves it exact to FP64
     rounding.
  3. The discrete free-space convolution of the brute-force equation
     (phi_ijk = sum rho G_{i-i',j-j',k-k'}), done two ways:
       potential_direct -- the literal O(M^2) double sum (small meshes only);
       potential_fft    -- cyclic convolution on the zero-padded 2M grid using
                           scipy.fft (pocketfft) as a library step
                           (Hadamard-product form).
  4. E = -grad(phi) by second-order central differences (the D-operators box
     of the structure figure).
  5. Interpolation of the mesh field back to the particles with the same
     weights as the assignment.

The point kernel of the brute-force equation (G = 1/r times the cell volume,
with the cell integral standing in at the singular origin) is available as
a variant of step 2.

Readings of the paper adopted where it is silent (each also listed in the
design notes of the repository):
  * phi = 1/(4 pi eps0) * sum_j rho_j * G_int(i-j); G_int already integrates
    over a cell (units m^2), so there is no separate h_x h_y h_z factor.
  * Nodes are vertex-centred: x_i = x0 + i*h, i = 0..n-1.
  * phi is returned on the extended box [-1, n] per axis (a one-node ghost
    layer), which the doubled grid gives exactly when the kernel value at
    offset n is the true G_int(n).
  * Where floating point decides an integer -- a particle's in/out-of-mesh
    status and its stencil node -- the decision is taken on
    s = (x - x0) * (1/h) evaluated in the run's dtype with two correctly
    rounded operations (difference, then product), as the run does.  The
    weights then come from the FP64 cell coordinate (x - x0) / h of the same
    input positions, so the oracle's result carries none of the dtype's
    position rounding.
  * eps0 = 8.8541878128e-12 F/m (CODATA 2018).
"""

import concurrent.futures
import math
import os

import numpy as np
import scipy.fft

EPS0 = 8.8541878128e-12  # F/m, CODATA 2018
COULOMB_K = 1.0 / (4.0 * math.pi * EPS0)


# --------------------------------------------------------------------------
# Mesh geometry
# --------------------------------------------------------------------------

def centred_origin(n, h):
    """Origin of an explicit-h mesh centred at 0: x0 = -(n-1) h / 2."""
    return tuple(-0.5 * (nd - 1) * hd for nd, hd in zip(n, h))


def fit_mesh(x, y, z, n):
    """Particle-fitted cubic mesh (the mesh-spacing remark of the PM section).

    h = max_d (hi_d - lo_d) / (n_d - 3); the origin centres the bounding box,
    x0_d = (lo_d + hi_d)/2 - (n_d - 1) h / 2, which leaves at least one empty
    node of margin on each side.  With no particles, or all particles at one
    point, h = 1 m and the box sits at the origin (lo = hi = 0 without
    particles).  Bounding-box values are the inputs as given (FP32 inputs are
    widened exactly); h and the origin are FP64.
    Returns (h, (x0, y0, z0)).
    """
    coords = [np.asarray(c, dtype=np.float64) for c in (x, y, z)]
    if coords[0].size == 0:
        lo = [0.0, 0.0, 0.0]
        hi = [0.0, 0.0, 0.0]
    else:
        lo = [float(c.min()) for c in coords]
        hi = [float(c.max()) for c in coords]
    h = 0.0
    for d in range(3):
        h = max(h, (hi[d] - lo[d]) / (n[d] - 3))
    if not h > 0.0:
        h = 1.0
    origin = tuple(0.5 * (lo[d] + hi[d]) - 0.5 * (n[d] - 1) * h for d in range(3))
    return h, origin


def cell_coordinates(pos, origin, h, dtype):
    """Cell coordinate of each position, for decisions and for weights.

    Returns (s_dec, s_exact) as FP64 arrays:
      s_dec   -- (pos - x0) * (1/h) in `dtype`: x0 and 1/h rounded from FP64 to
                 the dtype, then two correctly rounded dtype operations.  It
                 decides the in/out status and the stencil node.
      s_exact -- (pos - origin) / h in FP64 from the same input positions
                 (FP32 inputs widened exactly).  It gives the weights.
    """
    dt = np.dtype(dtype)
    x0 = dt.type(origin)
    inv = dt.type(1.0 / h)
    p = np.asarray(pos).astype(dt)
    s_dec = (p - x0) * inv
    s_exact = (p.astype(np.float64) - float(origin)) / float(h)
    return s_dec.astype(np.float64), s_exact


def _nearest_node(s_dec, dtype):
    """floor(s + 1/2) with the addition rounded in the dtype (halves go up)."""
    dt = np.dtype(dtype)
    return np.floor((s_dec.astype(dt) + dt.type(0.5)).astype(np.float64))


def cic_stencil(x, y, z, n, h, origin, dtype):
    """CIC cell index and fractional offsets of each particle.

    Returns (inside mask, i[3] int64 lower node index, f[3] float64 fraction).
    A particle is outside when s_d < 0 or s_d > n_d - 1 on any axis.  The
    lower node is min(floor(s), n-2), so a particle exactly on the last node
    goes entirely to it with f = 1.  Inside test and node use the dtype's
    s; the fraction f = s_exact - i is FP64.
    """
    cs = [cell_coordinates(c, o, hd, dtype) for c, o, hd in zip((x, y, z), origin, h)]
    inside = np.ones(cs[0][0].shape, dtype=bool)
    for d in range(3):
        inside &= (cs[d][0] >= 0.0) & (cs[d][0] <= n[d] - 1)
    idx, frac = [], []
    for d in range(3):
        sd = np.where(inside, cs[d][0], 0.0)
        se = np.where(inside, cs[d][1], 0.0)
        i = np.minimum(np.floor(sd), n[d] - 2).astype(np.int64)
        idx.append(i)
        frac.append(se - i)
    return inside, idx, frac


def _corner_weights(frac):
    """The eight trilinear weights, keyed by corner offset (cz, cy, cx)."""
    fx, fy, fz = frac
    wx = (1.0 - fx, fx)
    wy = (1.0 - fy, fy)
    wz = (1.0 - fz, fz)
    out = {}
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                out[(cz, cy, cx)] = wz[cz] * wy[cy] * wx[cx]
    return out


# --------------------------------------------------------------------------
# Assignment schemes of the interpolation box of the OPAL/IPPL structure
# figure ("NGP, CIC, TSI"): nearest grid point, cloud in cell (linear) and
# the triangular-shaped cloud (quadratic, 27 nodes).  The same weights assign
# charge to the mesh and interpolate the field back.
# --------------------------------------------------------------------------

SCHEMES = ("ngp", "cic", "tsc")


def stencil(x, y, z, n, h, origin, dtype, scheme="cic"):
    """Assignment stencil of each particle.

    Returns (inside, base[3], weights[3]): base[d] is the lowest stencil node
    on axis d and weights[d] the list of per-offset weights (1, 2 or 3 of
    them).  A particle is outside when s_d < 0 or s_d > n_d - 1 on any axis,
    or when its stencil would leave the mesh (TSC needs nearest node in
    [1, n-2]).  The nearest node is floor(s + 1/2) (halves round up).
      ngp: weight 1 at the nearest node.
      cic: lower node min(floor(s), n-2), weights (1-f, f).
      tsc: d = s - nearest; weights ((1/2 - d)^2 / 2, 3/4 - d^2, (1/2 + d)^2 / 2)
           at nearest - 1, nearest, nearest + 1.
    The inside test and the nodes use the dtype's s (s_dec of
    cell_coordinates); f and d use the FP64 s_exact.
    """
    if scheme not in SCHEMES:
        raise ValueError(scheme)
    cs = [cell_coordinates(c, o, hd, dtype) for c, o, hd in zip((x, y, z), origin, h)]
    inside = np.ones(cs[0][0].shape, dtype=bool)
    for d in range(3):
        inside &= (cs[d][0] >= 0.0) & (cs[d][0] <= n[d] - 1)
    near = [_nearest_node(c[0], dtype) for c in cs]
    if scheme == "tsc":
        for d in range(3):
            inside &= (near[d] >= 1) & (near[d] <= n[d] - 2)
    base, weights = [], []
    for d in range(3):
        sd = np.where(inside, cs[d][0], 0.0)
        se = np.where(inside, cs[d][1], 0.0)
        if scheme == "cic":
            i = np.minimum(np.floor(sd), n[d] - 2)
            f = se - i
            base.append(i.astype(np.int64))
            weights.append([1.0 - f, f])
        else:
            k = np.where(inside, near[d], 0.0)
            if scheme == "ngp":
                base.append(k.astype(np.int64))
                weights.append([np.ones_like(sd)])
            else:
                dd = se - k
                base.append((k - 1).astype(np.int64))
                weights.append([0.5 * (0.5 - dd) ** 2, 0.75 - dd * dd, 0.5 * (0.5 + dd) ** 2])
    return inside, base, weights


# Particles are taken in chunks of this many, which bounds the memory of the
# per-particle temporaries at large counts; every sum stays FP64.
_CHUNK = 1 << 22

# Host threads: chunks of particles are processed by a pool of this many
# threads (each chunk's arithmetic is the same as alone; the deposit adds the
# chunks' node sums in chunk order), and the FFTs of the convolution use as
# many workers.  set_threads(1) runs everything on one core.
_THREADS = max(1, min(os.cpu_count() or 1, 16))


def set_threads(num):
    """Number of host threads the oracle uses (chunk pool, FFT workers and the
    Green's function loops of the C part)."""
    global _THREADS
    _THREADS = max(1, int(num))
    if _LIB is not None:
        _LIB.oracle_set_threads(_THREADS)


def threads():
    return _THREADS


def _chunks(num):
    return [(lo, min(lo + _CHUNK, num)) for lo in range(0, num, _CHUNK)] or [(0, 0)]


def _map_chunks(fn, num):
    """fn(lo, hi) over the particle chunks, results in chunk order."""
    parts = _chunks(num)
    if _THREADS == 1 or len(parts) == 1:
        return [fn(lo, hi) for lo, hi in parts]
    with concurrent.futures.ThreadPoolExecutor(min(_THREADS, len(parts))) as ex:
        return list(ex.map(lambda c: fn(*c), parts))


def deposit(x, y, z, q, n, h, origin, dtype=np.float64, scheme="cic"):
    """Charge per node Q[nz, ny, nx] (coulomb) with the given scheme; (Q, n_outside)."""
    nx, ny, nz = n
    Q = np.zeros((nz, ny, nx), dtype=np.float64)
    n_out = 0
    parts = _map_chunks(lambda lo, hi: _deposit_part(x[lo:hi], y[lo:hi], z[lo:hi], q, n, h, origin, dtype,
                                                     scheme), np.asarray(x).size)
    for Qc, oc in parts:
        Q += Qc
        n_out += oc
    return Q, n_out


def _deposit_part(x, y, z, q, n, h, origin, dtype, scheme):
    nx, ny, nz = n
    inside, (bx, by, bz), (wx, wy, wz) = stencil(x, y, z, n, h, origin, dtype, scheme)
    sel = np.nonzero(inside)[0]
    Q = np.zeros(nx * ny * nz, dtype=np.float64)
    for cz, wzc in enumerate(wz):
        for cy, wyc in enumerate(wy):
            for cx, wxc in enumerate(wx):
                node = ((bz[sel] + cz) * ny + (by[sel] + cy)) * nx + (bx[sel] + cx)
                Q += np.bincount(node, weights=q * wzc[sel] * wyc[sel] * wxc[sel], minlength=nx * ny * nz)
    return Q.reshape(nz, ny, nx), int(inside.size - sel.size)


def gather(E, x, y, z, n, h, origin, dtype=np.float64, scheme="cic"):
    """Field at the particles, sum over the stencil of weight * E(node); 0 outside."""
    out = np.zeros((3, np.asarray(x).size), dtype=np.float64)

    def part(lo, hi):
        out[:, lo:hi] = _gather_part(E, x[lo:hi], y[lo:hi], z[lo:hi], n, h, origin, dtype, scheme)

    _map_chunks(part, out.shape[1])
    return out


def _gather_part(E, x, y, z, n, h, origin, dtype, scheme):
    inside, (bx, by, bz), (wx, wy, wz) = stencil(x, y, z, n, h, origin, dtype, scheme)
    out = np.zeros((3, inside.size), dtype=np.float64)
    for cz, wzc in enumerate(wz):
        for cy, wyc in enumerate(wy):
            for cx, wxc in enumerate(wx):
                w = wzc * wyc * wxc
                for d in range(3):
                    out[d] += w * E[d][bz + cz, by + cy, bx + cx]
    out[:, ~inside] = 0.0
    return out


# --------------------------------------------------------------------------
# 1. CIC deposit
# --------------------------------------------------------------------------

def deposit_cic(x, y, z, q, n, h, origin, dtype=np.float64):
    """Charge per node Q[nz, ny, nx] (coulomb) from particles of charge q each.

    Each inside particle adds q * w_x w_y w_z to the eight nodes around it.
    Returns (Q, n_outside).  rho = Q / (h_x h_y h_z).
    """
    nx, ny, nz = n
    Q = np.zeros((nz, ny, nx), dtype=np.float64)
    n_out = 0
    parts = _map_chunks(lambda lo, hi: _deposit_cic_part(x[lo:hi], y[lo:hi], z[lo:hi], q, n, h, origin, dtype),
                        np.asarray(x).size)
    for Qc, oc in parts:
        Q += Qc
        n_out += oc
    return Q, n_out


def _deposit_cic_part(x, y, z, q, n, h, origin, dtype):
    nx, ny, nz = n
    inside, (ix, iy, iz), frac = cic_stencil(x, y, z, n, h, origin, dtype)
    Q = np.zeros(nx * ny * nz, dtype=np.float64)
    sel = np.nonzero(inside)[0]
    ix, iy, iz = ix[sel], iy[sel], iz[sel]
    w = _corner_weights([f[sel] for f in frac])
    for (cz, cy, cx), wc in w.items():
        node = ((iz + cz) * ny + (iy + cy)) * nx + (ix + cx)
        Q += np.bincount(node, weights=q * wc, minlength=nx * ny * nz)
    return Q.reshape(nz, ny, nx), int(inside.size - sel.size)


# --------------------------------------------------------------------------
# 2. Integrated Green's function
# --------------------------------------------------------------------------

def _igf_lib():
    """The oracle's C library (igf_quad.c), built with gcc on first use."""
    global _LIB
    if _LIB is None:
        import ctypes
        from oracle import build as _build
        lib = ctypes.CDLL(_build.ensure_built())
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_igf_octant.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [dp]
        lib.oracle_igf_octant.restype = ctypes.c_int
        lib.oracle_igf_at.argtypes = [ctypes.c_int64, ip, ip, ip] + [ctypes.c_double] * 3 + [dp]
        lib.oracle_igf_at.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads(_THREADS)
        _LIB = lib
    return _LIB


_LIB = None


def _ptr(a, ctype):
    import ctypes
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def igf_at(a, b, c, h):
    """G_int(a, b, c): the integral of 1/r over the cell centred at (a hx, b hy, c hz).

    The alternating sum of the closed-form antiderivative
      F = yz ln(x+r) + xz ln(y+r) + xy ln(z+r)
          - x^2/2 atan(yz/(xr)) - y^2/2 atan(xz/(yr)) - z^2/2 atan(xy/(zr))
    over the eight cell corners, evaluated in 113-bit arithmetic so the
    cancellation of the sum (about 3 log10(offset) digits) leaves the FP64
    result exact to rounding at every offset.  Arrays broadcast; integer
    offsets (negative ones give the value at |offset|).
    """
    import ctypes
    a, b, c = np.broadcast_arrays(*(np.asarray(v) for v in (a, b, c)))
    shape = a.shape
    ai, bi, ci = (np.ascontiguousarray(np.rint(v).astype(np.int64).ravel()) for v in (a, b, c))
    out = np.empty(ai.size, dtype=np.float64)
    rc = _igf_lib().oracle_igf_at(ai.size, _ptr(ai, ctypes.c_int64), _ptr(bi, ctypes.c_int64),
                                  _ptr(ci, ctypes.c_int64), float(h[0]), float(h[1]), float(h[2]),
                                  _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("igf_at: bad arguments")
    out = out.reshape(shape)
    return out if shape else float(out)


def igf_octant(n, h):
    """G_int(a, b, c) for a in [0, nx], b in [0, ny], c in [0, nz]; array [c, b, a].

    Same closed form as igf_at, with F evaluated once per corner of the
    half-integer lattice (a - 1/2) h and differenced along each axis.
    """
    import ctypes
    nx, ny, nz = (int(v) for v in n)
    out = np.empty((nz + 1, ny + 1, nx + 1), dtype=np.float64)
    rc = _igf_lib().oracle_igf_octant(nx, ny, nz, float(h[0]), float(h[1]), float(h[2]),
                                      _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("igf_octant: bad arguments")
    return out


def point_kernel_octant(n, h):
    """The point kernel of the brute-force convolution equation, G = 1/r at the
    node offsets times the cell volume (the equation's h_x h_y h_z factor), on
    the octant [0, n] per axis; array [c, b, a].  G(0) is singular; the cell
    integral G_int(0) stands in for V * G(0)."""
    nx, ny, nz = n
    c, b, a = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    r = np.sqrt((a * h[0]) ** 2 + (b * h[1]) ** 2 + (c * h[2]) ** 2)
    V = h[0] * h[1] * h[2]
    with np.errstate(divide="ignore"):
        K = V / r
    K[0, 0, 0] = igf_at(0, 0, 0, h)
    return K


def kernel_octant(n, h, green="integrated"):
    """The convolution kernel on the octant: 'integrated' (G_int) or 'point'."""
    if green == "integrated":
        return igf_octant(n, h)
    if green == "point":
        return point_kernel_octant(n, h)
    raise ValueError(green)


# --------------------------------------------------------------------------
# 3. Discrete free-space convolution on the extended box [-1, n]^3
# --------------------------------------------------------------------------

def potential_direct(rho, h, green="integrated"):
    """Literal double sum: phi_i = K sum_j rho_j G_int(i - j), i in [-1, n]^3.

    rho is [nz, ny, nx] in C/m^3; returns phi_ext [nz+2, ny+2, nx+2] in volts,
    phi_ext[k+1, j+1, i+1] = phi at node (i, j, k).  O(M^2): small meshes only.
    """
    nz, ny, nx = rho.shape
    G = kernel_octant((nx + 1, ny + 1, nz + 1), h, green)  # offsets up to n+1 are needed
    phi = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.float64)
    ti = np.arange(-1, nx + 1)
    tj = np.arange(-1, ny + 1)
    tk = np.arange(-1, nz + 1)
    src = np.argwhere(rho != 0.0)
    for (k, j, i) in src:
        dz = np.abs(tk - k)[:, None, None]
        dy = np.abs(tj - j)[None, :, None]
        dx = np.abs(ti - i)[None, None, :]
        phi += rho[k, j, i] * G[dz, dy, dx]
    return COULOMB_K * phi


def doubled_kernel(n, h, green="integrated"):
    """K on the 2n grid: K[a] = G(min(a, 2n - a)) per axis (K[n] = G(n))."""
    nx, ny, nz = n
    G = kernel_octant(n, h, green)
    ax = np.minimum(np.arange(2 * nx), 2 * nx - np.arange(2 * nx))
    ay = np.minimum(np.arange(2 * ny), 2 * ny - np.arange(2 * ny))
    az = np.minimum(np.arange(2 * nz), 2 * nz - np.arange(2 * nz))
    return G[az[:, None, None], ay[None, :, None], ax[None, None, :]]


def potential_fft(rho, h, green="integrated"):
    """Hadamard-product form on the zero-padded 2n grid; phi_ext on [-1, n]^3.

    Cyclic convolution of rho (zero-padded to 2n) with K; for target indices
    -1..n every wrapped offset lands on its true |offset| <= n, so the result
    equals the literal sum there.
    """
    nz, ny, nx = rho.shape
    K = doubled_kernel((nx, ny, nz), h, green)
    shape = (2 * nz, 2 * ny, 2 * nx)
    Rk = scipy.fft.rfftn(rho, s=shape, axes=(0, 1, 2), workers=_THREADS)
    Kk = scipy.fft.rfftn(K, workers=_THREADS)
    del K
    Rk *= Kk
    del Kk
    full = scipy.fft.irfftn(Rk, s=shape, axes=(0, 1, 2), workers=_THREADS)
    idz = np.r_[2 * nz - 1, np.arange(nz + 1)]
    idy = np.r_[2 * ny - 1, np.arange(ny + 1)]
    idx = np.r_[2 * nx - 1, np.arange(nx + 1)]
    return COULOMB_K * full[np.ix_(idz, idy, idx)]


# --------------------------------------------------------------------------
# 4. Central-difference field
# --------------------------------------------------------------------------

def gradient(phi_ext, h):
    """E_d(i) = -(phi(i + e_d) - phi(i - e_d)) / (2 h_d), i in [0, n)^3.

    Returns E [3, nz, ny, nx] ordered (Ex, Ey, Ez), V/m.
    """
    hx, hy, hz = h
    Ex = -(phi_ext[1:-1, 1:-1, 2:] - phi_ext[1:-1, 1:-1, :-2]) / (2.0 * hx)
    Ey = -(phi_ext[1:-1, 2:, 1:-1] - phi_ext[1:-1, :-2, 1:-1]) / (2.0 * hy)
    Ez = -(phi_ext[2:, 1:-1, 1:-1] - phi_ext[:-2, 1:-1, 1:-1]) / (2.0 * hz)
    return np.stack([Ex, Ey, Ez])


# --------------------------------------------------------------------------
# 5. CIC gather
# --------------------------------------------------------------------------

def gather_cic(E, x, y, z, n, h, origin, dtype=np.float64):
    """E at the particles: sum over the 8 nodes of w * E(node); 0 outside."""
    out = np.zeros((3, np.asarray(x).size), dtype=np.float64)

    def part(lo, hi):
        out[:, lo:hi] = _gather_cic_part(E, x[lo:hi], y[lo:hi], z[lo:hi], n, h, origin, dtype)

    _map_chunks(part, out.shape[1])
    return out


def _gather_cic_part(E, x, y, z, n, h, origin, dtype):
    inside, (ix, iy, iz), frac = cic_stencil(x, y, z, n, h, origin, dtype)
    w = _corner_weights(frac)
    out = np.zeros((3, inside.size), dtype=np.float64)
    ixc = np.where(inside, ix, 0)
    iyc = np.where(inside, iy, 0)
    izc = np.where(inside, iz, 0)
    for (cz, cy, cx), wc in w.items():
        for d in range(3):
            out[d] += wc * E[d][izc + cz, iyc + cy, ixc + cx]
    out[:, ~inside] = 0.0
    return out


# --------------------------------------------------------------------------
# Whole path
# --------------------------------------------------------------------------

def solve_rho(rho, h, method="fft", green="integrated"):
    """rho [nz,ny,nx] (C/m^3) -> (phi_ext [nz+2,ny+2,nx+2], E [3,nz,ny,nx])."""
    rho = np.asarray(rho, dtype=np.float64)
    phi_ext = potential_fft(rho, h, green) if method == "fft" else potential_direct(rho, h, green)
    return phi_ext, gradient(phi_ext, h)


def solve_particles(x, y, z, q, n, h=None, origin=None, dtype=np.float64, method="fft", scheme="cic",
                    green="integrated"):
    """Particles (SoA) of charge q each -> field at the particles.

    h=None selects the particle-fitted cubic mesh; otherwise h is a 3-tuple and
    origin defaults to the mesh centred at 0.  scheme selects the assignment
    (ngp, cic, tsc), green the kernel (integrated, point).  Returns a dict with
    Q, rho, phi_ext, E_mesh, E (3 x Np), n_outside, h, origin.
    """
    if h is None:
        hc, origin = fit_mesh(x, y, z, n)
        h = (hc, hc, hc)
    elif origin is None:
        origin = centred_origin(n, h)
    Q, n_out = deposit(x, y, z, q, n, h, origin, dtype, scheme)
    rho = Q / (h[0] * h[1] * h[2])
    phi_ext, E_mesh = solve_rho(rho, h, method, green)
    E = gather(E_mesh, x, y, z, n, h, origin, dtype, scheme)
    return dict(Q=Q, rho=rho, phi_ext=phi_ext, E_mesh=E_mesh, E=E,
                n_outside=n_out, h=tuple(h), origin=tuple(origin))


def potential_at(rho, h, targets):
    """phi at a few target nodes (k, j, i) by the literal sum over all sources.

    Each target costs one pass over the whole mesh; use for sampled checks of
    large meshes.  Offsets may be -1..n (ghost layer).
    """
    nz, ny, nx = rho.shape
    G = igf_octant((nx + 1, ny + 1, nz + 1), h)
    out = []
    kk = np.arange(nz)[:, None, None]
    jj = np.arange(ny)[None, :, None]
    ii = np.arange(nx)[None, None, :]
    for (k, j, i) in targets:
        out.append(np.sum(rho * G[np.abs(kk - k), np.abs(jj - j), np.abs(ii - i)]))
    return COULOMB_K * np.asarray(out)
