"""Seeded synthetic initial states for the MHD update step.

This module only *builds inputs*: it holds none of the scheme's arithmetic and
is shared by the tests (for both the HIP path and the CPU oracle), the
benchmark and the closure data generator.

A state is a float64 numpy array of shape ``(8, nz, ny, nx)`` holding the
conserved fields of the paper's section II.A in the order
``rho, m_x, m_y, m_z, e, b_x, b_y, b_z``.  ``b`` is normalised by sqrt(4 pi)
and ``b_d`` is the flux through the low d-face of each cell (constrained
transport); ``e`` is the total energy density p/(gamma-1) + rho v^2/2 + b^2/2
with the cell-centred field taken as the mean of the two face values.
Grid spacing is h = 1/nx on every axis; cell (i, j, k) spans
[i h, (i+1) h] x [j h, (j+1) h] x [k h, (k+1) h].
"""
import numpy as np

GAMMA = 5.0 / 3.0
RHO, MX, MY, MZ, EN, BX, BY, BZ = range(8)


# --------------------------------------------------------------------------
# coordinates
# --------------------------------------------------------------------------

def centres(n):
    """cell-centre coordinates (x, y, z) broadcastable to (nz, ny, nx)"""
    nx, ny, nz = n
    h = 1.0 / nx
    x = ((np.arange(nx) + 0.5) * h)[None, None, :]
    y = ((np.arange(ny) + 0.5) * h)[None, :, None]
    z = ((np.arange(nz) + 0.5) * h)[:, None, None]
    return x, y, z


def faces(n, d):
    """coordinates of the low d-face centres of every cell"""
    nx, ny, nz = n
    h = 1.0 / nx
    x, y, z = centres(n)
    if d == 0:
        x = (np.arange(nx) * h)[None, None, :]
    elif d == 1:
        y = (np.arange(ny) * h)[None, :, None]
    else:
        z = (np.arange(nz) * h)[:, None, None]
    return x, y, z


def assemble(n, rho, v, p, b, gamma=GAMMA):
    """Build the conserved state on the grid n = (nx, ny, nz) from primitive
    cell-centred rho, v (3), p and face-centred b (3); every array is
    broadcast to (nz, ny, nx)."""
    shape = (n[2], n[1], n[0])
    rho = np.broadcast_to(rho, shape).astype(np.float64)
    p = np.broadcast_to(p, shape).astype(np.float64)
    v = [np.broadcast_to(c, shape).astype(np.float64) for c in v]
    b = [np.broadcast_to(c, shape).astype(np.float64) for c in b]
    s = np.empty((8,) + shape)
    s[RHO] = rho
    for d in range(3):
        s[MX + d] = rho * v[d]
        s[BX + d] = b[d]
    bc2 = sum((0.5 * (b[d] + np.roll(b[d], -1, axis=2 - d))) ** 2 for d in range(3))
    s[EN] = p / (gamma - 1.0) + 0.5 * rho * sum(c * c for c in v) + 0.5 * bc2
    return s


# --------------------------------------------------------------------------
# simple states
# --------------------------------------------------------------------------

def uniform(n, rho=1.0, v=(0.0, 0.0, 0.0), p=1.0, b=(1.0, 0.0, 0.0), gamma=GAMMA):
    nx, ny, nz = n
    one = np.ones((nz, ny, nx))
    return assemble(n, rho * one, [c * one for c in v], p * one, [c * one for c in b], gamma)


def vector_potential_b(n, A):
    """Discrete curl of an edge vector potential: A = (A_x, A_y, A_z) arrays
    on x-, y- and z-edges (A_x[k,j,i] at ((i+1/2)h, j h, k h), etc.).  The
    resulting face fluxes have zero discrete divergence in every cell."""
    nx = n[0]
    h = 1.0 / nx
    Ax, Ay, Az = A

    def dd(a, axis):  # forward difference a[i+1] - a[i] along axis (x=0)
        return np.roll(a, -1, axis=2 - axis) - a

    bx = (dd(Az, 1) - dd(Ay, 2)) / h
    by = (dd(Ax, 2) - dd(Az, 0)) / h
    bz = (dd(Ay, 0) - dd(Ax, 1)) / h
    return bx, by, bz


def random_smooth(n, seed, amp_v=0.15, amp_b=0.15, b0=(0.6, -0.4, 0.5),
                  rho0=1.0, p0=1.0, kmax=1, gamma=GAMMA):
    """Random smooth state: a few Fourier modes in rho, v, p and in an edge
    vector potential, plus a uniform field b0.  Divergence-free b."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    h = 1.0 / nx
    L = (1.0, ny * h, nz * h)

    def field(x, y, z, amp):
        out = np.zeros(np.broadcast_shapes(x.shape, y.shape, z.shape))
        for _ in range(4):
            k = rng.integers(-kmax, kmax + 1, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            a = rng.normal() * amp
            out = out + a * np.sin(2 * np.pi * (k[0] * x / L[0] + k[1] * y / L[1] + k[2] * z / L[2]) + ph)
        return out

    xc, yc, zc = centres(n)
    rho = rho0 * (1.0 + 0.2 * np.tanh(field(xc, yc, zc, 1.0)))
    v = [field(xc, yc, zc, amp_v) for _ in range(3)]
    p = p0 * (1.0 + 0.2 * np.tanh(field(xc, yc, zc, 1.0)))
    # edge positions for the vector potential
    xe = (np.arange(nx) * h)[None, None, :]
    ye = (np.arange(ny) * h)[None, :, None]
    ze = (np.arange(nz) * h)[:, None, None]
    Ax = field(xc, ye, ze, amp_b / (2 * np.pi))
    Ay = field(xe, yc, ze, amp_b / (2 * np.pi))
    Az = field(xe, ye, zc, amp_b / (2 * np.pi))
    shape = (nz, ny, nx)
    Ax, Ay, Az = (np.broadcast_to(a, shape) for a in (Ax, Ay, Az))
    bx, by, bz = vector_potential_b(n, (Ax, Ay, Az))
    b = [bx + b0[0], by + b0[1], bz + b0[2]]
    return assemble(n, rho, v, p, b, gamma)


# --------------------------------------------------------------------------
# linear waves of the ideal-MHD equations
# --------------------------------------------------------------------------

def mhd_jacobian(rho0, p0, B, gamma=GAMMA):
    """Jacobian of the 1D ideal-MHD equations in primitive variables
    W = (rho, v_x, v_y, v_z, p, b_y, b_z), linearised about a state at rest
    with uniform field B = (B_x, B_y, B_z), propagation along x:
    dW/dt + J dW/dx = 0 (equations (1)-(4) of the paper in 1D)."""
    Bx, By, Bz = B
    J = np.zeros((7, 7))
    J[0, 1] = rho0
    J[1, 4] = 1.0 / rho0
    J[1, 5] = By / rho0
    J[1, 6] = Bz / rho0
    J[2, 5] = -Bx / rho0
    J[3, 6] = -Bx / rho0
    J[4, 1] = gamma * p0
    J[5, 1] = By
    J[5, 2] = -Bx
    J[6, 1] = Bz
    J[6, 3] = -Bx
    return J


def wave_mode(mode, rho0, p0, B, gamma=GAMMA):
    """(speed, right eigenvector) of the rightward 'fast', 'alfven' or 'slow'
    mode, normalised so that its largest component is 1."""
    J = mhd_jacobian(rho0, p0, B, gamma)
    lam, R = np.linalg.eig(J)
    lam = lam.real
    R = R.real
    order = np.argsort(-lam)          # fast, alfven, slow, 0, -slow, -alf, -fast
    pick = {"fast": 0, "alfven": 1, "slow": 2}[mode]
    k = order[pick]
    r = R[:, k]
    r = r / r[np.argmax(np.abs(r))]
    return lam[k], r


def linear_wave(n, mode="fast", amp=1e-6, B=(1.0, 0.0, 0.0), rho0=1.0, p0=1.0,
                axis=0, t=0.0, v0=0.0, gamma=GAMMA):
    """Plane wave of amplitude amp along `axis` with wavelength = box length,
    exact solution of the linearised equations at time t.  The background
    field B and the wave are given in the frame (normal, t1, t2) of the axis
    and rotated cyclically onto (x, y, z).  v0 is a uniform background flow
    along the axis (the wave then travels at its speed + v0)."""
    lam, r = wave_mode(mode, rho0, p0, B, gamma)
    lam = lam + v0
    nx, ny, nz = n
    h = 1.0 / nx
    Lax = (nx, ny, nz)[axis] * h

    def phase(coord):
        return amp * np.sin(2 * np.pi * (coord - lam * t) / Lax)

    xc = centres(n)[axis]
    s = phase(xc)
    rho = rho0 + r[0] * s
    p = p0 + r[4] * s
    vloc = [v0 + r[1] * s, r[2] * s, r[3] * s]
    # transverse b components vary along the axis: their faces lie at the
    # cell centre along the axis; the normal component stays uniform
    bloc = [B[0] + 0 * s, B[1] + r[5] * s, B[2] + r[6] * s]
    v = [None] * 3
    b = [None] * 3
    for q in range(3):
        v[(axis + q) % 3] = vloc[q]
        b[(axis + q) % 3] = bloc[q]
    return assemble(n, rho, v, p, b, gamma)


def diagonal_wave(n, mode="fast", amp=1e-6, B=(1.0, 0.6, 0.4), rho0=1.0,
                  p0=1.0, t=0.0, gamma=GAMMA):
    """Linear wave travelling along the diagonal of the x-y plane, wave
    vector k = 2 pi (1/Lx, 1/Ly, 0).  B = (B_par, B_perp, B_z) is the
    background field in the wave frame (along k, in-plane normal to k, z).
    Every sweep then sees all field components vary along its axis.  The
    in-plane perturbation of b comes from a z vector potential on the z-edges,
    so the discrete div b is zero."""
    nx, ny, nz = n
    h = 1.0 / nx
    Lx, Ly = 1.0, ny * h
    kx, ky = 2 * np.pi / Lx, 2 * np.pi / Ly
    kk = np.hypot(kx, ky)
    cth, sth = kx / kk, ky / kk
    lam, r = wave_mode(mode, rho0, p0, B, gamma)
    xc, yc, zc = centres(n)

    def phase(x, y):
        return kx * x + ky * y - kk * lam * t

    sc = amp * np.sin(phase(xc, yc))
    rho = rho0 + r[0] * sc
    p = p0 + r[4] * sc
    vpar, vperp, vz = r[1] * sc, r[2] * sc, r[3] * sc
    v = [vpar * cth - vperp * sth, vpar * sth + vperp * cth, vz + 0 * zc]
    # uniform background on the faces
    b0x = B[0] * cth - B[1] * sth
    b0y = B[0] * sth + B[1] * cth
    # in-plane part from A_z = (amp r5 / |k|) cos(phase) on z-edges
    xe = (np.arange(nx) * h)[None, None, :]
    ye = (np.arange(ny) * h)[None, :, None]
    Az = np.broadcast_to((amp * r[5] / kk) * np.cos(phase(xe, ye)), (nz, ny, nx))
    zero = np.zeros((nz, ny, nx))
    bx, by, _ = vector_potential_b(n, (zero, zero, Az))
    # out-of-plane part: b_z on low z-faces (cell-centred in x and y)
    bz = B[2] + r[6] * amp * np.sin(phase(xc, yc)) + 0 * zc
    return assemble(n, rho, v, p, [bx + b0x, by + b0y, bz], gamma)


def cpaw(n, amp=0.1, B0=1.0, rho0=1.0, p0=0.1, axis=0, t=0.0, gamma=GAMMA):
    """Circularly polarised Alfven wave along `axis`: an exact nonlinear
    solution (|b| and p uniform) travelling at v_A = B0/sqrt(rho0)."""
    nx, ny, nz = n
    h = 1.0 / nx
    Lax = (nx, ny, nz)[axis] * h
    vA = B0 / np.sqrt(rho0)
    xc = centres(n)[axis]
    ph = 2 * np.pi * (xc - vA * t) / Lax
    bt1 = amp * np.sin(ph)
    bt2 = amp * np.cos(ph)
    vloc = [0 * ph, -bt1 / np.sqrt(rho0), -bt2 / np.sqrt(rho0)]
    bloc = [B0 + 0 * ph, bt1, bt2]
    v = [None] * 3
    b = [None] * 3
    for q in range(3):
        v[(axis + q) % 3] = vloc[q]
        b[(axis + q) % 3] = bloc[q]
    return assemble(n, rho0 + 0 * ph, v, p0 + 0 * ph, b, gamma)


# --------------------------------------------------------------------------
# shock tube and benchmark states
# --------------------------------------------------------------------------

def sod(n, axis=0, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), gamma=1.4):
    """Double Sod problem on a periodic box: the left state (rho, v, p) fills
    the middle half along `axis`, the right state the rest; b = 0.  The
    interface at 3/4 of the box is a standard Sod tube."""
    nx, ny, nz = n
    h = 1.0 / nx
    Lax = (nx, ny, nz)[axis] * h
    xc = centres(n)[axis] / Lax
    inside = (xc > 0.25) & (xc < 0.75)
    rho = np.where(inside, left[0], right[0])
    u = np.where(inside, left[1], right[1])
    p = np.where(inside, left[2], right[2])
    v = [0 * xc, 0 * xc, 0 * xc]
    v[axis] = u
    z = 0 * xc
    return assemble(n, rho, v, p, [z, z, z], gamma)


def brio_wu(n, axis=0, gamma=2.0):
    """Double Brio-Wu magnetised shock tube on a periodic box: along `axis`
    the middle half holds rho = 1, p = 1, b_t = +1 and the rest rho = 0.125,
    p = 0.1, b_t = -1, with a uniform normal field b_n = 0.75 and v = 0; b_t
    is the component after `axis` in cyclic order.  b_t varies only along
    `axis`, so the face field is divergence-free exactly."""
    nx, ny, nz = n
    h = 1.0 / nx
    Lax = (nx, ny, nz)[axis] * h
    xc = centres(n)[axis] / Lax
    inside = (xc > 0.25) & (xc < 0.75)
    rho = np.where(inside, 1.0, 0.125)
    p = np.where(inside, 1.0, 0.1)
    z = 0 * xc
    b = [z, z, z]
    b[axis] = z + 0.75
    b[(axis + 1) % 3] = np.where(inside, 1.0, -1.0)
    return assemble(n, rho, [z, z, z], p, b, gamma)


def field_loop(n, amp=1e-3, radius=0.15, v=(1.0, 0.5, 0.0), rho=1.0, p=1.0, gamma=GAMMA):
    """Advected magnetic field loop (a weak-field CT test in the x-y plane):
    the z-edge potential A_z = amp (radius - r) inside the circle of the given
    radius about the middle of the x-y box and 0 outside, b its discrete
    curl (exactly divergence-free, no b_z), uniform rho, p and velocity v.
    With v = (1, 1/2) and a box 1 x 1/2 (ny = nx/2) the loop crosses the
    box diagonally and is back in place at t = 1."""
    nx, ny, nz = n
    h = 1.0 / nx
    xe = (np.arange(nx) * h)[None, None, :]
    ye = (np.arange(ny) * h)[None, :, None]
    r = np.sqrt((xe - 0.5 * nx * h) ** 2 + (ye - 0.5 * ny * h) ** 2)
    Az = np.broadcast_to(np.where(r < radius, amp * (radius - r), 0.0), (nz, ny, nx))
    z = np.zeros((nz, ny, nx))
    b = vector_potential_b(n, (z, z, Az))
    return assemble(n, rho, [np.full((nz, ny, nx), c) for c in v], p, list(b), gamma)


def solenoidal_velocity(n, seed, kmin=1, kmax=8, slope=-4.0):
    """Gaussian random-phase solenoidal velocity field with per-mode power
    |v_k|^2 proportional to k^slope for integer |k| in [kmin, kmax], unit rms.
    Built on the half spectrum of a real transform (kx >= 0)."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    kx = np.fft.rfftfreq(nx, 1.0 / nx)[None, None, :]
    ky = np.fft.fftfreq(ny, 1.0 / ny)[None, :, None] * (nx / ny)
    kz = np.fft.fftfreq(nz, 1.0 / nz)[:, None, None] * (nx / nz)
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    kint = np.rint(kk)
    mask = (kint >= kmin) & (kint <= kmax)
    amp = np.where(mask, np.maximum(kk, 1e-30) ** (slope / 2.0), 0.0).astype(np.float32)
    shape = kk.shape
    vk = [amp * (rng.standard_normal(shape, dtype=np.float32)
                 + 1j * rng.standard_normal(shape, dtype=np.float32)) for _ in range(3)]
    # project out the component along k
    inv = np.where(kk > 0, 1.0 / np.maximum(kk, 1e-30) ** 2, 0.0).astype(np.float32)
    kv = (kx * vk[0] + ky * vk[1] + kz * vk[2]) * inv
    vk = [vk[0] - kx * kv, vk[1] - ky * kv, vk[2] - kz * kv]
    try:                               # threaded FFT when scipy is present
        import scipy.fft as sfft
        v = [sfft.irfftn(c, s=(nz, ny, nx), workers=-1).astype(np.float64) for c in vk]
    except ImportError:
        v = [np.fft.irfftn(c, s=(nz, ny, nx)).astype(np.float64) for c in vk]
    rms = np.sqrt(np.mean(v[0] ** 2 + v[1] ** 2 + v[2] ** 2))
    return [c / rms for c in v]


def turbulence(n, seed=2, mach=1.0, beta=1.0, rho0=1.0, p0=1.0, gamma=GAMMA):
    """Random-phase solenoidal velocity (P(k) ~ k^-4, 1 <= k <= 8) scaled to
    rms Mach `mach` with c_s = sqrt(gamma p0/rho0); uniform rho and p; a
    uniform field along z with plasma beta = 2 p0 / B0^2."""
    nx, ny, nz = n
    v = solenoidal_velocity(n, seed)
    cs = np.sqrt(gamma * p0 / rho0)
    v = [c * (mach * cs) for c in v]
    B0 = np.sqrt(2.0 * p0 / beta)
    one = np.ones((nz, ny, nx))
    return assemble(n, rho0 * one, v, p0 * one, [0 * one, 0 * one, B0 * one], gamma)


def orszag_tang(n, gamma=GAMMA):
    """3D Orszag-Tang-type state: v = (-sin 2 pi y, sin 2 pi x, 0.1 sin 2 pi z),
    b = (-sin 2 pi y, sin 4 pi x, 0)/sqrt(4 pi), rho = 25/(36 pi),
    p = 5/(12 pi).  Each b component is constant along its own axis, so the
    discrete div b vanishes."""
    xc, yc, zc = centres(n)
    s4p = np.sqrt(4.0 * np.pi)
    v = [-np.sin(2 * np.pi * yc) + 0 * xc + 0 * zc,
         np.sin(2 * np.pi * xc) + 0 * yc + 0 * zc,
         0.1 * np.sin(2 * np.pi * zc) + 0 * xc + 0 * yc]
    xb, yb, zb = faces(n, 0)
    bx = -np.sin(2 * np.pi * yb) / s4p + 0 * xb + 0 * zb
    xb, yb, zb = faces(n, 1)
    by = np.sin(4 * np.pi * xb) / s4p + 0 * yb + 0 * zb
    bz = 0 * xc + 0 * yc + 0 * zc
    rho = 25.0 / (36.0 * np.pi)
    p = 5.0 / (12.0 * np.pi)
    return assemble(n, rho + 0 * xc, v, p + 0 * xc, [bx, by, bz], gamma)


ENSEMBLE_SIZES = (32, 48, 64, 96, 128, 192, 256)


def ensemble_spec(nbox=64, seed=4, sizes=ENSEMBLE_SIZES):
    """Per-box (n, mach, beta, seed) of the uneven ensemble: n drawn from
    `sizes`, Mach uniform in [0.5, 3], beta log-uniform in [0.1, 10]."""
    rng = np.random.default_rng(seed)
    spec = []
    for b in range(nbox):
        n = int(rng.choice(sizes))
        mach = float(rng.uniform(0.5, 3.0))
        beta = float(10 ** rng.uniform(-1.0, 1.0))
        spec.append((n, mach, beta, seed * 1000 + b))
    return spec


# --------------------------------------------------------------------------
# device-side generation (torch) for grids too large to build on the host
# --------------------------------------------------------------------------

def orszag_tang_phases(seed):
    """random phase shifts (5 numbers in [0, 1)) of an Orszag-Tang-family
    member; seed 0 gives the unshifted state"""
    if seed == 0:
        return np.zeros(5)
    return np.random.default_rng(seed).uniform(0.0, 1.0, 5)


def orszag_tang_torch(n, seed=0, dtype=None, device="cuda", gamma=GAMMA):
    """The Orszag-Tang-type state of `orszag_tang`, with each sine shifted by
    a seeded phase (b_x(y), b_y(x) keep depending only on the transverse
    coordinate, so div b = 0 exactly), built directly in device memory as a
    torch tensor of shape (8, nz, ny, nx)."""
    import torch
    dtype = dtype or torch.float32
    nx, ny, nz = n
    h = 1.0 / nx
    ph = orszag_tang_phases(seed)
    tp = 2.0 * np.pi
    ar = lambda m, off: (torch.arange(m, device=device, dtype=torch.float64) + off) * h
    xc = ar(nx, 0.5).view(1, 1, nx)
    yc = ar(ny, 0.5).view(1, ny, 1)
    zc = ar(nz, 0.5).view(nz, 1, 1)
    rho = 25.0 / (36.0 * np.pi)
    p = 5.0 / (12.0 * np.pi)
    s4p = np.sqrt(4.0 * np.pi)
    out = torch.empty((8, nz, ny, nx), dtype=dtype, device=device)
    vx = -torch.sin(tp * (yc + ph[0]))
    vy = torch.sin(tp * (xc + ph[1]))
    vz = 0.1 * torch.sin(tp * (zc + ph[2]))
    bx = -torch.sin(tp * (yc + ph[3])) / s4p          # on x-faces, function of y
    by = torch.sin(2 * tp * (xc + ph[4])) / s4p       # on y-faces, function of x
    # cell-centred field = mean of the two faces along each axis: b_x and b_y
    # are constant along their own axis, so the mean equals the face value
    out[0] = rho
    out[1] = rho * vx
    out[2] = rho * vy
    out[3] = rho * vz
    ke = 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    out[4] = p / (gamma - 1.0) + ke + 0.5 * (bx * bx + by * by)
    out[5] = bx
    out[6] = by
    out[7] = 0.0
    return out
