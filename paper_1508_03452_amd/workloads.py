"""Seeded synthetic initial conditions shaped like the paper's runs.

This module only builds primitive fields (n, p, u, E, B, rho_c) and run
parameters.  It holds none of the lattice Boltzmann arithmetic, so both the
HIP library's callers and the oracle-based tests can use it.

All arrays are float64 numpy arrays of shape (nz, ny, nx); cell centres are
x_i = (i + 1/2 - N/2) dx in lattice units (dx = c = 1 unless stated).

Workloads (Sec. IV of the paper; sizes and seeds are this project's):
  alfven   -- small-amplitude Alfven wave on a periodic 256x4x4 box, ideal
              limit (sigma = 1e6), initial E from ideal Ohm's law (Eq. Ohm_ideal).
  sheet    -- self-similar resistive current sheet, 1024x4x4, x open,
              p = 50, B_y = erf(x / 2) (the erf profile of Eq. Current_sheet at
              the time where its width is two cells).
  kh       -- Kelvin-Helmholtz-driven reconnection slab, 1024x2048x1, x
              periodic, y open; tanh shear layer, antiparallel B_x, seeded
              transverse velocity noise.
  flare    -- 3-D flare-like box 256x256x512: quadrupole arcade plus a
              flux rope (Sec. IV, stellar flare), stratified density,
              seeded rope height, a driven shearing bottom face and open
              faces elsewhere.
  random   -- smooth random periodic state for parity tests.
"""
from dataclasses import dataclass, field
from math import erf, sqrt

import numpy as np

DEFAULT_PARAMS = dict(dx=1.0, c=1.0, mu0=1.0, tau=1.0, tau_h=0.5, alpha=0.1, Gamma=4.0 / 3.0, sigma=1.0,
                      nu=27.0 ** 0.5, divb_fix=0, null_band=64, collision=0, flux=0, b_prev=0)


@dataclass
class Workload:
    name: str
    shape: tuple           # (nx, ny, nz)
    bc: tuple              # ((lo, hi),) * 3 with "periodic" / "open" / "driven" (low z only)
    params: dict
    fields: dict           # n, p, u (3), E (3), B (3), rho_c (array or None)
    steps: int = 0
    meta: dict = field(default_factory=dict)
    driven: dict = None    # prescribed fields of a driven low-z face: n, p, u (3), B (3), each (ny, nx)
    force: tuple = None    # external force density ((Fx, Fy, Fz), gate), or None

    @property
    def ncells(self):
        nx, ny, nz = self.shape
        return nx * ny * nz


def _centres(n, dx=1.0):
    return (np.arange(n, dtype=np.float64) + 0.5 - n / 2.0) * dx


def _grid(shape, dx=1.0):
    nx, ny, nz = shape
    x = _centres(nx, dx)[None, None, :]
    y = _centres(ny, dx)[None, :, None]
    z = _centres(nz, dx)[:, None, None]
    return x, y, z


def _full(shape, v):
    nx, ny, nz = shape
    return np.full((nz, ny, nx), float(v))


def _params(**kw):
    d = dict(DEFAULT_PARAMS)
    d.update(kw)
    return d


PERIODIC3 = (("periodic", "periodic"),) * 3
KH_BC = (("periodic", "periodic"), ("open", "open"), ("periodic", "periodic"))


def alfven(nx=256, ny=4, nz=4, amp=0.01, sigma=1e6, steps=500):
    """Linear relativistic Alfven wave along a uniform B0 = 1 (n = p = 1)."""
    shape = (nx, ny, nz)
    x, _, _ = _grid(shape)
    Gamma = 4.0 / 3.0
    eps = 1.0 + 1.0 / (Gamma - 1.0)
    vA = 1.0 / sqrt(eps + 1.0 + 1.0)           # B0^2 / (eps + p + B0^2), B0 = 1
    s = np.broadcast_to(np.sin(2 * np.pi * (x + nx / 2.0) / nx), (nz, ny, nx)).copy()
    By = amp * s
    uy = -vA * amp * s
    zero = _full(shape, 0.0)
    u = (zero, uy, zero.copy())
    B = (_full(shape, 1.0), By, zero.copy())
    E = (zero.copy(), zero.copy(), uy.copy())   # E = -u x B with u = (0, u_y, 0), B = (1, B_y, 0)
    fields = dict(n=_full(shape, 1.0), p=_full(shape, 1.0), u=u, E=E, B=B, rho_c=_full(shape, 0.0))
    return Workload("alfven", shape, PERIODIC3, _params(sigma=sigma), fields, steps,
                    meta=dict(vA=vA, amp=amp, k=2 * np.pi / nx))


def sheet(nx=1024, ny=4, nz=4, sigma=100.0, p=50.0, steps=4000, width_cells=2.0):
    """Resistive current sheet: B_y = erf(x / width), rest frame, E = 0."""
    shape = (nx, ny, nz)
    x, _, _ = _grid(shape)
    t0 = sigma * (width_cells / 2.0) ** 2        # erf(x / (2 sqrt(t0 / sigma))) has that width
    By = np.broadcast_to(np.vectorize(erf)(x / (2.0 * np.sqrt(t0 / sigma))), (nz, ny, nx)).copy()
    zero = _full(shape, 0.0)
    fields = dict(n=_full(shape, 1.0), p=_full(shape, p), u=(zero, zero.copy(), zero.copy()),
                  E=(zero.copy(), zero.copy(), zero.copy()), B=(zero.copy(), By, zero.copy()),
                  rho_c=zero.copy())
    bc = (("open", "open"), ("periodic", "periodic"), ("periodic", "periodic"))
    return Workload("sheet", shape, bc, _params(sigma=sigma), fields, steps, meta=dict(t0=t0))


def alfven_box(n_cells=400, eta=0.118591, sigma=1e5, B0=1.0, By=0.1, x0=-0.8, x1=0.0, Gamma=4.0 / 3.0):
    """The Alfven-wave set-up of Sec. IV in the paper's units: [-1, 1] in n_cells cells, c = 1
    (dx / dt = sqrt 2), open ends, n = p = 1, B = (B0, By, B_z) with B_z = eta B0 sin(2 pi (3 s^2 - 2 s^3)),
    s = (x - x0) / (x1 - x0), inside (x0, x1) and 0 outside, u_z = -v_A B_z / B0 there, ideal-Ohm
    E = -u x B and rho_c from Gauss's law (None: the solver takes eps0 div E).  meta: v_A from the
    exact-wave formula of that section, the grid x, dt and the initial B_z."""
    shape = (n_cells, 1, 1)
    dx = 2.0 / n_cells
    x, _, _ = _grid(shape, dx)
    xs = x.ravel()
    eps = 1.0 + 1.0 / (Gamma - 1.0)                  # n c^2 + p / (Gamma - 1) with n = p = c = 1
    den = eps + 1.0 + B0 * B0 * (1.0 + eta * eta)
    vA = np.sqrt(2.0 * B0 * B0 / den / (1.0 + np.sqrt(1.0 - (2.0 * eta * B0 * B0 / den) ** 2)))
    sarg = (xs - x0) / (x1 - x0)
    inside = (xs > x0) & (xs < x1)
    Bz1 = np.where(inside, eta * B0 * np.sin(2.0 * np.pi * (3.0 * sarg ** 2 - 2.0 * sarg ** 3)), 0.0)
    uz1 = -vA / B0 * Bz1
    Bz = Bz1.reshape(1, 1, n_cells).copy()
    uz = uz1.reshape(1, 1, n_cells).copy()
    zero = _full(shape, 0.0)
    Bx, Byf = _full(shape, B0), _full(shape, By)
    # E = -u x B with u = (0, 0, u_z): E = (u_z B_y, -u_z B_x, 0)
    E = (uz * Byf, -uz * Bx, zero.copy())
    fields = dict(n=_full(shape, 1.0), p=_full(shape, 1.0), u=(zero.copy(), zero.copy(), uz),
                  E=E, B=(Bx, Byf, Bz), rho_c=None)
    bc = (("open", "open"), ("periodic", "periodic"), ("periodic", "periodic"))
    return Workload("alfven_box", shape, bc, _params(sigma=sigma, dx=dx, Gamma=Gamma), fields, 0,
                    meta=dict(vA=float(vA), x=xs.copy(), dt=dx / np.sqrt(2.0), Bz0=Bz1.copy(), x0=x0, x1=x1,
                              eta=eta, B0=B0))


def sheet_box(n_cells=100, sigma=100.0, t_start=1.0, p=50.0, half_width=1.5):
    """The current-sheet set-up of Sec. IV (self-similar current sheets) in the paper's units: the
    segment [-half_width, half_width] in n_cells cells (dx = 2 half_width / n_cells), c = 1 so that
    dx / dt = sqrt(2), open ends, B_y = erf(sqrt(sigma / t_start) x / 2) (B0 = 1), n = 1, p = 50,
    u = E = 0.  meta['t_start'] is the time the initial profile belongs to."""
    shape = (n_cells, 1, 1)
    dx = 2.0 * half_width / n_cells
    x, _, _ = _grid(shape, dx)
    By = np.vectorize(erf)(0.5 * np.sqrt(sigma / t_start) * x).reshape(1, 1, n_cells).copy()
    zero = _full(shape, 0.0)
    fields = dict(n=_full(shape, 1.0), p=_full(shape, p), u=(zero, zero.copy(), zero.copy()),
                  E=(zero.copy(), zero.copy(), zero.copy()), B=(zero.copy(), By, zero.copy()),
                  rho_c=zero.copy())
    bc = (("open", "open"), ("periodic", "periodic"), ("periodic", "periodic"))
    return Workload("sheet_box", shape, bc, _params(sigma=sigma, dx=dx), fields, 0,
                    meta=dict(t_start=t_start, dt=dx / np.sqrt(2.0), x=x.ravel().copy()))


def kh_box(n_cells=512, U0=0.2, dn=1.8, sigma=100.0, B0=0.06, u_pert=0.01, c=2.5, null_band=8):
    """The KH reconnection set-up of Sec. IV in the paper's units: [-0.5, 0.5]^2 in n_cells^2 cells,
    dx / dt = sqrt(2) c with c = 2.5, x periodic, y open; u_x = (U0 c / 2) tanh(y / a) with a = dx,
    n = 1 + (dn / 2) tanh(y / a), p = 1, B_x = B0 tanh(y / a), single-mode u_y =
    u_pert sin(2 pi x) exp(-y^2 / b^2) with b = 10 dx, ideal-Ohm E = -u x B.  U0 is in units of c.
    The null point is searched in the rows within null_band cells of y = 0."""
    shape = (n_cells, n_cells, 1)
    dx = 1.0 / n_cells
    x, y, _ = _grid(shape, dx)
    a, b = dx, 10.0 * dx
    th = np.broadcast_to(np.tanh(y / a), (1, n_cells, n_cells)).copy()
    ux = 0.5 * U0 * c * th
    uy = np.broadcast_to(u_pert * np.sin(2.0 * np.pi * x) * np.exp(-(y / b) ** 2), (1, n_cells, n_cells)).copy()
    n = 1.0 + 0.5 * dn * th
    Bx = B0 * th
    zero = _full(shape, 0.0)
    # E = -u x B with u = (u_x, u_y, 0), B = (B_x, 0, 0): E = (0, 0, u_y B_x)
    fields = dict(n=n, p=_full(shape, 1.0), u=(ux, uy, zero.copy()), E=(zero.copy(), zero.copy(), uy * Bx),
                  B=(Bx, zero.copy(), zero.copy()), rho_c=zero.copy())
    return Workload("kh_box", shape, KH_BC, _params(sigma=sigma, dx=dx, c=c, null_band=null_band), fields, 0,
                    meta=dict(U0=U0, dn=dn, B0=B0, dt=dx / (np.sqrt(2.0) * c)))


def kh(nx=1024, ny=2048, nz=1, v0=0.2, ratio=10.0, sigma=1e3, B0=0.1, noise=1e-3, seed=2015, a=1.0, b=10.0,
       steps=20000):
    """Kelvin-Helmholtz shear layer with an antiparallel field (Sec. IV, KH)."""
    shape = (nx, ny, nz)
    _, y, _ = _grid(shape)
    rng = np.random.Generator(np.random.PCG64(seed))
    th = np.broadcast_to(np.tanh(y / a), (nz, ny, nx)).copy()
    dn = 2.0 * (ratio - 1.0) / (ratio + 1.0)
    n = 1.0 + 0.5 * dn * th
    ux = v0 * th
    uy = noise * rng.uniform(-1.0, 1.0, size=(nz, ny, nx)) * np.exp(-(y / b) ** 2)
    zero = _full(shape, 0.0)
    Bx = B0 * th
    fields = dict(n=n, p=_full(shape, 1.0), u=(ux, uy, zero.copy()), E=(zero.copy(), zero.copy(), uy * Bx),
                  B=(Bx, zero.copy(), zero.copy()), rho_c=zero.copy())
    return Workload("kh", shape, KH_BC, _params(sigma=sigma), fields, steps, meta=dict(v0=v0, ratio=ratio, B0=B0))


def flare(nx=256, ny=256, nz=512, sigma=1e3, B0=0.06, seed=512, steps=10000, Lx=6.0, Lz=12.0, v_drive=0.1):
    """Flare-like 3-D box: quadrupole arcade + image current + flux rope.

    Flux function psi = psi_b + psi_i + psi_l (Sec. IV, stellar flare) in the
    x-z plane, B = curl(psi e_y), scaled so that max |B| = B0, with a
    uniform-twist axial B_y inside the rope.  The rope height is drawn from
    U[1.8, 2.2] with the seed.  Density n = max(0.05, exp(-z/2)), p = 1,
    u = 0, E = 0.  Physical box [-Lx/2, Lx/2]^2 x [0, Lz].  The bottom face is
    driven (ghost planes at the fields of the first plane with the shear
    u_x = v_drive tanh(y / 0.5) sin^2(pi (x + Lx/2) / Lx) (1 + 1e-3 U[-1, 1]),
    same seed); the other faces are open.  The sin^2 window takes the drive
    to zero at the x faces, as the paper's flare force vanishes at the side
    faces: a drive that pushes the fluid through an open (copy) face grows B
    without bound at that corner of the bottom plane.
    """
    shape = (nx, ny, nz)
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.uniform(1.8, 2.2)
    r0, cb = 0.5, 0.2534
    hphys = Lx / nx
    xs = (np.arange(nx) + 0.5) * hphys - Lx / 2.0
    zs = (np.arange(nz) + 0.5) * (Lz / nz)

    def psi(X, Z):
        pb = cb * np.log(((X + 0.3) ** 2 + (Z + 0.3) ** 2) * ((X - 0.3) ** 2 + (Z + 0.3) ** 2) /
                         (((X + 1.5) ** 2 + (Z + 0.3) ** 2) * ((X - 1.5) ** 2 + (Z + 0.3) ** 2)))
        pi_ = -r0 / 2.0 * np.log(X ** 2 + (Z + h) ** 2)
        r = np.sqrt(X ** 2 + (Z - h) ** 2)
        pl = np.where(r <= r0, r ** 2 / (2 * r0), r0 / 2 - r0 * np.log(r0) + r0 * np.log(np.maximum(r, 1e-300)))
        return pb + pi_ + pl

    X, Z = np.meshgrid(xs, zs, indexing="xy")        # (nz, nx)
    d = 1e-4
    # B = curl(psi e_y) = (-d psi/dz, 0, d psi/dx)
    bx = -(psi(X, Z + d) - psi(X, Z - d)) / (2 * d)
    bz = (psi(X + d, Z) - psi(X - d, Z)) / (2 * d)
    bmax = np.sqrt(bx ** 2 + bz ** 2).max()
    scale = B0 / bmax
    r = np.sqrt(X ** 2 + (Z - h) ** 2)
    by = np.where(r <= r0, scale * np.sqrt(np.maximum(2.0 * (1.0 - r ** 2 / r0 ** 2), 0.0)), 0.0)
    Bx = np.broadcast_to((bx * scale)[:, None, :], (nz, ny, nx)).copy()
    Bz = np.broadcast_to((bz * scale)[:, None, :], (nz, ny, nx)).copy()
    By = np.broadcast_to(by[:, None, :], (nz, ny, nx)).copy()
    n = np.broadcast_to(np.maximum(0.05, np.exp(-zs / 2.0))[:, None, None], (nz, ny, nx)).copy()
    zero = _full(shape, 0.0)
    fields = dict(n=n, p=_full(shape, 1.0), u=(zero, zero.copy(), zero.copy()),
                  E=(zero.copy(), zero.copy(), zero.copy()), B=(Bx, By, Bz), rho_c=zero.copy())
    # driven photosphere: shear u_x = v_drive tanh(y / 0.5) (1 + 1e-3 U[-1, 1]) below the first plane,
    # with the density, pressure and field of that plane
    ys = (np.arange(ny) + 0.5) * (Lx / ny) - Lx / 2.0
    jitter = 1.0 + 1e-3 * rng.uniform(-1.0, 1.0, size=(ny, nx))
    window = np.sin(np.pi * (xs + Lx / 2.0) / Lx) ** 2
    ux = v_drive * np.tanh(ys / 0.5)[:, None] * window[None, :] * jitter
    fz = np.zeros((ny, nx))
    driven = dict(n=n[0].copy(), p=np.ones((ny, nx)), u=(ux, fz, fz.copy()),
                  B=(Bx[0].copy(), By[0].copy(), Bz[0].copy()))
    bc = (("open", "open"), ("open", "open"), ("driven", "open"))
    return Workload("flare", shape, bc, _params(sigma=sigma), fields, steps, meta=dict(h=h, B0=B0, v_drive=v_drive),
                    driven=driven)


def flare_box(n=256, nz=None, sigma=100.0, B0=0.06, h=2.0, F0=0.05, gate=0.3, c=2.5):
    """The stellar-flare set-up of Sec. IV in the paper's units: [-3, 3]^2 x [0, 6] in n x n x nz cells
    (nz = n by default), c = 2.5 (dx / dt = 2.5 sqrt 2), all faces open, n = p = 1, u = 0, B = curl(psi e_y)
    scaled to max |B| = B0 plus the rope's B^y (flux rope at height h), and the external force of that
    section: F^x = F0 sin(pi x* / 3) cos(pi y / 6), F^y = F0 cos(pi x* / 3) sin(pi y / 6) in the two
    sub-boxes z <= 0.2343 (x* = x for x < 0, x - 3 for x >= 0), acting while the largest |beta| is below
    gate.  The paper obtains the initial E and J by iterating the code at fixed B and u; with u = 0 that
    iteration converges to the steady resistive balance J = curl B / mu0, E = J / sigma, which is used
    directly (central differences)."""
    nz = n if nz is None else nz
    shape = (n, n, nz)
    dx = 6.0 / n
    xs = (np.arange(n) + 0.5) * dx - 3.0
    ys = xs.copy()
    zs = (np.arange(nz) + 0.5) * dx
    r0, cb = 0.5, 0.2534

    def psi(X, Z):
        pb = cb * np.log(((X + 0.3) ** 2 + (Z + 0.3) ** 2) * ((X - 0.3) ** 2 + (Z + 0.3) ** 2) /
                         (((X + 1.5) ** 2 + (Z + 0.3) ** 2) * ((X - 1.5) ** 2 + (Z + 0.3) ** 2)))
        pi_ = -r0 / 2.0 * np.log(X ** 2 + (Z + h) ** 2)
        r = np.sqrt(X ** 2 + (Z - h) ** 2)
        pl = np.where(r <= r0, r ** 2 / (2 * r0), r0 / 2 - r0 * np.log(r0) + r0 * np.log(np.maximum(r, 1e-300)))
        return pb + pi_ + pl

    X, Z = np.meshgrid(xs, zs, indexing="xy")        # (nz, nx)
    d = 1e-4
    bx = -(psi(X, Z + d) - psi(X, Z - d)) / (2 * d)
    bz = (psi(X + d, Z) - psi(X - d, Z)) / (2 * d)
    scale = B0 / np.sqrt(bx ** 2 + bz ** 2).max()
    r = np.sqrt(X ** 2 + (Z - h) ** 2)
    by = np.where(r <= r0, scale * np.sqrt(np.maximum(2.0 * (1.0 - r ** 2 / r0 ** 2), 0.0)), 0.0)
    Bx = np.broadcast_to((bx * scale)[:, None, :], (nz, n, n)).copy()
    By = np.broadcast_to(by[:, None, :], (nz, n, n)).copy()
    Bz = np.broadcast_to((bz * scale)[:, None, :], (nz, n, n)).copy()
    # J = curl B (mu0 = 1) by central differences (one-sided on the faces); the fields vary in x and z only
    gx = lambda f: np.gradient(f, dx, axis=2)
    gz = lambda f: np.gradient(f, dx, axis=0)
    Jx = -gz(By)
    Jy = gz(Bx) - gx(Bz)
    Jz = gx(By)
    zero = _full(shape, 0.0)
    fields = dict(n=_full(shape, 1.0), p=_full(shape, 1.0), u=(zero, zero.copy(), zero.copy()),
                  E=(Jx / sigma, Jy / sigma, Jz / sigma), B=(Bx, By, Bz), rho_c=None)
    Xc = xs[None, None, :]
    Yc = ys[None, :, None]
    xstar = np.where(Xc < 0.0, Xc, Xc - 3.0)
    band = (zs <= 0.2343)[:, None, None]
    Fx = np.broadcast_to(np.where(band, F0 * np.sin(np.pi * xstar / 3.0) * np.cos(np.pi * Yc / 6.0), 0.0),
                         (nz, n, n)).copy()
    Fy = np.broadcast_to(np.where(band, F0 * np.cos(np.pi * xstar / 3.0) * np.sin(np.pi * Yc / 6.0), 0.0),
                         (nz, n, n)).copy()
    bc = (("open", "open"),) * 3
    return Workload("flare_box", shape, bc, _params(sigma=sigma, dx=dx, c=c), fields, 0,
                    meta=dict(h=h, B0=B0, F0=F0, dt=dx / (np.sqrt(2.0) * c)), force=((Fx, Fy, zero.copy()), gate))


def random_state(shape=(8, 8, 8), seed=0, vmax=0.3, amp=0.05, Bmag=0.3, Emag=0.05, sigma=10.0, modes=3,
                 bc=PERIODIC3, solenoidal=False, **params):
    """Smooth random state: a few random Fourier modes per field.  With
    solenoidal=True, B = Bmag x + curl of random vector-potential modes
    (divergence free) and E = -u x B (ideal Ohm)."""
    nx, ny, nz = shape
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, z = _grid(shape)
    X = (x + nx / 2.0) / nx
    Y = (y + ny / 2.0) / ny
    Z = (z + nz / 2.0) / nz

    def smooth(scale):
        f = np.zeros((nz, ny, nx))
        for _ in range(modes):
            k = rng.integers(0, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            f = f + rng.uniform(-1, 1) * np.cos(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
        return scale * f / modes

    n = 1.0 + smooth(amp * 4)
    p = 1.0 + smooth(amp * 4)
    u = [smooth(vmax) for _ in range(3)]
    B = [smooth(Bmag) + (Bmag if a == 0 else 0.0) for a in range(3)]
    E = [smooth(Emag) for _ in range(3)]
    rho_c = smooth(0.01)
    if solenoidal:
        B = [np.full((nz, ny, nx), float(Bmag)), np.zeros((nz, ny, nx)), np.zeros((nz, ny, nx))]
        for _ in range(modes):
            k = 2 * np.pi * rng.integers(1, 3, size=3) / np.array([nx, ny, nz], dtype=np.float64)
            a = rng.normal(size=3)
            ph = rng.uniform(0, 2 * np.pi)
            s = -np.sin(k[0] * (x + nx / 2.0) + k[1] * (y + ny / 2.0) + k[2] * (z + nz / 2.0) + ph)
            kxa = np.cross(k, a)
            for c in range(3):
                B[c] = B[c] + (Bmag / modes) * s * kxa[c]
        uv = np.stack(u, -1)
        E = list(np.moveaxis(-np.cross(uv, np.stack(B, -1)), -1, 0))
        rho_c = None
    fields = dict(n=n, p=p, u=tuple(u), E=tuple(np.ascontiguousarray(e) for e in E), B=tuple(B), rho_c=rho_c)
    return Workload("random", tuple(shape), bc, _params(sigma=sigma, **params), fields, 0)


def sweep_specs(n=64, seed=64, sizes=tuple(range(256, 1025, 64))):
    """Parameters of a batched KH sweep: per instance nx, ny uniform on `sizes`, sigma = 10^U[2, 5],
    v0 ~ U[0.05, 0.4], density ratio ~ U[1, 10], noise seed from the sweep seed.  Returns a list of
    dicts (nx, ny, sigma, v0, ratio, seed); fields come from kh() with these."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        out.append(dict(nx=int(rng.choice(sizes)), ny=int(rng.choice(sizes)), sigma=float(10.0 ** rng.uniform(2, 5)),
                        v0=float(rng.uniform(0.05, 0.4)), ratio=float(rng.uniform(1.0, 10.0)),
                        seed=int(rng.integers(0, 2 ** 31 - 1))))
    return out


def sweep_layout(spec):
    """(shape, bc, params) of a sweep instance, as kh() builds them, without its fields."""
    return (spec["nx"], spec["ny"], 1), KH_BC, _params(sigma=spec["sigma"])


def sweep_instance(spec):
    """The KH slab of one sweep instance."""
    return kh(nx=spec["nx"], ny=spec["ny"], v0=spec["v0"], ratio=spec["ratio"], sigma=spec["sigma"], seed=spec["seed"])


def mlp_init(seed=2024, n_in=6, n_h=32, n_out=2):
    """Initial weights of the learned recovery guess (uniform Glorot scale, zero biases), drawn here so
    that the library and the tests start from the same numbers.  Order: W1 (n_h x n_in), b1,
    W2 (n_h x n_h), b2, W3 (n_out x n_h), b3, flattened row-major."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for fan_in, fan_out in ((n_in, n_h), (n_h, n_h), (n_h, n_out)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        out.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        out.append(np.zeros(fan_out))
    return np.concatenate(out)


CONFIGS = {
    "alfven": alfven,
    "sheet": sheet,
    "kh": kh,
    "flare": flare,
}
