"""Seeded synthetic inputs for FSLBM runs: fill-level fields and obstacle masks.

This module only builds input arrays (volume fractions of simple bodies,
wall layers and a counter-based noise field). It holds none of the method's
arithmetic, so the CPU reference and the GPU library both consume exactly the
same arrays.

Layout of every field: numpy array of shape (nz, ny, nx), x fastest, i.e. the
linear cell index is x + nx*(y + ny*z). Cell (i, j, k) covers the unit box
[i, i+1] x [j, j+1] x [k, k+1] in cell-corner coordinates.

Fill levels follow the paper's definition of the fill level as the liquid
volume fraction of a cell (Sec. II). The paper initialises them by refining
each cell 100 times per axis (Sec. III.A.1); here the fractions are computed
by integrating the slice area of the body in closed form and the slice
position by Gauss-Legendre quadrature split at the slice-area kinks, which is
accurate to about 1e-9.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "sphere_fraction",
    "ellipsoid_fraction",
    "cylinder_fraction",
    "splitmix_uniform",
    "perturb_interface",
    "droplet",
    "bubble_probe",
    "sessile_droplet",
    "ellipsoid_droplet",
    "flat_film",
    "advected_bubble",
    "advection_errors",
    "lattice_units",
    "laplace_bubble",
    "renardy_units",
    "sessile_cap",
]

_GL_X, _GL_W = np.polynomial.legendre.leggauss(12)


def _chord_integral(a, b, r):
    """Integral of 2*sqrt(r^2 - x^2) over [a, b] with a, b clipped to [-r, r]."""
    def prim(x):
        xc = np.clip(x, -r, r)
        s = np.sqrt(np.maximum(r * r - xc * xc, 0.0))
        t = np.arcsin(np.clip(xc / np.maximum(r, 1e-300), -1.0, 1.0))
        return xc * s + r * r * t
    return prim(b) - prim(a)


def _quadrant_area(X, Y, r):
    """Area of {x <= X, y <= Y, x^2 + y^2 <= r^2} in closed form (vectorised).

    With s(x) = sqrt(r^2 - x^2), the column at abscissa x contributes the
    length max(0, min(Y, s) + s). For |Y| < r the columns split at
    |x| = xb = sqrt(r^2 - Y^2): where |x| >= xb the column is either the full
    chord (Y >= 0) or empty (Y < 0); where |x| < xb it is Y + s.
    """
    X, Y, r = np.broadcast_arrays(np.asarray(X, np.float64), np.asarray(Y, np.float64),
                                  np.asarray(r, np.float64))
    Xc = np.clip(X, -r, r)
    xb = np.sqrt(np.maximum(r * r - Y * Y, 0.0))
    full = _chord_integral(-r, Xc, r)
    # middle band |x| < xb: integral of (Y + s) over [-xb, min(Xc, xb)]
    hi = np.minimum(Xc, xb)
    w = np.maximum(hi - (-xb), 0.0)
    band = np.where(w > 0, Y * w + 0.5 * _chord_integral(-xb, np.maximum(hi, -xb), r), 0.0)
    # outer columns (|x| >= xb) with Y >= 0 carry the full chord
    outer = _chord_integral(-r, np.minimum(Xc, -xb), r) + np.where(
        Xc > xb, _chord_integral(xb, np.maximum(Xc, xb), r), 0.0)
    inside = np.abs(Y) < r
    res = np.where(Y >= r, full, np.where(inside, band + np.where(Y >= 0, outer, 0.0), 0.0))
    return np.where(r > 0, res, 0.0)


def _rect_disc_area(x0, x1, y0, y1, r):
    """Area of the disc of radius r (centre 0) inside [x0,x1] x [y0,y1]."""
    return (_quadrant_area(x1, y1, r) - _quadrant_area(x0, y1, r)
            - _quadrant_area(x1, y0, r) + _quadrant_area(x0, y0, r))


def _box_unit_sphere_volume(x0, x1, y0, y1, z0, z1):
    """Volume of the unit ball inside boxes [x0,x1]x[y0,y1]x[z0,z1] (arrays).

    Integrates the slice area A(z) = area(disc r(z) in rectangle) over z.
    A(z) is smooth except where r(z) crosses the distances from the axis to
    the rectangle's edges and corners; the z-interval is split there and each
    piece gets a 12-point Gauss-Legendre rule.
    """
    x0, x1, y0, y1, z0, z1 = (np.asarray(a, dtype=np.float64) for a in (x0, x1, y0, y1, z0, z1))
    za = np.clip(z0, -1.0, 1.0)
    zb = np.clip(z1, -1.0, 1.0)
    # Candidate radii where the slice area has a kink.
    dists = [np.abs(x0), np.abs(x1), np.abs(y0), np.abs(y1),
             np.hypot(x0, y0), np.hypot(x0, y1), np.hypot(x1, y0), np.hypot(x1, y1)]
    bps = [za, zb]
    for d in dists:
        zz = np.sqrt(np.maximum(1.0 - d * d, 0.0))
        for s in (zz, -zz):
            bps.append(np.clip(s, za, zb))
    bps.append(np.clip(np.zeros_like(za), za, zb))
    B = np.sort(np.stack(bps, axis=-1), axis=-1)
    vol = np.zeros(za.shape)
    for k in range(B.shape[-1] - 1):
        a = B[..., k]
        b = B[..., k + 1]
        h = b - a
        mid = 0.5 * (a + b)
        acc = np.zeros(za.shape)
        for xg, wg in zip(_GL_X, _GL_W):
            z = mid + 0.5 * h * xg
            r = np.sqrt(np.maximum(1.0 - z * z, 0.0))
            acc += wg * _rect_disc_area(x0, x1, y0, y1, r)
        vol += 0.5 * h * acc
    return vol


def ellipsoid_fraction(shape, center, semi_axes):
    """Liquid volume fraction of each cell inside an axis-aligned ellipsoid.

    shape = (nz, ny, nx); center = (cx, cy, cz) and semi_axes = (a, b, c) in
    cell-corner coordinates. The map (x-cx)/a etc. sends the ellipsoid to the
    unit ball and scales every cell volume by 1/(abc), so the fraction is
    abc * vol(unit ball ∩ mapped cell).
    """
    nz, ny, nx = shape
    cx, cy, cz = center
    a, b, c = semi_axes
    frac = np.zeros(shape, dtype=np.float64)
    # Only the bounding box of the body can hold liquid.
    lo = [max(0, int(np.floor(cc - s)) - 1) for cc, s in ((cz, c), (cy, b), (cx, a))]
    hi = [min(nn, int(np.ceil(cc + s)) + 1) for nn, cc, s in ((nz, cz, c), (ny, cy, b), (nx, cx, a))]
    if any(h <= l for l, h in zip(lo, hi)):
        return frac
    k, j, i = np.meshgrid(np.arange(lo[0], hi[0]), np.arange(lo[1], hi[1]),
                          np.arange(lo[2], hi[2]), indexing="ij")
    X0 = (i - cx) / a
    X1 = (i + 1 - cx) / a
    Y0 = (j - cy) / b
    Y1 = (j + 1 - cy) / b
    Z0 = (k - cz) / c
    Z1 = (k + 1 - cz) / c
    # A cell is entirely inside when its farthest corner is inside and
    # entirely outside when its nearest point is outside (scaled coordinates).
    far = np.maximum(X0 * X0, X1 * X1) + np.maximum(Y0 * Y0, Y1 * Y1) + np.maximum(Z0 * Z0, Z1 * Z1)

    def near1(l, h):
        return np.where((l <= 0) & (h >= 0), 0.0, np.minimum(l * l, h * h))

    near = near1(X0, X1) + near1(Y0, Y1) + near1(Z0, Z1)
    sub = np.zeros(X0.shape)
    sub[far <= 1.0] = 1.0
    cut = (near < 1.0) & (far > 1.0)
    idx = np.nonzero(cut)
    if idx[0].size:
        chunk = 100000
        vals = np.empty(idx[0].size)
        x0, x1, y0, y1, z0, z1 = X0[idx], X1[idx], Y0[idx], Y1[idx], Z0[idx], Z1[idx]
        for s in range(0, idx[0].size, chunk):
            sl = slice(s, s + chunk)
            v = _box_unit_sphere_volume(x0[sl], x1[sl], y0[sl], y1[sl], z0[sl], z1[sl])
            vals[sl] = v * (a * b * c)
        sub[idx] = np.clip(vals, 0.0, 1.0)
    frac[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = sub
    return frac


def sphere_fraction(shape, center, radius):
    """Liquid volume fraction of each cell inside a sphere (see ellipsoid_fraction)."""
    return ellipsoid_fraction(shape, center, (radius, radius, radius))


def cylinder_fraction(shape, center_xy, radius):
    """Liquid fraction of a cylinder along z (axis through center_xy = (cx, cy))."""
    nz, ny, nx = shape
    cx, cy = center_xy
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x0, x1, y0, y1 = i - cx, i + 1 - cx, j - cy, j + 1 - cy
    far = np.maximum(x0 * x0, x1 * x1) + np.maximum(y0 * y0, y1 * y1)
    near = (np.where((x0 <= 0) & (x1 >= 0), 0.0, np.minimum(x0 * x0, x1 * x1))
            + np.where((y0 <= 0) & (y1 >= 0), 0.0, np.minimum(y0 * y0, y1 * y1)))
    r2 = float(radius) ** 2
    area = _rect_disc_area(x0, x1, y0, y1, np.full(i.shape, float(radius)))
    area = np.where(far <= r2, 1.0, np.where(near >= r2, 0.0, np.clip(area, 0.0, 1.0)))
    return np.broadcast_to(area[None], shape).copy()


def splitmix_uniform(seed: int, n: int) -> np.ndarray:
    """Counter-based uniform numbers in [0, 1): SplitMix64 of (seed, index).

    SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the state for counter i
    is seed*golden + (i+1)*golden with golden = 0x9E3779B97F4A7C15, followed
    by the published 64-bit finaliser; the top 53 bits give the double.
    """
    golden = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) * golden + (np.arange(n, dtype=np.uint64) + np.uint64(1)) * golden
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def perturb_interface(fill: np.ndarray, amplitude: float = 1e-6, seed: int = 0) -> np.ndarray:
    """Add uniform noise in [-amplitude, amplitude) to cells with 0 < fill < 1.

    The noise value of cell i is SplitMix64(seed, i); the result is clamped to
    [0, 1]. Cells that are exactly 0 or 1 are left untouched.
    """
    out = fill.copy()
    u = splitmix_uniform(seed, fill.size).reshape(fill.shape)
    mask = (fill > 0.0) & (fill < 1.0)
    out[mask] = np.clip(fill[mask] + amplitude * (2.0 * u[mask] - 1.0), 0.0, 1.0)
    return out


def droplet(n: int, radius: float, noise: float = 1e-6, seed: int = 0):
    """Static spherical droplet of the given radius centred in a periodic n^3 box."""
    shape = (n, n, n)
    fill = sphere_fraction(shape, (n / 2, n / 2, n / 2), radius)
    if noise:
        fill = perturb_interface(fill, noise, seed)
    return fill, np.zeros(shape, dtype=np.uint8)


def bubble_probe(n: int, radius: float, noise: float = 0.0, seed: int = 0):
    """Gas bubble of the given radius in a liquid-filled periodic n^3 box."""
    shape = (n, n, n)
    fill = 1.0 - sphere_fraction(shape, (n / 2, n / 2, n / 2), radius)
    fill = np.clip(fill, 0.0, 1.0)
    if noise:
        fill = perturb_interface(fill, noise, seed)
    return fill, np.zeros(shape, dtype=np.uint8)


def advected_bubble(d: int):
    """Gas bubble of diameter d (cells) in a liquid-filled periodic box of
    3d x 2d x 2d (x, y, z), centred; the pure advection test of Sec. III.A
    translates it by d along x."""
    shape = (2 * d, 2 * d, 3 * d)
    fill = 1.0 - sphere_fraction(shape, (1.5 * d, d, d), d / 2.0)
    return np.clip(fill, 0.0, 1.0), np.zeros(shape, dtype=np.uint8)


def advection_errors(phi0: np.ndarray, phiT: np.ndarray, shift: int):
    """L1 and L2 errors of the advection test: phi(x + shift e_x, T) against
    phi(x, 0), normalised by the sums of |phi(x, 0)| and phi(x, 0)^2 over the
    whole periodic domain (Sec. III.A)."""
    moved = np.roll(phiT, -shift, axis=2)
    l1 = np.abs(moved - phi0).sum() / np.abs(phi0).sum()
    l2 = np.sqrt(((moved - phi0) ** 2).sum() / (phi0 ** 2).sum())
    return float(l1), float(l2)


def sessile_droplet(nx: int, ny: int, nz: int, radius: float, noise: float = 0.0, seed: int = 0):
    """Hemisphere on a no-slip wall.

    Obstacle layers fill k = 0 and k = nz-1; x and y are periodic. The wall
    plane is z = 1 (half-way between the obstacle layer and the first fluid
    layer) and the sphere centre is (nx/2, ny/2, 1).
    """
    shape = (nz, ny, nx)
    fill = sphere_fraction(shape, (nx / 2, ny / 2, 1.0), radius)
    obst = np.zeros(shape, dtype=np.uint8)
    obst[0] = 1
    obst[nz - 1] = 1
    fill[0] = 0.0
    fill[nz - 1] = 0.0
    if noise:
        fill = perturb_interface(fill, noise, seed)
    return fill, obst


def ellipsoid_droplet(n: int, semi_axes, noise: float = 1e-6, seed: int = 0):
    """Ellipsoidal droplet centred in a periodic n^3 box (oscillating-drop start)."""
    shape = (n, n, n)
    fill = ellipsoid_fraction(shape, (n / 2, n / 2, n / 2), semi_axes)
    if noise:
        fill = perturb_interface(fill, noise, seed)
    return fill, np.zeros(shape, dtype=np.uint8)


def flat_film(nx: int, ny: int, nz: int, height: float):
    """Liquid below the plane z = height between obstacle layers k=0 and k=nz-1."""
    shape = (nz, ny, nx)
    k = np.arange(nz, dtype=np.float64)
    col = np.clip(height - k, 0.0, 1.0)
    fill = np.broadcast_to(col[:, None, None], shape).copy()
    obst = np.zeros(shape, dtype=np.uint8)
    obst[0] = 1
    obst[nz - 1] = 1
    fill[0] = 0.0
    fill[nz - 1] = 0.0
    return fill, obst


def laplace_bubble(n: int, noise: float = 0.0, seed: int = 0):
    """The equilibrium-bubble setup of Sec. III.A.1 at dx = 1/n: a unit cube
    of liquid (n^3 fluid cells, periodic in x and y) between no-slip walls at
    z = 0 and z = 1, with a gas bubble of radius n/8 at its centre.

    Obstacle layers fill k = 0 and k = n+1, so the wall planes are z = 1 and
    z = n+1 in cell-corner coordinates and the centre is
    (n/2, n/2, n/2 + 1).
    """
    shape = (n + 2, n, n)
    fill = 1.0 - sphere_fraction(shape, (n / 2, n / 2, n / 2 + 1.0), n / 8.0)
    fill = np.clip(fill, 0.0, 1.0)
    obst = np.zeros(shape, dtype=np.uint8)
    obst[0] = 1
    obst[n + 1] = 1
    fill[0] = 0.0
    fill[n + 1] = 0.0
    if noise:
        fill = perturb_interface(fill, noise, seed)
    return fill, obst


def sessile_cap(n: int, theta_deg: float):
    """The equilibrium sessile droplet of Sec. III.B.1 at dx = 1/n: a
    spherical cap on the wall z = 0 of the unit cube (walls at z = 0 and 1,
    periodic in x and y) with the volume of a hemisphere of radius n/8 and
    the ideal height h and contact radius r of the contact angle theta
    (equations of that section). Obstacle layers fill k = 0 and k = n+1; the
    wall plane is z = 1 in cell-corner coordinates and the contact line is
    centred at (n/2, n/2). Returns fill, obstacle, h, r."""
    t = np.radians(theta_deg)
    R0 = n / 8.0
    V = 2.0 / 3.0 * np.pi * R0 ** 3
    h = (V / (np.pi * (1.0 / (1.0 - np.cos(t)) - 1.0 / 3.0))) ** (1.0 / 3.0)
    r = np.sqrt((6.0 * V / (np.pi * h) - h * h) / 3.0)
    Rs = h / (1.0 - np.cos(t))
    shape = (n + 2, n, n)
    fill = sphere_fraction(shape, (n / 2, n / 2, 1.0 + h - Rs), Rs)
    obst = np.zeros(shape, dtype=np.uint8)
    obst[0] = 1
    obst[n + 1] = 1
    fill[0] = 0.0
    fill[n + 1] = 0.0
    return fill, obst, float(h), float(r)


def renardy_units(n: int, dt: float = 1e-4):
    """(tau, sigma_L) of the equilibrium-bubble problem (Sec. III.A.1:
    liquid density 4, viscosity 1, surface tension 0.357 in units of the
    unit cube) at dx = 1/n and time step dt."""
    return lattice_units(1.0 / n, dt, 1.0 / 4.0, 0.357, 4.0)


def lattice_units(dx: float, dt: float, nu: float, sigma: float, rho: float):
    """Lattice relaxation time and surface tension for physical dx, dt.

    tau = 1/2 + 3 nu dt / dx^2 follows from nu = c_s^2 (tau - 1/2) with
    c_s^2 = 1/3 (Sec. II); sigma_L = sigma dt^2 / (rho dx^3) is the surface
    tension in lattice units (Sec. III.A.1 lists the resulting values).
    """
    tau = 0.5 + 3.0 * nu * dt / (dx * dx)
    sigma_l = sigma * dt * dt / (rho * dx ** 3)
    return tau, sigma_l
