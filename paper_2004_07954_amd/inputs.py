"""Seeded synthetic inputs for the WENO-ZN workloads.

This module holds initial conditions and random draws only -- none of the
scheme's arithmetic.  Both the HIP path and the CPU oracle are fed from it.
All states are conservative variables in SoA layout: [nvar, n] in 1D and
[4, ny, nx] (x fastest) in 2D.  Random numbers come from numpy's PCG64
``default_rng(seed)`` in fp64; the draw order is fixed as documented per function.
"""
import math

import numpy as np

GAMMA = 1.4


def cell_centres(xl, xr, n):
    """x_i = xl + (i + 1/2) dx, dx = (xr - xl)/n."""
    dx = (xr - xl) / n
    return xl + (np.arange(n) + 0.5) * dx, dx


def prim_to_cons_1d(rho, u, p, gamma=GAMMA):
    rho, u, p = np.broadcast_arrays(np.asarray(rho, float), np.asarray(u, float),
                                    np.asarray(p, float))
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def prim_to_cons_2d(rho, u, v, p, gamma=GAMMA):
    rho, u, v, p = np.broadcast_arrays(*(np.asarray(a, float) for a in (rho, u, v, p)))
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


# ------------------------------------------------------------------ advection
def advection_smooth(n, xl=-1.0, xr=1.0):
    """u0 = sin(pi x - sin(pi x)/pi) on a periodic [-1, 1] grid: shape [1, n]."""
    x, dx = cell_centres(xl, xr, n)
    return np.sin(np.pi * x - np.sin(np.pi * x) / np.pi)[None, :], dx


def advection_smooth_exact(x, t):
    y = x - t
    return np.sin(np.pi * y - np.sin(np.pi * y) / np.pi)


def single_jump(x):
    """The function with one jump at x = 0 (Sec. 3, eq:single) on [-1, 1].

    x <= 0 takes the left branch; the table of indicators around the jump prints
    u0(0) = 0, i.e. the left branch at x = 0 (reading kept in the design notes).
    """
    x = np.asarray(x, dtype=float)
    base = -np.sin(np.pi * x) - 0.5 * x ** 3
    return np.where(x <= 0.0, base, base + 1.0)


# ------------------------------------------------------------------ 1D Euler
# The linear advection cases of Sec. 4.2 on the periodic [-1, 1] (run to T = 6 on N = 200).
def four_waves(x, A=1.0):
    """Case 1 (eq:1st_case): Gaussians, square wave, triangle and half ellipse, divided by
    the reference value A.  Constants a = 0.5, z = -0.7, delta = 0.005, alpha = 10,
    beta = log 2 / (36 delta^2); the ellipse terms are centred at a - delta, a + delta and a."""
    x = np.asarray(x, dtype=np.float64)
    a, z, d, al = 0.5, -0.7, 0.005, 10.0
    be = math.log(2.0) / (36.0 * d * d)

    def G(zz):
        return np.exp(-be * (x - zz) ** 2)

    def F(aa):
        return np.sqrt(np.maximum(1.0 - al * al * (x - aa) ** 2, 0.0))

    u = np.zeros_like(x)
    m = (x >= -0.8) & (x <= -0.6)
    u[m] = ((G(z - d) + G(z + d) + 4.0 * G(z)) / 6.0)[m]
    u[(x >= -0.4) & (x <= -0.2)] = 1.0
    m = (x >= 0.0) & (x <= 0.2)
    u[m] = (1.0 - np.abs(10.0 * (x - 0.1)))[m]
    m = (x >= 0.4) & (x <= 0.6)
    u[m] = ((F(a - d) + F(a + d) + 4.0 * F(a)) / 6.0)[m]
    return u / A


def linear_case3(x):
    """Case 3 (eq:3rd_case)."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(x < -1.0 / 3.0, -x * np.sin(1.5 * np.pi * x * x),
                    np.where(x <= 1.0 / 3.0, np.abs(np.sin(2.0 * np.pi * x)),
                             2.0 * x - 1.0 - np.sin(3.0 * np.pi * x) / 6.0))


def linear_case(case, n, A=1.0):
    """Cell-centre data [1, n] of linear case 1, 2 (the single jump) or 3 on [-1, 1]; dx."""
    x, dx = cell_centres(-1.0, 1.0, n)
    if case == 1:
        u = four_waves(x, A)
    elif case == 2:
        u = single_jump(x)
    elif case == 3:
        u = linear_case3(x)
    else:
        raise ValueError("case must be 1, 2 or 3")
    return u[None, :], dx


def shu_osher_like(n, xl=-5.0, xr=5.0, gamma=GAMMA):
    """Left state (3.857143, 2.629369, 10.33333) for x < -4, right state
    (1 + 0.2 sin 5x, 0, 1); transmissive.  Returns (U[3, n], dx)."""
    x, dx = cell_centres(xl, xr, n)
    left = x < -4.0
    rho = np.where(left, 3.857143, 1.0 + 0.2 * np.sin(5.0 * x))
    u = np.where(left, 2.629369, 0.0)
    p = np.where(left, 10.33333, 1.0)
    return prim_to_cons_1d(rho, u, p, gamma), dx


def density_wave_1d(n, xl=-1.0, xr=1.0, amp=0.2, u0=1.0, p0=1.0, t=0.0, gamma=GAMMA):
    """rho = 1 + amp sin(pi (x - u0 t)), u = u0, p = p0: an exact periodic Euler solution."""
    x, dx = cell_centres(xl, xr, n)
    rho = 1.0 + amp * np.sin(np.pi * (x - u0 * t))
    return prim_to_cons_1d(rho, u0, p0, gamma), dx


def random_smooth_1d(n, seed, gamma=GAMMA):
    """Positive smooth-ish random state for parity tests (rho, p in [0.5, 1.5],
    u in [-0.5, 0.5]), periodic-friendly; draw order rho, u, p."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5, n)
    u = rng.uniform(-0.5, 0.5, n)
    p = rng.uniform(0.5, 1.5, n)
    return prim_to_cons_1d(rho, u, p, gamma)


def shock_tube_batch(batch, seed=4, nmin=256, nmax=16384, gamma=GAMMA):
    """Batched 1D shock tubes on [0, 1], jump at x = 0.5, transmissive.

    Draw order: lengths N_i = integers(nmin, nmax, endpoint=True) for all i first;
    then per instance rhoL, uL, pL, rhoR, uR, pR with rho ~ U[0.125, 5],
    u ~ U[-1, 1], p ~ U[0.1, 10].  Returns (U[3, sum N], offsets[B+1] int64, dx[B]).
    """
    rng = np.random.default_rng(seed)
    lens = rng.integers(nmin, nmax, size=batch, endpoint=True).astype(np.int64)
    offsets = np.zeros(batch + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lens)
    U = np.empty((3, int(offsets[-1])))
    dx = 1.0 / lens.astype(np.float64)
    for b in range(batch):
        rl = rng.uniform(0.125, 5.0); ul = rng.uniform(-1.0, 1.0); pl = rng.uniform(0.1, 10.0)
        rr = rng.uniform(0.125, 5.0); ur = rng.uniform(-1.0, 1.0); pr = rng.uniform(0.1, 10.0)
        x, _ = cell_centres(0.0, 1.0, int(lens[b]))
        left = x < 0.5
        U[:, offsets[b]:offsets[b + 1]] = prim_to_cons_1d(np.where(left, rl, rr),
                                                          np.where(left, ul, ur),
                                                          np.where(left, pl, pr), gamma)
    return U, offsets, dx


def smoothed_noise_periodic(n, sigma_cells, rng):
    """Periodic Gaussian smoothing (std sigma_cells, via FFT) of N(0,1) noise,
    normalised to unit standard deviation."""
    w = rng.standard_normal(n)
    k = np.fft.rfftfreq(n) * n  # integer wavenumbers
    filt = np.exp(-0.5 * (2.0 * np.pi * k * sigma_cells / n) ** 2)
    s = np.fft.irfft(np.fft.rfft(w) * filt, n)
    return s / s.std()


def adjoint_case(n=65536, seed=5, sigma_cells=256.0, gamma=GAMMA):
    """Periodic [0, 1]: rho0 = 1 + 0.2 sin 2 pi x + 0.05 n1, u = 0.5, p = 1;
    the target run starts from rho0 + 0.01 n2.  Draw order: n1, n2.
    Returns (U0[3, n], U0_target[3, n], dx)."""
    rng = np.random.default_rng(seed)
    x, dx = cell_centres(0.0, 1.0, n)
    n1 = smoothed_noise_periodic(n, sigma_cells, rng)
    n2 = smoothed_noise_periodic(n, sigma_cells, rng)
    rho0 = 1.0 + 0.2 * np.sin(2.0 * np.pi * x) + 0.05 * n1
    U0 = prim_to_cons_1d(rho0, 0.5, 1.0, gamma)
    Ut = prim_to_cons_1d(rho0 + 0.01 * n2, 0.5, 1.0, gamma)
    return U0, Ut, dx


def unit_directions(n, count, seed, smooth_cells=0.0):
    """Random unit directions; smooth_cells > 0 applies the periodic Gaussian smoothing of
    smoothed_noise_periodic (std in cells) before normalising."""
    rng = np.random.default_rng(seed)
    if smooth_cells > 0:
        d = np.stack([smoothed_noise_periodic(n, smooth_cells, rng) for _ in range(count)])
    else:
        d = rng.standard_normal((count, n))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


# ------------------------------------------------------------------ 2D Euler
def four_quadrant_random(nx, ny, seed=3, gamma=GAMMA):
    """Four-quadrant Riemann data on [0, 1]^2 split at (0.5, 0.5).

    Draw order: quadrants SW (x<.5, y<.5), SE, NW, NE; per quadrant rho ~ U[0.1, 2],
    u ~ U[-1, 1], v ~ U[-1, 1], p ~ U[0.1, 2].  Returns (U[4, ny, nx], dx, dy).
    """
    rng = np.random.default_rng(seed)
    states = []
    for _ in range(4):
        states.append((rng.uniform(0.1, 2.0), rng.uniform(-1.0, 1.0), rng.uniform(-1.0, 1.0),
                       rng.uniform(0.1, 2.0)))
    x, dx = cell_centres(0.0, 1.0, nx)
    y, dy = cell_centres(0.0, 1.0, ny)
    X, Y = np.meshgrid(x, y)  # [ny, nx]
    east = X >= 0.5
    north = Y >= 0.5
    q = (north.astype(int) * 2 + east.astype(int))  # 0 SW, 1 SE, 2 NW, 3 NE
    prim = np.zeros((4, ny, nx))
    for k, st in enumerate(states):
        for c in range(4):
            prim[c][q == k] = st[c]
    return prim_to_cons_2d(prim[0], prim[1], prim[2], prim[3], gamma), dx, dy


# The two 2D Riemann problems of Sec. 4.4 on [0, 1]^2 (eq:RM1, split at (0.8, 0.8), run to
# t = 0.8 on 400^2; eq:RM2, split at (0.5, 0.5), run to t = 0.25 on 1200^2 and 2400^2), as
# (rho, u, v, p) per quadrant.  Cells on a split line belong to the quadrant the equation's
# inequalities give them.
def riemann_2d(case, nx, ny=None, gamma=GAMMA):
    """Initial data of the 2D Riemann case 1 or 2; returns (U[4, ny, nx], dx, dy)."""
    ny = nx if ny is None else ny
    x, dx = cell_centres(0.0, 1.0, nx)
    y, dy = cell_centres(0.0, 1.0, ny)
    X, Y = np.meshgrid(x, y)
    prim = np.zeros((4, ny, nx))
    if case == 1:
        east, north = X >= 0.8, Y >= 0.8
        quads = [(east & north, (1.5, 0.0, 0.0, 1.5)),
                 (~east & north, (0.5323, 1.206, 0.0, 0.3)),
                 (~east & ~north, (0.138, 1.206, 1.206, 0.029)),
                 (east & ~north, (0.5323, 0.0, 1.206, 0.3))]
    elif case == 2:
        east, north = X > 0.5, Y > 0.5
        quads = [(~east & ~north, (0.8, 0.0, 0.0, 1.0)),
                 (~east & north, (1.0, 0.7276, 0.0, 1.0)),
                 (east & ~north, (1.0, 0.0, 0.7276, 1.0)),
                 (east & north, (0.5313, 0.0, 0.0, 0.4))]
    else:
        raise ValueError("case must be 1 or 2")
    for mask, st in quads:
        for c in range(4):
            prim[c][mask] = st[c]
    return prim_to_cons_2d(prim[0], prim[1], prim[2], prim[3], gamma), dx, dy


def density_wave_2d(nx, ny, amp=0.2, u0=1.0, v0=0.5, p0=1.0, t=0.0, gamma=GAMMA):
    """rho = 1 + amp sin(pi (x + y - (u0 + v0) t)) on the periodic [-1, 1]^2."""
    x, dx = cell_centres(-1.0, 1.0, nx)
    y, dy = cell_centres(-1.0, 1.0, ny)
    X, Y = np.meshgrid(x, y)
    rho = 1.0 + amp * np.sin(np.pi * (X + Y - (u0 + v0) * t))
    return prim_to_cons_2d(rho, u0, v0, p0, gamma), dx, dy


def random_smooth_2d(nx, ny, seed, gamma=GAMMA):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5, (ny, nx))
    u = rng.uniform(-0.5, 0.5, (ny, nx))
    v = rng.uniform(-0.5, 0.5, (ny, nx))
    p = rng.uniform(0.5, 1.5, (ny, nx))
    return prim_to_cons_2d(rho, u, v, p, gamma)


def rng_uniform(shape, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, shape)


__all__ = [k for k in dir() if not k.startswith("_") and k not in ("math", "np")]
