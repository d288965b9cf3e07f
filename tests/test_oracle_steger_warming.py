"""Pins of the oracle's Steger-Warming flux-vector splitting and of the 2D right-hand side
built on it (Sec. 4.4 uses this splitting for its 2D problems).

Expected values come from the Jacobian written out and diagonalised by LAPACK (the Euler
flux is homogeneous of degree one, F = A(U) U, so F^{+-} = R diag(lambda^{+-}) R^{-1} U),
from the physical flux, from supersonic states where one side vanishes exactly, and from
the exact 2D density wave.
"""
import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

G = 1.4


def _prim(U):
    rho, mx, my, E = U
    u, v = mx / rho, my / rho
    p = (G - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def _flux(U, d):
    rho, u, v, p = _prim(U)
    E = U[3]
    if d == 0:
        return np.array([rho * u, rho * u * u + p, rho * u * v, u * (E + p)])
    return np.array([rho * v, rho * u * v, rho * v * v + p, v * (E + p)])


def _jacobian(U, d):
    """dF/dU (d = 0) or dG/dU (d = 1) of 2D Euler, textbook form in (u, v, H)."""
    rho, u, v, p = _prim(U)
    H = (U[3] + p) / rho
    g1 = G - 1.0
    q2 = 0.5 * (u * u + v * v)
    if d == 0:
        return np.array([
            [0.0, 1.0, 0.0, 0.0],
            [g1 * q2 - u * u, (3.0 - G) * u, -g1 * v, g1],
            [-u * v, v, u, 0.0],
            [u * (g1 * q2 - H), H - g1 * u * u, -g1 * u * v, G * u]])
    return np.array([
        [0.0, 0.0, 1.0, 0.0],
        [-u * v, v, u, 0.0],
        [g1 * q2 - v * v, -g1 * u, (3.0 - G) * v, g1],
        [v * (g1 * q2 - H), -g1 * u * v, H - g1 * v * v, G * v]])


def _random_state(rng, mach=1.5):
    rho = rng.uniform(0.2, 3.0)
    p = rng.uniform(0.2, 5.0)
    c = np.sqrt(G * p / rho)
    u, v = rng.uniform(-mach, mach, 2) * c
    return I.prim_to_cons_2d(np.array(rho), u, v, np.array(p), G).reshape(4)


def test_jacobian_is_the_flux_derivative():
    """The test's own Jacobian against central differences of the flux (so that it can
    serve as the reference below)."""
    rng = np.random.default_rng(50)
    for _ in range(20):
        U = _random_state(rng)
        for d in (0, 1):
            h = 1e-6
            num = np.array([(_flux(U + h * e, d) - _flux(U - h * e, d)) / (2 * h)
                            for e in np.eye(4)]).T
            assert np.allclose(_jacobian(U, d), num, rtol=1e-7, atol=1e-7)
            assert np.allclose(_jacobian(U, d) @ U, _flux(U, d), rtol=1e-13, atol=1e-13)


def test_split_is_the_eigen_decomposition(orc):
    """F^{+-} = R diag((lambda +- |lambda|)/2) R^{-1} U with LAPACK's eigenvectors, both
    directions, sub- and supersonic states (any eigenvector scaling cancels)."""
    rng = np.random.default_rng(51)
    for _ in range(300):
        U = _random_state(rng, mach=2.5)
        for d in (0, 1):
            # the double eigenvalue u may come back as a tiny complex-conjugate pair: keep
            # complex arithmetic and take the real part of the product
            lam, R = np.linalg.eig(_jacobian(U, d))
            Ri = np.linalg.inv(R)
            lp = 0.5 * (lam.real + np.abs(lam.real))
            Fp_ref = (R @ np.diag(lp) @ Ri @ U).real
            Fm_ref = (R @ np.diag(lam.real - lp) @ Ri @ U).real
            Fp, Fm = orc.sw_split(U, d)
            scale = np.abs(_flux(U, d)).max() + np.abs(Fp_ref).max()
            assert np.abs(Fp - Fp_ref).max() <= 1e-12 * scale
            assert np.abs(Fm - Fm_ref).max() <= 1e-12 * scale
            assert np.abs(Fp + Fm - _flux(U, d)).max() <= 1e-13 * scale


def test_supersonic_states_are_one_sided(orc):
    """|u| > c: the whole flux goes to one side and the other is exactly zero."""
    for u, v in ((2.0, 0.3), (-2.0, 0.3), (0.3, 2.0), (0.3, -2.0)):
        U = I.prim_to_cons_2d(np.array(1.0), u, v, np.array(1.0 / G * 1.0), G).reshape(4)
        d = 0 if abs(u) > 1.5 else 1
        Fp, Fm = orc.sw_split(U, d)
        F = _flux(U, d)
        pos = (u if d == 0 else v) > 0
        assert np.array_equal(Fm if pos else Fp, np.zeros(4))
        assert np.allclose(Fp if pos else Fm, F, rtol=1e-14, atol=1e-15)


def _ghost(n, g, bc):
    return g % n if bc == 0 else min(max(g, 0), n - 1)


def test_rhs_x_only_against_assembled_reference(orc):
    """y-uniform data: the y fluxes cancel and L is the x reconstruction of the split fluxes,
    assembled here from the split and the scalar reconstruction (both pinned above and in
    the reconstruction pins) with the fluxes differenced by hand."""
    nx, ny, dx = 40, 6, 0.05
    rng = np.random.default_rng(52)
    row = np.array([_random_state(rng, mach=1.2) for _ in range(nx)]).T  # [4, nx]
    U = np.repeat(row[:, None, :], ny, axis=1)
    for bc in (0, 1):
        L = orc.rhs_2d_sw(U, dx, 0.07, bcx=bc, bcy=0)
        fh = np.zeros((4, nx + 1))
        for k in range(nx + 1):
            cells = [_ghost(nx, k - 1 + s, bc) for s in range(-2, 4)]
            sp = np.array([orc.sw_split(row[:, c], 0)[0] for c in cells]).T
            sm = np.array([orc.sw_split(row[:, c], 0)[1] for c in cells]).T
            for q in range(4):
                fh[q, k] = (orc.reconstruct(sp[q, 0:5])["fhat"]
                            + orc.reconstruct(sm[q, 5:0:-1])["fhat"])
        ref = -(fh[:, 1:] - fh[:, :-1]) / dx
        for j in range(ny):
            assert np.abs(L[:, j, :] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_transpose_symmetry(orc):
    """Swapping x and y (and u and v) transposes the RHS."""
    U = I.random_smooth_2d(13, 9, seed=53)
    L = orc.rhs_2d_sw(U, 0.1, 0.1, bcx=0, bcy=1)
    T = np.ascontiguousarray(U[[0, 2, 1, 3]].transpose(0, 2, 1))
    Lt = orc.rhs_2d_sw(T, 0.1, 0.1, bcx=1, bcy=0)
    want = L[[0, 2, 1, 3]].transpose(0, 2, 1)
    assert np.abs(Lt - want).max() <= 1e-12 * np.abs(L).max()


def test_uniform_state_and_conservation(orc):
    U = I.prim_to_cons_2d(np.full((7, 8), 0.9), 0.4, -0.2, np.full((7, 8), 1.3), G)
    assert np.abs(orc.rhs_2d_sw(U, 0.1, 0.1)).max() < 1e-12
    U = I.random_smooth_2d(24, 20, seed=54)
    L = orc.rhs_2d_sw(U, 0.05, 0.04, bcx=0, bcy=0)
    assert np.abs(L.sum(axis=(1, 2))).max() < 1e-11 * np.abs(L).max()


def test_fifth_order_on_density_wave(orc):
    """rho = 1 + 0.2 sin(pi (x + y)), u = 1, v = 0.5, p = 1 (no sonic point, so the split
    fluxes are smooth): the SW right-hand side converges at fifth order to the exact
    derivative."""
    errs = []
    for n in (32, 64, 128):
        U, dx, dy = I.density_wave_2d(n, n)
        x, _ = I.cell_centres(-1.0, 1.0, n)
        X, Y = np.meshgrid(x, x)
        rt = -0.2 * np.pi * np.cos(np.pi * (X + Y)) * 1.5  # rho_t = -(u + v) rho_x
        exact = np.array([rt, rt * 1.0, rt * 0.5, rt * 0.5 * 1.25])
        L = orc.rhs_2d_sw(U, dx, dy, bcx=0, bcy=0)
        errs.append(np.abs(L - exact).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders.min() > 4.85, orders


def test_run_dt_and_riemann_case_positivity(orc):
    """A short run of the paper's first Riemann case: the CFL dt of Sec. 4.4 from U^n, mass
    conservation up to the transmissive boundary fluxes (zero here: the states next to the
    boundary are uniform along it for the first steps), and positivity."""
    U0, dx, dy = I.riemann_2d(1, 48)
    U, dt = orc.rk3_run_2d_sw(U0, dx, dy, 5, cfl=0.5)
    rho, u, v, p = _prim(U0)
    c = np.sqrt(G * p / rho)
    dtx, dty = dx / np.max(np.abs(u) + c), dy / np.max(np.abs(v) + c)
    assert dt[0] == pytest.approx(0.5 * dtx * dty / (dtx + dty), rel=1e-14)
    r1, _, _, p1 = _prim(U)
    assert r1.min() > 0 and p1.min() > 0
