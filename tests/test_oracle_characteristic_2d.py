"""Pins of the oracle's 2D Euler scheme with each sweep's reconstruction in local
characteristic fields (the 1D procedure of Sec. 4.3 applied along x and along y of the
dimension-by-dimension scheme, eq:2d).

Expected values come from the flux Jacobian written out (itself checked against central
differences of the flux) and diagonalised by LAPACK, from the Roe property of the averaged
state, from the 1D characteristic scheme (to which a y-uniform state without v reduces), from
the exchange of x and y, and from the exact 2D density wave.
"""
import numpy as np

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


def _jacobian_uvH(u, v, H, d):
    """dF/dU (d = 0) or dG/dU (d = 1) of 2D Euler in terms of (u, v, H)."""
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


def _jacobian(U, d):
    rho, u, v, p = _prim(U)
    return _jacobian_uvH(u, v, (U[3] + p) / rho, d)


def _roe_uvH(UL, UR):
    """The Roe-averaged u, v, H written out (sqrt(rho) weights)."""
    rl, ul, vl, pl = _prim(UL)
    rr, ur, vr, pr = _prim(UR)
    hl, hr = (UL[3] + pl) / rl, (UR[3] + pr) / rr
    wl, wr = np.sqrt(rl), np.sqrt(rr)
    avg = lambda a, b: (wl * a + wr * b) / (wl + wr)
    return avg(ul, ur), avg(vl, vr), avg(hl, hr)


def _random_state(rng, mach=1.5):
    rho = rng.uniform(0.2, 3.0)
    p = rng.uniform(0.2, 5.0)
    c = np.sqrt(G * p / rho)
    u, v = rng.uniform(-mach, mach, 2) * c
    return I.prim_to_cons_2d(np.array(rho), u, v, np.array(p), G).reshape(4)


def test_jacobian_is_the_flux_derivative():
    rng = np.random.default_rng(60)
    for _ in range(20):
        U = _random_state(rng)
        for d in (0, 1):
            h = 1e-6
            num = np.array([(_flux(U + h * e, d) - _flux(U - h * e, d)) / (2 * h)
                            for e in np.eye(4)]).T
            assert np.allclose(_jacobian(U, d), num, rtol=1e-7, atol=1e-7)


def test_roe_property_and_eigen_decomposition(orc):
    """For 200 random pairs and both directions: the oracle's R and Lc diagonalise the
    Jacobian at the Roe average (R diag(lambda) Lc = A, Lc R = I, lambda = u_n - c, u_n,
    u_n, u_n + c as LAPACK finds them), and that Jacobian has the Roe property
    A (U_R - U_L) = F(U_R) - F(U_L)."""
    rng = np.random.default_rng(61)
    for _ in range(200):
        UL, UR = _random_state(rng), _random_state(rng)
        u, v, H = _roe_uvH(UL, UR)
        c = np.sqrt((G - 1.0) * (H - 0.5 * (u * u + v * v)))
        for d in (0, 1):
            A = _jacobian_uvH(u, v, H, d)
            scale = np.abs(_flux(UR, d) - _flux(UL, d)).max()
            assert np.abs(A @ (UR - UL) - (_flux(UR, d) - _flux(UL, d))).max() <= 1e-12 * scale
            R, Lc = orc.roe_eigen_2d(UL, UR, d)
            un = u if d == 0 else v
            lam = np.array([un - c, un, un, un + c])
            assert np.abs(Lc @ R - np.eye(4)).max() < 1e-12
            assert np.allclose(R @ np.diag(lam) @ Lc, A, rtol=1e-11, atol=1e-11 * np.abs(A).max())
            ev = np.sort(np.linalg.eigvals(A).real)
            assert np.allclose(ev, np.sort(lam), rtol=1e-10, atol=1e-10)


def test_alphas_are_the_eigenvalue_maxima(orc):
    """Per-field alphas: max over the cells of |lambda_k| of each cell's own Jacobian."""
    U = I.random_smooth_2d(11, 7, seed=62)
    _, a8 = orc.rhs_2d_char(U, 0.1, 0.1)
    cells = U.reshape(4, -1).T
    for d in (0, 1):
        lams = np.array([np.sort(np.linalg.eigvals(_jacobian(c, d)).real) for c in cells])
        want = np.abs(lams).max(axis=0)
        assert np.allclose(a8[4 * d:4 * d + 4], want, rtol=1e-12), (d, a8, want)


def test_reduces_to_the_1d_scheme(orc):
    """A state uniform in y with v = 0: the y sweep vanishes exactly, the y momentum stays
    exactly 0, and rho, rho u, E follow the 1D characteristic scheme."""
    for bc in (orc.BC_TRANSMISSIVE, orc.BC_PERIODIC):
        u1, dx = I.shu_osher_like(300)
        U = np.zeros((4, 5, 300))
        U[0], U[1], U[3] = u1[0], u1[1], u1[2]
        L, a8 = orc.rhs_2d_char(U, dx, 0.37, bcx=bc, bcy=orc.BC_PERIODIC)
        r, a3 = orc.rhs_1d_char(u1, dx, bc=bc)
        assert np.allclose(a8[[0, 1, 3]], a3, rtol=1e-15) and a8[2] == a8[1]
        assert np.all(L[2] == 0.0)
        for j in range(5):
            for c2, c1 in ((0, 0), (1, 1), (3, 2)):
                assert np.abs(L[c2, j] - r[c1]).max() <= 1e-13 * np.abs(r[c1]).max()


def test_transpose_symmetry(orc):
    """Swapping x and y (and u and v) transposes the RHS."""
    U = I.random_smooth_2d(13, 9, seed=63)
    L, a8 = orc.rhs_2d_char(U, 0.1, 0.07, bcx=0, bcy=1)
    T = np.ascontiguousarray(U[[0, 2, 1, 3]].transpose(0, 2, 1))
    Lt, at = orc.rhs_2d_char(T, 0.07, 0.1, bcx=1, bcy=0)
    want = L[[0, 2, 1, 3]].transpose(0, 2, 1)
    assert np.abs(Lt - want).max() <= 1e-13 * np.abs(L).max()
    assert np.array_equal(at, np.concatenate([a8[4:], a8[:4]]))


def test_uniform_state_and_conservation(orc):
    U = I.prim_to_cons_2d(np.full((7, 8), 0.9), 0.4, -0.2, np.full((7, 8), 1.3), G)
    assert np.abs(orc.rhs_2d_char(U, 0.1, 0.1)[0]).max() < 1e-12
    U = I.random_smooth_2d(24, 20, seed=64)
    L, _ = orc.rhs_2d_char(U, 0.05, 0.04, bcx=0, bcy=0)
    assert np.abs(L.sum(axis=(1, 2))).max() < 1e-11 * np.abs(L).max()


def test_differs_from_component_wise(orc):
    """Control: on the first Riemann case the characteristic and component-wise LF
    right-hand sides differ (the projection is not the identity)."""
    U, dx, dy = I.riemann_2d(1, 48)
    Lc, _ = orc.rhs_2d_char(U, dx, dy)
    Ll, _ = orc.rhs_2d(U, dx, dy)
    assert np.abs(Lc - Ll).max() > 1e-3 * np.abs(Ll).max()


def test_fifth_order_on_density_wave(orc):
    """rho = 1 + 0.2 sin(pi (x + y)), u = 1, v = 0.5, p = 1 on the periodic [-1, 1]^2: the
    right-hand side converges at fifth order to the exact derivative."""
    errs = []
    for n in (32, 64, 128):
        U, dx, dy = I.density_wave_2d(n, n)
        x, _ = I.cell_centres(-1.0, 1.0, n)
        X, Y = np.meshgrid(x, x)
        rt = -0.2 * np.pi * np.cos(np.pi * (X + Y)) * 1.5  # rho_t = -(u + v) rho_x
        exact = np.array([rt, rt * 1.0, rt * 0.5, rt * 0.5 * 1.25])
        L, _ = orc.rhs_2d_char(U, dx, dy, bcx=0, bcy=0)
        errs.append(np.abs(L - exact).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders.min() > 4.85, orders


def test_run_dt_and_positivity(orc):
    """A short run of the paper's first Riemann case: the CFL dt of Sec. 4.4 from U^n, and
    positive density and pressure."""
    U, dx, dy = I.riemann_2d(1, 64)
    u, dts = orc.rk3_run_2d_char(U, dx, dy, 10, cfl=0.5)
    rho, uu, vv, p = _prim(U)
    c = np.sqrt(G * p / rho)
    dtx, dty = dx / (np.abs(uu) + c).max(), dy / (np.abs(vv) + c).max()
    assert dts[0] == 0.5 * dtx * dty / (dtx + dty) or abs(dts[0] / (0.5 * dtx * dty / (dtx + dty)) - 1) < 1e-14
    r2, u2, v2, p2 = _prim(u)
    assert r2.min() > 0 and p2.min() > 0 and np.isfinite(u).all()
