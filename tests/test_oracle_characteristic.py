"""Pins of the oracle's characteristic-field scheme for 1D Euler (Sec. 4.3: Lax-Friedrichs
splitting with the WENO reconstruction done in local characteristic fields).

The expected values never come from the oracle's own eigenvector formulas: the Jacobian is
written out and diagonalised by LAPACK, Roe's defining property is checked on flux
differences, a pure contact discontinuity reduces the scheme to scalar upwind advection of
the density (a closed form derived below), and the smooth Euler density wave fixes the
order and the exact derivative.
"""
import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

G = 1.4


def _flux(U, g=G):
    rho, m, E = U
    u = m / rho
    p = (g - 1.0) * (E - 0.5 * rho * u * u)
    return np.array([m, m * u + p, u * (E + p)])


def _jacobian(u, H, g=G):
    """dF/dU of 1D Euler in terms of the velocity and the total enthalpy (textbook form)."""
    return np.array([
        [0.0, 1.0, 0.0],
        [0.5 * (g - 3.0) * u * u, (3.0 - g) * u, g - 1.0],
        [u * (0.5 * (g - 1.0) * u * u - H), H - (g - 1.0) * u * u, g * u],
    ])


def _random_state(rng):
    rho = rng.uniform(0.2, 3.0)
    u = rng.uniform(-2.0, 2.0)
    p = rng.uniform(0.2, 5.0)
    return np.array([rho, rho * u, p / (G - 1.0) + 0.5 * rho * u * u])


# ---------------------------------------------------------------- eigen-system at the Roe state
def test_roe_property_and_eigensystem(orc):
    """R diag(lambda) Lc is Roe's matrix: it maps U_R - U_L onto F(U_R) - F(U_L) for any two
    states, Lc R = I, and its eigenvalues are the sorted eigenvalues of the Jacobian."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        UL, UR = _random_state(rng), _random_state(rng)
        R, Lc = orc.roe_eigen(UL, UR)
        assert np.abs(Lc @ R - np.eye(3)).max() < 1e-13
        lam = np.diag(Lc @ _roe_matrix_from(R, Lc, UL, UR) @ R)
        A = R @ np.diag(lam) @ Lc
        dF = _flux(UR) - _flux(UL)
        assert np.allclose(A @ (UR - UL), dF, rtol=1e-12, atol=1e-12 * np.abs(dF).max())
        # A is the Jacobian at some state; its eigenvalues are u - c < u < u + c
        assert lam[0] < lam[1] < lam[2]
        assert lam[2] - lam[1] == pytest.approx(lam[1] - lam[0], rel=1e-12)


def _roe_matrix_from(R, Lc, UL, UR):
    """The Jacobian whose eigenvectors R claims to hold: recover (u, H) from the columns of R
    (row 1 of the middle column is u, row 2 of the first column is H - u c) and build dF/dU
    from its textbook form, so that a wrong eigenvector fails the diagonality check."""
    u = R[1, 1]
    c = R[1, 2] - u
    H = R[2, 0] + u * c
    A = _jacobian(u, H)
    D = Lc @ A @ R
    assert np.abs(D - np.diag(np.diag(D))).max() < 1e-11 * max(1.0, np.abs(D).max())
    # the sound speed of that state, from its definition
    assert c * c == pytest.approx((G - 1.0) * (H - 0.5 * u * u), rel=1e-12)
    return A


def test_roe_of_equal_states_is_the_jacobian(orc):
    """At U_L = U_R the Roe state is that state: R holds the Jacobian's eigenvectors with
    eigenvalues u - c, u, u + c of the state itself."""
    rng = np.random.default_rng(12)
    for _ in range(50):
        U = _random_state(rng)
        R, Lc = orc.roe_eigen(U, U)
        rho, u = U[0], U[1] / U[0]
        p = (G - 1.0) * (U[2] - 0.5 * rho * u * u)
        c = np.sqrt(G * p / rho)
        H = (U[2] + p) / rho
        A = _jacobian(u, H)
        lam = np.linalg.eigvals(A).real
        lam.sort()
        assert np.allclose(lam, [u - c, u, u + c], rtol=1e-12, atol=1e-12)
        assert np.allclose(A @ R, R @ np.diag([u - c, u, u + c]), rtol=1e-11, atol=1e-11)


# ---------------------------------------------------------------- the RHS against a LAPACK reference
def _ghost(n, g, bc):
    if bc == 0:
        return g % n
    return min(max(g, 0), n - 1)


def _rhs_char_reference(orc, U, dx, bc, a3):
    """The characteristic RHS with eigenvectors from numpy.linalg.eig of the Jacobian at the
    Roe state (any scaling and sign: WENO-ZN is odd and homogeneous of degree one up to the
    tiny epsilon), and the scalar reconstruction the paper defines (pinned elsewhere)."""
    n = U.shape[1]
    fh = np.zeros((3, n + 1))
    F = np.array([_flux(U[:, j]) for j in range(n)]).T
    for k in range(n + 1):
        cells = [_ghost(n, k - 1 + s, bc) for s in range(-2, 4)]  # cells i-2 .. i+3
        UL, UR = U[:, cells[2]], U[:, cells[3]]
        sL, sR = np.sqrt(UL[0]), np.sqrt(UR[0])
        uL, uR = UL[1] / UL[0], UR[1] / UR[0]
        HL = (UL[2] + (G - 1.0) * (UL[2] - 0.5 * UL[0] * uL * uL)) / UL[0]
        HR = (UR[2] + (G - 1.0) * (UR[2] - 0.5 * UR[0] * uR * uR)) / UR[0]
        u = (sL * uL + sR * uR) / (sL + sR)
        H = (sL * HL + sR * HR) / (sL + sR)
        lam, Rm = np.linalg.eig(_jacobian(u, H))
        order = np.argsort(lam.real)
        Rm = Rm[:, order].real
        Lm = np.linalg.inv(Rm)
        V = Lm @ U[:, cells]
        W = Lm @ F[:, cells]
        gh = np.zeros(3)
        for f in range(3):
            gp = 0.5 * (W[f] + a3[f] * V[f])
            gm = 0.5 * (W[f] - a3[f] * V[f])
            gh[f] = (orc.reconstruct(gp[0:5])["fhat"]
                     + orc.reconstruct(gm[5:0:-1])["fhat"])
        fh[:, k] = Rm @ gh
    return -(fh[:, 1:] - fh[:, :-1]) / dx


@pytest.mark.parametrize("bc", [0, 1])
def test_rhs_matches_lapack_eigenvectors(orc, bc):
    """Random positive states (periodic and transmissive): the oracle's characteristic RHS
    equals the one built from LAPACK eigenvectors, and its per-field alphas are the largest
    |eigenvalue| of the cell Jacobians, field by field."""
    U = I.random_smooth_1d(24, seed=21)
    dx = 0.1
    L, a3 = orc.rhs_1d_char(U, dx, bc=bc)
    lams = []
    for j in range(U.shape[1]):
        rho, u = U[0, j], U[1, j] / U[0, j]
        p = (G - 1.0) * (U[2, j] - 0.5 * rho * u * u)
        lam = np.sort(np.linalg.eigvals(_jacobian(u, (U[2, j] + p) / rho)).real)
        lams.append(np.abs(lam))
    assert np.allclose(a3, np.max(lams, axis=0), rtol=1e-12)
    ref = _rhs_char_reference(orc, U, dx, bc, a3)
    scale = np.abs(ref).max()
    assert np.abs(L - ref).max() <= 1e-11 * scale, np.abs(L - ref).max() / scale


def test_rhs_uses_given_alphas(orc):
    """Alphas passed in are used as given (the alpha of each field is a parameter of the
    split, not a property of the state)."""
    U = I.random_smooth_1d(20, seed=22)
    a3 = np.array([3.0, 1.5, 2.5])
    L, used = orc.rhs_1d_char(U, 0.05, bc=0, alpha3=a3)
    assert np.array_equal(used, a3)
    ref = _rhs_char_reference(orc, U, 0.05, 0, a3)
    assert np.abs(L - ref).max() <= 1e-11 * np.abs(ref).max()


# ---------------------------------------------------------------- closed form on a contact
@pytest.mark.parametrize("u0", [0.7, -0.7])
def test_contact_reduces_to_scalar_upwind_advection(orc, u0):
    """A pure contact (uniform u and p, any density): the jump lies along the middle right
    eigenvector (1, u, u^2/2), so the outer fields see constant data, the middle field sees
    rho - p/c^2 advected at speed u with alpha_2 = |u|, and the numerical flux is exactly
    F(rho*, u, p) with rho* the upwind WENO-ZN value of the density.  Hence
    L_rho = the scalar advection RHS of rho at speed u, L_m = u L_rho, L_E = u^2/2 L_rho.
    The component-wise scheme has no such property (its alpha is max(|u| + c))."""
    n = 64
    x, dx = I.cell_centres(-1.0, 1.0, n)
    rho = np.where(np.abs(x) < 0.4, 1.0, 0.125) + 0.05 * np.sin(3.0 * np.pi * x)
    U = I.prim_to_cons_1d(rho, u0, 1.0)
    L, a3 = orc.rhs_1d_char(U, dx, bc=orc.BC_PERIODIC)
    assert a3[1] == pytest.approx(abs(u0), rel=1e-15)
    Ladv, _ = orc.rhs_1d(rho[None, :], dx, sys=orc.SYS_ADV, bc=orc.BC_PERIODIC,
                         alpha=abs(u0), a=u0)
    scale = np.abs(Ladv).max()
    assert np.abs(L[0] - Ladv[0]).max() <= 1e-12 * scale
    assert np.abs(L[1] - u0 * Ladv[0]).max() <= 1e-12 * scale
    assert np.abs(L[2] - 0.5 * u0 * u0 * Ladv[0]).max() <= 1e-12 * scale
    Lc, _ = orc.rhs_1d(U, dx, bc=orc.BC_PERIODIC)
    assert np.abs(Lc[0] - Ladv[0]).max() > 1e-3 * scale  # the control differs


# ---------------------------------------------------------------- invariants
def test_uniform_state_is_steady(orc):
    U = I.prim_to_cons_1d(np.full(32, 0.8), -0.3, 1.7)
    L, _ = orc.rhs_1d_char(U, 0.1, bc=orc.BC_TRANSMISSIVE)
    assert np.abs(L).max() < 1e-12


def test_periodic_conservation(orc):
    """Fluxes telescope on a periodic grid: sum_i L_i dx = 0 for every component."""
    U = I.random_smooth_1d(96, seed=23)
    L, _ = orc.rhs_1d_char(U, 0.02, bc=orc.BC_PERIODIC)
    assert np.abs(L.sum(axis=1) * 0.02).max() < 1e-12 * np.abs(L).max()


def test_mirror_symmetry(orc):
    """x -> -x maps (rho, m, E) to (rho, -m, E) and swaps the acoustic fields; the RHS of the
    mirrored state is the mirrored RHS, so the minus-side reconstruction is the plus side
    read backwards."""
    U = I.random_smooth_1d(40, seed=24)
    M = U[:, ::-1] * np.array([1.0, -1.0, 1.0])[:, None]
    L, a3 = orc.rhs_1d_char(U, 0.05, bc=orc.BC_PERIODIC)
    Lm, am = orc.rhs_1d_char(M, 0.05, bc=orc.BC_PERIODIC)
    assert np.allclose(am, a3[::-1], rtol=1e-15)
    want = L[:, ::-1] * np.array([1.0, -1.0, 1.0])[:, None]
    assert np.abs(Lm - want).max() <= 1e-12 * np.abs(L).max()


# ---------------------------------------------------------------- order on the exact density wave
def test_fifth_order_on_density_wave(orc):
    """rho = 1 + 0.2 sin(pi x), u = 1, p = 1 is an exact Euler solution with
    L = -(rho_x, rho_x, rho_x / 2): the characteristic RHS converges at fifth order."""
    errs = []
    for n in (32, 64, 128, 256):
        U, dx = I.density_wave_1d(n)
        x, _ = I.cell_centres(-1.0, 1.0, n)
        rx = 0.2 * np.pi * np.cos(np.pi * x)
        exact = -np.array([rx, rx, 0.5 * rx])
        L, _ = orc.rhs_1d_char(U, dx, bc=orc.BC_PERIODIC)
        errs.append(np.abs(L - exact).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders.min() > 4.8, orders


def test_run_dt_alphas_and_conservation(orc):
    """TVD-RK3 run of the characteristic scheme: dt = cfl dx / max(|u| + c) of U^n, the
    recorded alphas of the first stage are those of the initial state, mass, momentum and
    energy are conserved on a periodic grid, and the density wave moves at u."""
    n = 128
    U0, dx = I.density_wave_1d(n)
    U, dt, al = orc.rk3_run_1d_char(U0, dx, 20, cfl=0.4, bc=orc.BC_PERIODIC)
    rho, u = U0[0], U0[1] / U0[0]
    c = np.sqrt(G * (G - 1.0) * (U0[2] - 0.5 * rho * u * u) / rho)
    assert dt[0] == pytest.approx(0.4 * dx / np.max(np.abs(u) + c), rel=1e-14)
    _, a3 = orc.rhs_1d_char(U0, dx, bc=orc.BC_PERIODIC)
    assert np.array_equal(al[0, 0], a3)
    assert np.abs(U.sum(axis=1) - U0.sum(axis=1)).max() < 1e-12 * n
    t = dt.sum()
    exact, _ = I.density_wave_1d(n, t=t)
    assert np.abs(U - exact).max() < 1e-6
