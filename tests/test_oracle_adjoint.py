"""Pins of the oracle's complex-step path, which provides the reference derivatives of the
discrete adjoint: its real part is the fp64 oracle, and its imaginary part agrees with central
finite differences of the fp64 oracle."""
import numpy as np

from paper_2004_07954_amd import inputs as I


def test_complex_rhs_real_part_is_the_rhs(orc):
    u = I.random_smooth_1d(60, seed=51)
    L, al = orc.rhs_1d(u, 0.02, bc=orc.BC_PERIODIC)
    Lc = orc.rhs_1d_complex(u.astype(complex), 0.02, al, bc=orc.BC_PERIODIC)
    np.testing.assert_array_equal(Lc.real, L)
    assert np.all(Lc.imag == 0.0)


def test_complex_step_matches_central_differences(orc):
    """d/dh L(u + h v) by the complex step against central differences of the real RHS
    (h = 1e-6): agreement to ~1e-6 relative (the finite-difference truncation level)."""
    u = I.random_smooth_1d(60, seed=52)
    v = np.random.default_rng(53).standard_normal(u.shape)
    _, al = orc.rhs_1d(u, 0.02, bc=orc.BC_PERIODIC)
    hc = 1e-30
    dc = orc.rhs_1d_complex(u + 1j * hc * v, 0.02, al, bc=orc.BC_PERIODIC).imag / hc
    h = 1e-6
    Lp, _ = orc.rhs_1d(u + h * v, 0.02, alpha=al, bc=orc.BC_PERIODIC)
    Lm, _ = orc.rhs_1d(u - h * v, 0.02, alpha=al, bc=orc.BC_PERIODIC)
    fd = (Lp - Lm) / (2 * h)
    assert np.abs(dc - fd).max() <= 1e-5 * np.abs(dc).max()


def test_complex_rk3_step(orc):
    """The complex TVD-RK3 step with a frozen schedule: real part equals the fp64 step; the
    directional derivative matches central differences of the fp64 step."""
    u = I.random_smooth_1d(50, seed=54)
    v = np.random.default_rng(55).standard_normal(u.shape)
    un, dt, al3 = orc.rk3_step_1d(u, 0.02, cfl=0.5, bc=orc.BC_PERIODIC)
    uc = orc.rk3_step_1d_complex(u + 1e-30j * v, 0.02, dt, al3, bc=orc.BC_PERIODIC)
    np.testing.assert_array_equal(uc.real, un)
    h = 1e-6
    up, _, _ = orc.rk3_step_1d(u + h * v, 0.02, dt=dt, alpha3=al3, bc=orc.BC_PERIODIC)
    um, _, _ = orc.rk3_step_1d(u - h * v, 0.02, dt=dt, alpha3=al3, bc=orc.BC_PERIODIC)
    fd = (up - um) / (2 * h)
    d = uc.imag / 1e-30
    assert np.abs(d - fd).max() <= 1e-5 * np.abs(d).max()


def test_abs_derivative_at_zero_is_zero(orc):
    """The kink of tau5 = |IS0 - IS2| at a symmetric stencil: the complex step takes the
    derivative of |x| at 0 as 0 (the reading used by the adjoint)."""
    n = 40
    i = np.arange(n)
    rho = 1.0 + 0.5 * (np.abs(i - 20) <= 1)  # symmetric plateau
    u = I.prim_to_cons_1d(rho, 0.0, 1.0)
    _, al = orc.rhs_1d(u, 0.05, bc=orc.BC_PERIODIC)
    d = orc.rhs_1d_complex(u + 1e-30j * np.ones_like(u), 0.05, al, bc=orc.BC_PERIODIC)
    assert np.isfinite(d.imag).all()
