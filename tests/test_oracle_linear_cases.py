"""Pins of the oracle on the paper's linear advection cases (Sec. 4.2, eq:26 with
eq:1st_case, eq:single and eq:3rd_case; N = 200, T = 6, periodic): the paper shows figures
only, so the pins are the properties it states.
  * self-similarity: with eps = 1e-40 the scheme is invariant under the reference value A of
    case 1 (A in {100, 1, 0.01}); a dimension-mismatched eps (1e-6) loses it (control);
  * non-oscillation near discontinuities: overshoot and undershoot after three periods stay
    within 1 % of the largest jump of the data;
  * resolution near discontinuities: the WENO-ZN maximum error (which sits at the jumps) is
    below WENO-Z's in all three cases, and WENO-ZN's L1 error below WENO-JS's.
"""
import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

N, T = 200, 6.0
JUMP = {1: 1.0, 2: 1.0, 3: 2.0}  # largest jump of the initial data (case 3: across x = +-1)


def _run(orc, u0, dx, scheme=0, eps=1e-40):
    nsteps = int(np.ceil(T / (0.5 * dx) - 1e-12))
    u, _, _ = orc.rk3_run_1d(u0, dx, nsteps, dt=T / nsteps, sys=orc.SYS_ADV, bc=orc.BC_PERIODIC,
                             prm=orc.params(scheme=scheme, q=1, eps=eps))
    return u[0]


def test_inputs_match_the_printed_definitions():
    """Spot values of the three initial conditions from their printed formulas."""
    x = np.array([-0.7, -0.3, 0.1, 0.5, 0.9])
    u = I.four_waves(x)
    assert u[1] == 1.0 and u[2] == 1.0 and u[4] == 0.0
    assert u[0] == pytest.approx((2 * np.exp(-np.log(2) / 36) + 4) / 6, rel=1e-14)
    assert u[3] == pytest.approx((2 * np.sqrt(1 - 100 * 0.005**2) + 4) / 6, rel=1e-14)
    assert np.allclose(I.four_waves(x, A=100.0), u / 100.0, rtol=0, atol=0)
    y = np.array([-0.5, 0.25, 0.5])
    v = I.linear_case3(y)
    assert v[0] == pytest.approx(0.5 * np.sin(1.5 * np.pi * 0.25), rel=1e-14)
    assert v[1] == pytest.approx(1.0, rel=1e-14)
    assert v[2] == pytest.approx(-np.sin(1.5 * np.pi) / 6, rel=1e-14)


@pytest.mark.parametrize("scheme", [0, 1])
def test_self_similarity_case1(orc, scheme):
    u1, dx = I.linear_case(1, N, 1.0)
    r1 = _run(orc, u1, dx, scheme)
    for A in (100.0, 0.01):
        uA, _ = I.linear_case(1, N, A)
        rA = _run(orc, uA, dx, scheme)
        assert np.abs(A * rA - r1).max() <= 1e-12


def test_self_similarity_control(orc):
    """An absolute eps of 1e-6 (the dimension mismatch the paper warns about) is not
    scale invariant."""
    u1, dx = I.linear_case(1, N, 1.0)
    r1 = _run(orc, u1, dx, 0, eps=1e-6)
    uA, _ = I.linear_case(1, N, 100.0)
    rA = _run(orc, uA, dx, 0, eps=1e-6)
    assert np.abs(100.0 * rA - r1).max() > 1e-4


@pytest.mark.parametrize("case", [1, 2, 3])
def test_non_oscillatory(orc, case):
    u0, dx = I.linear_case(case, N)
    r = _run(orc, u0, dx)
    assert r.max() - u0.max() <= 0.01 * JUMP[case]
    assert u0.min() - r.min() <= 0.01 * JUMP[case]


@pytest.mark.parametrize("case", [1, 2, 3])
def test_resolution_against_comparison_weights(orc, case):
    u0, dx = I.linear_case(case, N)
    e = {s: _run(orc, u0, dx, s, eps=1e-40 if s < 2 else 1e-6) - u0[0] for s in (0, 1, 2)}
    assert np.abs(e[0]).max() < np.abs(e[1]).max()
    assert np.abs(e[0]).sum() < np.abs(e[2]).sum()
