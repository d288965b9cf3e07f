"""Write adjoint_c5_quad_fd.txt: reference directional derivatives of the adjoint workload's
loss, computed by the CPU oracle alone (this script imports nothing else of the method).

Workload: 1D Euler, N = 65536 periodic on [0, 1], the seeded initial density of the adjoint
case (seed 5), U0 = (rho0, rho0 / 2, 1/0.4 + rho0 / 8), 400 TVD-RK3 steps (Sec. 4) with the
dt and per-stage Lax-Friedrichs alphas of the oracle's own fp64 run from U0 held fixed.
Loss J = 1/2 sum_i (rho_T,i - rho_target,i)^2 with rho_target the density of the target
state of the same case.

The derivative of J along a direction v of rho0 is the central difference
(J(rho0 + h v) - J(rho0 - h v)) / (2 h) of two runs in __float128 (the oracle's runs with
the state carried in 113-bit arithmetic), with h far below fp64 resolution, so that the
weights respond linearly (per-cell perturbations are ~1e-21, the neighbouring differences
of the data >= ~1e-12).  The truncation error of such steps is negligible; what limits the
quotient is the runs' rounding, which grows as 1/h.  Two step sizes a decade apart are
written for the first direction (1e-20, 1e-19: they agree to ~4e-12) and for the cells
(1e-22, 1e-21: they agree to ~1e-8, the rounding noise of the smaller step; a step of
1e-24 per cell was noisier still, ~1e-7).  The larger step is the reference.

Directions: 4 white-noise unit directions (inputs.unit_directions(65536, 4, seed=71)) and
8 single cells 8192 apart (offset from default_rng(72).integers(0, 8192)).  With the
schedule frozen a stage moves information by 3 cells, so the cells' influence regions
(3600 cells wide on each side after 400 steps) are disjoint, and one pair of runs with all
eight cells perturbed gives each cell's derivative from its own 8192-cell window.

Run: python tests/golden/make_adjoint_c5_pins.py  (about 15 runs of ~200 s on 8 threads).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import binding as orc  # noqa: E402
from paper_2004_07954_amd import inputs as I  # noqa: E402

N, NSTEPS = 65536, 400
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_c5_quad_fd.txt")


def state(rho_hi, rho_lo):
    hi = np.stack([rho_hi, 0.5 * rho_hi, 1.0 / 0.4 + 0.125 * rho_hi])
    lo = np.stack([rho_lo, 0.5 * rho_lo, 0.125 * rho_lo])
    return hi, lo


def main():
    t0 = time.time()
    u0, ut, dx = I.adjoint_case(n=N, seed=5, sigma_cells=256.0)
    rho0, target = u0[0], ut[0]
    base, _ = state(rho0, np.zeros(N))
    _, dts, als = orc.rk3_run_1d(base, dx, NSTEPS, cfl=0.5, bc=orc.BC_PERIODIC)

    def run(dr):
        hi, lo = state(rho0, dr)
        return orc.rk3_run_1d_f128(hi, lo, dx, dts, als, bc=orc.BC_PERIODIC)

    def pair(v, h):
        """Per-cell contributions to J(rho0 + h v) - J(rho0 - h v), divided by 2 h."""
        ph, pl = run(h * v)
        mh, ml = run(-h * v)
        d = (ph[0] - mh[0]) + (pl[0] - ml[0])        # rho+ - rho- (double-double)
        s = (ph[0] + mh[0]) - 2.0 * target           # rho+ + rho- - 2 target
        print("  pair done at %.0f s" % (time.time() - t0), flush=True)
        return 0.5 * d * s / (2.0 * h)

    rows = []
    dirs = I.unit_directions(N, 4, seed=71)
    for k in range(4):
        for h in ((1e-20, 1e-19) if k == 0 else (1e-20,)):
            print("direction %d, h = %g" % (k, h), flush=True)
            rows.append(("direction", k, h, float(np.sum(pair(dirs[k], h)))))
    off = int(np.random.default_rng(72).integers(0, 8192))
    cells = off + 8192 * np.arange(8)
    e = np.zeros(N)
    e[cells] = 1.0
    for h in (1e-22, 1e-21):
        print("cells, h = %g" % h, flush=True)
        contrib = pair(e, h)
        for c in cells:
            win = (np.arange(N) - c + N // 2) % N - N // 2
            rows.append(("cell", int(c), h, float(np.sum(contrib[np.abs(win) <= 4095]))))
    with open(OUT, "w") as fh:
        fh.write("# Directional derivatives of the adjoint workload's loss along directions of the\n"
                 "# initial density, by central differences of __float128 oracle runs with the\n"
                 "# oracle's fp64 schedule frozen (written by make_adjoint_c5_pins.py, which calls\n"
                 "# only the oracle).  kind index h dJ\n")
        for kind, idx, h, val in rows:
            fh.write("%s %d %.1e %.17e\n" % (kind, idx, h, val))
    print("wrote %s in %.0f s" % (OUT, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
