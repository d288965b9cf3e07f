"""The oracle's pins catch planted mistakes (CPU only).

Each mutant below is a copy of oracle/wenozn_oracle.cpp with one plausible slip of the kind a
transcription of the paper could make: a wrong coefficient, a dropped term, a flipped sign, a
wrong or shifted index, a transposed operand.  Every mutant is compiled and the oracle test
files (tests/test_oracle_*.py, which hold the pins to the paper's tables, closed forms,
orders and invariants) are run against it in a child interpreter: at least one test must fail
for every mutant.  The unmutated source must pass the same files (the control)."""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "wenozn_oracle.cpp")

# (name, what the slip is, exact text, replacement)
MUTANTS = [
    ("q0_coefficient", "candidate flux q0: 7/6 -> 5/6 (eq:4)",
     "T(1) / T(3) * a - T(7) / T(6) * b", "T(1) / T(3) * a - T(5) / T(6) * b"),
    ("is0_weight", "IS0: 13/12 -> 13/11 (eq:isjiang)",
     "r.IS[0] = T(13) / T(12)", "r.IS[0] = T(13) / T(11)"),
    ("is1_sign", "IS1: (b - d)^2 -> (b + d)^2 (eq:isjiang)",
     "T(1) / T(4) * sq(b - d)", "T(1) / T(4) * sq(b + d)"),
    ("tau5_index", "tau5 = |IS0 - IS1| instead of |IS0 - IS2|",
     "r.tau5 = absv(r.IS[0] - r.IS[2]);", "r.tau5 = absv(r.IS[0] - r.IS[1]);"),
    ("tau8_sign", "tau8: + e -> - e (eq:tau8)",
     "- T(4) * d + e);", "- T(4) * d - e);"),
    ("c_drops_tau5", "C: the -tau5 term of the numerator dropped (eq:function)",
     "(r.IS[0] + r.IS[2] - r.tau5 + eps)", "(r.IS[0] + r.IS[2] + eps)"),
    ("c_drops_a", "C: the constant A dropped (eq:function)",
     "r.C = A * ipow(", "r.C = ipow("),
    ("zn_exponent", "alpha_k: tau8/(IS_k + eps) squared instead of to the first power (eq:new)",
     "ipow(r.tau8 / (r.IS[k] + eps), P.q)", "ipow(r.tau8 / (r.IS[k] + eps), P.q + 1)"),
    ("linear_weights", "linear weights (1, 6, 3)/10 transposed to (3, 6, 1)/10",
     "{T(1) / T(10), T(6) / T(10), T(3) / T(10)}", "{T(3) / T(10), T(6) / T(10), T(1) / T(10)}"),
    ("mirror_shift", "f^- stencil mirrored about x_i instead of x_{i+1/2}",
     "reconstruct(M_[i + 3], M_[i + 2], M_[i + 1], M_[i], M_[i - 1], P)",
     "reconstruct(M_[i + 2], M_[i + 1], M_[i], M_[i - 1], M_[i - 2], P)"),
    ("lf_split_sign", "f^- = (F + alpha U)/2 instead of (F - alpha U)/2",
     "fm[v * np + j] = T(1) / T(2) * (F[v] - T(alpha) * U[v]);",
     "fm[v * np + j] = T(1) / T(2) * (F[v] + T(alpha) * U[v]);"),
    ("energy_flux", "1D energy flux u E instead of u (E + p)",
     "  F[2] = u * (E + p);\n}", "  F[2] = u * E;\n}"),
    ("wave_speed_abs", "max wave speed u + c instead of |u| + c",
     "return std::fabs(u) + std::sqrt(ph.gamma * p / rho);",
     "return u + std::sqrt(ph.gamma * p / rho);"),
    ("transmissive_bc", "transmissive ghosts copy the second cell instead of the edge cell",
     "return g < 0 ? 0 : n - 1;", "return g < 0 ? 1 : n - 2;"),
    ("rk3_coefficient", "TVD-RK3 second stage 3/4 U^n -> 1/4 U^n",
     "static const double RK_A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};",
     "static const double RK_A[3] = {0.0, 1.0 / 4.0, 1.0 / 3.0};"),
    ("g_flux_transposed", "2D y flux component rho u v written rho v v",
     "G[1] = rho * u * v;", "G[1] = rho * v * v;"),
    ("char_eigen_sign", "characteristic Lc[1][1] = -b1 u instead of b1 u",
     "  Lc[1][1] = b1 * u;\n", "  Lc[1][1] = -b1 * u;\n"),
    ("sw_split_sign", "Steger-Warming l2^{+-} with the sign of |l| flipped",
     "const T l2 = (un + s * absv(un)) / T(2);", "const T l2 = (un - s * absv(un)) / T(2);"),
]

CHILD = """
import sys
sys.path.insert(0, {root!r})
from oracle import build
build.LIB = sys.argv[1]
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                      "-W", "ignore::RuntimeWarning"] + sys.argv[2:]))
"""


def build_and_run(tmpdir, name, text):
    src = os.path.join(tmpdir, name + ".cpp")
    lib = os.path.join(tmpdir, "liboracle_" + name + ".so")
    with open(src, "w") as f:
        f.write(text)
    subprocess.run(["g++", "-std=c++17", "-O1", "-ffp-contract=off", "-fno-fast-math",
                    "-fopenmp", "-fPIC", "-shared", "-o", lib, src, "-lquadmath"],
                   check=True, timeout=300, capture_output=True)
    # (alphabetical order, which reaches a failing test fastest for most mutants: the
    # quad-precision table pin is slow when it has to run in full)
    tests = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    env = dict(os.environ, OMP_NUM_THREADS="2")
    try:
        r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT), lib] + tests,
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    except subprocess.TimeoutExpired:
        return name, None, "timed out"
    failed = [l for l in r.stdout.splitlines() if l.startswith("FAILED")]
    return name, r.returncode, failed[0] if failed else r.stdout[-300:]


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin(tmp_path):
    text = open(SRC).read()
    jobs = [("control", text)]
    for name, _, old, new in MUTANTS:
        assert old in text, "mutation site missing: " + name
        jobs.append((name, text.replace(old, new)))  # every occurrence
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        results = {n: (rc, msg) for n, rc, msg in
                   ex.map(lambda j: build_and_run(str(tmp_path), *j), jobs)}
    rc, msg = results.pop("control")
    assert rc == 0, "the unmutated oracle must pass its pins: " + str(msg)
    survivors = []
    for name, what, _, _ in MUTANTS:
        rc, msg = results[name]
        print("[mutant] %-18s %-70s caught by: %s" % (name, what, msg))
        if rc == 0:
            survivors.append(name)
    assert not survivors, "planted mistakes no pin catches: %s" % survivors
