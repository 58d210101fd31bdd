"""The FP64 sin/cos pairs (csrc/fastmath.hpp, host-compilable): the
polynomial pair (sincos_fold) against the C library, over the phase range the
engine uses and on special points; its error bound (1e-12) sits three orders
of magnitude inside the 1e-9 agreement the FP64 mode is held to. The
table-driven pair of the FP64 event folds (sincos_tab) against 40-digit
values (mpmath) of sin and cos of 2 pi y / TAB_N for the same y, and against
the C library for phases in radians."""
import os
import subprocess
import sys

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2502_15253_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include <cstring>
#include <cmath>
#include "fastmath.hpp"
int main(int argc, char** argv) {
  // "tab": sincos_tab of y; "rad": sincos_tab of x TAB_PER_RAD; else sincos_fold of x
  const int mode = argc > 1 ? (std::strcmp(argv[1], "tab") == 0 ? 1 : 2) : 0;
  double xs;
  while (std::scanf("%lf", &xs) == 1) {
    double s, c;
    if (mode == 0) nufold::sincos_fold(xs, s, c);
    else nufold::sincos_tab(mode == 1 ? xs : xs * nufold::TAB_PER_RAD, nufold::SINCOS_TAB, s, c);
    std::printf("%.17g %.17g %.17g %.17g\n", s, c, std::sin(xs), std::cos(xs));
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def binary(tmp_path_factory):
    d = tmp_path_factory.mktemp("fastmath")
    src = d / "t.cpp"
    src.write_text(PROGRAM)
    exe = d / "t"
    r = subprocess.run(["g++", "-O2", "-std=c++20", "-ffp-contract=off", f"-I{CSRC}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("g++ could not build the host copy: " + r.stderr[-300:])
    return str(exe)


def run(exe, xs, mode=None):
    out = subprocess.run([exe] + ([mode] if mode else []), input="\n".join(repr(float(x)) for x in xs), capture_output=True, text=True,
                         check=True).stdout
    return np.array([[float(v) for v in ln.split()] for ln in out.strip().splitlines()])


def test_sincos_error_bound_over_phase_range(binary):
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.uniform(-1e4, 1e4, 20000), rng.uniform(-10, 10, 20000),
                         np.arange(-64, 65) * np.pi / 4, [0.0, 1e-300, -1e-300, np.pi, -np.pi]])
    r = run(binary, xs)
    assert np.max(np.abs(r[:, 0] - r[:, 2])) < 1e-12
    assert np.max(np.abs(r[:, 1] - r[:, 3])) < 1e-12


def test_sincos_pythagoras_and_symmetry(binary):
    xs = np.linspace(-300.0, 300.0, 6001)
    r = run(binary, np.concatenate([xs, -xs]))
    n = len(xs)
    s, c = r[:n, 0], r[:n, 1]
    assert np.max(np.abs(s * s + c * c - 1.0)) < 3e-12
    assert np.array_equal(r[n:, 0], -s) and np.array_equal(r[n:, 1], c)


def test_table_pair_against_high_precision(binary):
    """sincos_tab(y) = sin, cos of 2 pi y / 256 to 1e-15 absolute, for y over
    the range of the engine's phases (|x| < 1e4 rad), near table points and
    half-way between them (the ends of the polynomials' interval), and for
    negative y (inverted mass ordering)."""
    import mpmath as mp
    mp.mp.dps = 40
    rng = np.random.default_rng(12)
    ys = np.concatenate([rng.uniform(-4.1e5, 4.1e5, 3000), rng.uniform(-300.0, 300.0, 3000),
                         np.arange(-600, 601) * 0.5, np.arange(-600, 601) * 0.5 + 1e-9,
                         np.arange(0, 256) + 0.4999999999, [0.0, 1e-300, -1e-300]])
    r = run(binary, ys, "tab")
    k = 2 * mp.pi / 256
    es = max(abs(float(mp.sin(k * mp.mpf(float(y))) - mp.mpf(float(v)))) for y, v in zip(ys, r[:, 0]))
    ec = max(abs(float(mp.cos(k * mp.mpf(float(y))) - mp.mpf(float(v)))) for y, v in zip(ys, r[:, 1]))
    assert es < 1e-15 and ec < 1e-15, (es, ec)


def test_table_pair_table_points_and_radians(binary):
    # whole y: the table's values, which are sin and cos of 2 pi i / 256
    # correctly rounded (40-digit values rounded once)
    import mpmath as mp
    mp.mp.dps = 40
    ys = np.arange(-512, 513).astype(float)
    r = run(binary, ys, "tab")
    want = np.array([[float(mp.sinpi(mp.mpf(int(y) % 256) / 128)), float(mp.cospi(mp.mpf(int(y) % 256) / 128))]
                     for y in ys])
    assert np.array_equal(r[:, :2], want)
    # phases in radians: the rounding of x TAB_PER_RAD adds about 1.1e-16 |x|
    rng = np.random.default_rng(13)
    xs = np.concatenate([rng.uniform(-1e4, 1e4, 20000), rng.uniform(-10, 10, 20000)])
    r = run(binary, xs, "rad")
    bound = 1e-15 + 3e-16 * np.abs(xs)
    assert np.all(np.abs(r[:, 0] - r[:, 2]) < bound) and np.all(np.abs(r[:, 1] - r[:, 3]) < bound)
    assert np.max(np.abs(r[:, 0] ** 2 + r[:, 1] ** 2 - 1.0)) < 1e-15
