"""The FP64 fold's sin/cos pair (csrc/fastmath.hpp, host-compilable) against
the C library, over the phase range the engine uses and on special points.
Its polynomial error bound (1e-12) sits three orders of magnitude inside the
1e-9 agreement the FP64 mode is held to."""
import os
import subprocess
import sys

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2502_15253_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include <cmath>
#include "fastmath.hpp"
int main() {
  double xs;
  while (std::scanf("%lf", &xs) == 1) {
    double s, c;
    nufold::sincos_fold(xs, s, c);
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


def run(exe, xs):
    out = subprocess.run([exe], input="\n".join(repr(float(x)) for x in xs), capture_output=True, text=True,
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
