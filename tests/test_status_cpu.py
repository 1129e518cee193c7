"""Convergence verdicts of the solvers with residuals that are not finite
(host logic, compiled here with the system C++ compiler; no GPU).

A NaN or infinite residual must never count as converged, and the worst
residual reported over several systems must keep a NaN (std::max would drop
it).  The GMRES driver, the refinement loop, the transient Newton loop and
the serving rounds all take their verdicts from these functions."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2305_06891_amd", "csrc", "convergence.hpp")

PROG = r"""
#include <cmath>
#include <cstdio>
#include <limits>
#include "convergence.hpp"
int main() {
  using namespace hm;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  const double inf = std::numeric_limits<double>::infinity();
  int bad = 0;
  bad += !(std::isnan(rel_residual(nan, 1.0)));
  bad += !(std::isnan(rel_residual(1.0, nan)));
  bad += !(std::isnan(rel_residual(inf, 1.0)));
  bad += !(rel_residual(0.0, 0.0) == 0.0);
  bad += !(rel_residual(2.0, 4.0) == 0.5);
  bad += !(std::isinf(rel_residual(1.0, 0.0)));
  bad += residual_met(nan, 1.0, 1e-6);
  bad += residual_met(inf, 1.0, 1e-6);
  bad += residual_met(1e-7, nan, 1e-6);
  bad += !residual_met(1e-7, 1.0, 1e-6);
  bad += residual_met(2e-6, 1.0, 1e-6);
  bad += !(std::isnan(max_keep_nan(0.0, nan)));
  bad += !(std::isnan(max_keep_nan(nan, 3.0)));
  bad += !(max_keep_nan(1.0, 3.0) == 3.0 && max_keep_nan(3.0, 1.0) == 3.0);
  bad += rel_met(nan, 1e-6);
  bad += !rel_met(1e-7, 1e-6);
  // the worst of several systems keeps the NaN wherever it sits
  double w = 0.0;
  const double rs[4] = {1e-9, nan, 1e-8, 1e-10};
  for (double r : rs) w = max_keep_nan(w, r);
  bad += !std::isnan(w);
  bad += rel_met(w, 1.0);
  std::printf("%d\n", bad);
  return bad == 0 ? 0 : 1;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_nonfinite_residuals_never_converge(tmp_path):
    src = tmp_path / "t.cpp"
    src.write_text(PROG)
    exe = tmp_path / "t"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", os.path.dirname(HDR), str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr


def test_solvers_take_their_verdicts_from_the_shared_tests():
    """The comparisons that decided convergence with plain `<=`/`>` (false
    for NaN) are gone from the solver sources."""
    csrc = os.path.join(ROOT, "paper_2305_06891_amd", "csrc")
    for name, needle in (("krylov.hip", "rel_residual("), ("solve.hip", "residual_met("),
                         ("server.hip", "residual_met("), ("api.hip", "max_keep_nan(")):
        with open(os.path.join(csrc, name)) as fh:
            assert needle in fh.read(), name
