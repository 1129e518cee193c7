// Convergence tests of the solvers (host code, no device headers): a
// residual that is not finite never counts as converged, and a maximum over
// residuals keeps a NaN instead of dropping it.
#pragma once

#include <cmath>
#include <limits>

namespace hm {

// |r|_2 / |b|_2, NaN when either norm is not finite; 0 for b = 0 and r = 0
// (a zero right-hand side is solved exactly by a zero start).
inline double rel_residual(double rn, double bn) {
  if (!std::isfinite(rn) || !std::isfinite(bn)) return std::numeric_limits<double>::quiet_NaN();
  if (bn > 0) return rn / bn;
  return rn == 0.0 ? 0.0 : std::numeric_limits<double>::infinity();
}

// |r| <= rtol |b| with both norms finite.
inline bool residual_met(double rn, double bn, double rtol) {
  return std::isfinite(rn) && std::isfinite(bn) && rn <= rtol * bn;
}

// max(acc, v) that propagates NaN from either side.
inline double max_keep_nan(double acc, double v) {
  if (std::isnan(acc)) return acc;
  if (std::isnan(v)) return v;
  return v > acc ? v : acc;
}

// A relative residual that met the tolerance (false for NaN).
inline bool rel_met(double rel, double rtol) { return rel <= rtol; }

}  // namespace hm
