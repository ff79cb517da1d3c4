// hlbm_stop.hpp -- the stop rule of the adjoint iteration (Algorithm 1: the
// adjoint runs until its variables reach a steady state).  Plain host C++,
// no HIP types, so that the rule can be checked on its own.
#pragma once

#include <cmath>

namespace hlbm {

enum StopDecision { STOP_CONTINUE = 0, STOP_CONVERGED = 1, STOP_DIVERGED = 2 };

// One residual check: dmax = max|phi_k - phi_(k-M)|, pmax = max|phi_k|.  The
// relative residual dmax / pmax (dmax alone while phi is still zero) is
// written to *res.  Converged when it is at most tol.  Diverged when either
// value is not finite, or when the residual has grown past 1e3 times the
// smallest residual of this solve (*min_res, updated here; start it at
// +infinity): a solve that had settled and then departs by three orders of
// magnitude is not heading for the steady state.
inline StopDecision adjoint_stop(double dmax, double pmax, double tol, double* min_res, double* res) {
  if (!std::isfinite(dmax) || !std::isfinite(pmax)) return STOP_DIVERGED;
  const double r = pmax > 0.0 ? dmax / pmax : dmax;
  *res = r;
  if (r <= tol) return STOP_CONVERGED;
  if (r > 1e3 * *min_res) return STOP_DIVERGED;
  if (r < *min_res) *min_res = r;
  return STOP_CONTINUE;
}

}  // namespace hlbm
