// Outer-iteration stop rule of the all-at-once solve (the control step of
// every sweep), as a pure function: the control kernel calls it once per
// sweep, and host test drivers call it on given sequences.
//
// Sweep k (0-based) has the update norm upd = max_n ||delta_n||_2, the
// iterate norm unrm = max_n ||u_n||_2, the residual norm res =
// max_n ||r_n||_2 of the iterate it started from, and the scalar averaged
// Jacobian c_bar of the new iterate.  With rel = upd / unrm and
// rho = upd / upd_prev, the error estimate is est = rho / (1 - rho) rel
// (k >= 1, rho < 1).  The loop stops
//   diverged  on NaN / Inf (any of upd, unrm, c_bar), or when the update has grown 1e3-fold over the
//             first one (k >= 2);
//   converged when est <= safety rtol and res has not grown over the previous
//             sweep's, or when rel <= 1e-3 rtol; in the unrefined mode also
//             when the update stops contracting (upd > upd_prev / 2, k >= 2);
//   out of iterations after max_iter sweeps.
#pragma once

#include "pint.h"

namespace pint {

struct StopIn {
  int k;              // index of the sweep just finished
  double upd, unrm, res;
  double cbar;        // the sweep's scalar averaged Jacobian (checked for NaN)
  double upd_prev;    // previous sweep's upd (k >= 1)
  double upd_first;   // sweep 0's upd (k >= 1)
  double res_prev;    // previous sweep's res; negative: not available
  double rtol, safety;
  int stagnate, max_iter;
};

struct StopOut {
  int status;  // PINT_OK / PINT_ENOCONV / PINT_EDIVERGED (meaningful when done)
  int done;
  double est, rel;
};

__host__ __device__ inline StopOut stop_rule(const StopIn& s) {
  StopOut o{PINT_OK, 0, 1e300, 0.0};
  const int k = s.k;
  o.rel = s.unrm > 0.0 ? s.upd / s.unrm : s.upd;
  const bool bad =
      !(s.upd == s.upd) || !(s.unrm == s.unrm) || !(s.cbar == s.cbar) || s.upd > 1e300 || s.unrm > 1e300;
  if (k >= 1 && s.upd_prev > 0.0) {
    const double rho = s.upd / s.upd_prev;
    if (rho < 1.0) o.est = rho / (1.0 - rho) * o.rel;
  }
  if (s.upd == 0.0) o.est = 0.0;
  const double upd_first = k == 0 ? s.upd : s.upd_first;
  const bool res_ok = k == 0 || s.res_prev < 0.0 || !(s.res > s.res_prev);
  if (bad || (k >= 2 && s.upd > 1e3 * upd_first)) {
    o.status = PINT_EDIVERGED;
    o.done = 1;
  } else if ((o.est <= s.safety * s.rtol && res_ok) || o.rel <= 1e-3 * s.rtol) {
    o.status = PINT_OK;
    o.done = 1;
  } else if (s.stagnate && k >= 2 && s.upd_prev > 0.0 && s.upd > 0.5 * s.upd_prev) {
    // unrefined mode: the update stopped contracting, the iterate sits on its
    // working-precision plateau
    o.status = PINT_OK;
    o.done = 1;
  } else if (k + 1 >= s.max_iter) {
    o.status = PINT_ENOCONV;
    o.done = 1;
  }
  return o;
}

}  // namespace pint
