// Host driver of the outer-iteration stop rule (csrc/stop_rule.hpp, the
// function the control kernel calls): reads one sweep per line,
//   upd unrm res c_bar
// after a header line "rtol safety stagnate max_iter", applies the rule with
// the same bookkeeping as the control kernel (previous update and residual,
// first update), and prints "k status done est" for every sweep until the
// rule stops the loop.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "stop_rule.hpp"

int main() {
  double rtol, safety;
  int stagnate, max_iter;
  if (std::scanf("%lf %lf %d %d", &rtol, &safety, &stagnate, &max_iter) != 4) return 2;
  double upd, unrm, res, cbar, upd_prev = 0.0, upd_first = 0.0, res_prev = -1.0;
  for (int k = 0; std::scanf("%lf %lf %lf %lf", &upd, &unrm, &res, &cbar) == 4; ++k) {
    pint::StopIn s{};
    s.k = k;
    s.upd = upd;
    s.unrm = unrm;
    s.res = res;
    s.cbar = cbar;
    s.upd_prev = upd_prev;
    s.upd_first = upd_first;
    s.res_prev = k >= 1 ? res_prev : -1.0;
    s.rtol = rtol;
    s.safety = safety;
    s.stagnate = stagnate;
    s.max_iter = max_iter;
    const pint::StopOut o = pint::stop_rule(s);
    std::printf("%d %d %d %.17g\n", k, o.status, o.done, o.est);
    if (o.done) break;
    if (k == 0) upd_first = upd;
    upd_prev = upd;
    res_prev = res;
  }
  return 0;
}
