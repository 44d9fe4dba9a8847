// mpt_window.h -- how long a kernel launch of the R16 step may be.  Plain
// C++ (host side of the library, and host tests).
#pragma once
#include <cmath>

namespace mpt {

// R16 storage: the times a launch of nsteps steps reads, t0 .. t0 +
// (nsteps - 1/2) dt, must span less than one met interval (with a margin
// far above rounding), so that its earlier met level moves by at most one
// and the three-level scale window of the step kernels covers it.
inline bool r16_launch_fits(int nsteps, double dt, double dt_met) {
  return nsteps >= 1 && ((double)nsteps - 0.5) * dt <= 0.999 * dt_met;
}

// The longest such launch; 0 when not even one step fits.
inline int r16_max_launch(double dt, double dt_met) {
  const double x = std::floor(0.999 * dt_met / dt + 0.5);
  int n = x > 1e9 ? 1000000000 : x < 0 ? 0 : (int)x;
  while (n > 0 && !r16_launch_fits(n, dt, dt_met)) --n;
  return n;
}

}  // namespace mpt
