// Host driver for the launch limit of the R16 step: reads (dt, dt_met)
// pairs as raw doubles from stdin, writes (n, fits(n), fits(n + 1)) per pair
// as raw doubles, n = r16_max_launch(dt, dt_met).
#include <cstdio>
#include <vector>

#include "mpt_window.h"

int main() {
  std::vector<double> x;
  double buf[4096];
  size_t got;
  while ((got = fread(buf, sizeof(double), 4096, stdin)) > 0) x.insert(x.end(), buf, buf + got);
  if (x.size() % 2) return 2;
  std::vector<double> y;
  for (size_t i = 0; i < x.size(); i += 2) {
    const int n = mpt::r16_max_launch(x[i], x[i + 1]);
    y.push_back((double)n);
    y.push_back(mpt::r16_launch_fits(n, x[i], x[i + 1]) ? 1.0 : 0.0);
    y.push_back(mpt::r16_launch_fits(n + 1, x[i], x[i + 1]) ? 1.0 : 0.0);
  }
  fwrite(y.data(), sizeof(double), y.size(), stdout);
  return 0;
}
