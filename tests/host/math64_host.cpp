// Host driver for the FP64 step functions: reads raw doubles from stdin,
// applies the function named by argv[1], writes raw doubles (two per input
// for sincospi, one per input pair for div) to stdout.
#include <cstdio>
#include <cstring>
#include <vector>

#include "mpt_math.h"

int main(int argc, char **argv) {
  if (argc != 2) return 2;
  std::vector<double> x;
  double buf[4096];
  size_t got;
  while ((got = fread(buf, sizeof(double), 4096, stdin)) > 0) x.insert(x.end(), buf, buf + got);
  std::vector<double> y;
  for (double v : x) {
    if (!strcmp(argv[1], "ln")) {
      y.push_back(mpt::m64::ln_pos(v));
    } else if (!strcmp(argv[1], "sqrt")) {
      y.push_back(mpt::m64::sqrt_pos(v));
    } else if (!strcmp(argv[1], "coslat")) {
      y.push_back(mpt::m64::cos_lat_deg(v));
    } else if (!strcmp(argv[1], "sincospi")) {
      double s, c;
      mpt::m64::sincospi_02(v, &s, &c);
      y.push_back(s);
      y.push_back(c);
    } else if (!strcmp(argv[1], "cospi")) {
      y.push_back(mpt::m64::cospi_02(v));
    } else if (strcmp(argv[1], "div")) {
      return 2;
    }
  }
  if (!strcmp(argv[1], "div")) {            // pairs (a, b) -> a / b
    y.clear();
    for (size_t q = 0; q + 1 < x.size(); q += 2) y.push_back(mpt::m64::div_1to4(x[q], x[q + 1]));
  }
  fwrite(y.data(), sizeof(double), y.size(), stdout);
  return 0;
}
