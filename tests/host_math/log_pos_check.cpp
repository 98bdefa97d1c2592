// Reads doubles (one hex float per line) and prints efm::log_pos of each
// (hex float per line): the host build of the logarithm the monitor kernels use.
#include <cstdio>
#include <cstdlib>

#include "logpos.h"

int main() {
  char buf[128];
  while (std::fgets(buf, sizeof buf, stdin)) {
    const double x = std::strtod(buf, nullptr);
    std::printf("%a\n", efm::log_pos(x));
  }
  return 0;
}
