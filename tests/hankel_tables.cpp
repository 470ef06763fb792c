// Host harness for the translation-table Bessel functions: prints
// z, then k s^t j_t(z) and k s^t y_t(z) for t = 0..10 (k = s = 1, w = z).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1806_04164_amd/csrc/pie_internal.h"

int main(int argc, char** argv) {
  for (int i = 1; i < argc; ++i) {
    const double z = std::atof(argv[i]);
    std::vector<double> o;
    pie::scaled_hankel(1.0, 1.0, z, 10, o);
    std::printf("%.17g", z);
    for (int t = 0; t <= 10; ++t) std::printf(" %.17g %.17g", o[2 * t], o[2 * t + 1]);
    std::printf("\n");
  }
  return 0;
}
