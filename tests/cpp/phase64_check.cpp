// Host check of the float64 near-field sine/cosine against the C library
// (long double) over the argument range of the near field and beyond.
#include <cmath>
#include <cstdio>

#include "../../paper_1606_02383_amd/csrc/phase64.h"

int main() {
  double worst_s = 0, worst_c = 0, at_s = 0, at_c = 0;
  const int n = 2000001;
  for (int i = 0; i < n; ++i) {
    const double x = -200.0 + 400.0 * i / (n - 1);
    double s, c;
    bemfmm::sincos_reduced(x, &s, &c);
    const long double rs = sinl((long double)x), rc = cosl((long double)x);
    const double es = (double)fabsl((long double)s - rs), ec = (double)fabsl((long double)c - rc);
    if (es > worst_s) worst_s = es, at_s = x;
    if (ec > worst_c) worst_c = ec, at_c = x;
  }
  // quadrant boundaries and tiny arguments
  const double special[] = {0.0, 1e-300, -1e-300, 1e-8, M_PI / 4, M_PI / 2, M_PI, 1.5 * M_PI,
                            2 * M_PI, -M_PI / 2, -M_PI, 100 * M_PI};
  for (double x : special) {
    double s, c;
    bemfmm::sincos_reduced(x, &s, &c);
    const double es = (double)fabsl((long double)s - sinl((long double)x));
    const double ec = (double)fabsl((long double)c - cosl((long double)x));
    if (es > worst_s) worst_s = es, at_s = x;
    if (ec > worst_c) worst_c = ec, at_c = x;
  }
  printf("max |sin error| %.3e at %.6f, max |cos error| %.3e at %.6f\n", worst_s, at_s, worst_c,
         at_c);
  return (worst_s < 5e-16 && worst_c < 5e-16) ? 0 : 1;
}
