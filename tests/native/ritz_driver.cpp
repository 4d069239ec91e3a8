// Reads complex upper Hessenberg matrices from stdin ("n" then n*n entries
// "re im", column-major) and prints their eigenvalues (ritz.h), the Leja
// ordering of them ("s" leading values) and the scale of the Newton step of
// each of those shifts, for a comparison with numpy.
#include <cstdio>
#include <vector>

#include "ritz.h"

int main() {
  int n, s;
  while (std::scanf("%d %d", &n, &s) == 2) {
    std::vector<ritz::cd> H((size_t)n * n);
    for (auto& z : H) {
      double re, im;
      if (std::scanf("%lf %lf", &re, &im) != 2) return 2;
      z = ritz::cd(re, im);
    }
    std::vector<ritz::cd> ev;
    const bool ok = ritz::hessenberg_eigenvalues(n, H.data(), n, ev);
    std::printf("%d %zu\n", ok ? 1 : 0, ev.size());
    for (const auto& z : ev) std::printf("%.17g %.17g\n", z.real(), z.imag());
    const auto lj = ritz::leja(ev, s);
    for (const auto& z : lj) std::printf("%.17g %.17g\n", z.real(), z.imag());
    for (double v : ritz::newton_scales(ev, lj)) std::printf("%.17g\n", v);
  }
  return 0;
}
