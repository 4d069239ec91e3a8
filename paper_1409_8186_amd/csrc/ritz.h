// Host-side helpers of s-step GMRES: the eigenvalues of a small complex upper
// Hessenberg matrix (the Ritz values of an Arnoldi cycle) by the shifted QR
// algorithm, and their Leja ordering, which spaces the shifts of a Newton
// Krylov basis v_i = (A - theta_i) v_{i-1} so that the basis stays well
// conditioned.  Plain C++ (std::complex), no device code.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace ritz {

using cd = std::complex<double>;

// Eigenvalues of the n x n upper Hessenberg matrix H (column-major, leading
// dimension ld; entries below the subdiagonal are ignored).  Single-shift QR
// with Wilkinson shifts and deflation at negligible subdiagonals; an
// exceptional shift every 10 iterations without deflation.  Returns false (and
// the current diagonal for the undeflated part) after 60 n iterations.
inline bool hessenberg_eigenvalues(int n, const cd* Hin, int ld, std::vector<cd>& ev) {
  ev.clear();
  if (n <= 0) return true;
  std::vector<cd> H((size_t)n * n);
  auto h = [&](int r, int c) -> cd& { return H[(size_t)c * n + r]; };
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < n; ++r) h(r, c) = r <= c + 1 ? Hin[(size_t)c * ld + r] : cd(0.0);
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, iter = 0, total = 0;
  bool ok = true;
  std::vector<double> cs(n);
  std::vector<cd> sn(n);
  while (hi >= 0) {
    if (hi == 0) {
      ev.push_back(h(0, 0));
      break;
    }
    int l = hi;
    while (l > 0) {
      const double scale = std::abs(h(l, l)) + std::abs(h(l - 1, l - 1));
      if (std::abs(h(l, l - 1)) <= eps * (scale > 0.0 ? scale : 1.0)) break;
      --l;
    }
    if (l == hi) {  // h(hi, hi) has split off
      ev.push_back(h(hi, hi));
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 60 * n) {
      ok = false;
      for (int k = hi; k >= 0; --k) ev.push_back(h(k, k));
      break;
    }
    // shift: eigenvalue of the trailing 2 x 2 block closer to its last entry
    cd mu;
    if (++iter % 10 == 0) {
      mu = h(hi, hi) + std::abs(h(hi, hi - 1));
    } else {
      const cd a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
      const cd half = 0.5 * (a - d);
      const cd disc = std::sqrt(half * half + b * c);
      const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
      mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    }
    // explicit shifted QR step on the active block l..hi: H - mu = QR, H <- RQ + mu
    for (int k = l; k <= hi; ++k) h(k, k) -= mu;
    for (int k = l; k < hi; ++k) {
      const cd x = h(k, k), y = h(k + 1, k);
      double c;
      cd s;
      if (std::abs(y) == 0.0) {
        c = 1.0;
        s = 0.0;
      } else if (std::abs(x) == 0.0) {
        c = 0.0;
        s = 1.0;
      } else {
        const double nx = std::abs(x), r = std::hypot(nx, std::abs(y));
        c = nx / r;
        s = (x / nx) * std::conj(y) / r;
      }
      cs[k] = c;
      sn[k] = s;
      for (int j = k; j <= hi; ++j) {  // rows k, k+1: [c s; -conj(s) c]
        const cd u = h(k, j), v = h(k + 1, j);
        h(k, j) = c * u + s * v;
        h(k + 1, j) = -std::conj(s) * u + c * v;
      }
    }
    for (int k = l; k < hi; ++k) {  // columns k, k+1 times the conjugate transpose
      const double c = cs[k];
      const cd s = sn[k];
      const int rmax = std::min(k + 2, hi);
      for (int i = l; i <= rmax; ++i) {
        const cd u = h(i, k), v = h(i, k + 1);
        h(i, k) = c * u + std::conj(s) * v;
        h(i, k + 1) = -s * u + c * v;
      }
    }
    for (int k = l; k <= hi; ++k) h(k, k) += mu;
  }
  return ok;
}

// s values picked from `vals` in Leja order: the one of largest modulus first,
// then each maximising the product of its distances to those already picked
// (a value equal to a picked one is not picked again).  With fewer distinct
// values than s, the order repeats from the start.
inline std::vector<cd> leja(const std::vector<cd>& vals, int s) {
  std::vector<cd> out;
  if (vals.empty() || s <= 0) return out;
  std::vector<char> used(vals.size(), 0);
  while ((int)out.size() < s) {
    int best = -1;
    double bestv = -1.0;
    for (size_t i = 0; i < vals.size(); ++i) {
      if (used[i]) continue;
      double v = 0.0;
      if (out.empty()) {
        v = std::abs(vals[i]);
      } else {
        // log of the product of distances (no overflow for many factors)
        bool dup = false;
        for (const cd& t : out) {
          const double d = std::abs(vals[i] - t);
          if (d == 0.0) dup = true;
          v += std::log(d > 0.0 ? d : 1e-300);
        }
        if (dup) continue;
        v += 1e6;  // keep any candidate above the -1 of "none"
      }
      if (v > bestv) {
        bestv = v;
        best = (int)i;
      }
    }
    if (best < 0) {  // nothing left: repeat the order so far
      const size_t k = out.size();
      for (size_t i = 0; (int)out.size() < s; ++i) out.push_back(out[i % k]);
      break;
    }
    used[best] = 1;
    out.push_back(vals[best]);
  }
  return out;
}

// Scale of each Newton step (A - theta_i) / sigma_i: sigma_i = max_k
// |vals_k - theta_i|, the largest factor the step applies to an eigenvector
// the Ritz values stand for, so the scaled basis keeps norms near one.  1 when
// that is zero or not finite.
inline std::vector<double> newton_scales(const std::vector<cd>& vals, const std::vector<cd>& shifts) {
  std::vector<double> sg(shifts.size(), 1.0);
  for (size_t i = 0; i < shifts.size(); ++i) {
    double mx = 0.0;
    for (const cd& v : vals) mx = std::max(mx, std::abs(v - shifts[i]));
    if (mx > 0.0 && std::isfinite(mx)) sg[i] = mx;
  }
  return sg;
}

}  // namespace ritz
