// SU(2) recoupling coefficients used by the GPU path.
//
// The paper evaluates all spin recoupling through Wigner 6j and 9j symbols and
// never through Clebsch-Gordan coefficients (section "Reduced MPS tensors").
// This file does the same: Racah's single-sum formula for the 6j symbol and
// the 9j symbol as a sum over products of three 6j symbols.  Spins are doubled.
//
// Reduced matrix elements follow <j' m'|T^k_q|j m> = <j m; k q|j' m'> <j'||T||j>
// (ket spin first, as in the paper's eq. tensordecomp).  With that convention:
//   * a product of operators on two subsystems (A on the first, B on the second)
//     <(j1' j2')J'||[A^k1 x B^k2]^K||(j1 j2)J> =
//        sqrt((2J+1)(2K+1)(2j1'+1)(2j2'+1)) {j1' j1 k1; j2' j2 k2; J' J K}
//        <j1'||A||j1> <j2'||B||j2>
//   * a product on one space (V first): coefficient of <j'||U||j''><j''||V||j>
//        (-1)^(K+j+j') sqrt((2K+1)(2j''+1)) {k1 k2 K; j j' j''}
//   * the conjugate tensor Tbar_q = (-1)^(k-q) (T_{-q})^dagger has
//        <j||Tbar||j'> = (-1)^(j'+k-j) sqrt((2j'+1)/(2j+1)) <j'||T||j>
//   * singlet recoupling <[a (x) [s (x) b]^a]^0 | [[a (x) s]^b (x) b]^0>
//        = (-1)^(a+s+b) sqrt((2a+1)(2b+1)) {a s b; b 0 a}
#include <cmath>
#include <cstdint>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "engine.h"

namespace sadmrg {

bool triangle(int a, int b, int c) { return c >= std::abs(a - b) && c <= a + b && ((a + b + c) & 1) == 0; }

static double fact(int n) {
  static const std::vector<double> f = [] {
    std::vector<double> v(171);
    v[0] = 1.0;
    for (int i = 1; i < 171; ++i) v[i] = v[i - 1] * i;
    return v;
  }();
  return f[n];
}

static double tri_delta(int a, int b, int c) {
  return std::sqrt(fact((a + b - c) / 2) * fact((a - b + c) / 2) * fact((-a + b + c) / 2) / fact((a + b + c) / 2 + 1));
}

double sixj(int a, int b, int c, int d, int e, int f) {
  if (!triangle(a, b, c) || !triangle(a, e, f) || !triangle(d, b, f) || !triangle(d, e, c)) return 0.0;
  const double pre = tri_delta(a, b, c) * tri_delta(a, e, f) * tri_delta(d, b, f) * tri_delta(d, e, c);
  const int lo = std::max(std::max(a + b + c, a + e + f), std::max(d + b + f, d + e + c));
  const int hi = std::min(std::min(a + b + d + e, a + c + d + f), b + c + e + f);
  double s = 0.0;
  for (int tt = lo; tt <= hi; tt += 2) {
    const int t = tt / 2;
    const double den = fact((tt - a - b - c) / 2) * fact((tt - a - e - f) / 2) * fact((tt - d - b - f) / 2) *
                       fact((tt - d - e - c) / 2) * fact((a + b + d + e - tt) / 2) * fact((a + c + d + f - tt) / 2) *
                       fact((b + c + e + f - tt) / 2);
    s += ((t & 1) ? -1.0 : 1.0) * fact(t + 1) / den;
  }
  return pre * s;
}

double ninej(int a, int b, int c, int d, int e, int f, int g, int h, int i) {
  const int lo = std::max(std::max(std::abs(a - i), std::abs(d - h)), std::abs(b - f));
  const int hi = std::min(std::min(a + i, d + h), b + f);
  double s = 0.0;
  for (int x = lo; x <= hi; x += 2) {
    const double t = sixj(a, b, c, f, i, x) * sixj(d, e, f, b, x, h) * sixj(g, h, i, x, a, d);
    s += ((x & 1) ? -1.0 : 1.0) * (x + 1) * t;
  }
  return s;
}

double coupling_product(int tj1, int tj2, int tJ, int tk1, int tk2, int tK, int tj1p, int tj2p, int tJp) {
  if (!triangle(tj1, tj2, tJ) || !triangle(tj1p, tj2p, tJp) || !triangle(tk1, tk2, tK) || !triangle(tj1, tk1, tj1p) ||
      !triangle(tj2, tk2, tj2p) || !triangle(tJ, tK, tJp))
    return 0.0;
  // memo per host thread: engines of a batch prepare their steps in parallel
  static thread_local std::unordered_map<uint64_t, double> cache;
  uint64_t key = 0;
  for (int v : {tj1, tj2, tJ, tk1, tk2, tK, tj1p, tj2p, tJp}) key = key * 64 + (uint64_t)v;
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const double v = std::sqrt((double)(tJ + 1) * (tK + 1) * (tj1p + 1) * (tj2p + 1)) *
                   ninej(tj1p, tj1, tk1, tj2p, tj2, tk2, tJp, tJ, tK);
  cache.emplace(key, v);
  return v;
}

double coupling_same(int tj, int tjm, int tjp, int tk1, int tk2, int tK) {
  if (!triangle(tj, tk2, tjm) || !triangle(tjm, tk1, tjp) || !triangle(tk1, tk2, tK) || !triangle(tj, tK, tjp))
    return 0.0;
  const int e = (tK + tj + tjp) / 2;
  return ((e & 1) ? -1.0 : 1.0) * std::sqrt((double)(tK + 1) * (tjm + 1)) * sixj(tk1, tk2, tK, tj, tjp, tjm);
}

double coupling_singlet(int tj, int tjp, int tk) { return coupling_product(tj, tj, 0, tk, tk, 0, tjp, tjp, 0); }

double recouple_singlet(int ta, int ts, int tb) {
  const int e = (ta + ts + tb) / 2;
  return ((e & 1) ? -1.0 : 1.0) * std::sqrt((double)(ta + 1) * (tb + 1)) * sixj(ta, ts, tb, tb, 0, ta);
}

double adjoint_factor(int tj_bra, int tj_ket, int tk) {
  const int e = (tj_bra + tk - tj_ket) / 2;
  return ((e & 1) ? -1.0 : 1.0) * std::sqrt((double)(tj_bra + 1) / (tj_ket + 1));
}

}  // namespace sadmrg
