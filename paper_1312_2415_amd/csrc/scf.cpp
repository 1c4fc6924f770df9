// DMRG-SCF: orbital optimisation around the DMRG active-space solver.
//
// Paper: arXiv:1312.2415 (CheMPS2), section "DMRG-SCF" of the library
// description: a state-specific complete-active-space self-consistent-field
// method with DMRG as the active-space solver; orbitals are doubly occupied
// (core), active or virtual per irrep; the orbitals are updated by the
// augmented-Hessian Newton-Raphson method with the exact Hessian until the
// orbital gradient drops below a threshold.  The active-space 1- and 2-RDMs
// come from the library's energy adjoint (section "CheMPS2 library", calc2DM).
//
// Conventions (real orbitals, chemist integrals g_pqrs = (pq|rs)):
//   D_pq = <E_pq>, d_pqrs = <E_pq E_rs - d_qr E_ps> = Gamma^A_{pr;qs},
//   E = e_nuc + sum h_pq D_pq + 1/2 sum g_pqrs d_pqrs;
//   orbital update phi'_p = sum_q phi_q R_qp, R = exp(-kappa), kappa
//   antisymmetric with parameters kappa_pq, p > q;
//   generalised Fock F_pq = sum_m D_pm h_qm + sum_mnt d_pmnt g_qmnt,
//   gradient dE/dkappa_pq = 2 (F_pq - F_qp),
//   Hessian (RDMs fixed) H_pq,rs = (1 - P_pq)(1 - P_rs) [2 D_pr h_qs
//     - (F_pr + F_rp) d_qs + 2 Y_pqrs],  Y_pqrs = sum_mn [(d_pmrn + d_pmnr)
//     g_qmsn + d_prmn g_qsmn]  (P_pq exchanges p and q).
// All of this is host arithmetic on L^2 to L^5 numbers; the DMRG solve and
// the RDMs run in the library's kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"

namespace sadmrg {

// h2 = R^T h R; g2_ijkl = sum_pqrs R_pi R_qj R_rk R_sl g_pqrs, one index at a time
void rotate_integrals(int L, const double* R, const double* h, const double* g, double* h2, double* g2) {
  const size_t L2 = (size_t)L * L, L3 = L2 * L, L4 = L3 * L;
  std::vector<double> t((size_t)L * L);
  for (int i = 0; i < L; ++i)
    for (int s = 0; s < L; ++s) {
      double v = 0.0;
      for (int p = 0; p < L; ++p) v += R[(size_t)p * L + i] * h[(size_t)p * L + s];
      t[(size_t)i * L + s] = v;
    }
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < L; ++j) {
      double v = 0.0;
      for (int s = 0; s < L; ++s) v += t[(size_t)i * L + s] * R[(size_t)s * L + j];
      h2[(size_t)i * L + j] = v;
    }
  // four passes; each transforms the leading index and rotates it to the back:
  // a[x][rest] -> b[rest][x'] with b = sum_x R_x x' a[x][rest]
  std::vector<double> a(g, g + L4), b(L4);
  for (int pass = 0; pass < 4; ++pass) {
    for (size_t rest = 0; rest < L3; ++rest)
      for (int xp = 0; xp < L; ++xp) {
        double v = 0.0;
        for (int x = 0; x < L; ++x) v += R[(size_t)x * L + xp] * a[(size_t)x * L3 + rest];
        b[rest * L + xp] = v;
      }
    a.swap(b);
  }
  std::copy(a.begin(), a.end(), g2);
}

// exp(A) of an antisymmetric A (Taylor series after scaling by 2^-s, then s
// squarings), re-orthonormalised column by column (modified Gram-Schmidt)
void expm_antisym(int L, const double* A, double* R) {
  const size_t n = (size_t)L * L;
  double nrm = 0.0;
  for (size_t i = 0; i < n; ++i) nrm = std::max(nrm, std::abs(A[i]));
  int s = 0;
  while (nrm * L > 0.25 && s < 60) {
    nrm *= 0.5;
    ++s;
  }
  const double sc = std::ldexp(1.0, -s);
  std::vector<double> X(n), T(n), E(n, 0.0), W(n);
  for (size_t i = 0; i < n; ++i) X[i] = A[i] * sc;
  for (int i = 0; i < L; ++i) E[(size_t)i * L + i] = 1.0;
  T = E;
  auto mul = [L](const std::vector<double>& P, const std::vector<double>& Q, std::vector<double>& out) {
    for (int i = 0; i < L; ++i)
      for (int j = 0; j < L; ++j) {
        double v = 0.0;
        for (int k = 0; k < L; ++k) v += P[(size_t)i * L + k] * Q[(size_t)k * L + j];
        out[(size_t)i * L + j] = v;
      }
  };
  for (int k = 1; k <= 18; ++k) {
    mul(T, X, W);
    for (size_t i = 0; i < n; ++i) T[i] = W[i] / k;
    for (size_t i = 0; i < n; ++i) E[i] += T[i];
  }
  for (int q = 0; q < s; ++q) {
    mul(E, E, W);
    E.swap(W);
  }
  for (int j = 0; j < L; ++j) {
    for (int k = 0; k < j; ++k) {
      double d = 0.0;
      for (int i = 0; i < L; ++i) d += E[(size_t)i * L + k] * E[(size_t)i * L + j];
      for (int i = 0; i < L; ++i) E[(size_t)i * L + j] -= d * E[(size_t)i * L + k];
    }
    double nn = 0.0;
    for (int i = 0; i < L; ++i) nn += E[(size_t)i * L + j] * E[(size_t)i * L + j];
    nn = 1.0 / std::sqrt(nn);
    for (int i = 0; i < L; ++i) E[(size_t)i * L + j] *= nn;
  }
  std::copy(E.begin(), E.end(), R);
}

// lowest eigenpair of a symmetric n x n matrix (cyclic Jacobi rotations)
static double lowest_eigenpair(int n, std::vector<double> A, std::vector<double>& vec) {
  std::vector<double> V((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double v = A[(size_t)i * n + j] * A[(size_t)i * n + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * std::max(tot, 1e-300)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (std::abs(apq) < 1e-300) continue;
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::abs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  int lo = 0;
  for (int i = 1; i < n; ++i)
    if (A[(size_t)i * n + i] < A[(size_t)lo * n + lo]) lo = i;
  vec.resize(n);
  for (int k = 0; k < n; ++k) vec[k] = V[(size_t)k * n + lo];
  return A[(size_t)lo * n + lo];
}

// Generalised Fock matrix, gradient over `pairs` (p > q) and, if hess is
// not null, the exact Hessian; occ lists the orbitals where D or d can be
// nonzero (core and active), which bounds every sum over m, n, t.
void orbital_derivatives(int L, const double* h, const double* g, const double* D, const double* d,
                         const std::vector<int>& occ, const std::vector<std::pair<int, int>>& pairs, double* F,
                         double* grad, double* hess) {
  auto G = [L, g](int p, int q, int r, int s) { return g[(((size_t)p * L + q) * L + r) * L + s]; };
  auto dd = [L, d](int p, int q, int r, int s) { return d[(((size_t)p * L + q) * L + r) * L + s]; };
  std::vector<double> Fl((size_t)L * L, 0.0);
  for (int p : occ)
    for (int q = 0; q < L; ++q) {
      double v = 0.0;
      for (int m : occ) v += D[(size_t)p * L + m] * h[(size_t)q * L + m];
      for (int m : occ)
        for (int n : occ)
          for (int t : occ) {
            const double x = dd(p, m, n, t);
            if (x != 0.0) v += x * G(q, m, n, t);
          }
      Fl[(size_t)p * L + q] = v;
    }
  if (F) std::copy(Fl.begin(), Fl.end(), F);
  const int np = (int)pairs.size();
  for (int a = 0; a < np; ++a) {
    const int p = pairs[a].first, q = pairs[a].second;
    grad[a] = 2.0 * (Fl[(size_t)p * L + q] - Fl[(size_t)q * L + p]);
  }
  if (!hess) return;
  auto Y = [&](int p, int q, int r, int s) {
    double v = 0.0;
    for (int m : occ)
      for (int n : occ) {
        const double x = dd(p, m, r, n) + dd(p, m, n, r), y = dd(p, r, m, n);
        if (x != 0.0) v += x * G(q, m, s, n);
        if (y != 0.0) v += y * G(q, s, m, n);
      }
    return v;
  };
  std::vector<char> isocc(L, 0);
  for (int m : occ) isocc[m] = 1;
  auto core = [&](int p, int q, int r, int s) {
    double v = 0.0;
    if (isocc[p] && isocc[r]) v += 2.0 * D[(size_t)p * L + r] * h[(size_t)q * L + s] + 2.0 * Y(p, q, r, s);
    if (q == s) v -= Fl[(size_t)p * L + r] + Fl[(size_t)r * L + p];
    return v;
  };
  for (int a = 0; a < np; ++a)
    for (int b = a; b < np; ++b) {
      const int p = pairs[a].first, q = pairs[a].second, r = pairs[b].first, s = pairs[b].second;
      const double v = core(p, q, r, s) - core(q, p, r, s) - core(p, q, s, r) + core(q, p, s, r);
      hess[(size_t)a * np + b] = v;
      hess[(size_t)b * np + a] = v;
    }
}

// augmented-Hessian step: lowest eigenvector (v0, v) of [[0, g^T], [g, H]],
// x = v / v0, scaled to norm <= max_step
std::vector<double> ah_step(const std::vector<double>& grad, const std::vector<double>& hess, double max_step) {
  const int n = (int)grad.size();
  std::vector<double> A((size_t)(n + 1) * (n + 1), 0.0);
  for (int i = 0; i < n; ++i) {
    A[(size_t)(i + 1)] = grad[i];
    A[(size_t)(i + 1) * (n + 1)] = grad[i];
    for (int j = 0; j < n; ++j) A[(size_t)(i + 1) * (n + 1) + j + 1] = hess[(size_t)i * n + j];
  }
  std::vector<double> v;
  lowest_eigenpair(n + 1, A, v);
  std::vector<double> x(n);
  if (std::abs(v[0]) < 1e-12) fail(-1, "augmented-Hessian step: the lowest eigenvector has no gradient component");
  double nx = 0.0;
  for (int i = 0; i < n; ++i) {
    x[i] = v[i + 1] / v[0];
    nx += x[i] * x[i];
  }
  nx = std::sqrt(nx);
  if (nx > max_step)
    for (double& e : x) e *= max_step / nx;
  return x;
}

}  // namespace sadmrg
