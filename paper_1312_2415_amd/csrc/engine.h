// Host engine of libsadmrg: symmetry tables, operator stores, task-list
// generation and the sweep driver.  Device work goes through kernels.h only.
#pragma once
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "kernels.h"

namespace sadmrg {

struct Failure {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);

// ---- SU(2) (su2.cpp), spins doubled
bool triangle(int a, int b, int c);
double sixj(int a, int b, int c, int d, int e, int f);
double ninej(int a, int b, int c, int d, int e, int f, int g, int h, int i);
double coupling_product(int tj1, int tj2, int tJ, int tk1, int tk2, int tK, int tj1p, int tj2p, int tJp);
double coupling_same(int tj, int tjm, int tjp, int tk1, int tk2, int tK);
double coupling_singlet(int tj, int tjp, int tk);
double recouple_singlet(int ta, int ts, int tb);
double adjoint_factor(int tj_bra, int tj_ket, int tk);

// ---- DMRG-SCF host arithmetic (scf.cpp)
void rotate_integrals(int L, const double* R, const double* h, const double* g, double* h2, double* g2);
void expm_antisym(int L, const double* A, double* R);
void orbital_derivatives(int L, const double* h, const double* g, const double* D, const double* d,
                         const std::vector<int>& occ, const std::vector<std::pair<int, int>>& pairs, double* F,
                         double* grad, double* hess);
std::vector<double> ah_step(const std::vector<double>& grad, const std::vector<double>& hess, double max_step);

// ---- symmetry sectors: (N left of the bond, 2j, irrep)
struct Sec {
  int N, tj, G;
};
inline bool operator<(const Sec& a, const Sec& b) { return std::tie(a.N, a.tj, a.G) < std::tie(b.N, b.tj, b.G); }
inline bool operator==(const Sec& a, const Sec& b) { return a.N == b.N && a.tj == b.tj && a.G == b.G; }

struct Basis {
  std::vector<Sec> sec;
  std::vector<int> dim;
  int find(const Sec& s) const;
  int64_t total() const;
};

// ---- owned device memory
struct DBuf {
  double* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) {
    o.p = nullptr;
    o.n = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) dev_free(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    release();
    p = (double*)dev_alloc(count * sizeof(double));
    n = count;
  }
  void ensure(size_t count) {
    if (count > n) alloc(count);
  }
};

// Device array of task records.  The host copy is kept until the next put so
// that an asynchronous upload never reads freed host memory.
template <class T>
struct DArr {
  T* p = nullptr;
  size_t cap = 0;
  size_t n = 0;
  std::vector<T> host;
  DArr() = default;
  DArr(const DArr&) = delete;
  DArr& operator=(const DArr&) = delete;
  DArr(DArr&& o) noexcept : p(o.p), cap(o.cap), n(o.n), host(std::move(o.host)) {
    o.p = nullptr;
    o.cap = o.n = 0;
  }
  DArr& operator=(DArr&& o) noexcept {
    if (this != &o) {
      if (p) dev_free(p);
      p = o.p, cap = o.cap, n = o.n, host = std::move(o.host);
      o.p = nullptr;
      o.cap = o.n = 0;
    }
    return *this;
  }
  ~DArr() {
    if (p) dev_free(p);
  }
  void put(const std::vector<T>& v, Stream st) {
    reserve(v.size());
    host = v;
    dev_h2d(p, host.data(), host.size() * sizeof(T), st);
  }
  // the same, taking the host copy over from the caller instead of copying it
  void put(std::vector<T>&& v, Stream st) {
    reserve(v.size());
    host = std::move(v);
    dev_h2d(p, host.data(), host.size() * sizeof(T), st);
  }

 private:
  void reserve(size_t count) {
    if (count > cap) {
      if (p) dev_free(p);
      cap = count + count / 4 + 16;
      p = (T*)dev_alloc(cap * sizeof(T));
    }
    n = count;
  }
};

}  // namespace sadmrg
