// libsadmrg host engine.
//
// Paper: arXiv:1312.2415 (CheMPS2).  Section references below are to that text.
//
// Data layout (all FP64, all in HBM):
//  * A block (left block at bond k = orbitals 0..k-1, or right block at bond k
//    = orbitals k..L-1 plus the singlet-embedding spin) stores its operators in
//    one buffer.  Every operator belongs to a quantum-number class (rank 2k,
//    particle change dN, irrep dG); all operators of a class share one
//    canonical element layout: every symmetry-allowed (bra, ket) sector pair,
//    dense row-major, in a fixed order.  Operator i of the class sits at its
//    own base offset with the same element offsets, so integral-weighted sums
//    over operators (complementary operators) are plain linear combinations.
//  * An enlarged block (block (x) one site, before truncation) uses the same
//    scheme on the enlarged sectors; its dense (m', m) blocks hold every
//    (sector, local state) piece pair.
//  * The two-site object psi: per sector m of the middle bond a dense
//    dimX(m) x dimY(m) row-major matrix; sectors concatenated in order.
#include "engine.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <exception>
#include <mutex>
#include <functional>
#include <thread>
#include <type_traits>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>
#include <set>

namespace sadmrg {

void fail(int code, const std::string& msg) { throw Failure{code, msg}; }
[[noreturn]] void dev_fail(const char* what) { throw Failure{-5, what}; }
[[noreturn]] void dev_fail_nomem(const char* what) { throw Failure{-4, what}; }

int Basis::find(const Sec& s) const {
  auto it = std::lower_bound(sec.begin(), sec.end(), s);
  if (it != sec.end() && *it == s) return int(it - sec.begin());
  return -1;
}
int64_t Basis::total() const {
  int64_t t = 0;
  for (int d : dim) t += d;
  return t;
}

static const int LOC_N[3] = {0, 1, 2};
static const int LOC_TJ[3] = {0, 1, 0};
static inline int loc_irrep(int n, int g) { return n == 1 ? g : 0; }

// ---------------------------------------------------------------------------
// Site operators: reduced elements <n'||o||n> on the local multiplets
// (empty, single, double), section "Reduced MPS tensors" local basis and the
// doublet operators of eqs. creaannih1/2.
// ---------------------------------------------------------------------------
struct SiteOp {
  int tk = 0, dN = 0;
  bool odd = false;
  double el[3][3] = {{0}};
};

static SiteOp site_product(const SiteOp& U, const SiteOp& V, int tK) {
  SiteOp r;
  r.tk = tK;
  r.dN = U.dN + V.dN;
  r.odd = U.odd ^ V.odd;
  for (int n1 = 0; n1 < 3; ++n1)
    for (int n2 = 0; n2 < 3; ++n2)
      for (int n3 = 0; n3 < 3; ++n3) {
        if (V.el[n2][n1] == 0.0 || U.el[n3][n2] == 0.0) continue;
        r.el[n3][n1] += coupling_same(LOC_TJ[n1], LOC_TJ[n2], LOC_TJ[n3], U.tk, V.tk, tK) * U.el[n3][n2] * V.el[n2][n1];
      }
  return r;
}

struct SiteOps {
  SiteOp I, CD, C, A0, B0, B1, AA0, E, CDE, EC, NUD;
  SiteOps() {
    const double s2 = std::sqrt(2.0);
    I.el[0][0] = I.el[1][1] = I.el[2][2] = 1.0;
    NUD.el[2][2] = 1.0;  // n_up n_down
    CD.tk = 1, CD.dN = 1, CD.odd = true, CD.el[1][0] = 1.0, CD.el[2][1] = -s2;  // b+
    C.tk = 1, C.dN = -1, C.odd = true, C.el[0][1] = -s2, C.el[1][2] = -1.0;     // b
    A0 = site_product(CD, CD, 0);                                              // [b+ b+]^0
    B0 = site_product(CD, C, 0);                                               // [b+ b]^0
    B1 = site_product(CD, C, 2);                                               // [b+ b]^1
    AA0 = site_product(C, C, 0);                                               // [b b]^0
    E = B0;                                                                    // E_kk = -sqrt2 [b+ b]^0
    for (auto& row : E.el)
      for (double& v : row) v *= -s2;
    CDE = site_product(CD, E, 1);  // b+ E_kk
    EC = site_product(E, C, 1);    // E_kk b
  }
  const SiteOp& B(int tj) const { return tj == 0 ? B0 : B1; }
};
static const SiteOps& SO() {
  static const SiteOps s;
  return s;
}

// ---------------------------------------------------------------------------
// Problem (the paper's Hamiltonian + Problem objects)
// ---------------------------------------------------------------------------
// A coefficient linear in the folded integrals: v = sum_i m_i W[e_i] (at most
// four entries).  Blocking formulas carry these so that the energy adjoint
// can route d E / d(coefficient) back to the integrals.
struct WLin {
  double v = 0.0;
  int n = 0;
  int64_t e[4] = {0, 0, 0, 0};
  double m[4] = {0.0, 0.0, 0.0, 0.0};
};
static inline WLin operator*(WLin a, double f) {
  a.v *= f;
  for (int i = 0; i < a.n; ++i) a.m[i] *= f;
  return a;
}
static inline WLin operator+(WLin a, const WLin& b) {
  a.v += b.v;
  for (int i = 0; i < b.n; ++i) {
    if (a.n >= 4) fail(-1, "internal: coefficient with more than four integrals");
    a.e[a.n] = b.e[i];
    a.m[a.n++] = b.m[i];
  }
  return a;
}
static inline WLin wconst(double v) {
  WLin a;
  a.v = v;
  return a;
}

struct Problem {
  int L = 0, order = 1;
  std::vector<int> orb;
  double e_const = 0.0;
  std::vector<double> h, eri, W;
  bool have_ints = false;
  bool count_method = false;  // record nonzero piece pairs for the method-work counter
  int N = -1, twoS = 0, irrep = 0;
  double w(int p, int q, int r, int s) const { return W[(((size_t)p * L + q) * L + r) * L + s]; }
  // q^j_ab(r,s): 2 W_abrs - W_rbas (j = 0), W_rbas (j = 1)
  double qc(int tj, int a, int b, int r, int s) const { return tj == 0 ? 2.0 * w(a, b, r, s) - w(r, b, a, s) : w(r, b, a, s); }
  int64_t wi(int p, int q, int r, int s) const { return (((int64_t)p * L + q) * L + r) * L + s; }
  WLin wl(int p, int q, int r, int s) const {
    WLin x;
    x.v = w(p, q, r, s);
    x.n = 1;
    x.e[0] = wi(p, q, r, s);
    x.m[0] = 1.0;
    return x;
  }
  WLin qcl(int tj, int a, int b, int r, int s) const {
    return tj == 0 ? wl(a, b, r, s) * 2.0 + wl(r, b, a, s) * -1.0 : wl(r, b, a, s);
  }
  bool bare_left(int k) const { return k <= L - k; }
  bool bare_right(int k) const { return L - k < k; }
  // section "Complementary operators", trick (a): one-body integrals folded
  // into the two-body ones, W_pqrs = (pq|rs) + [h_pq d_rs + h_rs d_pq]/(N-1)
  void fold() {
    W.assign((size_t)L * L * L * L, 0.0);
    for (int p = 0; p < L; ++p)
      for (int q = 0; q < L; ++q)
        for (int r = 0; r < L; ++r)
          for (int s = 0; s < L; ++s) {
            double v = eri[(((size_t)p * L + q) * L + r) * L + s];
            if (r == s) v += h[p * L + q] / (N - 1);
            if (p == q) v += h[r * L + s] / (N - 1);
            W[(((size_t)p * L + q) * L + r) * L + s] = v;
          }
  }
};

// ---------------------------------------------------------------------------
// Symmetry-sector tables (section "Reduced MPS tensors"; singlet embedding:
// left boundary (0,0,I0), right boundary (S,N,I)).
// ---------------------------------------------------------------------------
using SecCount = std::map<Sec, long long>;

static std::vector<SecCount> left_mult(const Problem& P) {
  std::vector<SecCount> out(P.L + 1);
  out[0][{0, 0, 0}] = 1;
  for (int k = 0; k < P.L; ++k)
    for (auto& [s, c] : out[k])
      for (int n = 0; n < 3; ++n)
        for (int tj = std::abs(s.tj - LOC_TJ[n]); tj <= s.tj + LOC_TJ[n]; tj += 2) {
          long long& v = out[k + 1][{s.N + LOC_N[n], tj, s.G ^ loc_irrep(n, P.orb[k])}];
          v = std::min<long long>(LLONG_MAX / 4, v + c);
        }
  return out;
}

static std::vector<SecCount> right_mult(const Problem& P) {
  std::vector<SecCount> out(P.L + 1);
  out[P.L][{P.N, P.twoS, P.irrep}] = 1;
  for (int k = P.L - 1; k >= 0; --k)
    for (auto& [b, c] : out[k + 1])
      for (int n = 0; n < 3; ++n) {
        const int N = b.N - LOC_N[n];
        if (N < 0) continue;
        for (int tj = std::abs(b.tj - LOC_TJ[n]); tj <= b.tj + LOC_TJ[n]; tj += 2) {
          long long& v = out[k][{N, tj, b.G ^ loc_irrep(n, P.orb[k])}];
          v = std::min<long long>(LLONG_MAX / 4, v + c);
        }
      }
  return out;
}

// D split equally over the sectors, capped by the FCI dimension (section "DMRG"
// of the library description): visit sectors by ascending cap, give each
// min(cap, floor(rest / sectors left)), then the remainder one by one in
// sector order to sectors below their cap.
static std::map<Sec, int> distribute(int D, const std::map<Sec, long long>& caps) {
  std::map<Sec, int> dims;
  long long sum = 0;
  for (auto& [s, c] : caps) sum += c;
  if (sum <= D) {
    for (auto& [s, c] : caps) dims[s] = (int)c;
    return dims;
  }
  std::vector<Sec> order;
  for (auto& [s, c] : caps) order.push_back(s);
  std::stable_sort(order.begin(), order.end(), [&](const Sec& a, const Sec& b) {
    if (caps.at(a) != caps.at(b)) return caps.at(a) < caps.at(b);
    return a < b;
  });
  long long rest = D;
  long long left = (long long)order.size();
  for (const Sec& s : order) {
    const long long d = std::min<long long>(caps.at(s), rest / left);
    dims[s] = (int)d;
    rest -= d;
    --left;
  }
  while (rest > 0) {
    bool moved = false;
    for (auto& [s, c] : caps) {
      if (rest == 0) break;
      if (dims[s] < c) {
        ++dims[s];
        --rest;
        moved = true;
      }
    }
    if (!moved) break;
  }
  std::map<Sec, int> out;
  for (auto& [s, d] : dims)
    if (d > 0) out[s] = d;
  return out;
}

static Basis to_basis(const std::map<Sec, int>& m) {
  Basis b;
  for (auto& [s, d] : m) {
    b.sec.push_back(s);
    b.dim.push_back(d);
  }
  return b;
}

// ---------------------------------------------------------------------------
// Enlarged bases
// ---------------------------------------------------------------------------
struct Piece {
  int sub, n, off;
};
struct Enl : Basis {
  std::vector<std::vector<Piece>> pieces;
  std::vector<std::vector<std::pair<int, int>>> where;  // [sub*3+n] -> (sector, offset)
};

static void finish_enl(Enl& E, const std::map<Sec, std::vector<std::pair<int, int>>>& tmp, const Basis& sub) {
  for (auto& [m, pcs] : tmp) {
    E.sec.push_back(m);
    std::vector<Piece> pv;
    int off = 0;
    for (auto& [a, n] : pcs) {
      pv.push_back({a, n, off});
      off += sub.dim[a];
    }
    E.dim.push_back(off);
    E.pieces.push_back(pv);
  }
  E.where.assign(sub.sec.size() * 3, {});
  for (int m = 0; m < (int)E.sec.size(); ++m)
    for (auto& p : E.pieces[m]) E.where[p.sub * 3 + p.n].push_back({m, p.off});
}

// left block at bond c-1 (x) site c-1 -> bond c ; pieces (a, n): a outer, n inner
static Enl left_enl(const Problem& P, int c, const Basis& sub, const std::set<Sec>* keep) {
  const int g = P.orb[c - 1];
  std::map<Sec, std::vector<std::pair<int, int>>> tmp;
  for (int a = 0; a < (int)sub.sec.size(); ++a)
    for (int n = 0; n < 3; ++n) {
      const Sec& s = sub.sec[a];
      for (int tj = std::abs(s.tj - LOC_TJ[n]); tj <= s.tj + LOC_TJ[n]; tj += 2) {
        Sec m{s.N + LOC_N[n], tj, s.G ^ loc_irrep(n, g)};
        if (keep && !keep->count(m)) continue;
        tmp[m].push_back({a, n});
      }
    }
  Enl E;
  finish_enl(E, tmp, sub);
  return E;
}

// site c (x) right block at bond c+1 -> bond c ; pieces (n, b): n outer, b inner
static Enl right_enl(const Problem& P, int c, const Basis& sub, const std::set<Sec>* keep) {
  const int g = P.orb[c];
  std::map<Sec, std::vector<std::pair<int, int>>> tmp;
  for (int n = 0; n < 3; ++n)
    for (int b = 0; b < (int)sub.sec.size(); ++b) {
      const Sec& s = sub.sec[b];
      const int N = s.N - LOC_N[n];
      if (N < 0) continue;
      for (int tj = std::abs(s.tj - LOC_TJ[n]); tj <= s.tj + LOC_TJ[n]; tj += 2) {
        Sec m{N, tj, s.G ^ loc_irrep(n, g)};
        if (keep && !keep->count(m)) continue;
        tmp[m].push_back({b, n});
      }
    }
  Enl E;
  finish_enl(E, tmp, sub);
  // the piece record keeps (sub = b, n)
  return E;
}

// ---------------------------------------------------------------------------
// Operator stores with canonical class layouts
// ---------------------------------------------------------------------------
enum Fam : int { F_H = 1, F_C = 2, F_S = 3, F_A = 4, F_B = 5, F_P = 6, F_Q = 7 };
static inline uint64_t K(int fam, int tj = 0, int i = 0, int j = 0) {
  return ((uint64_t)fam << 56) | ((uint64_t)tj << 48) | ((uint64_t)i << 24) | (uint64_t)j;
}

struct Layout {
  int tk = 0, dN = 0, dG = 0;
  std::vector<int> bra, ket;
  std::vector<int64_t> eoff;
  int64_t nnz = 0;
  std::unordered_map<int64_t, int> idx;
  int find(int b, int k) const {
    auto it = idx.find((int64_t)b * 65536 + k);
    return it == idx.end() ? -1 : it->second;
  }
  // adjoint element map (for dN == 0 classes), built on demand
  DArr<int> perm;
  DArr<double> fac;
  DArr<double> facT;  // fac[perm[e]]: factors of the transposed map (perm is an involution)
  bool adj_ready = false;
};

struct OpInfo {
  uint64_t key;
  int lay;
  bool odd;
  int64_t off;
};

// every Store gets a distinct generation number: a cached result derived
// from a store is valid while that store (not a later one at the same
// address) is the current block
static uint64_t next_store_gen() {
  static std::atomic<uint64_t> g{0};
  return ++g;
}

struct Store {
  uint64_t gen = next_store_gen();
  char side = 'L';
  int bond = 0;
  std::vector<int> orbs;
  Basis basis;
  std::vector<std::unique_ptr<Layout>> lays;
  std::map<std::tuple<int, int, int>, int> lay_of;
  std::vector<OpInfo> ops;
  std::unordered_map<uint64_t, int> by_key;
  DBuf data;
  int64_t total = 0;
  // structurally nonzero piece pairs of every block (kept only when the
  // method-work counter is on): sorted by block start, then offsets
  struct PieceRect {
    int64_t bstart;
    int roff, coff, rows, cols, ld;
    bool operator<(const PieceRect& o) const {
      return std::tie(bstart, roff, coff) < std::tie(o.bstart, o.roff, o.coff);
    }
    bool operator==(const PieceRect& o) const { return bstart == o.bstart && roff == o.roff && coff == o.coff; }
  };
  std::vector<PieceRect> pieces;
  bool has_pieces = false;

  int layout(int tk, int dN, int dG) {
    auto it = lay_of.find(std::make_tuple(tk, dN, dG));
    if (it != lay_of.end()) return it->second;
    return insert_layout(make_layout(tk, dN, dG));
  }
  int insert_layout(std::unique_ptr<Layout> L) {
    lay_of[std::make_tuple(L->tk, L->dN, L->dG)] = (int)lays.size();
    lays.push_back(std::move(L));
    return (int)lays.size() - 1;
  }
  // the blocks of the class (tk, dN, dG) over this basis
  std::unique_ptr<Layout> make_layout(int tk, int dN, int dG) const {
    auto L = std::make_unique<Layout>();
    L->tk = tk, L->dN = dN, L->dG = dG;
    const int ns = (int)basis.sec.size();
    // sector labels count the electrons left of the bond: an operator adding
    // dN electrons to a right block lowers the label by dN
    const int dl = side == 'R' ? -dN : dN;
    for (int b = 0; b < ns; ++b)
      for (int k = 0; k < ns; ++k) {
        const Sec &sb = basis.sec[b], &sk = basis.sec[k];
        if (sb.N != sk.N + dl || sb.G != (sk.G ^ dG) || !triangle(sk.tj, tk, sb.tj)) continue;
        L->idx[(int64_t)b * 65536 + k] = (int)L->bra.size();
        L->bra.push_back(b);
        L->ket.push_back(k);
        L->eoff.push_back(L->nnz);
        L->nnz += (int64_t)basis.dim[b] * basis.dim[k];
      }
    return L;
  }
  int add(uint64_t key, int tk, int dN, int dG, bool odd) {
    const int l = layout(tk, dN, dG);
    ops.push_back({key, l, odd, total});
    total += lays[l]->nnz;
    by_key[key] = (int)ops.size() - 1;
    return (int)ops.size() - 1;
  }
  int op(uint64_t key) const {
    auto it = by_key.find(key);
    return it == by_key.end() ? -1 : it->second;
  }
  int need(uint64_t key) const {
    const int o = op(key);
    if (o < 0) fail(-1, "internal: missing operator family in block");
    return o;
  }
  const Layout& lay(int o) const { return *lays[ops[o].lay]; }
  double* ptr(int o, int blk) const { return data.p + ops[o].off + lays[ops[o].lay]->eoff[blk]; }
  void allocate(Stream st) {
    data.alloc((size_t)std::max<int64_t>(total, 1));
    dev_zero(data.p, (size_t)std::max<int64_t>(total, 1) * 8, st);
  }
  // adjoint (d E / d element) of every operator, same layout (energy adjoint)
  DBuf adj;
  void alloc_adj(Stream st) {
    adj.alloc((size_t)std::max<int64_t>(total, 1));
    dev_zero(adj.p, (size_t)std::max<int64_t>(total, 1) * 8, st);
  }
  bool owns(const double* p) const { return data.p && p >= data.p && p < data.p + total; }
  double* adj_of(const double* p) const { return adj.p + (p - data.p); }
  void ensure_adjoint_map(int l, Stream st) {
    Layout& L = *lays[l];
    if (L.adj_ready) return;
    std::vector<int> perm(L.nnz);
    std::vector<double> fac(L.nnz);
    for (size_t b = 0; b < L.bra.size(); ++b) {
      const int B = L.bra[b], Kk = L.ket[b];
      const int src = L.find(Kk, B);  // original block (Kk <- B)
      if (src < 0) fail(-1, "internal: class not closed under adjoint");
      const double f = adjoint_factor(basis.sec[Kk].tj, basis.sec[B].tj, L.tk);
      const int rows = basis.dim[B], cols = basis.dim[Kk];
      for (int r = 0; r < rows; ++r)
        for (int c = 0; c < cols; ++c) {
          const int64_t e = L.eoff[b] + (int64_t)r * cols + c;
          perm[e] = (int)(L.eoff[src] + (int64_t)c * rows + r);
          fac[e] = f;
        }
    }
    std::vector<double> facT(L.nnz);
    for (int64_t q = 0; q < L.nnz; ++q) facT[q] = fac[perm[q]];
    L.perm.put(perm, st);
    L.fac.put(fac, st);
    L.facT.put(facT, st);
    L.adj_ready = true;
  }
};

// ---------------------------------------------------------------------------
// Expressions: linear combinations of stored operators (optionally the
// conjugate tensor Tbar), used as the block factor of a coupled product.
// ---------------------------------------------------------------------------
struct Ref {
  int store;  // 0: the block, 1: combination scratch, -1: identity
  int op;
  double c;
  bool adj;
};
using Expr = std::vector<Ref>;
struct Term {
  Expr x;
  SiteOp s;
  double coef;
  WLin wl;  // coef as a linear form of the integrals (n = 0: constant)
};
struct Def {
  uint64_t key;
  int tk, dN, dG;
  bool odd;
  std::vector<Term> terms, sym;  // sym terms are added together with their transpose
};

static Expr adjoint_expr(const Expr& e, const Store& X, const Store& T) {
  Expr out;
  for (const Ref& r : e) {
    Ref q = r;
    if (r.store >= 0 && r.adj) {  // Tbar(Tbar(T)) = (-1)^(2k) T
      const Store& S = r.store == 0 ? X : T;
      if (S.lay(r.op).tk & 1) q.c = -q.c;
    }
    q.adj = !r.adj;
    out.push_back(q);
  }
  return out;
}

// Combination scratch: integral-weighted sums of a block's operators
// (complementary operators assembled on the fly), computed before blocking.
struct Combos {
  Store T;  // same basis as the block
  struct In {
    int op;
    double c;
    bool adj;
    WLin w;  // c as a linear form of the integrals
  };
  std::vector<std::vector<In>> inputs;  // per scratch op
  std::vector<uint64_t> sig;            // dedup signature
  std::map<std::vector<double>, int> memo;

  // sum_i c_i op_i over block operators of one class; returns a Ref (store 1)
  // or an empty expression when all coefficients vanish.  A single constant
  // input becomes a scaled reference to the block operator itself.
  Expr make(const Store& X, const std::vector<In>& in, int tk, int dN, int dG, bool odd) {
    std::vector<In> nz;
    for (auto& i : in)
      if (i.c != 0.0 && i.op >= 0) nz.push_back(i);
    if (nz.empty()) return {};
    if (nz.size() == 1 && !nz[0].adj && nz[0].w.n == 0) return {Ref{0, nz[0].op, nz[0].c, false}};
    std::vector<double> key;
    for (auto& i : nz) {
      key.push_back(i.op);
      key.push_back(i.c);
      key.push_back(i.adj);
      key.push_back(i.w.n);
      for (int q = 0; q < i.w.n; ++q) {
        key.push_back((double)i.w.e[q]);
        key.push_back(i.w.m[q]);
      }
    }
    auto it = memo.find(key);
    if (it != memo.end()) return {Ref{1, it->second, 1.0, false}};
    const int o = T.add(K(0, 0, (int)inputs.size(), 0), tk, dN, dG, odd);
    inputs.push_back(nz);
    memo[key] = o;
    return {Ref{1, o, 1.0, false}};
  }

  void run(Store& X, Stream st) {
    if (T.ops.empty()) return;
    T.allocate(st);
    std::vector<ComboOut> outs;
    std::vector<ComboIn> ins;
    int64_t maxn = 0;
    for (size_t o = 0; o < T.ops.size(); ++o) {
      const int l = T.ops[o].lay;
      const Layout& L = *T.lays[l];
      const int xl = X.layout(L.tk, L.dN, L.dG);
      bool any_adj = false;
      for (auto& i : inputs[o]) any_adj |= i.adj;
      if (any_adj) X.ensure_adjoint_map(xl, st);
      ComboOut co;
      co.out = T.data.p + T.ops[o].off;
      co.nnz = L.nnz;
      co.i0 = (int)ins.size();
      for (auto& i : inputs[o]) {
        if (X.ops[i.op].lay != xl) fail(-1, "internal: combination over mismatched classes");
        ins.push_back({X.data.p + X.ops[i.op].off, i.c, i.adj ? 1 : 0});
      }
      co.i1 = (int)ins.size();
      co.perm = any_adj ? X.lays[xl]->perm.p : nullptr;
      co.fac = any_adj ? X.lays[xl]->fac.p : nullptr;
      outs.push_back(co);
      maxn = std::max(maxn, L.nnz);
    }
    d_outs.put(outs, st);
    d_ins.put(ins, st);
    launch_combo(d_outs.p, (int)outs.size(), d_ins.p, maxn, st);
  }
  DArr<ComboOut> d_outs;
  DArr<ComboIn> d_ins;
};

// ---------------------------------------------------------------------------
// Materialisation of enlarged-block operators from coupled products
//   out += coef * [X-expression (x) site operator]^K    (left: block first)
//   out += coef * [site operator (x) Y-expression]^K    (right: site first)
// Reduced elements via coupling_product (9j) and the fermion sign of the
// factor that is moved past the other one's electrons.
// ---------------------------------------------------------------------------
static thread_local bool tl_in_pool = false;

// Threads started for one loop and joined at its end (the loop of a host
// thread that finds the persistent workers below taken by another one).
template <class F>
static void parallel_for_spawned(size_t n, int nt, F& fn) {
  std::atomic<size_t> next{0};
  std::atomic<bool> stop{false};
  std::exception_ptr first;
  std::mutex mu;
  auto work = [&]() {
    const bool was = tl_in_pool;
    tl_in_pool = true;
    for (size_t j; !stop.load() && (j = next.fetch_add(1)) < n;) {
      try {
        fn(j);
      } catch (...) {
        std::lock_guard<std::mutex> lk(mu);
        if (!first) first = std::current_exception();
        stop = true;
      }
    }
    tl_in_pool = was;
  };
  DevPool* const mem = dev_pool_current();
  const int device = dev_get_device();
  auto worker = [&]() {
    dev_pool_bind(mem);
    try {
      dev_set_device(device);
    } catch (...) {
      std::lock_guard<std::mutex> lk(mu);
      if (!first) first = std::current_exception();
      stop = true;
    }
    work();
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
  work();
  for (auto& t : pool) t.join();
  if (first) std::rethrow_exception(first);
}

// Persistent host workers: started on first use and kept for the process,
// they take one loop at a time beside the thread that posts it, each bound
// to that thread's device and device-memory pool for the loop.  Starting
// threads for every loop (a few hundred loops per sweep) cost as much as
// some of the loops themselves.
struct HostWorkers {
  static constexpr int N = 15;  // workers beside the posting thread
  std::mutex mu;
  std::condition_variable cv_job, cv_done;
  std::vector<std::thread> th;
  bool busy = false, quit = false;
  uint64_t gen = 0;  // loops posted
  int want = 0, finished = 0;
  void (*call)(void*, size_t) = nullptr;
  void* ctx = nullptr;
  size_t n = 0;
  std::atomic<size_t> next{0};
  std::atomic<bool> stop{false};
  std::exception_ptr first;
  DevPool* mem = nullptr;
  int device = 0;

  ~HostWorkers() {
    {
      std::lock_guard<std::mutex> lk(mu);
      quit = true;
    }
    cv_job.notify_all();
    for (auto& x : th) x.join();
  }
  void failed(std::exception_ptr e) {
    std::lock_guard<std::mutex> lk(mu);
    if (!first) first = e;
    stop = true;
  }
  // the loop body, on the posting thread and on every worker taking part
  void work() {
    const bool was = tl_in_pool;
    tl_in_pool = true;
    for (size_t j; !stop.load() && (j = next.fetch_add(1)) < n;) {
      try {
        call(ctx, j);
      } catch (...) {
        failed(std::current_exception());
      }
    }
    tl_in_pool = was;
  }
  void loop(int id) {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      cv_job.wait(lk, [&] { return quit || (gen != seen && id < want); });
      if (quit) return;
      seen = gen;
      DevPool* const m = mem;
      const int dev = device;
      lk.unlock();
      DevPool* const prev = dev_pool_bind(m);
      try {
        dev_set_device(dev);
      } catch (...) {
        failed(std::current_exception());
      }
      work();
      dev_pool_bind(prev);
      lk.lock();
      if (++finished == want) cv_done.notify_all();
    }
  }
};

static HostWorkers& host_workers() {
  static HostWorkers w;
  return w;
}

// fn(j) for j < n on up to `threads` host threads (the calling one
// included); the first exception is rethrown after all have stopped.  A
// call from inside a worker runs serially (no nested loops).  Workers use
// the caller's device and device-memory pool.
template <class F>
static void parallel_for(size_t n, int threads, F&& fn) {
  const int nt = tl_in_pool ? 1 : (int)std::min<size_t>(n, (size_t)std::max(1, threads));
  if (nt <= 1) {
    for (size_t j = 0; j < n; ++j) fn(j);
    return;
  }
  typedef std::remove_reference_t<F> Fn;
  DevPool* const mem = dev_pool_current();
  const int device = dev_get_device();
  HostWorkers& W = host_workers();
  std::unique_lock<std::mutex> lk(W.mu);
  if (W.busy) {  // another host thread's loop holds the workers
    lk.unlock();
    parallel_for_spawned(n, nt, fn);
    return;
  }
  while ((int)W.th.size() < HostWorkers::N) {
    const int id = (int)W.th.size();
    W.th.emplace_back([&W, id] { W.loop(id); });
  }
  W.busy = true;
  W.call = [](void* c, size_t j) { (*static_cast<Fn*>(c))(j); };
  W.ctx = const_cast<void*>(static_cast<const void*>(&fn));
  W.n = n;
  W.next = 0;
  W.stop = false;
  W.first = nullptr;
  W.want = std::min(nt - 1, HostWorkers::N);
  W.finished = 0;
  W.mem = mem;
  W.device = device;
  ++W.gen;
  lk.unlock();
  W.cv_job.notify_all();
  W.work();
  lk.lock();
  W.cv_done.wait(lk, [&] { return W.finished == W.want; });
  const std::exception_ptr e = W.first;
  W.first = nullptr;
  W.call = nullptr;
  W.ctx = nullptr;
  W.busy = false;
  lk.unlock();
  if (e) std::rethrow_exception(e);
}

// host threads for the per-operator parts of an enlargement
static const int ENLARGE_HOST_THREADS = 16;

// fn on a host thread of its own (bound to the caller's device and
// device-memory pool) while the caller goes on, when `on`; otherwise fn runs
// in join().  join() (or the destructor, which swallows the error of an
// unwinding caller) waits for it and rethrows its exception.
struct Overlap {
  std::function<void()> fn;
  std::thread th;
  std::exception_ptr err;
  bool done = false;
  Overlap(bool on, std::function<void()> f) : fn(std::move(f)) {
    if (!on) return;
    DevPool* const mem = dev_pool_current();
    const int device = dev_get_device();
    th = std::thread([this, mem, device] {
      dev_pool_bind(mem);
      try {
        dev_set_device(device);
        fn();
      } catch (...) {
        err = std::current_exception();
      }
    });
  }
  void join() {
    if (done) return;
    done = true;
    if (th.joinable()) {
      th.join();
      if (err) std::rethrow_exception(err);
    } else {
      fn();
    }
  }
  ~Overlap() {
    if (th.joinable()) th.join();
  }
};

struct Entry {
  int64_t dst;  // element offset in the enlarged store
  int64_t bstart;  // element offset of the enlarged block it lies in
  int roff, coff;  // its position in that block (a piece pair)
  int rows, cols, ld;
  GatherSrc src;
  const Term* term;  // the term that produced it (scale = term->coef * unit)
  double unit;
};

struct Materializer {
  std::vector<Entry> entries;  // what emit_op appends to
  // parts[i]: the entries that write operator i of the enlarged store, in
  // emission order (each operator has its own region, so equal destinations
  // stay in one part)
  std::vector<std::vector<Entry>> parts;

  void emit_op(const Problem& P, const Store& X, const Store& T, const Enl& E, Store& Out, int outop,
               const Term& term, bool left, bool mirror) {
    const Layout& OL = Out.lay(outop);
    const int tK = OL.tk;
    for (const Ref& r : term.x) {
      if (r.store == -1) {  // identity on the block
        for (int a = 0; a < (int)X.basis.sec.size(); ++a)
          emit_block(P, E, Out, outop, OL, tK, term, r.c, a, a, 0, false, nullptr, 0, GS_IDENT, X.basis, left,
                     mirror);
        continue;
      }
      const Store& S = r.store == 0 ? X : T;
      const Layout& L = S.lay(r.op);
      const bool odd = S.ops[r.op].odd;
      for (size_t b = 0; b < L.bra.size(); ++b) {
        int bra = L.bra[b], ket = L.ket[b];
        double f = r.c;
        int kind = GS_NORMAL;
        const int ld = S.basis.dim[ket];
        if (r.adj) {
          f *= adjoint_factor(S.basis.sec[bra].tj, S.basis.sec[ket].tj, L.tk);
          std::swap(bra, ket);
          kind = GS_TRANS;
        }
        emit_block(P, E, Out, outop, OL, tK, term, f, bra, ket, L.tk, odd, S.ptr(r.op, (int)b), ld, kind, S.basis,
                   left, mirror);
      }
    }
  }

  void emit_block(const Problem& P, const Enl& E, Store& Out, int outop, const Layout& OL, int tK, const Term& term,
                  double f, int abra, int aket, int tkX, bool oddX, const double* src, int ld, int kind,
                  const Basis& sub, bool left, bool mirror) {
    const SiteOp& s = term.s;
    const Sec &sb = sub.sec[abra], &sk = sub.sec[aket];
    for (int nb = 0; nb < 3; ++nb)
      for (int nk = 0; nk < 3; ++nk) {
        const double sv = s.el[nb][nk];
        if (sv == 0.0) continue;
        for (auto& [mk, offk] : E.where[aket * 3 + nk])
          for (auto& [mb, offb] : E.where[abra * 3 + nb]) {
            const int tjk = E.sec[mk].tj, tjb = E.sec[mb].tj;
            if (!triangle(tjk, tK, tjb)) continue;
            double c9, sign;
            if (left) {
              c9 = coupling_product(sk.tj, LOC_TJ[nk], tjk, tkX, s.tk, tK, sb.tj, LOC_TJ[nb], tjb);
              sign = (s.odd && (sk.N & 1)) ? -1.0 : 1.0;
            } else {
              c9 = coupling_product(LOC_TJ[nk], sk.tj, tjk, s.tk, tkX, tK, LOC_TJ[nb], sb.tj, tjb);
              sign = (oddX && (LOC_N[nk] & 1)) ? -1.0 : 1.0;
            }
            if (c9 == 0.0) continue;
            const double scale = term.coef * f * c9 * sign * sv;
            const int blk = OL.find(mb, mk);
            if (blk < 0)
              fail(-1, "internal: enlarged block outside the class layout (op key " +
                           std::to_string(Out.ops[outop].key >> 56) + "/" +
                           std::to_string((Out.ops[outop].key >> 48) & 255) + " tk " + std::to_string(OL.tk) +
                           " dN " + std::to_string(OL.dN) + " dG " + std::to_string(OL.dG) + "; bra N" +
                           std::to_string(E.sec[mb].N) + " j" + std::to_string(E.sec[mb].tj) + " G" +
                           std::to_string(E.sec[mb].G) + ", ket N" + std::to_string(E.sec[mk].N) + " j" +
                           std::to_string(E.sec[mk].tj) + " G" + std::to_string(E.sec[mk].G) + ", X tk " +
                           std::to_string(tkX) + " site tk " + std::to_string(s.tk) + ")");
            const int cols_mk = E.dim[mk];
            Entry e;
            e.dst = Out.ops[outop].off + OL.eoff[blk] + (int64_t)offb * cols_mk + offk;
            e.bstart = Out.ops[outop].off + OL.eoff[blk];
            e.roff = offb;
            e.coff = offk;
            e.rows = sub.dim[abra];
            e.cols = sub.dim[aket];
            e.ld = cols_mk;
            e.src = {src, ld, kind, scale};
            e.term = &term;
            e.unit = f * c9 * sign * sv;
            entries.push_back(e);
            if (mirror) {  // transpose partner: block (mk <- mb) at (offk, offb)
              const int blk2 = OL.find(mk, mb);
              if (blk2 < 0) fail(-1, "internal: transpose block missing");
              Entry m;
              m.dst = Out.ops[outop].off + OL.eoff[blk2] + (int64_t)offk * E.dim[mb] + offb;
              m.bstart = Out.ops[outop].off + OL.eoff[blk2];
              m.roff = offk;
              m.coff = offb;
              m.rows = sub.dim[aket];
              m.cols = sub.dim[abra];
              m.ld = E.dim[mb];
              m.src = {src, ld, kind == GS_NORMAL ? GS_TRANS : (kind == GS_TRANS ? GS_NORMAL : GS_IDENT), scale};
              m.term = &term;
              m.unit = e.unit;
              entries.push_back(m);
            }
          }
      }
  }

  void run(Store& Out, Stream st) {
    // group equal destinations, keeping the emission order inside a group
    // (the order of the summands), one operator's part at a time on host
    // threads; every entry is one gather source, so each part's sources go
    // straight to their place in the final list (the destinations, fewer and
    // known only after grouping, are laid end to end afterwards)
    const size_t nseg = parts.size();
    std::vector<size_t> os(nseg + 1, 0);
    for (size_t i = 0; i < nseg; ++i) os[i + 1] = os[i] + parts[i].size();
    if (os[nseg] > (size_t)INT32_MAX) fail(-4, "enlargement with more than 2^31 gather sources");
    std::vector<GatherSrc> srcs(os[nseg]);
    std::vector<std::vector<GatherDst>> sd(nseg);
    parallel_for(nseg, ENLARGE_HOST_THREADS, [&](size_t i) {
      const std::vector<Entry>& pe = parts[i];
      const size_t n = pe.size();
      std::vector<std::pair<int64_t, uint32_t>> key(n);  // (destination, emission order)
      for (size_t k = 0; k < n; ++k) key[k] = {pe[k].dst, (uint32_t)k};
      std::sort(key.begin(), key.end());
      std::vector<GatherDst>& dl = sd[i];
      GatherSrc* const sl = srcs.data() + os[i];
      size_t ns = 0;
      for (size_t k = 0; k < n;) {
        const Entry& e0 = pe[key[k].second];
        GatherDst d{Out.data.p + e0.dst, e0.rows, e0.cols, e0.ld, (int)(os[i] + ns), 0};
        size_t j = k;
        for (; j < n && key[j].first == e0.dst; ++j) {
          const Entry& e = pe[key[j].second];
          if (e.rows != e0.rows || e.cols != e0.cols) fail(-1, "internal: overlapping sub-blocks of different shape");
          sl[ns++] = e.src;
        }
        d.s1 = (int)(os[i] + ns);
        dl.push_back(d);
        k = j;
      }
    });
    std::vector<size_t> od(nseg + 1, 0);
    for (size_t i = 0; i < nseg; ++i) od[i + 1] = od[i] + sd[i].size();
    std::vector<GatherDst> dsts(od[nseg]);
    parallel_for(nseg, ENLARGE_HOST_THREADS,
                 [&](size_t i) { std::copy(sd[i].begin(), sd[i].end(), dsts.begin() + (ptrdiff_t)od[i]); });
    n_entries = (int64_t)os[nseg];
    parts.clear();
    const int ndst = (int)dsts.size();
    d_dst.put(std::move(dsts), st);
    d_src.put(std::move(srcs), st);
    launch_gather(d_dst.p, ndst, d_src.p, st);
  }
  DArr<GatherDst> d_dst;
  DArr<GatherSrc> d_src;
  int64_t n_entries = 0;
};

// ---------------------------------------------------------------------------
// Blocking formulas: the operator families of an enlarged block in terms of
// the block's families and site operators (complementary operators, section
// "Complementary operators").  Families:
//   H          block Hamiltonian
//   C z        b+_z, z in the block
//   S w        sum_{p,r,s in block} W_{w p r s} b+_p E_rs, w outside
//   A j z z'   [b+_z b+_z']^j, B j z z' [b+_z b_z']^j   (z <= z', bare mode)
//   P j w w'   sum_{zz'} W_{z w z' w'} A^j_zz'           (w <= w' outside)
//   Q j a b    sum_{rs} q^j_ab(r,s) B^j_rs               (a <= b outside)
// ---------------------------------------------------------------------------
struct Blocker {
  const Problem& P;
  Store& X;    // block (at bond k)
  Combos& cb;  // scratch combinations of X
  bool bare;   // pair mode of X
  Blocker(const Problem& p, Store& x, Combos& c, bool b) : P(p), X(x), cb(c), bare(b) {}

  Expr C(int z) const { return {Ref{0, X.need(K(F_C, 0, z, 0)), 1.0, false}}; }
  static Expr scale(Expr e, double f) {
    for (auto& r : e) r.c *= f;
    return e;
  }
  int gz(int z) const { return P.orb[z]; }

  // sum_z c_z b+_z  (all z in the block share no constraint: grouped by irrep)
  Expr cdag(const std::vector<WLin>& coef) {
    // coefficients of orbitals with different irreps cannot mix; the caller's
    // integrals respect the point group, so at most one irrep is nonzero.
    std::vector<Combos::In> in;
    int g = -1;
    for (int z : X.orbs) {
      const double c = coef[z].v;
      if (c == 0.0) continue;
      if (g >= 0 && gz(z) != g) fail(-3, "integrals break the point-group symmetry");
      g = gz(z);
      in.push_back({X.need(K(F_C, 0, z, 0)), c, false, coef[z]});
    }
    if (in.empty()) return {};
    return cb.make(X, in, 1, 1, g, true);
  }

  Expr getP(int tj, int w, int wp) {
    const int g = gz(w) ^ gz(wp);
    const double sg = (tj == 2) ? -1.0 : 1.0;
    if (!bare) {
      if (tj == 2 && w == wp) return {};
      if (w <= wp) return {Ref{0, X.need(K(F_P, tj, w, wp)), 1.0, false}};
      return {Ref{0, X.need(K(F_P, tj, wp, w)), sg, false}};
    }
    std::vector<Combos::In> in;
    for (int z : X.orbs)
      for (int zp : X.orbs) {
        const double c = P.w(z, w, zp, wp);
        if (c == 0.0) continue;
        if (tj == 2 && z == zp) continue;
        const int a = std::min(z, zp), b = std::max(z, zp);
        const double f = (z <= zp) ? 1.0 : sg;
        in.push_back({X.need(K(F_A, tj, a, b)), c * f, false, P.wl(z, w, zp, wp) * f});
      }
    return cb.make(X, in, tj, 2, g, false);
  }

  Expr getQ(int tj, int a, int b) {
    const int g = gz(a) ^ gz(b);
    const double sg = (tj == 2) ? -1.0 : 1.0;
    if (!bare) {
      if (a <= b) return {Ref{0, X.need(K(F_Q, tj, a, b)), 1.0, false}};
      return {Ref{0, X.need(K(F_Q, tj, b, a)), sg, true}};
    }
    std::vector<Combos::In> in;
    for (int r : X.orbs)
      for (int s : X.orbs) {
        const double c = P.qc(tj, a, b, r, s);
        if (c == 0.0) continue;
        if (r <= s)
          in.push_back({X.need(K(F_B, tj, r, s)), c, false, P.qcl(tj, a, b, r, s)});
        else
          in.push_back({X.need(K(F_B, tj, s, r)), c * sg, true, P.qcl(tj, a, b, r, s) * sg});
      }
    return cb.make(X, in, tj, 0, g, false);
  }
};

static void add_term(Def& d, Expr x, const SiteOp& s, double coef) {
  if (x.empty() || coef == 0.0) return;
  d.terms.push_back({std::move(x), s, coef, wconst(coef)});
}
static void add_term_w(Def& d, Expr x, const SiteOp& s, const WLin& coef) {  // integral-valued coefficient
  if (x.empty() || coef.v == 0.0) return;
  d.terms.push_back({std::move(x), s, coef.v, coef});
}
static void add_sym(Def& d, Expr x, const SiteOp& s, double coef) {
  if (x.empty() || coef == 0.0) return;
  d.sym.push_back({std::move(x), s, coef, wconst(coef)});
}
static const Expr IDX = {Ref{-1, -1, 1.0, false}};

// Left: block at bond k (x) site k -> enlarged block at bond k+1
static std::vector<Def> defs_left(const Problem& P, Store& X, Combos& cb) {
  const int k = X.bond, L = P.L;
  const SiteOps& so = SO();
  const double s2 = std::sqrt(2.0), s3 = std::sqrt(3.0), s32 = std::sqrt(1.5);
  Blocker bk(P, X, cb, P.bare_left(k));
  std::vector<Def> defs;
  std::vector<WLin> coef(L);
  auto reset = [&] { std::fill(coef.begin(), coef.end(), WLin()); };

  for (int x : X.orbs) {
    Def d{K(F_C, 0, x, 0), 1, 1, P.orb[x], true, {}, {}};
    add_term(d, bk.C(x), so.I, 1.0);
    defs.push_back(d);
  }
  {
    Def d{K(F_C, 0, k, 0), 1, 1, P.orb[k], true, {}, {}};
    add_term(d, IDX, so.CD, 1.0);
    defs.push_back(d);
  }
  {  // H
    Def d{K(F_H), 0, 0, 0, false, {}, {}};
    add_term(d, {Ref{0, X.need(K(F_H)), 1.0, false}}, so.I, 1.0);
    add_term_w(d, IDX, so.NUD, P.wl(k, k, k, k));  // site Hamiltonian: W_kkkk n_up n_down
    add_sym(d, {Ref{0, X.need(K(F_S, 0, k, 0)), 1.0, false}}, so.C, -s2);
    reset();
    for (int x : X.orbs) coef[x] = P.wl(x, k, k, k);
    add_sym(d, bk.cdag(coef), so.EC, -s2);
    add_sym(d, bk.getP(0, k, k), so.AA0, -0.5);
    add_term(d, bk.getQ(0, k, k), so.B0, 1.0);
    add_term(d, bk.getQ(2, k, k), so.B1, s3);
    defs.push_back(d);
  }
  for (int y = k + 1; y < L; ++y) {  // S_y
    Def d{K(F_S, 0, y, 0), 1, 1, P.orb[y], true, {}, {}};
    add_term(d, {Ref{0, X.need(K(F_S, 0, y, 0)), 1.0, false}}, so.I, 1.0);
    add_term(d, bk.getQ(0, k, y), so.CD, -1.0 / s2);
    add_term(d, bk.getQ(2, k, y), so.CD, -s32);
    add_term(d, bk.getP(0, y, k), so.C, 1.0 / s2);
    add_term(d, bk.getP(2, y, k), so.C, -s32);
    reset();
    for (int s : X.orbs) coef[s] = P.wl(k, y, k, s);
    add_term(d, adjoint_expr(bk.cdag(coef), X, cb.T), so.A0, 1.0 / s2);
    reset();
    for (int r : X.orbs) coef[r] = P.wl(k, y, r, k) * (1.0 / s2) + P.wl(r, y, k, k) * -s2;
    add_term(d, bk.cdag(coef), so.B0, 1.0);
    reset();
    for (int r : X.orbs) coef[r] = P.wl(k, y, r, k);
    add_term(d, bk.cdag(coef), so.B1, s32);
    add_term_w(d, IDX, so.CDE, P.wl(k, y, k, k));
    defs.push_back(d);
  }
  std::vector<int> orbs = X.orbs;
  orbs.push_back(k);
  if (P.bare_left(k + 1)) {
    for (int x : orbs)
      for (int xp : orbs) {
        if (xp < x) continue;
        const int g = P.orb[x] ^ P.orb[xp];
        for (int tj : {0, 2}) {
          if (!(x == xp && tj == 2)) {
            Def d{K(F_A, tj, x, xp), tj, 2, g, false, {}, {}};
            if (xp < k)
              add_term(d, {Ref{0, X.need(K(F_A, tj, x, xp)), 1.0, false}}, so.I, 1.0);
            else if (x < k)
              add_term(d, bk.C(x), so.CD, 1.0);
            else
              add_term(d, IDX, so.A0, 1.0);
            defs.push_back(d);
          }
          Def d{K(F_B, tj, x, xp), tj, 0, g, false, {}, {}};
          if (xp < k)
            add_term(d, {Ref{0, X.need(K(F_B, tj, x, xp)), 1.0, false}}, so.I, 1.0);
          else if (x < k)
            add_term(d, bk.C(x), so.C, 1.0);
          else
            add_term(d, IDX, so.B(tj), 1.0);
          defs.push_back(d);
        }
      }
  } else {
    for (int w = k + 1; w < L; ++w)
      for (int wp = w; wp < L; ++wp) {
        const int g = P.orb[w] ^ P.orb[wp];
        for (int tj : {0, 2}) {
          const double sg = tj == 2 ? -1.0 : 1.0;
          if (!(w == wp && tj == 2)) {
            Def d{K(F_P, tj, w, wp), tj, 2, g, false, {}, {}};
            add_term(d, bk.getP(tj, w, wp), so.I, 1.0);
            reset();
            for (int z : X.orbs) coef[z] = P.wl(z, w, k, wp) + P.wl(k, w, z, wp) * sg;
            add_term(d, bk.cdag(coef), so.CD, 1.0);
            if (tj == 0) add_term_w(d, IDX, so.A0, P.wl(k, w, k, wp));
            defs.push_back(d);
          }
          Def d{K(F_Q, tj, w, wp), tj, 0, g, false, {}, {}};
          add_term(d, bk.getQ(tj, w, wp), so.I, 1.0);
          reset();
          for (int r : X.orbs) coef[r] = P.qcl(tj, w, wp, r, k);
          add_term(d, bk.cdag(coef), so.C, 1.0);
          reset();
          for (int s : X.orbs) coef[s] = P.qcl(tj, w, wp, k, s);
          add_term(d, adjoint_expr(bk.cdag(coef), X, cb.T), so.CD, sg);
          add_term_w(d, IDX, so.B(tj), P.qcl(tj, w, wp, k, k));
          defs.push_back(d);
        }
      }
  }
  return defs;
}

// Right: site k (x) block at bond k+1 -> enlarged block at bond k
static std::vector<Def> defs_right(const Problem& P, Store& Y, Combos& cb) {
  const int k = Y.bond - 1;
  const SiteOps& so = SO();
  const double s2 = std::sqrt(2.0), s3 = std::sqrt(3.0), s32 = std::sqrt(1.5);
  Blocker bk(P, Y, cb, P.bare_right(k + 1));
  std::vector<Def> defs;
  std::vector<WLin> coef(P.L);
  auto reset = [&] { std::fill(coef.begin(), coef.end(), WLin()); };

  for (int y : Y.orbs) {
    Def d{K(F_C, 0, y, 0), 1, 1, P.orb[y], true, {}, {}};
    add_term(d, bk.C(y), so.I, 1.0);
    defs.push_back(d);
  }
  {
    Def d{K(F_C, 0, k, 0), 1, 1, P.orb[k], true, {}, {}};
    add_term(d, IDX, so.CD, 1.0);
    defs.push_back(d);
  }
  {  // H
    Def d{K(F_H), 0, 0, 0, false, {}, {}};
    add_term(d, {Ref{0, Y.need(K(F_H)), 1.0, false}}, so.I, 1.0);
    add_term_w(d, IDX, so.NUD, P.wl(k, k, k, k));
    reset();
    for (int y : Y.orbs) coef[y] = P.wl(k, y, k, k);
    add_sym(d, adjoint_expr(bk.cdag(coef), Y, cb.T), so.CDE, -s2);
    add_sym(d, adjoint_expr({Ref{0, Y.need(K(F_S, 0, k, 0)), 1.0, false}}, Y, cb.T), so.CD, -s2);
    add_sym(d, adjoint_expr(bk.getP(0, k, k), Y, cb.T), so.A0, 0.5);
    add_term(d, bk.getQ(0, k, k), so.B0, 1.0);
    add_term(d, bk.getQ(2, k, k), so.B1, s3);
    defs.push_back(d);
  }
  for (int x = 0; x < k; ++x) {  // S_x
    Def d{K(F_S, 0, x, 0), 1, 1, P.orb[x], true, {}, {}};
    add_term(d, {Ref{0, Y.need(K(F_S, 0, x, 0)), 1.0, false}}, so.I, 1.0);
    add_term(d, bk.getQ(0, k, x), so.CD, -1.0 / s2);
    add_term(d, bk.getQ(2, k, x), so.CD, s32);
    add_term(d, bk.getP(0, x, k), so.C, 1.0 / s2);
    add_term(d, bk.getP(2, x, k), so.C, s32);
    // S_x = sum W_{p x r s} b+_p E_rs: x is the partner of the creator p, so
    // it stays in the second slot (needed when (pq|rs) != (qp|rs))
    reset();
    for (int s : Y.orbs) coef[s] = P.wl(k, x, k, s);
    add_term(d, adjoint_expr(bk.cdag(coef), Y, cb.T), so.A0, 1.0 / s2);
    reset();
    for (int r : Y.orbs) coef[r] = P.wl(k, x, r, k) * (1.0 / s2) + P.wl(r, x, k, k) * -s2;
    add_term(d, bk.cdag(coef), so.B0, 1.0);
    reset();
    for (int r : Y.orbs) coef[r] = P.wl(k, x, r, k);
    add_term(d, bk.cdag(coef), so.B1, -s32);
    add_term_w(d, IDX, so.CDE, P.wl(k, x, k, k));
    defs.push_back(d);
  }
  std::vector<int> orbs;
  orbs.push_back(k);
  for (int y : Y.orbs) orbs.push_back(y);
  if (P.bare_right(k)) {
    for (int y : orbs)
      for (int yp : orbs) {
        if (yp < y) continue;
        const int g = P.orb[y] ^ P.orb[yp];
        for (int tj : {0, 2}) {
          if (!(y == yp && tj == 2)) {
            Def d{K(F_A, tj, y, yp), tj, 2, g, false, {}, {}};
            if (y > k)
              add_term(d, {Ref{0, Y.need(K(F_A, tj, y, yp)), 1.0, false}}, so.I, 1.0);
            else if (yp > k)
              add_term(d, bk.C(yp), so.CD, 1.0);
            else
              add_term(d, IDX, so.A0, 1.0);
            defs.push_back(d);
          }
          Def d{K(F_B, tj, y, yp), tj, 0, g, false, {}, {}};
          if (y > k)
            add_term(d, {Ref{0, Y.need(K(F_B, tj, y, yp)), 1.0, false}}, so.I, 1.0);
          else if (yp > k)
            add_term(d, adjoint_expr(bk.C(yp), Y, cb.T), so.CD, 1.0);
          else
            add_term(d, IDX, so.B(tj), 1.0);
          defs.push_back(d);
        }
      }
  } else {
    for (int w = 0; w < k; ++w)
      for (int wp = w; wp < k; ++wp) {
        const int g = P.orb[w] ^ P.orb[wp];
        for (int tj : {0, 2}) {
          const double sg = tj == 2 ? -1.0 : 1.0;
          if (!(w == wp && tj == 2)) {
            Def d{K(F_P, tj, w, wp), tj, 2, g, false, {}, {}};
            add_term(d, bk.getP(tj, w, wp), so.I, 1.0);
            reset();
            for (int z : Y.orbs) coef[z] = P.wl(k, w, z, wp) + P.wl(z, w, k, wp) * sg;
            add_term(d, bk.cdag(coef), so.CD, 1.0);
            if (tj == 0) add_term_w(d, IDX, so.A0, P.wl(k, w, k, wp));
            defs.push_back(d);
          }
          Def d{K(F_Q, tj, w, wp), tj, 0, g, false, {}, {}};
          add_term(d, bk.getQ(tj, w, wp), so.I, 1.0);
          reset();
          for (int s : Y.orbs) coef[s] = P.qcl(tj, w, wp, k, s);
          add_term(d, adjoint_expr(bk.cdag(coef), Y, cb.T), so.CD, 1.0);
          reset();
          for (int r : Y.orbs) coef[r] = P.qcl(tj, w, wp, r, k);
          add_term(d, bk.cdag(coef), so.C, sg);
          add_term_w(d, IDX, so.B(tj), P.qcl(tj, w, wp, k, k));
          defs.push_back(d);
        }
      }
  }
  return defs;
}

// The blocking of one enlargement: the evaluated scratch combinations, the
// enlarged store's structure and its materialisation entries (host).
struct EnlargeTrace {
  Combos cb;
  std::vector<Def> defs;
  std::vector<int> opidx;  // operator of out for every definition
  std::unique_ptr<Store> out;
  Materializer mat;
};

// First part of an enlargement: the operator definitions, the combination
// scratch (its kernel enqueued on st) and the enlarged store's layouts.
static void trace_layouts(const Problem& P, Store& X, const Enl& E, bool left, Stream st, EnlargeTrace& tr) {
  tr.cb.T.side = X.side;
  tr.cb.T.bond = X.bond;
  tr.cb.T.basis = X.basis;
  tr.defs = left ? defs_left(P, X, tr.cb) : defs_right(P, X, tr.cb);
  tr.cb.run(X, st);
  tr.out = std::make_unique<Store>();
  Store& out = *tr.out;
  out.side = left ? 'L' : 'R';
  out.bond = left ? X.bond + 1 : X.bond - 1;
  out.orbs = X.orbs;
  if (left)
    out.orbs.push_back(X.bond);
  else
    out.orbs.insert(out.orbs.begin(), X.bond - 1);
  out.basis.sec = E.sec;
  out.basis.dim = E.dim;
  // the layouts of the operator classes, built on host threads and taken in
  // order of first use
  std::vector<std::tuple<int, int, int>> cls;
  {
    std::set<std::tuple<int, int, int>> seen;
    for (auto& d : tr.defs)
      if (seen.insert(std::make_tuple(d.tk, d.dN, d.dG)).second) cls.push_back(std::make_tuple(d.tk, d.dN, d.dG));
  }
  std::vector<std::unique_ptr<Layout>> built(cls.size());
  parallel_for(cls.size(), ENLARGE_HOST_THREADS, [&](size_t i) {
    built[i] = out.make_layout(std::get<0>(cls[i]), std::get<1>(cls[i]), std::get<2>(cls[i]));
  });
  for (auto& L : built) out.insert_layout(std::move(L));
  tr.opidx.clear();
  for (auto& d : tr.defs) tr.opidx.push_back(out.add(d.key, d.tk, d.dN, d.dG, d.odd));
}

// Second part (host only, reads the stores' layouts): the gather entries of
// every operator of the enlarged store `out` (the one trace_layouts built).
static void trace_entries(const Problem& P, const Store& X, const Enl& E, bool left, EnlargeTrace& tr, Store& out) {
  const std::vector<int>& opidx = tr.opidx;
  // the operators' entries are independent: emitted on host threads, one
  // list per operator (in operator order they are the serial emission order)
  std::vector<std::vector<Entry>> per(tr.defs.size());
  parallel_for(tr.defs.size(), ENLARGE_HOST_THREADS, [&](size_t i) {
    Materializer m;
    for (auto& t : tr.defs[i].terms) m.emit_op(P, X, tr.cb.T, E, out, opidx[i], t, left, false);
    for (auto& t : tr.defs[i].sym) m.emit_op(P, X, tr.cb.T, E, out, opidx[i], t, left, true);
    per[i] = std::move(m.entries);
  });
  if (P.count_method) {  // nonzero piece pairs of every enlarged block
    size_t tot = 0;
    for (auto& v : per) tot += v.size();
    std::vector<Store::PieceRect>& pr = out.pieces;
    pr.clear();
    pr.reserve(tot);
    for (auto& v : per)
      for (const Entry& e : v) pr.push_back({e.bstart, e.roff, e.coff, e.rows, e.cols, e.ld});
    std::sort(pr.begin(), pr.end());
    pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
    out.has_pieces = true;
  }
  tr.mat.parts = std::move(per);
}

static void trace_enlarge(const Problem& P, Store& X, const Enl& E, bool left, Stream st, EnlargeTrace& tr) {
  trace_layouts(P, X, E, left, st, tr);
  trace_entries(P, X, E, left, tr, *tr.out);
}

// Last part: the gather of the traced entries into `out` (allocated), then
// the nonzero piece pairs when the method counter is on; waits for the
// stream (the scratch combinations are released with the trace).
static void enlarge_finish(EnlargeTrace& tr, Store& out, Stream st, int64_t* n_entries) {
  tr.mat.run(out, st);
  if (n_entries) *n_entries += tr.mat.n_entries;
  if (out.has_pieces) {  // keep the piece pairs that hold a nonzero value
    std::vector<Store::PieceRect>& pr = out.pieces;
    std::vector<RectDesc> rd;
    rd.reserve(pr.size());
    for (const auto& q : pr) rd.push_back({q.bstart + (int64_t)q.roff * q.ld + q.coff, q.rows, q.cols, q.ld});
    DArr<RectDesc> d_rd;
    d_rd.put(rd, st);
    DBuf fl;
    fl.alloc(pr.size() / 8 + 1);
    launch_rects_nonzero(out.data.p, d_rd.p, (int)rd.size(), (unsigned char*)fl.p, st);
    std::vector<unsigned char> h(pr.size());
    dev_d2h(h.data(), fl.p, h.size(), st);
    size_t w = 0;
    for (size_t q = 0; q < pr.size(); ++q)
      if (h[q]) pr[w++] = pr[q];
    pr.resize(w);
  }
  dev_sync(st);
}

// Enlarge a block by one site: combinations, then materialisation.
static std::unique_ptr<Store> enlarge(const Problem& P, Store& X, const Enl& E, bool left, Stream st,
                                      int64_t* n_entries) {
  EnlargeTrace tr;
  trace_enlarge(P, X, E, left, st, tr);
  tr.out->allocate(st);
  enlarge_finish(tr, *tr.out, st, n_entries);
  return std::move(tr.out);
}

// ---------------------------------------------------------------------------
// Grouped-GEMM task lists (output tiles of at most 64 x 64) and the two-pass
// evaluation of block triple products  out += coef * opA(A) * B * opC(C):
//   pass 1: T = opA(A) * B   written once into a workspace slot,
//   pass 2: out += coef * T * opC(C), all products of one output block
//           accumulated by the same tiles (long K), split into flop-balanced
//           chunks whose partial tiles are added in a fixed order.
// ---------------------------------------------------------------------------
struct GemmList {
  static constexpr int TS = 64;
  struct Item {
    int tile;
    GTask t;
    double w;
  };
  std::vector<GTile> tiles;
  std::vector<Item> items;

  double flops = 0.0;  // 2 m n k of every task added
  double bytes = 0.0;  // each operand of every product, once

  int add_block(double* out, int rows, int cols, int ld, int mode) {
    const int first = (int)tiles.size();
    for (int r0 = 0; r0 < rows; r0 += TS)
      for (int c0 = 0; c0 < cols; c0 += TS)
        tiles.push_back(
            {out + (int64_t)r0 * ld + c0, nullptr, ld, std::min(TS, rows - r0), std::min(TS, cols - c0), mode, 0, 0});
    return first;
  }
  // block registered at `first` (rows x cols) += coef * opA(A)[rows x K] * opB(B)[K x cols]
  void add(int first, int rows, int cols, const GTask& base) {
    if (base.K <= 0 || rows <= 0 || cols <= 0) return;
    // the kernel addresses each operand of a tile with 32-bit byte offsets:
    // the largest element offset it forms, (64 ld + K) for storage contiguous
    // along k and (K + 32) ld + 64 otherwise, must stay below 2^28
    const int64_t lim = (int64_t)1 << 28;
    auto reach = [](bool kfast, int64_t ld, int64_t K) { return kfast ? 64 * ld + K + 64 : (K + 32) * ld + 64; };
    if (reach(!(base.flags & GT_TRANS_A), base.lda, base.K) >= lim ||
        reach((base.flags & GT_TRANS_B) != 0, base.ldb, base.K) >= lim)
      fail(-4, "block product too large for the grouped GEMM kernel");
    bytes += 8.0 * ((double)rows * base.K + (double)base.K * cols);
    const int ntc = (cols + TS - 1) / TS;
    for (int r0 = 0, tr = 0; r0 < rows; r0 += TS, ++tr)
      for (int c0 = 0, tc = 0; c0 < cols; c0 += TS, ++tc) {
        GTask t = base;
        t.a += (t.flags & GT_TRANS_A) ? (int64_t)r0 : (int64_t)r0 * t.lda;
        t.b += (t.flags & GT_TRANS_B) ? (int64_t)c0 * t.ldb : (int64_t)c0;
        const double w = 2.0 * std::min(TS, rows - r0) * std::min(TS, cols - c0) * t.K;
        items.push_back({first + tr * ntc + tc, t, w});
        flops += w;
      }
  }

  struct Plan {
    DArr<GTile> tiles;
    DArr<GTask> tasks;
    DArr<int> wstart;
    DArr<RTile> reds;
    DBuf part;
    int ntiles = 0, nwg = 0, nreds = 0;
    bool stream = false, f32 = false;
    int tag = 2;
    int xcd = 0;  // XCD count for the workgroup order (0: dispatch order)
    void run(Stream st, bool bf3 = false) const {
      launch_gemm(tiles.p, tasks.p, wstart.p, nwg, stream, tag, f32, st, f32 && bf3, xcd);
      launch_reduce(reds.p, nreds, f32, st);
    }
  };

  // Estimated workgroup cycles of one task in a tile with `cols` columns:
  // MFMA time of a wave (two 64-cycle MFMAs per k-step pair and 16-column
  // block) plus a fixed cost per staged chunk and per task.
  static double task_cost(int K, int cols) {
    const int ncb = (cols + 15) / 16;
    const int pairs = 4 * (K / GK_HOST) + (K % GK_HOST + 7) / 8;
    return 128.0 * ncb * pairs + 400.0 * ((K + GK_HOST - 1) / GK_HOST) + 200.0;
  }
  static constexpr int GK_HOST = 32;
  static constexpr double TILE_COST = 1500.0;
  // smallest estimated cost worth a workgroup of its own (about ten products):
  // below it a small problem would be cut into slivers that each pay the
  // workgroup start and a partial tile
  static constexpr double MIN_WG_COST = 30000.0;
  static int cus() {
    static const int n = std::max(1, dev_cu_count());
    return n;
  }
  // the tasks grouped by tile (tile order, insertion order within a tile):
  // tile i owns flat[cnt[i], cnt[i+1])
  void grouped(std::vector<int>& cnt, std::vector<GTask>& flat) const {
    cnt.assign(tiles.size() + 1, 0);
    bool sorted = true;  // items added tile by tile (every first pass) keep their order as they are
    for (size_t k = 0; k < items.size(); ++k) {
      cnt[items[k].tile + 1]++;
      sorted = sorted && (k == 0 || items[k - 1].tile <= items[k].tile);
    }
    for (size_t i = 0; i < tiles.size(); ++i) cnt[i + 1] += cnt[i];
    flat.resize(items.size());
    if (sorted) {
      for (size_t k = 0; k < items.size(); ++k) flat[k] = items[k].t;
      return;
    }
    std::vector<int> pos(cnt.begin(), cnt.end() - 1);
    for (auto& t : items) flat[pos[t.tile]++] = t.t;
  }
  // estimated cost of all tiles, summed in the order plan() sums it
  double total_cost() const {
    std::vector<int> cnt;
    std::vector<GTask> flat;
    grouped(cnt, flat);
    double total = 0.0;
    for (size_t i = 0; i < tiles.size(); ++i) {
      if (cnt[i] == cnt[i + 1] && tiles[i].mode == 0) continue;
      total += TILE_COST;
      for (int t = cnt[i]; t < cnt[i + 1]; ++t) total += task_cost(flat[t].K, tiles[i].cols);
    }
    return total;
  }

  // Assign the tiles, in order, to contiguous per-workgroup ranges of about
  // equal estimated cost, at most `gpc` workgroups per CU; gpc = 0 gives
  // every tile its own workgroup (the hardware then balances the load).  The
  // cost of a range is total / (gpc * CUs), or `target` when given (a batch
  // of problems sharing the launch), and never below MIN_WG_COST.  An
  // accumulating tile (mode 0) may be cut between two workgroups: its pieces
  // write partial tiles that a second kernel adds in a fixed order.
  void plan(Plan& pl, Stream st, int gpc, double target_cost = 0.0) {
    std::vector<int> cnt;
    std::vector<GTask> flat;
    grouped(cnt, flat);
    std::vector<double> cost(gpc > 0 ? flat.size() : 0);  // estimates: only ranges of tiles need them
    double total = 0.0;
    for (size_t i = 0; i < tiles.size() && gpc > 0; ++i) {
      if (cnt[i] == cnt[i + 1] && tiles[i].mode == 0) continue;
      total += TILE_COST;
      for (int t = cnt[i]; t < cnt[i + 1]; ++t) total += (cost[t] = task_cost(flat[t].K, tiles[i].cols));
    }
    const int G = gpc > 0 ? gpc * cus() : INT32_MAX;
    const double target = gpc > 0 ? std::max(target_cost > 0.0 ? target_cost : total / G, MIN_WG_COST) : 0.0;

    std::vector<GTile> chunks;
    std::vector<int> owner;  // source tile of every chunk
    std::vector<int> ws{0};
    chunks.reserve(tiles.size());
    owner.reserve(tiles.size());
    if (gpc <= 0) ws.reserve(tiles.size() + 1);
    double acc = 0.0;
    auto emit = [&](size_t i, int t0, int t1) {
      GTile c = tiles[i];
      c.t0 = t0;
      c.t1 = t1;
      chunks.push_back(c);
      owner.push_back((int)i);
    };
    auto cut = [&]() {
      if ((int)ws.size() < G && ws.back() < (int)chunks.size()) {
        ws.push_back((int)chunks.size());
        acc = 0.0;
      }
    };
    for (size_t i = 0; i < tiles.size(); ++i) {
      const int a = cnt[i], b = cnt[i + 1];
      if (gpc <= 0) {
        if (a < b || tiles[i].mode != 0) {
          emit(i, a, b);
          cut();
        }
        continue;
      }
      if (a == b) {
        if (tiles[i].mode == 0) continue;  // nothing to add
        emit(i, a, a);                     // overwrite with zeros
        if ((acc += TILE_COST) >= target) cut();
        continue;
      }
      acc += TILE_COST;
      int s = a;
      for (int t = a; t < b; ++t) {
        acc += cost[t];
        if (acc >= target && (tiles[i].mode == 0 || t + 1 == b) && (int)ws.size() < G) {
          emit(i, s, t + 1);
          s = t + 1;
          cut();
        }
      }
      if (s < b) emit(i, s, b);
    }
    if (ws.back() < (int)chunks.size()) ws.push_back((int)chunks.size());

    // partial tiles for the tiles that were cut (their pieces are adjacent)
    int64_t npart = 0;
    std::vector<RTile> reds;
    std::vector<int64_t> poff(chunks.size(), -1);
    for (size_t j = 0; j < chunks.size();) {
      size_t e = j + 1;
      while (e < chunks.size() && owner[e] == owner[j]) ++e;
      if (e - j > 1) {
        const GTile& t = tiles[owner[j]];
        reds.push_back({t.out, nullptr, t.ld, t.rows, t.cols, (int)(e - j)});
        for (size_t q = j; q < e; ++q) {
          poff[q] = npart;
          npart += (int64_t)t.rows * t.cols;
        }
      }
      j = e;
    }
    pl.part.alloc((size_t)std::max<int64_t>(npart, 1));
    for (size_t j = 0; j < chunks.size(); ++j) chunks[j].part = poff[j] >= 0 ? pl.part.p + poff[j] : nullptr;
    for (size_t j = 0, r = 0; j < chunks.size(); ++j)
      if (poff[j] >= 0 && (j == 0 || owner[j - 1] != owner[j])) reds[r++].part = chunks[j].part;
    pl.ntiles = (int)chunks.size();
    pl.nwg = (int)ws.size() - 1;
    pl.stream = gpc > 0;
    pl.nreds = (int)reds.size();
    pl.tiles.put(std::move(chunks), st);
    pl.tasks.put(std::move(flat), st);
    pl.wstart.put(std::move(ws), st);
    pl.reds.put(std::move(reds), st);
  }
};

// one product out[blk] += coef * opA(A)[rows x K1] * B[K1 x K2] * opC(C)[K2 x cols]
struct Triple {
  int blk;
  const double* a;
  const double* b;
  const double* c;
  int lda, ldb, ldc, K1, K2, flags;  // TT_* flags
  double coef;
};
struct OutBlk {
  double* out;
  int rows, cols, ld;
};

// Workgroups per CU of the grouped-GEMM plans (0 = one tile per workgroup):
// the first pass (one product per tile, short K) is best balanced by the
// hardware; the second (long accumulations) by cost-balanced ranges.
#ifndef GEMM_GPC_PASS1
#define GEMM_GPC_PASS1 0
#endif
#ifndef GEMM_GPC_PASS2
#define GEMM_GPC_PASS2 64
#endif
#ifndef GEMM_XCD_PASS1
#define GEMM_XCD_PASS1 0
#endif
#ifndef GEMM_XCD_PASS2
#define GEMM_XCD_PASS2 0
#endif
static constexpr int MI355X_XCDS = 8;  // XCDs of the device (256 CUs, 32 per XCD)

struct TwoPass {
  GemmList::Plan p1, p2;
  DBuf ws;
  double flops = 0.0;  // algorithmic: sum of the two GEMMs of every product
  double flops1 = 0.0, flops2 = 0.0;  // pass 1 / pass 2 shares
  // Algorithmic bytes of each pass: every GEMM reads its two operands once and
  // pass 1 writes its workspace tile once; pass 2 adds the output blocks once.
  double bytes1 = 0.0, bytes2 = 0.0;
  int64_t nprod = 0;
  void run(Stream st) const {
    p1.run(st);
    p2.run(st);
  }
};

// keep2: hand the accumulating pass's product list to the caller instead of
// planning it (a batch plans it with the cost target of the whole batch).
// Operand bytes a product streams from memory in each contraction order when
// every 64-wide output tile reads its panels of the two large factors
// (op(A), op(C) and the intermediate; the psi block is small and stays in the
// caches): left first, op(A) once per column tile of T, T and op(C) once per
// column / row tile of the output; right first, op(C) once per row tile of
// U, op(A) and U once per column / row tile of the output.
static void product_traffic(double R, double K1, double K2, double C, double& left, double& right) {
  auto tiles = [](double x) { return std::ceil(x / 64.0); };
  left = 8.0 * (R * K1 * tiles(K2) + R * K2 + R * K2 * tiles(C) + K2 * C * tiles(R));
  right = 8.0 * (K2 * C * tiles(K1) + K1 * C + R * K1 * tiles(C) + K1 * C * tiles(R));
}

// order: 0 = each product in the order with fewer flops; 1 = the order that
// streams fewer bytes (product_traffic), flops deciding ties.
static void build_two_pass(const std::vector<OutBlk>& outs, const std::vector<Triple>& tr, TwoPass& tp, Stream st,
                           bool sigma = false, GemmList* keep2 = nullptr, int gpc1 = GEMM_GPC_PASS1,
                           int gpc2 = GEMM_GPC_PASS2, int xcd1 = 0, int xcd2 = 0, int order = 0) {
  // Contraction order of every full product out[R x C] += c opA(A)[R x K1]
  // B'[K1 x K2] opC(C)[K2 x C] (B' = B or its transpose): left first (T =
  // opA(A) B' in the workspace, then out += c T opC(C): 2 R K2 (K1 + C)
  // flops) or right first (U = B' opC(C), then out += c opA(A) U: 2 K1 C
  // (K2 + R) flops), whichever does fewer flops; blocks whose sector
  // dimensions change across an operator make the two differ by up to a
  // factor of several.
  std::vector<int64_t> slot(tr.size(), -1);
  std::vector<char> right(tr.size(), 0);
  int64_t ws = 0;
  for (size_t i = 0; i < tr.size(); ++i)
    if (!(tr[i].flags & (TT_IDENT_A | TT_IDENT_C))) {
      const Triple& x = tr[i];
      const double R = outs[x.blk].rows, Cc = outs[x.blk].cols;
      const double fr = (double)x.K1 * Cc * (x.K2 + R), fl = R * x.K2 * (x.K1 + Cc);
      if (order == 1) {
        double bl, br;
        product_traffic(R, x.K1, x.K2, Cc, bl, br);
        right[i] = br < bl || (br == bl && fr < fl);
      } else {
        right[i] = fr < fl;
      }
      slot[i] = ws;
      ws += right[i] ? (int64_t)x.K1 * outs[x.blk].cols : (int64_t)outs[x.blk].rows * x.K2;
    }
  tp.ws.alloc((size_t)std::max<int64_t>(ws, 1));
  // output bytes: pass 1 writes every workspace slot once, pass 2 adds to
  // every output block once; operand bytes and flops are counted per task
  double wsb = 0.0, outb = 0.0;
  for (const OutBlk& o : outs) outb += 8.0 * (double)o.rows * o.cols;
  for (size_t i = 0; i < tr.size(); ++i)
    if (slot[i] >= 0) wsb += 8.0 * (right[i] ? (double)tr[i].K1 * outs[tr[i].blk].cols : (double)outs[tr[i].blk].rows * tr[i].K2);
  tp.p1.tag = sigma ? 0 : 2;
  tp.p2.tag = sigma ? 1 : 2;
  tp.nprod = (int64_t)tr.size();
  const int tag1 = tp.p1.tag, tag2 = tp.p2.tag;
  double g1f = 0.0, g1b = 0.0, g2f = 0.0, g2b = 0.0;
  // the two passes' product lists and plans are independent: built on two
  // host threads (pass 1: the T = op(A) B' or U = B' op(C) products into
  // workspace slots; pass 2: the accumulation into the output blocks)
  auto ntiles = [](int64_t r, int64_t c) { return ((r + GemmList::TS - 1) / GemmList::TS) * ((c + GemmList::TS - 1) / GemmList::TS); };
  parallel_for(2, 2, [&](size_t which) {
    if (which == 0) {
      GemmList g1;
      int64_t n1 = 0;  // tiles of the workspace slots, one task each
      for (size_t i = 0; i < tr.size(); ++i)
        if (slot[i] >= 0) n1 += right[i] ? ntiles(tr[i].K1, outs[tr[i].blk].cols) : ntiles(outs[tr[i].blk].rows, tr[i].K2);
      g1.tiles.reserve((size_t)n1);
      g1.items.reserve((size_t)n1);
      for (size_t i = 0; i < tr.size(); ++i) {
        const Triple& x = tr[i];
        if (x.flags & (TT_IDENT_A | TT_IDENT_C)) continue;
        const int R = outs[x.blk].rows, Cc = outs[x.blk].cols;
        const int trA = (x.flags & TT_TRANS_A) ? GT_TRANS_A : 0;
        const int trC = (x.flags & TT_TRANS_C) ? GT_TRANS_B : 0;
        const bool trB = (x.flags & TT_TRANS_B) != 0;  // middle factor transposed
        if (right[i]) {
          const int b1 = g1.add_block(tp.ws.p + slot[i], x.K1, Cc, Cc, 1);
          g1.add(b1, x.K1, Cc, GTask{x.b, x.c, x.ldb, x.ldc, x.K2, (trB ? GT_TRANS_A : 0) | trC, 1.0});
        } else {
          const int b1 = g1.add_block(tp.ws.p + slot[i], R, x.K2, x.K2, 1);
          g1.add(b1, R, x.K2, GTask{x.a, x.b, x.lda, x.ldb, x.K1, trA | (trB ? GT_TRANS_B : 0), 1.0});
        }
      }
      g1f = g1.flops;
      g1b = g1.bytes;
      g1.plan(tp.p1, st, gpc1);
    } else {
      GemmList g2;
      int64_t n2 = 0;  // one task per product and output tile
      for (size_t i = 0; i < tr.size(); ++i) n2 += ntiles(outs[tr[i].blk].rows, outs[tr[i].blk].cols);
      g2.items.reserve((size_t)n2);
      std::vector<int> first(outs.size());
      for (size_t b = 0; b < outs.size(); ++b)
        first[b] = g2.add_block(outs[b].out, outs[b].rows, outs[b].cols, outs[b].ld, 0);
      for (size_t i = 0; i < tr.size(); ++i) {
        const Triple& x = tr[i];
        const int R = outs[x.blk].rows, Cc = outs[x.blk].cols;
        const int trA = (x.flags & TT_TRANS_A) ? GT_TRANS_A : 0;
        const int trC = (x.flags & TT_TRANS_C) ? GT_TRANS_B : 0;
        const bool trB = (x.flags & TT_TRANS_B) != 0;
        if (x.flags & TT_IDENT_C)
          g2.add(first[x.blk], R, Cc, GTask{x.a, x.b, x.lda, x.ldb, x.K1, trA | (trB ? GT_TRANS_B : 0), x.coef});
        else if (x.flags & TT_IDENT_A)
          g2.add(first[x.blk], R, Cc, GTask{x.b, x.c, x.ldb, x.ldc, x.K2, trC | (trB ? GT_TRANS_A : 0), x.coef});
        else if (right[i])
          g2.add(first[x.blk], R, Cc, GTask{x.a, tp.ws.p + slot[i], x.lda, Cc, x.K1, trA, x.coef});
        else
          g2.add(first[x.blk], R, Cc, GTask{tp.ws.p + slot[i], x.c, x.K2, x.ldc, x.K2, trC, x.coef});
      }
      g2f = g2.flops;
      g2b = g2.bytes;
      if (keep2)
        *keep2 = std::move(g2);
      else
        g2.plan(tp.p2, st, gpc2);
    }
  });
  tp.flops1 = g1f;
  tp.flops2 = g2f;
  tp.flops = g1f + g2f;
  tp.bytes1 = g1b + wsb;
  tp.bytes2 = g2b + outb;
  tp.p1.tag = tag1;
  tp.p2.tag = tag2;
  tp.p1.xcd = xcd1;
  tp.p2.xcd = xcd2;
}

// A plan's records with every pointer moved from an FP64 buffer to its FP32
// mirror (same element offsets): the FP32 form of the same products.
struct PlanRegion {
  const double* b64;
  size_t n;
  float* b32;
};
static void mirror_plan(const GemmList::Plan& a, GemmList::Plan& b, const PlanRegion* reg, int nreg, Stream st) {
  auto remap = [&](const double* p) -> double* {
    if (!p) return nullptr;
    for (int r = 0; r < nreg; ++r)
      if (reg[r].b64 && p >= reg[r].b64 && p < reg[r].b64 + reg[r].n) return (double*)(reg[r].b32 + (p - reg[r].b64));
    fail(-5, "internal: product operand outside the known buffers");
  };
  std::vector<GTile> tl = a.tiles.host;
  for (GTile& t : tl) {
    t.out = remap(t.out);
    t.part = remap(t.part);
  }
  std::vector<GTask> tk = a.tasks.host;
  for (GTask& t : tk) {
    t.a = remap(t.a);
    t.b = remap(t.b);
  }
  std::vector<RTile> rd = a.reds.host;
  for (RTile& r : rd) {
    r.out = remap(r.out);
    r.part = remap(r.part);
  }
  b.tiles.put(tl, st);
  b.tasks.put(tk, st);
  b.wstart.put(a.wstart.host, st);
  b.reds.put(rd, st);
  b.ntiles = a.ntiles;
  b.nwg = a.nwg;
  b.nreds = a.nreds;
  b.stream = a.stream;
  b.tag = a.tag;
  b.xcd = a.xcd;
  b.f32 = true;
}

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct Tensor {  // per-sector dense matrices of one MPS site
  Basis rowsec;  // sectors (labels)
  std::vector<int> rows, cols;
  std::vector<int64_t> off;
  DBuf data;
  int find(const Sec& s) const { return rowsec.find(s); }
  double* at(int i) const { return data.p + off[i]; }
};

enum CenterKind { C_NONE, C_TWO, C_BOND_R, C_BOND_L, C_T0 };

struct Center {
  CenterKind kind = C_NONE;
  int pos = -1;         // two-site step i (C_TWO, C_T0) or bond c (C_BOND_*)
  Tensor t;             // matrices: TWO: psi per sector (dimX x dimY); BOND_R: (k_a x dimY(a));
                        // BOND_L: (dimX(b) x k_b); T0: (dimX(m) x d_m)
};

struct Step {
  int i = -1;
  std::unique_ptr<Store> X, Y;
  Enl EX, EY;
  Basis psi;  // sectors with dims as (dimX) ; dimY separately
  std::vector<int> dx, dy;
  std::vector<int64_t> off;
  int64_t n = 0;
  DBuf in, out, diag;
  TwoPass plan;
  // FP32 mirror of the sigma evaluation (built on first use): operator
  // stores, vectors, workspace and partial tiles as float arrays, and the
  // same plan with every record pointer moved to the mirror.
  std::vector<Triple> trs;  // the sigma products (kept for the energy adjoint)
  bool f32_ready = false;
  DBuf x32, y32, in32, out32, ws32, p1part32, p2part32;
  GemmList::Plan q1, q2;
  // the accumulating pass's products while its plan waits for the batch's
  // cost target
  GemmList g2;
  bool p2_pending = false;
  double flops = 0.0, bytes = 0.0;
  double method_flops = -1.0;  // with structurally zero piece pairs skipped (< 0: not counted)
  int64_t ntasks = 0;
  std::vector<std::array<int, 5>> shapes;  // per tile task: rows, K1, K2, cols, flags
  DBuf proj;                     // projection vectors of the lower states (excited-state solves)
  int nproj = 0;
  int site = -1;                 // i of the sites (i, i+1), kept when i is reset
  uint64_t genX = 0, genY = 0;   // generations of the blocks X and Y were built from
};

// Device bytes of enlarged blocks kept for reuse, over all engines of the
// process, and their ceiling (two fifths of the device memory).
static std::atomic<int64_t> g_enl_cache_bytes{0};
static int64_t enl_cache_budget() {
  static const int64_t b = (int64_t)(dev_total_memory() / 5 * 2);
  return b;
}

// stream of the noise draws of step i in pass p: NOISE_STREAM | p << 16 | i
static const uint64_t NOISE_STREAM = (uint64_t)0x4E4F << 40;

// binds a device-memory pool to the calling thread for one scope
// A timing event recorded on a stream, freed on every way out of its scope
// (an error between two events leaves none behind).
struct Event {
  void* p = nullptr;
  explicit Event(Stream st) : p(dev_event_record(st)) {}
  Event(const Event&) = delete;
  Event& operator=(const Event&) = delete;
  ~Event() {
    if (p) try {
        dev_event_free(p);
      } catch (...) {
      }
  }
  void* release() {
    void* q = p;
    p = nullptr;
    return q;
  }
};

struct PoolBind {
  DevPool* prev;
  explicit PoolBind(DevPool* p) : prev(p ? dev_pool_bind(p) : nullptr), set(p != nullptr) {}
  ~PoolBind() {
    if (set) dev_pool_bind(prev);
  }
  bool set;
};

// State of one Davidson solve (Davidson 1975; section "The effective
// Hamiltonian equation"), advanced phase by phase so that the solves of
// several engines on one stream can run in lockstep.
struct DavState {
  double* xres = nullptr;  // normalised Ritz vector on exit
  double tol = 0.0;        // residual-norm tolerance
  bool f32 = false;        // sigma with FP32 operands (FP32 or BF16x3 products)
  double eps = 6e-8;       // relative rounding of those products
  int ms = 2, k = 0, it = 1;
  double theta = 0.0, rbest = INFINITY;
  int stall = 0;
  bool conv = false, done = false;
};
// Small job arrays for the kernels, staged through page-locked memory: each
// upload is appended and copied asynchronously.  Space is reused only after
// reset(), which the caller issues right after a stream sync (when every
// copy and every kernel reading the arrays has finished); when the space
// runs out, a larger pair takes over and the old one is released at the
// next reset, so pointers handed out before stay valid until then.  Scalars
// the host needs come back through fetch(): one gather kernel and one copy.
struct Staging {
  Stream st = nullptr;
  DevPool* pool = nullptr;
  char* host = nullptr;
  char* dev = nullptr;
  size_t cap = 0, used = 0;
  double* sdev = nullptr;   // gathered scalars (device)
  double* shost = nullptr;  // gathered scalars (page-locked host)
  size_t scap = 0;
  std::vector<std::pair<void*, void*>> retired;  // (page-locked, device) to release at reset

  Staging(Stream s, DevPool* p) : st(s), pool(p) {}
  Staging(const Staging&) = delete;
  Staging& operator=(const Staging&) = delete;
  ~Staging() {
    try {
      dev_sync(st);
    } catch (...) {
    }
    release_retired();
    host_free_pinned(host);
    host_free_pinned(shost);
    PoolBind b(pool);
    if (dev) dev_free(dev);
    if (sdev) dev_free(sdev);
  }
  void release_retired() {
    PoolBind b(pool);
    for (auto& r : retired) {
      host_free_pinned(r.first);
      if (r.second) dev_free(r.second);
    }
    retired.clear();
  }
  void reset() {
    used = 0;
    release_retired();
  }
  template <class T>
  const T* up(const std::vector<T>& v) {
    const size_t b = std::max<size_t>(v.size() * sizeof(T), 8);
    size_t off = (used + 255) & ~(size_t)255;
    if (off + b > cap) {
      if (host || dev) retired.push_back({host, dev});
      cap = std::max<size_t>({2 * cap, b, (size_t)1 << 20});
      {
        PoolBind pb(pool);
        dev = (char*)dev_alloc(cap);
      }
      host = (char*)host_alloc_pinned(cap);
      off = 0;
    }
    if (!v.empty()) {
      std::memcpy(host + off, v.data(), v.size() * sizeof(T));
      dev_h2d_async(dev + off, host + off, v.size() * sizeof(T), st);
    }
    used = off + b;
    return (const T*)(dev + off);
  }
  // shost[i] = *src[i] once the stream has been synchronised
  void fetch(const std::vector<const double*>& src) {
    if (src.empty()) return;
    if (src.size() > scap) {
      if (shost || sdev) retired.push_back({shost, sdev});
      scap = std::max<size_t>(2 * src.size(), 64);
      {
        PoolBind pb(pool);
        sdev = (double*)dev_alloc(scap * sizeof(double));
      }
      shost = (double*)host_alloc_pinned(scap * sizeof(double));
    }
    const double* const* d = up(src);
    launch_scalars(d, (int)src.size(), sdev, st);
    dev_d2h_async(shost, sdev, src.size() * sizeof(double), st);
  }
};

struct Engine;
struct BatchLaunch;
static void davidson_lockstep(const std::vector<Engine*>& E, std::vector<DavState>& D, BatchLaunch* bl,
                              Staging& sg);

struct Engine {
  Problem P;
  Stream st = nullptr;
  int device = 0;
  uint64_t seed = 7;
  double dav_tol = 1e-9;
  int dav_max_sub = 32, dav_max_iter = 200;
  std::string err;
  std::vector<std::map<Sec, long long>> caps;
  std::vector<Basis> dims;  // bond dimensions (kept)
  std::vector<std::unique_ptr<Store>> Lb, Rb;
  // Renormalised blocks kept only at every ckpt-th bond (0: every bond):
  // the others are rebuilt from the nearest kept block and the MPS tensors
  // when a step needs them, and dropped again when the sweep has passed.
  int ckpt = 0;
  int64_t n_rebuilt = 0;    // blocks rebuilt since the statistics were reset
  double t_rebuilt = 0.0;   // host wall seconds of those rebuilds
  double block_bytes_max = 0.0;  // largest device bytes held by the blocks at once
  std::vector<Tensor> U, V;  // left tensors U[i]: bond i+1 sectors (dimX x k); right V[i]: bond i (k x dimY)
  Center cen;
  Step step;
  bool mps_ready = false;
  double emin = INFINITY, elast = NAN, wdisc = 0.0, wdisc_sweep = 0.0;
  std::vector<double> trace;
  bool warned = false;
  // statistics
  double t_sigma = 0, t_micro = 0, f_sigma = 0, t_block = 0, b_sigma = 0, max_enl_bytes = 0;
  double t_pass1 = 0, t_pass2 = 0, f_pass1 = 0, f_pass2 = 0, b_pass1 = 0, b_pass2 = 0;
  int64_t n_pass1 = 0, n_pass2 = 0;
  double t_sigma32 = 0, f_sigma32 = 0;
  // the method-work counter: method flops and performed flops of the FP64
  // sigma calls on steps where it was on
  double f_method = 0, f_method_perf = 0;
  int64_t n_sigma32 = 0;
  // host wall seconds of the parts of a micro-iteration outside Davidson
  enum { PH_ENLARGE, PH_TASKS, PH_PLAN, PH_DIAG, PH_GUESS, PH_SVD, PH_RENORM, PH_N };
  double t_phase[PH_N] = {};
  struct PhaseTimer {
    double& acc;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    explicit PhaseTimer(double& a) : acc(a) {}
    ~PhaseTimer() { acc += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
  };
  // noise (section "Convergence scheme"): uniform, magnitude <= 0.5 gamma
  // w_disc of the previous left- or right-sweep, added before each decomposition
  double noise = 0.0;
  double wd_prev = 0.0, wd_pass = 0.0;
  int64_t n_pass = 0;  // passes since the MPS was created or imported
  int prec = 0;             // 0: FP64 sigma; 1 / 2: FP32 / BF16x3 sigma in Davidson + FP64 refinement
  double mixed_tol = 1e-5;  // Davidson tolerance of the FP32 phase
  int refine_steps = 1;     // FP64 Davidson steps after the FP32 phase
  int renorm_prec = 0;      // renormalisation products: 0 FP64, 1 FP32, 2 BF16x3
  double refine_tol = 0.0;  // > 0: refinement steps stop once the FP64 residual norm is below it
  int64_t n_sigma = 0;
  // Davidson iterations replayed from a recorded launch sequence (0: the
  // host drives every iteration; k > 0: k replays between host checks)
  int dav_graph = 0;
  double t_dgraph = 0.0;  // seconds of the replayed segments (sigma and the rest)
  double t_dgraph_rec = 0.0;  // host seconds spent recording and instantiating
  Stream cap_stream = nullptr;  // recording stream when the work runs on the default stream
  double f_dgraph = 0.0;  // sigma flops inside them
  int64_t n_dgraph_sigma = 0, n_dgraph_replay = 0, n_dgraph_record = 0;
  // Davidson work buffers
  DBuf dV, dW, dHs, dsmall, dpartial, dx_, dax, dr, dt;
  double* hpin = nullptr;   // page-locked scalars read back after a stream sync
  std::unique_ptr<Staging> stage;  // job arrays of this engine's own Davidson
  DevPool* pool = nullptr;  // the context's device-memory pool
  bool defer_p2 = false;    // prepare() leaves the accumulating pass unplanned
  // workgroups per CU of the sigma plans (0 = one tile per workgroup), set by
  // sadmrg_autotune
  int gpc1 = GEMM_GPC_PASS1, gpc2 = GEMM_GPC_PASS2;
  // XCD-grouped workgroup order of the two sigma passes (0: dispatch order,
  // else the XCD count), set by sadmrg_set_xcd_order
  int xcd1 = GEMM_XCD_PASS1, xcd2 = GEMM_XCD_PASS2;
  // contraction order of the sigma products (0: fewer flops, 1: fewer bytes
  // streamed), set by sadmrg_set_contraction_order
  int corder = 0;
  // Enlarged blocks kept from the previous pass (section "Sweeping"): while
  // a left-to-right pass renews the left blocks, the right blocks are the
  // ones the previous right-to-left pass built, so the enlargement of the
  // right block at step i is the one that pass made at step i (and the
  // other way round).  Entry i of each side holds the enlarged store, the
  // generation of the block it came from and its enlarged basis.
  struct EnlCache {
    uint64_t src = 0;
    Basis E;
    std::unique_ptr<Store> st;
    int64_t bytes = 0;
  };
  std::vector<EnlCache> cacheX, cacheY;
  std::vector<std::pair<int, int>> cache_fifo;  // (side 0 = X / 1 = Y, site), oldest first
  bool enl_cache_on = true;
  bool enl_cache_on_saved = true;  // the setting while the method-work counter is on

  Engine() = default;
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;
  ~Engine() {
    clear_enl_cache();
    stage.reset();
    host_free_pinned(hpin);
    dev_stream_destroy(cap_stream);
  }

  void drop_cache_entry(EnlCache& c) {
    if (c.st) g_enl_cache_bytes -= c.bytes;
    c.st.reset();
    c.bytes = 0;
    c.src = 0;
  }
  void clear_enl_cache() {
    for (auto& c : cacheX) drop_cache_entry(c);
    for (auto& c : cacheY) drop_cache_entry(c);
    cache_fifo.clear();
  }
  // keep an enlarged store for the next pass if the byte ceiling allows,
  // giving up this engine's oldest entries first
  void cache_put(int side, int site, uint64_t src, const Basis& E, std::unique_ptr<Store> st) {
    if (!enl_cache_on || !st || site < 0) return;
    auto& vec = side == 0 ? cacheX : cacheY;
    if ((int)vec.size() < P.L) vec.resize(P.L);
    drop_cache_entry(vec[site]);
    const int64_t bytes = 8 * st->total;
    const int64_t cap = enl_cache_budget();
    size_t q = 0;
    while (true) {
      int64_t cur = g_enl_cache_bytes.load();
      if (cur + bytes <= cap) {
        if (g_enl_cache_bytes.compare_exchange_weak(cur, cur + bytes)) break;
        continue;
      }
      // evict the oldest of this engine's entries
      while (q < cache_fifo.size()) {
        auto [sd, k] = cache_fifo[q++];
        auto& v2 = sd == 0 ? cacheX : cacheY;
        if (k < (int)v2.size() && v2[k].st) {
          drop_cache_entry(v2[k]);
          break;
        }
      }
      if (q >= cache_fifo.size() && g_enl_cache_bytes.load() + bytes > cap) {
        cache_fifo.erase(cache_fifo.begin(), cache_fifo.begin() + q);
        return;  // does not fit
      }
    }
    cache_fifo.erase(cache_fifo.begin(), cache_fifo.begin() + q);
    EnlCache& c = vec[site];
    c.src = src;
    c.E.sec = E.sec;
    c.E.dim = E.dim;
    c.st = std::move(st);
    c.bytes = bytes;
    cache_fifo.push_back({side, site});
  }
  // the kept enlargement of block src for basis E, if there is one
  std::unique_ptr<Store> cache_take(int side, int site, const Store& src, const Basis& E) {
    auto& vec = side == 0 ? cacheX : cacheY;
    if (site < 0 || site >= (int)vec.size() || !vec[site].st) return nullptr;
    EnlCache& c = vec[site];
    std::unique_ptr<Store> out;
    if (c.src == src.gen && c.E.sec == E.sec && c.E.dim == E.dim) {
      g_enl_cache_bytes -= c.bytes;
      out = std::move(c.st);
      c.bytes = 0;
      c.src = 0;
    } else {
      drop_cache_entry(c);
    }
    return out;
  }

  void check_target() const {
    if (P.N < 0) fail(-1, "target not set");
    if (!P.have_ints) fail(-1, "integrals not set");
  }

  // ---- tables
  void build_caps() {
    auto lm = left_mult(P), rm = right_mult(P);
    caps.assign(P.L + 1, {});
    for (int k = 0; k <= P.L; ++k) {
      for (auto& [s, c] : lm[k]) {
        auto it = rm[k].find(s);
        if (it != rm[k].end()) caps[k][s] = std::min(c, it->second);
      }
      if (caps[k].empty()) fail(-2, "the target symmetry sector is empty");
    }
  }

  // ---- boundary blocks
  std::unique_ptr<Store> left_boundary() {
    auto s = std::make_unique<Store>();
    s->side = 'L';
    s->bond = 0;
    s->basis.sec = {{0, 0, 0}};
    s->basis.dim = {1};
    s->add(K(F_H), 0, 0, 0, false);
    for (int y = 0; y < P.L; ++y) s->add(K(F_S, 0, y, 0), 1, 1, P.orb[y], true);
    s->allocate(st);
    return s;
  }
  std::unique_ptr<Store> right_boundary() {
    auto s = std::make_unique<Store>();
    s->side = 'R';
    s->bond = P.L;
    s->basis.sec = {{P.N, P.twoS, P.irrep}};
    s->basis.dim = {1};
    s->add(K(F_H), 0, 0, 0, false);
    for (int x = 0; x < P.L; ++x) s->add(K(F_S, 0, x, 0), 1, 1, P.orb[x], true);
    s->allocate(st);
    return s;
  }

  // ---- renormalisation: left O' = U^T O U, right O' = V O V^T
  std::unique_ptr<Store> renormalize(const Store& E, const Tensor& T, const Basis& nb, bool left,
                                     const float* E32 = nullptr, int prec32 = 0) {
    auto out = std::make_unique<Store>();
    out->side = E.side;
    out->bond = E.bond;
    out->orbs = E.orbs;
    out->basis = nb;
    // the class layouts over the new basis, built on host threads in order of
    // first use, then the operators in the enlarged store's order
    {
      std::vector<int> cls;  // enlarged-store layouts in order of first use
      std::vector<char> seen(E.lays.size(), 0);
      for (auto& o : E.ops)
        if (!seen[(size_t)o.lay]) seen[(size_t)o.lay] = 1, cls.push_back(o.lay);
      std::vector<std::unique_ptr<Layout>> built(cls.size());
      parallel_for(cls.size(), ENLARGE_HOST_THREADS, [&](size_t q) {
        const Layout& L = *E.lays[(size_t)cls[q]];
        built[q] = out->make_layout(L.tk, L.dN, L.dG);
      });
      for (auto& L : built) out->insert_layout(std::move(L));
    }
    for (auto& o : E.ops) {
      const Layout& L = *E.lays[o.lay];
      out->add(o.key, L.tk, L.dN, L.dG, o.odd);
    }
    out->allocate(st);
    // every new sector's index in the enlarged basis and in the tensor
    const int nsec = (int)nb.sec.size();
    std::vector<int> emap((size_t)nsec), tmap((size_t)nsec);
    for (int j = 0; j < nsec; ++j) {
      emap[(size_t)j] = E.basis.find(nb.sec[(size_t)j]);
      tmap[(size_t)j] = T.find(nb.sec[(size_t)j]);
    }
    // the products of every operator (independent: built on host threads),
    // then laid end to end in operator order
    std::vector<std::vector<std::pair<OutBlk, Triple>>> per(out->ops.size());
    parallel_for(out->ops.size(), ENLARGE_HOST_THREADS, [&](size_t i) {
      const Layout& NL = out->lay((int)i);
      const Layout& EL = E.lay((int)i);
      std::vector<std::pair<OutBlk, Triple>>& pr = per[i];
      for (size_t b = 0; b < NL.bra.size(); ++b) {
        const int eb = emap[(size_t)NL.bra[b]], ek = emap[(size_t)NL.ket[b]];
        const int tb = tmap[(size_t)NL.bra[b]], tkk = tmap[(size_t)NL.ket[b]];
        if (eb < 0 || ek < 0 || tb < 0 || tkk < 0) fail(-1, "internal: renormalisation sector missing");
        const int eblk = EL.find(eb, ek);
        if (eblk < 0) continue;
        const int rows = nb.dim[NL.bra[b]], cols = nb.dim[NL.ket[b]];
        const OutBlk ob{out->ptr((int)i, (int)b), rows, cols, cols};
        Triple t{};
        t.b = E.ptr((int)i, eblk);
        t.ldb = E.basis.dim[ek];
        t.coef = 1.0;
        t.a = T.at(tb);
        t.lda = T.cols[tb];
        t.K1 = E.basis.dim[eb];
        t.c = T.at(tkk);
        t.ldc = T.cols[tkk];
        t.K2 = E.basis.dim[ek];
        t.flags = left ? TT_TRANS_A : TT_TRANS_C;  // left: U^T O U ; right: V O V^T
        pr.push_back({ob, t});
      }
    });
    size_t np = 0;
    for (auto& v : per) np += v.size();
    std::vector<OutBlk> outs;
    std::vector<Triple> trs;
    outs.reserve(np);
    trs.reserve(np);
    for (auto& v : per)
      for (auto& [ob, t] : v) {
        outs.push_back(ob);
        trs.push_back(t);
        trs.back().blk = (int)outs.size() - 1;
      }
    per.clear();
    TwoPass tp;
    build_two_pass(outs, trs, tp, st);
    if (prec32 == 0) {
      tp.run(st);
    } else {
      // The same products in reduced precision: FP32 copies of the enlarged
      // store (the sigma mirror when given), of the tensor, of the output,
      // workspace and partial tiles; FP32 (prec32 1) or BF16x3 (2) products
      // with FP32 accumulation; the new block converted back to FP64.
      DBuf e32, t32, o32, w32, q1p, q2p;
      auto fbuf = [](DBuf& b, int64_t count) { b.alloc((size_t)std::max<int64_t>((count + 1) / 2, 1)); };
      if (!E32) {
        fbuf(e32, E.total);
        launch_cvt_d2f((float*)e32.p, E.data.p, E.total, st);
        E32 = (const float*)e32.p;
      }
      fbuf(t32, (int64_t)T.data.n);
      launch_cvt_d2f((float*)t32.p, T.data.p, (int64_t)T.data.n, st);
      fbuf(o32, out->total);
      dev_zero(o32.p, o32.n * 8, st);
      fbuf(w32, (int64_t)tp.ws.n);
      fbuf(q1p, (int64_t)tp.p1.part.n);
      fbuf(q2p, (int64_t)tp.p2.part.n);
      const PlanRegion reg[] = {{E.data.p, (size_t)E.total, (float*)E32},
                                {T.data.p, T.data.n, (float*)t32.p},
                                {out->data.p, (size_t)out->total, (float*)o32.p},
                                {tp.ws.p, tp.ws.n, (float*)w32.p},
                                {tp.p1.part.p, tp.p1.part.n, (float*)q1p.p},
                                {tp.p2.part.p, tp.p2.part.n, (float*)q2p.p}};
      GemmList::Plan q1, q2;
      mirror_plan(tp.p1, q1, reg, 6, st);
      mirror_plan(tp.p2, q2, reg, 6, st);
      q1.run(st, prec32 == 2);
      q2.run(st, prec32 == 2);
      launch_cvt_f2d(out->data.p, (const float*)o32.p, out->total, st);
    }
    dev_sync(st);
    return out;
  }

  // ==========================================================================
  // Energy adjoint: the spin-summed 1- and 2-RDMs as derivatives of
  // E = <psi|H_eff|psi> at a two-site centre with respect to the folded
  // integrals W.  E is linear in W through the complementary operators of every
  // block; reverse-mode differentiation runs the sigma products, the
  // enlargements (materialisation, integral-weighted combinations) and the
  // renormalisations backwards with transposed products, and collects
  // d E / d W[e] on the host from the coefficients' linear forms.
  // ==========================================================================

  // Xbar, Ybar of the centre's enlarged stores from the sigma products:
  // for sigma[blk] += coef opA(A) B opC(C) and E = sum psi[blk] . sigma[blk],
  // Abar and Cbar are products of psi blocks with the other factor.
  void seed_adjoints() {
    Store &X = *step.X, &Y = *step.Y;
    X.alloc_adj(st);
    Y.alloc_adj(st);
    std::vector<OutBlk> outs;
    std::map<double*, int> oid;
    auto out_of = [&](Store& S, const double* blk, int rows, int cols) -> int {
      double* a = S.adj_of(blk);
      auto it = oid.find(a);
      if (it != oid.end()) return it->second;
      outs.push_back({a, rows, cols, cols});
      return oid[a] = (int)outs.size() - 1;
    };
    std::vector<Triple> at;
    for (const Triple& t : step.trs) {
      const int blk = t.blk;
      const double* O = step.in.p + step.off[blk];
      const int R = step.dx[blk], C = step.dy[blk];
      const bool hasA = !(t.flags & TT_IDENT_A), hasC = !(t.flags & TT_IDENT_C);
      const bool trA = (t.flags & TT_TRANS_A) != 0, trC = (t.flags & TT_TRANS_C) != 0;
      // sigma[blk] (R x C) += coef opA(A) [R x K1] B [K1 x K2] opC(C) [K2 x C];
      // without C, B is K1 x C; without A, B is R x K2
      if (hasA) {
        Triple a{};
        a.coef = t.coef;
        if (!trA) {  // A is R x K1
          a.blk = out_of(X, t.a, R, t.K1);
          a.a = O, a.lda = C, a.K1 = C;
          if (hasC) {  // Abar += O opC(C)^T B^T
            a.b = t.c, a.ldb = t.ldc, a.K2 = t.K2;
            a.c = t.b, a.ldc = t.ldb;
            a.flags = (trC ? 0 : TT_TRANS_B) | TT_TRANS_C;
          } else {  // Abar += O B^T
            a.b = t.b, a.ldb = t.ldb;
            a.flags = TT_IDENT_C | TT_TRANS_B;
          }
        } else {  // A is K1 x R
          a.blk = out_of(X, t.a, t.K1, R);
          a.a = t.b, a.lda = t.ldb;
          if (hasC) {  // Abar += B opC(C) O^T
            a.K1 = t.K2;
            a.b = t.c, a.ldb = t.ldc, a.K2 = C;
            a.c = O, a.ldc = C;
            a.flags = (trC ? TT_TRANS_B : 0) | TT_TRANS_C;
          } else {  // Abar += B O^T
            a.K1 = C;
            a.b = O, a.ldb = C;
            a.flags = TT_IDENT_C | TT_TRANS_B;
          }
        }
        at.push_back(a);
      }
      if (hasC) {
        Triple c{};
        c.coef = t.coef;
        if (!trC) {  // C is K2 x C
          c.blk = out_of(Y, t.c, t.K2, C);
          if (hasA) {  // Cbar += B^T opA(A)^T O
            c.a = t.b, c.lda = t.ldb, c.K1 = t.K1;
            c.b = t.a, c.ldb = t.lda, c.K2 = R;
            c.c = O, c.ldc = C;
            c.flags = TT_TRANS_A | (trA ? 0 : TT_TRANS_B);
          } else {  // Cbar += B^T O
            c.b = t.b, c.ldb = t.ldb, c.K2 = R;
            c.c = O, c.ldc = C;
            c.flags = TT_IDENT_A | TT_TRANS_B;
          }
        } else {  // C is C x K2
          c.blk = out_of(Y, t.c, C, t.K2);
          c.a = O, c.lda = C, c.K1 = R;
          if (hasA) {  // Cbar += O^T opA(A) B
            c.b = t.a, c.ldb = t.lda, c.K2 = t.K1;
            c.c = t.b, c.ldc = t.ldb;
            c.flags = TT_TRANS_A | (trA ? TT_TRANS_B : 0);
          } else {  // Cbar += O^T B
            c.b = t.b, c.ldb = t.ldb;
            c.flags = TT_IDENT_C | TT_TRANS_A;
          }
        }
        at.push_back(c);
      }
    }
    TwoPass tp;
    build_two_pass(outs, at, tp, st);
    tp.run(st);
    dev_sync(st);
  }

  // Ebar of an enlarged store from Rbar of the block renormalised from it:
  // left R = U^T E U  ->  Ebar = U Rbar U^T;  right R = V E V^T  ->  Ebar = V^T Rbar V
  void renorm_backward(const Store& R, Store& E, const Tensor& T, bool left) {
    E.alloc_adj(st);
    std::vector<OutBlk> outs;
    std::vector<Triple> trs;
    const Basis& nb = R.basis;
    for (size_t i = 0; i < R.ops.size(); ++i) {
      const Layout& NL = R.lay((int)i);
      const Layout& EL = E.lay((int)i);
      for (size_t b = 0; b < NL.bra.size(); ++b) {
        const Sec &sb = nb.sec[NL.bra[b]], &sk = nb.sec[NL.ket[b]];
        const int eb = E.basis.find(sb), ek = E.basis.find(sk);
        const int tb = T.find(sb), tkk = T.find(sk);
        if (eb < 0 || ek < 0 || tb < 0 || tkk < 0) fail(-1, "internal: renormalisation sector missing");
        const int eblk = EL.find(eb, ek);
        if (eblk < 0) continue;
        const int kb = nb.dim[NL.bra[b]], kk = nb.dim[NL.ket[b]];
        const int rows = E.basis.dim[eb], cols = E.basis.dim[ek];
        outs.push_back({E.adj.p + E.ops[i].off + EL.eoff[eblk], rows, cols, cols});
        Triple t{};
        t.blk = (int)outs.size() - 1;
        t.coef = 1.0;
        t.a = T.at(tb), t.lda = T.cols[tb], t.K1 = kb;
        t.b = R.adj.p + R.ops[i].off + NL.eoff[b], t.ldb = kk;
        t.c = T.at(tkk), t.ldc = T.cols[tkk], t.K2 = kk;
        t.flags = left ? TT_TRANS_C : TT_TRANS_A;
        trs.push_back(t);
      }
    }
    TwoPass tp;
    build_two_pass(outs, trs, tp, st);
    tp.run(st);
    dev_sync(st);
  }

  // Xbar of the block and d E / d W from Ebar of the store enlarged from it.
  void enlarge_backward(Store& X, EnlargeTrace& tr, std::vector<double>& G) {
    Store& Out = *tr.out;
    Store& T = tr.cb.T;
    X.alloc_adj(st);
    if (!T.ops.empty()) T.alloc_adj(st);
    // (1) transposed materialisation: every source block collects
    //     scale * op^T(Ebar sub-block) over the entries that read it
    struct Grp {
      double* dst;
      int rows, cols, ld;
      std::vector<GatherSrc> src;
    };
    std::map<double*, int> gid;
    std::vector<Grp> groups;
    std::vector<TraceJob> jobs;
    std::vector<const Entry*> jent;
    for (const std::vector<Entry>& part : tr.mat.parts)
      for (const Entry& en : part) {
        double* dsub = Out.adj.p + en.dst;
        if (en.src.kind == GS_IDENT) {  // identity on the block: the coefficient may be an integral
          if (en.term->wl.n > 0) {
            jobs.push_back({dsub, en.rows, en.ld});
            jent.push_back(&en);
          }
          continue;
        }
        const double* s = en.src.src;
        double* sadj = X.owns(s) ? X.adj_of(s) : (T.owns(s) ? T.adj_of(s) : nullptr);
        if (!sadj) fail(-1, "internal: materialisation source outside the block and its combinations");
        const bool trn = en.src.kind == GS_TRANS;
        auto it = gid.find(sadj);
        int g;
        if (it == gid.end()) {
          g = (int)groups.size();
          gid[sadj] = g;
          groups.push_back({sadj, trn ? en.cols : en.rows, trn ? en.rows : en.cols, en.src.ld, {}});
        } else {
          g = it->second;
        }
        groups[g].src.push_back({dsub, en.ld, en.src.kind, en.src.scale});
      }
    {
      std::vector<GatherDst> dsts;
      std::vector<GatherSrc> srcs;
      for (const Grp& g : groups) {
        GatherDst d{g.dst, g.rows, g.cols, g.ld, (int)srcs.size(), 0};
        for (const GatherSrc& s : g.src) srcs.push_back(s);
        d.s1 = (int)srcs.size();
        dsts.push_back(d);
      }
      DArr<GatherDst> ddst;
      DArr<GatherSrc> dsrc;
      ddst.put(dsts, st);
      dsrc.put(srcs, st);
      launch_gather(ddst.p, (int)dsts.size(), dsrc.p, st);
      dev_sync(st);
    }
    // (2) integral-valued coefficients of identity terms: d E / d coef = unit * trace
    if (!jobs.empty()) {
      DArr<TraceJob> dj;
      dj.put(jobs, st);
      DBuf tv;
      tv.alloc(jobs.size());
      launch_traces(dj.p, (int)jobs.size(), tv.p, st);
      std::vector<double> h(jobs.size());
      dev_d2h(h.data(), tv.p, h.size() * 8, st);
      for (size_t j = 0; j < jobs.size(); ++j) {
        const WLin& w = jent[j]->term->wl;
        const double d = jent[j]->unit * h[j];
        for (int q = 0; q < w.n; ++q) G[w.e[q]] += w.m[q] * d;
      }
    }
    if (T.ops.empty()) return;
    // (3) transposed combinations: Xbar[op_i] += c_i op_i^T(Tbar[o])
    {
      std::map<int, std::vector<std::pair<int, int>>> by_op;  // X op -> (combo, input index)
      for (size_t o = 0; o < T.ops.size(); ++o)
        for (size_t i = 0; i < tr.cb.inputs[o].size(); ++i) by_op[tr.cb.inputs[o][i].op].push_back({(int)o, (int)i});
      std::vector<ComboOut> outs;
      std::vector<ComboIn> ins;
      int64_t maxn = 0;
      for (auto& [op, lst] : by_op) {
        const int xl = X.ops[op].lay;
        bool any_adj = false;
        for (auto& [o, i] : lst) any_adj |= tr.cb.inputs[o][i].adj;
        if (any_adj) X.ensure_adjoint_map(xl, st);
        ComboOut co;
        co.out = X.adj.p + X.ops[op].off;
        co.nnz = X.lays[xl]->nnz;
        co.i0 = (int)ins.size();
        ins.push_back({co.out, 1.0, 0});
        for (auto& [o, i] : lst) {
          const Combos::In& in = tr.cb.inputs[o][i];
          ins.push_back({T.adj.p + T.ops[o].off, in.c, in.adj ? 1 : 0});
        }
        co.i1 = (int)ins.size();
        co.perm = any_adj ? X.lays[xl]->perm.p : nullptr;
        co.fac = any_adj ? X.lays[xl]->facT.p : nullptr;
        outs.push_back(co);
        maxn = std::max(maxn, co.nnz);
      }
      DArr<ComboOut> dout;
      DArr<ComboIn> din;
      dout.put(outs, st);
      din.put(ins, st);
      launch_combo(dout.p, (int)outs.size(), din.p, maxn, st);
      dev_sync(st);
    }
    // (4) d E / d c_i = < Tbar[o], op_i(X[op_i]) >, one GEMM per operator class
    std::map<int, std::vector<int>> combos_of_class;  // X layout -> combos
    for (size_t o = 0; o < T.ops.size(); ++o) {
      const Layout& L = *T.lays[T.ops[o].lay];
      combos_of_class[X.layout(L.tk, L.dN, L.dG)].push_back((int)o);
    }
    for (auto& [xl, cos] : combos_of_class) {
      const int64_t nnz = X.lays[xl]->nnz;
      if (nnz == 0) continue;
      std::map<std::pair<int, int>, int> col;  // (X op, adj) -> column
      for (int o : cos)
        for (const Combos::In& in : tr.cb.inputs[o]) col.emplace(std::make_pair(in.op, in.adj ? 1 : 0), 0);
      int nc = 0;
      for (auto& kv : col) kv.second = nc++;
      const int M = (int)cos.size();
      DBuf Am, Bm, Gm;
      Am.alloc((size_t)M * nnz);
      Bm.alloc((size_t)nc * nnz);
      Gm.alloc((size_t)M * nc);
      dev_zero(Gm.p, (size_t)M * nc * 8, st);
      for (int r = 0; r < M; ++r) dev_d2d(Am.p + (int64_t)r * nnz, T.adj.p + T.ops[cos[r]].off, (size_t)nnz * 8, st);
      std::vector<ComboOut> outs;
      std::vector<ComboIn> ins;
      bool any_adj = false;
      for (auto& [key, c] : col) {
        if (key.second) {
          any_adj = true;
          X.ensure_adjoint_map(xl, st);
          ComboOut co{Bm.p + (int64_t)c * nnz, nnz, (int)ins.size(), (int)ins.size() + 1, X.lays[xl]->perm.p,
                      X.lays[xl]->fac.p};
          ins.push_back({X.data.p + X.ops[key.first].off, 1.0, 1});
          outs.push_back(co);
        } else {
          dev_d2d(Bm.p + (int64_t)c * nnz, X.data.p + X.ops[key.first].off, (size_t)nnz * 8, st);
        }
      }
      if (any_adj) {
        DArr<ComboOut> dout;
        DArr<ComboIn> din;
        dout.put(outs, st);
        din.put(ins, st);
        launch_combo(dout.p, (int)outs.size(), din.p, nnz, st);
      }
      GemmList gl;
      const int first = gl.add_block(Gm.p, M, nc, nc, 0);
      gl.add(first, M, nc, GTask{Am.p, Bm.p, (int)nnz, (int)nnz, (int)nnz, GT_TRANS_B, 1.0});
      GemmList::Plan pl;
      gl.plan(pl, st, GEMM_GPC_PASS2);
      pl.run(st);
      std::vector<double> g((size_t)M * nc);
      dev_d2h(g.data(), Gm.p, g.size() * 8, st);
      for (int r = 0; r < M; ++r)
        for (const Combos::In& in : tr.cb.inputs[cos[r]]) {
          const double d = g[(size_t)r * nc + col[{in.op, in.adj ? 1 : 0}]];
          for (int q = 0; q < in.w.n; ++q) G[in.w.e[q]] += in.w.m[q] * d;
        }
    }
  }

  // d E / d W (L^4, accumulated into G) for E = <psi|H_eff|psi> / <psi|psi> at
  // the current two-site centre; returns E (without E_const).
  double energy_gradient(std::vector<double>& G) {
    if (!mps_ready) fail(-1, "no MPS");
    if (cen.kind != C_TWO) fail(-1, "RDMs need a two-site centre (after a sweep, a micro-iteration or an import)");
    const int i = cen.pos;
    prepare(i);
    const int64_t n = step.n;
    dsmall.ensure(8 * 64 + 64 * 64);
    dpartial.ensure(256 * 64);
    launch_dots(step.in.p, n, 1, step.in.p, n, dsmall.p, dpartial.p, st);
    launch_normalize(step.in.p, dsmall.p, n, st);
    sigma_fixed(false, false);  // H_0: the density matrices of the state itself
    launch_dots(step.in.p, n, 1, step.out.p, n, dsmall.p + 1, dpartial.p, st);
    double e;
    dev_d2h(&e, dsmall.p + 1, 8, st);
    G.assign((size_t)P.L * P.L * P.L * P.L, 0.0);
    seed_adjoints();
    // With checkpoints the walks rebuild the dropped blocks from the kept
    // ones below (left) or above (right) and drop each block again once its
    // adjoint has been passed on.
    {  // left blocks: bond i down to 0
      EnlargeTrace tr;
      trace_enlarge(P, lblock(i), step.EX, true, st, tr);
      if (tr.out->total != step.X->total) fail(-1, "internal: enlarged store mismatch in the adjoint");
      tr.out->adj = std::move(step.X->adj);
      for (int k = i;; --k) {
        enlarge_backward(*Lb[k], tr, G);
        tr.out->adj.release();
        if (k == 0) break;
        EnlargeTrace prev;
        std::set<Sec> keep(dims[k].sec.begin(), dims[k].sec.end());
        Store& Lp = lblock(k - 1);
        Enl E = left_enl(P, k, Lp.basis, &keep);
        trace_enlarge(P, Lp, E, true, st, prev);
        renorm_backward(*Lb[k], *prev.out, U[k - 1], true);
        Lb[k]->adj.release();
        if (k < i && !kept_bond(k)) Lb[k].reset();
        tr = std::move(prev);
      }
      Lb[0]->adj.release();
    }
    {  // right blocks: bond i+2 up to L
      EnlargeTrace tr;
      trace_enlarge(P, rblock(i + 2), step.EY, false, st, tr);
      if (tr.out->total != step.Y->total) fail(-1, "internal: enlarged store mismatch in the adjoint");
      tr.out->adj = std::move(step.Y->adj);
      for (int k = i + 2;; ++k) {
        enlarge_backward(*Rb[k], tr, G);
        tr.out->adj.release();
        if (k == P.L) break;
        EnlargeTrace prev;
        std::set<Sec> keep(dims[k].sec.begin(), dims[k].sec.end());
        Store& Rp = rblock(k + 1);
        Enl E = right_enl(P, k, Rp.basis, &keep);
        trace_enlarge(P, Rp, E, false, st, prev);
        renorm_backward(*Rb[k], *prev.out, V[k], false);
        Rb[k]->adj.release();
        if (k > i + 2 && !kept_bond(k)) Rb[k].reset();
        tr = std::move(prev);
      }
      Rb[P.L]->adj.release();
    }
    return e;
  }

  // The paper's calc2DM outputs from d E / d W (section "CheMPS2 library",
  // the DMRG object): gamma_pq = <E_pq>, Gamma^A_{ij;kl} = sum_{st}
  // <a+_is a+_jt a_lt a_ks> and Gamma^B_{ij;kl} = sum_{st} (-1)^(s-t) (same).
  // E is linear in the folded integrals W_pqrs = (pq|rs) + (h_pq d_rs + h_rs
  // d_pq)/(N-1), and every blocking formula reads W with each creator next to
  // its own annihilator partner, so the derivative holds for any W with the
  // symmetry of a real two-body operator, (pq|rs) = (rs|pq) = (qp|sr); its
  // average over those four images is D_pqrs = Gamma^A_{pr;qs} / 2, with no
  // symmetrisation over (pq|rs) = (qp|rs).  Gamma^B is the average over the
  // 2S+1 members of the multiplet (the singlet-embedding ghost is traced
  // out): for an SU(2)-invariant two-body density the spin structure leaves
  // Gamma^B_{ij;kl} = -(Gamma^A_{ij;kl} + 2 Gamma^A_{ij;lk}) / 3.
  // layout 0: rdm2[i][j][k][l] = Gamma^A_{ij;kl}; layout 1 (chemist):
  // rdm2[p][q][r][s] = Gamma^A_{pr;qs}, so E = E_c + sum h gamma + 1/2 sum
  // (pq|rs) rdm2_pqrs.  <S^2> = -N(N-4)/4 - 1/2 sum_ij Gamma^A_{ij;ji}.
  double rdms(double* rdm1, double* rdm2, int layout = 0, double* rdm2b = nullptr, double* s2 = nullptr) {
    std::vector<double> G;
    const double e = energy_gradient(G);
    const int L = P.L;
    auto ix = [L](int p, int q, int r, int s) { return (((size_t)p * L + q) * L + r) * L + s; };
    std::vector<double> GA((size_t)L * L * L * L);  // Gamma^A_{pr;qs} at [p][r][q][s]
    for (int p = 0; p < L; ++p)
      for (int q = 0; q < L; ++q)
        for (int r = 0; r < L; ++r)
          for (int s = 0; s < L; ++s)
            GA[ix(p, r, q, s)] =
                (G[ix(p, q, r, s)] + G[ix(r, s, p, q)] + G[ix(q, p, s, r)] + G[ix(s, r, q, p)]) / 2.0;
    if (rdm2) {
      if (layout == 0)
        std::copy(GA.begin(), GA.end(), rdm2);
      else
        for (int p = 0; p < L; ++p)
          for (int q = 0; q < L; ++q)
            for (int r = 0; r < L; ++r)
              for (int s = 0; s < L; ++s) rdm2[ix(p, q, r, s)] = GA[ix(p, r, q, s)];
    }
    if (rdm2b)
      for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j)
          for (int k = 0; k < L; ++k)
            for (int l = 0; l < L; ++l) rdm2b[ix(i, j, k, l)] = -(GA[ix(i, j, k, l)] + 2.0 * GA[ix(i, j, l, k)]) / 3.0;
    if (rdm1)  // gamma_ik = sum_j Gamma^A_{ij;kj} / (N - 1)
      for (int p = 0; p < L; ++p)
        for (int q = 0; q < L; ++q) {
          double v = 0.0;
          for (int j = 0; j < L; ++j) v += GA[ix(p, j, q, j)];
          rdm1[p * L + q] = v / (P.N - 1);
        }
    if (s2) {
      double t = 0.0;
      for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) t += GA[ix(i, j, j, i)];
      *s2 = -0.25 * P.N * (P.N - 4) - 0.5 * t;
    }
    return e + P.e_const;
  }

  // ---- excited states by projection (section "CheMPS2 library", the DMRG
  // object): after a state Psi_k is found it is pushed back with a weight
  // eta_k > 0 and the next solve uses H_m = H_0 + sum_k eta_k |Psi_k><Psi_k|,
  // which projects the lower states out of the target sector.  On the
  // current two-site space at sites (i, i+1) the extra term is
  //   sigma += sum_k eta_k <phi_k|x> phi_k,  phi_k = P_i Psi_k,
  // with P_i the projector onto the space of the current left states at bond
  // i, the two sites and the current right states at bond i+2.  Psi_k is kept
  // as its left-end object C (bond 1) and right-normalised tensors V_k[1..];
  // the overlaps are carried as environments updated with the sweep:
  //   OR[b] = <current right states at bond b | Psi_k's right states>,
  //   M[c]  = <current left states at bond c | Psi_k's part left of bond c>,
  // and at step i, X_i = (M[i] V_k[i]) recoupled into the left-enlarged basis
  // at bond i+1 (X_0 = C), phi_k = X_i V_k[i+1] OR[i+2]^T, M[i+1] = U[i]^T X_i.
  struct Lower {
    double eta = 0.0;
    std::vector<Basis> dims;  // Psi_k's bond bases
    Tensor C;                 // left-end object: bond-1 sectors, 1 x dims[1]
    std::vector<Tensor> V;    // V[1..L-1], right-normalised
    std::vector<Tensor> M;    // M[c], c = 1..L-1
    std::vector<Tensor> OR;   // OR[b], b = 2..L
    Tensor X;                 // X_i of the prepared step
  };
  std::vector<Lower> lower;
  DBuf projc, projpart;  // scalars and partial sums of the projector dots

  static void copy_meta(const Tensor& a, Tensor& b) {
    b.rowsec = a.rowsec;
    b.rows = a.rows;
    b.cols = a.cols;
  }
  void copy_tensor(const Tensor& a, Tensor& b) {
    copy_meta(a, b);
    alloc_tensor(b);
    int64_t tot = 0;
    for (size_t j = 0; j < a.rows.size(); ++j) tot += (int64_t)a.rows[j] * a.cols[j];
    if (tot) dev_d2d(b.data.p, a.data.p, (size_t)tot * 8, st);
  }
  void zero_tensor(Tensor& t) {
    int64_t tot = 0;
    for (size_t j = 0; j < t.rows.size(); ++j) tot += (int64_t)t.rows[j] * t.cols[j];
    dev_zero(t.data.p, (size_t)std::max<int64_t>(tot, 1) * 8, st);
  }
  void run_triples(const std::vector<OutBlk>& outs, const std::vector<Triple>& trs) {
    if (!trs.empty()) {
      TwoPass tp;
      build_two_pass(outs, trs, tp, st);
      tp.run(st);
    }
    dev_sync(st);
  }
  // the step a centre of this kind leads to (as sadmrg_prepare_step)
  int next_step() const {
    switch (cen.kind) {
      case C_TWO:
      case C_T0:
      case C_BOND_R:
        return cen.pos;
      case C_BOND_L:
        return cen.pos - 2;
      default:
        fail(-1, "no centre");
    }
  }
  // OR[c] = V[c] (1_site x OR[c+1]) V_k[c]^T over the right-enlarged pieces
  void lower_or(Lower& w, int c) {
    Tensor& o = w.OR[c];
    o = Tensor();
    for (size_t j = 0; j < dims[c].sec.size(); ++j) {
      const int kj = w.dims[c].find(dims[c].sec[j]);
      if (kj < 0 || V[c].find(dims[c].sec[j]) < 0 || w.V[c].find(dims[c].sec[j]) < 0) continue;
      o.rowsec.sec.push_back(dims[c].sec[j]);
      o.rowsec.dim.push_back(dims[c].dim[j]);
      o.rows.push_back(dims[c].dim[j]);
      o.cols.push_back(w.dims[c].dim[kj]);
    }
    alloc_tensor(o);
    zero_tensor(o);
    Enl ec = right_enl(P, c, dims[c + 1], nullptr), ek = right_enl(P, c, w.dims[c + 1], nullptr);
    std::vector<OutBlk> outs;
    std::vector<Triple> trs;
    for (size_t j = 0; j < o.rowsec.sec.size(); ++j) {
      const Sec& be = o.rowsec.sec[j];
      const int vc = V[c].find(be), vk = w.V[c].find(be), pc = ec.find(be), pk = ek.find(be);
      if (pc < 0 || pk < 0) continue;
      outs.push_back({o.at((int)j), o.rows[j], o.cols[j], o.cols[j]});
      for (const Piece& qc : ec.pieces[pc]) {
        const Sec& b = dims[c + 1].sec[qc.sub];
        const int ob = w.OR[c + 1].find(b);
        if (ob < 0) continue;
        for (const Piece& qk : ek.pieces[pk]) {
          if (qk.n != qc.n || !(w.dims[c + 1].sec[qk.sub] == b)) continue;
          Triple t{};
          t.blk = (int)outs.size() - 1;
          t.a = V[c].at(vc) + qc.off;
          t.lda = V[c].cols[vc];
          t.K1 = dims[c + 1].dim[qc.sub];
          t.b = w.OR[c + 1].at(ob);
          t.ldb = w.OR[c + 1].cols[ob];
          t.K2 = w.dims[c + 1].dim[qk.sub];
          t.c = w.V[c].at(vk) + qk.off;
          t.ldc = w.V[c].cols[vk];
          t.flags = TT_TRANS_C;
          t.coef = 1.0;
          trs.push_back(t);
        }
      }
    }
    run_triples(outs, trs);
  }
  // X_i: (M[i] V_k[i]) recoupled into the current left-enlarged basis at bond
  // i+1 (columns: Psi_k's bond i+1); X_0 is the left-end object
  void lower_x(Lower& w, int i) {
    if (i == 0) {
      copy_tensor(w.C, w.X);
      return;
    }
    Enl el = left_enl(P, i + 1, dims[i], nullptr), ek = right_enl(P, i, w.dims[i + 1], nullptr);
    Tensor& x = w.X;
    x = Tensor();
    for (size_t m = 0; m < el.sec.size(); ++m) {
      const int kj = w.dims[i + 1].find(el.sec[m]);
      if (kj < 0) continue;
      x.rowsec.sec.push_back(el.sec[m]);
      x.rowsec.dim.push_back(el.dim[m]);
      x.rows.push_back(el.dim[m]);
      x.cols.push_back(w.dims[i + 1].dim[kj]);
    }
    alloc_tensor(x);
    zero_tensor(x);
    std::vector<OutBlk> outs;
    std::vector<Triple> trs;
    const Tensor& M = w.M[i];
    for (size_t ja = 0; ja < M.rowsec.sec.size(); ++ja) {
      const Sec& a = M.rowsec.sec[ja];
      const int va = w.V[i].find(a), ea = ek.find(a), ai = dims[i].find(a);
      if (va < 0 || ea < 0 || ai < 0) continue;
      for (const Piece& pc : ek.pieces[ea]) {
        const Sec& be = w.dims[i + 1].sec[pc.sub];
        const int xb = x.find(be), eb = el.find(be);
        if (xb < 0 || eb < 0) continue;
        int roff = -1;
        for (const Piece& q : el.pieces[eb])
          if (q.sub == ai && q.n == pc.n) roff = q.off;
        if (roff < 0) continue;
        outs.push_back({x.at(xb) + (int64_t)roff * x.cols[xb], M.rows[ja], x.cols[xb], x.cols[xb]});
        Triple t{};
        t.blk = (int)outs.size() - 1;
        t.a = M.at((int)ja);
        t.lda = M.cols[ja];
        t.K1 = M.cols[ja];
        t.b = w.V[i].at(va) + pc.off;
        t.ldb = w.V[i].cols[va];
        t.flags = TT_IDENT_C;
        t.coef = recouple_singlet(a.tj, LOC_TJ[pc.n], be.tj);
        trs.push_back(t);
      }
    }
    run_triples(outs, trs);
  }
  // M[i+1] = U[i]^T X_i
  void lower_m(Lower& w, int i) {
    Tensor& o = w.M[i + 1];
    o = Tensor();
    for (size_t j = 0; j < U[i].rowsec.sec.size(); ++j) {
      const int xj = w.X.find(U[i].rowsec.sec[j]);
      if (xj < 0) continue;
      o.rowsec.sec.push_back(U[i].rowsec.sec[j]);
      o.rowsec.dim.push_back(U[i].cols[j]);
      o.rows.push_back(U[i].cols[j]);
      o.cols.push_back(w.X.cols[xj]);
    }
    alloc_tensor(o);
    zero_tensor(o);
    std::vector<OutBlk> outs;
    std::vector<Triple> trs;
    for (size_t j = 0; j < o.rowsec.sec.size(); ++j) {
      const int uj = U[i].find(o.rowsec.sec[j]), xj = w.X.find(o.rowsec.sec[j]);
      if (U[i].rows[uj] != w.X.rows[xj]) fail(-1, "internal: overlap environment shape mismatch");
      outs.push_back({o.at((int)j), o.rows[j], o.cols[j], o.cols[j]});
      Triple t{};
      t.blk = (int)outs.size() - 1;
      t.a = U[i].at(uj);
      t.lda = U[i].cols[uj];
      t.K1 = U[i].rows[uj];
      t.b = w.X.at(xj);
      t.ldb = w.X.cols[xj];
      t.flags = TT_TRANS_A | TT_IDENT_C;
      t.coef = 1.0;
      trs.push_back(t);
    }
    run_triples(outs, trs);
  }
  // every environment for the step the centre leads to
  void lower_rebuild() {
    if (lower.empty() || !mps_ready) return;
    const int L = P.L, i = next_step();
    for (Lower& w : lower) {
      w.M.clear();
      w.M.resize(L + 1);
      w.OR.clear();
      w.OR.resize(L + 1);
      Tensor& o = w.OR[L];  // boundary: one sector, <1|1>
      o.rowsec = dims[L];
      o.rows = {1};
      o.cols = {1};
      alloc_tensor(o);
      const double one = 1.0;
      dev_h2d(o.data.p, &one, 8, st);
      for (int b = L - 1; b >= i + 2; --b) lower_or(w, b);
      for (int c = 0; c < i; ++c) {
        lower_x(w, c);
        lower_m(w, c);
      }
    }
  }
  // snapshot of the current MPS (centre at the left end) as a lower state
  void lower_push(double eta) {
    if (!(eta > 0.0) || !std::isfinite(eta)) fail(-1, "eta must be positive");
    if (!mps_ready || cen.kind != C_TWO || cen.pos != 0)
      fail(-1, "push an excitation when the two-site centre is at the left end (after a sweep or an import there)");
    if (lower.size() >= 64) fail(-1, "at most 64 lower states");
    Lower w;
    w.eta = eta;
    w.dims = dims;
    w.V.resize(P.L);
    for (int k = 2; k < P.L; ++k) copy_tensor(V[k], w.V[k]);
    // the left-end object: one row per sector of bond 1 (bond 0 is one
    // state); row m = |row_m| (row_m / |row_m|): C holds the norms, V[1] the
    // normalised rows, Psi_k normalised as a whole
    const int ns = (int)cen.t.rows.size();
    std::vector<double> nrm(ns, 0.0);
    projc.ensure(64);
    projpart.ensure(256 * 64);
    for (int j = 0; j < ns; ++j) {
      if (cen.t.rows[j] != 1) fail(-1, "internal: left-end object with more than one row per sector");
      launch_dots(cen.t.at(j), cen.t.cols[j], 1, cen.t.at(j), cen.t.cols[j], projc.p, projpart.p, st);
      dev_d2h(&nrm[j], projc.p, 8, st);
    }
    double tot = 0.0;
    for (double v : nrm) tot += v;
    if (!(tot > 0.0)) fail(-1, "the current MPS is zero");
    Basis b1;
    std::vector<int> src;
    for (int j = 0; j < ns; ++j)
      if (nrm[j] > 0.0) {
        b1.sec.push_back(cen.t.rowsec.sec[j]);
        b1.dim.push_back(1);
        src.push_back(j);
      }
    w.dims[1] = b1;
    Tensor& v1 = w.V[1];
    v1.rowsec = b1;
    w.C.rowsec = b1;
    for (int j : src) {
      v1.rows.push_back(1);
      v1.cols.push_back(cen.t.cols[j]);
      w.C.rows.push_back(1);
      w.C.cols.push_back(1);
    }
    alloc_tensor(v1);
    alloc_tensor(w.C);
    std::vector<double> cv;
    for (size_t q = 0; q < src.size(); ++q) {
      const int j = src[q];
      dev_d2d(v1.at((int)q), cen.t.at(j), (size_t)cen.t.cols[j] * 8, st);
      launch_scal(v1.at((int)q), 1.0 / std::sqrt(nrm[j]), cen.t.cols[j], st);
      cv.push_back(std::sqrt(nrm[j] / tot));
    }
    dev_h2d(w.C.data.p, cv.data(), cv.size() * 8, st);
    lower.push_back(std::move(w));
    step.i = -1;  // the next prepare adds the projector
    lower_rebuild();
  }
  void lower_clear() {
    lower.clear();
    step.i = -1;
  }
  // phi_k of step i into step.proj (scaled by sqrt(eta_k)), added to the diagonal
  void lower_phi(int i) {
    const int K = (int)lower.size();
    step.nproj = K;
    if (!K) return;
    step.proj.alloc((size_t)K * std::max<int64_t>(step.n, 1));
    dev_zero(step.proj.p, (size_t)K * std::max<int64_t>(step.n, 1) * 8, st);
    for (int k = 0; k < K; ++k) {
      Lower& w = lower[k];
      lower_x(w, i);
      Enl ek = right_enl(P, i + 1, w.dims[i + 2], nullptr);
      std::vector<OutBlk> outs;
      std::vector<Triple> trs;
      double* base = step.proj.p + (int64_t)k * step.n;
      for (size_t m = 0; m < step.psi.sec.size(); ++m) {
        const Sec& ms = step.psi.sec[m];
        const int xm = w.X.find(ms), vm = w.V[i + 1].find(ms), em = ek.find(ms);
        if (xm < 0 || vm < 0 || em < 0) continue;
        for (const Piece& q : step.EY.pieces[m]) {
          const Sec& b = dims[i + 2].sec[q.sub];
          const int ob = w.OR[i + 2].find(b);
          if (ob < 0) continue;
          for (const Piece& qk : ek.pieces[em]) {
            if (qk.n != q.n || !(w.dims[i + 2].sec[qk.sub] == b)) continue;
            outs.push_back({base + step.off[m] + q.off, step.dx[m], dims[i + 2].dim[q.sub], step.dy[m]});
            Triple t{};
            t.blk = (int)outs.size() - 1;
            t.a = w.X.at(xm);
            t.lda = w.X.cols[xm];
            t.K1 = w.X.cols[xm];
            t.b = w.V[i + 1].at(vm) + qk.off;
            t.ldb = w.V[i + 1].cols[vm];
            t.K2 = w.dims[i + 2].dim[qk.sub];
            t.c = w.OR[i + 2].at(ob);
            t.ldc = w.OR[i + 2].cols[ob];
            t.flags = TT_TRANS_C;
            t.coef = std::sqrt(w.eta);
            trs.push_back(t);
          }
        }
      }
      run_triples(outs, trs);
    }
    launch_add_squares(step.diag.p, step.proj.p, step.n, K, step.n, st);
    dev_sync(st);
  }
  // y += sum_k (phi_k . x) phi_k (phi_k scaled by sqrt(eta_k)); x, y device vectors of the step
  void add_projectors(const double* x, double* y) {
    if (!step.nproj) return;
    projc.ensure(64);
    projpart.ensure(256 * 64);
    launch_dots(step.proj.p, step.n, step.nproj, x, step.n, projc.p, projpart.p, st);
    launch_combo_vec(step.proj.p, step.n, step.nproj, projc.p, 1.0, step.n, y, 1.0, st);
  }

  // ---- random initial MPS (section "DMRG" of the library description)
  void init_mps(int D) {
    check_target();
    if (D < 1) fail(-1, "D must be positive");
    build_caps();
    dims.assign(P.L + 1, {});
    for (int k = 0; k <= P.L; ++k) dims[k] = to_basis(distribute(D, caps[k]));
    U.clear();
    U.resize(P.L);
    V.clear();
    V.resize(P.L);
    DBuf work, tmp;
    for (int k = P.L - 1; k >= 1; --k) {
      std::set<Sec> keep(dims[k].sec.begin(), dims[k].sec.end());
      Enl E = right_enl(P, k, dims[k + 1], &keep);
      std::vector<int> ids;
      int64_t need = 0, wneed = 0;
      std::map<Sec, int> newd;
      for (int qi = 0; qi < (int)dims[k].sec.size(); ++qi) {
        const int e = E.find(dims[k].sec[qi]);
        if (e < 0) continue;
        ids.push_back(qi);
        const int d = dims[k].dim[qi], n = E.dim[e];
        need += (int64_t)d * n;
        const int r = std::min(d, n);
        wneed += (int64_t)d * n + (int64_t)r * r + r;
      }
      // random (d x n) per sector, SVD, keep the orthonormal rows
      tmp.alloc((size_t)std::max<int64_t>(need, 1));
      int64_t o = 0;
      std::vector<int64_t> offs;
      for (int qi : ids) {
        const int e = E.find(dims[k].sec[qi]);
        const int d = dims[k].dim[qi], n = E.dim[e];
        launch_fill_uniform(tmp.p + o, (int64_t)d * n, seed, ((uint64_t)k << 20) | (uint64_t)qi, st);
        offs.push_back(o);
        o += (int64_t)d * n;
      }
      Tensor t;
      int64_t toff = 0, uoff = 0;
      std::vector<SvdJob> jobs;
      std::vector<int> rr;
      for (size_t j = 0; j < ids.size(); ++j) {
        const int e = E.find(dims[k].sec[ids[j]]);
        const int d = dims[k].dim[ids[j]], n = E.dim[e];
        const int r = std::min(d, n);
        t.rowsec.sec.push_back(dims[k].sec[ids[j]]);
        t.rowsec.dim.push_back(r);
        t.rows.push_back(r);
        t.cols.push_back(n);
        t.off.push_back(toff);
        toff += (int64_t)r * n;
        uoff += (int64_t)d * r + r;
        rr.push_back(r);
        newd[dims[k].sec[ids[j]]] = r;
      }
      t.data.alloc((size_t)std::max<int64_t>(toff, 1));
      DBuf ubuf;
      ubuf.alloc((size_t)std::max<int64_t>(uoff, 1));
      work.alloc((size_t)std::max<int64_t>(wneed, 1));
      int64_t wo = 0, uo = 0;
      int maxs = 1;
      for (size_t j = 0; j < ids.size(); ++j) {
        const int e = E.find(dims[k].sec[ids[j]]);
        const int d = dims[k].dim[ids[j]], n = E.dim[e], r = rr[j];
        SvdJob jb{tmp.p + offs[j], d, n, n, ubuf.p + uo, ubuf.p + uo + (int64_t)d * r, t.at((int)j), work.p + wo};
        jobs.push_back(jb);
        uo += (int64_t)d * r + r;
        wo += (int64_t)d * n + (int64_t)r * r + r;
        maxs = std::max(maxs, r);
      }
      DArr<SvdJob> dj;
      dj.put(jobs, st);
      launch_svd(dj.p, (int)jobs.size(), maxs, st);
      dev_sync(st);
      V[k] = std::move(t);
      dims[k] = to_basis(newd);
    }
    // T0: random left tensor of site 0 (enlarged-left at bond 1 x bond 1)
    {
      std::set<Sec> keep(dims[1].sec.begin(), dims[1].sec.end());
      Enl E0 = left_enl(P, 1, dims[0], &keep);
      Tensor t;
      int64_t o = 0;
      std::vector<int> qis;
      for (int qi = 0; qi < (int)dims[1].sec.size(); ++qi) {
        const int e = E0.find(dims[1].sec[qi]);
        if (e < 0) continue;
        t.rowsec.sec.push_back(dims[1].sec[qi]);
        t.rowsec.dim.push_back(E0.dim[e]);
        t.rows.push_back(E0.dim[e]);
        t.cols.push_back(dims[1].dim[qi]);
        t.off.push_back(o);
        o += (int64_t)E0.dim[e] * dims[1].dim[qi];
        qis.push_back(qi);
      }
      t.data.alloc((size_t)std::max<int64_t>(o, 1));
      for (size_t j = 0; j < qis.size(); ++j)
        launch_fill_uniform(t.at((int)j), (int64_t)t.rows[j] * t.cols[j], seed, (uint64_t)qis[j], st);
      cen.kind = C_T0;
      cen.pos = 0;
      cen.t = std::move(t);
    }
    build_blocks_from_tensors(0);
    mps_ready = true;
    n_pass = 0;
    wd_prev = wd_pass = 0.0;
    lower_rebuild();
  }

  // Build left blocks 0..i and right blocks L..i+2 from the stored tensors.
  void build_blocks_from_tensors(int i) {
    clear_enl_cache();
    step = Step();
    Lb.clear();
    Rb.clear();
    Lb.resize(P.L + 1);
    Rb.resize(P.L + 1);
    Lb[0] = left_boundary();
    for (int k = 0; k < i; ++k) {  // the block below each new one is dropped unless kept
      build_left(k);
      if (!keep_left(k, i)) Lb[k].reset();
    }
    Rb[P.L] = right_boundary();
    for (int k = P.L - 1; k >= i + 2; --k) {
      build_right(k);
      if (!keep_right(k + 1, i)) Rb[k + 1].reset();
    }
    note_block_bytes();
    step.i = -1;
  }
  // left block at bond k+1 from the block at bond k and the tensor U[k]
  // (enlargement by site k, then renormalisation)
  void build_left(int k) {
    std::set<Sec> keep(dims[k + 1].sec.begin(), dims[k + 1].sec.end());
    Enl E = left_enl(P, k + 1, Lb[k]->basis, &keep);
    auto Xe = enlarge(P, *Lb[k], E, true, st, nullptr);
    Lb[k + 1] = renormalize(*Xe, U[k], dims[k + 1], true);
  }
  // right block at bond k from the block at bond k+1 and the tensor V[k]
  void build_right(int k) {
    std::set<Sec> keep(dims[k].sec.begin(), dims[k].sec.end());
    Enl E = right_enl(P, k, Rb[k + 1]->basis, &keep);
    auto Ye = enlarge(P, *Rb[k + 1], E, false, st, nullptr);
    Rb[k] = renormalize(*Ye, V[k], dims[k], false);
  }
  bool kept_bond(int b) const { return ckpt <= 0 || b == 0 || b == P.L || b % ckpt == 0; }
  // The left block at bond b, rebuilt upwards from the nearest block below
  // it when it was dropped (the blocks in between are rebuilt too and kept:
  // a right-to-left pass needs them next).
  Store& lblock(int b) {
    if (!Lb[b]) {
      const auto t0 = std::chrono::steady_clock::now();
      int c = b - 1;
      while (!Lb[c]) --c;  // Lb[0] is always kept
      for (int k = c; k < b; ++k)
        if (!Lb[k + 1]) {
          build_left(k);
          ++n_rebuilt;
        }
      t_rebuilt += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      note_block_bytes();
    }
    return *Lb[b];
  }
  // The right block at bond b, rebuilt downwards from the nearest block above.
  Store& rblock(int b) {
    if (!Rb[b]) {
      const auto t0 = std::chrono::steady_clock::now();
      int c = b + 1;
      while (!Rb[c]) ++c;  // Rb[L] is always kept
      for (int k = c - 1; k >= b; --k)
        if (!Rb[k]) {
          build_right(k);
          ++n_rebuilt;
        }
      t_rebuilt += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      note_block_bytes();
    }
    return *Rb[b];
  }
  // With checkpoints, keep around step i only the blocks a sweep through i
  // may need next: left bonds (cl, i+1] with cl the last kept bond below i,
  // right bonds [i+1, cr) with cr the first kept bond above i+2, and every
  // kept bond.
  bool keep_left(int k, int i) const {
    if (kept_bond(k)) return true;
    int cl = std::max(0, i - 1);
    while (cl > 0 && !kept_bond(cl)) --cl;
    return k > cl && k <= i + 1;
  }
  bool keep_right(int k, int i) const {
    if (kept_bond(k)) return true;
    int cr = std::min(P.L, i + 3);
    while (cr < P.L && !kept_bond(cr)) ++cr;
    return k >= i + 1 && k < cr;
  }
  void drop_blocks(int i) {
    if (ckpt <= 0) return;
    for (int k = 1; k < P.L; ++k) {
      if (Lb[k] && !keep_left(k, i)) Lb[k].reset();
      if (Rb[k] && !keep_right(k, i)) Rb[k].reset();
    }
  }
  void note_block_bytes() {
    double b = 0.0;
    for (auto& x : Lb)
      if (x) b += 8.0 * x->total;
    for (auto& x : Rb)
      if (x) b += 8.0 * x->total;
    block_bytes_max = std::max(block_bytes_max, b);
  }

  // ---- prepare the two-site step at sites (i, i+1)
  void prepare(int i) {
    if (step.i == i && step.X && step.Y) {
      build_guess();
      return;
    }
    auto t0 = std::chrono::steady_clock::now();
    const int c = i + 1;
    Store& Lk = lblock(i);
    Store& Rk = rblock(i + 2);
    Enl el0 = left_enl(P, c, Lk.basis, nullptr), er0 = right_enl(P, c, Rk.basis, nullptr);
    std::set<Sec> keep;
    for (auto& s : el0.sec)
      if (er0.find(s) >= 0) keep.insert(s);
    // the finished step's enlarged blocks may serve the next pass
    cache_put(0, step.site, step.genX, step.EX, std::move(step.X));
    cache_put(1, step.site, step.genY, step.EY, std::move(step.Y));
    step = Step();
    step.i = i;
    step.site = i;
    step.EX = left_enl(P, c, Lk.basis, &keep);
    step.EY = right_enl(P, c, Rk.basis, &keep);
    step.genX = Lk.gen;
    step.genY = Rk.gen;
    int64_t ne = 0;
    // An enlargement built here is traced in two parts: its layouts (and
    // device memory) first, so that the sigma products can be planned from
    // them on a host thread while this one emits and gathers the enlarged
    // operators' entries.
    EnlargeTrace trX, trY;
    bool freshX = false, freshY = false;
    {
      PhaseTimer pt(t_phase[PH_ENLARGE]);
      step.X = cache_take(0, i, Lk, step.EX);
      if (!step.X) {
        trace_layouts(P, Lk, step.EX, true, st, trX);
        step.X = std::move(trX.out);
        step.X->allocate(st);
        freshX = true;
      }
      step.Y = cache_take(1, i, Rk, step.EY);
      if (!step.Y) {
        trace_layouts(P, Rk, step.EY, false, st, trY);
        step.Y = std::move(trY.out);
        step.Y->allocate(st);
        freshY = true;
      }
    }
    // psi layout
    step.psi.sec = step.EX.sec;
    step.n = 0;
    for (size_t m = 0; m < step.EX.sec.size(); ++m) {
      step.dx.push_back(step.EX.dim[m]);
      step.dy.push_back(step.EY.dim[m]);
      step.off.push_back(step.n);
      step.n += (int64_t)step.EX.dim[m] * step.EY.dim[m];
    }
    step.psi.dim = step.dx;
    step.in.alloc((size_t)std::max<int64_t>(step.n, 1));
    step.out.alloc((size_t)std::max<int64_t>(step.n, 1));
    step.diag.alloc((size_t)std::max<int64_t>(step.n, 1));
    {
      // the planner reads the stores' layouts only; the method counter's
      // piece lists are written by the entries part, so it runs in order
      Overlap planner(!tl_in_pool && (freshX || freshY) && !P.count_method, [this] { build_sigma_tasks(); });
      PhaseTimer pt(t_phase[PH_ENLARGE]);
      if (freshX) {
        trace_entries(P, Lk, step.EX, true, trX, *step.X);
        enlarge_finish(trX, *step.X, st, &ne);
      }
      if (freshY) {
        trace_entries(P, Rk, step.EY, false, trY, *step.Y);
        enlarge_finish(trY, *step.Y, st, &ne);
      }
      planner.join();
    }
    drop_blocks(i);
    max_enl_bytes = std::max(max_enl_bytes, 8.0 * (double)(step.X->total + step.Y->total));
    {
      PhaseTimer pt(t_phase[PH_DIAG]);
      build_diag();
      lower_phi(i);
    }
    {
      PhaseTimer pt(t_phase[PH_GUESS]);
      build_guess();
      dev_sync(st);
    }
    t_block += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  struct HTerm {
    double coef;
    int x, y;  // op index in step.X / step.Y, -1 identity
    bool yadj, hc;
  };

  std::vector<HTerm> heff_terms() {
    std::vector<HTerm> ts;
    Store &X = *step.X, &Y = *step.Y;
    const double s2 = std::sqrt(2.0), s3 = std::sqrt(3.0);
    ts.push_back({1.0, X.need(K(F_H)), -1, false, false});
    ts.push_back({1.0, -1, Y.need(K(F_H)), false, false});
    for (int y : Y.orbs) ts.push_back({-s2, X.need(K(F_S, 0, y, 0)), Y.need(K(F_C, 0, y, 0)), true, true});
    for (int x : X.orbs) ts.push_back({-s2, X.need(K(F_C, 0, x, 0)), Y.need(K(F_S, 0, x, 0)), true, true});
    const int c = step.i + 1;
    const std::vector<int>& pr = P.bare_left(c) ? X.orbs : Y.orbs;
    const bool pairs_on_x = P.bare_left(c);
    for (int a : pr)
      for (int b : pr) {
        if (b < a) continue;
        for (int tj : {0, 2}) {
          const double cb = tj == 0 ? 1.0 : s3;
          if (pairs_on_x) {
            if (a < b) {
              ts.push_back({std::sqrt(tj + 1.0), X.need(K(F_A, tj, a, b)), Y.need(K(F_P, tj, a, b)), true, true});
              ts.push_back({cb, X.need(K(F_B, tj, a, b)), Y.need(K(F_Q, tj, a, b)), false, true});
            } else {
              if (tj == 0) ts.push_back({0.5, X.need(K(F_A, 0, a, a)), Y.need(K(F_P, 0, a, a)), true, true});
              ts.push_back({cb, X.need(K(F_B, tj, a, a)), Y.need(K(F_Q, tj, a, a)), false, false});
            }
          } else {
            if (a < b) {
              ts.push_back({std::sqrt(tj + 1.0), X.need(K(F_P, tj, a, b)), Y.need(K(F_A, tj, a, b)), true, true});
              ts.push_back({cb, X.need(K(F_Q, tj, a, b)), Y.need(K(F_B, tj, a, b)), false, true});
            } else {
              if (tj == 0) ts.push_back({0.5, X.need(K(F_P, 0, a, a)), Y.need(K(F_A, 0, a, a)), true, true});
              ts.push_back({cb, X.need(K(F_Q, tj, a, a)), Y.need(K(F_B, tj, a, a)), false, false});
            }
          }
        }
      }
    return ts;
  }

  // Flops of the sigma products with the structurally zero piece pairs of
  // the enlarged operator blocks skipped: a block of an enlarged operator
  // holds (sector, local state) piece pairs, and only those a blocking term
  // writes are nonzero.  For out += c op(A) B op(C), with nzA / nzC the
  // nonzero areas of op(A) / op(C), Rnz the rows of op(A) that hold a
  // nonzero piece and Cnz the columns of op(C): left first 2 nzA K2 + 2 Rnz
  // nzC, right first 2 K1 nzC + 2 nzA Cnz, the cheaper of the two (the
  // identity factors: one GEMM).
  double method_flops(const std::vector<OutBlk>& outs, const std::vector<Triple>& trs) const {
    const Store &X = *step.X, &Y = *step.Y;
    struct Shape {
      double area = 0.0;
      int rows_nz = 0, cols_nz = 0;  // of the stored block
    };
    auto shape = [](const Store& S, const double* p, int rows, int cols) {
      Shape sh;
      const int64_t b0 = p - S.data.p;
      Store::PieceRect key{b0, -1, -1, 0, 0};
      auto it = std::lower_bound(S.pieces.begin(), S.pieces.end(), key);
      std::vector<char> r(rows, 0), c(cols, 0);
      for (; it != S.pieces.end() && it->bstart == b0; ++it) {
        sh.area += (double)it->rows * it->cols;
        for (int q = 0; q < it->rows; ++q) r[it->roff + q] = 1;
        for (int q = 0; q < it->cols; ++q) c[it->coff + q] = 1;
      }
      for (char v : r) sh.rows_nz += v;
      for (char v : c) sh.cols_nz += v;
      return sh;
    };
    double f = 0.0;
    for (const Triple& t : trs) {
      const int R = outs[t.blk].rows, C = outs[t.blk].cols;
      Shape a, c;
      int aRnz = 0, cCnz = 0;
      if (!(t.flags & TT_IDENT_A)) {  // op(A) is R x K1
        const bool tr = t.flags & TT_TRANS_A;
        a = shape(X, t.a, tr ? t.K1 : R, tr ? R : t.K1);
        aRnz = tr ? a.cols_nz : a.rows_nz;
      }
      if (!(t.flags & TT_IDENT_C)) {  // op(C) is K2 x C
        const bool tr = t.flags & TT_TRANS_C;
        c = shape(Y, t.c, tr ? C : t.K2, tr ? t.K2 : C);
        cCnz = tr ? c.rows_nz : c.cols_nz;
      }
      if (t.flags & TT_IDENT_C)
        f += 2.0 * a.area * C;
      else if (t.flags & TT_IDENT_A)
        f += 2.0 * R * c.area;
      else
        f += std::min(2.0 * a.area * t.K2 + 2.0 * aRnz * c.area, 2.0 * t.K1 * c.area + 2.0 * a.area * cCnz);
    }
    return f;
  }

  void build_sigma_tasks() {
    auto tt0 = std::chrono::steady_clock::now();
    Store &X = *step.X, &Y = *step.Y;
    const int ns = (int)step.psi.sec.size();
    std::vector<OutBlk> outs(ns);
    for (int m = 0; m < ns; ++m) outs[m] = {step.out.p + step.off[m], step.dx[m], step.dy[m], step.dy[m]};
    std::vector<Triple> trs;
    double bytes = 0.0;
    std::set<std::pair<int, int>> touched;  // (store, op) operands read
    for (const HTerm& h : heff_terms()) {
      if (h.y < 0) {  // H_X (x) 1
        const Layout& L = X.lay(h.x);
        for (size_t b = 0; b < L.bra.size(); ++b) {
          const int m = L.bra[b];
          if (L.ket[b] != m) continue;
          Triple t{};
          t.blk = m;
          t.a = X.ptr(h.x, (int)b);
          t.lda = step.dx[m];
          t.K1 = step.dx[m];
          t.b = step.in.p + step.off[m];
          t.ldb = step.dy[m];
          t.flags = TT_IDENT_C;
          t.coef = h.coef;
          trs.push_back(t);
        }
        touched.insert({0, h.x});
        continue;
      }
      if (h.x < 0) {  // 1 (x) H_Y : psi H^T
        const Layout& L = Y.lay(h.y);
        for (size_t b = 0; b < L.bra.size(); ++b) {
          const int m = L.bra[b];
          if (L.ket[b] != m) continue;
          Triple t{};
          t.blk = m;
          t.b = step.in.p + step.off[m];
          t.ldb = step.dy[m];
          t.c = Y.ptr(h.y, (int)b);
          t.ldc = step.dy[m];
          t.K2 = step.dy[m];
          t.flags = TT_IDENT_A | TT_TRANS_C;
          t.coef = h.coef;
          trs.push_back(t);
        }
        touched.insert({1, h.y});
        continue;
      }
      const Layout& XL = X.lay(h.x);
      const Layout& YL = Y.lay(h.y);
      const int tk = XL.tk;
      const bool yodd = Y.ops[h.y].odd;
      touched.insert({0, h.x});
      touched.insert({1, h.y});
      for (size_t b = 0; b < XL.bra.size(); ++b) {
        const int mb = XL.bra[b], mk = XL.ket[b];
        int yb;
        double fy = 1.0;
        if (h.yadj) {
          yb = YL.find(mk, mb);
          if (yb < 0) continue;
          fy = adjoint_factor(step.psi.sec[mk].tj, step.psi.sec[mb].tj, tk);
        } else {
          yb = YL.find(mb, mk);
          if (yb < 0) continue;
        }
        const double cs = coupling_singlet(step.psi.sec[mk].tj, step.psi.sec[mb].tj, tk);
        const double sign = (yodd && (step.psi.sec[mk].N & 1)) ? -1.0 : 1.0;
        const double f = h.coef * cs * sign * fy;
        if (f == 0.0) continue;
        const double* xa = X.ptr(h.x, (int)b);
        const double* yc = Y.ptr(h.y, yb);
        {  // sigma[mb] += f X[mb,mk] psi[mk] Yeff[mb,mk]^T
          Triple t{};
          t.blk = mb;
          t.a = xa;
          t.lda = step.dx[mk];
          t.K1 = step.dx[mk];
          t.b = step.in.p + step.off[mk];
          t.ldb = step.dy[mk];
          t.c = yc;
          t.K2 = step.dy[mk];
          if (h.yadj) {
            t.ldc = step.dy[mb];  // stored (mk <- mb): dy[mk] x dy[mb]
            t.flags = 0;
          } else {
            t.ldc = step.dy[mk];  // stored (mb <- mk): dy[mb] x dy[mk]
            t.flags = TT_TRANS_C;
          }
          t.coef = f;
          trs.push_back(t);
        }
        if (h.hc) {  // sigma[mk] += f X[mb,mk]^T psi[mb] Yeff[mb,mk]
          Triple t{};
          t.blk = mk;
          t.a = xa;
          t.lda = step.dx[mk];
          t.K1 = step.dx[mb];
          t.b = step.in.p + step.off[mb];
          t.ldb = step.dy[mb];
          t.c = yc;
          t.K2 = step.dy[mb];
          if (h.yadj) {
            t.ldc = step.dy[mb];
            t.flags = TT_TRANS_A | TT_TRANS_C;
          } else {
            t.ldc = step.dy[mk];
            t.flags = TT_TRANS_A;
          }
          t.coef = f;
          trs.push_back(t);
        }
      }
    }
    for (auto& [s, o] : touched) bytes += 8.0 * (s == 0 ? X.lay(o).nnz : Y.lay(o).nnz);
    bytes += 16.0 * step.n;
    t_phase[PH_TASKS] += std::chrono::duration<double>(std::chrono::steady_clock::now() - tt0).count();
    PhaseTimer pt(t_phase[PH_PLAN]);
    build_two_pass(outs, trs, step.plan, st, true, defer_p2 ? &step.g2 : nullptr, gpc1, gpc2, xcd1, xcd2,
                   corder);
    step.p2_pending = defer_p2;
    step.flops = step.plan.flops;
    step.bytes = bytes;
    step.ntasks = (int64_t)trs.size();
    step.method_flops = (X.has_pieces && Y.has_pieces) ? method_flops(outs, trs) : -1.0;
    step.shapes.clear();
    step.shapes.reserve(trs.size());
    for (auto& t : trs) step.shapes.push_back({outs[t.blk].rows, t.K1, t.K2, outs[t.blk].cols, t.flags});
    step.trs = std::move(trs);
  }

  void build_diag() {
    Store &X = *step.X, &Y = *step.Y;
    const int ns = (int)step.psi.sec.size();
    std::vector<std::vector<DiagTask>> per(ns);
    for (const HTerm& h : heff_terms()) {
      if (h.y < 0 || h.x < 0) {
        const bool xs = h.y < 0;
        const Store& S = xs ? X : Y;
        const int o = xs ? h.x : h.y;
        const Layout& L = S.lay(o);
        for (size_t b = 0; b < L.bra.size(); ++b) {
          const int m = L.bra[b];
          if (L.ket[b] != m) continue;
          DiagTask d{};
          if (xs) {
            d.x = S.ptr(o, (int)b);
            d.sx = step.dx[m] + 1;
          } else {
            d.y = S.ptr(o, (int)b);
            d.sy = step.dy[m] + 1;
          }
          d.coef = h.coef;
          per[m].push_back(d);
        }
        continue;
      }
      const Layout& XL = X.lay(h.x);
      const Layout& YL = Y.lay(h.y);
      const int tk = XL.tk;
      for (size_t b = 0; b < XL.bra.size(); ++b) {
        const int m = XL.bra[b];
        if (XL.ket[b] != m) continue;
        const int yb = YL.find(m, m);
        if (yb < 0) continue;
        double fy = h.yadj ? adjoint_factor(step.psi.sec[m].tj, step.psi.sec[m].tj, tk) : 1.0;
        const double cs = coupling_singlet(step.psi.sec[m].tj, step.psi.sec[m].tj, tk);
        const double sign = (Y.ops[h.y].odd && (step.psi.sec[m].N & 1)) ? -1.0 : 1.0;
        DiagTask d{X.ptr(h.x, (int)b), Y.ptr(h.y, yb), step.dx[m] + 1, step.dy[m] + 1,
                   h.coef * cs * sign * fy * (h.hc ? 2.0 : 1.0)};
        if (d.coef != 0.0) per[m].push_back(d);
      }
    }
    std::vector<DiagSec> secs;
    std::vector<DiagTask> tasks;
    for (int m = 0; m < ns; ++m) {
      DiagSec s{step.diag.p + step.off[m], step.dx[m], step.dy[m], (int)tasks.size(), 0};
      for (auto& d : per[m]) tasks.push_back(d);
      s.t1 = (int)tasks.size();
      secs.push_back(s);
    }
    DArr<DiagSec> ds;
    DArr<DiagTask> dt;
    ds.put(secs, st);
    dt.put(tasks, st);
    launch_diag(ds.p, (int)secs.size(), dt.p, st);
    dev_sync(st);
  }

  // initial guess of the micro-iteration in step.in (section "The effective
  // Hamiltonian equation": the current two-site object)
  void build_guess() {
    dev_zero(step.in.p, (size_t)std::max<int64_t>(step.n, 1) * 8, st);
    const int i = step.i;
    const int ns = (int)step.psi.sec.size();
    std::vector<OutBlk> outs;
    std::vector<Triple> trs;
    if (cen.kind == C_TWO && cen.pos == i) {
      std::vector<GatherDst> dsts;
      std::vector<GatherSrc> srcs;
      for (int m = 0; m < ns; ++m) {
        const int j = cen.t.find(step.psi.sec[m]);
        if (j < 0) continue;
        if (cen.t.rows[j] != step.dx[m] || cen.t.cols[j] != step.dy[m]) fail(-1, "internal: centre shape mismatch");
        srcs.push_back({cen.t.at(j), cen.t.cols[j], GS_NORMAL, 1.0});
        dsts.push_back({step.in.p + step.off[m], step.dx[m], step.dy[m], step.dy[m], (int)srcs.size() - 1,
                        (int)srcs.size()});
      }
      DArr<GatherDst> dd;
      DArr<GatherSrc> ds;
      dd.put(dsts, st);
      ds.put(srcs, st);
      launch_gather(dd.p, (int)dsts.size(), ds.p, st);
      dev_sync(st);
      return;
    }
    if (cen.kind == C_T0 && i == 0) {  // psi = T0 V[1]
      for (int m = 0; m < ns; ++m) {
        const int j = cen.t.find(step.psi.sec[m]);
        const int v = V[1].find(step.psi.sec[m]);
        if (j < 0 || v < 0) continue;
        if (V[1].cols[v] != step.dy[m]) fail(-1, "internal: right tensor shape mismatch");
        outs.push_back({step.in.p + step.off[m], step.dx[m], step.dy[m], step.dy[m]});
        Triple t{};
        t.blk = (int)outs.size() - 1;
        t.a = cen.t.at(j);
        t.lda = cen.t.cols[j];
        t.K1 = cen.t.cols[j];
        t.b = V[1].at(v);
        t.ldb = V[1].cols[v];
        t.flags = TT_IDENT_C;
        t.coef = 1.0;
        trs.push_back(t);
      }
    } else if (cen.kind == C_BOND_R && cen.pos == i) {
      // C[a] rows of bond i, columns (n, b) of the right-enlarged basis at bond i
      Enl Er = right_enl(P, i, dims[i + 1], nullptr);
      for (size_t ja = 0; ja < cen.t.rowsec.sec.size(); ++ja) {
        const Sec& a = cen.t.rowsec.sec[ja];
        const int ea = Er.find(a);
        if (ea < 0) continue;
        const int ai = Lb[i]->basis.find(a);
        for (auto& pc : Er.pieces[ea]) {
          const Sec& b = dims[i + 1].sec[pc.sub];
          const int m = step.psi.find(b);
          const int v = V[i + 1].find(b);
          if (m < 0 || v < 0 || ai < 0) continue;
          int roff = -1;
          for (auto& q : step.EX.pieces[m])
            if (q.sub == ai && q.n == pc.n) roff = q.off;
          if (roff < 0) continue;
          if (V[i + 1].cols[v] != step.dy[m]) fail(-1, "internal: right tensor shape mismatch");
          const double r = recouple_singlet(a.tj, LOC_TJ[pc.n], b.tj);
          const int rows = cen.t.rows[ja];
          outs.push_back({step.in.p + step.off[m] + (int64_t)roff * step.dy[m], rows, step.dy[m], step.dy[m]});
          Triple t{};
          t.blk = (int)outs.size() - 1;
          t.b = cen.t.at((int)ja) + pc.off;
          t.ldb = cen.t.cols[ja];
          t.K2 = dims[i + 1].dim[pc.sub];
          t.c = V[i + 1].at(v);
          t.ldc = V[i + 1].cols[v];
          t.flags = TT_IDENT_A;
          t.coef = r;
          trs.push_back(t);
        }
      }
    } else if (cen.kind == C_BOND_L && cen.pos == i + 2) {
      // C[b] rows (a, n) of the left-enlarged basis at bond i+2, columns bond i+2
      Enl El = left_enl(P, i + 2, dims[i + 1], nullptr);
      for (size_t jb = 0; jb < cen.t.rowsec.sec.size(); ++jb) {
        const Sec& b = cen.t.rowsec.sec[jb];
        const int eb = El.find(b);
        if (eb < 0) continue;
        const int bi = Rb[i + 2]->basis.find(b);
        for (auto& pc : El.pieces[eb]) {
          const Sec& a = dims[i + 1].sec[pc.sub];
          const int m = step.psi.find(a);
          const int u = U[i].find(a);
          if (m < 0 || u < 0 || bi < 0) continue;
          int coff = -1;
          for (auto& q : step.EY.pieces[m])
            if (q.sub == bi && q.n == pc.n) coff = q.off;
          if (coff < 0) continue;
          if (U[i].rows[u] != step.dx[m]) fail(-1, "internal: left tensor shape mismatch");
          const double r = recouple_singlet(a.tj, LOC_TJ[pc.n], b.tj);
          const int cols = cen.t.cols[jb];
          outs.push_back({step.in.p + step.off[m] + coff, step.dx[m], cols, step.dy[m]});
          Triple t{};
          t.blk = (int)outs.size() - 1;
          t.a = U[i].at(u);
          t.lda = U[i].cols[u];
          t.K1 = U[i].cols[u];
          t.b = cen.t.at((int)jb) + (int64_t)pc.off * cen.t.cols[jb];
          t.ldb = cen.t.cols[jb];
          t.flags = TT_IDENT_C;
          t.coef = r;
          trs.push_back(t);
        }
      }
    } else {
      fail(-1, "internal: no centre for this step");
    }
    TwoPass tp;
    build_two_pass(outs, trs, tp, st);
    tp.run(st);
    dev_sync(st);
  }

  // ---- FP32 mirror of the prepared step's sigma
  static void alloc_f32(DBuf& b, int64_t count) { b.alloc((size_t)std::max<int64_t>((count + 1) / 2, 1)); }

  void ensure_f32() {
    Step& S = step;
    if (S.f32_ready) return;
    Store &X = *S.X, &Y = *S.Y;
    alloc_f32(S.x32, X.total);
    alloc_f32(S.y32, Y.total);
    alloc_f32(S.in32, S.n);
    alloc_f32(S.out32, S.n);
    alloc_f32(S.ws32, (int64_t)S.plan.ws.n);
    alloc_f32(S.p1part32, (int64_t)S.plan.p1.part.n);
    alloc_f32(S.p2part32, (int64_t)S.plan.p2.part.n);
    launch_cvt_d2f((float*)S.x32.p, X.data.p, X.total, st);
    launch_cvt_d2f((float*)S.y32.p, Y.data.p, Y.total, st);
    const PlanRegion reg[] = {{X.data.p, (size_t)X.total, (float*)S.x32.p},
                              {Y.data.p, (size_t)Y.total, (float*)S.y32.p},
                              {S.in.p, (size_t)S.n, (float*)S.in32.p},
                              {S.out.p, (size_t)S.n, (float*)S.out32.p},
                              {S.plan.ws.p, S.plan.ws.n, (float*)S.ws32.p},
                              {S.plan.p1.part.p, S.plan.p1.part.n, (float*)S.p1part32.p},
                              {S.plan.p2.part.p, S.plan.p2.part.n, (float*)S.p2part32.p}};
    mirror_plan(S.plan.p1, S.q1, reg, 7, st);
    mirror_plan(S.plan.p2, S.q2, reg, 7, st);
    S.f32_ready = true;
  }

  // ---- sigma on the prepared step: step.out = H_eff step.in (FP64, or with
  // FP32 operands and FP32 accumulation when f32)
  void sigma_fixed(bool f32 = false, bool proj = true) {
    if (step.p2_pending) fail(-1, "internal: sigma plan incomplete");
    struct AddProj {  // the excited-state projectors, after the products
      Engine& e;
      bool on;
      ~AddProj() noexcept(false) {
        if (on && !std::uncaught_exceptions()) e.add_projectors(e.step.in.p, e.step.out.p);
      }
    } addp{*this, proj};
    if (f32) ensure_f32();
    const GemmList::Plan& p1 = f32 ? step.q1 : step.plan.p1;
    const GemmList::Plan& p2 = f32 ? step.q2 : step.plan.p2;
    const Event e0(st);
    if (f32) {
      launch_cvt_d2f((float*)step.in32.p, step.in.p, step.n, st);
      dev_zero(step.out32.p, step.out32.n * 8, st);  // whole mirror (n floats, rounded up)
    } else {
      dev_zero(step.out.p, (size_t)std::max<int64_t>(step.n, 1) * 8, st);
    }
    const Event e1(st);
    const bool bf3 = f32 && prec == 2;
    p1.run(st, bf3);
    const Event e2(st);
    launch_gemm(p2.tiles.p, p2.tasks.p, p2.wstart.p, p2.nwg, p2.stream, p2.tag, p2.f32, st, bf3, p2.xcd);
    const Event e3(st);
    launch_reduce(p2.reds.p, p2.nreds, p2.f32, st);
    if (f32) launch_cvt_f2d(step.out.p, (const float*)step.out32.p, step.n, st);
    const Event e4(st);
    const double t0 = dev_event_elapsed(e0.p, e1.p), t1 = dev_event_elapsed(e1.p, e2.p),
                 t2 = dev_event_elapsed(e2.p, e3.p), t3 = dev_event_elapsed(e3.p, e4.p);
    if (f32) {
      t_sigma32 += t0 + t1 + t2 + t3;
      f_sigma32 += step.flops;
      ++n_sigma32;
      return;
    }
    t_sigma += t1 + t2 + t3;
    if (step.method_flops >= 0.0) {
      f_method += step.method_flops;
      f_method_perf += step.flops;
    }
    t_pass1 += t1;
    t_pass2 += t2;
    ++n_sigma;
    f_sigma += step.flops;
    f_pass1 += step.plan.flops1;
    f_pass2 += step.plan.flops2;
    b_pass1 += step.plan.bytes1;
    b_pass2 += step.plan.bytes2;
    ++n_pass1;
    if (step.plan.p2.ntiles > 0) ++n_pass2;
    b_sigma += step.bytes;
  }
  void sigma_vec(const double* x, double* y, bool f32 = false) {
    dev_d2d(step.in.p, x, (size_t)step.n * 8, st);
    sigma_fixed(f32);
    dev_d2d(y, step.out.p, (size_t)step.n * 8, st);
  }
  // The launches of sigma_fixed (step.in to step.out) with no host wait, no
  // allocation and no timing events, for a recorded sequence; the GEMM
  // passes do nothing while *gate != 0.  record_prepare() first makes the
  // buffers it uses.
  void record_prepare(bool f32) {
    if (step.p2_pending) fail(-1, "internal: sigma plan incomplete");
    if (f32) ensure_f32();
    if (step.nproj) {
      projc.ensure(64);
      projpart.ensure(256 * 64);
    }
  }
  void sigma_record(bool f32, const int* gate) {
    const GemmList::Plan& p1 = f32 ? step.q1 : step.plan.p1;
    const GemmList::Plan& p2 = f32 ? step.q2 : step.plan.p2;
    if (f32) {
      launch_cvt_d2f((float*)step.in32.p, step.in.p, step.n, st);
      dev_zero(step.out32.p, step.out32.n * 8, st);
    } else {
      dev_zero(step.out.p, (size_t)std::max<int64_t>(step.n, 1) * 8, st);
    }
    const bool bf3 = f32 && prec == 2;
    launch_gemm(p1.tiles.p, p1.tasks.p, p1.wstart.p, p1.nwg, p1.stream, p1.tag, p1.f32, st, f32 && bf3, p1.xcd, gate);
    launch_reduce(p1.reds.p, p1.nreds, p1.f32, st, gate);
    launch_gemm(p2.tiles.p, p2.tasks.p, p2.wstart.p, p2.nwg, p2.stream, p2.tag, p2.f32, st, bf3, p2.xcd, gate);
    launch_reduce(p2.reds.p, p2.nreds, p2.f32, st, gate);
    if (f32) launch_cvt_f2d(step.out.p, (const float*)step.out32.p, step.n, st);
    add_projectors(step.in.p, step.out.p);
  }
  // the parts of sigma_vec around the two GEMM passes, for a launch shared
  // with other engines (same operations in the same order)
  void sigma_in(const double* x, bool f32) {
    if (step.p2_pending) fail(-1, "internal: sigma plan incomplete");
    if (f32) ensure_f32();
    dev_d2d(step.in.p, x, (size_t)step.n * 8, st);
    if (f32) {
      launch_cvt_d2f((float*)step.in32.p, step.in.p, step.n, st);
      dev_zero(step.out32.p, step.out32.n * 8, st);
    } else {
      dev_zero(step.out.p, (size_t)std::max<int64_t>(step.n, 1) * 8, st);
    }
  }
  void sigma_out(double* y, bool f32) {
    if (f32) launch_cvt_f2d(step.out.p, (const float*)step.out32.p, step.n, st);
    add_projectors(step.in.p, step.out.p);
    dev_d2d(y, step.out.p, (size_t)step.n * 8, st);
  }
  // Pick the sigma plans' workgroups per CU by timing the prepared step:
  // every candidate pair (first pass: one tile per workgroup or 8 ranges per
  // CU; accumulating pass: 12..64 ranges per CU) is planned and its FP64 sigma
  // timed over `reps` calls; the fastest pair is kept for this context and
  // the step is re-planned with it.  out[2 * c], out[2 * c + 1]: the pair's
  // gpc values, out[2 * ncand + c]: its mean ms per sigma.
  static constexpr int TUNE_G1[2] = {0, 8};
  static constexpr int TUNE_G2[6] = {12, 16, 24, 32, 48, 64};
  static constexpr int TUNE_N = 12;
  void autotune(int reps, double* out) {
    if (step.i < 0 || !step.X || !step.Y) fail(-1, "no prepared step");
    if (reps < 1) fail(-1, "reps must be positive");
    const int ns = (int)step.psi.sec.size();
    std::vector<OutBlk> outs(ns);
    for (int m = 0; m < ns; ++m) outs[m] = {step.out.p + step.off[m], step.dx[m], step.dy[m], step.dy[m]};
    launch_fill_uniform(step.in.p, step.n, 99, 0x5455, st);  // timing input
    const double ts = t_sigma, fs = f_sigma, tp1 = t_pass1, tp2 = t_pass2, fp1 = f_pass1, fp2 = f_pass2,
                 bp1 = b_pass1, bp2 = b_pass2, bs = b_sigma;
    const int64_t nsg = n_sigma, np1 = n_pass1, np2 = n_pass2;
    int best = -1;
    double best_ms = INFINITY;
    for (int c = 0; c < TUNE_N; ++c) {
      const int g1 = TUNE_G1[c / 6], g2 = TUNE_G2[c % 6];
      TwoPass tp;
      build_two_pass(outs, step.trs, tp, st, true, nullptr, g1, g2, xcd1, xcd2, corder);
      std::swap(tp, step.plan);
      sigma_fixed(false);  // warm-up
      const double t0 = t_sigma;
      for (int r = 0; r < reps; ++r) sigma_fixed(false);
      const double ms = 1e3 * (t_sigma - t0) / reps;
      std::swap(tp, step.plan);
      if (out) {
        out[2 * c] = g1;
        out[2 * c + 1] = g2;
        out[2 * TUNE_N + c] = ms;
      }
      if (ms < best_ms) best_ms = ms, best = c;
    }
    // the timing calls do not count in the statistics
    t_sigma = ts, f_sigma = fs, t_pass1 = tp1, t_pass2 = tp2, f_pass1 = fp1, f_pass2 = fp2;
    b_pass1 = bp1, b_pass2 = bp2, b_sigma = bs, n_sigma = nsg, n_pass1 = np1, n_pass2 = np2;
    gpc1 = TUNE_G1[best / 6];
    gpc2 = TUNE_G2[best % 6];
    TwoPass tp;
    build_two_pass(outs, step.trs, tp, st, true, nullptr, gpc1, gpc2, xcd1, xcd2, corder);
    std::swap(tp, step.plan);
    step.flops = step.plan.flops;
    step.f32_ready = false;
    dev_sync(st);
  }

  // relative rounding of the reduced-precision sigma products: FP32 (2^-24),
  // BF16x3 (the dropped lo*lo term and the split remainder, about 2^-16)
  double reduced_eps() const { return prec == 2 ? 1.5e-5 : 6e-8; }
  // plan the accumulating pass left open by prepare() (target: cost per
  // workgroup range; 0 = this problem alone)
  void plan_pass2(double target) {
    if (!step.p2_pending) return;
    const int tag = step.plan.p2.tag;
    step.g2.plan(step.plan.p2, st, gpc2, target);
    step.plan.p2.tag = tag;
    step.g2 = GemmList();
    step.p2_pending = false;
  }

  // ---- Davidson (Davidson 1975; section "The effective Hamiltonian equation")
  // tol: residual-norm tolerance; f32: sigma with FP32 operands.
  double davidson(double* xres, int* iters, bool* conv, double tol, bool f32) {
    if (!stage) stage = std::make_unique<Staging>(st, pool);
    stage->st = st;
    std::vector<Engine*> E{this};
    std::vector<DavState> D(1);
    D[0].xres = xres;
    D[0].tol = tol;
    D[0].f32 = f32;
    D[0].eps = reduced_eps();
    davidson_lockstep(E, D, nullptr, *stage);
    *iters = D[0].it;
    *conv = D[0].conv;
    return D[0].theta;
  }

  // Work buffers of one solve.  Small-matrix layout in dsmall: eigenvalues,
  // eigenvectors (64 x 64), coefficients, norms.
  double* dav_evals() { return dsmall.p; }
  double* dav_evecs() { return dsmall.p + 64; }
  double* dav_coef() { return dsmall.p + 64 + 64 * 64; }
  double* dav_nrm() { return dav_coef() + 64; }
  double* dav_nrm2() { return dav_coef() + 65; }
  void dav_alloc(DavState& d) {
    const int64_t n = step.n;
    d.ms = std::max(2, std::min(dav_max_sub, 64));
    d.k = 0;
    d.it = 1;
    d.theta = 0.0;
    d.rbest = INFINITY;
    d.stall = 0;
    d.conv = d.done = false;
    dV.ensure((size_t)d.ms * n);
    dW.ensure((size_t)d.ms * n);
    dHs.ensure((size_t)d.ms * d.ms);
    dsmall.ensure(8 * 64 + 64 * 64);
    dpartial.ensure(256 * 64);
    dx_.ensure(n);
    dax.ensure(n);
    dr.ensure(n);
    dt.ensure(n);
  }
  // vector whose sigma is due, and where it goes
  double* dav_x(const DavState& d) { return dV.p + (int64_t)d.k * step.n; }
  double* dav_y(const DavState& d) { return dW.p + (int64_t)d.k * step.n; }
  // a zero guess becomes the constant vector (rare; synchronous)
  void dav_zero_guess() {
    const int64_t n = step.n;
    std::vector<double> one(n, 1.0);
    dev_h2d(dV.p, one.data(), (size_t)n * 8, st);
    launch_dots(dV.p, n, 1, dV.p, n, dav_nrm(), dpartial.p, st);
  }
  // the preconditioned residual collapsed: orthogonalise the residual itself;
  // false if that vanishes too (rare; synchronous)
  bool dav_residual_direction(DavState& d) {
    const int64_t n = step.n;
    dev_d2d(dt.p, dr.p, (size_t)n * 8, st);
    for (int pass = 0; pass < 2; ++pass) {
      launch_dots(dV.p, n, d.k, dt.p, n, dav_coef(), dpartial.p, st);
      launch_combo_vec(dV.p, n, d.k, dav_coef(), -1.0, n, dt.p, 1.0, st);
    }
    launch_dots(dt.p, n, 1, dt.p, n, dav_nrm2(), dpartial.p, st);
    double tn;
    dev_d2h(&tn, dav_nrm2(), 8, st);
    return tn > 1e-28;
  }
  // subspace full: restart from the current Ritz vector, then the new
  // direction (already normalised) is orthogonalised against it
  void dav_restart(DavState& d) {
    const int64_t n = step.n;
    dev_d2d(dV.p, dx_.p, (size_t)n * 8, st);
    dev_d2d(dW.p, dax.p, (size_t)n * 8, st);
    launch_dots(dV.p, n, 1, dV.p, n, dav_nrm(), dpartial.p, st);
    // x is unit (orthonormal basis, unit Ritz coefficients); W follows x
    launch_dots(dV.p, n, 1, dW.p, n, dHs.p, dpartial.p, st);
    d.k = 1;
    launch_dots(dV.p, n, 1, dt.p, n, dav_coef(), dpartial.p, st);
    launch_combo_vec(dV.p, n, 1, dav_coef(), -1.0, n, dt.p, 1.0, st);
    launch_dots(dt.p, n, 1, dt.p, n, dav_nrm2(), dpartial.p, st);
    launch_normalize(dt.p, dav_nrm2(), n, st);
  }

  // ---- SVD and truncation (section "The reduced two-site object"): SVD per
  // (j_M, N_M, I_M) sector, keep the D largest kappa = s / sqrt(2 j_M + 1).
  struct Split {
    Basis kept;
    std::vector<int> ms;  // psi sector index of each kept sector
    DBuf ubuf, sbuf, vbuf;
    std::vector<int64_t> uo, so, vo;
    std::vector<int> r;
    double wd = 0.0;
  };

  void svd_truncate(const double* psi, int D, Split& sp) {
    const int ns = (int)step.psi.sec.size();
    sp.uo.resize(ns);
    sp.so.resize(ns);
    sp.vo.resize(ns);
    sp.r.resize(ns);
    int64_t nu = 0, nsv = 0, nv = 0, nw = 0;
    int maxs = 1;
    for (int m = 0; m < ns; ++m) {
      const int r = std::min(step.dx[m], step.dy[m]);
      sp.r[m] = r;
      sp.uo[m] = nu;
      nu += (int64_t)step.dx[m] * r;
      sp.so[m] = nsv;
      nsv += r;
      sp.vo[m] = nv;
      nv += (int64_t)r * step.dy[m];
      nw += (int64_t)step.dx[m] * step.dy[m] + (int64_t)r * r + r;
      maxs = std::max(maxs, r);
    }
    sp.ubuf.alloc((size_t)std::max<int64_t>(nu, 1));
    sp.sbuf.alloc((size_t)std::max<int64_t>(nsv, 1));
    sp.vbuf.alloc((size_t)std::max<int64_t>(nv, 1));
    DBuf work;
    work.alloc((size_t)std::max<int64_t>(nw, 1));
    std::vector<SvdJob> jobs;
    int64_t wo = 0;
    for (int m = 0; m < ns; ++m) {
      jobs.push_back({psi + step.off[m], step.dx[m], step.dy[m], step.dy[m], sp.ubuf.p + sp.uo[m],
                      sp.sbuf.p + sp.so[m], sp.vbuf.p + sp.vo[m], work.p + wo});
      wo += (int64_t)step.dx[m] * step.dy[m] + (int64_t)sp.r[m] * sp.r[m] + sp.r[m];
    }
    DArr<SvdJob> dj;
    dj.put(jobs, st);
    // matrices with 64 or more singular values are orthogonalised by block
    // rounds (a workgroup per pair of column blocks, sweeps repeated until
    // converged), the others in one workgroup each
    std::vector<SvdJob> small, big;
    std::vector<int> pbase{0};
    int maxs_small = 1, maxs_big = 1, rounds = 0;
    for (const SvdJob& jb : jobs) {
      const int r = std::min(jb.rows, jb.cols);
      if (r >= 64 && svd_block_fits(jb.rows, jb.cols)) {
        big.push_back(jb);
        pbase.push_back(pbase.back() + svd_block_pairs(jb.rows, jb.cols));
        rounds = std::max(rounds, svd_block_rounds(jb.rows, jb.cols));
        maxs_big = std::max(maxs_big, r);
      } else {
        small.push_back(jb);
        maxs_small = std::max(maxs_small, r);
      }
    }
    (void)maxs;
    DArr<SvdJob> dsmall, dbig;
    DArr<int> dpb, dfl;
    if (!small.empty()) {
      dsmall.put(small, st);
      launch_svd(dsmall.p, (int)small.size(), maxs_small, st, 0);
    }
    if (!big.empty()) {
      const int nb = (int)big.size();
      dbig.put(big, st);
      dpb.put(pbase, st);
      // two flag arrays: the sweep's and the previous one's (a job whose
      // previous sweep rotated nothing significant is skipped)
      std::vector<int> fl(2 * nb, 1);
      dfl.put(fl, st);
      launch_svd(dbig.p, nb, maxs_big, st, 1);
      for (int sweep = 0; sweep < 60; ++sweep) {
        const int* act = dfl.p + nb * (sweep % 2);
        int* cur = dfl.p + nb * ((sweep + 1) % 2);
        dev_zero(cur, sizeof(int) * nb, st);
        for (int r = 0; r < rounds; ++r) launch_svd_block(dbig.p, dpb.p, nb, pbase.back(), r, act, cur, st);
        dev_d2h(fl.data(), cur, sizeof(int) * nb, st);
        if (std::none_of(fl.begin(), fl.begin() + nb, [](int f) { return f != 0; })) break;
      }
      launch_svd(dbig.p, nb, maxs_big, st, 2);
    }
    launch_svd_signs(dj.p, (int)jobs.size(), st);
    std::vector<double> s(nsv);
    dev_d2h(s.data(), sp.sbuf.p, (size_t)nsv * 8, st);
    struct Cand {
      double kappa;
      int m, a;
    };
    std::vector<Cand> cand;
    double norm2 = 0.0;
    for (int m = 0; m < ns; ++m)
      for (int a = 0; a < sp.r[m]; ++a) {
        const double v = s[sp.so[m] + a];
        cand.push_back({v / std::sqrt(step.psi.sec[m].tj + 1.0), m, a});
        norm2 += v * v;
      }
    std::stable_sort(cand.begin(), cand.end(), [](const Cand& x, const Cand& y) {
      if (x.kappa != y.kappa) return x.kappa > y.kappa;
      if (x.m != y.m) return x.m < y.m;
      return x.a < y.a;
    });
    std::vector<int> kept(ns, 0);
    double disc = 0.0;
    for (size_t c = 0; c < cand.size(); ++c) {
      if ((int)c < D)
        kept[cand[c].m]++;
      else
        disc += s[sp.so[cand[c].m] + cand[c].a] * s[sp.so[cand[c].m] + cand[c].a];
    }
    sp.wd = disc / std::max(norm2, 1e-300);
    sp.kept = Basis();
    sp.ms.clear();
    for (int m = 0; m < ns; ++m)
      if (kept[m] > 0) {
        sp.kept.sec.push_back(step.psi.sec[m]);
        sp.kept.dim.push_back(kept[m]);
        sp.ms.push_back(m);
      }
  }

  // copy the leading (rows x cols) part of row-major matrices (ld) into a
  // compact tensor, optionally scaling rows/cols by singular values
  void compact(Tensor& t, const std::vector<const double*>& src, const std::vector<int>& ld) {
    std::vector<GatherDst> dsts;
    std::vector<GatherSrc> srcs;
    for (size_t j = 0; j < src.size(); ++j) {
      srcs.push_back({src[j], ld[j], GS_NORMAL, 1.0});
      dsts.push_back({t.at((int)j), t.rows[j], t.cols[j], t.cols[j], (int)j, (int)j + 1});
    }
    DArr<GatherDst> dd;
    DArr<GatherSrc> ds;
    dd.put(dsts, st);
    ds.put(srcs, st);
    launch_gather(dd.p, (int)dsts.size(), ds.p, st);
    dev_sync(st);
  }

  void alloc_tensor(Tensor& t) {
    int64_t o = 0;
    t.off.clear();
    for (size_t j = 0; j < t.rows.size(); ++j) {
      t.off.push_back(o);
      o += (int64_t)t.rows[j] * t.cols[j];
    }
    t.data.alloc((size_t)std::max<int64_t>(o, 1));
  }

  // ---- one micro-iteration
  // <x|H|x> / <x|x> with the FP64 sigma
  // FP64 refinement of an FP32 Davidson solution x (unit; the solve's last
  // Ritz value still in dav_evals()): Davidson steps in FP64 on the subspace
  // {x, t}, t the preconditioned FP64 residual made orthonormal to x.  The
  // phases of a step: after y = H x is in dr, refine_dir forms t in dt; after
  // w = H t is in dax, refine_dots enqueues the inner products (read back
  // into hpin[0..4]); refine_update solves the 2 x 2 problem on the host,
  // replaces x by the lowest Ritz vector and returns its FP64 Rayleigh
  // quotient.  With `more`, it also leaves H x of the new vector in dr (as
  // the same combination of y and w) and its Rayleigh quotient in
  // dav_evals(), ready for the next step: one more FP64 sigma per step.
  void refine_dir(const double* x) {
    const int64_t n = step.n;
    launch_residual(dr.p, x, dav_evals(), n, dt.p, st);
    if (refine_tol > 0.0) launch_dots(dt.p, n, 1, dt.p, n, dav_nrm(), dpartial.p, st);  // |r|^2 of x
    launch_precond(dt.p, step.diag.p, dav_evals(), n, dt.p, st);
    for (int pass = 0; pass < 2; ++pass) {
      launch_dots(x, n, 1, dt.p, n, dav_coef(), dpartial.p, st);
      launch_combo_vec(x, n, 1, dav_coef(), -1.0, n, dt.p, 1.0, st);
    }
    launch_dots(dt.p, n, 1, dt.p, n, dav_nrm2(), dpartial.p, st);
    launch_normalize(dt.p, dav_nrm2(), n, st);
  }
  void refine_dots(const double* x) {
    const int64_t n = step.n;
    double* c = dav_coef();
    launch_dots(x, n, 1, dr.p, n, c + 1, dpartial.p, st);   // x.Hx
    launch_dots(x, n, 1, x, n, c + 2, dpartial.p, st);      // x.x
    launch_dots(x, n, 1, dax.p, n, c + 3, dpartial.p, st);  // x.Ht
    launch_dots(dt.p, n, 1, dax.p, n, c + 4, dpartial.p, st);  // t.Ht
    if (!hpin) hpin = (double*)host_alloc_pinned(8 * sizeof(double));
    dev_d2h_async(hpin, dav_nrm2(), 8, st);  // |t|^2 before normalisation
    dev_d2h_async(hpin + 1, c + 1, 32, st);
  }
  double refine_update(double* x, bool more = false, bool* moved = nullptr) {
    const int64_t n = step.n;
    const double tt = hpin[0], xy = hpin[1], xx = hpin[2], xw = hpin[3], tw = hpin[4];
    const double a = xy / xx;
    if (moved) *moved = false;
    if (!(tt > 1e-28) || !(xx > 0) || !std::isfinite(xw) || !std::isfinite(tw)) return a;
    const double sx = std::sqrt(xx);
    const double b = xw / sx, c = tw;
    const double lam = 0.5 * (a + c) - std::sqrt(0.25 * (a - c) * (a - c) + b * b);
    double p = b, q = lam - a;  // (H - lam) v = 0, two equivalent rows
    const double p2 = lam - c, q2 = b;
    if (p2 * p2 + q2 * q2 > p * p + q * q) p = p2, q = q2;
    const double nv = std::sqrt(p * p + q * q);
    if (!(nv > 0) || !std::isfinite(lam) || lam > a) return a;
    p /= nv;
    q /= nv;
    if (p < 0) p = -p, q = -q;  // keep the sign of x
    launch_scal(x, p / sx, n, st);
    launch_axpy(x, dt.p, q, n, st);
    if (more) {
      launch_scal(dr.p, p / sx, n, st);
      launch_axpy(dr.p, dax.p, q, n, st);
      hpin[6] = lam;  // read by the copy before the next step's host update
      dev_h2d_async(dav_evals(), hpin + 6, sizeof(double), st);
    }
    if (moved) *moved = true;
    return lam;
  }
  // the residual norm of the vector refine_dir last worked on (synchronises)
  double refine_residual() {
    double r2 = 0.0;
    dev_d2h(&r2, dav_nrm(), 8, st);
    return std::sqrt(std::max(0.0, r2));
  }
  double refine64(double* x) {
    sigma_vec(x, dr.p, false);
    double th = NAN;
    for (int k = 0; k < refine_steps; ++k) {
      refine_dir(x);
      if (refine_tol > 0.0 && k > 0 && refine_residual() <= refine_tol) break;
      sigma_vec(dt.p, dax.p, false);
      refine_dots(x);
      dev_sync(st);
      bool moved = false;
      th = refine_update(x, k + 1 < refine_steps, &moved);
      if (!moved) break;
    }
    return th;
  }
  double micro(int i, int D, bool right, bool do_svd) {
    auto t0 = std::chrono::steady_clock::now();
    prepare(i);
    DBuf x;
    x.alloc((size_t)std::max<int64_t>(step.n, 1));
    int its = 0;
    bool conv = false;
    double th;
    if (prec >= 1) {
      // FP32 (or BF16x3) sigma until the residual reaches mixed_tol, then one FP64
      // Davidson step from that vector (two FP64 sigma): the reported energy
      // is the FP64 Ritz value of the refined vector
      th = davidson(x.p, &its, &conv, std::max(dav_tol, mixed_tol), true);
      th = refine64(x.p);
    } else {
      th = davidson(x.p, &its, &conv, dav_tol, false);
    }
    const double e = micro_finish(i, D, right, do_svd, x.p, th, conv);
    t_micro += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return e;
  }

  // everything after the centre solve: energy bookkeeping, noise, SVD and
  // truncation, the new site tensor, renormalisation, the centre move
  double micro_finish(int i, int D, bool right, bool do_svd, double* x, double th, bool conv) {
    if (!conv) warned = true;
    const double e = th + P.e_const;
    emin = std::min(emin, e);
    elast = e;
    trace.push_back(e);
    const int ns = (int)step.psi.sec.size();
    if (!do_svd) {  // keep the optimised object as the guess of the next step
      Tensor t;
      t.rowsec = step.psi;
      for (int m = 0; m < ns; ++m) {
        t.rows.push_back(step.dx[m]);
        t.cols.push_back(step.dy[m]);
      }
      alloc_tensor(t);
      dev_d2d(t.data.p, x, (size_t)step.n * 8, st);
      cen.kind = C_TWO;
      cen.pos = i;
      cen.t = std::move(t);
      return e;
    }
    if (noise > 0.0 && wd_prev > 0.0) {
      // the eigenvector's arbitrary sign is fixed first (<x, u> >= 0) so that
      // the noisy object does not depend on it
      DBuf u;
      u.alloc((size_t)std::max<int64_t>(step.n, 1));
      launch_fill_uniform(u.p, step.n, seed, NOISE_STREAM | ((uint64_t)n_pass << 16) | (uint64_t)i, st);
      dsmall.ensure(8 * 64 + 64 * 64);
      dpartial.ensure(256 * 64);
      launch_dots(x, step.n, 1, u.p, step.n, dsmall.p, dpartial.p, st);
      double xu;
      dev_d2h(&xu, dsmall.p, 8, st);
      if (xu < 0.0) launch_axpy(x, x, -2.0, step.n, st);
      launch_axpy(x, u.p, 0.5 * noise * wd_prev, step.n, st);
      dev_sync(st);
    }
    Split sp;
    {
      PhaseTimer pt(t_phase[PH_SVD]);
      svd_truncate(x, D, sp);
    }
    PhaseTimer pt(t_phase[PH_RENORM]);
    wdisc_sweep = std::max(wdisc_sweep, sp.wd);
    wd_pass = std::max(wd_pass, sp.wd);
    const int c = i + 1;
    const int nk = (int)sp.kept.sec.size();
    if (right) {
      Tensor u;  // U[i]: (dimX(m) x k_m)
      u.rowsec = sp.kept;
      std::vector<const double*> src;
      std::vector<int> ld;
      for (int j = 0; j < nk; ++j) {
        const int m = sp.ms[j];
        u.rows.push_back(step.dx[m]);
        u.cols.push_back(sp.kept.dim[j]);
        src.push_back(sp.ubuf.p + sp.uo[m]);
        ld.push_back(sp.r[m]);
      }
      alloc_tensor(u);
      compact(u, src, ld);
      Tensor cc;  // centre on bond c: s Vt  (k_m x dimY(m))
      cc.rowsec = sp.kept;
      src.clear();
      ld.clear();
      for (int j = 0; j < nk; ++j) {
        const int m = sp.ms[j];
        cc.rows.push_back(sp.kept.dim[j]);
        cc.cols.push_back(step.dy[m]);
        src.push_back(sp.vbuf.p + sp.vo[m]);
        ld.push_back(step.dy[m]);
      }
      alloc_tensor(cc);
      compact(cc, src, ld);
      for (int j = 0; j < nk; ++j)
        launch_scale_rows(cc.at(j), cc.rows[j], cc.cols[j], cc.cols[j], sp.sbuf.p + sp.so[sp.ms[j]], st);
      dims[c] = sp.kept;
      U[i] = std::move(u);
      Lb[c] = renormalize(*step.X, U[i], dims[c], true, step.f32_ready ? (const float*)step.x32.p : nullptr,
                          renorm_prec);
      note_block_bytes();
      for (Lower& w : lower) lower_m(w, i);
      cen.kind = C_BOND_R;
      cen.pos = c;
      cen.t = std::move(cc);
    } else {
      Tensor v;  // V[i+1]: (k_m x dimY(m))
      v.rowsec = sp.kept;
      std::vector<const double*> src;
      std::vector<int> ld;
      for (int j = 0; j < nk; ++j) {
        const int m = sp.ms[j];
        v.rows.push_back(sp.kept.dim[j]);
        v.cols.push_back(step.dy[m]);
        src.push_back(sp.vbuf.p + sp.vo[m]);
        ld.push_back(step.dy[m]);
      }
      alloc_tensor(v);
      compact(v, src, ld);
      Tensor cc;  // centre: U s (dimX(m) x k_m)
      cc.rowsec = sp.kept;
      src.clear();
      ld.clear();
      for (int j = 0; j < nk; ++j) {
        const int m = sp.ms[j];
        cc.rows.push_back(step.dx[m]);
        cc.cols.push_back(sp.kept.dim[j]);
        src.push_back(sp.ubuf.p + sp.uo[m]);
        ld.push_back(sp.r[m]);
      }
      alloc_tensor(cc);
      compact(cc, src, ld);
      for (int j = 0; j < nk; ++j)
        launch_scale_cols(cc.at(j), cc.rows[j], cc.cols[j], cc.cols[j], sp.sbuf.p + sp.so[sp.ms[j]], st);
      dims[c] = sp.kept;
      V[i + 1] = std::move(v);
      Rb[c] = renormalize(*step.Y, V[i + 1], dims[c], false, step.f32_ready ? (const float*)step.y32.p : nullptr,
                          renorm_prec);
      note_block_bytes();
      for (Lower& w : lower) lower_or(w, c);
      cen.kind = C_BOND_L;
      cen.pos = c;
      cen.t = std::move(cc);
    }
    dev_sync(st);
    step.i = -1;  // blocks changed
    return e;
  }

  // left-to-right micro-iterations from the current centre (test / benchmark hook)
  double advance(int D, int n) {
    if (!mps_ready) fail(-1, "no MPS");
    if (!((cen.kind == C_T0 && cen.pos == 0) || (cen.kind == C_TWO) || cen.kind == C_BOND_R))
      fail(-1, "advance needs a centre reached by a left-to-right move");
    int i = cen.pos;
    double e = INFINITY;
    for (int s = 0; s < n && i <= P.L - 3; ++s, ++i) e = std::min(e, micro(i, D, true, true));
    return e;
  }

  void end_pass() {
    wd_prev = wd_pass;
    wd_pass = 0.0;
    ++n_pass;
  }

  double sweep(int D) {
    if (!mps_ready) fail(-1, "call sadmrg_init_mps or sadmrg_mps_import first");
    const int L = P.L;
    double e = INFINITY;
    wdisc_sweep = 0.0;
    // a left-to-right pass needs the centre at step 0
    if (!((cen.kind == C_T0 && cen.pos == 0) || (cen.kind == C_TWO && cen.pos == 0)))
      fail(-1, "internal: sweep must start with the centre at the left end");
    for (int i = 0; i <= L - 2; ++i) e = std::min(e, micro(i, D, true, i < L - 2));
    end_pass();
    for (int i = L - 2; i >= 0; --i) e = std::min(e, micro(i, D, false, i > 0));
    end_pass();
    wdisc = wdisc_sweep;
    return e;
  }
};

// ---------------------------------------------------------------------------
// Independent problems in lockstep.  The paper computes each state of its
// carbon-dimer study (section "Bond dissociation curves") as a separate
// calculation in its own symmetry sector, and parallelises within one
// calculation over the sparse blocks (section "DMRG" of the library
// description).  Small calculations cannot fill the GPU alone, so several
// engines that share one stream advance step by step together: their sigma
// products go out as one launch per GEMM pass, with the accumulating pass
// balanced over the whole batch, and the host waits for the stream once per
// Davidson phase for all of them.
// ---------------------------------------------------------------------------
struct BatchLaunch {
  Stream st = nullptr;
  Staging stage;             // job arrays and descriptors of the shared launches
  std::vector<Stream> priv;  // one stream per engine for its own phases
  // timing: event pairs around the shared launches, read at the end
  std::vector<std::pair<void*, void*>> ev64, ev32;
  double f64 = 0.0, f32 = 0.0;  // algorithmic flops of the shared launches
  int64_t n64 = 0, n32 = 0;     // shared launches (one per pass pair)
  // host wall time of the phases of the batched micro-iterations: step
  // preparation, Davidson, FP64 refinement (mixed precision), decomposition
  // and update
  double w_prepare = 0.0, w_davidson = 0.0, w_rayleigh = 0.0, w_finish = 0.0;

  BatchLaunch(Stream s, DevPool* p, size_t n) : st(s), stage(s, p) {
    for (size_t k = 0; k < n; ++k) priv.push_back(dev_stream_create());
  }
  BatchLaunch(const BatchLaunch&) = delete;
  BatchLaunch& operator=(const BatchLaunch&) = delete;
  ~BatchLaunch() {
    try {
      dev_sync(st);
    } catch (...) {
    }
    for (Stream s : priv) dev_stream_destroy(s);
    for (auto& e : ev64) dev_event_free(e.first), dev_event_free(e.second);
    for (auto& e : ev32) dev_event_free(e.first), dev_event_free(e.second);
  }
  // seconds in the shared launches (synchronises)
  void times(double& t64, double& t32) {
    t64 = t32 = 0.0;
    for (auto& e : ev64) t64 += dev_event_elapsed(e.first, e.second);
    for (auto& e : ev32) t32 += dev_event_elapsed(e.first, e.second);
  }

  // The GEMM passes of the sigma of every engine, shared: each engine's
  // step.in (FP64 or its FP32 mirror) must be in place and its output zeroed.
  void gemm_passes(const std::vector<Engine*>& E, bool use32) {
    std::vector<GSeg> s1, s2, sr;
    std::vector<int> b1, b2, br;
    int nw1 = 0, nw2 = 0, nr = 0;
    bool stream2 = true;
    double fl = 0.0;
    for (Engine* e : E) {
      const Step& S = e->step;
      const GemmList::Plan& p1 = use32 ? S.q1 : S.plan.p1;
      const GemmList::Plan& p2 = use32 ? S.q2 : S.plan.p2;
      if (p1.stream || p1.nreds != 0) fail(-1, "internal: first pass must be one tile per workgroup");
      stream2 = p2.stream;
      if (p1.nwg > 0) {
        s1.push_back({p1.tiles.p, p1.tasks.p, nullptr, nullptr});
        b1.push_back(nw1);
        nw1 += p1.nwg;
      }
      if (p2.nwg > 0) {
        s2.push_back({p2.tiles.p, p2.tasks.p, p2.wstart.p, nullptr});
        b2.push_back(nw2);
        nw2 += p2.nwg;
      }
      if (p2.nreds > 0) {
        sr.push_back({nullptr, nullptr, nullptr, p2.reds.p});
        br.push_back(nr);
        nr += p2.nreds;
      }
      fl += S.flops;
    }
    const GSeg* d1 = stage.up(s1);
    const GSeg* d2 = stage.up(s2);
    const GSeg* dr = stage.up(sr);
    const int* e1 = stage.up(b1);
    const int* e2 = stage.up(b2);
    const int* er = stage.up(br);
    Event t0(st);
    const bool bf3 = use32 && !E.empty() && E[0]->prec == 2;
    launch_gemm_seg(d1, e1, (int)s1.size(), nw1, false, use32, st, bf3);
    launch_gemm_seg(d2, e2, (int)s2.size(), nw2, stream2, use32, st, bf3);
    launch_reduce_seg(dr, er, (int)sr.size(), nr, use32, st);
    Event t1(st);
    (use32 ? ev32 : ev64).push_back({t0.p, t1.p});
    t0.release();
    t1.release();
    (use32 ? f32 : f64) += fl;
    ++(use32 ? n32 : n64);
  }

  // y_e = H_eff(e) x_e for every engine e (the single-engine operations
  // around the GEMM passes as job lists)
  void sigma(const std::vector<Engine*>& E, const std::vector<const double*>& x, const std::vector<double*>& y,
             bool use32);

  // The shared sigma of step.in into step.out of every engine as launches
  // with no host work, for a recorded sequence: descriptors and job lists
  // are uploaded once (prepare), then launched (record) as often as needed;
  // gates[e]: engine e's GEMM workgroups do nothing while *gates[e] != 0.
  // The arrays live in the staging area sg (valid until its next reset).
  struct Rec {
    const GSeg *s1 = nullptr, *s2 = nullptr, *sr = nullptr;
    const int *b1 = nullptr, *b2 = nullptr, *br = nullptr;
    const EwJob *pre = nullptr, *post = nullptr;
    int ns1 = 0, ns2 = 0, nsr = 0, npre = 0, npost = 0;
    int nw1 = 0, nw2 = 0, nr = 0;
    bool stream2 = true, use32 = false, bf3 = false;
    int64_t maxn = 0;
  };
  void record_prepare(Rec& r, const std::vector<Engine*>& E, bool use32, const std::vector<const int*>& gates,
                      Staging& sg);
  void record(const Rec& r) const {
    launch_ew_batch(r.pre, r.npre, r.maxn, st);
    launch_gemm_seg(r.s1, r.b1, r.ns1, r.nw1, false, r.use32, st, r.bf3);
    launch_gemm_seg(r.s2, r.b2, r.ns2, r.nw2, r.stream2, r.use32, st, r.bf3);
    launch_reduce_seg(r.sr, r.br, r.nsr, r.nr, r.use32, st);
    launch_ew_batch(r.post, r.npost, r.maxn, st);
  }
};

// host threads for the per-engine parts of a batched micro-iteration
// (preparation, decomposition and update); the engines touch disjoint
// memory and keep their own stream order
static const int BATCH_HOST_THREADS = 16;

// For one per-engine phase the engine works on a stream of its own, so that
// its waits do not include the other engines' work: the private stream
// first follows the shared one, and the shared one follows the private
// stream at the end; the engine's work thus stays in one total order.
struct OwnStream {
  Engine& e;
  Stream shared;
  OwnStream(Engine& en, Stream priv) : e(en), shared(en.st) {
    dev_stream_order(priv, shared);
    e.st = priv;
  }
  ~OwnStream() {
    try {
      dev_stream_order(shared, e.st);
    } catch (...) {
    }
    e.st = shared;
  }
};

// Job lists of one launch of the batched Davidson helpers
struct EwList {
  std::vector<EwJob> v;
  int64_t maxn = 0;
  void add(int kind, const double* a, const double* b, const double* sc, double* y, int64_t n) {
    v.push_back({a, b, sc, y, n, kind});
    maxn = std::max(maxn, n);
  }
  void run(Staging& sg, Stream st) {
    if (!v.empty()) launch_ew_batch(sg.up(v), (int)v.size(), maxn, st);
    v.clear();
    maxn = 0;
  }
};
struct DotList {
  std::vector<DotJob> v;
  int maxk = 0;
  void add(const double* V, int64_t ldv, int k, const double* x, int64_t n, double* out, double* part) {
    v.push_back({V, x, out, part, ldv, n, k});
    maxk = std::max(maxk, k);
  }
  void run(Staging& sg, Stream st) {
    if (!v.empty()) launch_dots_batch(sg.up(v), (int)v.size(), maxk, st);
    v.clear();
    maxk = 0;
  }
};
struct ComboList {
  std::vector<ComboJob> v;
  int64_t maxn = 0;
  void add(const double* V, int64_t ldv, int k, const double* coef, double alpha, int64_t n, double* y, double beta) {
    v.push_back({V, coef, y, ldv, n, k, alpha, beta});
    maxn = std::max(maxn, n);
  }
  void run(Staging& sg, Stream st) {
    if (!v.empty()) launch_combo_batch(sg.up(v), (int)v.size(), maxn, st);
    v.clear();
    maxn = 0;
  }
};

void BatchLaunch::sigma(const std::vector<Engine*>& E, const std::vector<const double*>& x,
                        const std::vector<double*>& y, bool use32) {
  EwList ew;
  for (size_t k = 0; k < E.size(); ++k) {
    Engine& e = *E[k];
    if (e.step.p2_pending) fail(-1, "internal: sigma plan incomplete");
    const int64_t n = e.step.n;
    if (use32) {
      {
        PoolBind b(e.pool);
        e.ensure_f32();
      }
      ew.add(EW_D2F, x[k], nullptr, nullptr, e.step.in32.p, n);
      ew.add(EW_ZERO, nullptr, nullptr, nullptr, e.step.out32.p, (int64_t)e.step.out32.n);
    } else {
      ew.add(EW_COPY, x[k], nullptr, nullptr, e.step.in.p, n);
      ew.add(EW_ZERO, nullptr, nullptr, nullptr, e.step.out.p, std::max<int64_t>(n, 1));
    }
  }
  ew.run(stage, st);
  gemm_passes(E, use32);
  for (size_t k = 0; k < E.size(); ++k) {
    Engine& e = *E[k];
    if (use32)
      ew.add(EW_F2D, e.step.out32.p, nullptr, nullptr, y[k], e.step.n);
    else
      ew.add(EW_COPY, e.step.out.p, nullptr, nullptr, y[k], e.step.n);
  }
  ew.run(stage, st);
}

void BatchLaunch::record_prepare(Rec& r, const std::vector<Engine*>& E, bool use32,
                                 const std::vector<const int*>& gates, Staging& sg) {
  std::vector<GSeg> s1, s2, sr;
  std::vector<int> b1, b2, br;
  std::vector<EwJob> pre, post;
  r = Rec();
  r.use32 = use32;
  r.bf3 = use32 && !E.empty() && E[0]->prec == 2;
  for (size_t k = 0; k < E.size(); ++k) {
    Engine& e = *E[k];
    {
      PoolBind b(e.pool);
      e.record_prepare(use32);
    }
    const Step& S = e.step;
    const GemmList::Plan& p1 = use32 ? S.q1 : S.plan.p1;
    const GemmList::Plan& p2 = use32 ? S.q2 : S.plan.p2;
    if (p1.stream || p1.nreds != 0) fail(-1, "internal: first pass must be one tile per workgroup");
    r.stream2 = p2.stream;
    if (p1.nwg > 0) {
      s1.push_back({p1.tiles.p, p1.tasks.p, nullptr, nullptr, gates[k]});
      b1.push_back(r.nw1);
      r.nw1 += p1.nwg;
    }
    if (p2.nwg > 0) {
      s2.push_back({p2.tiles.p, p2.tasks.p, p2.wstart.p, nullptr, gates[k]});
      b2.push_back(r.nw2);
      r.nw2 += p2.nwg;
    }
    if (p2.nreds > 0) {
      sr.push_back({nullptr, nullptr, nullptr, p2.reds.p, gates[k]});
      br.push_back(r.nr);
      r.nr += p2.nreds;
    }
    const int64_t n = S.n;
    r.maxn = std::max(r.maxn, std::max<int64_t>(n, (int64_t)S.out32.n));
    if (use32) {
      pre.push_back({S.in.p, nullptr, nullptr, S.in32.p, n, EW_D2F});
      pre.push_back({nullptr, nullptr, nullptr, S.out32.p, (int64_t)S.out32.n, EW_ZERO});
      post.push_back({S.out32.p, nullptr, nullptr, S.out.p, n, EW_F2D});
    } else {
      pre.push_back({nullptr, nullptr, nullptr, S.out.p, std::max<int64_t>(n, 1), EW_ZERO});
    }
  }
  r.s1 = sg.up(s1), r.ns1 = (int)s1.size();
  r.s2 = sg.up(s2), r.ns2 = (int)s2.size();
  r.sr = sg.up(sr), r.nsr = (int)sr.size();
  r.b1 = sg.up(b1);
  r.b2 = sg.up(b2);
  r.br = sg.up(br);
  r.pre = sg.up(pre), r.npre = (int)pre.size();
  r.post = sg.up(post), r.npost = (int)post.size();
}

// Davidson solves of engines that share one stream, in lockstep.  Every
// stage is one launch over all solves that take part in it (the helpers'
// job-list forms, each job with the arithmetic of the single-solve kernel),
// and the host waits for the stream twice per iteration, once for all
// solves.  With bl, the sigma products of an iteration share their GEMM
// launches; without it (one engine) each engine runs its own sigma.
static void davidson_lockstep(const std::vector<Engine*>& E, std::vector<DavState>& D, BatchLaunch* bl,
                              Staging& sg) {
  const size_t ne = E.size();
  if (ne == 0) return;
  const Stream st = E[0]->st;
  sg.st = st;
  sg.reset();
  EwList ew;
  DotList dots;
  ComboList cb;
  std::vector<SyevJob> sy;
  std::vector<const double*> sc;
  auto N = [&](size_t k) { return E[k]->step.n; };
  auto sync = [&]() {
    dev_sync(st);
    sg.reset();
  };
  // sigma of V_k into W_k, then row k of the projected matrix
  auto sigma_round = [&](const std::vector<size_t>& idx) {
    if (idx.empty()) return;
    if (!bl || idx.size() == 1) {
      for (size_t k : idx) {
        PoolBind b(E[k]->pool);
        E[k]->sigma_vec(E[k]->dav_x(D[k]), E[k]->dav_y(D[k]), D[k].f32);
      }
    } else {
      std::vector<Engine*> e;
      std::vector<const double*> x;
      std::vector<double*> y;
      const bool use32 = D[idx[0]].f32;
      for (size_t k : idx) {
        if (D[k].f32 != use32) fail(-1, "internal: one shared launch has one precision");
        e.push_back(E[k]);
        x.push_back(E[k]->dav_x(D[k]));
        y.push_back(E[k]->dav_y(D[k]));
      }
      bl->sigma(e, x, y, use32);
    }
    for (size_t k : idx) {
      Engine& g = *E[k];
      const int64_t n = N(k);
      dots.add(g.dV.p, n, D[k].k + 1, g.dW.p + (int64_t)D[k].k * n, n, g.dHs.p + (int64_t)D[k].k * D[k].ms,
               g.dpartial.p);
    }
    dots.run(sg, st);
    for (size_t k : idx) ++D[k].k;
  };
  // normalised Ritz vector into xres
  auto finish = [&](const std::vector<size_t>& idx) {
    if (idx.empty()) return;
    for (size_t k : idx) {
      Engine& g = *E[k];
      dots.add(g.dx_.p, N(k), 1, g.dx_.p, N(k), g.dav_nrm(), g.dpartial.p);
      ew.add(EW_COPY, g.dx_.p, nullptr, nullptr, D[k].xres, N(k));
    }
    dots.run(sg, st);
    ew.run(sg, st);
    for (size_t k : idx) {
      ew.add(EW_NORMALIZE, nullptr, nullptr, E[k]->dav_nrm(), D[k].xres, N(k));
      D[k].done = true;
    }
    ew.run(sg, st);
  };

  std::vector<size_t> all(ne);
  for (size_t k = 0; k < ne; ++k) {
    all[k] = k;
    PoolBind b(E[k]->pool);
    E[k]->dav_alloc(D[k]);
  }
  // V_0 = guess / |guess| (the guess is in step.in)
  for (size_t k : all) ew.add(EW_COPY, E[k]->step.in.p, nullptr, nullptr, E[k]->dV.p, N(k));
  ew.run(sg, st);
  for (size_t k : all) dots.add(E[k]->dV.p, N(k), 1, E[k]->dV.p, N(k), E[k]->dav_nrm(), E[k]->dpartial.p);
  dots.run(sg, st);
  sc.clear();
  for (size_t k : all) sc.push_back(E[k]->dav_nrm());
  sg.fetch(sc);
  sync();
  {
    std::vector<double> h0(sg.shost, sg.shost + ne);
    for (size_t k : all)
      if (!(h0[k] > 0)) {
        PoolBind b(E[k]->pool);
        E[k]->dav_zero_guess();
      }
  }
  for (size_t k : all) ew.add(EW_NORMALIZE, nullptr, nullptr, E[k]->dav_nrm(), E[k]->dV.p, N(k));
  ew.run(sg, st);
  sigma_round(all);
  std::vector<size_t> act, cont, fin, next;

  // Recorded iterations: one iteration of every solve (Ritz pair, residual,
  // convergence test, correction, restart, sigma, new row) is recorded once
  // as a fixed launch sequence that reads each solve's state from device
  // memory, and replayed dav_graph times between two host checks; the host
  // only finishes the solves that the replays marked done.  The arithmetic
  // is that of the host-driven loop below, step for step.
  bool graph = E[0]->dav_graph > 0;
  for (size_t k : all) graph = graph && N(k) > 1 && D[k].f32 == D[0].f32;
  if (graph) {
    const int seg = E[0]->dav_graph;
    const bool use32 = D[0].f32;
    PoolBind pb(sg.pool);
    std::vector<DGState> hs(ne);
    int msmax = 1;
    int64_t nmax = 1;
    for (size_t k : all) {
      hs[k] = DGState{D[k].k, D[k].it, 0, 0, 0, 0, 0, 0, INFINITY, 0.0};
      msmax = std::max(msmax, D[k].ms);
      nmax = std::max(nmax, N(k));
    }
    // the state and job arrays stay in the staging area until the final sync
    DGState* const dst = const_cast<DGState*>(sg.up(hs));
    std::vector<DGJob> hj(ne);
    std::vector<const int*> gates(ne);
    for (size_t k : all) {
      Engine& g = *E[k];
      gates[k] = &dst[k].done;
      hj[k] = DGJob{dst + k, g.dV.p, g.dW.p, g.dHs.p, g.dav_evals(), g.dav_evecs(), g.dav_coef(), g.dav_nrm(),
                    g.dav_nrm2(), g.dx_.p, g.dax.p, g.dr.p, g.dt.p, g.dpartial.p, g.step.diag.p, g.step.in.p,
                    g.step.out.p, N(k), D[k].ms, g.dav_max_iter, use32 ? 1 : 0, 0, D[k].tol, D[k].eps};
    }
    const DGJob* const J = sg.up(hj);
    const bool shared = bl && ne > 1;
    BatchLaunch::Rec rec;
    if (shared) {
      bl->record_prepare(rec, E, use32, gates, sg);
    } else {
      for (size_t k : all) {
        PoolBind b(E[k]->pool);
        E[k]->record_prepare(use32);
      }
    }
    const int nj = (int)ne;
    const int C = DG_GATE_COLLAPSE, R = DG_GATE_RESTART;
    // The legacy default stream cannot be recorded: the sequence is then
    // recorded on a stream of its own (recording runs nothing) and replayed
    // on the default stream.  The engines (and the shared launch) record on
    // that stream while the recording lasts.
    struct Capture {  // ends an interrupted recording, restores the streams, frees the graph
      Stream st, rs = nullptr;
      const std::vector<Engine*>& E;
      BatchLaunch* bl;
      bool open = false, swapped = false;
      void* ex = nullptr;
      Capture(Stream s, const std::vector<Engine*>& e, BatchLaunch* b) : st(s), E(e), bl(b) {}
      void begin() {
        rs = st;
        if (!st) {
          if (!E[0]->cap_stream) E[0]->cap_stream = dev_stream_create();
          rs = E[0]->cap_stream;
          for (Engine* e : E) e->st = rs;
          if (bl) bl->st = rs;
          swapped = true;
        }
        dev_capture_begin(rs);
        open = true;
      }
      void restore() {
        if (!swapped) return;
        for (Engine* e : E) e->st = st;
        if (bl) bl->st = st;
        swapped = false;
      }
      void end() {
        open = false;
        ex = dev_capture_end(rs);
        restore();
      }
      ~Capture() {
        if (open) dev_capture_abort(rs);
        restore();
        dev_graph_free(ex);
      }
    } cap(st, E, bl);
    const auto tr0 = std::chrono::steady_clock::now();
    cap.begin();
    {
      const Stream st = cap.rs;  // the recording stream, for the launches of this block
      launch_dg_scalar(J, nj, DG_TOP, st);
      launch_dg_syev(J, nj, st);
      launch_dg_combo(J, nj, DGC_RITZ_X, 0, nmax, st);
      launch_dg_combo(J, nj, DGC_RITZ_AX, 0, nmax, st);
      launch_dg_ew(J, nj, DGE_RESIDUAL, 0, nmax, st);
      launch_dg_dots(J, nj, DGD_RR, 0, 1, st);
      launch_dg_scalar(J, nj, DG_CHECK, st);
      launch_dg_ew(J, nj, DGE_PRECOND, 0, nmax, st);
      for (int pass = 0; pass < 2; ++pass) {
        launch_dg_dots(J, nj, DGD_VT, 0, msmax, st);
        launch_dg_combo(J, nj, DGC_ORTH, 0, nmax, st);
      }
      launch_dg_dots(J, nj, DGD_TT, 0, 1, st);
      launch_dg_scalar(J, nj, DG_COLLAPSE, st);
      launch_dg_ew(J, nj, DGE_COPY_RT, C, nmax, st);  // the residual itself instead
      for (int pass = 0; pass < 2; ++pass) {
        launch_dg_dots(J, nj, DGD_VT, C, msmax, st);
        launch_dg_combo(J, nj, DGC_ORTH, C, nmax, st);
      }
      launch_dg_dots(J, nj, DGD_TT, C, 1, st);
      launch_dg_scalar(J, nj, DG_COLLAPSE2, st);
      launch_dg_ew(J, nj, DGE_NORMALIZE_T, 0, nmax, st);
      launch_dg_scalar(J, nj, DG_RESTART_FLAG, st);
      launch_dg_ew(J, nj, DGE_RESTART_COPY, R, nmax, st);  // V_0 = x, W_0 = Ax
      launch_dg_dots(J, nj, DGD_V0W0, R, 1, st);
      launch_dg_dots(J, nj, DGD_V0T, R, 1, st);
      launch_dg_combo(J, nj, DGC_ORTH0, R, nmax, st);
      launch_dg_dots(J, nj, DGD_TT, R, 1, st);
      launch_dg_ew(J, nj, DGE_NORMALIZE_T, R, nmax, st);
      launch_dg_scalar(J, nj, DG_RESTART_K, st);
      launch_dg_ew(J, nj, DGE_APPEND, 0, nmax, st);
      launch_dg_ew(J, nj, DGE_LOAD, 0, nmax, st);
      if (shared)
        bl->record(rec);
      else
        for (size_t k : all) E[k]->sigma_record(use32, gates[k]);
      launch_dg_ew(J, nj, DGE_STORE, 0, nmax, st);
      launch_dg_dots(J, nj, DGD_ROW, 0, msmax, st);
      launch_dg_scalar(J, nj, DG_ADVANCE, st);
    }
    cap.end();
    void* const ex = cap.ex;
    const double trec = std::chrono::duration<double>(std::chrono::steady_clock::now() - tr0).count();
    for (size_t k : all) {
      ++E[k]->n_dgraph_record;
      E[k]->t_dgraph_rec += trec / (double)ne;
    }
    std::vector<DGState> prev = hs;
    while (true) {
      const Event e0(st);
      for (int r = 0; r < seg; ++r) dev_graph_launch(ex, st);
      const Event e1(st);
      sc.clear();
      for (size_t k : all) sc.push_back(E[k]->dav_evals());
      sg.fetch(sc);
      dev_d2h(hs.data(), dst, ne * sizeof(DGState), st);  // waits for the stream
      const double tseg = dev_event_elapsed(e0.p, e1.p);
      std::vector<double> th(sg.shost, sg.shost + ne);
      fin.clear();
      bool live = false;
      for (size_t k : all) {
        Engine& g = *E[k];
        const int nsig = hs[k].it - prev[k].it;
        g.t_dgraph += tseg / (double)ne;
        g.n_dgraph_replay += seg;
        g.n_dgraph_sigma += nsig;
        g.f_dgraph += nsig * g.step.flops;
        if (D[k].done) continue;
        if (hs[k].done) {
          D[k].theta = th[k];
          D[k].k = hs[k].k;
          D[k].it = hs[k].state == 2 ? g.dav_max_iter : hs[k].it;
          D[k].conv = hs[k].state != 2;
          fin.push_back(k);
        } else {
          live = true;
        }
      }
      finish(fin);
      prev = hs;
      if (!live) break;
    }
    sync();
    return;
  }

  while (true) {
    act.clear();
    fin.clear();
    for (size_t k = 0; k < ne; ++k) {
      if (D[k].done) continue;
      if (D[k].it > E[k]->dav_max_iter) {  // out of iterations
        D[k].it = E[k]->dav_max_iter;
        fin.push_back(k);
        continue;
      }
      act.push_back(k);
    }
    finish(fin);
    if (act.empty()) break;
    // Ritz pair of the subspace and its residual norm
    sy.clear();
    sc.clear();
    for (size_t k : act) {
      Engine& g = *E[k];
      if (N(k) == 1) continue;
      sy.push_back({g.dHs.p, g.dav_evals(), g.dav_evecs(), D[k].k, D[k].ms});
      cb.add(g.dV.p, N(k), D[k].k, g.dav_evecs(), 1.0, N(k), g.dx_.p, 0.0);  // x = V s
      cb.add(g.dW.p, N(k), D[k].k, g.dav_evecs(), 1.0, N(k), g.dax.p, 0.0);  // ax = W s
      ew.add(EW_RESIDUAL, g.dax.p, g.dx_.p, g.dav_evals(), g.dr.p, N(k));
      dots.add(g.dr.p, N(k), 1, g.dr.p, N(k), g.dav_nrm(), g.dpartial.p);
    }
    if (!sy.empty()) launch_syev_batch(sg.up(sy), (int)sy.size(), st);
    cb.run(sg, st);
    ew.run(sg, st);
    dots.run(sg, st);
    for (size_t k : act) {
      if (N(k) == 1) {
        sc.push_back(E[k]->dHs.p);
        sc.push_back(E[k]->dHs.p);
      } else {
        sc.push_back(E[k]->dav_evals());
        sc.push_back(E[k]->dav_nrm());
      }
    }
    sg.fetch(sc);
    sync();
    // convergence test; otherwise the preconditioned, orthogonalised residual
    cont.clear();
    fin.clear();
    for (size_t j = 0; j < act.size(); ++j) {
      const size_t k = act[j];
      DavState& d = D[k];
      d.theta = sg.shost[2 * j];
      if (N(k) == 1) {
        ew.add(EW_COPY, E[k]->dV.p, nullptr, nullptr, d.xres, 1);
        d.it = 1;
        d.conv = d.done = true;
        continue;
      }
      const double rn = std::sqrt(std::max(0.0, sg.shost[2 * j + 1]));
      if (rn <= d.tol) {
        d.conv = true;
        fin.push_back(k);
        continue;
      }
      // reduced-precision sigma has a residual floor set by its rounding
      // (observed near 10 eps |theta| for FP32): close to it, stop when the
      // residual has not improved by 10 % for four iterations
      if (d.f32 && rn < 100.0 * d.eps * std::max(1.0, std::fabs(d.theta))) {
        if (rn < 0.9 * d.rbest) {
          d.rbest = rn;
          d.stall = 0;
        } else if (++d.stall >= 4) {
          d.conv = true;
          fin.push_back(k);
          continue;
        }
      }
      cont.push_back(k);
    }
    ew.run(sg, st);  // the one-element copies
    finish(fin);
    if (cont.empty()) continue;
    for (size_t k : cont) {
      Engine& g = *E[k];
      ew.add(EW_PRECOND, g.dr.p, g.step.diag.p, g.dav_evals(), g.dt.p, N(k));
    }
    ew.run(sg, st);
    for (int pass = 0; pass < 2; ++pass) {
      for (size_t k : cont) {
        Engine& g = *E[k];
        dots.add(g.dV.p, N(k), D[k].k, g.dt.p, N(k), g.dav_coef(), g.dpartial.p);
        cb.add(g.dV.p, N(k), D[k].k, g.dav_coef(), -1.0, N(k), g.dt.p, 1.0);
      }
      dots.run(sg, st);
      cb.run(sg, st);
    }
    sc.clear();
    for (size_t k : cont) {
      Engine& g = *E[k];
      dots.add(g.dt.p, N(k), 1, g.dt.p, N(k), g.dav_nrm2(), g.dpartial.p);
      sc.push_back(g.dav_nrm2());
    }
    dots.run(sg, st);
    sg.fetch(sc);
    sync();
    // the new direction into V_k (restarting from the Ritz vector when full)
    next.clear();
    fin.clear();
    {
      std::vector<double> tn(sg.shost, sg.shost + cont.size());
      for (size_t j = 0; j < cont.size(); ++j) {
        const size_t k = cont[j];
        if (!(tn[j] > 1e-28)) {  // preconditioned residual collapsed
          PoolBind b(E[k]->pool);
          if (!E[k]->dav_residual_direction(D[k])) {
            D[k].conv = true;
            fin.push_back(k);
            continue;
          }
        }
        next.push_back(k);
      }
    }
    finish(fin);
    for (size_t k : next) ew.add(EW_NORMALIZE, nullptr, nullptr, E[k]->dav_nrm2(), E[k]->dt.p, N(k));
    ew.run(sg, st);
    for (size_t k : next)
      if (D[k].k >= D[k].ms) {
        PoolBind b(E[k]->pool);
        E[k]->dav_restart(D[k]);
      }
    for (size_t k : next) ew.add(EW_COPY, E[k]->dt.p, nullptr, nullptr, E[k]->dav_x(D[k]), N(k));
    ew.run(sg, st);
    sigma_round(next);
    for (size_t k : next) ++D[k].it;
  }
  sync();
}

// One sweep (left-to-right then right-to-left pass; section "Sweeping") of
// every engine, the micro-iterations of all engines in lockstep: step r of
// each engine still sweeping, then step r + 1.  Engines keep their own
// schedule position, noise and statistics; only the launches are shared.
static bool batch_sweep(const std::vector<Engine*>& E, const std::vector<int>& Dk, std::vector<double>& emin,
                        BatchLaunch& bl) {
  const size_t n = E.size();
  std::vector<int> nsteps(n);
  int maxs = 0;
  for (size_t k = 0; k < n; ++k) {
    Engine& e = *E[k];
    if (!e.mps_ready) fail(-1, "call sadmrg_init_mps or sadmrg_mps_import first");
    if (!((e.cen.kind == C_T0 && e.cen.pos == 0) || (e.cen.kind == C_TWO && e.cen.pos == 0)))
      fail(-1, "a batched sweep starts with every centre at the left end");
    e.wdisc_sweep = 0.0;
    e.warned = false;
    nsteps[k] = 2 * (e.P.L - 1);
    maxs = std::max(maxs, nsteps[k]);
  }
  emin.assign(n, INFINITY);
  const int prec = E[0]->prec;
  const bool use32 = prec >= 1;
  for (int r = 0; r < maxs; ++r) {
    std::vector<Engine*> ea;
    std::vector<size_t> ka;
    std::vector<int> si;
    std::vector<char> sright, ssvd;
    for (size_t k = 0; k < n; ++k) {
      if (r >= nsteps[k]) continue;
      const int L = E[k]->P.L;
      const bool right = r <= L - 2;
      const int i = right ? r : 2 * L - 3 - r;
      ea.push_back(E[k]);
      ka.push_back(k);
      si.push_back(i);
      sright.push_back(right);
      ssvd.push_back(right ? i < L - 2 : i > 0);
    }
    const size_t na = ea.size();
    std::vector<DBuf> xb(na);
    auto clock = std::chrono::steady_clock::now();
    auto lap = [&clock]() {
      const auto t = std::chrono::steady_clock::now();
      const double d = std::chrono::duration<double>(t - clock).count();
      clock = t;
      return d;
    };
    parallel_for(na, BATCH_HOST_THREADS, [&](size_t j) {
      Engine& e = *ea[j];
      PoolBind b(e.pool);
      OwnStream os(e, bl.priv[ka[j]]);
      struct Defer {
        Engine& e;
        ~Defer() { e.defer_p2 = false; }
      } df{e};
      e.defer_p2 = true;
      e.prepare(si[j]);
      xb[j].alloc((size_t)std::max<int64_t>(e.step.n, 1));
    });
    // the accumulating pass balanced over the whole batch
    double tot = 0.0;
    for (Engine* e : ea)
      if (e->step.p2_pending) tot += e->step.g2.total_cost();
    const int gpc2 = E[0]->gpc2;
    const double target = gpc2 > 0 ? tot / ((double)gpc2 * GemmList::cus()) : 0.0;
    for (Engine* e : ea) {
      PoolBind b(e->pool);
      e->plan_pass2(target);
    }
    bl.w_prepare += lap();
    std::vector<DavState> ds(na);
    for (size_t j = 0; j < na; ++j) {
      ds[j].xres = xb[j].p;
      ds[j].tol = use32 ? std::max(ea[j]->dav_tol, ea[j]->mixed_tol) : ea[j]->dav_tol;
      ds[j].f32 = use32;
      ds[j].eps = ea[j]->reduced_eps();
    }
    davidson_lockstep(ea, ds, &bl, bl.stage);
    bl.w_davidson += lap();
    std::vector<double> th(na);
    for (size_t j = 0; j < na; ++j) th[j] = ds[j].theta;
    if (use32) {  // FP64 refinement of the FP32 solutions, sigma shared
      auto shared_sigma = [&](std::vector<const double*> xs, std::vector<double*> ys) {
        if (na == 1) {
          PoolBind b(ea[0]->pool);
          ea[0]->sigma_vec(xs[0], ys[0], false);
        } else {
          bl.sigma(ea, xs, ys, false);
        }
      };
      std::vector<const double*> xs, ts;
      std::vector<double*> ys, ws;
      for (size_t j = 0; j < na; ++j) {
        xs.push_back(xb[j].p);
        ys.push_back(ea[j]->dr.p);
        ts.push_back(ea[j]->dt.p);
        ws.push_back(ea[j]->dax.p);
      }
      shared_sigma(xs, ys);
      const int steps = E[0]->refine_steps;
      const double rtol = E[0]->refine_tol;
      std::vector<char> live(na, 1);  // still refining (a step that could not move x ends it)
      for (int k = 0; k < steps; ++k) {
        std::vector<Engine*> ek;
        std::vector<const double*> tk;
        std::vector<double*> wk;
        for (size_t j = 0; j < na; ++j) {
          if (!live[j]) continue;
          PoolBind b(ea[j]->pool);
          ea[j]->refine_dir(xb[j].p);
        }
        if (rtol > 0.0 && k > 0) {  // residual norms of the refined vectors: done below rtol
          std::vector<const double*> rn;
          std::vector<size_t> idx;
          for (size_t j = 0; j < na; ++j)
            if (live[j]) rn.push_back(ea[j]->dav_nrm()), idx.push_back(j);
          bl.stage.fetch(rn);
          dev_sync(bl.st);
          for (size_t q = 0; q < idx.size(); ++q)
            if (std::sqrt(std::max(0.0, bl.stage.shost[q])) <= rtol) live[idx[q]] = 0;
          bl.stage.reset();
        }
        for (size_t j = 0; j < na; ++j) {
          if (!live[j]) continue;
          ek.push_back(ea[j]);
          tk.push_back(ts[j]);
          wk.push_back(ws[j]);
        }
        if (ek.empty()) break;
        if (ek.size() == 1) {
          PoolBind b(ek[0]->pool);
          ek[0]->sigma_vec(tk[0], wk[0], false);
        } else {
          bl.sigma(ek, tk, wk, false);
        }
        for (size_t j = 0; j < na; ++j) {
          if (!live[j]) continue;
          PoolBind b(ea[j]->pool);
          ea[j]->refine_dots(xb[j].p);
        }
        dev_sync(bl.st);
        bl.stage.reset();
        for (size_t j = 0; j < na; ++j) {
          if (!live[j]) continue;
          PoolBind b(ea[j]->pool);
          bool moved = false;
          th[j] = ea[j]->refine_update(xb[j].p, k + 1 < steps, &moved);
          live[j] = moved;
        }
      }
    }
    bl.w_rayleigh += lap();
    parallel_for(na, BATCH_HOST_THREADS, [&](size_t j) {
      Engine& e = *ea[j];
      PoolBind b(e.pool);
      OwnStream os(e, bl.priv[ka[j]]);
      const double en = e.micro_finish(si[j], Dk[ka[j]], sright[j], ssvd[j], xb[j].p, th[j], ds[j].conv);
      emin[ka[j]] = std::min(emin[ka[j]], en);
      if ((sright[j] && si[j] == e.P.L - 2) || (!sright[j] && si[j] == 0)) e.end_pass();
      if (!sright[j] && si[j] == 0) e.wdisc = e.wdisc_sweep;
      xb[j].release();
    });
    bl.w_finish += lap();
  }
  bool warned = false;
  for (Engine* e : E) warned = warned || e->warned;
  return warned;
}

}  // namespace sadmrg

// ===========================================================================
// MPS exchange and the C ABI
// ===========================================================================
namespace sadmrg {

static const int64_t MPS_MAGIC = 0x3154535053414453LL;

struct Reader {
  const char* p;
  size_t n, o = 0;
  int64_t i64() {
    if (o + 8 > n) fail(-1, "MPS blob truncated");
    int64_t v;
    std::memcpy(&v, p + o, 8);
    o += 8;
    return v;
  }
  void dbl(double* d, size_t cnt) {
    if (o + 8 * cnt > n) fail(-1, "MPS blob truncated");
    std::memcpy(d, p + o, 8 * cnt);
    o += 8 * cnt;
  }
};

static void import_mps(Engine& E, const void* blob, size_t bytes) {
  Problem& P = E.P;
  E.check_target();
  Reader r{(const char*)blob, bytes};
  if (r.i64() != MPS_MAGIC) fail(-1, "MPS blob: bad magic");
  const int64_t L = r.i64(), N = r.i64(), twoS = r.i64(), irrep = r.i64(), ci = r.i64();
  if (L != P.L || N != P.N || twoS != P.twoS || irrep != P.irrep) fail(-1, "MPS blob does not match the problem");
  if (ci < 0 || ci > L - 2) fail(-1, "MPS blob: bad centre");
  E.build_caps();
  E.dims.assign(P.L + 1, {});
  for (int k = 0; k <= P.L; ++k) {
    const int64_t ns = r.i64();
    for (int64_t j = 0; j < ns; ++j) {
      Sec s{(int)r.i64(), (int)r.i64(), (int)r.i64()};
      const int64_t d = r.i64();
      if (!E.dims[k].sec.empty() && !(E.dims[k].sec.back() < s)) fail(-1, "MPS blob: sectors not sorted");
      E.dims[k].sec.push_back(s);
      E.dims[k].dim.push_back((int)d);
    }
  }
  E.U.clear();
  E.U.resize(P.L);
  E.V.clear();
  E.V.resize(P.L);
  std::vector<double> buf;
  auto read_tensor = [&](Tensor& t) {
    E.alloc_tensor(t);
    int64_t tot = 0;
    for (size_t j = 0; j < t.rows.size(); ++j) tot += (int64_t)t.rows[j] * t.cols[j];
    buf.resize(tot);
    r.dbl(buf.data(), tot);
    dev_h2d(t.data.p, buf.data(), tot * 8, E.st);
  };
  for (int k = 0; k < ci; ++k) {
    Enl El = left_enl(P, k + 1, E.dims[k], nullptr);
    Tensor t;
    t.rowsec = E.dims[k + 1];
    for (size_t j = 0; j < E.dims[k + 1].sec.size(); ++j) {
      const int e = El.find(E.dims[k + 1].sec[j]);
      if (e < 0) fail(-1, "MPS blob: sector unreachable from the left");
      t.rows.push_back(El.dim[e]);
      t.cols.push_back(E.dims[k + 1].dim[j]);
    }
    read_tensor(t);
    E.U[k] = std::move(t);
  }
  for (int k = (int)ci + 2; k < P.L; ++k) {
    Enl Er = right_enl(P, k, E.dims[k + 1], nullptr);
    Tensor t;
    t.rowsec = E.dims[k];
    for (size_t j = 0; j < E.dims[k].sec.size(); ++j) {
      const int e = Er.find(E.dims[k].sec[j]);
      if (e < 0) fail(-1, "MPS blob: sector unreachable from the right");
      t.rows.push_back(E.dims[k].dim[j]);
      t.cols.push_back(Er.dim[e]);
    }
    read_tensor(t);
    E.V[k] = std::move(t);
  }
  {
    Enl El = left_enl(P, (int)ci + 1, E.dims[ci], nullptr), Er = right_enl(P, (int)ci + 1, E.dims[ci + 2], nullptr);
    Tensor t;
    for (size_t m = 0; m < El.sec.size(); ++m) {
      const int e = Er.find(El.sec[m]);
      if (e < 0) continue;
      t.rowsec.sec.push_back(El.sec[m]);
      t.rowsec.dim.push_back(El.dim[m]);
      t.rows.push_back(El.dim[m]);
      t.cols.push_back(Er.dim[e]);
    }
    read_tensor(t);
    E.cen.kind = C_TWO;
    E.cen.pos = (int)ci;
    E.cen.t = std::move(t);
  }
  if (r.o != r.n) fail(-1, "MPS blob: trailing bytes");
  E.build_blocks_from_tensors((int)ci);
  E.mps_ready = true;
  E.n_pass = 0;
  E.wd_prev = E.wd_pass = 0.0;
  E.lower_rebuild();
}

static void export_mps(Engine& E, std::vector<char>& out) {
  if (E.cen.kind != C_TWO) fail(-1, "export needs a two-site centre (call after a micro-iteration or import)");
  const int ci = E.cen.pos;
  auto put = [&](int64_t v) {
    const char* b = (const char*)&v;
    out.insert(out.end(), b, b + 8);
  };
  auto putT = [&](const Tensor& t) {
    int64_t tot = 0;
    for (size_t j = 0; j < t.rows.size(); ++j) tot += (int64_t)t.rows[j] * t.cols[j];
    std::vector<double> h(tot);
    dev_d2h(h.data(), t.data.p, tot * 8, E.st);
    const char* b = (const char*)h.data();
    out.insert(out.end(), b, b + tot * 8);
  };
  put(MPS_MAGIC);
  put(E.P.L), put(E.P.N), put(E.P.twoS), put(E.P.irrep), put(ci);
  for (int k = 0; k <= E.P.L; ++k) {
    put((int64_t)E.dims[k].sec.size());
    for (size_t j = 0; j < E.dims[k].sec.size(); ++j) {
      put(E.dims[k].sec[j].N), put(E.dims[k].sec[j].tj), put(E.dims[k].sec[j].G), put(E.dims[k].dim[j]);
    }
  }
  for (int k = 0; k < ci; ++k) putT(E.U[k]);
  for (int k = ci + 2; k < E.P.L; ++k) putT(E.V[k]);
  putT(E.cen.t);
}

// Discarded-weight extrapolation (section "Extrapolation"): the least-squares
// line E = E0 + C1 w through the (w, E) pairs with w > 0; a pair with w = 0 is
// an exact energy at its D and is returned as E0 (the lowest of them); one
// truncated pair carries no slope.
static void fit_line(int n, const double* w, const double* e, double* e0, double* c1) {
  double best_exact = INFINITY;
  int nt = 0;
  double sw = 0.0, se = 0.0;
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(w[i]) || !std::isfinite(e[i]) || w[i] < 0.0) fail(-1, "bad (w, E) pair");
    if (w[i] == 0.0) {
      best_exact = std::min(best_exact, e[i]);
    } else {
      ++nt;
      sw += w[i];
      se += e[i];
    }
  }
  if (std::isfinite(best_exact)) {
    *e0 = best_exact;
    *c1 = 0.0;
    return;
  }
  if (nt == 1) {
    *e0 = se;
    *c1 = 0.0;
    return;
  }
  // centred normal equations of the two-parameter fit
  const double mw = sw / nt, me = se / nt;
  double sxx = 0.0, sxy = 0.0;
  for (int i = 0; i < n; ++i) {
    sxx += (w[i] - mw) * (w[i] - mw);
    sxy += (w[i] - mw) * (e[i] - me);
  }
  if (!(sxx > 0.0)) {  // all weights equal: no slope can be fitted
    *e0 = me;
    *c1 = 0.0;
    return;
  }
  *c1 = sxy / sxx;
  *e0 = me - *c1 * mw;
}

}  // namespace sadmrg

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
#include "../../include/sadmrg.h"

struct sadmrg_ctx {
  sadmrg::DevPool* pool = nullptr;  // outlives e: released by sadmrg_destroy
  sadmrg::Engine e;
  std::string err;
};

namespace {
struct PoolScope {  // binds a context's device-memory pool for one call
  sadmrg::DevPool* prev;
  explicit PoolScope(sadmrg::DevPool* p) : prev(sadmrg::dev_pool_bind(p)) {}
  ~PoolScope() { sadmrg::dev_pool_bind(prev); }
};
}  // namespace

using sadmrg::Failure;

template <class F>
static int guard(sadmrg_ctx* c, F&& f) {
  if (!c) return SADMRG_EINVAL;
  PoolScope scope(c->pool);
  try {
    c->err.clear();
    return f();
  } catch (const Failure& x) {
    c->err = x.msg;
    return x.code;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return SADMRG_ENOMEM;
  } catch (const std::exception& x) {
    c->err = x.what();
    return SADMRG_EINVAL;
  }
}

extern "C" {

const char* sadmrg_version(void) { return "sadmrg 0.1 (gfx950, FP64)"; }

int sadmrg_create(sadmrg_ctx** out, int L, int group_order, const int* orb_irrep, int device) {
  if (!out) return SADMRG_EINVAL;
  *out = nullptr;
  if (L < 2 || L > 4096 || !orb_irrep) return SADMRG_EINVAL;
  if (group_order != 1 && group_order != 2 && group_order != 4 && group_order != 8) return SADMRG_EINVAL;
  for (int i = 0; i < L; ++i)
    if (orb_irrep[i] < 0 || orb_irrep[i] >= group_order) return SADMRG_EINVAL;
  auto* c = new (std::nothrow) sadmrg_ctx();
  if (!c) return SADMRG_ENOMEM;
  c->pool = sadmrg::dev_pool_create();
  int rc = guard(c, [&] {
    const int nd = sadmrg::dev_count();
    if (nd <= 0) sadmrg::fail(SADMRG_EDEVICE, "no HIP device available");
    if (device < 0 || device >= nd) sadmrg::fail(SADMRG_EINVAL, "device index out of range");
    sadmrg::dev_set_device(device);
    sadmrg::scratch_init(device);
    c->e.device = device;
    c->e.pool = c->pool;
    c->e.P.L = L;
    c->e.P.order = group_order;
    c->e.P.orb.assign(orb_irrep, orb_irrep + L);
    return 0;
  });
  if (rc != 0) {
    sadmrg_destroy(c);
    return rc;
  }
  *out = c;
  return 0;
}

void sadmrg_destroy(sadmrg_ctx* ctx) {
  if (!ctx) return;
  sadmrg::DevPool* pool = ctx->pool;
  {
    PoolScope scope(pool);
    try {
      sadmrg::dev_sync(ctx->e.st);
    } catch (...) {
    }
    delete ctx;  // device blocks return to the pool
  }
  sadmrg::dev_pool_destroy(pool);
}

int sadmrg_set_allocator(sadmrg_ctx* ctx, sadmrg_alloc_fn alloc_fn, sadmrg_free_fn free_fn, void* user) {
  return guard(ctx, [&] {
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) sadmrg::fail(SADMRG_EINVAL, "give both callbacks or neither");
    sadmrg::dev_sync(ctx->e.st);
    if (!sadmrg::dev_pool_set_allocator(ctx->pool, alloc_fn, free_fn, user, ctx->e.device))
      sadmrg::fail(SADMRG_EINVAL, "the context already holds device memory: set the allocator right after creation");
    return 0;
  });
}

int sadmrg_set_stream(sadmrg_ctx* ctx, void* hip_stream) {
  return guard(ctx, [&] {
    sadmrg::dev_sync(ctx->e.st);  // cached blocks are idle before the stream changes
    ctx->e.st = hip_stream;
    return 0;
  });
}

int sadmrg_set_integrals(sadmrg_ctx* ctx, double e_const, const double* h, const double* eri, double sym_tol) {
  return guard(ctx, [&] {
    auto& P = ctx->e.P;
    if (!h || !eri) sadmrg::fail(SADMRG_EINVAL, "null integrals");
    const int L = P.L;
    const size_t n4 = (size_t)L * L * L * L;
    for (size_t i = 0; i < (size_t)L * L; ++i)
      if (!std::isfinite(h[i])) sadmrg::fail(SADMRG_EINTEG, "h contains NaN/Inf");
    for (size_t i = 0; i < n4; ++i)
      if (!std::isfinite(eri[i])) sadmrg::fail(SADMRG_EINTEG, "eri contains NaN/Inf");
    if (!std::isfinite(e_const)) sadmrg::fail(SADMRG_EINTEG, "E_const is not finite");
    auto E4 = [&](int p, int q, int r, int s) { return eri[(((size_t)p * L + q) * L + r) * L + s]; };
    for (int p = 0; p < L; ++p)
      for (int q = 0; q < L; ++q) {
        if (std::abs(h[p * L + q] - h[q * L + p]) > sym_tol) sadmrg::fail(SADMRG_EINTEG, "h is not symmetric");
        if (P.orb[p] != P.orb[q] && std::abs(h[p * L + q]) > sym_tol)
          sadmrg::fail(SADMRG_EINTEG, "h breaks the point-group symmetry");
      }
    for (int p = 0; p < L; ++p)
      for (int q = 0; q < L; ++q)
        for (int r = 0; r < L; ++r)
          for (int s = 0; s < L; ++s) {
            const double v = E4(p, q, r, s);
            if (std::abs(v - E4(r, s, p, q)) > sym_tol || std::abs(v - E4(q, p, s, r)) > sym_tol)
              sadmrg::fail(SADMRG_EINTEG, "eri lacks the symmetry (pq|rs) = (rs|pq) = (qp|sr)");
            if ((P.orb[p] ^ P.orb[q] ^ P.orb[r] ^ P.orb[s]) != 0 && std::abs(v) > sym_tol)
              sadmrg::fail(SADMRG_EINTEG, "eri breaks the point-group symmetry");
          }
    P.e_const = e_const;
    P.h.assign(h, h + (size_t)L * L);
    P.eri.assign(eri, eri + n4);
    // symmetry-forbidden elements within tolerance are set to exact zeros
    for (int p = 0; p < L; ++p)
      for (int q = 0; q < L; ++q)
        if (P.orb[p] != P.orb[q]) P.h[p * L + q] = 0.0;
    for (int p = 0; p < L; ++p)
      for (int q = 0; q < L; ++q)
        for (int r = 0; r < L; ++r)
          for (int s = 0; s < L; ++s)
            if ((P.orb[p] ^ P.orb[q] ^ P.orb[r] ^ P.orb[s]) != 0) P.eri[(((size_t)p * L + q) * L + r) * L + s] = 0.0;
    P.have_ints = true;
    if (P.N >= 2) P.fold();
    ctx->e.mps_ready = false;
    return 0;
  });
}

int sadmrg_set_target(sadmrg_ctx* ctx, int N, int twoS, int irrep) {
  return guard(ctx, [&] {
    auto& P = ctx->e.P;
    if (N < 2 || N > 2 * P.L || twoS < 0 || twoS > N || ((N - twoS) & 1) || irrep < 0 || irrep >= P.order ||
        twoS > 2 * P.L - N)
      sadmrg::fail(SADMRG_ESYMM, "inconsistent (N, 2S, irrep)");
    P.N = N;
    P.twoS = twoS;
    P.irrep = irrep;
    if (P.have_ints) P.fold();
    ctx->e.mps_ready = false;
    ctx->e.lower_clear();  // lower states of another sector
    return 0;
  });
}

int sadmrg_set_davidson(sadmrg_ctx* ctx, double tol, int max_sub, int max_iter) {
  return guard(ctx, [&] {
    if (!(tol > 0) || max_sub < 2 || max_sub > 64 || max_iter < 1) sadmrg::fail(SADMRG_EINVAL, "bad Davidson settings");
    ctx->e.dav_tol = tol;
    ctx->e.dav_max_sub = max_sub;
    ctx->e.dav_max_iter = max_iter;
    return 0;
  });
}

int sadmrg_set_seed(sadmrg_ctx* ctx, uint64_t seed) {
  return guard(ctx, [&] {
    ctx->e.seed = seed;
    return 0;
  });
}

int sadmrg_init_mps(sadmrg_ctx* ctx, int D) {
  return guard(ctx, [&] {
    ctx->e.init_mps(D);
    return 0;
  });
}

int sadmrg_sweep(sadmrg_ctx* ctx, int D, double* e_min) {
  return guard(ctx, [&] {
    if (D < 1) sadmrg::fail(SADMRG_EINVAL, "D must be positive");
    ctx->e.warned = false;
    const double e = ctx->e.sweep(D);
    if (e_min) *e_min = e;
    return ctx->e.warned ? SADMRG_WARN_NOT_CONVERGED : 0;
  });
}

int sadmrg_batch_sweep(sadmrg_ctx* const* ctxs, int n, const int* D, double* e_min, double* stats) {
  if (!ctxs || n < 1 || !D) return SADMRG_EINVAL;
  for (int k = 0; k < n; ++k) {
    if (!ctxs[k]) return SADMRG_EINVAL;
    ctxs[k]->err.clear();
    for (int j = 0; j < k; ++j)
      if (ctxs[j] == ctxs[k]) {
        ctxs[k]->err = "a context appears twice in the batch";
        return SADMRG_EINVAL;
      }
  }
  auto fail_all = [&](int code, const std::string& msg) {
    for (int k = 0; k < n; ++k) ctxs[k]->err = msg;
    return code;
  };
  sadmrg::Engine& e0 = ctxs[0]->e;
  for (int k = 0; k < n; ++k) {
    const sadmrg::Engine& e = ctxs[k]->e;
    if (D[k] < 1) return fail_all(SADMRG_EINVAL, "D must be positive");
    if (e.device != e0.device || e.st != e0.st)
      return fail_all(SADMRG_EINVAL, "batched contexts must share one device and one stream");
    if (e.prec != e0.prec || e.refine_steps != e0.refine_steps || e.refine_tol != e0.refine_tol ||
        e.dav_graph != e0.dav_graph || e.renorm_prec != e0.renorm_prec)
      return fail_all(SADMRG_EINVAL, "batched contexts must share one precision mode, refinement and recording");
  }
  try {
    std::vector<sadmrg::Engine*> E;
    for (int k = 0; k < n; ++k) E.push_back(&ctxs[k]->e);
    std::vector<double> em;
    bool warned;
    double t64 = 0.0, t32 = 0.0;
    sadmrg::BatchLaunch bl(e0.st, ctxs[0]->pool, (size_t)n);
    warned = sadmrg::batch_sweep(E, std::vector<int>(D, D + n), em, bl);
    bl.times(t64, t32);
    if (e_min)
      for (int k = 0; k < n; ++k) e_min[k] = em[k];
    if (stats) {
      stats[0] = t64;
      stats[1] = bl.f64;
      stats[2] = (double)bl.n64;
      stats[3] = t32;
      stats[4] = bl.f32;
      stats[5] = (double)bl.n32;
      stats[6] = bl.w_prepare;
      stats[7] = bl.w_davidson;
      stats[8] = bl.w_rayleigh;
      stats[9] = bl.w_finish;
    }
    return warned ? SADMRG_WARN_NOT_CONVERGED : 0;
  } catch (const sadmrg::Failure& x) {
    return fail_all(x.code, x.msg);
  } catch (const std::bad_alloc&) {
    return fail_all(SADMRG_ENOMEM, "host allocation failed");
  } catch (const std::exception& x) {
    return fail_all(SADMRG_EINVAL, x.what());
  }
}

int sadmrg_solve(sadmrg_ctx* ctx, int n, const int* D, const double* e_conv, const int* max_sweeps,
                 const double* noise, double* e_min) {
  return guard(ctx, [&] {
    if (n < 1 || !D || !e_conv || !max_sweeps) sadmrg::fail(SADMRG_EINVAL, "bad schedule");
    for (int i = 0; i < n; ++i) {
      if (D[i] < 1 || max_sweeps[i] < 1 || !(e_conv[i] >= 0)) sadmrg::fail(SADMRG_EINVAL, "bad schedule entry");
      if (noise && !(noise[i] >= 0.0)) sadmrg::fail(SADMRG_EINVAL, "noise must be non-negative");
    }
    auto& E = ctx->e;
    if (!E.mps_ready) E.init_mps(D[0]);
    E.warned = false;
    double prev = INFINITY;
    struct NoiseReset {  // the noise applies to this schedule only
      sadmrg::Engine& e;
      ~NoiseReset() { e.noise = 0.0; }
    } reset{E};
    for (int i = 0; i < n; ++i) {
      E.noise = noise ? noise[i] : 0.0;
      for (int s = 0; s < max_sweeps[i]; ++s) {
        const double e = E.sweep(D[i]);
        const bool done = std::abs(e - prev) < e_conv[i];
        prev = e;
        if (done) break;
      }
    }
    if (e_min) *e_min = E.emin;
    return E.warned ? SADMRG_WARN_NOT_CONVERGED : 0;
  });
}

int sadmrg_extrapolate(int n, const double* w, const double* e, double* e0, double* c1) {
  if (n < 1 || !w || !e || !e0 || !c1) return SADMRG_EINVAL;
  try {
    sadmrg::fit_line(n, w, e, e0, c1);
  } catch (const sadmrg::Failure& f) {
    return f.code;
  }
  return 0;
}

int sadmrg_solve_extrapolated(sadmrg_ctx* ctx, int n, const int* D, const double* e_conv, const int* max_sweeps,
                              const double* noise, double* points, double* e0, double* c1) {
  return guard(ctx, [&] {
    if (n < 1 || !D || !e_conv || !max_sweeps) sadmrg::fail(SADMRG_EINVAL, "bad schedule");
    auto& E = ctx->e;
    std::vector<double> ws(n), es(n);
    int warn = 0;
    for (int i = 0; i < n; ++i) {
      const double nz = noise ? noise[i] : 0.0;
      const int rc = sadmrg_solve(ctx, 1, D + i, e_conv + i, max_sweeps + i, &nz, nullptr);
      if (rc < 0) throw sadmrg::Failure{rc, ctx->err};
      if (rc > 0) warn = rc;
      // E(D): lowest energy of the stage's last macro-iteration; w(D): its
      // largest discarded weight
      const size_t per = 2 * (size_t)(E.P.L - 1);
      const size_t nt = E.trace.size();
      double lo = INFINITY;
      for (size_t k = nt > per ? nt - per : 0; k < nt; ++k) lo = std::min(lo, E.trace[k]);
      ws[i] = E.wdisc;
      es[i] = lo;
      if (points) {
        points[3 * i] = D[i];
        points[3 * i + 1] = ws[i];
        points[3 * i + 2] = es[i];
      }
    }
    double a = 0.0, b = 0.0;
    sadmrg::fit_line(n, ws.data(), es.data(), &a, &b);
    if (e0) *e0 = a;
    if (c1) *c1 = b;
    return warn;
  });
}

int sadmrg_rotate_integrals(int L, const double* R, const double* h, const double* eri, double* h_out,
                            double* eri_out) {
  if (L < 1 || !R || !h || !eri || !h_out || !eri_out) return SADMRG_EINVAL;
  try {
    sadmrg::rotate_integrals(L, R, h, eri, h_out, eri_out);
  } catch (const std::bad_alloc&) {
    return SADMRG_ENOMEM;
  }
  return 0;
}

int sadmrg_rotation(int L, const double* kappa, double* R) {
  if (L < 1 || !kappa || !R) return SADMRG_EINVAL;
  for (int p = 0; p < L; ++p)
    for (int q = 0; q < L; ++q)
      if (!std::isfinite(kappa[(size_t)p * L + q]) ||
          std::abs(kappa[(size_t)p * L + q] + kappa[(size_t)q * L + p]) > 1e-12)
        return SADMRG_EINVAL;
  try {
    sadmrg::expm_antisym(L, kappa, R);
  } catch (const std::bad_alloc&) {
    return SADMRG_ENOMEM;
  }
  return 0;
}

int sadmrg_orbital_derivatives(int L, const double* h, const double* eri, const double* D, const double* d,
                               int npairs, const int* pairs, double* grad, double* hess, double* fock) {
  if (L < 1 || !h || !eri || !D || !d || npairs < 0 || (npairs > 0 && (!pairs || !grad))) return SADMRG_EINVAL;
  std::vector<std::pair<int, int>> pr;
  for (int a = 0; a < npairs; ++a) {
    const int p = pairs[2 * a], q = pairs[2 * a + 1];
    if (p < 0 || p >= L || q < 0 || q >= L || p == q) return SADMRG_EINVAL;
    pr.push_back({p, q});
  }
  std::vector<int> occ;  // orbitals where D or d is nonzero
  const size_t L3 = (size_t)L * L * L;
  for (int p = 0; p < L; ++p) {
    bool nz = false;
    for (int q = 0; q < L && !nz; ++q) nz = D[(size_t)p * L + q] != 0.0;
    for (size_t r = 0; r < L3 && !nz; ++r) nz = d[(size_t)p * L3 + r] != 0.0;
    if (nz) occ.push_back(p);
  }
  std::vector<double> g(std::max(npairs, 1));
  try {
    sadmrg::orbital_derivatives(L, h, eri, D, d, occ, pr, fock, npairs ? grad : g.data(), hess);
  } catch (const std::bad_alloc&) {
    return SADMRG_ENOMEM;
  }
  return 0;
}

int sadmrg_dmrgscf(sadmrg_ctx* ctx, int Lt, const int* orb_irrep, const int* cls, double e_nuc, const double* h,
                   const double* eri, int n_sched, const int* D, const double* e_conv, const int* max_sweeps,
                   const double* noise, double grad_tol, int max_iter, double max_step, double* U,
                   double* history, int* n_iter, double* energy) {
  return guard(ctx, [&] {
    using namespace sadmrg;
    auto& E = ctx->e;
    if (Lt < 2 || !orb_irrep || !cls || !h || !eri || max_iter < 1 || !(grad_tol > 0.0) || !(max_step > 0.0))
      fail(SADMRG_EINVAL, "bad DMRG-SCF arguments");
    if (n_sched < 1 || !D || !e_conv || !max_sweeps) fail(SADMRG_EINVAL, "bad schedule");
    std::vector<int> core, act;
    for (int p = 0; p < Lt; ++p) {
      if (cls[p] < 0 || cls[p] > 2) fail(SADMRG_EINVAL, "orbital class must be 0 (core), 1 (active) or 2 (virtual)");
      if (orb_irrep[p] < 0 || orb_irrep[p] >= E.P.order) fail(SADMRG_EINVAL, "orbital irrep out of range");
      if (cls[p] == 0) core.push_back(p);
      if (cls[p] == 1) act.push_back(p);
    }
    const int La = (int)act.size();
    if (La != E.P.L) fail(SADMRG_EINVAL, "the context must have one orbital per active orbital");
    for (int t = 0; t < La; ++t)
      if (orb_irrep[act[t]] != E.P.orb[t]) fail(SADMRG_EINVAL, "active orbital irreps differ from the context's");
    if (E.P.N < 2) fail(SADMRG_ESYMM, "set the active-space target (N, 2S, irrep) on the context first");
    std::vector<std::pair<int, int>> pairs;  // non-redundant rotations
    for (int p = 0; p < Lt; ++p)
      for (int q = 0; q < p; ++q)
        if (cls[p] != cls[q] && orb_irrep[p] == orb_irrep[q]) pairs.push_back({p, q});
    const size_t n2 = (size_t)Lt * Lt, n4 = n2 * n2;
    std::vector<double> R(n2, 0.0), ht(n2), gt(n4), ha((size_t)La * La), ga((size_t)La * La * La * La);
    if (U)
      std::copy(U, U + n2, R.begin());
    else
      for (int p = 0; p < Lt; ++p) R[(size_t)p * Lt + p] = 1.0;
    std::vector<double> g1((size_t)La * La), G2((size_t)La * La * La * La), Dm(n2), dm(n4);
    auto gi = [&](int p, int q, int r, int s) { return gt[(((size_t)p * Lt + q) * Lt + r) * Lt + s]; };
    double e = 0.0;
    int it = 0;
    for (; it < max_iter; ++it) {
      rotate_integrals(Lt, R.data(), h, eri, ht.data(), gt.data());
      // core energy and the active-space Hamiltonian in the core's field
      double e_core = e_nuc;
      for (int c : core) e_core += 2.0 * ht[(size_t)c * Lt + c];
      for (int c : core)
        for (int c2 : core) e_core += 2.0 * gi(c, c, c2, c2) - gi(c, c2, c2, c);
      for (int t = 0; t < La; ++t)
        for (int u = 0; u < La; ++u) {
          double v = ht[(size_t)act[t] * Lt + act[u]];
          for (int c : core) v += 2.0 * gi(act[t], act[u], c, c) - gi(act[t], c, c, act[u]);
          ha[(size_t)t * La + u] = v;
        }
      for (int t = 0; t < La; ++t)
        for (int u = 0; u < La; ++u)
          for (int v = 0; v < La; ++v)
            for (int w = 0; w < La; ++w) ga[(((size_t)t * La + u) * La + v) * La + w] = gi(act[t], act[u], act[v], act[w]);
      // warm start: the converged MPS of the previous orbitals
      std::vector<char> blob;
      if (E.mps_ready) {
        size_t nb = 0;
        int rc = sadmrg_mps_export(ctx, nullptr, &nb);
        if (rc == 0) {
          blob.resize(nb);
          rc = sadmrg_mps_export(ctx, blob.data(), &nb);
        }
        if (rc != 0) blob.clear();
      }
      int rc = sadmrg_set_integrals(ctx, e_core, ha.data(), ga.data(), 1e-9);
      if (rc < 0) throw Failure{rc, ctx->err};
      if (!blob.empty()) {
        rc = sadmrg_mps_import(ctx, blob.data(), blob.size());
        if (rc < 0) throw Failure{rc, ctx->err};
      }
      rc = sadmrg_solve(ctx, n_sched, D, e_conv, max_sweeps, noise, nullptr);
      if (rc < 0) throw Failure{rc, ctx->err};
      e = E.rdms(g1.data(), G2.data(), 1);  // chemist: G2[t][u][v][w] = d_tuvw
      // full-space RDMs of (closed-shell core) x (active state)
      std::fill(Dm.begin(), Dm.end(), 0.0);
      std::fill(dm.begin(), dm.end(), 0.0);
      auto DD = [&](int p, int q) -> double& { return Dm[(size_t)p * Lt + q]; };
      auto dd = [&](int p, int q, int r, int s) -> double& { return dm[(((size_t)p * Lt + q) * Lt + r) * Lt + s]; };
      for (int c : core) DD(c, c) = 2.0;
      for (int t = 0; t < La; ++t)
        for (int u = 0; u < La; ++u) DD(act[t], act[u]) = g1[(size_t)t * La + u];
      for (int c : core)
        for (int c2 : core) {
          dd(c, c, c2, c2) += 4.0;
          dd(c, c2, c2, c) -= 2.0;
        }
      for (int c : core)
        for (int t = 0; t < La; ++t)
          for (int u = 0; u < La; ++u) {
            const double gtu = g1[(size_t)t * La + u];
            dd(c, c, act[t], act[u]) += 2.0 * gtu;
            dd(act[t], act[u], c, c) += 2.0 * gtu;
            dd(c, act[u], act[t], c) -= gtu;
            dd(act[t], c, c, act[u]) -= gtu;
          }
      for (int t = 0; t < La; ++t)
        for (int u = 0; u < La; ++u)
          for (int v = 0; v < La; ++v)
            for (int w = 0; w < La; ++w)
              dd(act[t], act[u], act[v], act[w]) = G2[(((size_t)t * La + u) * La + v) * La + w];
      std::vector<int> occ(core);
      occ.insert(occ.end(), act.begin(), act.end());
      std::sort(occ.begin(), occ.end());
      const int np = (int)pairs.size();
      std::vector<double> grad(std::max(np, 1)), hess((size_t)np * np);
      orbital_derivatives(Lt, ht.data(), gt.data(), Dm.data(), dm.data(), occ, pairs, nullptr, grad.data(),
                          nullptr);
      double gn = 0.0;
      for (int a = 0; a < np; ++a) gn += grad[a] * grad[a];
      gn = std::sqrt(gn);
      if (history) {
        history[2 * it] = e;
        history[2 * it + 1] = gn;
      }
      if (gn < grad_tol || np == 0) {
        ++it;
        break;
      }
      orbital_derivatives(Lt, ht.data(), gt.data(), Dm.data(), dm.data(), occ, pairs, nullptr, grad.data(),
                          hess.data());
      grad.resize(np);
      const std::vector<double> x = ah_step(grad, hess, max_step);
      std::vector<double> K(n2, 0.0), Rs(n2), Rn(n2);
      for (int a = 0; a < np; ++a) {  // R <- R exp(-kappa)
        K[(size_t)pairs[a].first * Lt + pairs[a].second] = -x[a];
        K[(size_t)pairs[a].second * Lt + pairs[a].first] = x[a];
      }
      expm_antisym(Lt, K.data(), Rs.data());
      for (int p = 0; p < Lt; ++p)
        for (int q = 0; q < Lt; ++q) {
          double v = 0.0;
          for (int k = 0; k < Lt; ++k) v += R[(size_t)p * Lt + k] * Rs[(size_t)k * Lt + q];
          Rn[(size_t)p * Lt + q] = v;
        }
      R.swap(Rn);
    }
    if (U) std::copy(R.begin(), R.end(), U);
    if (n_iter) *n_iter = std::min(it, max_iter);
    if (energy) *energy = e;
    return 0;
  });
}

int sadmrg_push_excitation(sadmrg_ctx* ctx, double eta) {
  return guard(ctx, [&] {
    ctx->e.lower_push(eta);
    return 0;
  });
}

int sadmrg_clear_excitations(sadmrg_ctx* ctx) {
  return guard(ctx, [&] {
    ctx->e.lower_clear();
    return 0;
  });
}

int sadmrg_set_method_counter(sadmrg_ctx* ctx, int on) {
  return guard(ctx, [&] {
    auto& E = ctx->e;
    if (on && !E.P.count_method) {  // kept enlargements carry no piece lists
      E.enl_cache_on_saved = E.enl_cache_on;
      E.enl_cache_on = false;
      E.clear_enl_cache();
    }
    if (!on && E.P.count_method) E.enl_cache_on = E.enl_cache_on_saved;
    E.P.count_method = on != 0;
    E.step.i = -1;
    return 0;
  });
}

int sadmrg_stats_method(sadmrg_ctx* ctx, double* method_flops, double* performed_flops, double* step_method_flops) {
  return guard(ctx, [&] {
    if (method_flops) *method_flops = ctx->e.f_method;
    if (performed_flops) *performed_flops = ctx->e.f_method_perf;
    if (step_method_flops) *step_method_flops = ctx->e.step.method_flops;
    return 0;
  });
}

int sadmrg_get_energy(sadmrg_ctx* ctx, double* e_min, double* e_last, double* wdisc_max) {
  return guard(ctx, [&] {
    if (e_min) *e_min = ctx->e.emin;
    if (e_last) *e_last = ctx->e.elast;
    if (wdisc_max) *wdisc_max = ctx->e.wdisc;
    return 0;
  });
}

int sadmrg_get_trace(sadmrg_ctx* ctx, double* out, int* n) {
  return guard(ctx, [&] {
    if (!n) sadmrg::fail(SADMRG_EINVAL, "null count");
    const int have = (int)ctx->e.trace.size();
    if (out) std::copy(ctx->e.trace.begin(), ctx->e.trace.begin() + std::min(have, *n), out);
    *n = have;
    return 0;
  });
}

int sadmrg_mps_import(sadmrg_ctx* ctx, const void* blob, size_t bytes) {
  return guard(ctx, [&] {
    if (!blob) sadmrg::fail(SADMRG_EINVAL, "null blob");
    sadmrg::import_mps(ctx->e, blob, bytes);
    return 0;
  });
}

int sadmrg_mps_export(sadmrg_ctx* ctx, void* blob, size_t* bytes) {
  return guard(ctx, [&] {
    if (!bytes) sadmrg::fail(SADMRG_EINVAL, "null size");
    std::vector<char> out;
    sadmrg::export_mps(ctx->e, out);
    if (blob) {
      if (*bytes < out.size()) sadmrg::fail(SADMRG_EINVAL, "export buffer too small");
      std::memcpy(blob, out.data(), out.size());
    }
    *bytes = out.size();
    return 0;
  });
}

int sadmrg_prepare_step(sadmrg_ctx* ctx) {
  return guard(ctx, [&] {
    auto& E = ctx->e;
    if (!E.mps_ready) sadmrg::fail(SADMRG_EINVAL, "no MPS");
    int i;
    switch (E.cen.kind) {
      case sadmrg::C_TWO:
      case sadmrg::C_T0:
        i = E.cen.pos;
        break;
      case sadmrg::C_BOND_R:
        i = E.cen.pos;
        break;
      case sadmrg::C_BOND_L:
        i = E.cen.pos - 2;
        break;
      default:
        sadmrg::fail(SADMRG_EINVAL, "no centre");
    }
    E.prepare(i);
    return 0;
  });
}

int sadmrg_psi_layout(sadmrg_ctx* ctx, int* nsec, int64_t* desc, int64_t* n) {
  return guard(ctx, [&] {
    auto& S = ctx->e.step;
    if (S.i < 0 || !S.X) sadmrg::fail(SADMRG_EINVAL, "no prepared step");
    if (nsec) *nsec = (int)S.psi.sec.size();
    if (n) *n = S.n;
    if (desc)
      for (size_t m = 0; m < S.psi.sec.size(); ++m) {
        int64_t* d = desc + 6 * m;
        d[0] = S.psi.sec[m].N, d[1] = S.psi.sec[m].tj, d[2] = S.psi.sec[m].G;
        d[3] = S.dx[m], d[4] = S.dy[m], d[5] = S.off[m];
      }
    return 0;
  });
}

int sadmrg_sigma(sadmrg_ctx* ctx, const double* x, double* y, int on_device) {
  return guard(ctx, [&] {
    auto& E = ctx->e;
    auto& S = E.step;
    if (S.i < 0 || !S.X) sadmrg::fail(SADMRG_EINVAL, "no prepared step");
    if (!x || !y) sadmrg::fail(SADMRG_EINVAL, "null vector");
    const bool f32 = E.prec != 0;
    if (on_device) {
      E.sigma_vec(x, y, f32);
      sadmrg::dev_sync(E.st);
    } else {
      sadmrg::dev_h2d(S.in.p, x, (size_t)S.n * 8, E.st);
      E.sigma_fixed(f32);
      sadmrg::dev_d2h(y, S.out.p, (size_t)S.n * 8, E.st);
    }
    return 0;
  });
}

int sadmrg_heff_diagonal(sadmrg_ctx* ctx, double* d, int on_device) {
  return guard(ctx, [&] {
    auto& E = ctx->e;
    auto& S = E.step;
    if (S.i < 0 || !S.X) sadmrg::fail(SADMRG_EINVAL, "no prepared step");
    if (on_device)
      sadmrg::dev_d2d(d, S.diag.p, (size_t)S.n * 8, E.st);
    else
      sadmrg::dev_d2h(d, S.diag.p, (size_t)S.n * 8, E.st);
    sadmrg::dev_sync(E.st);
    return 0;
  });
}

int sadmrg_debug_guess(sadmrg_ctx* ctx, double* out, int on_device) {
  return guard(ctx, [&] {
    auto& E = ctx->e;
    auto& S = E.step;
    if (S.i < 0 || !S.X) sadmrg::fail(SADMRG_EINVAL, "no prepared step");
    if (!out) sadmrg::fail(SADMRG_EINVAL, "null vector");
    if (on_device)
      sadmrg::dev_d2d(out, S.in.p, (size_t)S.n * 8, E.st);
    else
      sadmrg::dev_d2h(out, S.in.p, (size_t)S.n * 8, E.st);
    sadmrg::dev_sync(E.st);
    return 0;
  });
}

int sadmrg_sigma_noalloc(sadmrg_ctx* ctx, const double* x, double* y) {
  return guard(ctx, [&] {
    using namespace sadmrg;
    auto& E = ctx->e;
    auto& S = E.step;
    if (S.i < 0 || !S.X) fail(SADMRG_EINVAL, "no prepared step");
    if (!x || !y) fail(SADMRG_EINVAL, "null vector");
    if (E.prec != 0) fail(SADMRG_EINVAL, "the allocation-free sigma is FP64: set precision mode 0");
    if (!E.lower.empty()) fail(SADMRG_EINVAL, "the allocation-free sigma has no excited-state projectors");
    if (S.p2_pending) fail(SADMRG_EINVAL, "sigma plan incomplete");
    char* base = (char*)scratch_ptr(E.device);
    std::mutex* use = scratch_lock(E.device);
    if (!base || !use) fail(SADMRG_EDEVICE, "static workspace not initialised on this device");
    const GemmList::Plan* pl[2] = {&S.plan.p1, &S.plan.p2};
    // regions of the static array, each 256-byte aligned: psi in, sigma out,
    // the first pass's workspace, the partial tiles of both passes, then the
    // launch records of both passes with their pointers moved into the array
    size_t off = 0;
    auto take = [&](size_t bytes) {
      const size_t at = off;
      off += (bytes + 255) / 256 * 256;
      return at;
    };
    const size_t o_in = take((size_t)S.n * 8), o_out = take((size_t)S.n * 8);
    const size_t o_ws = take(S.plan.ws.n * 8);
    const size_t o_part[2] = {take(pl[0]->part.n * 8), take(pl[1]->part.n * 8)};
    size_t o_tiles[2], o_tasks[2], o_ws0[2], o_reds[2];
    for (int q = 0; q < 2; ++q) {
      o_tiles[q] = take(pl[q]->tiles.host.size() * sizeof(GTile));
      o_tasks[q] = take(pl[q]->tasks.host.size() * sizeof(GTask));
      o_ws0[q] = take(pl[q]->wstart.host.size() * sizeof(int));
      o_reds[q] = take(pl[q]->reds.host.size() * sizeof(RTile));
    }
    if (off > scratch_bytes())
      fail(SADMRG_EINVAL, "prepared step needs " + std::to_string(off) + " bytes of workspace; the allocation-free sigma holds at most " +
                              std::to_string(scratch_bytes()));
    struct Region {
      const double* from;
      size_t n;
      size_t to;
    };
    const Region reg[] = {{S.in.p, (size_t)S.n, o_in},
                          {S.out.p, (size_t)S.n, o_out},
                          {S.plan.ws.p, S.plan.ws.n, o_ws},
                          {pl[0]->part.p, pl[0]->part.n, o_part[0]},
                          {pl[1]->part.p, pl[1]->part.n, o_part[1]}};
    auto remap = [&](const double* p) -> double* {
      if (!p) return nullptr;
      for (const Region& r : reg)
        if (r.from && p >= r.from && p < r.from + r.n) return (double*)(base + r.to) + (p - r.from);
      return const_cast<double*>(p);  // operator stores: read in place
    };
    // the records, remapped, in one host image of the record regions
    const size_t rec0 = o_tiles[0];
    std::vector<char> img(off - rec0);
    for (int q = 0; q < 2; ++q) {
      GTile* tl = (GTile*)(img.data() + (o_tiles[q] - rec0));
      for (size_t j = 0; j < pl[q]->tiles.host.size(); ++j) {
        tl[j] = pl[q]->tiles.host[j];
        tl[j].out = remap(tl[j].out);
        tl[j].part = remap(tl[j].part);
      }
      GTask* tk = (GTask*)(img.data() + (o_tasks[q] - rec0));
      for (size_t j = 0; j < pl[q]->tasks.host.size(); ++j) {
        tk[j] = pl[q]->tasks.host[j];
        tk[j].a = remap(tk[j].a);
        tk[j].b = remap(tk[j].b);
      }
      if (!pl[q]->wstart.host.empty())
        std::memcpy(img.data() + (o_ws0[q] - rec0), pl[q]->wstart.host.data(), pl[q]->wstart.host.size() * sizeof(int));
      RTile* rd = (RTile*)(img.data() + (o_reds[q] - rec0));
      for (size_t j = 0; j < pl[q]->reds.host.size(); ++j) {
        rd[j] = pl[q]->reds.host[j];
        rd[j].out = remap(rd[j].out);
        rd[j].part = (const double*)remap(rd[j].part);
      }
    }
    // one call at a time per device: the array keeps the last call's contents
    std::lock_guard<std::mutex> lk(*use);
    dev_h2d(base + rec0, img.data(), img.size(), E.st);
    dev_d2d(base + o_in, x, (size_t)S.n * 8, E.st);
    dev_zero(base + o_out, (size_t)S.n * 8, E.st);  // pass 2 accumulates into it
    for (int q = 0; q < 2; ++q) {
      launch_gemm((const GTile*)(base + o_tiles[q]), (const GTask*)(base + o_tasks[q]), (const int*)(base + o_ws0[q]),
                  pl[q]->nwg, pl[q]->stream, pl[q]->tag, false, E.st, false, pl[q]->xcd);
      launch_reduce((const RTile*)(base + o_reds[q]), pl[q]->nreds, false, E.st);
    }
    dev_d2d(y, base + o_out, (size_t)S.n * 8, E.st);
    dev_sync(E.st);
    return 0;
  });
}

int sadmrg_debug_plan_stats(sadmrg_ctx* ctx, int64_t* out) {
  return guard(ctx, [&] {
    auto& S = ctx->e.step;
    if (S.i < 0 || !S.X) sadmrg::fail(SADMRG_EINVAL, "no prepared step");
    if (!out) sadmrg::fail(SADMRG_EINVAL, "null output");
    const sadmrg::GemmList::Plan* pl[2] = {&S.plan.p1, &S.plan.p2};
    for (int q = 0; q < 2; ++q) {
      out[3 * q + 0] = pl[q]->ntiles;
      out[3 * q + 1] = pl[q]->nwg;
      out[3 * q + 2] = pl[q]->nreds;
    }
    return 0;
  });
}

int sadmrg_sigma_counters(sadmrg_ctx* ctx, double* flops, double* bytes, int64_t* tasks) {
  return guard(ctx, [&] {
    auto& S = ctx->e.step;
    if (S.i < 0 || !S.X) sadmrg::fail(SADMRG_EINVAL, "no prepared step");
    if (flops) *flops = S.flops;
    if (bytes) *bytes = S.bytes;
    if (tasks) *tasks = S.ntasks;
    return 0;
  });
}

int sadmrg_stats(sadmrg_ctx* ctx, double* t_sigma, int64_t* n_sigma, double* t_micro, double* flops_sigma,
                 double* t_blocking) {
  return guard(ctx, [&] {
    auto& E = ctx->e;
    if (t_sigma) *t_sigma = E.t_sigma;
    if (n_sigma) *n_sigma = E.n_sigma;
    if (t_micro) *t_micro = E.t_micro;
    if (flops_sigma) *flops_sigma = E.f_sigma;
    if (t_blocking) *t_blocking = E.t_block;
    return 0;
  });
}

int sadmrg_stats_bytes(sadmrg_ctx* ctx, double* bytes_sigma, double* max_enlarged_bytes) {
  return guard(ctx, [&] {
    if (bytes_sigma) *bytes_sigma = ctx->e.b_sigma;
    if (max_enlarged_bytes) *max_enlarged_bytes = ctx->e.max_enl_bytes;
    return 0;
  });
}

int sadmrg_advance(sadmrg_ctx* ctx, int D, int n, double* e_min) {
  return guard(ctx, [&] {
    if (D < 1 || n < 0) sadmrg::fail(SADMRG_EINVAL, "bad arguments");
    const double e = ctx->e.advance(D, n);
    if (e_min) *e_min = e;
    return 0;
  });
}

int sadmrg_debug_task_shapes(sadmrg_ctx* ctx, int* out, int64_t* n) {
  return guard(ctx, [&] {
    auto& S = ctx->e.step;
    if (S.i < 0 || !S.X) sadmrg::fail(SADMRG_EINVAL, "no prepared step");
    if (!n) sadmrg::fail(SADMRG_EINVAL, "null count");
    if (out) {
      const int64_t m = std::min<int64_t>(*n, (int64_t)S.shapes.size());
      for (int64_t i = 0; i < m; ++i)
        for (int q = 0; q < 5; ++q) out[5 * i + q] = S.shapes[i][q];
    }
    *n = (int64_t)S.shapes.size();
    return 0;
  });
}

int sadmrg_stats_passes(sadmrg_ctx* ctx, double* pass1, double* pass2) {
  return guard(ctx, [&] {
    auto& E = ctx->e;
    if (pass1) {
      pass1[0] = E.t_pass1;
      pass1[1] = E.f_pass1;
      pass1[2] = E.b_pass1;
      pass1[3] = (double)E.n_pass1;
    }
    if (pass2) {
      pass2[0] = E.t_pass2;
      pass2[1] = E.f_pass2;
      pass2[2] = E.b_pass2;
      pass2[3] = (double)E.n_pass2;
    }
    return 0;
  });
}

int sadmrg_rdm(sadmrg_ctx* ctx, double* rdm1, double* rdm2, double* energy) {
  return guard(ctx, [&] {
    auto& E = ctx->e;
    if (E.P.N < 2) sadmrg::fail(SADMRG_ESYMM, "no target");
    const double e = E.rdms(rdm1, rdm2);
    if (energy) *energy = e;
    return 0;
  });
}

int sadmrg_calc2dm(sadmrg_ctx* ctx, double* gamma_a, double* gamma_b, int layout, double* rdm1, double* s2,
                   double* energy) {
  return guard(ctx, [&] {
    auto& E = ctx->e;
    if (layout != 0 && layout != 1) sadmrg::fail(SADMRG_EINVAL, "layout must be 0 (paper) or 1 (chemist)");
    if (E.P.N < 2) sadmrg::fail(SADMRG_ESYMM, "no target");
    const double e = E.rdms(rdm1, gamma_a, layout, gamma_b, s2);
    if (energy) *energy = e;
    return 0;
  });
}

int sadmrg_get_s2(sadmrg_ctx* ctx, double* s2) {
  return guard(ctx, [&] {
    if (!s2) sadmrg::fail(SADMRG_EINVAL, "null output");
    if (ctx->e.P.N < 2) sadmrg::fail(SADMRG_ESYMM, "no target");
    ctx->e.rdms(nullptr, nullptr, 0, nullptr, s2);
    return 0;
  });
}

int sadmrg_set_precision(sadmrg_ctx* ctx, int mode, double mixed_tol) {
  return guard(ctx, [&] {
    if (mode < 0 || mode > 2)
      sadmrg::fail(SADMRG_EINVAL, "precision mode must be 0 (FP64), 1 (FP32 mixed) or 2 (BF16x3 mixed)");
    if (mode > 0 && !(mixed_tol > 0.0)) sadmrg::fail(SADMRG_EINVAL, "mixed_tol must be positive");
    ctx->e.prec = mode;
    if (mode > 0) ctx->e.mixed_tol = mixed_tol;
    return 0;
  });
}

int sadmrg_set_refinement(sadmrg_ctx* ctx, int steps) {
  return guard(ctx, [&] {
    if (steps < 1 || steps > 8) sadmrg::fail(SADMRG_EINVAL, "refinement steps must be in 1..8");
    ctx->e.refine_steps = steps;
    return 0;
  });
}

int sadmrg_set_block_checkpoints(sadmrg_ctx* ctx, int interval) {
  return guard(ctx, [&] {
    auto& E = ctx->e;
    if (interval < 0) sadmrg::fail(SADMRG_EINVAL, "checkpoint interval must be >= 0");
    E.ckpt = interval;
    if (interval > 0 && E.enl_cache_on) {  // the kept enlargements would hold what the checkpoints save
      E.enl_cache_on = false;
      E.clear_enl_cache();
    }
    if (E.mps_ready && interval > 0) {
      const int i = E.step.i >= 0 ? E.step.i : (E.cen.pos >= 0 ? std::min(E.cen.pos, E.P.L - 2) : 0);
      E.drop_blocks(std::max(0, i));
    }
    return 0;
  });
}

int sadmrg_stats_blocks(sadmrg_ctx* ctx, int64_t* rebuilt, double* seconds, double* max_bytes, int* held) {
  return guard(ctx, [&] {
    const auto& E = ctx->e;
    if (rebuilt) *rebuilt = E.n_rebuilt;
    if (seconds) *seconds = E.t_rebuilt;
    if (max_bytes) *max_bytes = E.block_bytes_max;
    if (held) {
      int n = 0;
      for (auto& x : E.Lb) n += x ? 1 : 0;
      for (auto& x : E.Rb) n += x ? 1 : 0;
      *held = n;
    }
    return 0;
  });
}

int sadmrg_set_davidson_graph(sadmrg_ctx* ctx, int replays) {
  return guard(ctx, [&] {
    if (replays < 0 || replays > 64) sadmrg::fail(SADMRG_EINVAL, "replays must be in 0..64");
    ctx->e.dav_graph = replays;
    return 0;
  });
}

int sadmrg_stats_graph(sadmrg_ctx* ctx, double* seconds, double* record_seconds, double* sigma_flops,
                       int64_t* sigma_calls, int64_t* replays, int64_t* records) {
  return guard(ctx, [&] {
    const auto& E = ctx->e;
    if (seconds) *seconds = E.t_dgraph;
    if (record_seconds) *record_seconds = E.t_dgraph_rec;
    if (sigma_flops) *sigma_flops = E.f_dgraph;
    if (sigma_calls) *sigma_calls = E.n_dgraph_sigma;
    if (replays) *replays = E.n_dgraph_replay;
    if (records) *records = E.n_dgraph_record;
    return 0;
  });
}

int sadmrg_set_renorm_precision(sadmrg_ctx* ctx, int mode) {
  return guard(ctx, [&] {
    if (mode < 0 || mode > 2) sadmrg::fail(SADMRG_EINVAL, "renormalisation precision must be 0, 1 or 2");
    ctx->e.renorm_prec = mode;
    return 0;
  });
}

int sadmrg_set_refinement_tol(sadmrg_ctx* ctx, double tol) {
  return guard(ctx, [&] {
    if (!(tol >= 0.0) || !std::isfinite(tol)) sadmrg::fail(SADMRG_EINVAL, "refinement tolerance must be >= 0");
    ctx->e.refine_tol = tol;
    return 0;
  });
}

int sadmrg_stats_mixed(sadmrg_ctx* ctx, double* t_sigma32, int64_t* n_sigma32, double* flops_sigma32) {
  return guard(ctx, [&] {
    if (t_sigma32) *t_sigma32 = ctx->e.t_sigma32;
    if (n_sigma32) *n_sigma32 = ctx->e.n_sigma32;
    if (flops_sigma32) *flops_sigma32 = ctx->e.f_sigma32;
    return 0;
  });
}

int sadmrg_debug_copy_probe(sadmrg_ctx* ctx, int64_t n, int reps, double* seconds) {
  return guard(ctx, [&] {
    if (n <= 0 || reps <= 0) sadmrg::fail(SADMRG_EINVAL, "copy probe: n and reps must be positive");
    sadmrg::DBuf a, b;
    a.alloc((size_t)n);
    b.alloc((size_t)n);
    sadmrg::launch_fill_uniform(a.p, n, 1, 2, ctx->e.st);
    double t = 0.0;
    for (int r = 0; r < reps; ++r) {
      const sadmrg::Event e0(ctx->e.st);
      sadmrg::launch_copy(b.p, a.p, n, ctx->e.st);
      const sadmrg::Event e1(ctx->e.st);
      t += sadmrg::dev_event_elapsed(e0.p, e1.p);
    }
    sadmrg::dev_sync(ctx->e.st);
    if (seconds) *seconds = t / reps;
    return 0;
  });
}

int sadmrg_debug_gemm_probe(sadmrg_ctx* ctx, int nprod, int K, int reps, double* seconds, double* bytes) {
  return guard(ctx, [&] {
    using namespace sadmrg;
    if (nprod <= 0 || K <= 0 || K > 4096 || reps <= 0) fail(SADMRG_EINVAL, "gemm probe: bad sizes");
    const int64_t per = (int64_t)64 * K;  // one 64 x K panel
    DBuf a, b, c;
    a.alloc((size_t)nprod * per);
    b.alloc((size_t)nprod * per);
    c.alloc((size_t)nprod * 64 * 64);
    launch_fill_uniform(a.p, (int64_t)nprod * per, 3, 4, ctx->e.st);
    launch_fill_uniform(b.p, (int64_t)nprod * per, 5, 6, ctx->e.st);
    GemmList gl;
    for (int q = 0; q < nprod; ++q) {  // c_q = a_q (64 x K) * b_q (K x 64), operands of their own
      const int blk = gl.add_block(c.p + (int64_t)q * 4096, 64, 64, 64, 1);
      gl.add(blk, 64, 64, GTask{a.p + q * per, b.p + q * per, K, 64, K, 0, 1.0});
    }
    GemmList::Plan pl;
    gl.plan(pl, ctx->e.st, 0);
    pl.tag = 0;  // the sigma pass-1 kernel
    double t = 0.0;
    for (int r = 0; r < reps; ++r) {
      const Event e0(ctx->e.st);
      launch_gemm(pl.tiles.p, pl.tasks.p, pl.wstart.p, pl.nwg, pl.stream, pl.tag, false, ctx->e.st);
      const Event e1(ctx->e.st);
      t += dev_event_elapsed(e0.p, e1.p);
    }
    dev_sync(ctx->e.st);
    if (seconds) *seconds = t / reps;
    if (bytes) *bytes = 8.0 * ((double)nprod * 2 * per + (double)nprod * 4096);
    return 0;
  });
}

int sadmrg_stats_reset(sadmrg_ctx* ctx) {
  return guard(ctx, [&] {
    auto& E = ctx->e;
    E.t_sigma = E.t_micro = E.f_sigma = E.t_block = E.b_sigma = E.max_enl_bytes = 0;
    E.t_pass1 = E.t_pass2 = E.f_pass1 = E.f_pass2 = E.b_pass1 = E.b_pass2 = 0;
    E.n_pass1 = E.n_pass2 = 0;
    E.t_sigma32 = E.f_sigma32 = 0;
    E.n_sigma32 = 0;
    E.n_sigma = 0;
    E.f_method = E.f_method_perf = 0;
    E.t_dgraph = E.f_dgraph = E.t_dgraph_rec = 0;
    E.n_rebuilt = 0;
    E.t_rebuilt = E.block_bytes_max = 0;
    E.n_dgraph_sigma = E.n_dgraph_replay = E.n_dgraph_record = 0;
    for (double& t : E.t_phase) t = 0.0;
    return 0;
  });
}

int sadmrg_set_contraction_order(sadmrg_ctx* ctx, int mode) {
  return guard(ctx, [&] {
    if (mode != 0 && mode != 1) sadmrg::fail(SADMRG_EINVAL, "contraction order mode must be 0 or 1");
    ctx->e.corder = mode;
    ctx->e.step.i = -1;  // re-plan on the next step
    return 0;
  });
}

int sadmrg_set_xcd_order(sadmrg_ctx* ctx, int pass1, int pass2) {
  return guard(ctx, [&] {
    ctx->e.xcd1 = pass1 ? sadmrg::MI355X_XCDS : 0;
    ctx->e.xcd2 = pass2 ? sadmrg::MI355X_XCDS : 0;
    ctx->e.step.i = -1;  // re-plan on the next step
    return 0;
  });
}

int sadmrg_set_launch_shape(sadmrg_ctx* ctx, int gpc1, int gpc2) {
  return guard(ctx, [&] {
    if (gpc1 < 0 || gpc1 > 64 || gpc2 < 0 || gpc2 > 64)
      sadmrg::fail(SADMRG_EINVAL, "workgroups per CU must be in 0..64");
    ctx->e.gpc1 = gpc1;
    ctx->e.gpc2 = gpc2;
    ctx->e.step.i = -1;  // the next prepared step is planned with them
    return 0;
  });
}

int sadmrg_autotune(sadmrg_ctx* ctx, int reps, int* gpc1, int* gpc2, double* table) {
  return guard(ctx, [&] {
    ctx->e.autotune(reps, table);
    if (gpc1) *gpc1 = ctx->e.gpc1;
    if (gpc2) *gpc2 = ctx->e.gpc2;
    return 0;
  });
}

int sadmrg_device_memory(int device, size_t* free_bytes, size_t* total_bytes) {
  if (!free_bytes || !total_bytes) return SADMRG_EINVAL;
  try {
    const int nd = sadmrg::dev_count();
    if (device < 0 || device >= nd) return SADMRG_EINVAL;
    sadmrg::dev_set_device(device);
    sadmrg::dev_memory_info(free_bytes, total_bytes);
    return 0;
  } catch (...) {
    return SADMRG_EDEVICE;
  }
}

int sadmrg_set_enlarge_cache(sadmrg_ctx* ctx, int on) {
  return guard(ctx, [&] {
    if (on != 0 && on != 1) sadmrg::fail(SADMRG_EINVAL, "on must be 0 or 1");
    ctx->e.enl_cache_on = on != 0;
    if (!on) ctx->e.clear_enl_cache();
    return 0;
  });
}

int sadmrg_stats_phases(sadmrg_ctx* ctx, double* out) {
  return guard(ctx, [&] {
    if (!out) sadmrg::fail(SADMRG_EINVAL, "null output");
    for (int k = 0; k < sadmrg::Engine::PH_N; ++k) out[k] = ctx->e.t_phase[k];
    return 0;
  });
}

const char* sadmrg_last_error(const sadmrg_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int sadmrg_debug_coupling(int which, const int* a, double* out) {
  if (!a || !out) return SADMRG_EINVAL;
  if (which == 0)
    *out = sadmrg::coupling_product(a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], a[8]);
  else if (which == 1)
    *out = sadmrg::coupling_same(a[0], a[1], a[2], a[3], a[4], a[5]);
  else if (which == 2)
    *out = sadmrg::sixj(a[0], a[1], a[2], a[3], a[4], a[5]);
  else
    return SADMRG_EINVAL;
  return 0;
}

}  // extern "C"
