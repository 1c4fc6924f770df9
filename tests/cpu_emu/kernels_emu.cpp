// CPU stand-in for the device layer of libsadmrg (kernels.h), for running the
// engine's host code under ThreadSanitizer / AddressSanitizer on a machine
// without a GPU.  Test infrastructure only: it is linked into the test driver
// executable next to engine.cpp, su2.cpp, scf.cpp and pool.cpp, never into
// the library the Python binding loads.
//
// "Device" memory is host memory; every launch runs to completion on the
// calling thread (so stream order is program order); the arithmetic follows
// the record semantics documented in kernels.h.  The recorded-iteration
// (graph) kernels are not emulated.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../paper_1312_2415_amd/csrc/kernels.h"

namespace sadmrg {

[[noreturn]] void dev_fail(const char* what);

// ---- memory -----------------------------------------------------------------
static constexpr size_t EMU_TOTAL = (size_t)64 << 30;
static std::atomic<int64_t> g_used{0};
static std::mutex g_size_mu;
static std::map<void*, size_t> g_sizes;

void* dev_raw_alloc(size_t bytes) {
  void* p = std::aligned_alloc(256, (bytes + 255) / 256 * 256);
  if (!p) return nullptr;
  {
    std::lock_guard<std::mutex> lk(g_size_mu);
    g_sizes[p] = bytes;
  }
  g_used += (int64_t)bytes;
  return p;
}
void dev_raw_free(void* p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(g_size_mu);
    auto it = g_sizes.find(p);
    if (it != g_sizes.end()) {
      g_used -= (int64_t)it->second;
      g_sizes.erase(it);
    }
  }
  std::free(p);
}
bool dev_raw_meminfo(size_t* fr, size_t* tot) {
  *tot = EMU_TOTAL;
  const int64_t u = g_used.load();
  *fr = u >= (int64_t)EMU_TOTAL ? 0 : EMU_TOTAL - (size_t)u;
  return true;
}
void dev_h2d(void* dst, const void* src, size_t bytes, Stream) {
  if (bytes) std::memcpy(dst, src, bytes);
}
void dev_d2h(void* dst, const void* src, size_t bytes, Stream) {
  if (bytes) std::memcpy(dst, src, bytes);
}
void dev_d2d(void* dst, const void* src, size_t bytes, Stream) {
  if (bytes) std::memmove(dst, src, bytes);
}
void dev_zero(void* p, size_t bytes, Stream) {
  if (bytes) std::memset(p, 0, bytes / 8 * 8);
}
void dev_sync(Stream) {}
void* host_alloc_pinned(size_t bytes) {
  void* p = std::malloc(bytes ? bytes : 8);
  if (!p) dev_fail("host allocation failed");
  return p;
}
void host_free_pinned(void* p) { std::free(p); }
void dev_h2d_async(void* dst, const void* src, size_t bytes, Stream) {
  if (bytes) std::memcpy(dst, src, bytes);
}
void dev_d2h_async(void* dst, const void* src, size_t bytes, Stream) {
  if (bytes) std::memcpy(dst, src, bytes);
}
void dev_set_device(int) {}
int dev_get_device() { return 0; }
size_t dev_total_memory() { return EMU_TOTAL; }
void dev_memory_info(size_t* fr, size_t* tot) { dev_raw_meminfo(fr, tot); }
int dev_count() { return 1; }
int dev_cu_count() { return 256; }

// ---- events and streams -------------------------------------------------------
struct EmuEvent {
  std::chrono::steady_clock::time_point t;
};
void* dev_event_record(Stream) { return new EmuEvent{std::chrono::steady_clock::now()}; }
double dev_event_elapsed(void* a, void* b) {
  return std::chrono::duration<double>(((EmuEvent*)b)->t - ((EmuEvent*)a)->t).count();
}
void dev_event_free(void* e) { delete (EmuEvent*)e; }
void dev_event_wait(void*) {}
Stream dev_stream_create() { return (Stream) new char[1]; }
void dev_stream_destroy(Stream s) { delete[] (char*)s; }
void dev_stream_order(Stream, Stream) {}

// ---- static workspace of the allocation-free entry point -------------------------
// held until the process ends, as the device array it stands in for
static constexpr size_t EMU_SCRATCH = (size_t)32 << 20;
struct AlignedFree {
  void operator()(void* p) const { std::free(p); }
};
static std::mutex g_scratch_mu;
static std::map<int, std::unique_ptr<void, AlignedFree>> g_scratch;
static std::map<int, std::unique_ptr<std::mutex>> g_scratch_lock;
void scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch.count(device)) return;
  g_scratch[device].reset(std::aligned_alloc(256, EMU_SCRATCH));
  g_scratch_lock[device] = std::make_unique<std::mutex>();
}
void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(device);
  return it == g_scratch.end() ? nullptr : it->second.get();
}
std::mutex* scratch_lock(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_lock.find(device);
  return it == g_scratch_lock.end() ? nullptr : it->second.get();
}
size_t scratch_bytes() { return EMU_SCRATCH; }

// ---- grouped GEMM ------------------------------------------------------------------
template <typename T>
static void tile_run(const GTile& t, const GTask* tasks) {
  std::vector<double> acc((size_t)t.rows * t.cols, 0.0);
  for (int q = t.t0; q < t.t1; ++q) {
    const GTask& k = tasks[q];
    const T* A = (const T*)k.a;
    const T* B = (const T*)k.b;
    const bool ta = k.flags & GT_TRANS_A, tb = k.flags & GT_TRANS_B;
    for (int r = 0; r < t.rows; ++r)
      for (int c = 0; c < t.cols; ++c) {
        double s = 0.0;
        for (int x = 0; x < k.K; ++x) {
          const double a = ta ? A[(int64_t)x * k.lda + r] : A[(int64_t)r * k.lda + x];
          const double b = tb ? B[(int64_t)c * k.ldb + x] : B[(int64_t)x * k.ldb + c];
          s += a * b;
        }
        acc[(size_t)r * t.cols + c] += k.coef * s;
      }
  }
  T* out = (T*)t.out;
  T* part = (T*)t.part;
  for (int r = 0; r < t.rows; ++r)
    for (int c = 0; c < t.cols; ++c) {
      const double v = acc[(size_t)r * t.cols + c];
      if (part)
        part[(int64_t)r * t.cols + c] = (T)v;
      else if (t.mode == 1)
        out[(int64_t)r * t.ld + c] = (T)v;
      else
        out[(int64_t)r * t.ld + c] += (T)v;
    }
}
static void plan_run(const GTile* tiles, const GTask* tasks, const int* wstart, int nwg, bool stream, bool f32) {
  const int a = stream ? wstart[0] : 0, b = stream ? wstart[nwg] : nwg;
  for (int i = a; i < b; ++i) {
    if (f32)
      tile_run<float>(tiles[i], tasks);
    else
      tile_run<double>(tiles[i], tasks);
  }
}
std::atomic<int> emu_fail_gemms{0};  // the test driver's injected failure: GEMM launch number n from now fails
void launch_gemm(const GTile* tiles, const GTask* tasks, const int* wstart, int nwg, bool stream, int, bool f32,
                 Stream, bool, int, const int* gate) {
  if (emu_fail_gemms.load() > 0 && emu_fail_gemms.fetch_sub(1) == 1) dev_fail("emulation: injected GEMM failure");
  if (nwg <= 0 || (gate && *gate)) return;
  plan_run(tiles, tasks, wstart, nwg, stream, f32);
}
template <typename T>
static void reduce_run(const RTile& t) {
  T* out = (T*)t.out;
  const T* part = (const T*)t.part;
  const int n = t.rows * t.cols;
  for (int e = 0; e < n; ++e) {
    double s = 0.0;
    for (int p = 0; p < t.nparts; ++p) s += part[(int64_t)p * n + e];
    out[(int64_t)(e / t.cols) * t.ld + e % t.cols] += (T)s;
  }
}
void launch_reduce(const RTile* reds, int nred, bool f32, Stream, const int* gate) {
  if (gate && *gate) return;
  for (int i = 0; i < nred; ++i) {
    if (f32)
      reduce_run<float>(reds[i]);
    else
      reduce_run<double>(reds[i]);
  }
}
void launch_gemm_seg(const GSeg* segs, const int* base, int nseg, int nwg, bool stream, bool f32, Stream, bool) {
  if (emu_fail_gemms.load() > 0 && emu_fail_gemms.fetch_sub(1) == 1) dev_fail("emulation: injected GEMM failure");
  for (int s = 0; s < nseg; ++s) {
    if (segs[s].gate && *segs[s].gate) continue;
    const int n = (s + 1 < nseg ? base[s + 1] : nwg) - base[s];
    plan_run(segs[s].tiles, segs[s].tasks, segs[s].wstart, n, stream, f32);
  }
}
void launch_reduce_seg(const GSeg* segs, const int* base, int nseg, int nred, bool f32, Stream st) {
  for (int s = 0; s < nseg; ++s) {
    const int n = (s + 1 < nseg ? base[s + 1] : nred) - base[s];
    launch_reduce(segs[s].reds, n, f32, st, segs[s].gate);
  }
}

// ---- element-wise and gather kernels ---------------------------------------------
void launch_traces(const TraceJob* jobs, int njobs, double* out, Stream) {
  for (int j = 0; j < njobs; ++j) {
    double s = 0.0;
    for (int r = 0; r < jobs[j].n; ++r) s += jobs[j].p[(int64_t)r * (jobs[j].ld + 1)];
    out[j] = s;
  }
}
void launch_cvt_d2f(float* dst, const double* src, int64_t n, Stream) {
  for (int64_t i = 0; i < n; ++i) dst[i] = (float)src[i];
}
void launch_cvt_f2d(double* dst, const float* src, int64_t n, Stream) {
  for (int64_t i = 0; i < n; ++i) dst[i] = (double)src[i];
}
std::atomic<int> emu_fail_gathers{0};  // the test driver's injected failure: gather number n from now fails
void launch_gather(const GatherDst* dsts, int ndst, const GatherSrc* srcs, Stream) {
  if (emu_fail_gathers.load() > 0 && emu_fail_gathers.fetch_sub(1) == 1) dev_fail("emulation: injected gather failure");
  for (int i = 0; i < ndst; ++i) {
    const GatherDst& d = dsts[i];
    for (int r = 0; r < d.rows; ++r)
      for (int c = 0; c < d.cols; ++c) {
        double v = 0.0;
        for (int s = d.s0; s < d.s1; ++s) {
          const GatherSrc& g = srcs[s];
          if (g.kind == GS_NORMAL)
            v += g.scale * g.src[(int64_t)r * g.ld + c];
          else if (g.kind == GS_TRANS)
            v += g.scale * g.src[(int64_t)c * g.ld + r];
          else if (r == c)
            v += g.scale;
        }
        d.dst[(int64_t)r * d.ld + c] = v;
      }
  }
}
void launch_combo(const ComboOut* outs, int nout, const ComboIn* ins, int64_t, Stream) {
  for (int o = 0; o < nout; ++o) {
    const ComboOut& x = outs[o];
    for (int64_t e = 0; e < x.nnz; ++e) {
      double v = 0.0;
      for (int i = x.i0; i < x.i1; ++i) v += ins[i].adj ? ins[i].coef * x.fac[e] * ins[i].in[x.perm[e]] : ins[i].coef * ins[i].in[e];
      x.out[e] = v;
    }
  }
}
void launch_diag(const DiagSec* secs, int nsec, const DiagTask* tasks, Stream) {
  for (int i = 0; i < nsec; ++i) {
    const DiagSec& s = secs[i];
    for (int r = 0; r < s.rows; ++r)
      for (int c = 0; c < s.cols; ++c) {
        double v = 0.0;
        for (int t = s.t0; t < s.t1; ++t) {
          const DiagTask& d = tasks[t];
          v += d.coef * (d.x ? d.x[(int64_t)r * d.sx] : 1.0) * (d.y ? d.y[(int64_t)c * d.sy] : 1.0);
        }
        s.out[(int64_t)r * s.cols + c] = v;
      }
  }
}

// ---- SVD (one-sided Jacobi, the layout of SvdJob) ----------------------------------
// The working copy lives in the job's work buffer as on the device: M (m x n,
// column j at j*m), V (n x n, column j at j*n), then the norm slot (n).
struct SvdView {
  bool tall;
  int m, n;
  double *M, *V, *nrm;
  explicit SvdView(const SvdJob& jb)
      : tall(jb.rows >= jb.cols), m(tall ? jb.rows : jb.cols), n(tall ? jb.cols : jb.rows), M(jb.work),
        V(jb.work + (size_t)m * n), nrm(jb.work + (size_t)m * n + (size_t)n * n) {}
};
// one Jacobi rotation of columns p, q of M (and V); returns true when the
// pair was rotated and both columns hold more than 1e-13 of the norm
static bool svd_rotate(double* mp, double* mq, double* vp, double* vq, int m, int n, double tol, double fro2) {
  double al = 0, be = 0, ga = 0;
  for (int i = 0; i < m; ++i) {
    al += mp[i] * mp[i];
    be += mq[i] * mq[i];
    ga += mp[i] * mq[i];
  }
  if (std::fabs(ga) <= tol * std::sqrt(al * be) || ga == 0.0) return false;
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
  for (int i = 0; i < m; ++i) {
    const double x = mp[i], y = mq[i];
    mp[i] = cs * x - sn * y;
    mq[i] = sn * x + cs * y;
  }
  for (int i = 0; i < n; ++i) {
    const double x = vp[i], y = vq[i];
    vp[i] = cs * x - sn * y;
    vq[i] = sn * x + cs * y;
  }
  return al > 1e-26 * fro2 && be > 1e-26 * fro2;
}
static void svd_load(const SvdJob& jb) {
  SvdView w(jb);
  for (int j = 0; j < w.n; ++j)
    for (int i = 0; i < w.m; ++i)
      w.M[(size_t)j * w.m + i] = w.tall ? jb.a[(int64_t)i * jb.lda + j] : jb.a[(int64_t)j * jb.lda + i];
  for (size_t e = 0; e < (size_t)w.n * w.n; ++e) w.V[e] = (e / w.n == e % w.n) ? 1.0 : 0.0;
  double fro2 = 0.0;
  for (size_t e = 0; e < (size_t)w.m * w.n; ++e) fro2 += w.M[e] * w.M[e];
  w.nrm[0] = fro2;
}
static void svd_sweeps_serial(const SvdJob& jb) {
  SvdView w(jb);
  const double fro2 = w.nrm[0];
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rot = false;
    for (int p = 0; p < w.n; ++p)
      for (int q = p + 1; q < w.n; ++q)
        rot |= svd_rotate(w.M + (size_t)p * w.m, w.M + (size_t)q * w.m, w.V + (size_t)p * w.n, w.V + (size_t)q * w.n,
                          w.m, w.n, 1e-15, fro2);
    if (!rot) break;
  }
}
static void svd_output(const SvdJob& jb) {
  SvdView w(jb);
  const int m = w.m, n = w.n;
  const bool tall = w.tall;
  const double* M = w.M;
  const double* V = w.V;
  std::vector<double> nrm(n);
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < m; ++i) s += M[(size_t)j * m + i] * M[(size_t)j * m + i];
    nrm[j] = std::sqrt(s);
  }
  std::vector<int> ord(n);
  for (int j = 0; j < n; ++j) ord[j] = j;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return nrm[a] > nrm[b]; });
  const double smax = n ? nrm[ord[0]] : 0.0;
  for (int k = 0; k < n; ++k) jb.s[k] = nrm[ord[k]];
  auto put = [&](int i, int k, double v) {
    if (tall)
      jb.u[(int64_t)i * n + k] = v;
    else
      jb.vt[(int64_t)k * jb.cols + i] = v;
  };
  auto get = [&](int i, int k) { return tall ? jb.u[(int64_t)i * n + k] : jb.vt[(int64_t)k * jb.cols + i]; };
  for (int k = 0; k < n; ++k) {
    const int j = ord[k];
    const double s = nrm[j];
    if (s > 1e-13 * smax && s != 0.0) {
      for (int i = 0; i < m; ++i) put(i, k, M[(size_t)j * m + i] / s);
      continue;
    }
    for (int a = 0; a < m; ++a) {  // completion with unit vectors e_t, t = k, k+1, ... mod m
      const int tt = (k + a) % m;
      for (int i = 0; i < m; ++i) put(i, k, i == tt ? 1.0 : 0.0);
      for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
        std::vector<double> d(k, 0.0);
        for (int kk = 0; kk < k; ++kk)
          for (int i = 0; i < m; ++i) d[kk] += get(i, kk) * get(i, k);
        for (int i = 0; i < m; ++i) {
          double v = get(i, k);
          for (int kk = 0; kk < k; ++kk) v -= d[kk] * get(i, kk);
          put(i, k, v);
        }
      }
      double nn = 0;
      for (int i = 0; i < m; ++i) nn += get(i, k) * get(i, k);
      if (nn > 0.5 * (double)(m - k) / (double)m) {
        for (int i = 0; i < m; ++i) put(i, k, get(i, k) / std::sqrt(nn));
        break;
      }
    }
  }
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < n; ++i) {
      const double v = V[(size_t)ord[k] * n + i];
      if (tall)
        jb.vt[(int64_t)k * jb.cols + i] = v;
      else
        jb.u[(int64_t)i * n + k] = v;
    }
}
void launch_svd(const SvdJob* jobs, int njobs, int, Stream, int phase) {
  for (int j = 0; j < njobs; ++j) {
    if (phase != 2) svd_load(jobs[j]);
    if (phase == 0) svd_sweeps_serial(jobs[j]);
    if (phase != 1) svd_output(jobs[j]);
  }
}
// Block rounds as the device runs them: workgroup b takes block pair b -
// pair_base[k] of job k; the pairs of one round touch disjoint columns, so
// running them one after another is the same computation.
static constexpr int EMU_SVB_W = 16;
std::atomic<long> emu_svd_block_pairs_run{0};  // block pairs processed (read by the test driver)
std::atomic<long> emu_svd_rotations{0};        // column pairs tried by the block rounds
std::atomic<bool> emu_svd_block_off{false};    // the test driver's switch to the one-workgroup path
bool svd_block_fits(int rows, int cols) { return !emu_svd_block_off && rows + cols <= 600; }
int svd_block_pairs(int rows, int cols) {
  const int nblk = (std::min(rows, cols) + EMU_SVB_W - 1) / EMU_SVB_W;
  return (nblk + (nblk & 1)) / 2;
}
int svd_block_rounds(int rows, int cols) {
  const int nblk = (std::min(rows, cols) + EMU_SVB_W - 1) / EMU_SVB_W;
  return nblk + (nblk & 1) - 1;
}
void launch_svd_block(const SvdJob* jobs, const int* pair_base, int njobs, int npairs, int round, const int* active,
                      int* flags, Stream) {
  for (int b = 0; b < npairs; ++b) {
    int k = 0;
    while (k + 1 < njobs && pair_base[k + 1] <= b) ++k;
    if (!active[k]) continue;
    SvdView w(jobs[k]);
    const int nblk = (w.n + EMU_SVB_W - 1) / EMU_SVB_W, npb = nblk + (nblk & 1);
    if (round >= npb - 1) continue;
    const int pr = b - pair_base[k];
    const int ba = (pr == 0) ? 0 : ((pr - 1 + round) % (npb - 1)) + 1;
    const int bb = ((npb - 2 - pr + round) % (npb - 1)) + 1;
    std::vector<int> cols;
    for (int blk : {ba, bb})
      if (blk < nblk)
        for (int c = blk * EMU_SVB_W; c < std::min((blk + 1) * EMU_SVB_W, w.n); ++c) cols.push_back(c);
    const int nc = (int)cols.size();
    const int na = ba < nblk ? std::min((ba + 1) * EMU_SVB_W, w.n) - ba * EMU_SVB_W : 0;
    const bool cross = round > 0;  // later rounds: only the pairs across the two blocks
    if (nc < 2 || (cross && (na == 0 || na == nc))) continue;
    ++emu_svd_block_pairs_run;
    const double tol = std::fmax(1e-15, w.m * 2.220446049250313e-16);
    const int npl = nc + (nc & 1);
    bool sig = false;
    auto rot = [&](int p, int q) {
      ++emu_svd_rotations;
      sig |= svd_rotate(w.M + (size_t)cols[p] * w.m, w.M + (size_t)cols[q] * w.m, w.V + (size_t)cols[p] * w.n,
                        w.V + (size_t)cols[q] * w.n, w.m, w.n, tol, w.nrm[0]);
    };
    if (cross) {
      for (int r = 0; r < EMU_SVB_W; ++r)
        for (int wv = 0; wv < EMU_SVB_W; ++wv) {
          const int p = wv, q = na + (wv + r) % EMU_SVB_W;
          if (p < na && q < nc) rot(p, q);
        }
    } else {
      for (int r = 0; r < npl - 1; ++r)
        for (int wv = 0; wv < npl / 2; ++wv) {
          const int la = (wv == 0) ? 0 : ((wv - 1 + r) % (npl - 1)) + 1;
          const int lb = ((npl - 2 - wv + r) % (npl - 1)) + 1;
          const int p = std::min(la, lb), q = std::max(la, lb);
          if (q >= nc || p == q) continue;
          rot(p, q);
        }
    }
    if (sig) flags[k] = 1;
  }
}
void launch_svd_signs(const SvdJob* jobs, int njobs, Stream) {
  for (int q = 0; q < njobs; ++q) {
    const SvdJob& j = jobs[q];
    const int r = std::min(j.rows, j.cols);
    for (int a = 0; a < r; ++a) {
      double best = -1.0;
      int idx = 0;
      for (int row = 0; row < j.rows; ++row)
        if (std::fabs(j.u[(int64_t)row * r + a]) > best) best = std::fabs(j.u[(int64_t)row * r + a]), idx = row;
      if (j.u[(int64_t)idx * r + a] < 0.0) {
        for (int row = 0; row < j.rows; ++row) j.u[(int64_t)row * r + a] = -j.u[(int64_t)row * r + a];
        for (int c = 0; c < j.cols; ++c) j.vt[(int64_t)a * j.cols + c] = -j.vt[(int64_t)a * j.cols + c];
      }
    }
  }
}

// ---- Davidson helpers ----------------------------------------------------------
void launch_dots(const double* V, int64_t ldv, int k, const double* x, int64_t n, double* out, double*, Stream) {
  for (int j = 0; j < k; ++j) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += V[j * ldv + i] * x[i];
    out[j] = s;
  }
}
void launch_combo_vec(const double* V, int64_t ldv, int k, const double* coef, double alpha, int64_t n, double* y,
                      double beta, Stream) {
  for (int64_t i = 0; i < n; ++i) {
    double s = 0;
    for (int j = 0; j < k; ++j) s += coef[j] * V[j * ldv + i];
    y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + alpha * s;
  }
}
void launch_residual(const double* ax, const double* x, const double* theta, int64_t n, double* r, Stream) {
  for (int64_t i = 0; i < n; ++i) r[i] = ax[i] - theta[0] * x[i];
}
static double guard_den(double d) { return std::fabs(d) < 1e-12 ? (d < 0 ? -1e-12 : 1e-12) : d; }
void launch_precond(const double* r, const double* diag, const double* theta, int64_t n, double* t, Stream) {
  for (int64_t i = 0; i < n; ++i) t[i] = r[i] / guard_den(theta[0] - diag[i]);
}
void launch_normalize(double* y, const double* nrm2, int64_t n, Stream) {
  const double f = 1.0 / std::sqrt(nrm2[0]);
  for (int64_t i = 0; i < n; ++i) y[i] *= f;
}
// symmetric k x k (lower triangle, leading dim ld): cyclic Jacobi
void launch_syev_small(const double* H, int k, int ld, double* evals, double* evecs, Stream) {
  std::vector<double> a((size_t)k * k), v((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j <= i; ++j) a[(size_t)i * k + j] = a[(size_t)j * k + i] = H[(int64_t)i * ld + j];
  for (int i = 0; i < k; ++i) v[(size_t)i * k + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool any = false;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = a[(size_t)p * k + q];
        if (std::fabs(apq) <= 1e-300 || std::fabs(apq) <= 1e-17 * std::sqrt(std::fabs(a[(size_t)p * k + p] * a[(size_t)q * k + q]) + 1e-300))
          continue;
        any = true;
        const double th = (a[(size_t)q * k + q] - a[(size_t)p * k + p]) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(1.0 + th * th));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int j = 0; j < k; ++j) {
          const double x = a[(size_t)p * k + j], y = a[(size_t)q * k + j];
          a[(size_t)p * k + j] = c * x - s * y;
          a[(size_t)q * k + j] = s * x + c * y;
        }
        for (int i = 0; i < k; ++i) {
          const double x = a[(size_t)i * k + p], y = a[(size_t)i * k + q];
          a[(size_t)i * k + p] = c * x - s * y;
          a[(size_t)i * k + q] = s * x + c * y;
          const double vx = v[(size_t)i * k + p], vy = v[(size_t)i * k + q];
          v[(size_t)i * k + p] = c * vx - s * vy;
          v[(size_t)i * k + q] = s * vx + c * vy;
        }
      }
    if (!any) break;
  }
  std::vector<int> ord(k);
  for (int j = 0; j < k; ++j) ord[j] = j;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return a[(size_t)x * k + x] < a[(size_t)y * k + y]; });
  for (int j = 0; j < k; ++j) {
    evals[j] = a[(size_t)ord[j] * k + ord[j]];
    for (int i = 0; i < k; ++i) evecs[(int64_t)j * k + i] = v[(size_t)i * k + ord[j]];
  }
}
void launch_dots_batch(const DotJob* jobs, int njobs, int, Stream st) {
  for (int q = 0; q < njobs; ++q) launch_dots(jobs[q].V, jobs[q].ldv, jobs[q].k, jobs[q].x, jobs[q].n, jobs[q].out, nullptr, st);
}
void launch_combo_batch(const ComboJob* jobs, int njobs, int64_t, Stream st) {
  for (int q = 0; q < njobs; ++q)
    launch_combo_vec(jobs[q].V, jobs[q].ldv, jobs[q].k, jobs[q].coef, jobs[q].alpha, jobs[q].n, jobs[q].y, jobs[q].beta, st);
}
void launch_ew_batch(const EwJob* jobs, int njobs, int64_t, Stream) {
  for (int q = 0; q < njobs; ++q) {
    const EwJob& j = jobs[q];
    for (int64_t i = 0; i < j.n; ++i) switch (j.kind) {
        case EW_COPY: j.y[i] = j.a[i]; break;
        case EW_ZERO: j.y[i] = 0.0; break;
        case EW_RESIDUAL: j.y[i] = j.a[i] - j.s[0] * j.b[i]; break;
        case EW_PRECOND: j.y[i] = j.a[i] / guard_den(j.s[0] - j.b[i]); break;
        case EW_NORMALIZE: j.y[i] *= 1.0 / std::sqrt(j.s[0]); break;
        case EW_D2F: ((float*)j.y)[i] = (float)j.a[i]; break;
        case EW_F2D: j.y[i] = (double)((const float*)j.a)[i]; break;
        default: break;
      }
  }
}
void launch_syev_batch(const SyevJob* jobs, int njobs, Stream st) {
  for (int q = 0; q < njobs; ++q) launch_syev_small(jobs[q].H, jobs[q].k, jobs[q].ld, jobs[q].evals, jobs[q].evecs, st);
}

// ---- recorded iterations: not emulated -------------------------------------------
void launch_dg_scalar(const DGJob*, int, int, Stream) { dev_fail("emulation: recorded iterations not available"); }
void launch_dg_dots(const DGJob*, int, int, int, int, Stream) { dev_fail("emulation: recorded iterations not available"); }
void launch_dg_ew(const DGJob*, int, int, int, int64_t, Stream) { dev_fail("emulation: recorded iterations not available"); }
void launch_dg_combo(const DGJob*, int, int, int, int64_t, Stream) { dev_fail("emulation: recorded iterations not available"); }
void launch_dg_syev(const DGJob*, int, Stream) { dev_fail("emulation: recorded iterations not available"); }
void dev_capture_begin(Stream) { dev_fail("emulation: graphs not available"); }
void* dev_capture_end(Stream) { dev_fail("emulation: graphs not available"); }
void dev_capture_abort(Stream) {}
void dev_graph_launch(void*, Stream) { dev_fail("emulation: graphs not available"); }
void dev_graph_free(void*) {}

// ---- small helpers ------------------------------------------------------------------
void launch_scalars(const double* const* src, int n, double* dst, Stream) {
  for (int i = 0; i < n; ++i) dst[i] = src[i][0];
}
static uint64_t sm64(uint64_t x) {  // SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014)
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
void launch_fill_uniform(double* p, int64_t n, uint64_t seed, uint64_t stream, Stream) {
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t k = sm64(seed ^ sm64(stream * 0x100000001B3ull + (uint64_t)i));
    p[i] = (double)(k >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  }
}
void launch_axpy(double* y, const double* x, double a, int64_t n, Stream) {
  for (int64_t i = 0; i < n; ++i) y[i] += a * x[i];
}
void launch_rects_nonzero(const double* base, const RectDesc* rects, int n, unsigned char* flag, Stream) {
  for (int r = 0; r < n; ++r) {
    unsigned char f = 0;
    for (int i = 0; i < rects[r].rows && !f; ++i)
      for (int j = 0; j < rects[r].cols; ++j)
        if (base[rects[r].off + (int64_t)i * rects[r].ld + j] != 0.0) {
          f = 1;
          break;
        }
    flag[r] = f;
  }
}
void launch_add_squares(double* y, const double* V, int64_t ldv, int k, int64_t n, Stream) {
  for (int64_t i = 0; i < n; ++i) {
    double v = y[i];
    for (int j = 0; j < k; ++j) v += V[j * ldv + i] * V[j * ldv + i];
    y[i] = v;
  }
}
void launch_scal(double* y, double a, int64_t n, Stream) {
  for (int64_t i = 0; i < n; ++i) y[i] *= a;
}
void launch_copy(double* dst, const double* src, int64_t n, Stream) {
  if (n > 0) std::memmove(dst, src, (size_t)n * 8);
}
void launch_scale_rows(double* a, int rows, int cols, int ld, const double* s, Stream) {
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) a[(int64_t)r * ld + c] *= s[r];
}
void launch_scale_cols(double* a, int rows, int cols, int ld, const double* s, Stream) {
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) a[(int64_t)r * ld + c] *= s[c];
}

}  // namespace sadmrg
