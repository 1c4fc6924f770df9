// Device interface of libsadmrg: kernel launchers, the task records they
// consume, and the device-memory calls.  The host engine talks to the GPU only
// through this header.
#pragma once
#include <cstddef>
#include <cstdint>
#include <mutex>

namespace sadmrg {

using Stream = void*;  // hipStream_t

// ---------------------------------------------------------------------------
// Device memory (HIP runtime); failures throw through dev_fail().
// ---------------------------------------------------------------------------
void* dev_alloc(size_t bytes);
void dev_free(void* p);
// The raw calls under the pools (pool.cpp): a new device block or null, its
// release, and the free / total bytes of the current device (false when the
// runtime cannot tell).
void* dev_raw_alloc(size_t bytes);
void dev_raw_free(void* p);
bool dev_raw_meminfo(size_t* free_bytes, size_t* total_bytes);
// Per-context cache of device blocks (see kernels.hip); bind returns the
// previously bound pool.  Destroy only after the context's stream is idle.
struct DevPool;
// Caller-supplied allocator of a pool: alloc returns a device block of at
// least `bytes` on `device` (null on failure), free returns one.
using DevAllocFn = void* (*)(size_t bytes, int device, void* user);
using DevFreeFn = void (*)(void* ptr, size_t bytes, int device, void* user);
// false if the pool already owns blocks (they came from the other allocator)
bool dev_pool_set_allocator(DevPool* pool, DevAllocFn a, DevFreeFn f, void* user, int device);
DevPool* dev_pool_create();
void dev_pool_destroy(DevPool* pool);
DevPool* dev_pool_bind(DevPool* pool);
DevPool* dev_pool_current();  // the pool bound to the calling thread
void dev_h2d(void* dst, const void* src, size_t bytes, Stream st);
void dev_d2h(void* dst, const void* src, size_t bytes, Stream st);
void dev_d2d(void* dst, const void* src, size_t bytes, Stream st);
void dev_zero(void* p, size_t bytes, Stream st);  // fill kernel (no memset node)
void dev_sync(Stream st);
// Page-locked host memory and copies that do not wait for the stream: the
// host side must stay untouched until the stream has passed the copy.
void* host_alloc_pinned(size_t bytes);
void host_free_pinned(void* p);
void dev_h2d_async(void* dst, const void* pinned_src, size_t bytes, Stream st);
void dev_d2h_async(void* pinned_dst, const void* src, size_t bytes, Stream st);
void dev_set_device(int device);
int dev_get_device();  // the calling thread's current device
size_t dev_total_memory();  // bytes of device memory of the current device
void dev_memory_info(size_t* free_bytes, size_t* total_bytes);  // current device
int dev_count();
// event timing: returns an opaque event handle recorded on st
void* dev_event_record(Stream st);
double dev_event_elapsed(void* a, void* b);  // seconds, synchronises b
void dev_event_free(void* e);
void dev_event_wait(void* e);  // the host waits until the stream has passed e
// Streams of default priority; dev_stream_order(a, b): work enqueued on a
// from now on starts after the work already enqueued on b.
Stream dev_stream_create();
void dev_stream_destroy(Stream s);
void dev_stream_order(Stream a, Stream b);

// Static per-device workspace of the allocation-free sigma entry point.
// scratch_init(device) must run with that device current (context creation
// does it); scratch_ptr returns the device address it found (null before),
// scratch_lock a host mutex that serialises the entry point's calls on that
// device, scratch_bytes the array's size.
void scratch_init(int device);
void* scratch_ptr(int device);
std::mutex* scratch_lock(int device);
size_t scratch_bytes();

// Flags of a block triple product  out += coef * opA(A) * B * opC(C)  (the
// host evaluates it as two grouped GEMMs): transpose A / C, identity A / C.
enum : int { TT_TRANS_A = 1, TT_TRANS_C = 2, TT_IDENT_A = 4, TT_IDENT_C = 8, TT_TRANS_B = 16 };

// out[r*ld + c] += sum_{p < nparts} part[p*rows*cols + r*cols + c]  (fixed order)
struct RTile {
  double* out;
  const double* part;
  int ld, rows, cols, nparts;
};

// dst[rows x cols] (leading dim ld) = sum_s scale_s * src_s, where src_s is a
// (rows x cols) block, the transpose of a (cols x rows) block, or the identity.
enum : int { GS_NORMAL = 0, GS_TRANS = 1, GS_IDENT = 2 };

struct GatherDst {
  double* dst;
  int rows, cols, ld;
  int s0, s1;
};

struct GatherSrc {
  const double* src;
  int ld;
  int kind;
  double scale;
};

// Linear combinations of operators sharing one element layout:
//   out[e] = sum_entries coef * (adj ? fac[e] * in[perm[e]] : in[e]),  e < nnz
struct ComboOut {
  double* out;
  int64_t nnz;
  int i0, i1;         // input-entry range
  const int* perm;    // adjoint element map of the layout (may be null)
  const double* fac;  // adjoint factors of the layout (may be null)
};
struct ComboIn {
  const double* in;
  double coef;
  int adj;
};

// Diagonal of the effective Hamiltonian: out[r*cols + c] = sum coef * x[r*sx] * y[c*sy]
struct DiagTask {
  const double* x;  // null = identity (value 1)
  const double* y;
  int sx, sy;
  double coef;
};
struct DiagSec {
  double* out;
  int rows, cols;
  int t0, t1;
};

// One-sided Jacobi SVD of a (rows x cols, leading dim lda) matrix:
//   A = U diag(s) Vt,  r = min(rows, cols), s descending,
//   U (rows x r, ld r) and Vt (r x cols, ld cols) orthonormal; columns of the
//   long-side factor whose singular value vanishes are completed by
//   Gram-Schmidt.  work needs rows*cols + r*r + r doubles.
struct SvdJob {
  const double* a;
  int rows, cols, lda;
  double* u;
  double* s;
  double* vt;
  double* work;
};


// Grouped GEMM: each output tile (<= 64 x 64) gets
//   mode 0: out += sum_t coef_t * opA(A_t)[rows x K_t] * opB(B_t)[K_t x cols]
//   mode 1: out  = (same sum)        (when part == nullptr)
// or writes the sum to `part` (a partial of a split tile, reduced later).
// `a` / `b` point at the tile's first row / column.
enum : int { GT_TRANS_A = 1, GT_TRANS_B = 2 };
struct GTile {
  double* out;
  double* part;
  int ld, rows, cols, mode;
  int t0, t1;
};
struct GTask {
  const double* a;
  const double* b;
  int lda, ldb, K, flags;
  double coef;
};
// stream: workgroup g processes the tiles [wstart[g], wstart[g+1]) in order
// (nwg groups); otherwise workgroup g processes tile g (nwg = tile count,
// wstart unused).
// tag: 0 = sigma pass 1, 1 = sigma pass 2, 2 = other (separate kernel symbols for profiling)
// f32: operands, outputs and partial tiles are float arrays (the record
// pointers keep their double* type and are reinterpreted).
// bf3 (with f32): BF16x3 products on the FP32 data (hi*hi + hi*lo + lo*hi of
// the BF16 splits, FP32 accumulation).
// nx > 1: workgroups are ordered so that consecutive tiles (or ranges) run
// on one of nx XCDs (the dispatcher deals workgroups to the XCDs in turn);
// results do not depend on it.
// gate (device int, optional): the launch does nothing while *gate != 0
void launch_gemm(const GTile* tiles, const GTask* tasks, const int* wstart, int nwg, bool stream, int tag, bool f32,
                 Stream st, bool bf3 = false, int nx = 0, const int* gate = nullptr);
// Number of compute units of the current device.
int dev_cu_count();
void launch_reduce(const RTile* reds, int nred, bool f32, Stream st, const int* gate = nullptr);
// Several independent plans in one launch: plan s owns the workgroups
// [base[s], base[s+1]) of the grid (base ascending from 0, nwg in total) and
// reads its own records: tiles + tasks (+ wstart when stream) for the GEMM,
// reds for the reduction.  Both arrays live in device memory.
struct GSeg {
  const GTile* tiles;
  const GTask* tasks;
  const int* wstart;
  const RTile* reds;
  const int* gate;  // optional: the plan's workgroups do nothing while *gate != 0
};
void launch_gemm_seg(const GSeg* segs, const int* base, int nseg, int nwg, bool stream, bool f32, Stream st,
                     bool bf3 = false);
void launch_reduce_seg(const GSeg* segs, const int* base, int nseg, int nred, bool f32, Stream st);
// out[j] = sum_{r < n_j} p_j[r * (ld_j + 1)]  (traces of square sub-blocks)
struct TraceJob {
  const double* p;
  int n, ld;
};
void launch_traces(const TraceJob* jobs, int njobs, double* out, Stream st);
// dst[i] = (float)src[i] / (double)src[i], i < n
void launch_cvt_d2f(float* dst, const double* src, int64_t n, Stream st);
void launch_cvt_f2d(double* dst, const float* src, int64_t n, Stream st);
void launch_gather(const GatherDst* dsts, int ndst, const GatherSrc* srcs, Stream st);
void launch_combo(const ComboOut* outs, int nout, const ComboIn* ins, int64_t max_nnz, Stream st);
void launch_diag(const DiagSec* secs, int nsec, const DiagTask* tasks, Stream st);
// phase 0: the whole decomposition in one workgroup per job; 1: only the
// working copy for the block rounds; 2: only the outputs of a working copy
// the block rounds have orthogonalised.
void launch_svd(const SvdJob* jobs, int njobs, int max_short, Stream st, int phase = 0);
// Block rounds of the one-sided Jacobi sweep for larger jobs (after phase 1,
// before phase 2): job k owns workgroups [pair_base[k], pair_base[k+1]) (its
// svd_block_pairs), npairs in total, pair_base ascending from 0; round r of
// a sweep (svd_block_rounds of them for a job; later rounds leave it alone);
// flags[k] is set when the round rotated a significant pair of job k; jobs
// with active[k] == 0 are skipped.  A job fits when svd_block_fits (its
// blocks' columns of M and V in LDS).
bool svd_block_fits(int rows, int cols);
int svd_block_pairs(int rows, int cols);
int svd_block_rounds(int rows, int cols);
void launch_svd_block(const SvdJob* jobs, const int* pair_base, int njobs, int npairs, int round,
                      const int* active, int* flags, Stream st);
// Sign convention of singular vectors: for every column a of U (rows x r,
// leading dimension r) the entry of largest magnitude (lowest row among ties)
// is made positive; row a of Vt (r x cols, leading dimension cols) follows.
void launch_svd_signs(const SvdJob* jobs, int njobs, Stream st);

// Davidson helpers (device pointers; k <= 64)
// out[j] = dot(V + j*ldv, x) for j < k; deterministic two-stage reduction (partial: 256*k doubles)
void launch_dots(const double* V, int64_t ldv, int k, const double* x, int64_t n, double* out, double* partial,
                 Stream st);
// y = beta*y + alpha * sum_j coef[j] * V_j   (coef on device)
void launch_combo_vec(const double* V, int64_t ldv, int k, const double* coef, double alpha, int64_t n, double* y,
                      double beta, Stream st);
// r = ax - theta[0] * x
void launch_residual(const double* ax, const double* x, const double* theta, int64_t n, double* r, Stream st);
// t = r / (theta[0] - diag), denominator guarded away from zero
void launch_precond(const double* r, const double* diag, const double* theta, int64_t n, double* t, Stream st);
// y *= 1 / sqrt(nrm2[0])
void launch_normalize(double* y, const double* nrm2, int64_t n, Stream st);
// eigen-decomposition of a symmetric k x k matrix given by its lower triangle
// (leading dim ld), k <= 64: evals ascending, eigenvector j at evecs + j*k
void launch_syev_small(const double* H, int k, int ld, double* evals, double* evecs, Stream st);
// The Davidson helpers over job lists: one launch serves many independent
// solves, each job with the arithmetic of the single-solve call.
// out[j] = dot(V + j*ldv, x), j < k; part holds 256*k doubles
struct DotJob {
  const double* V;
  const double* x;
  double* out;
  double* part;
  int64_t ldv, n;
  int k;
};
void launch_dots_batch(const DotJob* jobs, int njobs, int max_k, Stream st);
// y = beta*y + alpha * sum_j coef[j] * V_j
struct ComboJob {
  const double* V;
  const double* coef;
  double* y;
  int64_t ldv, n;
  int k;
  double alpha, beta;
};
void launch_combo_batch(const ComboJob* jobs, int njobs, int64_t max_n, Stream st);
// element-wise, i < n:  COPY y = a;  ZERO y = 0;  RESIDUAL y = a - s[0] b;
// PRECOND y = a / (s[0] - b) (guarded as launch_precond);  NORMALIZE
// y *= 1/sqrt(s[0]);  D2F (float)y = a;  F2D y = (float)a
enum : int { EW_COPY = 0, EW_ZERO, EW_RESIDUAL, EW_PRECOND, EW_NORMALIZE, EW_D2F, EW_F2D };
struct EwJob {
  const double* a;
  const double* b;
  const double* s;
  double* y;
  int64_t n;
  int kind;
};
void launch_ew_batch(const EwJob* jobs, int njobs, int64_t max_n, Stream st);
struct SyevJob {
  const double* H;
  double* evals;
  double* evecs;
  int k, ld;
};
void launch_syev_batch(const SyevJob* jobs, int njobs, Stream st);
// ---- Davidson iterations as one fixed launch sequence (recorded once into a
// graph and replayed).  Each solve keeps its subspace size and flags in
// device memory; the kernels read them, so the same sequence serves every
// iteration, and a finished solve's kernels return at once.  Every kernel
// does exactly the arithmetic of the job-list helpers above.
struct DGState {
  int k;         // vectors in the subspace
  int it;        // iteration number
  int done;      // nonzero: the solve has finished
  int state;     // 1 converged, 2 out of iterations, 3 residual vanished
  int collapse;  // the preconditioned residual vanished: the residual is tried
  int restart;   // the subspace is full: restart from the Ritz vector
  int stall;     // reduced-precision floor: iterations without 10 % progress
  int pad;
  double rbest;  // best residual norm near the reduced-precision floor
  double pad2;
};
struct DGJob {
  DGState* s;
  double* V;  // ms vectors of length n (ld n)
  double* W;  // their sigma images
  double* Hs;  // projected matrix, lower triangle, ld ms
  double* evals;
  double* evecs;
  double* coef;
  double* nrm;   // |r|^2
  double* nrm2;  // |t|^2
  double* x;
  double* ax;
  double* r;
  double* t;
  double* part;  // 256 * ms partial sums
  const double* diag;
  double* in;         // the sigma input of the problem
  const double* out;  // and its output
  int64_t n;
  int ms, max_it, f32, pad;
  double tol, eps;
};
// scalar steps (one thread per solve)
enum : int { DG_TOP = 0, DG_CHECK, DG_COLLAPSE, DG_COLLAPSE2, DG_RESTART_FLAG, DG_RESTART_K, DG_ADVANCE };
// inner products
enum : int { DGD_ROW = 0, DGD_RR, DGD_VT, DGD_TT, DGD_V0W0, DGD_V0T };
// element-wise steps
enum : int { DGE_PRECOND = 0, DGE_COPY_RT, DGE_NORMALIZE_T, DGE_RESTART_COPY, DGE_APPEND, DGE_LOAD, DGE_STORE,
             DGE_RESIDUAL };
// linear combinations
enum : int { DGC_RITZ_X = 0, DGC_RITZ_AX, DGC_ORTH, DGC_ORTH0 };
// extra condition of a step: none, the collapse flag, the restart flag
enum : int { DG_GATE_NONE = 0, DG_GATE_COLLAPSE, DG_GATE_RESTART };
void launch_dg_scalar(const DGJob* jobs, int njobs, int which, Stream st);
void launch_dg_dots(const DGJob* jobs, int njobs, int which, int gate, int max_k, Stream st);
void launch_dg_ew(const DGJob* jobs, int njobs, int which, int gate, int64_t max_n, Stream st);
void launch_dg_combo(const DGJob* jobs, int njobs, int which, int gate, int64_t max_n, Stream st);
void launch_dg_syev(const DGJob* jobs, int njobs, Stream st);
// Stream capture into a graph and its replay
void dev_capture_begin(Stream st);
void* dev_capture_end(Stream st);  // instantiated graph
void dev_capture_abort(Stream st);  // ends a recording and drops it
void dev_graph_launch(void* exec, Stream st);
void dev_graph_free(void* exec);

// dst[i] = *src[i], i < n (src: device array of device pointers)
void launch_scalars(const double* const* src, int n, double* dst, Stream st);
// uniform [-1,1) numbers from the SplitMix64 counter generator
void launch_fill_uniform(double* p, int64_t n, uint64_t seed, uint64_t stream, Stream st);
// y[i] += a * x[i], i < n
void launch_axpy(double* y, const double* x, double a, int64_t n, Stream st);
// flag[r] = 1 if the (rows x cols, leading dim ld) sub-block at base + off
// holds a nonzero value, else 0, r < n
struct RectDesc {
  int64_t off;
  int rows, cols, ld;
};
void launch_rects_nonzero(const double* base, const RectDesc* rects, int n, unsigned char* flag, Stream st);
// y[i] += sum_{j < k} V[j * ldv + i]^2, i < n
void launch_add_squares(double* y, const double* V, int64_t ldv, int k, int64_t n, Stream st);
// y[i] *= a, i < n
void launch_scal(double* y, double a, int64_t n, Stream st);
// Plain streaming copy dst[i] = src[i] (reference kernel for HBM byte counters).
void launch_copy(double* dst, const double* src, int64_t n, Stream st);
// a[r][c] *= s[r]  /  a[r][c] *= s[c]
void launch_scale_rows(double* a, int rows, int cols, int ld, const double* s, Stream st);
void launch_scale_cols(double* a, int rows, int cols, int ld, const double* s, Stream st);

}  // namespace sadmrg
