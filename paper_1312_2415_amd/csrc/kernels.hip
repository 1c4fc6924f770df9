// HIP kernels for gfx950 (CDNA4, wave64).
//
// The hot contraction of the method -- the action of the effective two-site
// Hamiltonian and the renormalisation of block operators (paper, section
// "CheMPS2 library": the two OpenMP hot spots) -- is a sum of block triple
// products  coef * op(A) * B * op(C)  over symmetry-sector pairs.  The host
// evaluates them as two grouped GEMMs (gemm_kernel, FP64 matrix cores); split
// output tiles are combined by reduce_kernel in a fixed order, so every output
// element is written deterministically (no floating-point atomics).
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>

namespace sadmrg {

[[noreturn]] void dev_fail(const char* what);        // defined by the engine (throws)
[[noreturn]] void dev_fail_nomem(const char* what);  // same, as an out-of-memory error

static void hip_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    static thread_local char buf[512];
    snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
    dev_fail(buf);
  }
}

static void check_launch(const char* what) { hip_ok(hipGetLastError(), what); }

// ---------------------------------------------------------------------------
// Raw device memory for the context pools (pool.cpp).
// ---------------------------------------------------------------------------
void* dev_raw_alloc(size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}
void dev_raw_free(void* p) { (void)hipFree(p); }
bool dev_raw_meminfo(size_t* free_bytes, size_t* total_bytes) {
  if (hipMemGetInfo(free_bytes, total_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

void dev_h2d(void* dst, const void* src, size_t bytes, Stream st) {
  // uploads happen between kernels, never inside the sigma loop: synchronise so
  // that the host source may be released as soon as this returns
  if (bytes) hip_ok(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, (hipStream_t)st), "hipMemcpyAsync H2D");
  hip_ok(hipStreamSynchronize((hipStream_t)st), "hipStreamSynchronize");
}
void dev_d2h(void* dst, const void* src, size_t bytes, Stream st) {
  if (bytes) hip_ok(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, (hipStream_t)st), "hipMemcpyAsync D2H");
  hip_ok(hipStreamSynchronize((hipStream_t)st), "hipStreamSynchronize");
}
void dev_d2d(void* dst, const void* src, size_t bytes, Stream st) {
  if (!bytes) return;
  // whole doubles: a plain copy kernel (a fraction of the host cost of the
  // runtime's copy, which matters for the many short vector copies)
  if (bytes % 8 == 0 && (uintptr_t)dst % 8 == 0 && (uintptr_t)src % 8 == 0) {
    launch_copy((double*)dst, (const double*)src, (int64_t)(bytes / 8), st);
    return;
  }
  hip_ok(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)st), "hipMemcpyAsync D2D");
}
__global__ void zero_kernel(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}
void dev_zero(void* p, size_t bytes, Stream st) {
  const int64_t n = (int64_t)(bytes / 8);
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>(8192, (n + 255) / 256);
  hipLaunchKernelGGL(zero_kernel, dim3(nb), dim3(256), 0, (hipStream_t)st, (double*)p, n);
  check_launch("zero");
}
void dev_sync(Stream st) { hip_ok(hipStreamSynchronize((hipStream_t)st), "hipStreamSynchronize"); }
void* host_alloc_pinned(size_t bytes) {
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes ? bytes : 8, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    dev_fail("hipHostMalloc failed");
  }
  return p;
}
void host_free_pinned(void* p) {
  if (p) (void)hipHostFree(p);
}
void dev_h2d_async(void* dst, const void* src, size_t bytes, Stream st) {
  if (bytes) hip_ok(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, (hipStream_t)st), "hipMemcpyAsync H2D");
}
void dev_d2h_async(void* dst, const void* src, size_t bytes, Stream st) {
  if (bytes) hip_ok(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, (hipStream_t)st), "hipMemcpyAsync D2H");
}
void dev_set_device(int device) { hip_ok(hipSetDevice(device), "hipSetDevice"); }
int dev_get_device() {
  int d = 0;
  hip_ok(hipGetDevice(&d), "hipGetDevice");
  return d;
}
void dev_memory_info(size_t* fr, size_t* tot) { hip_ok(hipMemGetInfo(fr, tot), "hipMemGetInfo"); }
size_t dev_total_memory() {
  size_t fr = 0, tot = 0;
  hip_ok(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
  return tot;
}
int dev_count() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}
void* dev_event_record(Stream st) {
  hipEvent_t e;
  hip_ok(hipEventCreate(&e), "hipEventCreate");
  hip_ok(hipEventRecord(e, (hipStream_t)st), "hipEventRecord");
  return (void*)e;
}
double dev_event_elapsed(void* a, void* b) {
  hip_ok(hipEventSynchronize((hipEvent_t)b), "hipEventSynchronize");
  float ms = 0;
  hip_ok(hipEventElapsedTime(&ms, (hipEvent_t)a, (hipEvent_t)b), "hipEventElapsedTime");
  return ms * 1e-3;
}
void dev_event_free(void* e) {
  if (e) (void)hipEventDestroy((hipEvent_t)e);
}
void dev_event_wait(void* e) { hip_ok(hipEventSynchronize((hipEvent_t)e), "hipEventSynchronize"); }
Stream dev_stream_create() {
  hipStream_t s = nullptr;
  hip_ok(hipStreamCreate(&s), "hipStreamCreate");
  return (Stream)s;
}
void dev_stream_destroy(Stream s) {
  if (s) (void)hipStreamDestroy((hipStream_t)s);
}
void dev_stream_order(Stream a, Stream b) {
  if (a == b) return;
  hipEvent_t e;
  hip_ok(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
  hip_ok(hipEventRecord(e, (hipStream_t)b), "hipEventRecord");
  hip_ok(hipStreamWaitEvent((hipStream_t)a, e, 0), "hipStreamWaitEvent");
  (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------------------
// Static device workspace of the allocation-free sigma entry point
// (sadmrg_sigma_noalloc): one copy per device, held until the process ends.
// In host code the array's name is not a device address: scratch_init looks
// the address up once per device, with that device current, and every later
// use (kernel arguments, copies, fills) goes through the address it keeps.
// ---------------------------------------------------------------------------
static constexpr size_t SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;
static std::map<int, std::unique_ptr<std::mutex>> g_scratch_use;

void scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return;
  int cur = -1;
  hip_ok(hipGetDevice(&cur), "hipGetDevice");
  if (cur != device) dev_fail("scratch_init: the device is not current");
  void* p = nullptr;
  hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  if (!p) dev_fail("hipGetSymbolAddress(scratch) returned a null address");
  g_scratch_ptr[device] = p;
  g_scratch_use[device] = std::make_unique<std::mutex>();
}
void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}
std::mutex* scratch_lock(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_use.find(device);
  return it == g_scratch_use.end() ? nullptr : it->second.get();
}
size_t scratch_bytes() { return SCRATCH_BYTES; }

namespace {


}  // namespace

// ---------------------------------------------------------------------------
// FP64 matrix-core helper.  Lane layout of v_mfma_f64_16x16x4f64 (checked on
// gfx950): A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, D[i][j] in lane
// j + 16 (i % 4), register i / 4.
// ---------------------------------------------------------------------------
typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ inline d4_t mfma16(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}


// ---------------------------------------------------------------------------
// Grouped GEMM on the FP64 matrix cores.
//
// Output tiles of at most 64 x 64; a tile sums the products of its task range
// [t0, t1).  Workgroup g (4 wavefronts) processes the tiles
// [wstart[g], wstart[g+1]) in order, as one stream of (tile, task, k-chunk)
// items, so the loads of the next tile start while the current one is still
// being multiplied; the host balances the ranges by estimated cost.  Wave w
// owns rows [16w, 16w+16) of a tile as four 16 x 16 accumulator blocks.
// Items are staged through LDS in chunks of GK = 32 along K.  opA is kept in
// LDS as [row][k] and opB as [col][k] (row stride SLD doubles), so that every
// lane reads its MFMA operands for two k-steps with one 16-byte LDS read.
// The k index of the product is permuted inside a chunk (k-step pair p, lane
// group g, step parity e -> k = 8p + 2g + e), identically for both operands.
//
// Global loads are raw buffer loads whose descriptor covers exactly the bytes
// of the task's operand inside the tile (record count = extent), and every
// element's full byte offset goes into the vector offset, so the hardware
// range check returns zero for anything past the extent: rows/cols beyond a
// ragged tile edge and, for mn-contiguous storage, k beyond K.  For
// k-contiguous storage the last (ragged) chunk of a task masks k >= K
// explicitly.  Elements of rows (cols) beyond the tile that still fall inside
// the extent are real data of the operand; they only reach output rows
// (cols) that are never written.  The next chunk is loaded into registers
// while the current one is multiplied out of LDS (one LDS buffer of 34 KB:
// four workgroups per CU).  Task and tile records are read one ahead.
// ---------------------------------------------------------------------------
constexpr int GK = 32;
constexpr unsigned G_OOB = 0x80000000u;  // offset past every record count
constexpr int G_RSRC_W3 = 0x00020000;   // raw buffer, 32-bit data format

typedef unsigned int u2_t __attribute__((ext_vector_type(2)));
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// Element-type traits of the grouped GEMM.  SLD: LDS row stride in elements
// (16-byte aligned rows; 68 / 36 dwords = 4 mod 32 banks, so 16-byte reads of
// 8 consecutive lanes are conflict-free).  VEC: elements per 16-byte read =
// MFMA k-steps served by one read.  Accumulator row of (lane group lk,
// register r) in a 16 x 16 block: FP64 lk + 4r, FP32 4lk + r.
template <typename T>
struct GT;
template <>
struct GT<double> {
  static constexpr int SLD = 34, VEC = 2;
  typedef d2_t V;
  typedef d4_t Acc;
  __device__ static double load(__amdgpu_buffer_rsrc_t rs, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0));
  }
  __device__ static Acc mfma(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct GT<float> {
  static constexpr int SLD = 36, VEC = 4;
  typedef f4_t V;
  typedef f4_t Acc;
  __device__ static float load(__amdgpu_buffer_rsrc_t rs, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
  }
  __device__ static Acc mfma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lk, int r) { return 4 * lk + r; }
};

// Task records are read with a uniform index; the compiler cannot prove the
// loaded values uniform once LDS stores intervene, so every word is moved to
// a scalar register explicitly (buffer descriptors built from them must be
// scalar).
__device__ inline int g_u(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline uint64_t g_u64(uint64_t v) {
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return lo | (hi << 32);
}
__device__ inline GTask g_task(const GTask* __restrict__ tasks, int i) {
  const GTask t = tasks[i];
  GTask u;
  u.a = (const double*)g_u64((uint64_t)t.a);
  u.b = (const double*)g_u64((uint64_t)t.b);
  u.lda = g_u(t.lda);
  u.ldb = g_u(t.ldb);
  u.K = g_u(t.K);
  u.flags = g_u(t.flags);
  u.coef = __builtin_bit_cast(double, g_u64(__builtin_bit_cast(uint64_t, t.coef)));
  return u;
}

__device__ inline GTile g_tile(const GTile* __restrict__ tiles, int i) {
  const GTile t = tiles[i];
  GTile u;
  u.out = (double*)g_u64((uint64_t)t.out);
  u.part = (double*)g_u64((uint64_t)t.part);
  u.ld = g_u(t.ld);
  u.rows = g_u(t.rows);
  u.cols = g_u(t.cols);
  u.mode = g_u(t.mode);
  u.t0 = g_u(t.t0);
  u.t1 = g_u(t.t1);
  return u;
}

// One operand of the current task.  k-fast storage (contiguous along k: opA
// not transposed, opB transposed): thread element q is (mn, k) =
// (tid/32 + 8q, tid%32); mn-fast storage: (tid%64, tid/64 + 4q).  Record
// pointers are typed double* on the host; the element type T of the launch
// decides how they are read.
struct GOp {
  __amdgpu_buffer_rsrc_t rs;
  unsigned base;   // byte offset of element q = 0 at k0 = 0 (per thread)
  unsigned qstep;  // byte step between elements q and q+1 (uniform)
  unsigned kstep;  // byte step per unit of k0 (uniform)
  bool kfast;
};

template <typename T>
__device__ inline void g_op(GOp& o, const double* ptr, int ld, bool kfast, int ext, int K, int tid) {
  constexpr unsigned ES = sizeof(T);
  const int nrec = (kfast ? (ext - 1) * ld + K : (K - 1) * ld + ext) * (int)ES;
  o.rs = __builtin_amdgcn_make_buffer_rsrc((void*)ptr, (short)0, nrec, G_RSRC_W3);
  o.kfast = kfast;
  o.base = kfast ? (unsigned)((tid / 32) * ld + tid % 32) * ES : (unsigned)((tid / 64) * ld + tid % 64) * ES;
  o.qstep = kfast ? (unsigned)ld * 8u * ES : (unsigned)ld * 4u * ES;
  o.kstep = kfast ? ES : (unsigned)ld * ES;
}

template <typename T>
__device__ inline void g_fetch(T (&r)[8], const GOp& o, int k0, int K, int tid) {
  unsigned b = o.base;
  if (o.kfast && k0 + GK > K && k0 + tid % 32 >= K) b = G_OOB;
  const unsigned adv = (unsigned)k0 * o.kstep;
#pragma unroll
  for (int q = 0; q < 8; ++q) r[q] = GT<T>::load(o.rs, b + (q * o.qstep + adv));
}

// LDS position of element q: [mn][k] with row stride SLD.
template <typename T>
__device__ inline int g_lds(bool kfast, int tid, int q) {
  constexpr int SLD = GT<T>::SLD;
  return kfast ? (tid / 32 + 8 * q) * SLD + tid % 32 : (tid % 64) * SLD + tid / 64 + 4 * q;
}

template <typename T>
__device__ inline void g_store(const T (&ra)[8], const T (&rb)[8], double coef, int flags, T* sA, T* sB, int tid) {
  const bool kfa = !(flags & GT_TRANS_A), kfb = (flags & GT_TRANS_B) != 0;
  const T c = (T)coef;
  if (kfa) {
#pragma unroll
    for (int q = 0; q < 8; ++q) sA[g_lds<T>(true, tid, q)] = c * ra[q];
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) sA[g_lds<T>(false, tid, q)] = c * ra[q];
  }
  if (kfb) {
#pragma unroll
    for (int q = 0; q < 8; ++q) sB[g_lds<T>(true, tid, q)] = rb[q];
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) sB[g_lds<T>(false, tid, q)] = rb[q];
  }
}

// acc[b] += A[16 rows][k] * B[k][16b .. 16b+15], b < NCB, over the first np
// groups of 4*VEC values of k of the staged chunk.  Inside a group, lane
// group lk reads VEC consecutive k with one 16-byte read and feeds them to
// VEC successive MFMA k-steps (k = 4*VEC*p + VEC*lk + e), for both operands.
template <typename T, int NCB>
__device__ inline void g_mac(typename GT<T>::Acc (&acc)[4], const T* sA, const T* sB, int np, int r0, int li, int lk) {
  typedef typename GT<T>::V V;
  constexpr int SLD = GT<T>::SLD, VEC = GT<T>::VEC;
  const T* pa = sA + (r0 + li) * SLD + VEC * lk;
  const T* pb = sB + li * SLD + VEC * lk;
  for (int p = 0; p < np; ++p) {
    const V av = *(const V*)(pa + 4 * VEC * p);
    V bv[NCB];
#pragma unroll
    for (int b = 0; b < NCB; ++b) bv[b] = *(const V*)(pb + 16 * b * SLD + 4 * VEC * p);
#pragma unroll
    for (int e = 0; e < VEC; ++e)
#pragma unroll
      for (int b = 0; b < NCB; ++b) acc[b] = GT<T>::mfma(av[e], bv[b][e], acc[b]);
  }
}

template <typename T>
__device__ inline void g_mac_any(typename GT<T>::Acc (&acc)[4], const T* sA, const T* sB, int kc, int ncb, int r0,
                                 int li, int lk) {
  const int np = (kc + 4 * GT<T>::VEC - 1) / (4 * GT<T>::VEC);
  if (ncb == 4)
    g_mac<T, 4>(acc, sA, sB, np, r0, li, lk);
  else if (ncb == 3)
    g_mac<T, 3>(acc, sA, sB, np, r0, li, lk);
  else if (ncb == 2)
    g_mac<T, 2>(acc, sA, sB, np, r0, li, lk);
  else
    g_mac<T, 1>(acc, sA, sB, np, r0, li, lk);
}

// BF16x3 products on FP32 data: every staged value x is split at the LDS
// store into hi = bf16(x) and lo = bf16(x - hi) (round to nearest; x = hi +
// lo to about 2^-17 |x|), and a product is hi*hi + hi*lo + lo*hi (the lo*lo
// term, about 2^-16 of it, is dropped) with FP32 accumulation, on the
// 16x16x32 BF16 MFMA.  The four LDS planes (A hi, A lo, B hi, B lo) are
// [mn][k] with row stride SLDB; lane group lk feeds k = 8 lk .. 8 lk + 7 of
// a chunk to the MFMA, the same k slots for both operands.
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
constexpr int SLDB = 40;                // bf16 row stride (80 B: 16-byte aligned rows)
constexpr int BF_PLANE = 64 * SLDB;     // elements of one plane
__device__ inline int g_lds_bf(bool kfast, int tid, int q) {
  return kfast ? (tid / 32 + 8 * q) * SLDB + tid % 32 : (tid % 64) * SLDB + tid / 64 + 4 * q;
}
__device__ inline void g_store_bf3(const float (&ra)[8], const float (&rb)[8], double coef, int flags, __bf16* sH,
                                   int tid) {
  const bool kfa = !(flags & GT_TRANS_A), kfb = (flags & GT_TRANS_B) != 0;
  const float c = (float)coef;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float a = c * ra[q], b = rb[q];
    const __bf16 ah = (__bf16)a, bh = (__bf16)b;
    const int ia = g_lds_bf(kfa, tid, q), ib = g_lds_bf(kfb, tid, q);
    sH[ia] = ah;
    sH[BF_PLANE + ia] = (__bf16)(a - (float)ah);
    sH[2 * BF_PLANE + ib] = bh;
    sH[3 * BF_PLANE + ib] = (__bf16)(b - (float)bh);
  }
}
template <int NCB>
__device__ inline void g_mac_bf3(f4_t (&acc)[4], const __bf16* sH, int r0, int li, int lk) {
  const int oa = (r0 + li) * SLDB + 8 * lk;
  const bf8_t ah = *(const bf8_t*)(sH + oa), al = *(const bf8_t*)(sH + BF_PLANE + oa);
#pragma unroll
  for (int b = 0; b < NCB; ++b) {
    const int ob = (li + 16 * b) * SLDB + 8 * lk;
    const bf8_t bh = *(const bf8_t*)(sH + 2 * BF_PLANE + ob), bl = *(const bf8_t*)(sH + 3 * BF_PLANE + ob);
    acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[b], 0, 0, 0);
    acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[b], 0, 0, 0);
    acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[b], 0, 0, 0);
  }
}
__device__ inline void g_mac_bf3_any(f4_t (&acc)[4], const __bf16* sH, int ncb, int r0, int li, int lk) {
  if (ncb == 4)
    g_mac_bf3<4>(acc, sH, r0, li, lk);
  else if (ncb == 3)
    g_mac_bf3<3>(acc, sH, r0, li, lk);
  else if (ncb == 2)
    g_mac_bf3<2>(acc, sH, r0, li, lk);
  else
    g_mac_bf3<1>(acc, sH, r0, li, lk);
}

struct GOut {  // what the epilogue of a tile needs
  double* out;
  double* part;
  int ld, rows, cols, mode;
};
__device__ inline GOut g_out(const GTile& t) { return GOut{t.out, t.part, t.ld, t.rows, t.cols, t.mode}; }

template <typename T>
__device__ inline void g_write(const GOut& tile, const typename GT<T>::Acc (&acc)[4], int r0, int li, int lk) {
  T* const out = (T*)tile.out;
  T* const part = (T*)tile.part;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int col = 16 * b + li;
    if (col >= tile.cols) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int orow = r0 + GT<T>::row(lk, r);
      if (orow >= tile.rows) continue;
      if (part)
        part[orow * tile.cols + col] = acc[b][r];
      else if (tile.mode == 1)
        out[(int64_t)orow * tile.ld + col] = acc[b][r];
      else
        out[(int64_t)orow * tile.ld + col] += acc[b][r];
    }
  }
}

// Workgroup order across the XCDs.  The dispatcher hands consecutive
// workgroups of a launch to the XCDs in turn (workgroup b to XCD b mod nx),
// and each XCD has its own L2.  With nx > 1 workgroup b takes item
// start(x) + b / nx with x = b mod nx, where XCD x owns the contiguous items
// [start(x), start(x+1)) of an even split: consecutive items (the tiles of
// one product, which share operand panels) then run on one XCD, close in
// time.  A bijection of [0, n) for any n.
__device__ __forceinline__ unsigned xcd_item(unsigned b, unsigned n, int nx) {
  if (nx <= 1) return b;
  const unsigned q = n / (unsigned)nx, r = n % (unsigned)nx, x = b % (unsigned)nx, j = b / (unsigned)nx;
  return x * q + min(x, r) + j;
}

// One tile per workgroup (blockIdx.x = tile), no state carried between tiles:
// the hardware dispatcher balances short, independent tiles best.
// TAG only separates the symbols of the launch sites for profiling:
// 0 = sigma pass 1, 1 = sigma pass 2, 2 = renormalisation / other products.
template <typename T, bool BF3 = false>
__device__ __forceinline__ void gemm_tile_body(const GTile* __restrict__ tiles, const GTask* __restrict__ tasks,
                                               const unsigned bid) {
  typedef typename GT<T>::Acc Acc;
  static_assert(!BF3 || sizeof(T) == 4, "BF16x3 products take FP32 data");
  __shared__ __attribute__((aligned(16))) T sA[BF3 ? 4 : 64 * GT<T>::SLD];
  __shared__ __attribute__((aligned(16))) T sB[BF3 ? 4 : 64 * GT<T>::SLD];
  __shared__ __attribute__((aligned(16))) __bf16 sH[BF3 ? 4 * BF_PLANE : 8];
  const GTile tile = tiles[bid];
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid / 64);  // wave index, scalar
  const int l = tid % 64;
  const int li = l % 16, lk = l / 16;
  const int r0 = 16 * w;
  const bool active = r0 < tile.rows;
  const int ncb = (tile.cols + 15) / 16;
  Acc acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = (Acc){0, 0, 0, 0};

  if (tile.t0 < tile.t1) {
    int t = tile.t0, k0 = 0;  // stream position of the next fetch
    GTask cur = g_task(tasks, t);
    GTask nxt = t + 1 < tile.t1 ? g_task(tasks, t + 1) : cur;
    GOp A, B;
    g_op<T>(A, cur.a, cur.lda, !(cur.flags & GT_TRANS_A), tile.rows, cur.K, tid);
    g_op<T>(B, cur.b, cur.ldb, (cur.flags & GT_TRANS_B) != 0, tile.cols, cur.K, tid);
    T ra[8], rb[8];
    int kc, flags;
    double coef;
    auto next = [&]() {
      g_fetch<T>(ra, A, k0, cur.K, tid);
      g_fetch<T>(rb, B, k0, cur.K, tid);
      kc = min(GK, cur.K - k0);
      coef = cur.coef;
      flags = cur.flags;
      k0 += GK;
      if (k0 >= cur.K) {
        k0 = 0;
        if (++t < tile.t1) {
          cur = nxt;
          if (t + 1 < tile.t1) nxt = g_task(tasks, t + 1);
          g_op<T>(A, cur.a, cur.lda, !(cur.flags & GT_TRANS_A), tile.rows, cur.K, tid);
          g_op<T>(B, cur.b, cur.ldb, (cur.flags & GT_TRANS_B) != 0, tile.cols, cur.K, tid);
        }
      }
    };
    next();
    while (true) {
      if constexpr (BF3)
        g_store_bf3(ra, rb, coef, flags, sH, tid);
      else
        g_store<T>(ra, rb, coef, flags, sA, sB, tid);
      const int np = (kc + 4 * GT<T>::VEC - 1) / (4 * GT<T>::VEC);
      __syncthreads();
      const bool more = t < tile.t1;
      if (more) next();
      if constexpr (BF3) {
        if (active) g_mac_bf3_any(acc, sH, ncb, r0, li, lk);
      } else if (active) {
        if (ncb == 4)
          g_mac<T, 4>(acc, sA, sB, np, r0, li, lk);
        else if (ncb == 3)
          g_mac<T, 3>(acc, sA, sB, np, r0, li, lk);
        else if (ncb == 2)
          g_mac<T, 2>(acc, sA, sB, np, r0, li, lk);
        else
          g_mac<T, 1>(acc, sA, sB, np, r0, li, lk);
      }
      if (!more) break;
      __syncthreads();
    }
  }
  if (active) g_write<T>(g_out(tile), acc, r0, li, lk);
}

// gate: when given and nonzero the launch does nothing (a finished solve in a
// recorded Davidson sequence)
template <typename T, int TAG>
__global__ __launch_bounds__(256, 4) void gemm_tile_kernel(const GTile* __restrict__ tiles,
                                                           const GTask* __restrict__ tasks, int nx,
                                                           const int* __restrict__ gate) {
  if (gate && *gate) return;
  gemm_tile_body<T>(tiles, tasks, xcd_item(blockIdx.x, gridDim.x, nx));
}
// the same with BF16x3 products on FP32 data
template <int TAG>
__global__ __launch_bounds__(256, 4) void gemm_tile_bf3_kernel(const GTile* __restrict__ tiles,
                                                               const GTask* __restrict__ tasks, int nx,
                                                               const int* __restrict__ gate) {
  if (gate && *gate) return;
  gemm_tile_body<float, true>(tiles, tasks, xcd_item(blockIdx.x, gridDim.x, nx));
}

// Workgroup g streams the tiles [wstart[g], wstart[g+1]).
// TAG only separates the symbols of the launch sites for profiling:
// 0 = sigma pass 1, 1 = sigma pass 2, 2 = renormalisation / other products.
template <typename T, bool BF3 = false>
__device__ __forceinline__ void gemm_stream_body(const GTile* __restrict__ tiles, const GTask* __restrict__ tasks,
                                                 const int* __restrict__ wstart, const unsigned bid) {
  typedef typename GT<T>::Acc Acc;
  static_assert(!BF3 || sizeof(T) == 4, "BF16x3 products take FP32 data");
  __shared__ __attribute__((aligned(16))) T sA[BF3 ? 4 : 64 * GT<T>::SLD];
  __shared__ __attribute__((aligned(16))) T sB[BF3 ? 4 : 64 * GT<T>::SLD];
  __shared__ __attribute__((aligned(16))) __bf16 sH[BF3 ? 4 * BF_PLANE : 8];
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid / 64);  // wave index, scalar
  const int l = tid % 64;
  const int li = l % 16, lk = l / 16;
  const int r0 = 16 * w;
  int ft = wstart[bid];
  const int fe = wstart[bid + 1];
  if (ft >= fe) return;

  // fetch side: tile ft (record FT), task t (record cur) at chunk k0; the
  // next task of the tile (nxt), the next tile (NT) and its first task (ncur)
  GTile FT = g_tile(tiles, ft);
  GTile NT = ft + 1 < fe ? g_tile(tiles, ft + 1) : FT;
  int t = FT.t0, k0 = 0;
  GTask cur{}, nxt{}, ncur{};
  GOp A, B;
  if (FT.t0 < FT.t1) {
    cur = g_task(tasks, t);
    nxt = t + 1 < FT.t1 ? g_task(tasks, t + 1) : cur;
    g_op<T>(A, cur.a, cur.lda, !(cur.flags & GT_TRANS_A), FT.rows, cur.K, tid);
    g_op<T>(B, cur.b, cur.ldb, (cur.flags & GT_TRANS_B) != 0, FT.cols, cur.K, tid);
  }
  if (ft + 1 < fe && NT.t0 < NT.t1) ncur = g_task(tasks, NT.t0);

  // the staged item: registers + description
  T ra[8], rb[8];
  GOut MT;  // tile of the staged item
  int kc, flags;
  bool last;
  double coef;
  auto issue = [&]() {
    MT = g_out(FT);
    if (t < FT.t1) {
      g_fetch<T>(ra, A, k0, cur.K, tid);
      g_fetch<T>(rb, B, k0, cur.K, tid);
      kc = min(GK, cur.K - k0);
      coef = cur.coef;
      flags = cur.flags;
      k0 += GK;
      if (k0 >= cur.K) {
        k0 = 0;
        if (++t < FT.t1) {
          cur = nxt;
          if (t + 1 < FT.t1) nxt = g_task(tasks, t + 1);
          g_op<T>(A, cur.a, cur.lda, !(cur.flags & GT_TRANS_A), FT.rows, cur.K, tid);
          g_op<T>(B, cur.b, cur.ldb, (cur.flags & GT_TRANS_B) != 0, FT.cols, cur.K, tid);
        }
      }
    } else {  // a tile without products: its output is written as zero
      kc = 0;
      coef = 0.0;
      flags = 0;
    }
    last = t >= FT.t1;
    if (last && ++ft < fe) {
      FT = NT;
      t = FT.t0;
      k0 = 0;
      if (t < FT.t1) {
        cur = ncur;
        nxt = t + 1 < FT.t1 ? g_task(tasks, t + 1) : cur;
        g_op<T>(A, cur.a, cur.lda, !(cur.flags & GT_TRANS_A), FT.rows, cur.K, tid);
        g_op<T>(B, cur.b, cur.ldb, (cur.flags & GT_TRANS_B) != 0, FT.cols, cur.K, tid);
      }
      if (ft + 1 < fe) {
        NT = g_tile(tiles, ft + 1);
        if (NT.t0 < NT.t1) ncur = g_task(tasks, NT.t0);
      }
    }
  };

  Acc acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = (Acc){0, 0, 0, 0};
  issue();
  while (true) {
    if (kc > 0) {
      if constexpr (BF3)
        g_store_bf3(ra, rb, coef, flags, sH, tid);
      else
        g_store<T>(ra, rb, coef, flags, sA, sB, tid);
    }
    const GOut mt = MT;
    const int kcc = kc;
    const bool mlast = last;
    __syncthreads();
    const bool more = ft < fe;
    if (more) issue();
    const bool active = r0 < mt.rows;
    if constexpr (BF3) {
      if (active && kcc > 0) g_mac_bf3_any(acc, sH, (mt.cols + 15) / 16, r0, li, lk);
    } else {
      if (active && kcc > 0) g_mac_any<T>(acc, sA, sB, kcc, (mt.cols + 15) / 16, r0, li, lk);
    }
    if (mlast) {
      if (active) g_write<T>(mt, acc, r0, li, lk);
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = (Acc){0, 0, 0, 0};
    }
    if (!more) break;
    __syncthreads();
  }
}

template <typename T, int TAG>
__global__ __launch_bounds__(256, 3) void gemm_stream_kernel(const GTile* __restrict__ tiles,
                                                             const GTask* __restrict__ tasks,
                                                             const int* __restrict__ wstart, int nx,
                                                             const int* __restrict__ gate) {
  if (gate && *gate) return;
  gemm_stream_body<T>(tiles, tasks, wstart, xcd_item(blockIdx.x, gridDim.x, nx));
}
template <int TAG>
__global__ __launch_bounds__(256, 3) void gemm_stream_bf3_kernel(const GTile* __restrict__ tiles,
                                                                 const GTask* __restrict__ tasks,
                                                                 const int* __restrict__ wstart, int nx,
                                                                 const int* __restrict__ gate) {
  if (gate && *gate) return;
  gemm_stream_body<float, true>(tiles, tasks, wstart, xcd_item(blockIdx.x, gridDim.x, nx));
}

// Several plans in one launch (independent problems batched together): plan s
// owns the workgroups [base[s], base[s+1]), base ascending from 0.  Every
// wavefront finds its plan with one vector load and a ballot per 64 plans.
__device__ __forceinline__ int seg_find(const int* __restrict__ base, const int nseg, const int bid) {
  const int lane = threadIdx.x % 64;
  int s = 0;
  for (int c = 0; c < nseg; c += 64) {
    const int j = c + lane;
    const bool le = j < nseg && base[j] <= bid;
    const unsigned long long m = __ballot(le);
    s += __popcll(m);
    if (m != ~0ull) break;
  }
  return __builtin_amdgcn_readfirstlane(s - 1);
}

// The descriptor as the kernels read it: record pointers typed as global
// memory, so that their loads stay scalar as for kernel-argument pointers.
#define G_GLOBAL __attribute__((address_space(1)))
struct GSegDev {
  const G_GLOBAL GTile* tiles;
  const G_GLOBAL GTask* tasks;
  const G_GLOBAL int* wstart;
  const G_GLOBAL RTile* reds;
  const G_GLOBAL int* gate;
};
static_assert(sizeof(GSegDev) == sizeof(GSeg), "descriptor layout");

template <typename T, bool BF3>
__device__ __forceinline__ void gemm_tile_seg_body(const GSeg* __restrict__ segs,
                                                               const int* __restrict__ base, int nseg) {
  const int s = seg_find(base, nseg, blockIdx.x);
  const GSegDev* const d = (const GSegDev*)segs;
  if (d[s].gate && *d[s].gate) return;
  gemm_tile_body<T, BF3>((const GTile*)d[s].tiles, (const GTask*)d[s].tasks, blockIdx.x - base[s]);
}

template <typename T, bool BF3>
__device__ __forceinline__ void gemm_stream_seg_body(const GSeg* __restrict__ segs,
                                                                 const int* __restrict__ base, int nseg) {
  const int s = seg_find(base, nseg, blockIdx.x);
  const GSegDev* const d = (const GSegDev*)segs;
  if (d[s].gate && *d[s].gate) return;
  gemm_stream_body<T, BF3>((const GTile*)d[s].tiles, (const GTask*)d[s].tasks, (const int*)d[s].wstart,
                      blockIdx.x - base[s]);
}

template <typename T>
__global__ __launch_bounds__(256, 4) void gemm_tile_seg_kernel(const GSeg* __restrict__ segs,
                                                               const int* __restrict__ base, int nseg) {
  gemm_tile_seg_body<T, false>(segs, base, nseg);
}
__global__ __launch_bounds__(256, 4) void gemm_tile_seg_bf3_kernel(const GSeg* __restrict__ segs,
                                                                   const int* __restrict__ base, int nseg) {
  gemm_tile_seg_body<float, true>(segs, base, nseg);
}
template <typename T>
__global__ __launch_bounds__(256, 3) void gemm_stream_seg_kernel(const GSeg* __restrict__ segs,
                                                                 const int* __restrict__ base, int nseg) {
  gemm_stream_seg_body<T, false>(segs, base, nseg);
}
__global__ __launch_bounds__(256, 3) void gemm_stream_seg_bf3_kernel(const GSeg* __restrict__ segs,
                                                                     const int* __restrict__ base, int nseg) {
  gemm_stream_seg_body<float, true>(segs, base, nseg);
}

template <typename T>
static void launch_gemm_t(const GTile* tiles, const GTask* tasks, const int* wstart, int nwg, bool stream, int tag,
                          hipStream_t hs, int nx, const int* gate) {
  if (stream) {
    if (tag == 0)
      hipLaunchKernelGGL((gemm_stream_kernel<T, 0>), dim3(nwg), dim3(256), 0, hs, tiles, tasks, wstart, nx, gate);
    else if (tag == 1)
      hipLaunchKernelGGL((gemm_stream_kernel<T, 1>), dim3(nwg), dim3(256), 0, hs, tiles, tasks, wstart, nx, gate);
    else
      hipLaunchKernelGGL((gemm_stream_kernel<T, 2>), dim3(nwg), dim3(256), 0, hs, tiles, tasks, wstart, nx, gate);
  } else {
    if (tag == 0)
      hipLaunchKernelGGL((gemm_tile_kernel<T, 0>), dim3(nwg), dim3(256), 0, hs, tiles, tasks, nx, gate);
    else if (tag == 1)
      hipLaunchKernelGGL((gemm_tile_kernel<T, 1>), dim3(nwg), dim3(256), 0, hs, tiles, tasks, nx, gate);
    else
      hipLaunchKernelGGL((gemm_tile_kernel<T, 2>), dim3(nwg), dim3(256), 0, hs, tiles, tasks, nx, gate);
  }
}
static void launch_gemm_bf3(const GTile* tiles, const GTask* tasks, const int* wstart, int nwg, bool stream, int tag,
                            hipStream_t hs, int nx, const int* gate) {
  if (stream) {
    if (tag == 0)
      hipLaunchKernelGGL((gemm_stream_bf3_kernel<0>), dim3(nwg), dim3(256), 0, hs, tiles, tasks, wstart, nx, gate);
    else if (tag == 1)
      hipLaunchKernelGGL((gemm_stream_bf3_kernel<1>), dim3(nwg), dim3(256), 0, hs, tiles, tasks, wstart, nx, gate);
    else
      hipLaunchKernelGGL((gemm_stream_bf3_kernel<2>), dim3(nwg), dim3(256), 0, hs, tiles, tasks, wstart, nx, gate);
  } else {
    if (tag == 0)
      hipLaunchKernelGGL((gemm_tile_bf3_kernel<0>), dim3(nwg), dim3(256), 0, hs, tiles, tasks, nx, gate);
    else if (tag == 1)
      hipLaunchKernelGGL((gemm_tile_bf3_kernel<1>), dim3(nwg), dim3(256), 0, hs, tiles, tasks, nx, gate);
    else
      hipLaunchKernelGGL((gemm_tile_bf3_kernel<2>), dim3(nwg), dim3(256), 0, hs, tiles, tasks, nx, gate);
  }
}

void launch_gemm(const GTile* tiles, const GTask* tasks, const int* wstart, int nwg, bool stream, int tag, bool f32,
                 Stream st, bool bf3, int nx, const int* gate) {
  if (nwg <= 0) return;
  if (f32 && bf3)
    launch_gemm_bf3(tiles, tasks, wstart, nwg, stream, tag, (hipStream_t)st, nx, gate);
  else if (f32)
    launch_gemm_t<float>(tiles, tasks, wstart, nwg, stream, tag, (hipStream_t)st, nx, gate);
  else
    launch_gemm_t<double>(tiles, tasks, wstart, nwg, stream, tag, (hipStream_t)st, nx, gate);
  check_launch("gemm");
}

void launch_gemm_seg(const GSeg* segs, const int* base, int nseg, int nwg, bool stream, bool f32, Stream st,
                     bool bf3) {
  if (nwg <= 0 || nseg <= 0) return;
  const hipStream_t hs = (hipStream_t)st;
  if (f32 && bf3) {
    if (stream)
      hipLaunchKernelGGL(gemm_stream_seg_bf3_kernel, dim3(nwg), dim3(256), 0, hs, segs, base, nseg);
    else
      hipLaunchKernelGGL(gemm_tile_seg_bf3_kernel, dim3(nwg), dim3(256), 0, hs, segs, base, nseg);
    check_launch("gemm_seg");
    return;
  }
  if (stream) {
    if (f32)
      hipLaunchKernelGGL(gemm_stream_seg_kernel<float>, dim3(nwg), dim3(256), 0, hs, segs, base, nseg);
    else
      hipLaunchKernelGGL(gemm_stream_seg_kernel<double>, dim3(nwg), dim3(256), 0, hs, segs, base, nseg);
  } else {
    if (f32)
      hipLaunchKernelGGL(gemm_tile_seg_kernel<float>, dim3(nwg), dim3(256), 0, hs, segs, base, nseg);
    else
      hipLaunchKernelGGL(gemm_tile_seg_kernel<double>, dim3(nwg), dim3(256), 0, hs, segs, base, nseg);
  }
  check_launch("gemm_seg");
}

int dev_cu_count() {
  int dev = 0, n = 0;
  hip_ok(hipGetDevice(&dev), "hipGetDevice");
  hip_ok(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
  return n;
}

// Ordered sum of a tile's partial results: eight interleaved accumulators
// keep loads in flight; the combination order is fixed, so results are
// reproducible run to run.  A tile (at most 64 x 64) is shared by
// REDUCE_SPLIT workgroups, each summing every REDUCE_SPLIT-th run of 256
// elements.
constexpr int REDUCE_SPLIT = 4;
template <typename T>
__device__ __forceinline__ void reduce_body(const RTile* __restrict__ reds, const unsigned bid) {
  const RTile t = reds[bid];
  const T* const part = (const T*)t.part;
  T* const out = (T*)t.out;
  const int n = t.rows * t.cols;
  // blockIdx.y takes every gridDim.y-th run of 256 elements of the tile
  for (int e = blockIdx.y * 256 + threadIdx.x; e < n; e += 256 * gridDim.y) {
    T v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const T* p = part + e;
    int q = 0;
    for (; q + 8 <= t.nparts; q += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] += p[(int64_t)(q + u) * n];
    }
    for (int u = 0; q < t.nparts; ++q, ++u) v[u] += p[(int64_t)q * n];
    const T s = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    out[(int64_t)(e / t.cols) * t.ld + e % t.cols] += s;
  }
}
template <typename T>
__global__ __launch_bounds__(256) void reduce_kernel(const RTile* __restrict__ reds, const int* __restrict__ gate) {
  if (gate && *gate) return;
  reduce_body<T>(reds, blockIdx.x);
}
template <typename T>
__global__ __launch_bounds__(256) void reduce_seg_kernel(const GSeg* __restrict__ segs, const int* __restrict__ base,
                                                         int nseg) {
  const int s = seg_find(base, nseg, blockIdx.x);
  const GSegDev* const d = (const GSegDev*)segs;
  if (d[s].gate && *d[s].gate) return;
  reduce_body<T>((const RTile*)d[s].reds, blockIdx.x - base[s]);
}

void launch_reduce(const RTile* reds, int nred, bool f32, Stream st, const int* gate) {
  if (nred <= 0) return;
  if (f32)
    hipLaunchKernelGGL(reduce_kernel<float>, dim3(nred, REDUCE_SPLIT), dim3(256), 0, (hipStream_t)st, reds, gate);
  else
    hipLaunchKernelGGL(reduce_kernel<double>, dim3(nred, REDUCE_SPLIT), dim3(256), 0, (hipStream_t)st, reds, gate);
  check_launch("reduce");
}

void launch_reduce_seg(const GSeg* segs, const int* base, int nseg, int nred, bool f32, Stream st) {
  if (nred <= 0 || nseg <= 0) return;
  if (f32)
    hipLaunchKernelGGL(reduce_seg_kernel<float>, dim3(nred, REDUCE_SPLIT), dim3(256), 0, (hipStream_t)st, segs, base,
                       nseg);
  else
    hipLaunchKernelGGL(reduce_seg_kernel<double>, dim3(nred, REDUCE_SPLIT), dim3(256), 0, (hipStream_t)st, segs, base,
                       nseg);
  check_launch("reduce_seg");
}

// ---------------------------------------------------------------------------
// Traces of square sub-blocks: one workgroup per job, fixed-order reduction.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void traces_kernel(const TraceJob* __restrict__ jobs, double* __restrict__ out) {
  const TraceJob j = jobs[blockIdx.x];
  __shared__ double red[256];
  double v = 0.0;
  for (int r = threadIdx.x; r < j.n; r += 256) v += j.p[(int64_t)r * (j.ld + 1)];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}
void launch_traces(const TraceJob* jobs, int njobs, double* out, Stream st) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(traces_kernel, dim3(njobs), dim3(256), 0, (hipStream_t)st, jobs, out);
  check_launch("traces");
}

// ---------------------------------------------------------------------------
// Precision conversions (FP64 <-> FP32 copies of operands and vectors).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cvt_d2f_kernel(float* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = (float)src[i];
}
__global__ __launch_bounds__(256) void cvt_f2d_kernel(double* __restrict__ dst, const float* __restrict__ src, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = (double)src[i];
}
void launch_cvt_d2f(float* dst, const double* src, int64_t n, Stream st) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>((n + 255) / 256, 256 * 32);
  hipLaunchKernelGGL(cvt_d2f_kernel, dim3(nb), dim3(256), 0, (hipStream_t)st, dst, src, n);
  check_launch("cvt_d2f");
}
void launch_cvt_f2d(double* dst, const float* src, int64_t n, Stream st) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>((n + 255) / 256, 256 * 32);
  hipLaunchKernelGGL(cvt_f2d_kernel, dim3(nb), dim3(256), 0, (hipStream_t)st, dst, src, n);
  check_launch("cvt_f2d");
}

// ---------------------------------------------------------------------------
// Gather-accumulate of scaled (possibly transposed / identity) blocks.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gather_kernel(const GatherDst* __restrict__ dsts,
                                                     const GatherSrc* __restrict__ srcs) {
  const GatherDst d = dsts[blockIdx.x];
  const int n = d.rows * d.cols;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = e / d.cols, c = e % d.cols;
    double v = 0.0;
    for (int s = d.s0; s < d.s1; ++s) {
      const GatherSrc g = srcs[s];
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

void launch_gather(const GatherDst* dsts, int ndst, const GatherSrc* srcs, Stream st) {
  if (ndst <= 0) return;
  hipLaunchKernelGGL(gather_kernel, dim3(ndst), dim3(256), 0, (hipStream_t)st, dsts, srcs);
  check_launch("gather");
}

// ---------------------------------------------------------------------------
// Linear combinations of operators that share one element layout (the
// integral-weighted complementary-operator sums).  Grid: (element chunks, outputs).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void combo_ops_kernel(const ComboOut* __restrict__ outs,
                                                        const ComboIn* __restrict__ ins) {
  const ComboOut o = outs[blockIdx.y];
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < o.nnz; e += (int64_t)gridDim.x * 256) {
    double v = 0.0;
    for (int i = o.i0; i < o.i1; ++i) {
      const ComboIn c = ins[i];
      v += c.adj ? c.coef * o.fac[e] * c.in[o.perm[e]] : c.coef * c.in[e];
    }
    o.out[e] = v;
  }
}

void launch_combo(const ComboOut* outs, int nout, const ComboIn* ins, int64_t max_nnz, Stream st) {
  if (nout <= 0 || max_nnz <= 0) return;
  const int nb = (int)std::min<int64_t>(1024, (max_nnz + 255) / 256);
  for (int o0 = 0; o0 < nout; o0 += 65535) {
    const int cnt = std::min(65535, nout - o0);
    hipLaunchKernelGGL(combo_ops_kernel, dim3(nb, cnt), dim3(256), 0, (hipStream_t)st, outs + o0, ins);
  }
  check_launch("combo");
}

// ---------------------------------------------------------------------------
// Diagonal of H_eff.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void diag_kernel(const DiagSec* __restrict__ secs,
                                                   const DiagTask* __restrict__ tasks) {
  const DiagSec s = secs[blockIdx.x];
  const int n = s.rows * s.cols;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = e / s.cols, c = e % s.cols;
    double v = 0.0;
    for (int t = s.t0; t < s.t1; ++t) {
      const DiagTask d = tasks[t];
      const double xv = d.x ? d.x[(int64_t)r * d.sx] : 1.0;
      const double yv = d.y ? d.y[(int64_t)c * d.sy] : 1.0;
      v += d.coef * xv * yv;
    }
    s.out[e] = v;
  }
}

void launch_diag(const DiagSec* secs, int nsec, const DiagTask* tasks, Stream st) {
  if (nsec <= 0) return;
  hipLaunchKernelGGL(diag_kernel, dim3(nsec), dim3(256), 0, (hipStream_t)st, secs, tasks);
  check_launch("diag");
}

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD, one workgroup per sector matrix.
// Works on the tall orientation M (m x n, m >= n): columns are rotated until
// mutually orthogonal; M V = U S.  Column pairs are visited in round-robin
// (tournament) order, so n/2 disjoint pairs are processed concurrently: a
// group of G lanes per pair, G chosen per matrix so that a round's pairs
// are all in flight at once where they fit (G = 8 from 65 pairs up, 16, 32,
// 64 for fewer); a round is then a single pass of dependent memory accesses
// instead of several.
// ---------------------------------------------------------------------------
#ifndef SVD_WAVES_N
#define SVD_WAVES_N 16
#endif
constexpr int SVD_WAVES = SVD_WAVES_N;

// Sum over the G lanes of a group (butterfly: every lane of the group ends
// with the same value, bit for bit).
template <int G>
__device__ inline double group_sum(double v) {
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// Jacobi sweeps over the columns of M (m x n) and V (n x n), column j
// contiguous, until a sweep rotates no pair of columns that both hold more
// than 1e-13 of the matrix norm (fro2 = squared Frobenius norm), at most 60
// sweeps.  Pairs of smaller columns are still rotated, but do not keep the
// sweeps going: in a rank-deficient matrix they are rounding noise whose
// relative inner products never settle, and the decomposition replaces them
// (vanishing singular values) anyway.
template <int G>
__device__ void svd_sweeps(double* M, double* V, int m, int n, double fro2) {
  constexpr int PAIRS = SVD_WAVES * (64 / G);  // pairs processed at once
  const int tid = threadIdx.x;
  const int gl = tid % G, grp = tid / G;  // lane within its pair group, group index
  __shared__ int s_rot;
  const int np = (n % 2) ? n + 1 : n;  // tournament with a dummy when n is odd
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      // pairs (p, q) of the round-robin schedule: position 0 fixed, others rotate
      for (int pr = grp; pr < np / 2; pr += PAIRS) {
        // circle method: slot 0 fixed, slots 1..np-1 rotate; pair (slot pr, slot np-1-pr)
        const int a = (pr == 0) ? 0 : ((pr - 1 + round) % (np - 1)) + 1;
        const int b = ((np - 2 - pr + round) % (np - 1)) + 1;
        const int p = min(a, b), q = max(a, b);
        if (q >= n || p == q) continue;
        double* mp = M + (int64_t)p * m;
        double* mq = M + (int64_t)q * m;
        double al = 0, be = 0, ga = 0;
        for (int i = gl; i < m; i += G) {
          const double x = mp[i], y = mq[i];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        al = group_sum<G>(al);
        be = group_sum<G>(be);
        ga = group_sum<G>(ga);
        if (fabs(ga) <= 1e-15 * sqrt(al * be) || ga == 0.0) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
        for (int i = gl; i < m; i += G) {
          const double x = mp[i], y = mq[i];
          mp[i] = cs * x - sn * y;
          mq[i] = sn * x + cs * y;
        }
        double* vp = V + (int64_t)p * n;
        double* vq = V + (int64_t)q * n;
        for (int i = gl; i < n; i += G) {
          const double x = vp[i], y = vq[i];
          vp[i] = cs * x - sn * y;
          vq[i] = sn * x + cs * y;
        }
        if (gl == 0 && al > 1e-26 * fro2 && be > 1e-26 * fro2) s_rot = 1;
      }
      __syncthreads();
    }
    if (s_rot == 0) break;
    __syncthreads();
  }
}

// phase 0: the whole decomposition; 1: only the working copy (M, V = 1, and
// the squared norm of A in the norm slot, for svd_block_kernel); 2: only the
// outputs of a working copy the block rounds have orthogonalised.
__global__ __launch_bounds__(64 * SVD_WAVES) void svd_kernel(const SvdJob* __restrict__ jobs, int phase) {
  const SvdJob jb = jobs[blockIdx.x];
  const bool tall = jb.rows >= jb.cols;
  const int m = tall ? jb.rows : jb.cols;  // long side
  const int n = tall ? jb.cols : jb.rows;  // short side (number of singular values)
  double* M = jb.work;                     // m x n, column j contiguous: M[j*m + i]
  double* V = M + (int64_t)m * n;          // n x n, column j contiguous
  double* nrm = V + (int64_t)n * n;        // n
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int nth = blockDim.x;
  const double* A = jb.a;
  if (phase != 2) {
    // load (column-major working copy of the tall orientation)
    for (int e = tid; e < m * n; e += nth) {
      const int j = e / m, i = e % m;  // column j, row i of the tall matrix
      M[e] = tall ? A[(int64_t)i * jb.lda + j] : A[(int64_t)j * jb.lda + i];
    }
    for (int e = tid; e < n * n; e += nth) V[e] = (e / n == e % n) ? 1.0 : 0.0;
    __shared__ double s_fro[SVD_WAVES];
    {
      double f = 0;
      for (int e = tid; e < m * n; e += nth) f += M[e] * M[e];
      f = wave_sum(f);
      if (lane == 0) s_fro[wv] = f;
    }
    __syncthreads();
    double fro2 = 0;
    for (int w = 0; w < SVD_WAVES; ++w) fro2 += s_fro[w];
    if (phase == 1) {
      if (tid == 0) nrm[0] = fro2;
      return;
    }

    const int half = (n + 1) / 2;  // pairs per round
    if (half <= SVD_WAVES)
      svd_sweeps<64>(M, V, m, n, fro2);
    else if (half <= 2 * SVD_WAVES)
      svd_sweeps<32>(M, V, m, n, fro2);
    else if (half <= 4 * SVD_WAVES)
      svd_sweeps<16>(M, V, m, n, fro2);
    else
      svd_sweeps<8>(M, V, m, n, fro2);
  }
  __syncthreads();
  // column norms
  for (int j = wv; j < n; j += SVD_WAVES) {
    double s = 0;
    for (int i = lane; i < m; i += 64) s += M[(int64_t)j * m + i] * M[(int64_t)j * m + i];
    s = wave_sum(s);
    if (lane == 0) nrm[j] = sqrt(s);
  }
  __syncthreads();
  // sort order (descending), stable: rank of column j
  __shared__ int s_ord[1024];
  for (int j = tid; j < n; j += nth) {
    int rank = 0;
    for (int i = 0; i < n; ++i) rank += (nrm[i] > nrm[j]) || (nrm[i] == nrm[j] && i < j);
    s_ord[rank] = j;
  }
  __syncthreads();
  // outputs: long-side factor columns L_k = M_col / s (m x n), short-side V (n x n)
  // tall:  A = L S V^T  -> U = L (rows x r), Vt = V^T (r x cols)
  // wide:  A^T = L S V^T -> A = V S L^T -> U = V (rows x r), Vt = L^T (r x cols)
  double* U = jb.u;
  double* S = jb.s;
  double* VT = jb.vt;
  const double smax = nrm[s_ord[0]];
  for (int k = tid; k < n; k += nth) S[k] = nrm[s_ord[k]];
  // long-side factor: column k is M's column s_ord[k] / s while s is not
  // vanishing (the columns are sorted, so those are a prefix) ...
  auto put = [&](int i, int k, double v) {
    if (tall)
      U[(int64_t)i * n + k] = v;
    else
      VT[(int64_t)k * jb.cols + i] = v;
  };
  auto get = [&](int i, int k) -> double { return tall ? U[(int64_t)i * n + k] : VT[(int64_t)k * jb.cols + i]; };
  int kt = 0;
  while (kt < n && nrm[s_ord[kt]] > 1e-13 * smax && nrm[s_ord[kt]] != 0.0) ++kt;
  for (int e = tid; e < kt * m; e += nth) {
    const int k = e / m, i = e % m;
    put(i, k, M[(int64_t)s_ord[k] * m + i] / nrm[s_ord[k]]);
  }
  __syncthreads();
  // ... and the vanishing ones complete the set: column k from the unit
  // vector e_t (t = k, k+1, ... mod m) orthogonalised twice against every
  // earlier column at once (classical Gram-Schmidt: the inner products one
  // wave per column, then one update pass), kept once the squared norm left
  // exceeds half the average share (m - k) / m of the complement, which the
  // best unit vector always reaches
  __shared__ double s_d[1024];
  __shared__ double s_red2[SVD_WAVES];
  for (int k = kt; k < n; ++k) {
    for (int a = 0; a < m; ++a) {
      const int tt = (k + a) % m;
      for (int i = tid; i < m; i += nth) put(i, k, i == tt ? 1.0 : 0.0);
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass) {
        for (int kk = wv; kk < k; kk += SVD_WAVES) {
          double d = 0;
          for (int i = lane; i < m; i += 64) d += get(i, kk) * get(i, k);
          d = wave_sum(d);
          if (lane == 0) s_d[kk] = d;
        }
        __syncthreads();
        for (int i = tid; i < m; i += nth) {
          double v = get(i, k);
          for (int kk = 0; kk < k; ++kk) v -= s_d[kk] * get(i, kk);
          put(i, k, v);
        }
        __syncthreads();
      }
      double d = 0;
      for (int i = tid; i < m; i += nth) d += get(i, k) * get(i, k);
      d = wave_sum(d);
      if (lane == 0) s_red2[wv] = d;
      __syncthreads();
      double nn = 0;
      for (int w = 0; w < SVD_WAVES; ++w) nn += s_red2[w];
      __syncthreads();
      if (nn > 0.5 * (double)(m - k) / (double)m) {
        const double inv = 1.0 / sqrt(nn);
        for (int i = tid; i < m; i += nth) put(i, k, get(i, k) * inv);
        __syncthreads();
        break;
      }
    }
  }
  // short-side factor
  for (int e = tid; e < n * n; e += nth) {
    const int k = e / n, i = e % n;  // column k (sorted) of V, row i
    const double v = V[(int64_t)s_ord[k] * n + i];
    if (tall)
      VT[(int64_t)k * jb.cols + i] = v;  // Vt[k][i]
    else
      U[(int64_t)i * n + k] = v;  // U[i][k]
  }
}

void launch_svd(const SvdJob* jobs, int njobs, int max_short, Stream st, int phase) {
  if (njobs <= 0) return;
  if (max_short > 1024) dev_fail("svd: sector matrix too large (short side > 1024)");
  if (phase < 0 || phase > 2) dev_fail("svd: phase must be 0, 1 or 2");
  hipLaunchKernelGGL(svd_kernel, dim3(njobs), dim3(64 * SVD_WAVES), 0, (hipStream_t)st, jobs, phase);
  check_launch("svd");
}

// ---------------------------------------------------------------------------
// Block one-sided Jacobi for the larger sector matrices: the working copy's
// columns are cut into blocks of SVB_W; in round r of a sweep the blocks are
// paired by the same round-robin schedule as single columns, and every pair
// of blocks is a workgroup of its own, so a matrix is worked on by many
// compute units at once.  A workgroup loads the pair's columns of M and V
// into LDS, rotates pairs of them (one wave per column pair, all in LDS) and
// writes them back: in round 0, where every block is visited once, one sweep
// of the single-column method over all columns of the two blocks; in the
// later rounds only the pairs across the two blocks, so every pair of
// columns is visited once per sweep.  The memory traffic per rotation falls
// by the width of a block and the rounds of a sweep by its square.  flags[job] is set when a pair of columns that both hold more than
// 1e-13 of the matrix norm was rotated (the convergence test of the
// single-workgroup sweeps), so the host repeats sweeps until no flag is set;
// a job whose previous sweep set no flag (active[k] == 0) is left alone.
// ---------------------------------------------------------------------------
constexpr int SVB_W = 16;                 // columns per block
constexpr int SVB_LDS = 2 * SVB_W * 600;  // doubles of LDS: the pair's columns of M and V, m + n <= 600
__global__ __launch_bounds__(1024) void svd_block_kernel(const SvdJob* __restrict__ jobs,
                                                         const int* __restrict__ pair_base, int njobs, int round,
                                                         const int* __restrict__ active, int* __restrict__ flags) {
  __shared__ double sMV[SVB_LDS];
  __shared__ int s_flag;
  // job of this workgroup: the last k with pair_base[k] <= blockIdx.x
  int k = 0;
  {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (pair_base[mid] <= (int)blockIdx.x)
        lo = mid;
      else
        hi = mid - 1;
    }
    k = lo;
  }
  if (!active[k]) return;  // converged in an earlier sweep
  const SvdJob jb = jobs[k];
  const bool tall = jb.rows >= jb.cols;
  const int m = tall ? jb.rows : jb.cols, n = tall ? jb.cols : jb.rows;
  double* M = jb.work;
  double* V = M + (int64_t)m * n;
  const double fro2 = V[(int64_t)n * n];  // phase 1 left it in the norm slot
  const int nblk = (n + SVB_W - 1) / SVB_W, npb = nblk + (nblk & 1);
  if (round >= npb - 1) return;
  const int pr = (int)blockIdx.x - pair_base[k];
  const int ba = (pr == 0) ? 0 : ((pr - 1 + round) % (npb - 1)) + 1;
  const int bb = ((npb - 2 - pr + round) % (npb - 1)) + 1;
  // local columns: block ba then block bb (a block at or past nblk is empty)
  const int a0 = ba * SVB_W, a1 = ba < nblk ? min(a0 + SVB_W, n) : a0;
  const int b0 = bb * SVB_W, b1 = bb < nblk ? min(b0 + SVB_W, n) : b0;
  const int na = a1 - a0, nc = na + (b1 - b0);
  const bool cross = round > 0;  // only the pairs across the two blocks
  if (nc < 2 || (cross && (na == 0 || na == nc))) return;
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  double* sM = sMV;               // local column c at c * m
  double* sV = sMV + 2 * SVB_W * m;  // local column c at c * n
  auto gcol = [&](int c) { return c < na ? a0 + c : b0 + (c - na); };
  for (int e = tid; e < nc * m; e += 1024) {
    const int c = e / m, i = e % m;
    sM[e] = M[(int64_t)gcol(c) * m + i];
  }
  for (int e = tid; e < nc * n; e += 1024) {
    const int c = e / n, i = e % n;
    sV[e] = V[(int64_t)gcol(c) * n + i];
  }
  if (tid == 0) s_flag = 0;
  __syncthreads();
  const double tol = fmax(1e-15, (double)m * 2.220446049250313e-16);
  const int npl = nc + (nc & 1);
  const int nr = cross ? SVB_W : npl - 1;
  for (int r = 0; r < nr; ++r) {
    // wave wv takes local pair wv of round r (at most SVB_W pairs, 16 waves):
    // across the blocks column wv of the first with column (wv + r) mod SVB_W
    // of the second, else the round-robin pair of all columns
    int p = 0, q = 0;
    if (cross) {
      p = wv;
      q = na + (wv + r) % SVB_W;
    } else if (wv < npl / 2) {
      const int la = (wv == 0) ? 0 : ((wv - 1 + r) % (npl - 1)) + 1;
      const int lb = ((npl - 2 - wv + r) % (npl - 1)) + 1;
      p = min(la, lb);
      q = max(la, lb);
    }
    if (q < nc && p != q && p < (cross ? na : nc)) {
      double* mp = sM + p * m;
      double* mq = sM + q * m;
      double al = 0, be = 0, ga = 0;
      for (int i = lane; i < m; i += 64) {
        const double x = mp[i], y = mq[i];
        al += x * x;
        be += y * y;
        ga += x * y;
      }
      al = wave_sum(al);
      be = wave_sum(be);
      ga = wave_sum(ga);
      if (!(fabs(ga) <= tol * sqrt(al * be) || ga == 0.0)) {
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
        for (int i = lane; i < m; i += 64) {
          const double x = mp[i], y = mq[i];
          mp[i] = cs * x - sn * y;
          mq[i] = sn * x + cs * y;
        }
        double* vp = sV + p * n;
        double* vq = sV + q * n;
        for (int i = lane; i < n; i += 64) {
          const double x = vp[i], y = vq[i];
          vp[i] = cs * x - sn * y;
          vq[i] = sn * x + cs * y;
        }
        if (lane == 0 && al > 1e-26 * fro2 && be > 1e-26 * fro2) s_flag = 1;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < nc * m; e += 1024) {
    const int c = e / m, i = e % m;
    M[(int64_t)gcol(c) * m + i] = sM[e];
  }
  for (int e = tid; e < nc * n; e += 1024) {
    const int c = e / n, i = e % n;
    V[(int64_t)gcol(c) * n + i] = sV[e];
  }
  if (tid == 0 && s_flag) flags[k] = 1;
}

bool svd_block_fits(int rows, int cols) { return rows + cols <= SVB_LDS / (2 * SVB_W); }
int svd_block_pairs(int rows, int cols) {
  const int nblk = (min(rows, cols) + SVB_W - 1) / SVB_W;
  return (nblk + (nblk & 1)) / 2;
}
int svd_block_rounds(int rows, int cols) {
  const int nblk = (min(rows, cols) + SVB_W - 1) / SVB_W;
  return nblk + (nblk & 1) - 1;
}
void launch_svd_block(const SvdJob* jobs, const int* pair_base, int njobs, int npairs, int round,
                      const int* active, int* flags, Stream st) {
  if (njobs <= 0 || npairs <= 0) return;
  hipLaunchKernelGGL(svd_block_kernel, dim3(npairs), dim3(1024), 0, (hipStream_t)st, jobs, pair_base, njobs, round,
                     active, flags);
  check_launch("svd_block");
}

__global__ __launch_bounds__(256) void svd_signs_kernel(const SvdJob* __restrict__ jobs) {
  const SvdJob j = jobs[blockIdx.x];
  const int r = min(j.rows, j.cols);
  __shared__ double bv[256];
  __shared__ int bi[256];
  for (int a = 0; a < r; ++a) {
    double best = -1.0;
    int idx = 0x7fffffff;
    for (int row = threadIdx.x; row < j.rows; row += 256) {
      const double v = fabs(j.u[(int64_t)row * r + a]);
      if (v > best) {  // rows visited in increasing order: ties keep the lowest
        best = v;
        idx = row;
      }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = idx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        const double ov = bv[threadIdx.x + w];
        const int oi = bi[threadIdx.x + w];
        if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
          bv[threadIdx.x] = ov;
          bi[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    const bool flip = bi[0] < j.rows && j.u[(int64_t)bi[0] * r + a] < 0.0;
    __syncthreads();
    if (flip) {
      for (int row = threadIdx.x; row < j.rows; row += 256) j.u[(int64_t)row * r + a] = -j.u[(int64_t)row * r + a];
      for (int c = threadIdx.x; c < j.cols; c += 256) j.vt[(int64_t)a * j.cols + c] = -j.vt[(int64_t)a * j.cols + c];
    }
    __syncthreads();
  }
}

void launch_svd_signs(const SvdJob* jobs, int njobs, Stream st) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(svd_signs_kernel, dim3(njobs), dim3(256), 0, (hipStream_t)st, jobs);
  check_launch("svd_signs");
}

// ---------------------------------------------------------------------------
// Davidson vector kernels
// ---------------------------------------------------------------------------
constexpr int RB = 256;
constexpr int RCH = 256;  // partial-sum chunks per vector

__global__ __launch_bounds__(RB) void dots_stage1(const double* __restrict__ V, int64_t ldv,
                                                  const double* __restrict__ x, int64_t n,
                                                  double* __restrict__ partial) {
  const int j = blockIdx.y;
  const int64_t chunk = (n + RCH - 1) / RCH;
  const int64_t b = blockIdx.x * chunk, e = min(n, b + chunk);
  const double* v = V + j * ldv;
  double s = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += RB) s += v[i] * x[i];
  __shared__ double red[RB / 64];
  s = wave_sum(s);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < RB / 64; ++w) t += red[w];
    partial[(int64_t)j * RCH + blockIdx.x] = t;
  }
}

__global__ void dots_stage2(const double* __restrict__ partial, int k, double* __restrict__ out) {
  const int j = blockIdx.x;
  double s = 0;
  for (int i = threadIdx.x; i < RCH; i += 64) s += partial[(int64_t)j * RCH + i];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[j] = s;
}

void launch_dots(const double* V, int64_t ldv, int k, const double* x, int64_t n, double* out, double* partial,
                 Stream st) {
  if (k <= 0) return;
  hipLaunchKernelGGL(dots_stage1, dim3(RCH, k), dim3(RB), 0, (hipStream_t)st, V, ldv, x, n, partial);
  hipLaunchKernelGGL(dots_stage2, dim3(k), dim3(64), 0, (hipStream_t)st, partial, k, out);
}

__global__ void combo_kernel(const double* __restrict__ V, int64_t ldv, int k, const double* __restrict__ coef,
                             double alpha, int64_t n, double* __restrict__ y, double beta) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0;
    for (int j = 0; j < k; ++j) s += coef[j] * V[j * ldv + i];
    y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + alpha * s;
  }
}

void launch_combo_vec(const double* V, int64_t ldv, int k, const double* coef, double alpha, int64_t n, double* y,
                      double beta, Stream st) {
  int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(combo_kernel, dim3(nb), dim3(256), 0, (hipStream_t)st, V, ldv, k, coef, alpha, n, y, beta);
}

__global__ void residual_kernel(const double* ax, const double* x, const double* theta, int64_t n, double* r) {
  const double th = theta[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = ax[i] - th * x[i];
}

void launch_residual(const double* ax, const double* x, const double* theta, int64_t n, double* r, Stream st) {
  int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(residual_kernel, dim3(nb), dim3(256), 0, (hipStream_t)st, ax, x, theta, n, r);
}

__global__ void precond_kernel(const double* r, const double* diag, const double* theta, int64_t n, double* t) {
  const double th = theta[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double d = th - diag[i];
    if (fabs(d) < 1e-12) d = d < 0 ? -1e-12 : 1e-12;
    t[i] = r[i] / d;
  }
}

void launch_precond(const double* r, const double* diag, const double* theta, int64_t n, double* t, Stream st) {
  int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(precond_kernel, dim3(nb), dim3(256), 0, (hipStream_t)st, r, diag, theta, n, t);
}

__global__ void normalize_kernel(double* y, const double* nrm2, int64_t n) {
  const double f = 1.0 / sqrt(nrm2[0]);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] *= f;
}

void launch_normalize(double* y, const double* nrm2, int64_t n, Stream st) {
  int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(normalize_kernel, dim3(nb), dim3(256), 0, (hipStream_t)st, y, nrm2, n);
}

// Cyclic Jacobi eigen-decomposition of a small symmetric matrix, one
// workgroup of SYEV_T threads.  Round-robin ordering: k/2 disjoint rotations
// per round, whose row and column updates are spread over all threads (each
// element's arithmetic does not depend on the thread count).
constexpr int SYEV_MAX = 64;
constexpr int SYEV_T = 256;

__device__ __forceinline__ void syev_body(const double* __restrict__ H, const int k, const int ld,
                                          double* __restrict__ evals, double* __restrict__ evecs) {
  __shared__ double a[SYEV_MAX][SYEV_MAX + 1];
  __shared__ double v[SYEV_MAX][SYEV_MAX + 1];
  __shared__ double rc[SYEV_MAX / 2], rs[SYEV_MAX / 2];
  __shared__ int rp[SYEV_MAX / 2], rq[SYEV_MAX / 2];
  __shared__ int s_any;
  const int lane = threadIdx.x;
  for (int e = lane; e < k * k; e += SYEV_T) {
    const int i = e / k, j = e % k;
    a[i][j] = (i >= j) ? H[i * ld + j] : H[j * ld + i];  // lower triangle is authoritative
    v[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int np = (k % 2) ? k + 1 : k;
  for (int sweep = 0; sweep < 100 && k > 1; ++sweep) {
    if (lane == 0) s_any = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      if (lane < np / 2) {
        const int pr = lane;
        const int x = (pr == 0) ? 0 : ((pr - 1 + round) % (np - 1)) + 1;
        const int y = ((np - 2 - pr + round) % (np - 1)) + 1;
        int p = min(x, y), q = max(x, y);
        double c = 1.0, s = 0.0;
        if (q < k && p != q) {
          const double apq = a[p][q];
          if (fabs(apq) > 1e-300 && fabs(apq) > 1e-17 * sqrt(fabs(a[p][p] * a[q][q]) + 1e-300)) {
            const double th = (a[q][q] - a[p][p]) / (2.0 * apq);
            const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            s_any = 1;
          }
        } else {
          p = q = -1;
        }
        rp[pr] = p;
        rq[pr] = q;
        rc[pr] = c;
        rs[pr] = s;
      }
      __syncthreads();
      // rows: a <- J^T a
      for (int e = lane; e < (np / 2) * k; e += SYEV_T) {
        const int pr = e / k, j = e % k;
        const int p = rp[pr], q = rq[pr];
        if (p < 0) continue;
        const double c = rc[pr], s = rs[pr];
        const double x = a[p][j], y = a[q][j];
        a[p][j] = c * x - s * y;
        a[q][j] = s * x + c * y;
      }
      __syncthreads();
      // cols: a <- a J ; v <- v J
      for (int e = lane; e < (np / 2) * k; e += SYEV_T) {
        const int pr = e / k, i = e % k;
        const int p = rp[pr], q = rq[pr];
        if (p < 0) continue;
        const double c = rc[pr], s = rs[pr];
        const double x = a[i][p], y = a[i][q];
        a[i][p] = c * x - s * y;
        a[i][q] = s * x + c * y;
        const double vx = v[i][p], vy = v[i][q];
        v[i][p] = c * vx - s * vy;
        v[i][q] = s * vx + c * vy;
      }
      __syncthreads();
    }
    if (s_any == 0) break;
    __syncthreads();
  }
  // sort ascending (selection by rank)
  __shared__ int ord[SYEV_MAX];
  for (int j = lane; j < k; j += SYEV_T) {
    int rank = 0;
    for (int i = 0; i < k; ++i) rank += (a[i][i] < a[j][j]) || (a[i][i] == a[j][j] && i < j);
    ord[rank] = j;
  }
  __syncthreads();
  for (int j = lane; j < k; j += SYEV_T) evals[j] = a[ord[j]][ord[j]];
  for (int e = lane; e < k * k; e += SYEV_T) {
    const int j = e / k, i = e % k;
    evecs[j * k + i] = v[i][ord[j]];  // eigenvector j contiguous
  }
}

__global__ __launch_bounds__(SYEV_T) void syev_kernel(const double* __restrict__ H, int k, int ld,
                                                  double* __restrict__ evals, double* __restrict__ evecs) {
  syev_body(H, k, ld, evals, evecs);
}

void launch_syev_small(const double* H, int k, int ld, double* evals, double* evecs, Stream st) {
  hipLaunchKernelGGL(syev_kernel, dim3(1), dim3(SYEV_T), 0, (hipStream_t)st, H, k, ld, evals, evecs);
}

// ---------------------------------------------------------------------------
// The same Davidson helpers over job lists (one launch for many solves).  Each
// job gets the arithmetic of the single-solve kernel above: the same
// partial-sum chunks and reduction order for the inner products, the same
// element formulas, the same Jacobi solver.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RB) void dots_batch_stage1(const DotJob* __restrict__ jobs) {
  const DotJob jb = jobs[blockIdx.z];
  const int j = blockIdx.y;
  if (j >= jb.k) return;
  const int64_t n = jb.n;
  const int64_t chunk = (n + RCH - 1) / RCH;
  const int64_t b = blockIdx.x * chunk, e = min(n, b + chunk);
  const double* v = jb.V + j * jb.ldv;
  const double* x = jb.x;
  double s = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += RB) s += v[i] * x[i];
  __shared__ double red[RB / 64];
  s = wave_sum(s);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < RB / 64; ++w) t += red[w];
    jb.part[(int64_t)j * RCH + blockIdx.x] = t;
  }
}

__global__ void dots_batch_stage2(const DotJob* __restrict__ jobs) {
  const DotJob jb = jobs[blockIdx.y];
  const int j = blockIdx.x;
  if (j >= jb.k) return;
  double s = 0;
  for (int i = threadIdx.x; i < RCH; i += 64) s += jb.part[(int64_t)j * RCH + i];
  s = wave_sum(s);
  if (threadIdx.x == 0) jb.out[j] = s;
}

void launch_dots_batch(const DotJob* jobs, int njobs, int max_k, Stream st) {
  if (njobs <= 0 || max_k <= 0) return;
  hipLaunchKernelGGL(dots_batch_stage1, dim3(RCH, max_k, njobs), dim3(RB), 0, (hipStream_t)st, jobs);
  hipLaunchKernelGGL(dots_batch_stage2, dim3(max_k, njobs), dim3(64), 0, (hipStream_t)st, jobs);
  check_launch("dots_batch");
}

__global__ void combo_batch_kernel(const ComboJob* __restrict__ jobs) {
  const ComboJob jb = jobs[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < jb.n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0;
    for (int j = 0; j < jb.k; ++j) s += jb.coef[j] * jb.V[j * jb.ldv + i];
    jb.y[i] = (jb.beta == 0.0 ? 0.0 : jb.beta * jb.y[i]) + jb.alpha * s;
  }
}

void launch_combo_batch(const ComboJob* jobs, int njobs, int64_t max_n, Stream st) {
  if (njobs <= 0) return;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (max_n + 255) / 256));
  hipLaunchKernelGGL(combo_batch_kernel, dim3(nb, njobs), dim3(256), 0, (hipStream_t)st, jobs);
  check_launch("combo_batch");
}

__global__ void ew_batch_kernel(const EwJob* __restrict__ jobs) {
  const EwJob jb = jobs[blockIdx.y];
  const int64_t n = jb.n;
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, step = (int64_t)gridDim.x * blockDim.x;
  switch (jb.kind) {
    case EW_COPY:
      for (int64_t i = i0; i < n; i += step) jb.y[i] = jb.a[i];
      break;
    case EW_ZERO:
      for (int64_t i = i0; i < n; i += step) jb.y[i] = 0.0;
      break;
    case EW_RESIDUAL: {
      const double th = jb.s[0];
      for (int64_t i = i0; i < n; i += step) jb.y[i] = jb.a[i] - th * jb.b[i];
      break;
    }
    case EW_PRECOND: {
      const double th = jb.s[0];
      for (int64_t i = i0; i < n; i += step) {
        double d = th - jb.b[i];
        if (fabs(d) < 1e-12) d = d < 0 ? -1e-12 : 1e-12;
        jb.y[i] = jb.a[i] / d;
      }
      break;
    }
    case EW_NORMALIZE: {
      const double f = 1.0 / sqrt(jb.s[0]);
      for (int64_t i = i0; i < n; i += step) jb.y[i] *= f;
      break;
    }
    case EW_D2F:
      for (int64_t i = i0; i < n; i += step) ((float*)jb.y)[i] = (float)jb.a[i];
      break;
    case EW_F2D:
      for (int64_t i = i0; i < n; i += step) jb.y[i] = (double)((const float*)jb.a)[i];
      break;
    default:
      break;
  }
}

void launch_ew_batch(const EwJob* jobs, int njobs, int64_t max_n, Stream st) {
  if (njobs <= 0) return;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (max_n + 255) / 256));
  hipLaunchKernelGGL(ew_batch_kernel, dim3(nb, njobs), dim3(256), 0, (hipStream_t)st, jobs);
  check_launch("ew_batch");
}

__global__ __launch_bounds__(SYEV_T) void syev_batch_kernel(const SyevJob* __restrict__ jobs) {
  const SyevJob jb = jobs[blockIdx.x];
  syev_body(jb.H, jb.k, jb.ld, jb.evals, jb.evecs);
}

void launch_syev_batch(const SyevJob* jobs, int njobs, Stream st) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(syev_batch_kernel, dim3(njobs), dim3(SYEV_T), 0, (hipStream_t)st, jobs);
  check_launch("syev_batch");
}

// ---------------------------------------------------------------------------
// Davidson iterations as a fixed launch sequence.  Each kernel reads the
// solve's subspace size and flags from its DGState and runs only while the
// solve is live (and, for the collapse and restart branches, while their
// flag is set); its arithmetic is that of the corresponding job-list helper.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool dg_live(const DGJob& j, int gate) {
  const DGState* s = j.s;
  if (s->done) return false;
  if (gate == DG_GATE_COLLAPSE) return s->collapse != 0;
  if (gate == DG_GATE_RESTART) return s->restart != 0;
  return true;
}

__global__ void dg_scalar_kernel(const DGJob* __restrict__ jobs, int njobs, int which) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= njobs) return;
  const DGJob j = jobs[q];
  DGState* s = j.s;
  if (s->done) return;
  switch (which) {
    case DG_TOP:  // out of iterations: the previous Ritz vector is the result
      if (s->it > j.max_it) {
        s->state = 2;
        s->done = 1;
      }
      break;
    case DG_CHECK: {
      const double th = j.evals[0];
      const double rn = sqrt(fmax(0.0, j.nrm[0]));
      if (rn <= j.tol) {
        s->state = 1;
        s->done = 1;
      } else if (j.f32 && rn < 100.0 * j.eps * fmax(1.0, fabs(th))) {
        // the reduced-precision floor: stop when four iterations gain < 10 %
        if (rn < 0.9 * s->rbest) {
          s->rbest = rn;
          s->stall = 0;
        } else if (++s->stall >= 4) {
          s->state = 1;
          s->done = 1;
        }
      }
      break;
    }
    case DG_COLLAPSE:
      s->collapse = !(j.nrm2[0] > 1e-28);
      break;
    case DG_COLLAPSE2:
      if (s->collapse && !(j.nrm2[0] > 1e-28)) {
        s->state = 3;
        s->done = 1;
      }
      s->collapse = 0;
      break;
    case DG_RESTART_FLAG:
      s->restart = s->k >= j.ms;
      break;
    case DG_RESTART_K:
      if (s->restart) s->k = 1;
      s->restart = 0;
      break;
    case DG_ADVANCE:
      s->k += 1;
      s->it += 1;
      break;
    default:
      break;
  }
}

void launch_dg_scalar(const DGJob* jobs, int njobs, int which, Stream st) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(dg_scalar_kernel, dim3((njobs + 63) / 64), dim3(64), 0, (hipStream_t)st, jobs, njobs, which);
  check_launch("dg_scalar");
}

// the operands of an inner-product step: out[j] = V_j . x, j < cnt
__device__ __forceinline__ void dg_dot_args(const DGJob& jb, int which, const double*& V, const double*& x,
                                            double*& out, int& cnt) {
  const int k = jb.s->k;
  switch (which) {
    case DGD_ROW:  // row k of the projected matrix: V_j . W_k, j <= k
      V = jb.V, x = jb.W + (int64_t)k * jb.n, out = jb.Hs + (int64_t)k * jb.ms, cnt = k + 1;
      break;
    case DGD_RR:
      V = jb.r, x = jb.r, out = jb.nrm, cnt = 1;
      break;
    case DGD_VT:
      V = jb.V, x = jb.t, out = jb.coef, cnt = k;
      break;
    case DGD_TT:
      V = jb.t, x = jb.t, out = jb.nrm2, cnt = 1;
      break;
    case DGD_V0W0:
      V = jb.V, x = jb.W, out = jb.Hs, cnt = 1;
      break;
    default:  // DGD_V0T
      V = jb.V, x = jb.t, out = jb.coef, cnt = 1;
      break;
  }
}

// One workgroup per (chunk, solve) takes the vectors j < cnt in turn (the
// count is only known on the device); each partial sum is formed exactly as
// by the job-list helper.
__global__ __launch_bounds__(RB) void dg_dots_stage1(const DGJob* __restrict__ jobs, int which, int gate) {
  const DGJob jb = jobs[blockIdx.y];
  if (!dg_live(jb, gate)) return;
  const double *V, *x;
  double* out;
  int cnt;
  dg_dot_args(jb, which, V, x, out, cnt);
  const int64_t n = jb.n;
  const int64_t chunk = (n + RCH - 1) / RCH;
  const int64_t b = blockIdx.x * chunk, e = min(n, b + chunk);
  __shared__ double red[RB / 64];
  for (int j = 0; j < cnt; ++j) {
    const double* v = V + j * n;
    double s = 0;
    for (int64_t i = b + threadIdx.x; i < e; i += RB) s += v[i] * x[i];
    s = wave_sum(s);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int w = 0; w < RB / 64; ++w) t += red[w];
      jb.part[(int64_t)j * RCH + blockIdx.x] = t;
    }
    __syncthreads();
  }
}

__global__ void dg_dots_stage2(const DGJob* __restrict__ jobs, int which, int gate) {
  const DGJob jb = jobs[blockIdx.y];
  if (!dg_live(jb, gate)) return;
  const double *V, *x;
  double* out;
  int cnt;
  dg_dot_args(jb, which, V, x, out, cnt);
  const int j = blockIdx.x;
  if (j >= cnt) return;
  double s = 0;
  for (int i = threadIdx.x; i < RCH; i += 64) s += jb.part[(int64_t)j * RCH + i];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[j] = s;
}

void launch_dg_dots(const DGJob* jobs, int njobs, int which, int gate, int max_k, Stream st) {
  if (njobs <= 0 || max_k <= 0) return;
  hipLaunchKernelGGL(dg_dots_stage1, dim3(RCH, njobs), dim3(RB), 0, (hipStream_t)st, jobs, which, gate);
  hipLaunchKernelGGL(dg_dots_stage2, dim3(max_k, njobs), dim3(64), 0, (hipStream_t)st, jobs, which, gate);
  check_launch("dg_dots");
}

__global__ void dg_ew_kernel(const DGJob* __restrict__ jobs, int which, int gate) {
  const DGJob jb = jobs[blockIdx.y];
  if (!dg_live(jb, gate)) return;
  const int64_t n = jb.n;
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, step = (int64_t)gridDim.x * blockDim.x;
  const int k = jb.s->k;
  switch (which) {
    case DGE_PRECOND: {
      const double th = jb.evals[0];
      for (int64_t i = i0; i < n; i += step) {
        double d = th - jb.diag[i];
        if (fabs(d) < 1e-12) d = d < 0 ? -1e-12 : 1e-12;
        jb.t[i] = jb.r[i] / d;
      }
      break;
    }
    case DGE_RESIDUAL: {
      const double th = jb.evals[0];
      for (int64_t i = i0; i < n; i += step) jb.r[i] = jb.ax[i] - th * jb.x[i];
      break;
    }
    case DGE_COPY_RT:
      for (int64_t i = i0; i < n; i += step) jb.t[i] = jb.r[i];
      break;
    case DGE_NORMALIZE_T: {
      const double f = 1.0 / sqrt(jb.nrm2[0]);
      for (int64_t i = i0; i < n; i += step) jb.t[i] *= f;
      break;
    }
    case DGE_RESTART_COPY:
      for (int64_t i = i0; i < n; i += step) {
        jb.V[i] = jb.x[i];
        jb.W[i] = jb.ax[i];
      }
      break;
    case DGE_APPEND: {
      double* v = jb.V + (int64_t)k * n;
      for (int64_t i = i0; i < n; i += step) v[i] = jb.t[i];
      break;
    }
    case DGE_LOAD: {
      const double* v = jb.V + (int64_t)k * n;
      for (int64_t i = i0; i < n; i += step) jb.in[i] = v[i];
      break;
    }
    case DGE_STORE: {
      double* w = jb.W + (int64_t)k * n;
      for (int64_t i = i0; i < n; i += step) w[i] = jb.out[i];
      break;
    }
    default:
      break;
  }
}

void launch_dg_ew(const DGJob* jobs, int njobs, int which, int gate, int64_t max_n, Stream st) {
  if (njobs <= 0) return;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (max_n + 255) / 256));
  hipLaunchKernelGGL(dg_ew_kernel, dim3(nb, njobs), dim3(256), 0, (hipStream_t)st, jobs, which, gate);
  check_launch("dg_ew");
}

// y = beta y + alpha sum_{j < cnt} coef[j] V_j with the combo helper's arithmetic
__global__ void dg_combo_kernel(const DGJob* __restrict__ jobs, int which, int gate) {
  const DGJob jb = jobs[blockIdx.y];
  if (!dg_live(jb, gate)) return;
  const double* V;
  const double* coef;
  double* y;
  int cnt;
  double alpha, beta;
  const int k = jb.s->k;
  switch (which) {
    case DGC_RITZ_X:
      V = jb.V, coef = jb.evecs, y = jb.x, cnt = k, alpha = 1.0, beta = 0.0;
      break;
    case DGC_RITZ_AX:
      V = jb.W, coef = jb.evecs, y = jb.ax, cnt = k, alpha = 1.0, beta = 0.0;
      break;
    case DGC_ORTH:
      V = jb.V, coef = jb.coef, y = jb.t, cnt = k, alpha = -1.0, beta = 1.0;
      break;
    default:  // DGC_ORTH0
      V = jb.V, coef = jb.coef, y = jb.t, cnt = 1, alpha = -1.0, beta = 1.0;
      break;
  }
  const int64_t n = jb.n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0;
    for (int j = 0; j < cnt; ++j) s += coef[j] * V[j * n + i];
    y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + alpha * s;
  }
}

void launch_dg_combo(const DGJob* jobs, int njobs, int which, int gate, int64_t max_n, Stream st) {
  if (njobs <= 0) return;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (max_n + 255) / 256));
  hipLaunchKernelGGL(dg_combo_kernel, dim3(nb, njobs), dim3(256), 0, (hipStream_t)st, jobs, which, gate);
  check_launch("dg_combo");
}

__global__ __launch_bounds__(SYEV_T) void dg_syev_kernel(const DGJob* __restrict__ jobs) {
  const DGJob jb = jobs[blockIdx.x];
  if (jb.s->done) return;
  syev_body(jb.Hs, jb.s->k, jb.ms, jb.evals, jb.evecs);
}

void launch_dg_syev(const DGJob* jobs, int njobs, Stream st) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(dg_syev_kernel, dim3(njobs), dim3(SYEV_T), 0, (hipStream_t)st, jobs);
  check_launch("dg_syev");
}

void dev_capture_begin(Stream st) {
  hip_ok(hipStreamBeginCapture((hipStream_t)st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
}
void* dev_capture_end(Stream st) {
  hipGraph_t g = nullptr;
  hip_ok(hipStreamEndCapture((hipStream_t)st, &g), "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  hip_ok(e, "hipGraphInstantiate");
  return (void*)ex;
}
void dev_capture_abort(Stream st) {
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture((hipStream_t)st, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
}
void dev_graph_launch(void* exec, Stream st) {
  hip_ok(hipGraphLaunch((hipGraphExec_t)exec, (hipStream_t)st), "hipGraphLaunch");
}
void dev_graph_free(void* exec) {
  if (exec) (void)hipGraphExecDestroy((hipGraphExec_t)exec);
}

__global__ void scalars_kernel(const double* const* __restrict__ src, int n, double* __restrict__ dst) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i][0];
}

void launch_scalars(const double* const* src, int n, double* dst, Stream st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scalars_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)st, src, n, dst);
  check_launch("scalars");
}

// SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014).
__device__ inline uint64_t sm64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void fill_uniform_kernel(double* p, int64_t n, uint64_t seed, uint64_t stream) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = sm64(seed ^ sm64(stream * 0x100000001B3ull + (uint64_t)i));
    p[i] = (double)(k >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  }
}

void launch_fill_uniform(double* p, int64_t n, uint64_t seed, uint64_t stream, Stream st) {
  if (n <= 0) return;
  int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(fill_uniform_kernel, dim3(nb), dim3(256), 0, (hipStream_t)st, p, n, seed, stream);
}

__global__ void axpy_kernel(double* y, const double* x, double a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}
void launch_axpy(double* y, const double* x, double a, int64_t n, Stream st) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(axpy_kernel, dim3(nb), dim3(256), 0, (hipStream_t)st, y, x, a, n);
  check_launch("axpy");
}

__global__ void scal_kernel(double* y, double a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] *= a;
}

void launch_scal(double* y, double a, int64_t n, Stream st) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(scal_kernel, dim3(nb), dim3(256), 0, (hipStream_t)st, y, a, n);
  check_launch("scal");
}

__global__ void scale_rows_kernel(double* a, int rows, int cols, int ld, const double* s) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < rows * cols; e += gridDim.x * blockDim.x) {
    const int r = e / cols, c = e % cols;
    a[(int64_t)r * ld + c] *= s[r];
  }
}
__global__ void scale_cols_kernel(double* a, int rows, int cols, int ld, const double* s) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < rows * cols; e += gridDim.x * blockDim.x) {
    const int r = e / cols, c = e % cols;
    a[(int64_t)r * ld + c] *= s[c];
  }
}

void launch_scale_rows(double* a, int rows, int cols, int ld, const double* s, Stream st) {
  if (rows * cols <= 0) return;
  hipLaunchKernelGGL(scale_rows_kernel, dim3(std::min(1024, (rows * cols + 255) / 256)), dim3(256), 0, (hipStream_t)st, a, rows,
                     cols, ld, s);
}
void launch_scale_cols(double* a, int rows, int cols, int ld, const double* s, Stream st) {
  if (rows * cols <= 0) return;
  hipLaunchKernelGGL(scale_cols_kernel, dim3(std::min(1024, (rows * cols + 255) / 256)), dim3(256), 0, (hipStream_t)st, a, rows,
                     cols, ld, s);
}


// ---------------------------------------------------------------------------
// Streaming copy: reads 8n bytes and writes 8n bytes, nothing else.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void copy_kernel(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

void launch_copy(double* dst, const double* src, int64_t n, Stream st) {
  if (n <= 0) return;
  // up to 256 workgroups per CU: a 1 GiB copy then streams at about 6 TB/s
  // (a quarter of that grid reached 4.5 TB/s)
  const int64_t want = (n + 255) / 256;
  const int nb = (int)std::min<int64_t>(want, 256 * 256);
  hipLaunchKernelGGL(copy_kernel, dim3(nb), dim3(256), 0, (hipStream_t)st, dst, src, n);
  check_launch("copy");
}


__global__ void add_squares_kernel(double* y, const double* V, int64_t ldv, int k, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = y[i];
    for (int j = 0; j < k; ++j) {
      const double x = V[j * ldv + i];
      v += x * x;
    }
    y[i] = v;
  }
}
void launch_add_squares(double* y, const double* V, int64_t ldv, int k, int64_t n, Stream st) {
  if (n <= 0 || k <= 0) return;
  const int nb = (int)std::min<int64_t>(8192, (n + 255) / 256);
  hipLaunchKernelGGL(add_squares_kernel, dim3(nb), dim3(256), 0, (hipStream_t)st, y, V, ldv, k, n);
  check_launch("add_squares");
}


__global__ void rects_nonzero_kernel(const double* base, const RectDesc* rects, int n, unsigned char* flag) {
  const int r = blockIdx.x;
  if (r >= n) return;
  const RectDesc d = rects[r];
  int any = 0;
  const int64_t tot = (int64_t)d.rows * d.cols;
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
    const int64_t rr = e / d.cols, cc = e % d.cols;
    if (base[d.off + rr * d.ld + cc] != 0.0) any = 1;
  }
  __shared__ int hit;
  if (threadIdx.x == 0) hit = 0;
  __syncthreads();
  if (any) atomicOr(&hit, 1);
  __syncthreads();
  if (threadIdx.x == 0) flag[r] = (unsigned char)hit;
}
void launch_rects_nonzero(const double* base, const RectDesc* rects, int n, unsigned char* flag, Stream st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(rects_nonzero_kernel, dim3(n), dim3(256), 0, (hipStream_t)st, base, rects, n, flag);
  check_launch("rects_nonzero");
}

}  // namespace sadmrg
