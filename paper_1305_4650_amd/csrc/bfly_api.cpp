// Host side of libbfly: argument validation (before any HIP call), plans,
// workspace sizing and carving, and the C ABI of include/bfly.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/bfly.h"
#include "bfly_internal.h"

struct bfly_plan_s {
  int d = 0;
  int64_t N = 0;
  int L = 0;
  int q = 0;
  int r = 0;
  int phase = 0;
  double src_lo[3] = {0, 0, 0}, src_hi[3] = {0, 0, 0};
  double tgt_lo[3] = {0, 0, 0}, tgt_hi[3] = {0, 0, 0};
  double z[bfly::kQMax] = {};
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int ok() {
  g_last_error.clear();
  return BFLY_OK;
}

int q_max(int d) { return d == 1 ? 16 : (d == 2 ? 12 : 5); }

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Geometry of one apply in its own roles (adjoint swaps the boxes).
bfly::Geo make_geo(const bfly_plan_s& p, bool adjoint) {
  bfly::Geo g;
  std::memset(&g, 0, sizeof g);
  g.d = p.d;
  g.L = p.L;
  g.q = p.q;
  g.r = p.r;
  // middle switch (Sec. 1.4); the adjoint's levels mirror the forward's, so
  // its switch at L - floor(L/2) makes it the exact transpose of the forward
  g.ls = adjoint ? p.L - p.L / 2 : p.L / 2;
  g.phase = p.phase;
  g.adj = adjoint ? 1 : 0;
  g.nc = 1 << p.d;
  g.Nd = (double)p.N;
  const double* slo = adjoint ? p.tgt_lo : p.src_lo;
  const double* shi = adjoint ? p.tgt_hi : p.src_hi;
  const double* tlo = adjoint ? p.src_lo : p.tgt_lo;
  const double* thi = adjoint ? p.src_hi : p.tgt_hi;
  for (int j = 0; j < p.d; ++j) {
    g.slo[j] = slo[j];
    g.sD[j] = shi[j] - slo[j];
    g.tlo[j] = tlo[j];
    g.tD[j] = thi[j] - tlo[j];
  }
  for (int k = 0; k < p.q; ++k) g.z[k] = p.z[k];
  return g;
}

struct Layout {
  size_t w, keys, keys_sorted, idx, perm, offs, tocc, tmp, total;
  size_t tmp_bytes;
};

int layout(const bfly_plan_s& p, int64_t n_in, int nrhs, int prec, Layout* out) {
  bfly::Geo g = make_geo(p, false);
  size_t tmp_bytes = 0;
  hipError_t e = bfly::sort_storage_bytes(n_in, p.d * p.L, &tmp_bytes);
  if (e != hipSuccess) return fail(BFLY_EDEVICE, "sort storage query failed: %s", hipGetErrorString(e));
  const size_t n = (size_t)(n_in > 0 ? n_in : 0);
  const size_t P = (size_t)1 << (p.d * p.L);
  Layout L;
  size_t off = 0;
  L.w = off;
  off += up(bfly::weight_bytes(g, nrhs, prec));
  L.keys = off;
  off += up(4 * n);
  L.keys_sorted = off;
  off += up(4 * n);
  L.idx = 0;  // the single-apply sort numbers the points itself
  L.perm = off;
  off += up(4 * n);
  L.offs = off;
  off += up(4 * (P + 2));  // offsets, then the empty-leaf flag
  L.tocc = off;
  off += up(bfly::tocc_bytes(p.d, p.L));
  L.tmp = off;
  off += up(tmp_bytes);
  L.total = off;
  L.tmp_bytes = tmp_bytes;
  *out = L;
  return BFLY_OK;
}

// FP64 and FP32 are implemented; SPLIT32 is a valid mode that the library
// does not provide (see include/bfly.h)
int check_prec(int prec) {
  if (prec == BFLY_SPLIT32)
    return fail(BFLY_EUNSUPPORTED,
                "precision mode SPLIT32 is not implemented: on gfx950 a double-float multiply-add (18 FP32 "
                "instructions) is about 7x slower than an FP64 one, so the FP64 mode serves that accuracy");
  if (prec != BFLY_FP64 && prec != BFLY_FP32) return fail(BFLY_EINVAL, "unknown precision mode %d", prec);
  return BFLY_OK;
}

int check_plan(const bfly_plan_s* p) {
  if (!p) return fail(BFLY_EINVAL, "plan is NULL");
  return BFLY_OK;
}

// The workspace of one apply, carved into its pieces.
bfly::Work carve(const bfly_plan_s& p, const Layout& L, void* ws) {
  char* base = static_cast<char*>(ws);
  bfly::Work w;
  w.W = base + L.w;
  w.keys = reinterpret_cast<uint32_t*>(base + L.keys);
  w.keys_sorted = reinterpret_cast<uint32_t*>(base + L.keys_sorted);
  w.idx = nullptr;
  w.perm = reinterpret_cast<int32_t*>(base + L.perm);
  w.offs = reinterpret_cast<int32_t*>(base + L.offs);
  w.empty = w.offs + ((int64_t)1 << (p.d * p.L)) + 1;
  w.tocc = reinterpret_cast<uint8_t*>(base + L.tocc);
  w.sort_tmp = base + L.tmp;
  w.sort_tmp_bytes = L.tmp_bytes;
  return w;
}

int check_sticky() {
  hipError_t e = hipPeekAtLastError();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(BFLY_EDEVICE, "earlier device work failed: %s", hipGetErrorString(e));
  }
  return BFLY_OK;
}

// ---- workspace of bfly_apply_noalloc ----
// For callers that cannot allocate device memory: the workspace of an apply
// lives in this array, one copy per GPU (the runtime places it in each
// device's memory when the library's code is loaded there; it stays until
// the process ends).  Host code never uses the array's name as an address:
// its device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocBytes = BFLY_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
int scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(BFLY_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(BFLY_EDEVICE, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(BFLY_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BFLY_OK;
}

// One apply after host-side validation.  ws == nullptr with noalloc = true
// takes the workspace from the library's device array (bfly_apply_noalloc).
int apply_common(bfly_plan_t plan, bool adjoint, int64_t n_in, const double* pin, const void* vin,
                 int64_t ldin, int64_t n_out, const double* pout, void* vout, int64_t ldout, int nrhs,
                 int prec, void* ws, size_t ws_bytes, void* stream, bool noalloc = false) {
  if (int rc = check_plan(plan)) return rc;
  const char* nin = adjoint ? "n_tgt" : "n_src";
  const char* nout = adjoint ? "n_src" : "n_tgt";
  if (n_in < 0 || n_in >= ((int64_t)1 << 31)) return fail(BFLY_EINVAL, "%s out of range", nin);
  if (n_out < 0 || n_out >= ((int64_t)1 << 31)) return fail(BFLY_EINVAL, "%s out of range", nout);
  if (nrhs < 1 || nrhs > 4096) return fail(BFLY_EINVAL, "nrhs must be in [1, 4096]");
  if (int rc = check_prec(prec)) return rc;
  if (ldin < n_in || ldin < 1) return fail(BFLY_EINVAL, "leading dimension of the input < number of inputs");
  if (ldout < n_out || ldout < 1) return fail(BFLY_EINVAL, "leading dimension of the output < number of outputs");
  if (n_in > 0 && (!pin || !vin)) return fail(BFLY_EINVAL, "input points or values are NULL");
  if (n_out > 0 && (!pout || !vout)) return fail(BFLY_EINVAL, "output points or values are NULL");
  Layout L;
  if (int rc = layout(*plan, n_in, nrhs, prec, &L)) return rc;
  if (noalloc) {
    if (L.total > kNoAllocBytes)
      return fail(BFLY_EWORKSPACE, "apply needs %zu bytes of workspace; bfly_apply_noalloc holds at most %zu",
                  L.total, kNoAllocBytes);
    if (int rc = scratch_of_current_device(&ws)) return rc;
    ws_bytes = kNoAllocBytes;
  }
  if (!ws || ws_bytes < L.total)
    return fail(BFLY_EWORKSPACE, "workspace of %zu bytes given, %zu required", ws ? ws_bytes : (size_t)0,
                L.total);
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(BFLY_EINVAL, "workspace must be 256-byte aligned");
  if (int rc = check_sticky()) return rc;
  bfly::Work w = carve(*plan, L, ws);
  bfly::Geo g = make_geo(*plan, adjoint);
  hipError_t e = bfly::run_apply(g, prec, n_in, pin, static_cast<const double*>(vin), ldin, n_out, pout,
                                 static_cast<double*>(vout), ldout, nrhs, w, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(BFLY_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return ok();
}

// ---- autotuning (bfly_tune) ----

// All ways of covering n stages by launches of 1..kmax stages each.
void compositions(int n, int kmax, std::vector<int>& cur, std::vector<std::vector<int>>& out) {
  if (n == 0) {
    out.push_back(cur);
    return;
  }
  for (int k = 1; k <= std::min(n, kmax); ++k) {
    cur.push_back(k);
    compositions(n - k, kmax, cur, out);
    cur.pop_back();
  }
}

// The greedy cover: launches of kmax stages, the last one shorter.
std::vector<int> greedy(int n, int kmax) {
  std::vector<int> v;
  for (int l = 0; l < n; l += kmax) v.push_back(std::min(kmax, n - l));
  return v;
}

bfly::TuneParams with_split(bfly::TuneParams p, const std::vector<int>& a, const std::vector<int>& b) {
  p.nsplit = 0;
  for (int k : a)
    if (p.nsplit < 16) p.split[p.nsplit++] = k;
  for (int k : b)
    if (p.nsplit < 16) p.split[p.nsplit++] = k;
  return p;
}

int tune_common(bfly_plan_t plan, int adjoint, int64_t n_in, const double* pin, const void* vin, int64_t ldin,
                int64_t n_out, const double* pout, void* vout, int64_t ldout, int nrhs, int prec, void* ws,
                size_t ws_bytes, double max_ms, double* best_ms, void* stream) {
  if (adjoint != 0 && adjoint != 1) return fail(BFLY_EINVAL, "adjoint must be 0 or 1");
  if (!(max_ms >= 0.0)) return fail(BFLY_EINVAL, "max_ms must be >= 0");
  // validation and one apply with the current shapes (also a warm-up)
  if (int rc = apply_common(plan, adjoint != 0, n_in, pin, vin, ldin, n_out, pout, vout, ldout, nrhs, prec, ws,
                            ws_bytes, stream))
    return rc;
  Layout L;
  if (int rc = layout(*plan, n_in, nrhs, prec, &L)) return rc;
  const bfly::Work w = carve(*plan, L, ws);
  const bfly::Geo g = make_geo(*plan, adjoint != 0);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  bfly::ShapeLimits lim;
  hipError_t e = bfly::shape_limits(g, prec, &lim);
  if (e != hipSuccess) return fail(BFLY_EDEVICE, "shape query failed: %s", hipGetErrorString(e));
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess) {
    if (ev0) (void)hipEventDestroy(ev0);
    return fail(BFLY_EDEVICE, "hipEventCreate failed");
  }
  double spent = 0.0;
  int reps = 3;
  // time per apply of one candidate (a warm-up apply, then reps applies)
  auto measure = [&](const bfly::TuneParams& p, double* ms) -> hipError_t {
    hipError_t err = bfly::run_apply(g, prec, n_in, pin, static_cast<const double*>(vin), ldin, n_out, pout,
                                     static_cast<double*>(vout), ldout, nrhs, w, st, &p);
    if (err == hipSuccess) err = hipEventRecord(ev0, st);
    for (int i = 0; i < reps && err == hipSuccess; ++i)
      err = bfly::run_apply(g, prec, n_in, pin, static_cast<const double*>(vin), ldin, n_out, pout,
                            static_cast<double*>(vout), ldout, nrhs, w, st, &p);
    if (err == hipSuccess) err = hipEventRecord(ev1, st);
    if (err == hipSuccess) err = hipEventSynchronize(ev1);
    float t = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, ev0, ev1);
    *ms = (double)t / reps;
    spent += (double)t * (reps + 1) / reps;
    return err;
  };
  bfly::TuneParams best;  // all zero: the built-in shapes
  double best_t = 0.0;
  e = measure(best, &best_t);
  if (e == hipSuccess && best_t < 1.0) {  // short applies: more repetitions against timer noise
    reps = 10;
    e = measure(best, &best_t);
  }
  // a candidate replaces the best only if it is faster by more than the noise
  auto consider = [&](const bfly::TuneParams& p) {
    if (e != hipSuccess || (max_ms > 0.0 && spent >= max_ms)) return;
    double t = 0.0;
    e = measure(p, &t);
    if (e == hipSuccess && t < best_t * 0.995) {
      best = p;
      best_t = t;
    }
  };
  const bool chunked = lim.rc > 1 && nrhs >= lim.rc;
  const int kmax = chunked ? lim.kmax_rc : lim.kmax_one;
  if (g.ls > 0) {
    // stages per launch: every cover of the column-space half with the
    // built-in row-space cover, then every cover of the row-space half with
    // the best column-space one (the built-in covers take launches of kcol /
    // krow stages, the last shorter)
    std::vector<std::vector<int>> col, row;
    std::vector<int> cur;
    compositions(g.ls, kmax, cur, col);
    compositions(g.L - g.ls, kmax, cur, row);
    std::vector<int> col_best = greedy(g.ls, chunked ? lim.kcol_rc : lim.kcol_one);
    const std::vector<int> row0 = greedy(g.L - g.ls, chunked ? lim.krow_rc : lim.krow_one);
    for (const auto& c : col) {
      const double before = best_t;
      consider(with_split(best, c, row0));
      if (best_t < before) col_best = c;
    }
    for (const auto& r : row) consider(with_split(best, col_best, r));
  }
  // units per workgroup block, per launch kind
  for (int ub : {1, 2, 3, 4, 6, 8}) {
    bfly::TuneParams p = best;
    p.ub_first = ub;
    consider(p);
  }
  for (int ub : {1, 2, 3, 4, 6, 8}) {
    bfly::TuneParams p = best;
    p.ub_second = ub;
    consider(p);
  }
  // one right-hand side per workgroup instead of chunks
  if (lim.rc > 1 && nrhs >= lim.rc) {
    bfly::TuneParams p = best;
    p.rc_one = 1;
    consider(p);
  }
  // leave the chosen shapes' result in the outputs
  if (e == hipSuccess)
    e = bfly::run_apply(g, prec, n_in, pin, static_cast<const double*>(vin), ldin, n_out, pout,
                        static_cast<double*>(vout), ldout, nrhs, w, st, &best);
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (e != hipSuccess) return fail(BFLY_EDEVICE, "tuning run failed: %s", hipGetErrorString(e));
  e = bfly::tune_store(g, nrhs, prec, best, best_t);
  if (e != hipSuccess) return fail(BFLY_EINVAL, "could not write the tuning cache (BFLY_TUNE_CACHE)");
  if (best_ms) *best_ms = best_t;
  return ok();
}

// ---- batched applies ----

// An instance of at least this many leaves fills the GPU by itself (its
// narrowest launch has thousands of workgroups): a batched apply runs it as a
// single apply, in order on the stream, and batches only the smaller ones
// level-synchronously.  (MI355X, 48 hyperbolic-Radon instances with N from
// 128 to 1024 and 8 right-hand sides: level-synchronous launches over all of
// them were 2-4% slower than back-to-back single applies, the small
// instances' weights no longer staying in cache from one launch to the next.)
constexpr uint64_t kSoloLeaves = (uint64_t)1 << 14;

bool solo(const bfly_batch_item& it) { return ((uint64_t)1 << (it.plan->d * it.plan->L)) >= kSoloLeaves; }

struct BLayout {
  std::vector<size_t> w;     // weights of each instance
  std::vector<uint32_t> leafbase;  // first key of each batched (not solo) instance
  size_t keys = 0, keys_sorted = 0, idx = 0, perm = 0, offs = 0, desc = 0, tmp = 0, total = 0, tmp_bytes = 0;
  int64_t n_small = 0;       // input points of the batched instances (the one sort)
  uint64_t leaves = 0;       // leaves of the batched instances (its key space)
  int bits = 0;              // key bits of that sort
};

int check_item(const bfly_batch_item& it, int k) {
  if (int rc = check_plan(it.plan)) return fail(rc, "item %d: plan is NULL", k);
  if (it.adjoint != 0 && it.adjoint != 1) return fail(BFLY_EINVAL, "item %d: adjoint must be 0 or 1", k);
  if (it.nrhs < 1 || it.nrhs > 4096) return fail(BFLY_EINVAL, "item %d: nrhs must be in [1, 4096]", k);
  if (it.n_in < 0 || it.n_in >= ((int64_t)1 << 31)) return fail(BFLY_EINVAL, "item %d: n_in out of range", k);
  if (it.n_out < 0 || it.n_out >= ((int64_t)1 << 31)) return fail(BFLY_EINVAL, "item %d: n_out out of range", k);
  if (it.ld_in < it.n_in || it.ld_in < 1) return fail(BFLY_EINVAL, "item %d: ld_in < n_in", k);
  if (it.ld_out < it.n_out || it.ld_out < 1) return fail(BFLY_EINVAL, "item %d: ld_out < n_out", k);
  if (it.n_in > 0 && (!it.pts_in || !it.in)) return fail(BFLY_EINVAL, "item %d: input points or values are NULL", k);
  if (it.n_out > 0 && (!it.pts_out || !it.out))
    return fail(BFLY_EINVAL, "item %d: output points or values are NULL", k);
  return BFLY_OK;
}

int batch_layout(int n, const bfly_batch_item* items, int prec, BLayout* out) {
  if (n < 1 || n > 4096) return fail(BFLY_EINVAL, "n_items must be in [1, 4096]");
  if (!items) return fail(BFLY_EINVAL, "items is NULL");
  if (int rc = check_prec(prec)) return rc;
  BLayout L;
  size_t off = 0;
  uint64_t leaves_all = 0;
  int64_t n_all = 0;
  // the point and leaf buffers are shared in stream order: the instances run
  // as single applies use them one after another (their own n and N^d), then
  // the batched instances use them together (one key space)
  int64_t n_max = 0;
  uint64_t leaves_max = 0;
  for (int k = 0; k < n; ++k) {
    if (int rc = check_item(items[k], k)) return rc;
    const bfly_plan_s& p = *items[k].plan;
    L.w.push_back(off);
    off += up(bfly::weight_bytes(make_geo(p, items[k].adjoint != 0), items[k].nrhs, prec));
    const uint64_t P = (uint64_t)1 << (p.d * p.L);
    leaves_all += P;
    n_all += items[k].n_in;
    if (leaves_all > ((uint64_t)1 << 31)) return fail(BFLY_EINVAL, "total leaves of the batch exceed 2^31");
    if (n_all >= ((int64_t)1 << 31)) return fail(BFLY_EINVAL, "total input points of the batch reach 2^31");
    if (solo(items[k])) {
      L.leafbase.push_back(0);
      n_max = std::max(n_max, items[k].n_in);
      leaves_max = std::max(leaves_max, P);
    } else {
      L.leafbase.push_back((uint32_t)L.leaves);
      L.leaves += P;
      L.n_small += items[k].n_in;
    }
  }
  n_max = std::max(n_max, L.n_small);
  leaves_max = std::max(leaves_max, L.leaves);
  while (L.bits < 32 && ((uint64_t)1 << L.bits) < L.leaves) ++L.bits;
  // sort scratch: the batched sort of n_small keys, and each single apply's
  // own sort (the scratch size is not monotone in n: the tile size changes)
  hipError_t e = bfly::sort_storage_bytes(L.n_small, L.bits, &L.tmp_bytes);
  if (e != hipSuccess) return fail(BFLY_EDEVICE, "sort storage query failed: %s", hipGetErrorString(e));
  for (int k = 0; k < n; ++k) {
    if (!solo(items[k])) continue;
    size_t b = 0;
    e = bfly::sort_storage_bytes(items[k].n_in, items[k].plan->d * items[k].plan->L, &b);
    if (e != hipSuccess) return fail(BFLY_EDEVICE, "sort storage query failed: %s", hipGetErrorString(e));
    L.tmp_bytes = std::max(L.tmp_bytes, b);
  }
  const size_t nt = (size_t)n_max;
  L.keys = off;
  off += up(4 * nt);
  L.keys_sorted = off;
  off += up(4 * nt);
  L.idx = off;
  off += up(4 * nt);
  L.perm = off;
  off += up(4 * nt);
  L.offs = off;
  off += up(4 * (leaves_max + 2));  // offsets, then the empty-leaf flag
  L.desc = off;
  off += up(2 * (size_t)n * sizeof(bfly::ItemDesc));
  L.tmp = off;
  off += up(L.tmp_bytes);
  L.total = off;
  *out = std::move(L);
  return BFLY_OK;
}

int apply_batched(int n, const bfly_batch_item* items, int prec, void* ws, size_t ws_bytes, void* stream) {
  BLayout L;
  if (int rc = batch_layout(n, items, prec, &L)) return rc;
  if (!ws || ws_bytes < L.total)
    return fail(BFLY_EWORKSPACE, "workspace of %zu bytes given, %zu required", ws ? ws_bytes : (size_t)0,
                L.total);
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(BFLY_EINVAL, "workspace must be 256-byte aligned");
  if (int rc = check_sticky()) return rc;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  bfly::Work w;
  w.keys = reinterpret_cast<uint32_t*>(base + L.keys);
  w.keys_sorted = reinterpret_cast<uint32_t*>(base + L.keys_sorted);
  w.idx = reinterpret_cast<int32_t*>(base + L.idx);
  w.perm = reinterpret_cast<int32_t*>(base + L.perm);
  w.offs = reinterpret_cast<int32_t*>(base + L.offs);
  w.empty = w.offs + L.leaves + 1;
  w.sort_tmp = base + L.tmp;
  w.sort_tmp_bytes = L.tmp_bytes;
  std::vector<bfly::Geo> geo(n);
  std::vector<bfly::BinInst> bins;
  std::vector<bfly::BatchInst> inst;
  int64_t n_small = 0;
  hipError_t e = hipSuccess;
  for (int k = 0; k < n && e == hipSuccess; ++k) {
    const bfly_batch_item& it = items[k];
    geo[k] = make_geo(*it.plan, it.adjoint != 0);
    if (solo(it)) {
      // a single apply on the shared buffers (in stream order, before the
      // batched instances reuse them)
      bfly::Work ws1 = w;
      ws1.W = base + L.w[k];
      ws1.idx = nullptr;
      ws1.empty = w.offs + ((int64_t)1 << (it.plan->d * it.plan->L)) + 1;
      ws1.tocc = nullptr;
      e = bfly::run_apply(geo[k], prec, it.n_in, it.pts_in, static_cast<const double*>(it.in), it.ld_in, it.n_out,
                          it.pts_out, static_cast<double*>(it.out), it.ld_out, it.nrhs, ws1, st);
      continue;
    }
    bins.emplace_back();
    inst.emplace_back();
    n_small += it.n_in;
    bins.back().pts = it.pts_in;
    bins.back().n = it.n_in;
    bins.back().G = &geo[k];
    bins.back().leafbase = L.leafbase[k];
    bfly::BatchInst& b = inst.back();
    b.G = geo[k];
    b.W = base + L.w[k];
    b.nrhs = it.nrhs;
    b.pts_in = it.pts_in;
    b.vals_in = static_cast<const double*>(it.in);
    b.ld_in = it.ld_in;
    b.offs = w.offs + L.leafbase[k];
    b.n_out = it.n_out;
    b.pts_out = it.pts_out;
    b.vals_out = static_cast<double*>(it.out);
    b.ld_out = it.ld_out;
  }
  if (e != hipSuccess) return fail(BFLY_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  if (inst.empty()) return ok();
  const int nb = (int)inst.size();
  if (n_small != L.n_small) return fail(BFLY_EINVAL, "internal: batched point count mismatch");
  e = bfly::bin_batch(bins.data(), nb, n_small, L.leaves, w, st);
  if (e != hipSuccess) return fail(BFLY_EDEVICE, "binning launch failed: %s", hipGetErrorString(e));
  // groups of instances sharing d, q, phase and direction, in order of first appearance
  std::vector<int> done(nb, 0);
  int desc_next = 0;
  for (int k = 0; k < nb && e == hipSuccess; ++k) {
    if (done[k]) continue;
    std::vector<bfly::BatchInst> grp;
    for (int j = k; j < nb; ++j) {
      const bfly::Geo& a = inst[k].G;
      const bfly::Geo& b = inst[j].G;
      if (!done[j] && a.d == b.d && a.q == b.q && a.phase == b.phase && a.adj == b.adj) {
        grp.push_back(inst[j]);
        done[j] = 1;
      }
    }
    bfly::BatchGroup bg;
    bg.inst = grp.data();
    bg.n = (int)grp.size();
    bg.perm = w.perm;
    bg.empty = w.empty;
    bg.desc = reinterpret_cast<bfly::ItemDesc*>(base + L.desc) + desc_next;
    bg.stream = st;
    bfly::tune_batch_from_env(bg);
    desc_next += 2 * bg.n;
    const int d = grp[0].G.d;
    e = d == 1 ? bfly::run_batch_d1(bg, prec) : (d == 2 ? bfly::run_batch_d2(bg, prec) : bfly::run_batch_d3(bg, prec));
  }
  if (e != hipSuccess) return fail(BFLY_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return ok();
}

}  // namespace

extern "C" {

int bfly_plan(int d, int64_t N, const double* src_lo, const double* src_hi, const double* tgt_lo,
              const double* tgt_hi, int phase_id, int q, bfly_plan_t* out) {
  if (!out) return fail(BFLY_EINVAL, "out is NULL");
  *out = nullptr;
  if (d < 1 || d > 3) return fail(BFLY_EINVAL, "d must be 1, 2 or 3 (got %d)", d);
  if (N < 1 || (N & (N - 1)) != 0) return fail(BFLY_EINVAL, "N must be a power of two >= 1");
  int L = 0;
  while (((int64_t)1 << L) < N) ++L;
  if ((int64_t)d * L > 30) return fail(BFLY_EINVAL, "N^d must be below 2^31");
  if (q < 2 || q > q_max(d)) return fail(BFLY_EINVAL, "q must be in [2, %d] for d = %d", q_max(d), d);
  if (!src_lo || !src_hi || !tgt_lo || !tgt_hi) return fail(BFLY_EINVAL, "box corner pointer is NULL");
  for (int j = 0; j < d; ++j) {
    if (!std::isfinite(src_lo[j]) || !std::isfinite(src_hi[j]) || !(src_hi[j] > src_lo[j]))
      return fail(BFLY_EINVAL, "source box must be finite with hi > lo in every dimension");
    if (!std::isfinite(tgt_lo[j]) || !std::isfinite(tgt_hi[j]) || !(tgt_hi[j] > tgt_lo[j]))
      return fail(BFLY_EINVAL, "target box must be finite with hi > lo in every dimension");
  }
  if (phase_id < 0 || phase_id > 4) return fail(BFLY_EINVAL, "unknown phase id %d", phase_id);
  if (phase_id == BFLY_PHASE_HYPRADON2 && d != 2) return fail(BFLY_EUNSUPPORTED, "HYPRADON2 needs d = 2");
  if (phase_id == BFLY_PHASE_GENRADON3 && d != 3) return fail(BFLY_EUNSUPPORTED, "GENRADON3 needs d = 3");
  if (phase_id == BFLY_PHASE_GENRADON3_PI && d != 3)
    return fail(BFLY_EUNSUPPORTED, "GENRADON3_PI needs d = 3");
  bfly_plan_s* p = new (std::nothrow) bfly_plan_s;
  if (!p) return fail(BFLY_ENOMEM, "plan allocation failed");
  p->d = d;
  p->N = N;
  p->L = L;
  p->q = q;
  p->r = 1;
  for (int j = 0; j < d; ++j) p->r *= q;
  p->phase = phase_id;
  for (int j = 0; j < d; ++j) {
    p->src_lo[j] = src_lo[j];
    p->src_hi[j] = src_hi[j];
    p->tgt_lo[j] = tgt_lo[j];
    p->tgt_hi[j] = tgt_hi[j];
  }
  // Chebyshev nodes of the first kind (the grid of Sec. 1.4), stored exactly
  // antisymmetric, z[q-1-k] = -z[k] (the level kernels use the reflection)
  for (int k = 0; k < q; ++k) p->z[k] = std::cos((double)(2 * k + 1) * M_PI / (double)(2 * q));
  for (int k = 0; k < q / 2; ++k) p->z[q - 1 - k] = -p->z[k];
  if (q % 2) p->z[q / 2] = 0.0;
  *out = p;
  return ok();
}

int bfly_plan_destroy(bfly_plan_t plan) {
  delete plan;
  return ok();
}

int bfly_plan_info(bfly_plan_t plan, int64_t* out5) {
  if (int rc = check_plan(plan)) return rc;
  if (!out5) return fail(BFLY_EINVAL, "out is NULL");
  out5[0] = plan->d;
  out5[1] = plan->N;
  out5[2] = plan->q;
  out5[3] = plan->r;
  out5[4] = plan->L / 2;
  return ok();
}

int bfly_workspace_size(bfly_plan_t plan, int64_t n_in, int nrhs, int prec, size_t* bytes) {
  if (int rc = check_plan(plan)) return rc;
  if (!bytes) return fail(BFLY_EINVAL, "bytes is NULL");
  if (n_in < 0 || n_in >= ((int64_t)1 << 31)) return fail(BFLY_EINVAL, "n_in out of range");
  if (nrhs < 1 || nrhs > 4096) return fail(BFLY_EINVAL, "nrhs must be in [1, 4096]");
  if (int rc = check_prec(prec)) return rc;
  Layout L;
  if (int rc = layout(*plan, n_in, nrhs, prec, &L)) return rc;
  *bytes = L.total;
  return ok();
}

int bfly_apply(bfly_plan_t plan, int64_t n_src, const double* y, const void* g, int64_t ldg, int64_t n_tgt,
               const double* x, void* f, int64_t ldf, int nrhs, int prec, void* ws, size_t ws_bytes,
               void* stream) {
  return apply_common(plan, false, n_src, y, g, ldg, n_tgt, x, f, ldf, nrhs, prec, ws, ws_bytes, stream);
}

int bfly_apply_noalloc(bfly_plan_t plan, int64_t n_src, const double* y, const void* g, int64_t ldg, int64_t n_tgt,
                       const double* x, void* f, int64_t ldf, int nrhs, int prec, void* stream) {
  return apply_common(plan, false, n_src, y, g, ldg, n_tgt, x, f, ldf, nrhs, prec, nullptr, 0, stream, true);
}

int bfly_apply_adjoint(bfly_plan_t plan, int64_t n_tgt, const double* x, const void* f_in, int64_t ldf,
                       int64_t n_src, const double* y, void* g_out, int64_t ldg, int nrhs, int prec, void* ws,
                       size_t ws_bytes, void* stream) {
  return apply_common(plan, true, n_tgt, x, f_in, ldf, n_src, y, g_out, ldg, nrhs, prec, ws, ws_bytes, stream);
}

int bfly_batch_workspace_size(int n_items, const bfly_batch_item* items, int prec, size_t* bytes) {
  if (!bytes) return fail(BFLY_EINVAL, "bytes is NULL");
  BLayout L;
  if (int rc = batch_layout(n_items, items, prec, &L)) return rc;
  *bytes = L.total;
  return ok();
}

int bfly_apply_batched(int n_items, const bfly_batch_item* items, int prec, void* ws, size_t ws_bytes,
                       void* stream) {
  return apply_batched(n_items, items, prec, ws, ws_bytes, stream);
}

int bfly_tune(bfly_plan_t plan, int adjoint, int64_t n_in, const double* pts_in, const void* in, int64_t ld_in,
              int64_t n_out, const double* pts_out, void* out, int64_t ld_out, int nrhs, int prec, void* ws,
              size_t ws_bytes, double max_ms, double* best_ms, void* stream) {
  return tune_common(plan, adjoint, n_in, pts_in, in, ld_in, n_out, pts_out, out, ld_out, nrhs, prec, ws, ws_bytes,
                     max_ms, best_ms, stream);
}

int bfly_tune_reset(void) {
  bfly::tune_clear();
  return ok();
}

int bfly_timing_enable(int on) {
  bfly::timing_set(on != 0);
  return ok();
}

int bfly_timing_read(double* ms, int64_t* launches, int64_t* stages, int64_t* inits, int64_t* switches) {
  if (!ms || !launches || !stages || !inits || !switches) return fail(BFLY_EINVAL, "output arrays are NULL");
  hipError_t e = bfly::timing_read(ms, launches, stages, inits, switches);
  if (e != hipSuccess) return fail(BFLY_EDEVICE, "timing events failed: %s", hipGetErrorString(e));
  return ok();
}

int bfly_timing_launches(int cap, int* count, int* kind, int* stages, int* inits, int* switches, double* ms) {
  if (cap < 0 || !count) return fail(BFLY_EINVAL, "cap < 0 or count is NULL");
  if (cap > 0 && (!kind || !stages || !inits || !switches || !ms)) return fail(BFLY_EINVAL, "output arrays are NULL");
  std::vector<bfly::LaunchRecord> rec((size_t)cap);
  const int n = bfly::timing_launches(cap, rec.data());
  for (int i = 0; i < n && i < cap; ++i) {
    kind[i] = rec[i].kind;
    stages[i] = rec[i].stages;
    inits[i] = rec[i].inits;
    switches[i] = rec[i].switches;
    ms[i] = rec[i].ms;
  }
  *count = n;
  return ok();
}

const char* bfly_status_string(int status) {
  switch (status) {
    case BFLY_OK:
      return "success";
    case BFLY_EINVAL:
      return "invalid argument";
    case BFLY_EUNSUPPORTED:
      return "unsupported configuration";
    case BFLY_ENOMEM:
      return "host allocation failed";
    case BFLY_EDEVICE:
      return "device error";
    case BFLY_EWORKSPACE:
      return "workspace too small";
    default:
      return "unknown status";
  }
}

const char* bfly_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
