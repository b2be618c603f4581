// Host side of the C ABI (include/nmf.h): argument validation, the workspace
// plan, the one-time set-up of A (CSR copy, transposed copy, SpMM work plans),
// and the launch sequence of every ALS iteration.  All device work is done by
// the kernels in k_*.hip; nothing here computes the factorization.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <atomic>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "nmf_internal.h"

using namespace nmfk;

namespace {

thread_local std::string g_create_error = "no error";

nmf_status fail(nmf_handle* h, nmf_status st, const std::string& msg) {
  if (h)
    h->last_error = msg;
  else
    g_create_error = msg;
  return st;
}

#define HIPCHK(h, expr)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail((h), NMF_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool is_device_ptr(const void* p) {
  if (p == nullptr) return false;
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  const hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged ||
         attr.type == hipMemoryTypeUnified;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Sequential carve-up of the workspace; the same walk sizes it (base == 0).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(char* b) : base(b) {}
  template <typename P>
  P* take(size_t count) {
    off = align_up(off, 256);
    P* p = base ? reinterpret_cast<P*>(base + off) : nullptr;
    off += count * sizeof(P);
    return p;
  }
};

struct PlanSizes {
  int64_t items, heavy, parts;
};

PlanSizes plan_bounds(int64_t rows, int64_t nnz) {
  const int64_t chunks = (nnz + kChunk - 1) / kChunk;
  return PlanSizes{rows + 2 * chunks + 1, chunks + 1, 2 * chunks + 1};
}

struct HostPlan {
  std::vector<WorkItem> items;
  std::vector<int32_t> rows, nchunks, part0;
  int32_t parts = 0;
};

// Work items for one orientation: groups of up to max_rows consecutive
// short rows (total at most kChunk nonzeros), and kChunk-long pieces of
// every longer row.
HostPlan build_plan(const int64_t* rp, int64_t rows, int max_rows) {
  HostPlan p;
  int64_t r = 0;
  while (r < rows) {
    const int64_t len = rp[r + 1] - rp[r];
    if (len > kChunk) {
      const int32_t nch = static_cast<int32_t>((len + kChunk - 1) / kChunk);
      const int32_t hidx = static_cast<int32_t>(p.nchunks.size());
      p.rows.push_back(static_cast<int32_t>(r));
      p.nchunks.push_back(nch);
      p.part0.push_back(p.parts);
      for (int32_t j = 0; j < nch; ++j) {
        WorkItem w;
        w.r0 = static_cast<int32_t>(r);
        w.r1 = static_cast<int32_t>(r + 1);
        w.p0 = rp[r] + static_cast<int64_t>(j) * kChunk;
        w.p1 = std::min(rp[r + 1], w.p0 + kChunk);
        w.heavy = hidx;
        w.part = p.parts + j;
        p.items.push_back(w);
      }
      p.parts += nch;
      ++r;
      continue;
    }
    const int64_t start = r;
    int64_t total = 0;
    while (r < rows && r - start < max_rows) {
      const int64_t l = rp[r + 1] - rp[r];
      if (l > kChunk || (r > start && total + l > kChunk)) break;
      total += l;
      ++r;
    }
    WorkItem w;
    w.r0 = static_cast<int32_t>(start);
    w.r1 = static_cast<int32_t>(r);
    w.p0 = rp[start];
    w.p1 = rp[r];
    w.heavy = -1;
    w.part = -1;
    p.items.push_back(w);
  }
  return p;
}

struct Layout {
  size_t bytes = 0;
};

// Assign every device buffer of a handle (h may be a dummy when sizing).
size_t carve(nmf_handle* h, char* base, const nmf_config& c, int64_t nnz, const PlanSizes& pa,
             const PlanSizes& pt) {
  Carver cv(base);
  const int64_t n = c.n, m = c.m;
  const int k = c.k;
  const size_t elt = c.dtype == NMF_F64 ? 8 : 4;
  const size_t cand = c.dtype == NMF_F64 ? 16 : 8;
  const int64_t rmax = std::max(n, m);
  const int mw = (k + 31) / 32;
  // A and its transpose
  h->planA.rows = n;
  h->planA.rowptr = cv.take<int64_t>(n + 1);
  h->planA.col = cv.take<int32_t>(nnz);
  h->planA.val = cv.take<char>(nnz * elt);
  h->planAt.rows = m;
  h->planAt.rowptr = cv.take<int64_t>(m + 1);
  // (the fused V-half kernel's stream is padded: see vh_stream_cap)
  const int64_t nnz_at = vhalf_fits(elt, n, m, k, nnz) ? vh_stream_cap(m, nnz) : nnz;
  h->planAt.col = cv.take<int32_t>(nnz_at);
  h->planAt.val = cv.take<char>(nnz_at * elt);
  // per term: its nonzeros in the V-half stream (the gathered-entry count)
  h->planAt.sdf = cv.take<int32_t>(n);
  if (vhalf_fits(elt, n, m, k, nnz)) h->planAt.warm_col = cv.take<int32_t>(kMaxWarm);
  // room for the V half's hot block when one can exist (the fused V-half
  // kernel serves the problem and the flag is not set): see do_create
  if (vhalf_fits(elt, n, m, k, nnz) && !(c.flags & NMF_FLAG_NO_HOT)) {
    const int hot_max = static_cast<int>(std::min<int64_t>(kMaxHot, (n + 15) / 16 * 16));
    h->planAt.hot_col = cv.take<int32_t>(kMaxHot);
    h->planAt.hot = cv.take<char>(m * hot_max * elt);
  }
  for (int o = 0; o < 2; ++o) {
    Plan& p = o == 0 ? h->planA : h->planAt;
    const PlanSizes& s = o == 0 ? pa : pt;
    p.items = cv.take<WorkItem>(s.items);
    p.heavy_row = cv.take<int32_t>(s.heavy);
    p.heavy_nchunks = cv.take<int32_t>(s.heavy);
    p.heavy_part0 = cv.take<int32_t>(s.heavy);
    p.partials = cv.take<char>(s.parts * k * elt);
  }
  auto factor = [&](Factor& f, int64_t rows) {
    f.rows = rows;
    f.row_ptr = cv.take<int32_t>(rows + 1);
    f.topic = cv.take<uint8_t>(rows * k);
    f.val = cv.take<char>(rows * k * elt);
    f.slot = cv.take<int32_t>(rows);
    f.rowid = cv.take<int32_t>(rows);
    // U's copy, when the fused V-half kernel reads it, needs only 16-byte
    // groups: k rounded up to 4 (a smaller working set for the L2s)
    f.ld = (vhalf_fits(elt, n, m, k, nnz) && &f != &h->V) ? (k + 3) / 4 * 4 : dense_ld(k, elt);
    f.dense = cv.take<char>(rows * f.ld * elt);
    f.counts = cv.take<int32_t>(4);
    f.meta = cv.take<int2>(rows);
    f.packed = cv.take<char>(rows * k * 2 * elt);
    f.rowtab = cv.take<int2>((rows + 31) / 32);
  };
  factor(h->U[0], n);
  factor(h->U[1], n);
  factor(h->V, m);
  h->vpre = cv.take<char>(m * k * elt);
  h->upre = cv.take<char>(n * k * elt);
  h->cbuf = cv.take<char>(n * k * elt);
  h->lossB = cv.take<char>(m * k * elt);
  h->lossC = cv.take<char>(n * k * elt);
  h->sel.hist = cv.take<uint32_t>(static_cast<size_t>(k) * kBins);
  h->sel.sel = cv.take<ColSel>(k);
  // candidate lists: per column kSelSub sub-lists, each with room for all
  // the candidates of the collect blocks that append to it
  const int64_t nsel = (rmax + kSelBlockRows - 1) / kSelBlockRows;
  h->sel.cand_sub = (nsel + kSelSub - 1) / kSelSub * kSelBlockRows;
  h->sel.cand_stride = kSelSub * h->sel.cand_sub;
  h->sel.cand_cnt = cv.take<int32_t>(static_cast<size_t>(k) * kSelSub * kCntStride);
  h->sel.candA = cv.take<char>(static_cast<size_t>(k) * h->sel.cand_stride * cand);
  h->sel.candB = cv.take<char>(static_cast<size_t>(k) * h->sel.cand_stride * cand);
  h->sel.mask = cv.take<uint32_t>(rmax * mw);
  h->sel.ticket = cv.take<int32_t>(16);
  h->sel.scan_part = cv.take<int32_t>(2 * ((rmax + 255) / 256 + 1));
  h->gram_partials = cv.take<char>(static_cast<size_t>(kGramBlocks) * k * (k + 1) / 2 * elt);
  h->gram_ticket = cv.take<int32_t>(4);
  h->gU.G = cv.take<double>(static_cast<size_t>(k) * k);
  h->gU.W = cv.take<double>(static_cast<size_t>(k) * k);
  h->gU.dead = cv.take<int32_t>(4);
  h->gV.G = cv.take<double>(static_cast<size_t>(k) * k);
  h->gV.W = cv.take<double>(static_cast<size_t>(k) * k);
  h->gV.dead = cv.take<int32_t>(4);
  h->lossG = cv.take<double>(2 * static_cast<size_t>(k) * k);
  h->met.partials = cv.take<double>(kMetricBlocks * 4);
  h->met.ticket = cv.take<int32_t>(4);
  h->met.ring = cv.take<double>(static_cast<size_t>(kHistRing) * H_FIELDS);
  h->met.it = cv.take<int64_t>(1);
  h->met.max_nnz = cv.take<int64_t>(1);
  h->met.nA2 = cv.take<double>(1);
  h->met.loss_parts = cv.take<double>(kMetricBlocks);
  h->met.out = cv.take<double>(4);
  h->met.gathered = cv.take<unsigned long long>(2 * kGathSlots);
  h->status = cv.take<int32_t>(4);
  h->scratch_i = cv.take<int32_t>(4);
  return align_up(cv.off, 256);
}

nmf_status check_config(const nmf_config* c) {
  if (c == nullptr) return fail(nullptr, NMF_ERR_INVALID_ARG, "config is NULL");
  if (c->n < 1 || c->m < 1) return fail(nullptr, NMF_ERR_INVALID_ARG, "n and m must be >= 1");
  // row indices and per-row offsets are held in 32 bits
  if (c->n >= (int64_t(1) << 29) || c->m >= (int64_t(1) << 29))
    return fail(nullptr, NMF_ERR_UNSUPPORTED, "n and m must be below 2^29");
  if (c->k < 1) return fail(nullptr, NMF_ERR_INVALID_ARG, "k must be >= 1");
  if (c->k > kMaxK) return fail(nullptr, NMF_ERR_UNSUPPORTED, "k must be <= 128");
  if (c->k > c->n || c->k > c->m) return fail(nullptr, NMF_ERR_INVALID_ARG, "k must be <= min(n, m)");
  if (c->t_u < 1 || c->t_v < 1) return fail(nullptr, NMF_ERR_INVALID_ARG, "t_u and t_v must be >= 1");
  if (c->mode != NMF_MODE_COLUMN && c->mode != NMF_MODE_NONE && c->mode != NMF_MODE_WHOLE)
    return fail(nullptr, NMF_ERR_UNSUPPORTED, "mode not supported");
  if (c->dtype != NMF_F32 && c->dtype != NMF_F64) return fail(nullptr, NMF_ERR_UNSUPPORTED, "dtype");
  // int32 element offsets into the k-wide matrices, and 32-bit byte offsets
  // into the dense factor copies the SpMM gathers from
  const int64_t elt = c->dtype == NMF_F32 ? 4 : 8;
  const int64_t ld = dense_ld(c->k, elt);
  if (c->n * ld * elt >= (int64_t(1) << 32) || c->m * ld * elt >= (int64_t(1) << 32))
    return fail(nullptr, NMF_ERR_UNSUPPORTED, "a dense factor (rows x k, k padded to 64 bytes) must be below 4 GiB");
  return NMF_OK;
}

// Host work of handle creation split over threads: f(part, begin, end) for
// `parts` consecutive ranges given by bounds[0..parts] (the last range on the
// calling thread; a range whose thread cannot be started runs inline).
template <class F>
void par_ranges(const std::vector<int64_t>& bounds, F&& f) {
  const int parts = static_cast<int>(bounds.size()) - 1;
  std::vector<std::thread> th;
  for (int t = 0; t < parts; ++t) {
    const int64_t b = bounds[t], e = bounds[t + 1];
    if (t + 1 == parts) {
      f(t, b, e);
      break;
    }
    try {
      th.emplace_back([&f, t, b, e] { f(t, b, e); });
    } catch (...) {
      f(t, b, e);
    }
  }
  for (auto& x : th) x.join();
}

// Threads for host work over `work` elements: one per 2^20, at most the
// hardware's, at most 32.
int host_parts(int64_t work) {
  const int64_t hw = std::max<unsigned>(1u, std::thread::hardware_concurrency());
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>({hw, int64_t{32}, work >> 20})));
}

// [0, n) in `parts` equal ranges.
std::vector<int64_t> even_bounds(int64_t n, int parts) {
  std::vector<int64_t> b(parts + 1);
  for (int t = 0; t <= parts; ++t) b[t] = n * t / parts;
  return b;
}

// Rows [0, n) in `parts` ranges of about equal nonzero counts (row pointer rp).
std::vector<int64_t> nnz_bounds(const int64_t* rp, int64_t n, int parts) {
  std::vector<int64_t> b(parts + 1);
  b[0] = 0;
  b[parts] = n;
  for (int t = 1; t < parts; ++t) {
    const int64_t want = rp[n] / parts * t;
    b[t] = std::max(b[t - 1], static_cast<int64_t>(std::lower_bound(rp, rp + n + 1, want) - rp));
    b[t] = std::min(b[t], n);
  }
  return b;
}

template <typename T>
bool values_ok(const T* v, int64_t count, bool* any_pos) {
  bool pos = false;
  for (int64_t i = 0; i < count; ++i) {
    const T x = v[i];
    if (!(x >= T(0)) || !std::isfinite(x)) return false;
    if (x > T(0)) pos = true;
  }
  if (any_pos) *any_pos = pos;
  return true;
}

template <typename T>
bool values_ok_par(const T* v, int64_t count, bool* any_pos) {
  const int parts = host_parts(count);
  std::vector<char> ok(parts, 1), pos(parts, 0);
  par_ranges(even_bounds(count, parts), [&](int t, int64_t b, int64_t e) {
    bool p = false;
    ok[t] = values_ok(v + b, e - b, &p) ? 1 : 0;
    pos[t] = p ? 1 : 0;
  });
  bool all = true, any = false;
  for (int t = 0; t < parts; ++t) {
    all = all && ok[t];
    any = any || pos[t];
  }
  if (any_pos) *any_pos = any;
  return all;
}

// host <- or -> device copy on the handle's stream, then wait
nmf_status copy_sync(nmf_handle* h, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return NMF_OK;
  HIPCHK(h, hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return NMF_OK;
}

nmf_status sync_status(nmf_handle* h) {
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int32_t st = 0;
  HIPCHK(h, hipMemcpy(&st, h->status, sizeof(st), hipMemcpyDeviceToHost));
  if (st == NMF_ERR_NOT_SPD) return fail(h, NMF_ERR_NOT_SPD, "Gram matrix is not positive definite");
  if (st == NMF_ERR_NONFINITE) return fail(h, NMF_ERR_NONFINITE, "non-finite value (e.g. ||U|| = 0)");
  if (st != 0) return fail(h, static_cast<nmf_status>(st), "device error");
  return NMF_OK;
}

// ---- stage timing: events in a pool; interval i = (event i-1, event i)
constexpr size_t kProfPool = 1024;

nmf_status prof_fold(nmf_handle* h) {
  if (h->prof_used == 0) return NMF_OK;
  HIPCHK(h, hipEventSynchronize(h->prof_ev[h->prof_used - 1]));
  for (size_t i = 1; i < h->prof_used; ++i) {
    const int st = h->prof_stage[i];
    if (st < 0) continue;
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, h->prof_ev[i - 1], h->prof_ev[i]));
    h->prof_ms[st] += ms;
    h->prof_cnt[st] += 1;
  }
  h->prof_used = 0;
  return NMF_OK;
}

// A mark where stage `closing` ends and stage `next` begins (-1: none).  An
// event is recorded only where a bracketed stage (one in prof_mask) ends or
// begins, so unbracketed stages run back to back; an opening mark directly
// after the mark that already opened the same stage records nothing.
nmf_status prof_mark(nmf_handle* h, int closing, int next) {
  if (!h->prof_on) return NMF_OK;
  const bool close = closing >= 0 && ((h->prof_mask >> closing) & 1u);
  const bool open = next >= 0 && ((h->prof_mask >> next) & 1u);
  if (closing < 0 && next == h->prof_open) return NMF_OK;
  if (!close && !open) {
    h->prof_open = -2;
    return NMF_OK;
  }
  if (h->prof_used == kProfPool) {
    nmf_status s = prof_fold(h);
    if (s != NMF_OK) return s;
  }
  HIPCHK(h, hipEventRecord(h->prof_ev[h->prof_used], h->stream));
  // an interval counts only when its first event opened the stage it closes
  h->prof_stage[h->prof_used] = (close && h->prof_used > 0 && h->prof_open == closing) ? closing : -1;
  ++h->prof_used;
  h->prof_open = open ? next : -2;
  return NMF_OK;
}

#define PROF(h, st, nx)                            \
  do {                                             \
    nmf_status ps_ = prof_mark((h), (st), (nx));   \
    if (ps_ != NMF_OK) return ps_;                 \
  } while (0)

// Load a dense rows x k factor (host or device) into a stored factor.
// A factor's gather metadata follows the SpMM that gathers it: U is gathered
// by the V half (threshold sparse_row[0]), V by the U half (sparse_row[1]).
int sparse_row_of(const nmf_handle* h, const Factor& f) {
  if (&f == &h->V) return h->sparse_row[1];
  return h->use_vhalf ? 0 : h->sparse_row[0];
}

template <typename T>
nmf_status load_factor(nmf_handle* h, const void* src, Factor& f) {
  const size_t bytes = static_cast<size_t>(f.rows) * h->k * sizeof(T);
  T* stage = static_cast<T*>(h->sel.candB);
  if (!is_device_ptr(src)) {
    if (!values_ok(static_cast<const T*>(src), f.rows * h->k, nullptr))
      return fail(h, NMF_ERR_INVALID_INPUT, "factor has a negative or non-finite value");
    nmf_status s = copy_sync(h, stage, src, bytes);
    if (s != NMF_OK) return s;
  } else {
    HIPCHK(h, hipMemcpyAsync(stage, src, bytes, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemsetAsync(h->scratch_i, 0, sizeof(int32_t), h->stream));
    HIPCHK(h, check_input<T>(h, stage, f.rows * h->k, h->scratch_i));
    int32_t flag = 0;
    HIPCHK(h, hipMemcpyAsync(&flag, h->scratch_i, sizeof(flag), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (flag) return fail(h, NMF_ERR_INVALID_INPUT, "factor has a negative or non-finite value");
  }
  HIPCHK(h, mark_nonzero<T>(h, stage, f.rows));
  HIPCHK(h, repack<T>(h, stage, f.rows, f, sparse_row_of(h, f)));
  return NMF_OK;
}

template <typename T>
nmf_status refresh_max(nmf_handle* h) {
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int32_t cu[4] = {0}, cv[4] = {0};
  HIPCHK(h, hipMemcpy(cu, h->U[h->cur_u].counts, sizeof(cu), hipMemcpyDeviceToHost));
  HIPCHK(h, hipMemcpy(cv, h->V.counts, sizeof(cv), hipMemcpyDeviceToHost));
  int64_t cur = static_cast<int64_t>(cu[0]) + (h->have_v ? cv[0] : 0);
  int64_t old = 0;
  HIPCHK(h, hipMemcpy(&old, h->met.max_nnz, sizeof(old), hipMemcpyDeviceToHost));
  if (cur > old) HIPCHK(h, hipMemcpy(h->met.max_nnz, &cur, sizeof(cur), hipMemcpyHostToDevice));
  return NMF_OK;
}

// `next`: the stage enqueued after this half (-1: none), for the profiling marks.
template <typename T>
nmf_status v_half(nmf_handle* h, int next) {
  Factor& U = h->U[h->cur_u];
  T* vpre = static_cast<T*>(h->vpre);
  PROF(h, -1, NMF_STAGE_SPMM_V);
  HIPCHK(h, spmm<T>(h, h->planAt, U, h->gU.W, vpre, nullptr, false, nullptr, h->sparse_row[0], h->wide[0], h->waves[0]));
  PROF(h, NMF_STAGE_SPMM_V, NMF_STAGE_SELECT_V);
  HIPCHK(h, select_topt<T>(h, vpre, h->m, h->cfg.t_v, h->cfg.mode, h->V));
  PROF(h, NMF_STAGE_SELECT_V, NMF_STAGE_REPACK_V);
  HIPCHK(h, repack<T>(h, vpre, h->m, h->V, sparse_row_of(h, h->V)));
  PROF(h, NMF_STAGE_REPACK_V, NMF_STAGE_GRAM_V);
  HIPCHK(h, gram<T>(h, h->V, h->gV));
  PROF(h, NMF_STAGE_GRAM_V, next);
  h->have_v = true;
  h->have_pre_v = true;
  return NMF_OK;
}

template <typename T>
nmf_status u_half(nmf_handle* h, bool keep_c, int next) {
  const int nxt = 1 - h->cur_u;
  Factor& Un = h->U[nxt];
  T* upre = static_cast<T*>(h->upre);
  PROF(h, -1, NMF_STAGE_SPMM_U);
  HIPCHK(h, spmm<T>(h, h->planA, h->V, h->gV.W, upre, keep_c ? static_cast<T*>(h->cbuf) : nullptr,
                    false, nullptr, h->sparse_row[1], h->wide[1], h->waves[1]));
  PROF(h, NMF_STAGE_SPMM_U, NMF_STAGE_SELECT_U);
  HIPCHK(h, select_topt<T>(h, upre, h->n, h->cfg.t_u, h->cfg.mode, Un));
  PROF(h, NMF_STAGE_SELECT_U, NMF_STAGE_REPACK_U);
  HIPCHK(h, repack<T>(h, upre, h->n, Un, sparse_row_of(h, Un)));
  PROF(h, NMF_STAGE_REPACK_U, NMF_STAGE_GRAM_U);
  HIPCHK(h, gram<T>(h, Un, h->gU));
  PROF(h, NMF_STAGE_GRAM_U, next);
  h->have_pre_u = true;
  return NMF_OK;
}

template <typename T>
nmf_status refresh_w(nmf_handle* h) {
  if (!h->w_stale) return NMF_OK;
  HIPCHK(h, gram<T>(h, h->U[h->cur_u], h->gU));
  h->w_stale = false;
  return NMF_OK;
}

template <typename T>
nmf_status do_steps(nmf_handle* h, int32_t iters) {
  const bool rec = !(h->cfg.flags & NMF_FLAG_NO_METRICS);
  if (iters > 0) {
    nmf_status s = refresh_w<T>(h);
    if (s != NMF_OK) return s;
  }
  h->prof_open = -2;
  for (int32_t i = 0; i < iters; ++i) {
    nmf_status s = v_half<T>(h, NMF_STAGE_SPMM_U);
    if (s != NMF_OK) return s;
    s = u_half<T>(h, rec, NMF_STAGE_METRICS);
    if (s != NMF_OK) return s;
    const int nxt = 1 - h->cur_u;
    HIPCHK(h, metrics<T>(h, h->U[nxt], h->U[h->cur_u], rec ? static_cast<T*>(h->cbuf) : nullptr, rec));
    PROF(h, NMF_STAGE_METRICS, i + 1 < iters ? NMF_STAGE_SPMM_V : -1);
    h->cur_u = nxt;
    ++h->iters_done;
    h->metrics_valid = rec;
  }
  return NMF_OK;
}

template <typename T>
nmf_status do_create(nmf_handle* h, const int64_t* rp_in, const int32_t* col_in, const void* val_in,
                     const void* u0, const void* v0) {
  const int64_t n = h->n, m = h->m, nnz = h->nnz;
  // A on the host for validation, the transpose and the work plans (the
  // loops over nonzeros run on host threads, each over a range of rows)
  std::unique_ptr<int64_t[]> rp_h;
  std::unique_ptr<int32_t[]> col_h;
  std::unique_ptr<T[]> val_h;
  const int64_t* rp = rp_in;
  const int32_t* col = col_in;
  const T* val = static_cast<const T*>(val_in);
  if (is_device_ptr(rp_in)) {
    rp_h.reset(new (std::nothrow) int64_t[n + 1]);
    if (!rp_h) return fail(h, NMF_ERR_DEVICE, "out of host memory");
    HIPCHK(h, hipMemcpy(rp_h.get(), rp_in, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    rp = rp_h.get();
  }
  if (rp[0] != 0 || rp[n] != nnz) return fail(h, NMF_ERR_INVALID_ARG, "row pointer must start at 0 and end at nnz");
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) return fail(h, NMF_ERR_INVALID_ARG, "row pointer decreases");
  if (nnz > 0 && is_device_ptr(col_in)) {
    col_h.reset(new (std::nothrow) int32_t[nnz]);
    if (!col_h) return fail(h, NMF_ERR_DEVICE, "out of host memory");
    HIPCHK(h, hipMemcpy(col_h.get(), col_in, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    col = col_h.get();
  }
  if (nnz > 0 && is_device_ptr(val_in)) {
    val_h.reset(new (std::nothrow) T[nnz]);
    if (!val_h) return fail(h, NMF_ERR_DEVICE, "out of host memory");
    HIPCHK(h, hipMemcpy(val_h.get(), val_in, nnz * sizeof(T), hipMemcpyDeviceToHost));
    val = val_h.get();
  }
  const int parts = host_parts(nnz);
  const std::vector<int64_t> rows_of = nnz_bounds(rp, n, parts);  // each part's rows
  {
    // 1: a column out of range, 2: not increasing (the first row that fails decides)
    std::vector<int64_t> bad_row(parts, n);
    std::vector<int> bad_kind(parts, 0);
    par_ranges(rows_of, [&](int t, int64_t b, int64_t e) {
      for (int64_t i = b; i < e && bad_kind[t] == 0; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
          const int32_t j = col[p];
          if (j < 0 || j >= m) {
            bad_kind[t] = 1;
            bad_row[t] = i;
            break;
          }
          if (p > rp[i] && j <= col[p - 1]) {
            bad_kind[t] = 2;
            bad_row[t] = i;
            break;
          }
        }
    });
    for (int t = 0; t < parts; ++t) {
      if (bad_kind[t] == 1) return fail(h, NMF_ERR_INVALID_ARG, "column index out of range");
      if (bad_kind[t] == 2) return fail(h, NMF_ERR_INVALID_ARG, "column indices not strictly increasing in a row");
    }
  }
  bool any_pos = false;
  if (!values_ok_par(val, nnz, &any_pos)) return fail(h, NMF_ERR_INVALID_INPUT, "A has a negative or non-finite value");
  if (!any_pos) return fail(h, NMF_ERR_INVALID_INPUT, "||A|| = 0");
  // hot terms (float32): rows of A with at least kHotDensity * m nonzeros,
  // most nonzeros first (ties: lower row), at most kMaxHot; their entries
  // leave the V-half stream for a dense docs x hot block
  std::vector<int32_t> hot;
  if (vhalf_fits(sizeof(T), n, m, h->k, nnz) && !(h->cfg.flags & NMF_FLAG_NO_HOT)) {
    const int64_t need = std::max<int64_t>(kHotMinNnz, static_cast<int64_t>(std::ceil(kHotDensity * m)));
    for (int64_t i = 0; i < n; ++i)
      if (rp[i + 1] - rp[i] >= need) hot.push_back(static_cast<int32_t>(i));
    std::stable_sort(hot.begin(), hot.end(),
                     [&](int32_t a, int32_t b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; });
    if (hot.size() > static_cast<size_t>(kMaxHot)) hot.resize(kMaxHot);
  }
  const int n_hot = static_cast<int>(hot.size());
  const int hot_ld = (n_hot + 15) / 16 * 16;
  std::vector<int32_t> hot_of(n_hot ? n : 0, -1);
  for (int x = 0; x < n_hot; ++x) hot_of[hot[x]] = x;
  // warm terms (fused V-half kernel): the most frequent of the rest, at
  // least kHotMinNnz nonzeros each, most first (ties: lower row), at most
  // kMaxWarm; their rows of U are read from LDS
  std::vector<int32_t> warm;
  if (h->use_vhalf) {
    for (int64_t i = 0; i < n; ++i)
      if ((!n_hot || hot_of[i] < 0) && rp[i + 1] - rp[i] >= kHotMinNnz) warm.push_back(static_cast<int32_t>(i));
    std::stable_sort(warm.begin(), warm.end(),
                     [&](int32_t a, int32_t b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; });
    // as many as the kernel's LDS holds beside its hot rows, W and U's row table
    const int64_t base = (static_cast<int64_t>(hot_ld) * 64 * 4 + static_cast<int64_t>(h->k) * h->k * 8 +
                          (n + 31) / 32 * 8 + 15) / 16 * 16;
    const int64_t room = std::max<int64_t>(0, (int64_t{160} * 1024 - base) / (64 * 4));
    if (static_cast<int64_t>(warm.size()) > std::min<int64_t>(kMaxWarm, room))
      warm.resize(static_cast<size_t>(std::min<int64_t>(kMaxWarm, room)));
  }
  std::vector<int32_t> warm_of(warm.empty() ? 0 : n, -1);
  for (size_t w = 0; w < warm.size(); ++w) warm_of[warm[w]] = static_cast<int32_t>(w);
  std::vector<T> hot_block(static_cast<size_t>(n_hot ? m : 0) * hot_ld, T(0));
  // transpose of the rest (stable counting sort: rows ascending within each
  // column); for the fused V-half kernel every document's run is padded to
  // a multiple of four with term -1, value 0.  Each part counts its rows'
  // nonzeros per column; a part's entries of column j then start at the
  // column's start plus the earlier parts' counts, so the result does not
  // depend on the number of parts.
  const bool skip_hot = n_hot > 0;
  // per part: its count, then its offset, per column (allocated here: the
  // worker threads allocate nothing)
  std::vector<std::vector<int32_t>> pc(parts, std::vector<int32_t>(m, 0));
  par_ranges(rows_of, [&](int t, int64_t b, int64_t e) {
    int32_t* c = pc[t].data();
    for (int64_t i = b; i < e; ++i)
      if (!skip_hot || hot_of[i] < 0)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) ++c[col[p]];
  });
  std::vector<int64_t> cp(m + 1, 0);
  const int cparts = host_parts(m * static_cast<int64_t>(parts) * 4);
  const std::vector<int64_t> cols_of = even_bounds(m, cparts);
  par_ranges(cols_of, [&](int, int64_t b, int64_t e) {
    for (int64_t j = b; j < e; ++j) {
      int64_t c = 0;
      for (int t = 0; t < parts; ++t) {
        const int32_t x = pc[t][j];
        pc[t][j] = static_cast<int32_t>(c);  // within-column offset of part t (a column holds < 2^29)
        c += x;
      }
      cp[j + 1] = h->use_vhalf ? (c + 3) & ~int64_t{3} : c;
    }
  });
  for (int64_t j = 0; j < m; ++j) cp[j + 1] += cp[j];
  const int64_t nnz_t = cp[m];
  std::unique_ptr<int32_t[]> crow_p(new (std::nothrow) int32_t[nnz_t > 0 ? nnz_t : 1]);
  std::unique_ptr<T[]> cval_p(new (std::nothrow) T[nnz_t > 0 ? nnz_t : 1]);
  if (!crow_p || !cval_p) return fail(h, NMF_ERR_DEVICE, "out of host memory");
  int32_t* crow = crow_p.get();
  T* cval = cval_p.get();
  par_ranges(rows_of, [&](int t, int64_t b, int64_t e) {
    int32_t* off = pc[t].data();
    for (int64_t i = b; i < e; ++i) {
      const int x = skip_hot ? hot_of[i] : -1;
      for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
        const int32_t j = col[p];
        if (x >= 0) {
          hot_block[static_cast<size_t>(j) * hot_ld + x] = val[p];
          continue;
        }
        const int64_t q = cp[j] + off[j]++;
        crow[q] = (!warm.empty() && warm_of[i] >= 0) ? -2 - warm_of[i] : static_cast<int32_t>(i);
        cval[q] = val[p];
      }
    }
  });
  if (h->use_vhalf) {
    // each document's padding after its own entries (the last part's
    // offset has reached the column's count)
    par_ranges(cols_of, [&](int, int64_t b, int64_t e) {
      for (int64_t j = b; j < e; ++j)
        for (int64_t q = cp[j] + pc[parts - 1][j]; q < cp[j + 1]; ++q) {
          crow[q] = -1;
          cval[q] = T(0);
        }
    });
  }
  // rows per light item = the epilogue row group of the SpMM instantiation
  const int group = spmm_row_group(h->k);
  HostPlan pa = build_plan(rp, n, group);
  // (the fused V-half kernel needs no work items)
  HostPlan pt = h->use_vhalf ? HostPlan{} : build_plan(cp.data(), m, group);
  const PlanSizes ba = plan_bounds(n, nnz), bt = plan_bounds(m, nnz);
  if (static_cast<int64_t>(pa.items.size()) > ba.items || static_cast<int64_t>(pt.items.size()) > bt.items ||
      pa.parts > ba.parts || pt.parts > bt.parts)
    return fail(h, NMF_ERR_WORKSPACE, "internal: work plan exceeds its bound");
  auto upload_plan = [&](Plan& p, const HostPlan& hp) -> nmf_status {
    p.n_items = static_cast<int32_t>(hp.items.size());
    p.n_heavy = static_cast<int32_t>(hp.nchunks.size());
    p.n_parts = hp.parts;
    HIPCHK(h, hipMemcpy(p.items, hp.items.data(), hp.items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    if (!hp.nchunks.empty()) {
      HIPCHK(h, hipMemcpy(p.heavy_nchunks, hp.nchunks.data(), hp.nchunks.size() * 4, hipMemcpyHostToDevice));
      HIPCHK(h, hipMemcpy(p.heavy_part0, hp.part0.data(), hp.part0.size() * 4, hipMemcpyHostToDevice));
      HIPCHK(h, hipMemcpy(p.heavy_row, hp.rows.data(), hp.rows.size() * 4, hipMemcpyHostToDevice));
    }
    return NMF_OK;
  };
  nmf_status s;
  if ((s = upload_plan(h->planA, pa)) != NMF_OK) return s;
  if ((s = upload_plan(h->planAt, pt)) != NMF_OK) return s;
  HIPCHK(h, hipMemcpy(h->planA.rowptr, rp, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->planAt.rowptr, cp.data(), (m + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->planA.col, col, nnz * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->planA.val, val, nnz * sizeof(T), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->planAt.col, crow, nnz_t * sizeof(int32_t), hipMemcpyHostToDevice));
  h->planA.nnz = nnz;
  h->planAt.nnz = nnz_t;
  HIPCHK(h, hipMemcpy(h->planAt.val, cval, nnz_t * sizeof(T), hipMemcpyHostToDevice));
  if (h->use_vhalf) {
    // the fused V-half kernel's four spare entries past the padded stream
    // (its aligned reads at a document's end reach them): no term, value 0
    HIPCHK(h, hipMemset(h->planAt.col + nnz_t, 0xFF, 4 * sizeof(int32_t)));
    HIPCHK(h, hipMemset(static_cast<char*>(h->planAt.val) + nnz_t * sizeof(T), 0, 4 * sizeof(T)));
  }
  if (n_hot && (h->planAt.hot == nullptr || h->planAt.hot_col == nullptr))
    return fail(h, NMF_ERR_WORKSPACE, "internal: no room for the hot block");
  h->planAt.n_hot = n_hot;
  h->planAt.hot_ld = hot_ld;
  h->planAt.n_warm = static_cast<int32_t>(warm.size());
  if (!warm.empty())
    HIPCHK(h, hipMemcpy(h->planAt.warm_col, warm.data(), warm.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  {
    // each term's nonzeros in the V-half stream (hot terms: none)
    std::vector<int32_t> sdf(n);
    for (int64_t i = 0; i < n; ++i)
      sdf[i] = (n_hot && hot_of[i] >= 0) ? 0 : static_cast<int32_t>(rp[i + 1] - rp[i]);
    HIPCHK(h, hipMemcpy(h->planAt.sdf, sdf.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  if (n_hot) {
    HIPCHK(h, hipMemcpy(h->planAt.hot_col, hot.data(), n_hot * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->planAt.hot, hot_block.data(), hot_block.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  // state that must start at zero
  const int k = h->k;
  HIPCHK(h, hipMemset(h->sel.hist, 0, static_cast<size_t>(k) * kBins * 4));
  HIPCHK(h, hipMemset(h->sel.cand_cnt, 0, static_cast<size_t>(k) * kSelSub * kCntStride * 4));
  HIPCHK(h, hipMemset(h->sel.mask, 0, static_cast<size_t>(std::max(n, m)) * h->mask_words * 4));
  HIPCHK(h, hipMemset(h->sel.ticket, 0, 16 * 4));
  HIPCHK(h, hipMemset(h->gram_ticket, 0, 16));
  HIPCHK(h, hipMemset(h->met.ticket, 0, 16));
  HIPCHK(h, hipMemset(h->met.it, 0, 8));
  HIPCHK(h, hipMemset(h->met.max_nnz, 0, 8));
  HIPCHK(h, hipMemset(h->met.gathered, 0, 2 * kGathSlots * sizeof(unsigned long long)));
  HIPCHK(h, hipMemset(h->status, 0, 16));
  HIPCHK(h, hipMemset(h->gU.dead, 0, 16));
  HIPCHK(h, hipMemset(h->gV.dead, 0, 16));
  for (int f = 0; f < 3; ++f) {
    Factor& F = f < 2 ? h->U[f] : h->V;
    HIPCHK(h, hipMemset(F.counts, 0, 16));
  }
  HIPCHK(h, sum_squares<T>(h, static_cast<const T*>(h->planA.val), nnz, h->met.nA2));
  // initial factors
  if ((s = load_factor<T>(h, u0, h->U[0])) != NMF_OK) return s;
  if ((s = load_factor<T>(h, u0, h->U[1])) != NMF_OK) return s;
  h->cur_u = 0;
  if (v0 != nullptr) {
    if ((s = load_factor<T>(h, v0, h->V)) != NMF_OK) return s;
    h->have_v = true;
    HIPCHK(h, gram<T>(h, h->V, h->gV));
  }
  HIPCHK(h, gram<T>(h, h->U[0], h->gU));
  if ((s = refresh_max<T>(h)) != NMF_OK) return s;
  return sync_status(h);
}

template <typename T>
nmf_status do_error(nmf_handle* h, double* E) {
  if (!h->have_v) return fail(h, NMF_ERR_STATE, "no V yet: take a step or pass v0");
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  if (h->metrics_valid && h->iters_done > 0) {
    int64_t it = 0;
    HIPCHK(h, hipMemcpy(&it, h->met.it, 8, hipMemcpyDeviceToHost));
    double rec[H_FIELDS];
    HIPCHK(h, hipMemcpy(rec, h->met.ring + ((it - 1) % kHistRing) * H_FIELDS, sizeof(rec), hipMemcpyDeviceToHost));
    *E = rec[H_E];
    return NMF_OK;
  }
  // on demand: C = A V (raw), then ||A||^2 - 2 <U, C> + <G_U, G_V>
  T* C = static_cast<T*>(h->cbuf);
  HIPCHK(h, spmm<T>(h, h->planA, h->V, nullptr, C, nullptr, true, nullptr, h->sparse_row[1]));
  HIPCHK(h, densify<T>(h, h->U[h->cur_u], static_cast<T*>(h->lossC)));
  HIPCHK(h, loss_dot<T>(h, static_cast<const T*>(h->lossC), C, h->gU.G, h->gV.G, h->met.out));
  s = sync_status(h);
  if (s != NMF_OK) return s;
  double L = 0, nA2 = 0;
  HIPCHK(h, hipMemcpy(&L, h->met.out, 8, hipMemcpyDeviceToHost));
  HIPCHK(h, hipMemcpy(&nA2, h->met.nA2, 8, hipMemcpyDeviceToHost));
  *E = std::sqrt(L > 0 ? L : 0.0) / std::sqrt(nA2);
  return NMF_OK;
}

// Sequential ALS (Algorithm 3): blocks of k2 topics, `iters` iterations per
// block, each block starting from the initial guess U0 = the first k2
// columns of U when the call begins.  The handle's factors keep their full
// width k = eta k2 (later blocks' columns zero); every iteration records E
// and R in the history like an iteration of Algorithm 2.
template <typename T>
nmf_status do_sequential(nmf_handle* h, int32_t k2, int32_t iters) {
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  const int k = h->k;
  const int eta = k / k2;
  const bool rec = !(h->cfg.flags & NMF_FLAG_NO_METRICS);
  h->prof_open = -2;
  h->w_stale = true;  // only block inverses are formed: the records carry no conditioning
  T* upre = static_cast<T*>(h->upre);
  T* vpre = static_cast<T*>(h->vpre);
  T* C = static_cast<T*>(h->cbuf);
  T* U0b = static_cast<T*>(h->lossC);                // n x k2: the initial guess of every block
  double* Gb = h->lossG;                             // k2 x k2 block of a Gram matrix
  double* W22 = h->lossG + static_cast<size_t>(k2) * k2;  // its inverse
  HIPCHK(h, densify<T>(h, h->U[h->cur_u], upre));
  HIPCHK(h, seq_save<T>(h, upre, U0b, h->n, k2));
  // With k2 < k the products gather and store only the block's columns.  C
  // (A V, read by the metrics) then keeps in the columns of every finished
  // block what that block's last U half stored there (A V of those columns,
  // which stay fixed); columns of later blocks stay zero.
  const bool window = k2 < k;
  if (window) HIPCHK(h, seq_setup<T>(h, C, nullptr, h->n, 0, 0));  // C <- 0
  for (int b = 0; b < eta; ++b) {
    const int k1 = b * k2;
    // U = [finished blocks | U0 | 0]
    Factor& Uc = h->U[h->cur_u];
    HIPCHK(h, densify<T>(h, Uc, upre));
    HIPCHK(h, seq_setup<T>(h, upre, U0b, h->n, k1, k2));
    HIPCHK(h, mark_nonzero<T>(h, upre, h->n));
    HIPCHK(h, repack<T>(h, upre, h->n, Uc, sparse_row_of(h, Uc)));
    HIPCHK(h, gram_plain<T>(h, Uc, h->gU.G));
    for (int32_t it = 0; it < iters; ++it) {
      Factor& Uo = h->U[h->cur_u];
      const int nxt = 1 - h->cur_u;
      Factor& Un = h->U[nxt];
      // V half: V2 = (A^T U2 - V1 U1^T U2) (U2^T U2)^-1
      const ColWindow win{k1, k2, k, k1};
      PROF(h, -1, NMF_STAGE_SPMM_V);
      // (U[nxt] is rebuilt after the U half's product: until then its buffers
      // hold the narrow copy of U's block columns and the row filter bits)
      if (window)
        HIPCHK(h, spmm_window<T>(h, h->planAt, Uo, vpre, win, h->sparse_row[0], Un));
      else
        HIPCHK(h, spmm<T>(h, h->planAt, Uo, nullptr, vpre, nullptr, true, nullptr, h->sparse_row[0]));
      HIPCHK(h, block_inverse(h, h->gU.G, k1, k2, Gb, W22, h->scratch_i));
      HIPCHK(h, seq_solve<T>(h, vpre, vpre, h->m, h->V, h->gU.G, W22, k1, k2));
      PROF(h, NMF_STAGE_SPMM_V, NMF_STAGE_SELECT_V);
      HIPCHK(h, select_topt<T>(h, vpre, h->m, h->cfg.t_v, h->cfg.mode, h->V));
      PROF(h, NMF_STAGE_SELECT_V, NMF_STAGE_REPACK_V);
      HIPCHK(h, repack<T>(h, vpre, h->m, h->V, sparse_row_of(h, h->V)));
      PROF(h, NMF_STAGE_REPACK_V, NMF_STAGE_GRAM_V);
      HIPCHK(h, gram_plain<T>(h, h->V, h->gV.G));
      HIPCHK(h, seq_max(h, Uo, h->V));
      PROF(h, NMF_STAGE_GRAM_V, NMF_STAGE_SPMM_U);
      // U half: U2 = (A V2 - U1 V1^T V2) (V2^T V2)^-1
      if (window)
        HIPCHK(h, spmm_window<T>(h, h->planA, h->V, C, win, h->sparse_row[1], Un));
      else
        HIPCHK(h, spmm<T>(h, h->planA, h->V, nullptr, C, nullptr, true, nullptr, h->sparse_row[1]));
      HIPCHK(h, block_inverse(h, h->gV.G, k1, k2, Gb, W22, h->scratch_i));
      HIPCHK(h, seq_solve<T>(h, C, upre, h->n, Uo, h->gV.G, W22, k1, k2));
      PROF(h, NMF_STAGE_SPMM_U, NMF_STAGE_SELECT_U);
      HIPCHK(h, select_topt<T>(h, upre, h->n, h->cfg.t_u, h->cfg.mode, Un));
      PROF(h, NMF_STAGE_SELECT_U, NMF_STAGE_REPACK_U);
      HIPCHK(h, repack<T>(h, upre, h->n, Un, sparse_row_of(h, Un)));
      PROF(h, NMF_STAGE_REPACK_U, NMF_STAGE_GRAM_U);
      HIPCHK(h, gram_plain<T>(h, Un, h->gU.G));
      HIPCHK(h, seq_max(h, Un, h->V));
      PROF(h, NMF_STAGE_GRAM_U, NMF_STAGE_METRICS);
      HIPCHK(h, metrics<T>(h, Un, Uo, C, rec));
      PROF(h, NMF_STAGE_METRICS, it + 1 < iters ? NMF_STAGE_SPMM_V : -1);
      h->cur_u = nxt;
      ++h->iters_done;
      h->have_v = h->have_pre_v = h->have_pre_u = true;
      h->metrics_valid = rec;
    }
  }
  h->w_stale = true;  // gU.W / gV.W were not kept up to date
  return NMF_OK;
}

// The top-t rule applied once to the current U and V (their dense forms go
// through the select and the repack of an iteration), then their Gram
// matrices and inverses are rebuilt.
template <typename T>
nmf_status do_enforce(nmf_handle* h, int32_t mode, int64_t t_u, int64_t t_v) {
  if (!h->have_v) return fail(h, NMF_ERR_STATE, "no V yet: take a step or pass v0");
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  Factor& U = h->U[h->cur_u];
  T* xu = static_cast<T*>(h->lossC);  // n x k scratch
  T* xv = static_cast<T*>(h->lossB);  // m x k scratch
  HIPCHK(h, densify<T>(h, U, xu));
  HIPCHK(h, select_topt<T>(h, xu, h->n, t_u, mode, U));
  HIPCHK(h, repack<T>(h, xu, h->n, U, sparse_row_of(h, U)));
  HIPCHK(h, densify<T>(h, h->V, xv));
  HIPCHK(h, select_topt<T>(h, xv, h->m, t_v, mode, h->V));
  HIPCHK(h, repack<T>(h, xv, h->m, h->V, sparse_row_of(h, h->V)));
  HIPCHK(h, gram<T>(h, U, h->gU));
  HIPCHK(h, gram<T>(h, h->V, h->gV));
  h->metrics_valid = false;
  return sync_status(h);
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

nmf_status nmf_workspace_size(const nmf_config* cfg, int64_t nnz, size_t* bytes) {
  nmf_status s = check_config(cfg);
  if (s != NMF_OK) return s;
  if (nnz < 0 || bytes == nullptr) return fail(nullptr, NMF_ERR_INVALID_ARG, "nnz < 0 or bytes NULL");
  nmf_handle dummy;
  dummy.cfg = *cfg;
  *bytes = carve(&dummy, nullptr, *cfg, nnz, plan_bounds(cfg->n, nnz), plan_bounds(cfg->m, nnz));
  return NMF_OK;
}

}  // extern "C"

namespace {

// nmf_create with the workspace already chosen; `caller_ws` asks for the
// checks of a caller's workspace (the static one is known to be device
// memory of the right alignment).
nmf_status create_impl(const nmf_config* cfg, const int64_t* a_rowptr, const int32_t* a_col, const void* a_val,
                       int64_t nnz, const void* u0, const void* v0, void* workspace, size_t ws_bytes,
                       void* hip_stream, nmf_handle** out, bool caller_ws) {
  if (out == nullptr) return fail(nullptr, NMF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  nmf_status s = check_config(cfg);
  if (s != NMF_OK) return s;
  if (a_rowptr == nullptr || (nnz > 0 && (a_col == nullptr || a_val == nullptr)) || u0 == nullptr)
    return fail(nullptr, NMF_ERR_INVALID_ARG, "a required pointer is NULL");
  if (nnz < 1) return fail(nullptr, NMF_ERR_INVALID_INPUT, "||A|| = 0 (no nonzeros)");
  if (nnz >= (int64_t(1) << 40)) return fail(nullptr, NMF_ERR_UNSUPPORTED, "nnz too large");
  size_t need = 0;
  nmf_workspace_size(cfg, nnz, &need);
  if (workspace == nullptr || ws_bytes < need)
    return fail(nullptr, NMF_ERR_WORKSPACE, "workspace smaller than nmf_workspace_size()");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(nullptr, NMF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (caller_ws && !is_device_ptr(workspace))
    return fail(nullptr, NMF_ERR_WORKSPACE, "workspace must be device memory");
  nmf_handle* h = new (std::nothrow) nmf_handle();
  if (h == nullptr) return fail(nullptr, NMF_ERR_DEVICE, "out of host memory");
  h->cfg = *cfg;
  h->n = cfg->n;
  h->m = cfg->m;
  h->k = cfg->k;
  h->nnz = nnz;
  h->elt = cfg->dtype == NMF_F64 ? 8 : 4;
  h->mask_words = (cfg->k + 31) / 32;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->ws = static_cast<char*>(workspace);
  h->ws_bytes = ws_bytes;
  if (hipGetDevice(&h->device) != hipSuccess ||
      hipDeviceGetAttribute(&h->num_cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) {
    delete h;
    return fail(nullptr, NMF_ERR_DEVICE, "no HIP device");
  }
  h->hist_cus = h->num_cus;
  // float32 with k <= 64 (32-bit byte offsets into V_pre): the fused V-half
  // kernel, whose gathers read every nonempty row of U from its compact
  // dense copy
  h->use_vhalf = vhalf_fits(h->elt, h->n, h->m, h->k, nnz);
  if (h->use_vhalf) h->waves[0] = 16;
  if (h->k > 64) {
    // rows twice as wide (two topics per lane): the wide step for the V
    // half, and for the U half rows of up to three entries gathered entry by
    // entry in 16-wave blocks (1M x 5M, k = 100: U half 21.5 -> 17.8 ms,
    // V half 25.9 -> 25.1 ms)
    h->wide[0] = true;
    h->sparse_row[1] = 3;
    h->waves[1] = 16;
  }
  carve(h, h->ws, *cfg, nnz, plan_bounds(cfg->n, nnz), plan_bounds(cfg->m, nnz));
  try {
    s = h->elt == 8 ? do_create<double>(h, a_rowptr, a_col, a_val, u0, v0)
                    : do_create<float>(h, a_rowptr, a_col, a_val, u0, v0);
  } catch (const std::bad_alloc&) {
    s = fail(h, NMF_ERR_DEVICE, "out of host memory");
  } catch (...) {
    s = fail(h, NMF_ERR_DEVICE, "host error while creating the handle");
  }
  if (s != NMF_OK) {
    g_create_error = h->last_error;
    (void)hipStreamSynchronize(h->stream);
    delete h;
    return s;
  }
  *out = h;
  return NMF_OK;
}

}  // namespace

// The static workspace of nmf_create_static: one array per device (each
// GPU the library runs on holds its own copy until the process ends).  Host
// code never passes the array's name to a kernel or a copy: it is a host-side
// stand-in there.  The device address is taken once per device with
// hipGetSymbolAddress, with that device current, and kept in `g_static`.
static __device__ __align__(256) unsigned char scratch[NMF_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxStaticDevices = 64;
struct StaticWorkspace {
  void* ptr = nullptr;    // device address of `scratch` on this device
  bool in_use = false;    // a live handle owns it
};
std::mutex g_static_mu;
StaticWorkspace g_static[kMaxStaticDevices];

}  // namespace

extern "C" {

nmf_status nmf_create(const nmf_config* cfg, const int64_t* a_rowptr, const int32_t* a_col,
                      const void* a_val, int64_t nnz, const void* u0, const void* v0,
                      void* workspace, size_t ws_bytes, void* hip_stream, nmf_handle** out) {
  return create_impl(cfg, a_rowptr, a_col, a_val, nnz, u0, v0, workspace, ws_bytes, hip_stream, out, true);
}

nmf_status nmf_create_static(const nmf_config* cfg, const int64_t* a_rowptr, const int32_t* a_col,
                             const void* a_val, int64_t nnz, const void* u0, const void* v0, void* hip_stream,
                             nmf_handle** out) {
  if (out == nullptr) return fail(nullptr, NMF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  nmf_status s = check_config(cfg);
  if (s != NMF_OK) return s;
  if (nnz < 0) return fail(nullptr, NMF_ERR_INVALID_ARG, "nnz < 0");
  size_t need = 0;
  s = nmf_workspace_size(cfg, nnz, &need);
  if (s != NMF_OK) return s;
  if (need > NMF_STATIC_WORKSPACE_BYTES)
    return fail(nullptr, NMF_ERR_WORKSPACE,
                "problem needs " + std::to_string(need) + " bytes of workspace; the static workspace holds " +
                    std::to_string(static_cast<unsigned long long>(NMF_STATIC_WORKSPACE_BYTES)) +
                    " (use nmf_create with a caller workspace)");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxStaticDevices)
    return fail(nullptr, NMF_ERR_DEVICE, "no HIP device for the static workspace");
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticWorkspace& sw = g_static[dev];
  if (sw.in_use)
    return fail(nullptr, NMF_ERR_STATE,
                "the static workspace of device " + std::to_string(dev) +
                    " belongs to a live handle; destroy that handle first");
  if (sw.ptr == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(nullptr, NMF_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    sw.ptr = p;
  }
  s = create_impl(cfg, a_rowptr, a_col, a_val, nnz, u0, v0, sw.ptr, NMF_STATIC_WORKSPACE_BYTES, hip_stream, out,
                  false);
  if (s == NMF_OK) {
    sw.in_use = true;
    (*out)->static_dev = dev;
  }
  return s;
}

nmf_status nmf_als_step(nmf_handle* h, int32_t iters) {
  if (h == nullptr) return fail(nullptr, NMF_ERR_INVALID_ARG, "handle is NULL");
  if (iters < 0) return fail(h, NMF_ERR_INVALID_ARG, "iters < 0");
  return h->elt == 8 ? do_steps<double>(h, iters) : do_steps<float>(h, iters);
}

nmf_status nmf_half_step(nmf_handle* h, int32_t which) {
  if (h == nullptr) return fail(nullptr, NMF_ERR_INVALID_ARG, "handle is NULL");
  if (which != 0 && which != 1) return fail(h, NMF_ERR_INVALID_ARG, "which must be 0 or 1");
  if (which == 1 && !h->have_v) return fail(h, NMF_ERR_STATE, "no V yet");
  nmf_status s = h->elt == 8 ? refresh_w<double>(h) : refresh_w<float>(h);
  if (s != NMF_OK) return s;
  h->prof_open = -2;
  if (which == 0) {
    s = h->elt == 8 ? v_half<double>(h, -1) : v_half<float>(h, -1);
  } else {
    s = h->elt == 8 ? u_half<double>(h, false, -1) : u_half<float>(h, false, -1);
    if (s == NMF_OK) h->cur_u = 1 - h->cur_u;
  }
  h->metrics_valid = false;
  return s;
}

nmf_status nmf_error(nmf_handle* h, double* E) {
  if (h == nullptr || E == nullptr) return fail(h, NMF_ERR_INVALID_ARG, "NULL argument");
  return h->elt == 8 ? do_error<double>(h, E) : do_error<float>(h, E);
}

nmf_status nmf_residual(nmf_handle* h, double* R) {
  if (h == nullptr || R == nullptr) return fail(h, NMF_ERR_INVALID_ARG, "NULL argument");
  if (h->iters_done == 0) return fail(h, NMF_ERR_STATE, "no iteration completed");
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  int64_t it = 0;
  HIPCHK(h, hipMemcpy(&it, h->met.it, 8, hipMemcpyDeviceToHost));
  if (it == 0) return fail(h, NMF_ERR_STATE, "no iteration completed");
  double rec[H_FIELDS];
  HIPCHK(h, hipMemcpy(rec, h->met.ring + ((it - 1) % kHistRing) * H_FIELDS, sizeof(rec), hipMemcpyDeviceToHost));
  *R = rec[H_R];
  return NMF_OK;
}

nmf_status nmf_history(nmf_handle* h, double* E, double* R, int64_t* nnz_u, int64_t* nnz_v,
                       int32_t cap, int32_t* len) {
  if (h == nullptr || len == nullptr || cap < 0) return fail(h, NMF_ERR_INVALID_ARG, "bad argument");
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  int64_t it = 0;
  HIPCHK(h, hipMemcpy(&it, h->met.it, 8, hipMemcpyDeviceToHost));
  std::vector<double> ring(static_cast<size_t>(kHistRing) * H_FIELDS);
  HIPCHK(h, hipMemcpy(ring.data(), h->met.ring, ring.size() * 8, hipMemcpyDeviceToHost));
  int64_t have = std::min<int64_t>(it, kHistRing);
  int64_t cnt = std::min<int64_t>(have, cap);
  for (int64_t i = 0; i < cnt; ++i) {
    const int64_t idx = (it - cnt + i) % kHistRing;
    const double* r = &ring[idx * H_FIELDS];
    if (E) E[i] = r[H_E];
    if (R) R[i] = r[H_R];
    if (nnz_u) nnz_u[i] = static_cast<int64_t>(r[H_NNZU]);
    if (nnz_v) nnz_v[i] = static_cast<int64_t>(r[H_NNZV]);
  }
  *len = static_cast<int32_t>(cnt);
  return NMF_OK;
}

nmf_status nmf_history_field(nmf_handle* h, int32_t field, double* out, int32_t cap, int32_t* len) {
  static_assert(H_FIELDS == NMF_HIST_NUM_FIELDS, "history record layout");
  if (h == nullptr || out == nullptr || len == nullptr || cap < 0 || field < 0 || field >= H_FIELDS)
    return fail(h, NMF_ERR_INVALID_ARG, "bad argument");
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  int64_t it = 0;
  HIPCHK(h, hipMemcpy(&it, h->met.it, 8, hipMemcpyDeviceToHost));
  std::vector<double> ring(static_cast<size_t>(kHistRing) * H_FIELDS);
  HIPCHK(h, hipMemcpy(ring.data(), h->met.ring, ring.size() * 8, hipMemcpyDeviceToHost));
  const int64_t cnt = std::min<int64_t>(std::min<int64_t>(it, kHistRing), cap);
  for (int64_t i = 0; i < cnt; ++i) out[i] = ring[((it - cnt + i) % kHistRing) * H_FIELDS + field];
  *len = static_cast<int32_t>(cnt);
  return NMF_OK;
}

nmf_status nmf_max_nnz(nmf_handle* h, int64_t* max_nnz_uv) {
  if (h == nullptr || max_nnz_uv == nullptr) return fail(h, NMF_ERR_INVALID_ARG, "NULL argument");
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  HIPCHK(h, hipMemcpy(max_nnz_uv, h->met.max_nnz, 8, hipMemcpyDeviceToHost));
  return NMF_OK;
}

nmf_status nmf_get_factors(nmf_handle* h, void* u_dense, void* v_dense) {
  if (h == nullptr) return fail(nullptr, NMF_ERR_INVALID_ARG, "handle is NULL");
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  for (int f = 0; f < 2; ++f) {
    void* dst = f == 0 ? u_dense : v_dense;
    if (dst == nullptr) continue;
    if (f == 1 && !h->have_v) return fail(h, NMF_ERR_STATE, "no V yet");
    Factor& F = f == 0 ? h->U[h->cur_u] : h->V;
    const size_t bytes = static_cast<size_t>(F.rows) * h->k * h->elt;
    void* stage = is_device_ptr(dst) ? dst : h->sel.candB;
    if (h->elt == 8)
      HIPCHK(h, densify<double>(h, F, static_cast<double*>(stage)));
    else
      HIPCHK(h, densify<float>(h, F, static_cast<float*>(stage)));
    if (stage != dst) {
      s = copy_sync(h, dst, stage, bytes);
      if (s != NMF_OK) return s;
    }
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return NMF_OK;
}

nmf_status nmf_get_sparse(nmf_handle* h, int32_t which, int32_t* row_ptr, uint8_t* topic, void* val,
                          int64_t* nnz) {
  if (h == nullptr || nnz == nullptr || (which != 0 && which != 1))
    return fail(h, NMF_ERR_INVALID_ARG, "bad argument");
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  if (which == 1 && !h->have_v) return fail(h, NMF_ERR_STATE, "no V yet");
  Factor& F = which == 0 ? h->U[h->cur_u] : h->V;
  int32_t counts[4];
  HIPCHK(h, hipMemcpy(counts, F.counts, sizeof(counts), hipMemcpyDeviceToHost));
  *nnz = counts[0];
  if (row_ptr && (s = copy_sync(h, row_ptr, F.row_ptr, (F.rows + 1) * 4)) != NMF_OK) return s;
  if (topic && (s = copy_sync(h, topic, F.topic, counts[0])) != NMF_OK) return s;
  if (val && (s = copy_sync(h, val, F.val, static_cast<size_t>(counts[0]) * h->elt)) != NMF_OK) return s;
  return NMF_OK;
}

nmf_status nmf_set_factors(nmf_handle* h, const void* u, const void* u_prev, const void* v) {
  if (h == nullptr || u == nullptr) return fail(h, NMF_ERR_INVALID_ARG, "handle or u is NULL");
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  const bool f64 = h->elt == 8;
  const int prev = 1 - h->cur_u;
  s = f64 ? load_factor<double>(h, u_prev ? u_prev : u, h->U[prev]) : load_factor<float>(h, u_prev ? u_prev : u, h->U[prev]);
  if (s != NMF_OK) return s;
  s = f64 ? load_factor<double>(h, u, h->U[h->cur_u]) : load_factor<float>(h, u, h->U[h->cur_u]);
  if (s != NMF_OK) return s;
  if (v != nullptr) {
    s = f64 ? load_factor<double>(h, v, h->V) : load_factor<float>(h, v, h->V);
    if (s != NMF_OK) return s;
    h->have_v = true;
    HIPCHK(h, f64 ? gram<double>(h, h->V, h->gV) : gram<float>(h, h->V, h->gV));
  }
  HIPCHK(h, f64 ? gram<double>(h, h->U[h->cur_u], h->gU) : gram<float>(h, h->U[h->cur_u], h->gU));
  h->metrics_valid = false;
  return sync_status(h);
}

nmf_status nmf_get_pre(nmf_handle* h, int32_t which, void* dst) {
  if (h == nullptr || dst == nullptr || (which != 0 && which != 1))
    return fail(h, NMF_ERR_INVALID_ARG, "bad argument");
  if ((which == 0 && !h->have_pre_v) || (which == 1 && !h->have_pre_u))
    return fail(h, NMF_ERR_STATE, "no such half-step has run");
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  const int64_t rows = which == 0 ? h->m : h->n;
  return copy_sync(h, dst, which == 0 ? h->vpre : h->upre, static_cast<size_t>(rows) * h->k * h->elt);
}

nmf_status nmf_loss_fwd(nmf_handle* h, const void* U, const void* V, double* loss_dev) {
  if (h == nullptr || U == nullptr || V == nullptr || loss_dev == nullptr)
    return fail(h, NMF_ERR_INVALID_ARG, "NULL argument");
  // every operand is read or written by kernels: host memory would fault
  if (!is_device_ptr(U) || !is_device_ptr(V) || !is_device_ptr(loss_dev))
    return fail(h, NMF_ERR_INVALID_ARG, "U, V and the loss must be device memory");
  // the products below are skipped while the sticky status is set
  nmf_status st = sync_status(h);
  if (st != NMF_OK) return st;
  double* GU = h->lossG;
  double* GV = h->lossG + static_cast<size_t>(h->k) * h->k;
  if (h->elt == 8) {
    HIPCHK(h, spmm<double>(h, h->planA, h->V, nullptr, static_cast<double*>(h->lossC), nullptr, true, static_cast<const double*>(V), 0));
    HIPCHK(h, gram_dense<double>(h, static_cast<const double*>(U), h->n, GU));
    HIPCHK(h, gram_dense<double>(h, static_cast<const double*>(V), h->m, GV));
    HIPCHK(h, loss_dot<double>(h, static_cast<const double*>(U), static_cast<const double*>(h->lossC), GU, GV, loss_dev));
  } else {
    HIPCHK(h, spmm<float>(h, h->planA, h->V, nullptr, static_cast<float*>(h->lossC), nullptr, true, static_cast<const float*>(V), 0));
    HIPCHK(h, gram_dense<float>(h, static_cast<const float*>(U), h->n, GU));
    HIPCHK(h, gram_dense<float>(h, static_cast<const float*>(V), h->m, GV));
    HIPCHK(h, loss_dot<float>(h, static_cast<const float*>(U), static_cast<const float*>(h->lossC), GU, GV, loss_dev));
  }
  return sync_status(h);
}

nmf_status nmf_loss_bwd(nmf_handle* h, const void* U, const void* V, const double* g_scale, void* gU,
                        void* gV) {
  if (h == nullptr || U == nullptr || V == nullptr) return fail(h, NMF_ERR_INVALID_ARG, "NULL argument");
  if (!is_device_ptr(U) || !is_device_ptr(V) || (g_scale != nullptr && !is_device_ptr(g_scale)) ||
      (gU != nullptr && !is_device_ptr(gU)) || (gV != nullptr && !is_device_ptr(gV)))
    return fail(h, NMF_ERR_INVALID_ARG, "U, V, the scale and the gradients must be device memory");
  nmf_status st = sync_status(h);
  if (st != NMF_OK) return st;
  double* GU = h->lossG;
  double* GV = h->lossG + static_cast<size_t>(h->k) * h->k;
  if (h->elt == 8) {
    using T = double;
    if (gU) {
      HIPCHK(h, spmm<T>(h, h->planA, h->V, nullptr, static_cast<T*>(h->lossC), nullptr, true, static_cast<const T*>(V), 0));
      HIPCHK(h, gram_dense<T>(h, static_cast<const T*>(V), h->m, GV));
      HIPCHK(h, grad_combine<T>(h, static_cast<const T*>(U), static_cast<const T*>(h->lossC), GV, g_scale, h->n, static_cast<T*>(gU)));
    }
    if (gV) {
      HIPCHK(h, spmm<T>(h, h->planAt, h->U[0], nullptr, static_cast<T*>(h->lossB), nullptr, true, static_cast<const T*>(U), 0));
      HIPCHK(h, gram_dense<T>(h, static_cast<const T*>(U), h->n, GU));
      HIPCHK(h, grad_combine<T>(h, static_cast<const T*>(V), static_cast<const T*>(h->lossB), GU, g_scale, h->m, static_cast<T*>(gV)));
    }
  } else {
    using T = float;
    if (gU) {
      HIPCHK(h, spmm<T>(h, h->planA, h->V, nullptr, static_cast<T*>(h->lossC), nullptr, true, static_cast<const T*>(V), 0));
      HIPCHK(h, gram_dense<T>(h, static_cast<const T*>(V), h->m, GV));
      HIPCHK(h, grad_combine<T>(h, static_cast<const T*>(U), static_cast<const T*>(h->lossC), GV, g_scale, h->n, static_cast<T*>(gU)));
    }
    if (gV) {
      HIPCHK(h, spmm<T>(h, h->planAt, h->U[0], nullptr, static_cast<T*>(h->lossB), nullptr, true, static_cast<const T*>(U), 0));
      HIPCHK(h, gram_dense<T>(h, static_cast<const T*>(U), h->n, GU));
      HIPCHK(h, grad_combine<T>(h, static_cast<const T*>(V), static_cast<const T*>(h->lossB), GU, g_scale, h->m, static_cast<T*>(gV)));
    }
  }
  return sync_status(h);
}

// Rebuild a stored factor (0: U, 1: V) from its dense form so that its
// gather metadata matches the current thresholds.
nmf_status reload_meta(nmf_handle* h, int which) {
  if (which == 1 && !h->have_v) return NMF_OK;
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  Factor& F = which == 0 ? h->U[h->cur_u] : h->V;
  void* stage = h->sel.candA;  // rows x k scratch, free between selections
  if (h->elt == 8) {
    HIPCHK(h, densify<double>(h, F, static_cast<double*>(stage)));
    HIPCHK(h, mark_nonzero<double>(h, static_cast<double*>(stage), F.rows));
    HIPCHK(h, repack<double>(h, static_cast<double*>(stage), F.rows, F, sparse_row_of(h, F)));
  } else {
    HIPCHK(h, densify<float>(h, F, static_cast<float*>(stage)));
    HIPCHK(h, mark_nonzero<float>(h, static_cast<float*>(stage), F.rows));
    HIPCHK(h, repack<float>(h, static_cast<float*>(stage), F.rows, F, sparse_row_of(h, F)));
  }
  return sync_status(h);
}

nmf_status nmf_sequential(nmf_handle* h, int32_t k2, int32_t iters) {
  if (h == nullptr) return fail(nullptr, NMF_ERR_INVALID_ARG, "handle is NULL");
  if (k2 < 1 || h->k % k2 != 0) return fail(h, NMF_ERR_INVALID_ARG, "k2 must divide k");
  if (iters < 1) return fail(h, NMF_ERR_INVALID_ARG, "iters < 1");
  if (h->cfg.mode != NMF_MODE_COLUMN && h->cfg.mode != NMF_MODE_NONE)
    return fail(h, NMF_ERR_UNSUPPORTED, "sequential ALS runs in NMF_MODE_COLUMN or NMF_MODE_NONE");
  return h->elt == 8 ? do_sequential<double>(h, k2, iters) : do_sequential<float>(h, k2, iters);
}

nmf_status nmf_enforce(nmf_handle* h, int32_t mode, int64_t t_u, int64_t t_v) {
  if (h == nullptr) return fail(nullptr, NMF_ERR_INVALID_ARG, "handle is NULL");
  if (mode != NMF_MODE_COLUMN && mode != NMF_MODE_WHOLE)
    return fail(h, NMF_ERR_INVALID_ARG, "mode must be NMF_MODE_COLUMN or NMF_MODE_WHOLE");
  if (t_u < 1 || t_v < 1) return fail(h, NMF_ERR_INVALID_ARG, "t_u and t_v must be >= 1");
  return h->elt == 8 ? do_enforce<double>(h, mode, t_u, t_v) : do_enforce<float>(h, mode, t_u, t_v);
}

nmf_status nmf_topic_counts(nmf_handle* h, const int32_t* labels, int32_t n_labels, int64_t* counts) {
  if (h == nullptr || labels == nullptr || counts == nullptr) return fail(h, NMF_ERR_INVALID_ARG, "NULL argument");
  if (n_labels < 1 || n_labels > kBins) return fail(h, NMF_ERR_INVALID_ARG, "n_labels must be in 1..256");
  if (!h->have_v) return fail(h, NMF_ERR_STATE, "no V yet");
  nmf_status s = sync_status(h);
  if (s != NMF_OK) return s;
  // scratch: the labels in the m x k pre-selection area of the loss, the
  // counts in the select's histogram (k x 256 words, zero between selects)
  const int32_t* lab = labels;
  if (!is_device_ptr(labels)) {
    s = copy_sync(h, h->lossB, labels, static_cast<size_t>(h->m) * sizeof(int32_t));
    if (s != NMF_OK) return s;
    lab = static_cast<const int32_t*>(h->lossB);
  }
  const size_t n = static_cast<size_t>(h->k) * n_labels;
  HIPCHK(h, topic_counts(h, h->V, lab, n_labels, h->sel.hist));
  std::vector<uint32_t> c(n);
  HIPCHK(h, hipMemcpyAsync(c.data(), h->sel.hist, n * sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, fill_i32(h->stream, reinterpret_cast<int32_t*>(h->sel.hist), 0, static_cast<int64_t>(n)));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (size_t i = 0; i < n; ++i) counts[i] = c[i];
  return NMF_OK;
}

nmf_status nmf_accuracy_from_counts(const int64_t* counts, int32_t k, int32_t n_labels, double* acc) {
  if (counts == nullptr || acc == nullptr || k < 1 || n_labels < 1)
    return fail(nullptr, NMF_ERR_INVALID_ARG, "NULL pointer, k < 1 or n_labels < 1");
  for (int64_t i = 0; i < static_cast<int64_t>(k) * n_labels; ++i)
    if (counts[i] < 0) return fail(nullptr, NMF_ERR_INVALID_ARG, "negative count");
  const int64_t nj = n_labels;
  for (int32_t c = 0; c < k; ++c) {
    const int64_t* row = counts + static_cast<int64_t>(c) * n_labels;
    int64_t nd = 0, same2 = 0;  // documents, twice the same-label pairs
    for (int64_t l = 0; l < nj; ++l) {
      nd += row[l];
      same2 += row[l] * (row[l] - 1);
    }
    if (nd <= 1 || nj <= 1) {
      acc[c] = 1.0;
      continue;
    }
    // twice alpha and beta, so that everything stays integral
    const int64_t q = nd / nj, r = nd % nj;
    const int64_t alpha2 = q * (nj * (q - 1) + 2 * r);
    const int64_t beta2 = nd * (nd - 1);
    acc[c] = static_cast<double>(same2 - alpha2) / static_cast<double>(beta2 - alpha2);
  }
  return NMF_OK;
}

nmf_status nmf_topic_accuracy(nmf_handle* h, const int32_t* labels, int32_t n_labels, double* acc) {
  if (h == nullptr || acc == nullptr) return fail(h, NMF_ERR_INVALID_ARG, "NULL argument");
  if (n_labels < 1 || n_labels > kBins) return fail(h, NMF_ERR_INVALID_ARG, "n_labels must be in 1..256");
  std::vector<int64_t> counts(static_cast<size_t>(h->k) * n_labels);
  nmf_status s = nmf_topic_counts(h, labels, n_labels, counts.data());
  if (s != NMF_OK) return s;
  s = nmf_accuracy_from_counts(counts.data(), h->k, n_labels, acc);
  if (s != NMF_OK) return fail(h, s, g_create_error);
  return NMF_OK;
}

nmf_status nmf_get_param(nmf_handle* h, int32_t param, int64_t* value) {
  if (h == nullptr || value == nullptr) return fail(h, NMF_ERR_INVALID_ARG, "NULL argument");
  switch (param) {
    case NMF_PARAM_SPARSE_ROW_V:
    case NMF_PARAM_SPARSE_ROW_U:
      *value = h->sparse_row[param];
      return NMF_OK;
    case NMF_PARAM_WIDE_V:
    case NMF_PARAM_WIDE_U:
      *value = h->wide[param - NMF_PARAM_WIDE_V] ? 1 : 0;
      return NMF_OK;
    case NMF_PARAM_WAVES_V:
    case NMF_PARAM_WAVES_U:
      *value = h->waves[param - NMF_PARAM_WAVES_V];
      return NMF_OK;
    default:
      return fail(h, NMF_ERR_INVALID_ARG, "unknown parameter");
  }
}

nmf_status nmf_set_param(nmf_handle* h, int32_t param, int64_t value) {
  if (h == nullptr) return fail(nullptr, NMF_ERR_INVALID_ARG, "handle is NULL");
  switch (param) {
    case NMF_PARAM_SPARSE_ROW_V:
    case NMF_PARAM_SPARSE_ROW_U:
      if (value < 0 || value > kMaxK) return fail(h, NMF_ERR_INVALID_ARG, "sparse-row threshold out of range");
      h->sparse_row[param] = static_cast<int>(value);
      // the stored factor's gather metadata depends on the threshold:
      // rebuild it for the factor this half-step gathers
      return param == NMF_PARAM_SPARSE_ROW_V ? reload_meta(h, 0) : reload_meta(h, 1);
    case NMF_PARAM_WIDE_V:
    case NMF_PARAM_WIDE_U:
      if (value != 0 && value != 1) return fail(h, NMF_ERR_INVALID_ARG, "step form must be 0 or 1");
      h->wide[param - NMF_PARAM_WIDE_V] = value != 0;
      return NMF_OK;
    case NMF_PARAM_WAVES_V:
    case NMF_PARAM_WAVES_U:
      if (value != 1 && value != 2 && value != 4 && value != 8 && value != 16)
        return fail(h, NMF_ERR_INVALID_ARG, "waves per block must be 1, 2, 4, 8 or 16");
      h->waves[param - NMF_PARAM_WAVES_V] = static_cast<int>(value);
      return NMF_OK;
    default:
      return fail(h, NMF_ERR_INVALID_ARG, "unknown parameter");
  }
}

nmf_status nmf_profile(nmf_handle* h, int32_t enable) {
  return nmf_profile_stages(h, enable != 0 ? (1u << NMF_NUM_STAGES) - 1u : 0u);
}

nmf_status nmf_profile_stages(nmf_handle* h, uint32_t stages) {
  if (h == nullptr) return fail(nullptr, NMF_ERR_INVALID_ARG, "handle is NULL");
  if (stages >> NMF_NUM_STAGES) return fail(h, NMF_ERR_INVALID_ARG, "unknown stage bit");
  if (h->prof_ev.empty()) {
    h->prof_ev.resize(kProfPool);
    h->prof_stage.resize(kProfPool, -1);
    for (auto& e : h->prof_ev) HIPCHK(h, hipEventCreate(&e));
  }
  nmf_status s = prof_fold(h);
  if (s != NMF_OK) return s;
  h->prof_on = stages != 0;
  h->prof_mask = stages;
  h->prof_open = -2;
  if (h->prof_on)
    for (int i = 0; i < NMF_NUM_STAGES; ++i) {
      h->prof_ms[i] = 0;
      h->prof_cnt[i] = 0;
    }
  return NMF_OK;
}

nmf_status nmf_profile_read(nmf_handle* h, double* ms, int64_t* count, int32_t n_stages) {
  if (h == nullptr || n_stages < 0 || n_stages > NMF_NUM_STAGES) return fail(h, NMF_ERR_INVALID_ARG, "bad argument");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  nmf_status s = prof_fold(h);
  if (s != NMF_OK) return s;
  for (int i = 0; i < n_stages; ++i) {
    if (ms) ms[i] = h->prof_ms[i];
    if (count) count[i] = h->prof_cnt[i];
  }
  return NMF_OK;
}

const char* nmf_last_error(const nmf_handle* h) {
  return h ? h->last_error.c_str() : g_create_error.c_str();
}

void nmf_destroy(nmf_handle* h) {
  if (h == nullptr) return;
  (void)hipStreamSynchronize(h->stream);
  for (auto& e : h->prof_ev) (void)hipEventDestroy(e);
  if (h->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static[h->static_dev].in_use = false;
  }
  delete h;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
//
// A batch is one handle per problem, all on one stream, plus the fused
// launch plans: every problem's launches of one iteration are recorded (for
// each parity of the current-U slot), and launch j of every problem becomes
// one launch of the kernel's batched form whose blocks are mapped to
// (problem, block of that problem's own grid).  Problems whose launch j is a
// different kernel (another template instance) get a launch of their own at
// the same position.

struct nmf_batch {
  struct Launch {
    const void* fn;
    unsigned blocks;
    unsigned block;
    size_t lds;
    const void* args;  // device: the members' argument structs
    const void* map;   // device: BlockMap per block
  };
  std::vector<nmf_handle*> h;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<Launch> plan[2];  // one iteration starting at current-U slot 0 / 1
  hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [loop, fused][start slot]
  char* tables = nullptr;       // device: the fused launches' argument structs and block maps
  size_t table_bytes = 0;
  std::string last_error;
};

namespace {

thread_local std::string g_batch_error = "no error";

nmf_status batch_fail(nmf_batch* b, nmf_status s, const std::string& msg) {
  if (b)
    b->last_error = msg;
  else
    g_batch_error = msg;
  return s;
}

#define BCHK(b, expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return batch_fail((b), NMF_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Upper bound of the fused-table bytes one problem adds (both slots): its
// argument structs and one BlockMap per block of every launch of an
// iteration (grid bounds as in the launchers).
size_t batch_table_bound(const nmf_config& c, int64_t nnz) {
  const int64_t ch = nnz / kChunk + 2;
  auto sel = [&](int64_t r) { return 2 * ((r + 63) / 64 + 1) + (c.k + 3) / 4 + c.k; };
  auto rep = [&](int64_t r) { return 2 * ((r + 255) / 256 + 1); };
  const int64_t gram = kGramBlocks + 130 + 1;
  const int64_t blocks = (c.m + 2 * ch + 1) + ch + (c.n + 2 * ch + 1) + ch + sel(c.m) + sel(c.n) + rep(c.m) +
                         rep(c.n) + 2 * gram + kMetricBlocks + 1 + (c.m + 63) / 64 + 1;
  const int64_t launches = 48;
  return 2 * (static_cast<size_t>(blocks) * sizeof(BlockMap) + launches * (512 + 512));
}

// The host-side state one iteration changes, to undo a recorded or captured
// iteration and to apply replayed ones.
struct HostState {
  int cur_u;
  int64_t iters_done;
  bool have_v, have_pre_v, have_pre_u, metrics_valid, prof_on;
};
HostState save_state(const nmf_handle* h) {
  return HostState{h->cur_u, h->iters_done, h->have_v, h->have_pre_v, h->have_pre_u, h->metrics_valid, h->prof_on};
}
void restore_state(nmf_handle* h, const HostState& s) {
  h->cur_u = s.cur_u;
  h->iters_done = s.iters_done;
  h->have_v = s.have_v;
  h->have_pre_v = s.have_pre_v;
  h->have_pre_u = s.have_pre_u;
  h->metrics_valid = s.metrics_valid;
  h->prof_on = s.prof_on;
}
void advance_state(nmf_handle* h, int32_t iters) {
  if (iters <= 0) return;
  if (iters & 1) h->cur_u = 1 - h->cur_u;
  h->iters_done += iters;
  h->have_v = h->have_pre_v = h->have_pre_u = true;
  h->metrics_valid = !(h->cfg.flags & NMF_FLAG_NO_METRICS);
}

nmf_status steps_of(nmf_handle* h, int32_t iters) {
  return h->elt == 8 ? do_steps<double>(h, iters) : do_steps<float>(h, iters);
}

nmf_status build_plans(nmf_batch* b, char* tables, size_t table_bytes) {
  std::vector<char> stage;
  size_t used = 0;
  auto put = [&](const void* src, size_t bytes) {
    used = align_up(used, 256);
    const size_t at = used;
    if (stage.size() < used + bytes) stage.resize(used + bytes);
    std::memcpy(stage.data() + at, src, bytes);
    used += bytes;
    return at;
  };
  struct Pending {
    int slot;
    const void* fn;
    unsigned blocks, block;
    size_t lds, args_at, map_at;
  };
  std::vector<Pending> pend;
  const size_t np = b->h.size();
  for (int slot = 0; slot < 2; ++slot) {
    std::vector<std::vector<LaunchRecord>> recs(np);
    for (size_t i = 0; i < np; ++i) {
      nmf_handle* h = b->h[i];
      const HostState st = save_state(h);
      h->prof_on = false;
      h->cur_u = slot;
      h->rec = &recs[i];
      h->hist_cus = h->batch_cus > 0 ? h->batch_cus : h->num_cus;
      nmf_status s = steps_of(h, 1);
      h->hist_cus = h->num_cus;
      h->rec = nullptr;
      restore_state(h, st);
      if (s != NMF_OK) return batch_fail(b, s, "recording problem " + std::to_string(i) + ": " + h->last_error);
    }
    const size_t L = recs[0].size();
    for (size_t i = 1; i < np; ++i)
      if (recs[i].size() != L) return batch_fail(b, NMF_ERR_DEVICE, "internal: launch sequences differ");
    for (size_t j = 0; j < L; ++j) {
      std::vector<std::pair<const void*, unsigned>> keys;
      std::vector<std::vector<size_t>> members;
      for (size_t i = 0; i < np; ++i) {
        const LaunchRecord& r = recs[i][j];
        if (r.grid == 0) continue;
        size_t g = 0;
        while (g < keys.size() && (keys[g].first != r.batched || keys[g].second != r.block)) ++g;
        if (g == keys.size()) {
          keys.emplace_back(r.batched, r.block);
          members.emplace_back();
        }
        members[g].push_back(i);
      }
      for (size_t g = 0; g < keys.size(); ++g) {
        std::vector<unsigned char> args;
        std::vector<BlockMap> map;
        size_t lds = 0;
        for (size_t mi = 0; mi < members[g].size(); ++mi) {
          const LaunchRecord& r = recs[members[g][mi]][j];
          args.insert(args.end(), r.args.begin(), r.args.end());
          for (unsigned blk = 0; blk < r.grid; ++blk)
            map.push_back(BlockMap{static_cast<int32_t>(mi), static_cast<int32_t>(blk),
                                   static_cast<int32_t>(r.grid), 0});
          lds = std::max(lds, r.lds);
        }
        Pending p;
        p.slot = slot;
        p.fn = keys[g].first;
        p.blocks = static_cast<unsigned>(map.size());
        p.block = keys[g].second;
        p.lds = lds;
        p.args_at = put(args.data(), args.size());
        p.map_at = put(map.data(), map.size() * sizeof(BlockMap));
        pend.push_back(p);
      }
    }
  }
  if (used > table_bytes) return batch_fail(b, NMF_ERR_WORKSPACE, "internal: fused tables exceed their bound");
  BCHK(b, hipMemcpy(tables, stage.data(), used, hipMemcpyHostToDevice));
  for (const Pending& p : pend)
    b->plan[p.slot].push_back(nmf_batch::Launch{p.fn, p.blocks, p.block, p.lds, tables + p.args_at, tables + p.map_at});
  return NMF_OK;
}

// Drop the fused plans and every captured graph, then record the plans
// again (after the members' tuning parameters changed).
nmf_status rebuild_plans(nmf_batch* b) {
  BCHK(b, hipStreamSynchronize(b->stream));
  for (auto& row : b->exec)
    for (auto& e : row) {
      if (e) (void)hipGraphExecDestroy(e);
      e = nullptr;
    }
  b->plan[0].clear();
  b->plan[1].clear();
  return build_plans(b, b->tables, b->table_bytes);
}

nmf_status launch_plan(nmf_batch* b, int slot) {
  for (const nmf_batch::Launch& L : b->plan[slot]) {
    void* kargs[2] = {const_cast<void**>(&L.args), const_cast<void**>(&L.map)};
    BCHK(b, hipLaunchKernel(L.fn, dim3(L.blocks), dim3(L.block), kargs, L.lds, b->stream));
  }
  return NMF_OK;
}

// Every problem must sit at the same current-U slot for the fused plans.
nmf_status common_slot(nmf_batch* b, int* slot) {
  *slot = b->h[0]->cur_u;
  for (nmf_handle* h : b->h)
    if (h->cur_u != *slot)
      return batch_fail(b, NMF_ERR_STATE, "problems were stepped separately: their iterates are out of step");
  return NMF_OK;
}

// One iteration of the batch without graphs (fused or loop); the host state
// is advanced.
nmf_status batch_iteration(nmf_batch* b, bool fused) {
  if (fused) {
    int slot;
    nmf_status s = common_slot(b, &slot);
    if (s != NMF_OK) return s;
    if ((s = launch_plan(b, slot)) != NMF_OK) return s;
    for (nmf_handle* h : b->h) advance_state(h, 1);
    return NMF_OK;
  }
  for (size_t i = 0; i < b->h.size(); ++i) {
    nmf_status s = steps_of(b->h[i], 1);
    if (s != NMF_OK) return batch_fail(b, s, "problem " + std::to_string(i) + ": " + b->h[i]->last_error);
  }
  return NMF_OK;
}

// Capture two iterations starting at the current slot as a graph; the host
// state is left as it was.
nmf_status capture_pair(nmf_batch* b, bool fused, int slot, hipGraphExec_t* exec) {
  std::vector<HostState> st;
  for (nmf_handle* h : b->h) st.push_back(save_state(h));
  BCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  nmf_status s = NMF_OK;
  for (int it = 0; it < 2 && s == NMF_OK; ++it) s = batch_iteration(b, fused);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(b->stream, &g);
  for (size_t i = 0; i < b->h.size(); ++i) restore_state(b->h[i], st[i]);
  if (s != NMF_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (ec != hipSuccess) return batch_fail(b, NMF_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
  const hipError_t ei = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return batch_fail(b, NMF_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
  (void)slot;
  return NMF_OK;
}

}  // namespace

extern "C" {

nmf_status nmf_batch_workspace_size(int32_t count, const nmf_config* cfgs, const int64_t* nnz, size_t* bytes) {
  if (count < 1 || cfgs == nullptr || nnz == nullptr || bytes == nullptr)
    return batch_fail(nullptr, NMF_ERR_INVALID_ARG, "count < 1 or a NULL argument");
  size_t total = 0, tables = 0;
  for (int32_t i = 0; i < count; ++i) {
    size_t w = 0;
    nmf_status s = nmf_workspace_size(&cfgs[i], nnz[i], &w);
    if (s != NMF_OK) return batch_fail(nullptr, s, "problem " + std::to_string(i) + ": " + nmf_last_error(nullptr));
    total += align_up(w, 256);
    tables += batch_table_bound(cfgs[i], nnz[i]);
  }
  *bytes = total + align_up(tables, 256);
  return NMF_OK;
}

static nmf_status nmf_batch_create_impl(int32_t count, const nmf_config* cfgs, const int64_t* const* a_rowptr,
                            const int32_t* const* a_col, const void* const* a_val, const int64_t* nnz,
                            const void* const* u0, void* workspace, size_t ws_bytes, void* hip_stream,
                            nmf_batch** out) {
  if (out == nullptr) return batch_fail(nullptr, NMF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (count < 1 || cfgs == nullptr || a_rowptr == nullptr || a_col == nullptr || a_val == nullptr ||
      nnz == nullptr || u0 == nullptr)
    return batch_fail(nullptr, NMF_ERR_INVALID_ARG, "count < 1 or a NULL array");
  size_t need = 0;
  nmf_status s = nmf_batch_workspace_size(count, cfgs, nnz, &need);
  if (s != NMF_OK) return s;
  if (workspace == nullptr || ws_bytes < need)
    return batch_fail(nullptr, NMF_ERR_WORKSPACE, "workspace smaller than nmf_batch_workspace_size()");
  nmf_batch* b = new (std::nothrow) nmf_batch();
  if (b == nullptr) return batch_fail(nullptr, NMF_ERR_DEVICE, "out of host memory");
  b->stream = static_cast<hipStream_t>(hip_stream);
  if (b->stream == nullptr) {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return batch_fail(nullptr, NMF_ERR_DEVICE, "cannot create a stream");
    }
    b->own_stream = true;
  }
  char* base = static_cast<char*>(workspace);
  size_t off = 0;
  for (int32_t i = 0; i < count && s == NMF_OK; ++i) {
    size_t w = 0;
    nmf_workspace_size(&cfgs[i], nnz[i], &w);
    nmf_handle* h = nullptr;
    s = nmf_create(&cfgs[i], a_rowptr[i], a_col[i], a_val[i], nnz[i], u0[i], nullptr, base + off, w, b->stream, &h);
    if (s != NMF_OK) {
      batch_fail(nullptr, s, "problem " + std::to_string(i) + ": " + nmf_last_error(nullptr));
      break;
    }
    b->h.push_back(h);
    off += align_up(w, 256);
  }
  if (s == NMF_OK) {
    // each problem's histogram pass is sized for its share of the GPU (by
    // select work, (n + m) k), four times over so that the fused launch
    // still balances; a problem alone uses every compute unit
    double total = 0;
    for (nmf_handle* h : b->h) total += static_cast<double>(h->n + h->m) * h->k;
    for (nmf_handle* h : b->h) {
      const double w = static_cast<double>(h->n + h->m) * h->k;
      const int share = static_cast<int>(std::ceil(4.0 * h->num_cus * w / total));
      h->batch_cus = std::max(1, std::min(h->num_cus, share));
    }
    b->tables = base + off;
    b->table_bytes = ws_bytes - off;
    s = build_plans(b, b->tables, b->table_bytes);
    if (s != NMF_OK) g_batch_error = b->last_error;
  }
  if (s != NMF_OK) {
    const std::string msg = g_batch_error;
    nmf_batch_destroy(b);
    g_batch_error = msg;
    return s;
  }
  *out = b;
  return NMF_OK;
}

static nmf_status nmf_batch_step_impl(nmf_batch* b, int32_t iters, int32_t how) {
  if (b == nullptr) return batch_fail(nullptr, NMF_ERR_INVALID_ARG, "batch is NULL");
  if (iters < 0) return batch_fail(b, NMF_ERR_INVALID_ARG, "iters < 0");
  if (how < NMF_BATCH_LOOP || how > NMF_BATCH_FUSED_GRAPH) return batch_fail(b, NMF_ERR_INVALID_ARG, "unknown mode");
  const bool fused = how == NMF_BATCH_FUSED || how == NMF_BATCH_FUSED_GRAPH;
  const bool graph = how == NMF_BATCH_LOOP_GRAPH || how == NMF_BATCH_FUSED_GRAPH;
  nmf_status s;
  if (!graph) {
    for (int32_t it = 0; it < iters; ++it)
      if ((s = batch_iteration(b, fused)) != NMF_OK) return s;
    return NMF_OK;
  }
  int slot;
  if ((s = common_slot(b, &slot)) != NMF_OK) return s;
  hipGraphExec_t& ex = b->exec[fused ? 1 : 0][slot];
  if (iters >= 2 && ex == nullptr && (s = capture_pair(b, fused, slot, &ex)) != NMF_OK) return s;
  for (int32_t it = 0; it + 1 < iters; it += 2) {
    BCHK(b, hipGraphLaunch(ex, b->stream));
    for (nmf_handle* h : b->h) advance_state(h, 2);
  }
  if (iters & 1) return batch_iteration(b, fused);
  return NMF_OK;
}

nmf_status nmf_batch_errors(nmf_batch* b, double* E, int32_t* status) {
  if (b == nullptr) return batch_fail(nullptr, NMF_ERR_INVALID_ARG, "batch is NULL");
  BCHK(b, hipStreamSynchronize(b->stream));
  nmf_status first = NMF_OK;
  for (size_t i = 0; i < b->h.size(); ++i) {
    double e = __builtin_nan("");
    nmf_status s = nmf_error(b->h[i], &e);
    if (E) E[i] = e;
    if (status) status[i] = s;
    if (s != NMF_OK && first == NMF_OK) {
      first = s;
      b->last_error = "problem " + std::to_string(i) + ": " + b->h[i]->last_error;
    }
  }
  return first;
}

static nmf_status nmf_batch_set_param_impl(nmf_batch* b, int32_t i, int32_t param, int64_t value) {
  if (b == nullptr) return batch_fail(nullptr, NMF_ERR_INVALID_ARG, "batch is NULL");
  if (i < -1 || i >= static_cast<int32_t>(b->h.size())) return batch_fail(b, NMF_ERR_INVALID_ARG, "no such problem");
  BCHK(b, hipStreamSynchronize(b->stream));
  for (size_t j = 0; j < b->h.size(); ++j) {
    if (i >= 0 && static_cast<int32_t>(j) != i) continue;
    nmf_status s = nmf_set_param(b->h[j], param, value);
    if (s != NMF_OK) return batch_fail(b, s, "problem " + std::to_string(j) + ": " + b->h[j]->last_error);
  }
  return rebuild_plans(b);
}

static nmf_status nmf_batch_tune_impl(nmf_batch* b, int32_t iters, int32_t* chosen) {
  if (b == nullptr) return batch_fail(nullptr, NMF_ERR_INVALID_ARG, "batch is NULL");
  if (iters < 1) return batch_fail(b, NMF_ERR_INVALID_ARG, "iters < 1");
  int slot;
  nmf_status s = common_slot(b, &slot);
  if (s != NMF_OK) return s;
  // SpMM forms tried for each half: {wide step, entry-by-entry threshold, waves per block}
  static const int kCands[][3] = {{0, 1, 16}, {0, 1, 8}, {0, 3, 8}, {0, 0, 16}, {1, 3, 8},
                                  {1, 1, 8},  {1, 3, 16}, {1, 0, 8}, {1, 2, 4}, {0, 2, 4}};
  const int n_cands = static_cast<int>(sizeof(kCands) / sizeof(kCands[0]));
  auto apply = [&](int half, const int* c) -> nmf_status {
    const int32_t params[3] = {half == 0 ? NMF_PARAM_WIDE_V : NMF_PARAM_WIDE_U,
                               half == 0 ? NMF_PARAM_SPARSE_ROW_V : NMF_PARAM_SPARSE_ROW_U,
                               half == 0 ? NMF_PARAM_WAVES_V : NMF_PARAM_WAVES_U};
    for (size_t j = 0; j < b->h.size(); ++j)
      for (int q = 0; q < 3; ++q) {
        nmf_status st = nmf_set_param(b->h[j], params[q], c[q]);
        if (st != NMF_OK) return batch_fail(b, st, "problem " + std::to_string(j) + ": " + b->h[j]->last_error);
      }
    return rebuild_plans(b);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BCHK(b, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return batch_fail(b, NMF_ERR_DEVICE, "hipEventCreate failed");
  }
  int best[2] = {0, 0};
  for (int half = 0; half < 2 && s == NMF_OK; ++half) {
    float best_ms = 0.f;
    for (int c = 0; c < n_cands && s == NMF_OK; ++c) {
      if ((s = apply(half, kCands[c])) != NMF_OK) break;
      // one untimed iteration under the new form, then `iters` timed ones
      if ((s = batch_iteration(b, true)) != NMF_OK) break;
      if (hipEventRecord(e0, b->stream) != hipSuccess) s = batch_fail(b, NMF_ERR_DEVICE, "hipEventRecord failed");
      for (int32_t it = 0; it < iters && s == NMF_OK; ++it) s = batch_iteration(b, true);
      if (s != NMF_OK) break;
      float ms = 0.f;
      if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        s = batch_fail(b, NMF_ERR_DEVICE, "timing a tuning trial failed");
        break;
      }
      if (c == 0 || ms < best_ms) {
        best_ms = ms;
        best[half] = c;
      }
    }
    if (s == NMF_OK) s = apply(half, kCands[best[half]]);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != NMF_OK) return s;
  if (chosen)
    for (int half = 0; half < 2; ++half)
      for (int q = 0; q < 3; ++q) chosen[half * 3 + q] = kCands[best[half]][q];
  return NMF_OK;
}

nmf_handle* nmf_batch_problem(nmf_batch* b, int32_t i) {
  if (b == nullptr || i < 0 || static_cast<size_t>(i) >= b->h.size()) return nullptr;
  return b->h[i];
}

const char* nmf_batch_last_error(const nmf_batch* b) {
  return b ? b->last_error.c_str() : g_batch_error.c_str();
}

void nmf_batch_destroy(nmf_batch* b) {
  if (b == nullptr) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (auto& row : b->exec)
    for (auto& e : row)
      if (e) (void)hipGraphExecDestroy(e);
  for (nmf_handle* h : b->h) nmf_destroy(h);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

// The batch entry points that build host containers: a host allocation
// failure (or any other host exception) becomes an error status instead of
// escaping the C ABI.
nmf_status nmf_batch_create(int32_t count, const nmf_config* cfgs, const int64_t* const* a_rowptr,
                            const int32_t* const* a_col, const void* const* a_val, const int64_t* nnz,
                            const void* const* u0, void* workspace, size_t ws_bytes, void* hip_stream,
                            nmf_batch** out) {
  try {
    return nmf_batch_create_impl(count, cfgs, a_rowptr, a_col, a_val, nnz, u0, workspace, ws_bytes, hip_stream,
                                 out);
  } catch (const std::bad_alloc&) {
    return batch_fail(nullptr, NMF_ERR_DEVICE, "out of host memory");
  } catch (...) {
    return batch_fail(nullptr, NMF_ERR_DEVICE, "host error while creating the batch");
  }
}

nmf_status nmf_batch_step(nmf_batch* b, int32_t iters, int32_t how) {
  try {
    return nmf_batch_step_impl(b, iters, how);
  } catch (const std::bad_alloc&) {
    return batch_fail(b, NMF_ERR_DEVICE, "out of host memory");
  } catch (...) {
    return batch_fail(b, NMF_ERR_DEVICE, "host error in a batch step");
  }
}

nmf_status nmf_batch_set_param(nmf_batch* b, int32_t i, int32_t param, int64_t value) {
  try {
    return nmf_batch_set_param_impl(b, i, param, value);
  } catch (const std::bad_alloc&) {
    return batch_fail(b, NMF_ERR_DEVICE, "out of host memory");
  } catch (...) {
    return batch_fail(b, NMF_ERR_DEVICE, "host error while setting a parameter");
  }
}

nmf_status nmf_batch_tune(nmf_batch* b, int32_t iters, int32_t* chosen) {
  try {
    return nmf_batch_tune_impl(b, iters, chosen);
  } catch (const std::bad_alloc&) {
    return batch_fail(b, NMF_ERR_DEVICE, "out of host memory");
  } catch (...) {
    return batch_fail(b, NMF_ERR_DEVICE, "host error while tuning");
  }
}

}  // extern "C"
