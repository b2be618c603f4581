// Internal declarations shared by the host library (nmf_api.cpp) and the HIP
// kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nmf.h"

namespace nmfk {

constexpr int kMaxK = 128;       // topics supported (2 per lane at most)
constexpr int kMaxHot = 128;     // most hot columns split off the V-half stream (float32)
constexpr int kMaxWarm = 256;    // most warm terms, whose rows of U the V-half kernel keeps in LDS
constexpr double kHotDensity = 0.0625;  // a hot column holds at least this share of the rows
constexpr int64_t kHotMinNnz = 16;     // ... and at least this many nonzeros
constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kChunk = 1024;     // nonzeros per SpMM work item; longer rows are split

// Most output rows a light SpMM work item carries (the rows of one epilogue
// batch): 8 with one topic per lane, 4 with two.
inline int spmm_row_group(int k) { return k > 64 ? 4 : 8; }
constexpr int kBins = 256;       // radix digit width of the top-t select (8 bits)
constexpr int kHistRing = 4096;  // iterations kept in the device history ring
constexpr int kGramBlocks = 240; // Gram partial blocks (fixed: deterministic sums)
constexpr int kMetricBlocks = 1024;
constexpr int kSelBlockRows = 64;  // rows of the selected matrix per select collect block
constexpr int kSelSub = 16;        // candidate sub-lists per column (collect block b appends to b % 16)
constexpr int kCntStride = 64;     // ints between candidate counters (256 bytes)

// History record fields (float64 each), in the order of NMF_HIST_*.
enum { H_E = 0, H_R, H_NNZU, H_NNZV, H_DEADU, H_DEADV, H_VIFU, H_VIFV, H_GATHV, H_GATHU, H_FIELDS };
constexpr int kGathSlots = 16;  // spread slots of each gathered-entries counter

// One unit of SpMM work for one wave, over the nonzeros [p0, p1) of the
// plan's arrays (row-compressed, rows ascending, columns ascending in a row).
//  light (heavy < 0): output rows [r0, r1), every row at most kChunk long.
//  heavy (heavy >= 0): one kChunk piece of the long row r0; its raw sum goes
//    to partial slot `part`; a second kernel adds the row's partials in chunk
//    order and runs the epilogue.
struct WorkItem {
  int32_t r0, r1;
  int64_t p0, p1;
  int32_t heavy;
  int32_t part;
};

// SpMM plan for one orientation of A (CSR of A: U half; CSR of A^T: V half).
struct Plan {
  int64_t rows = 0;
  int64_t nnz = 0;            // entries in col/val (the fused V-half stream: padding included)
  int64_t* rowptr = nullptr;  // [rows + 1]
  int32_t* col = nullptr;     // [nnz]
  void* val = nullptr;        // [nnz] T
  WorkItem* items = nullptr;  // [n_items]
  int32_t n_items = 0;
  int32_t n_heavy = 0;
  int32_t n_parts = 0;
  int32_t* heavy_row = nullptr;      // [n_heavy] row of each long row
  int32_t* heavy_nchunks = nullptr;  // [n_heavy]
  int32_t* heavy_part0 = nullptr;    // [n_heavy]
  void* partials = nullptr;          // [n_parts][k] T
  // Hot rows of the gathered factor (float32 only): the columns of the
  // streamed orientation that hold the most nonzeros are kept out of the CSR
  // above and stored as a dense block, hot[r * hot_ld + h] = entry of row r
  // in hot column h (hot_ld a multiple of 16, zero-padded), multiplied on the
  // matrix cores.
  int32_t n_hot = 0;
  int32_t hot_ld = 0;
  int32_t* hot_col = nullptr;  // [kMaxHot]: factor row of hot column h
  void* hot = nullptr;         // [rows][hot_ld] T
  // Warm columns (fused V-half stream only): the next most frequent terms
  // after the hot ones stay in the stream, but their entries carry term
  // -2 - w and the kernel reads factor row warm_col[w] from LDS
  int32_t n_warm = 0;
  int32_t* warm_col = nullptr;  // [kMaxWarm]
  // Per row of the gathered factor: how many of this plan's streamed
  // nonzeros lie in its column (the hot ones excluded); the gathered-entry
  // count of a product is sum over rows of this times the row's entries
  int32_t* sdf = nullptr;      // [rows of the gathered factor]
};

// The fused V-half kernel serves float32 factors with k <= 64 whose byte
// offsets into V_pre, the hot block and the stream fit 32 bits and whose U row table
// (8 bytes per 32 terms) fits its LDS share; the hot block exists only then.
constexpr int64_t kVhTabWords = 8192;  // at most 262144 terms
// Its stream pads every document's nonzeros to a multiple of four (term -1,
// value 0), so that each lane's four-nonzero reads are 16-byte aligned, and
// keeps four spare entries past the end: vh_stream_cap entries in all.
inline int64_t vh_stream_cap(int64_t m, int64_t nnz) { return nnz + 3 * m + 4; }
inline bool vhalf_fits(size_t elt, int64_t n, int64_t m, int k, int64_t nnz) {
  return elt == 4 && k <= 64 && (m + 16) * k * 4 < (int64_t{1} << 32) &&
         vh_stream_cap(m, nnz) * 4 < (int64_t{1} << 32) &&
         (m + 16) * kMaxHot * 4 < (int64_t{1} << 32) && (n + 31) / 32 <= kVhTabWords;
}

// A factor as stored (row-compressed sparse) plus the gather cache the SpMM
// reads: every nonempty row expanded to a dense row (rows 16-byte aligned at
// least, so one lane can load four floats or two doubles of a row at once).
struct Factor {
  int64_t rows = 0;
  int32_t* row_ptr = nullptr;  // [rows + 1]
  uint8_t* topic = nullptr;    // [rows * k]
  void* val = nullptr;         // [rows * k] T
  int32_t* slot = nullptr;     // [rows]: -1 empty, else compact row index
  int32_t* rowid = nullptr;    // [rows]: compact row index -> row
  void* dense = nullptr;       // [rows][ld] T: compact dense rows 0..R-1, zero past k
  int32_t ld = 0;              // row pitch of `dense`: k rounded up to 64 bytes (dense_ld), or
                               // to 4 for U when the fused V-half kernel serves the problem
  int32_t* counts = nullptr;   // device [0] = nnz, [1] = R (nonempty rows)
  // SpMM gather metadata: per row {compact dense row (rows with more entries
  // than the gathering SpMM's threshold) or first stored entry, entry count};
  // per entry {value, topic}
  int2* meta = nullptr;        // [rows]
  void* packed = nullptr;      // [rows * k] FactorEnt<T>
  // Row table: word w = {bit i set when row 32 w + i is nonempty, number of
  // nonempty rows before row 32 w}, so a row's compact index is found from
  // one word (the fused V-half kernel keeps U's table in LDS)
  int2* rowtab = nullptr;      // [(rows + 31) / 32]
};

// One stored factor entry as the SpMM gathers it (8 bytes for float).
template <typename T>
struct FactorEnt {
  T v;
  uint32_t t;
};

// Row pitch of a factor's compact dense copy: k rounded up to whole 64-byte
// lines (16 floats or 8 doubles), so that each quarter of a wave reading a
// row (lanes = topics) touches exactly one cache line.
inline int32_t dense_ld(int32_t k, size_t elt) {
  const int32_t v = static_cast<int32_t>(64 / elt);
  return (k + v - 1) / v * v;
}


// Gram matrix of a factor and its inverse.
struct Gram {
  double* G = nullptr;  // [k][k] F^T F
  double* W = nullptr;  // [k][k] inverse of G
  int32_t* dead = nullptr;  // device: number of dead topics
};

// Per-column selection state of the top-t select.
struct ColSel {
  int32_t b1;    // first digit of the threshold
  int32_t need;  // entries still to take from the b1 bin
  int32_t all;   // 1: the column keeps every positive entry
  int32_t npos;  // positive entries in the column
};

struct SelectWs {
  uint32_t* hist = nullptr;     // [k][kBins], zero between uses (cleared by refine)
  ColSel* sel = nullptr;        // [k]
  int32_t* cand_cnt = nullptr;  // [k][kSelSub] counters kCntStride ints apart, zero between uses
  int64_t cand_sub = 0;         // entries per sub-list (per column)
  void* candA = nullptr;        // [k][rows_max] candidates (row, key)
  void* candB = nullptr;        // [k][rows_max] ping-pong buffer
  int64_t cand_stride = 0;      // entries per column
  uint32_t* mask = nullptr;     // [rows_max][mask_words], zero between uses
  int32_t* ticket = nullptr;    // [4], zero between uses
  int32_t* scan_part = nullptr; // [2][scan blocks + 1]
};

struct Metrics {
  double* partials = nullptr;   // [kMetricBlocks][4]
  int32_t* ticket = nullptr;    // [1]
  double* ring = nullptr;       // [kHistRing][H_FIELDS]
  int64_t* it = nullptr;        // device iteration counter
  int64_t* max_nnz = nullptr;   // device storage high-water mark
  double* nA2 = nullptr;        // ||A||_F^2
  double* loss_parts = nullptr; // [kMetricBlocks]
  double* out = nullptr;        // [4] scalar results of on-demand queries
  // factor entries the products gathered since the last record: [0] V half,
  // [1] U half, each spread over kGathSlots words (one atomic add per wave)
  unsigned long long* gathered = nullptr;  // [2][kGathSlots]
};

}  // namespace nmfk

namespace nmfk {

// One block of a batched launch: the problem it serves and the block of that
// problem's own grid it plays (blk of nblk).
struct BlockMap {
  int32_t prob;
  int32_t blk;
  int32_t nblk;
  int32_t pad;
};

// Launches recorded instead of issued (to build a batched replay): the
// batched form of the kernel, its argument struct, the problem's own grid,
// the block size and the dynamic LDS bytes.
struct LaunchRecord {
  const void* batched = nullptr;
  std::vector<unsigned char> args;
  unsigned grid = 0;
  unsigned block = 0;
  size_t lds = 0;
};

}  // namespace nmfk

struct nmf_handle {
  nmf_config cfg{};
  int64_t n = 0, m = 0, nnz = 0;
  int k = 0;
  size_t elt = 4;  // sizeof(T)
  int mask_words = 1;
  hipStream_t stream = nullptr;
  int device = 0;
  int static_dev = -1;  // device whose static workspace this handle owns (nmf_create_static), else -1
  int num_cus = 256;
  // Compute units this problem's histogram pass is sized for: all of them
  // alone and in a batch's per-problem loop, its share of the GPU in a
  // batch's fused launches (block counts only; no result depends on it).
  int hist_cus = 256;
  int batch_cus = 0;  // that share (0: not in a batch)
  char* ws = nullptr;
  size_t ws_bytes = 0;

  nmfk::Plan planA;   // CSR of A: rows = terms (U half)
  nmfk::Plan planAt;  // CSR of A^T: rows = docs (V half)
  nmfk::Factor U[2];  // current and previous U
  int cur_u = 0;
  nmfk::Factor V;
  nmfk::Gram gU, gV;
  void* vpre = nullptr;  // [m][k] T clamped pre-selection V
  void* upre = nullptr;  // [n][k] T clamped pre-selection U
  void* cbuf = nullptr;  // [n][k] T raw A V of the last U half
  void* lossB = nullptr; // [m][k] T scratch of the loss entry points
  void* lossC = nullptr; // [n][k] T
  double* lossG = nullptr; // [2][k][k]
  nmfk::SelectWs sel;
  void* gram_partials = nullptr;  // [kGramBlocks][k][k] T
  int32_t* gram_ticket = nullptr;
  nmfk::Metrics met;
  int32_t* status = nullptr;      // sticky device status (nmf_status value)
  int32_t* scratch_i = nullptr;   // small device scratch for host queries

  // host-side state
  int64_t iters_done = 0;
  bool have_v = false;
  bool w_stale = false;  // gU.W is not the inverse of U's Gram (after a sequential run)
  bool have_pre_v = false, have_pre_u = false;
  bool metrics_valid = false;  // the newest history record describes the current U, V
  // float32 with k <= 64: the V half is the fused kernel of k_vhalf.hip
  // (its own queue replaces the entry-by-entry gathers: NMF_PARAM_SPARSE_ROW_V
  // and NMF_PARAM_WIDE_V do not apply)
  bool use_vhalf = false;
  int sparse_row[2] = {1, 1};                 // NMF_PARAM_SPARSE_ROW_V / _U
  bool wide[2] = {false, true};               // NMF_PARAM_WIDE_V / _U
  int waves[2] = {16, 8};                     // NMF_PARAM_WAVES_V / _U: waves per SpMM block
  // stage timing (nmf_profile)
  bool prof_on = false;
  uint32_t prof_mask = 0;               // stages bracketed while prof_on (bit s = stage s)
  int prof_open = -2;                   // stage the last mark opened (-2: none)
  std::vector<hipEvent_t> prof_ev;      // pool
  std::vector<int> prof_stage;          // stage of the interval ending at event i
  size_t prof_used = 0;
  double prof_ms[NMF_NUM_STAGES] = {0};
  int64_t prof_cnt[NMF_NUM_STAGES] = {0};
  std::string last_error;
  // when set, kernel launches are appended here instead of being issued
  std::vector<nmfk::LaunchRecord>* rec = nullptr;
};

namespace nmfk {

// Column window of a raw product: factor columns [c0, c0 + kw) only, stored
// into X (row pitch x_ld) from column x_c0 on.  Sequential ALS solves k2
// columns at a time and gathers only those.
struct ColWindow {
  int32_t c0;
  int32_t kw;
  int32_t x_ld;
  int32_t x_c0;
};

// Kernel launchers (one translation unit each), instantiated for float and
// double.  All enqueue on h->stream and return hipSuccess or the launch error.
template <typename T>
hipError_t spmm(nmf_handle* h, const Plan& p, const Factor& F, const double* W, T* X, T* C,
                bool raw, const T* dense_in, int sparse_row, bool wide = false, int waves = 8);
template <typename T>
hipError_t select_topt(nmf_handle* h, const T* X, int64_t rows, int64_t t, int mode,
                       const Factor& out_f);
template <typename T>
hipError_t mark_nonzero(nmf_handle* h, const T* X, int64_t rows);
// sparse_row: the threshold of the SpMM that will gather this factor (it
// decides what the per-row metadata points to).
template <typename T>
hipError_t repack(nmf_handle* h, const T* X, int64_t rows, const Factor& out_f, int sparse_row);
template <typename T>
hipError_t gram(nmf_handle* h, const Factor& F, const Gram& g);
template <typename T>
hipError_t metrics(nmf_handle* h, const Factor& Unew, const Factor& Uold, const T* C,
                   bool record);
template <typename T>
hipError_t densify(nmf_handle* h, const Factor& F, T* out);
template <typename T>
hipError_t check_input(nmf_handle* h, const T* x, int64_t count, int32_t* flag);
template <typename T>
hipError_t sum_squares(nmf_handle* h, const T* x, int64_t count, double* out);
template <typename T>
hipError_t loss_dot(nmf_handle* h, const T* U, const T* C, const double* GU, const double* GV,
                    double* loss_out);
template <typename T>
hipError_t gram_dense(nmf_handle* h, const T* F, int64_t rows, double* G);
template <typename T>
hipError_t grad_combine(nmf_handle* h, const T* F, const T* B, const double* G,
                        const double* g_scale, int64_t rows, T* out);
hipError_t fill_i32(hipStream_t s, int32_t* p, int32_t v, int64_t count);
// V half of float32 problems with k <= 64 (k_vhalf.hip): the whole product
// A^T U (hot block on the matrix cores, the rest streamed), the float64
// solve with W and the clamp in one kernel (W null: X receives the raw
// sums).  U's row metadata must point every nonempty row at its compact
// dense row (gather threshold 0).
hipError_t vhalf(nmf_handle* h, const Plan& p, const Factor& F, const float* dense_in, float* X, const double* W,
                 int waves);
// An empty launch record (keeps every product's launch sequence equally long).
hipError_t vhalf_placeholder(nmf_handle* h);
// Raw sums of the fused V-half kernel over a column window; F holds only the
// window's columns (compact rows of pitch F.ld, as narrow_rows writes them).
hipError_t vhalf_window(nmf_handle* h, const Plan& p, const Factor& F, float* X, const ColWindow& win);
// Raw product over a column window: the SpMM stream skipping (row filter in
// LDS) the nonzeros whose factor row stores nothing in the window, or the
// fused V-half kernel on a narrow copy of the window's columns.  S is a
// factor of F's shape whose buffers are free during the call (its values
// take the filter bits, its dense rows the narrow copy).
template <typename T>
hipError_t spmm_window(nmf_handle* h, const Plan& p, const Factor& F, T* X, const ColWindow& win, int sparse_row,
                       const Factor& S);
// (k_seq.hip) bits[w] bit i: row 32 w + i of F stores an entry in [c0, c0 + kw).
hipError_t window_bits(nmf_handle* h, const Factor& F, int c0, int kw, uint32_t* bits);
// (k_seq.hip, float) out[s][0, ldn) <- columns [c0, c0 + kw) of F's compact
// dense row s (zero past kw), for every compact row s.
hipError_t narrow_rows(nmf_handle* h, const Factor& F, int c0, int kw, int ldn, float* out);

// Sequential ALS (k_seq.hip, k_gram.hip).
template <typename T>
hipError_t gram_plain(nmf_handle* h, const Factor& F, double* G);
hipError_t block_inverse(nmf_handle* h, const double* G, int k1, int k2, double* Gb, double* W22, int32_t* dead);
template <typename T>
hipError_t seq_solve(nmf_handle* h, const T* B, T* X, int64_t rows, const Factor& F_old, const double* G,
                     const double* W22, int k1, int k2);
template <typename T>
hipError_t seq_setup(nmf_handle* h, T* X, const T* U0b, int64_t rows, int k1, int k2);
template <typename T>
hipError_t seq_save(nmf_handle* h, const T* X, T* U0b, int64_t rows, int k2);
hipError_t seq_max(nmf_handle* h, const Factor& a, const Factor& b);
// counts[c * n_labels + l] += documents with label l storing an entry in topic c
hipError_t topic_counts(nmf_handle* h, const Factor& F, const int32_t* labels, int32_t n_labels, uint32_t* counts);

}  // namespace nmfk
