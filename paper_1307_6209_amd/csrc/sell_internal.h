// Internal declarations shared by the host orchestration and the kernels of
// the SELL-C-sigma library (gfx950). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sellcs.h"

namespace sell {

// One work unit of an spMVM launch: a row slice ("item") of a chunk and the
// range of chunk columns it covers. Items are (chunk, half) pairs: a chunk of
// C <= 64 rows is one item; C = 128 is two items of 64 rows. A unit with
// nseg == 1 covers the whole item and writes y directly; otherwise it is
// segment seg of nseg of split slice sid, and it stores its row sums for the
// combining kernel.
struct Unit {
  int32_t item;
  int32_t seg;
  int32_t nseg;
  int32_t sid;
};

// A row slice whose chunk is split: its nseg segments stored their row sums
// at partial[poff + seg*rpw + r] (block form: see k_spmmv); a second kernel
// adds them in segment order.
struct SplitDesc {
  int32_t item;
  int32_t nseg;
  int64_t poff;
};

// Work unit of the batched kernel (adds the matrix index; mat < 0: an empty
// unit that only fills the grid).
struct BUnit {
  int32_t mat;
  int32_t item;
  int32_t seg;
  int32_t nseg;
  int32_t sid;
  int32_t pad[3];
};

// Geometry of a chunk height on a 64-lane wavefront whose lanes each hold
// V consecutive slots of a wave step (V > 1 only for C <= 64).
struct Geom {
  int C;    // chunk height
  int V;    // slots (rows) per lane
  int rpw;  // rows of one item (min(C, 64))
  int T;    // chunk columns per wave step (64 * V / rpw)
  int wpc;  // items (waves) per chunk (C / 64 for C = 128, else 1)
};

inline Geom geom_of(int C, int V = 1) {
  Geom g;
  g.C = C;
  g.V = V;
  g.rpw = C < 64 ? C : 64;
  g.T = 64 * V / g.rpw;
  g.wpc = C > 64 ? C / 64 : 1;
  return g;
}

// Waves per workgroup of the kernels that give each wave one work unit.
constexpr int kWavesPerBlock = 4;
// Waves per workgroup of the persistent batched kernel: one (its waves run
// slices of different lengths; a workgroup holds its CU slots until its
// last wave ends).
constexpr int kBatchPersistentWaves = 1;
// Accelerator dies (XCDs) of the device, each with its own L2; the hardware
// dispatcher sends workgroup b of a launch to XCD b mod kXcds.
constexpr int kXcds = 8;

// Segments of split chunks are whole multiples of this many chunk columns,
// so that every kernel's step width (at most 64 columns) divides them.
constexpr int kSegAlign = 64;

// Arguments of the spMVM kernels (by value).
struct SpmvArgs {
  const void *val;
  const int32_t *col;
  const int64_t *cs;
  const int32_t *cl;
  const int32_t *perm;  // nullptr: identity
  const void *x;
  void *y;
  int64_t nrows;
  int64_t nwork;        // items (no unit list) or units
  const Unit *units;    // nullptr: wave w handles item w whole
  const SplitDesc *splits;
  int64_t nsplit;
  void *partial;
  int32_t seg_cols;     // chunk columns per segment (multiple of kSegAlign)
  const int32_t *rl;    // single-vector product: length of every row in sorted
                        // order (N_c * C entries), or nullptr
  // block form only
  int32_t k;            // right-hand sides
  int32_t kt;           // right-hand sides per pass (ktile)
};

// Per-matrix descriptor of the batched kernel (device resident).
struct BatchMat {
  const void *val;
  const int32_t *col;
  const int64_t *cs;
  const int32_t *cl;
  const int32_t *perm;
  const void *x;
  void *y;
  int64_t nrows;
};

// Split row slice of the batched kernel.
struct BSplitDesc {
  int32_t mat;
  int32_t item;
  int32_t nseg;
  int32_t pad;
  int64_t poff;
};

struct BatchArgs {
  const BatchMat *mats;
  const BUnit *units;
  int64_t nunits;
  const int32_t *slice;  // persistent form: nwaves + 1 unit offsets; nullptr: one unit per wave
  int32_t nwaves;
  const BSplitDesc *splits;
  int64_t nsplit;
  void *partial;
  int32_t seg_cols;
};

// x window of a product workgroup (LDS staging): groups of G consecutive
// chunks (G = kXwChunksWide when the windows of that many fit, else
// kXwChunks), at most kXwMaxSlots slots each.
constexpr int kXwChunks = 4;
constexpr int kXwChunksWide = 8;
constexpr int kXwMaxSlots = 8192;
struct XwArgs {
  const uint16_t *lcol;   // window position of every slot
  const int64_t *segoff;  // ngroups + 1 segment offsets
  const int32_t *seg;     // per segment: start column, window position, length
  int32_t wcap;           // LDS elements reserved for the window (the largest one)
  int32_t gc;             // chunks per group (one wave each): kXwChunks or kXwChunksWide
};
// Most segments a group's window may have (its table is staged in LDS too).
constexpr int kXwMaxSeg = 1024;

enum DtypeCombo {
  COMBO_F64_F64 = 0,   // val f64, x f64, acc f64
  COMBO_F32_F32 = 1,   // val f32, x f32, acc f32
  COMBO_F32_F64 = 2,   // val f32, x f32, acc f64
  COMBO_BF16_F32 = 3,  // val bf16, x f32, acc f32
  COMBO_BF16_F64 = 4,  // val bf16, x f32, acc f64
};

// Kernel launchers (return hipError of the launch).
// Each launcher enqueues the product kernel and, when rows are split, the
// kernel that adds their segment sums.
// skip_zero: slots holding value 0 skip their gather (for padding-heavy layouts).
hipError_t launch_spmv(int combo, int C, int U, int V, bool skip_zero, const SpmvArgs &a, hipStream_t s);
hipError_t launch_spmmv(int C, int KV, const SpmvArgs &a, hipStream_t s);
// Block form with LPR lanes per row (LPR 4: k = 16; LPR 8: k = 32 or 64;
// C >= 16): one pass, a.kt == a.k.
hipError_t launch_spmmv_rows(int C, int LPR, const SpmvArgs &a, hipStream_t s);
// Product with the x window staged in LDS (C in 8..64, V 1 or 2, no split
// chunks); lds_bytes: the largest window times the x element size, rounded
// up to 8 bytes, plus 8 bytes per segment of the largest segment table.
hipError_t launch_spmv_xw(int combo, int C, int V, int U, const SpmvArgs &a, const XwArgs &w, size_t lds_bytes,
                          hipStream_t s);
hipError_t launch_batch(int combo, int C, int U, const BatchArgs &a, hipStream_t s);
// Resident waves per CU of the persistent batched kernel (its grid size).
int batch_waves_per_cu(int combo, int C, int U);

// Build kernels.
hipError_t build_rowlen(const int64_t *rpt, int64_t n, int64_t nnz, int32_t *len, uint32_t *flags,
                        unsigned long long *sumsq, int32_t *maxlen, hipStream_t s);
hipError_t build_colcheck(const int32_t *col, int64_t nnz, int64_t ncols, uint32_t *flags, hipStream_t s);
// Sorted row order for sigma > 1. keys_a/keys_b: two scratch arrays of n uint64.
hipError_t build_sort(const int32_t *len, int64_t n, int64_t sigma, uint64_t *keys_a, uint64_t *keys_b,
                      int32_t *perm, hipStream_t s);
hipError_t build_chunkwidth(const int32_t *len, const int32_t *perm, int64_t n, int C, int64_t nchunks,
                            int32_t *cl, int64_t *csz, hipStream_t s);
// Exclusive scan of n int64 values (in-place allowed); tmp needs scan_tmp_elems(n) int64.
int64_t scan_tmp_elems(int64_t n);
hipError_t build_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s);
// cmap: column map applied to every stored column index (nullptr: none).
hipError_t build_fill(const int64_t *rpt, const int32_t *col, const double *val, int64_t n, int C,
                      const int32_t *perm, const int32_t *len, const int64_t *cs, int64_t nchunks,
                      int64_t padded, const int32_t *cmap, int32_t *scol, void *sval, int val_dtype,
                      hipStream_t s);
hipError_t build_invert(const int32_t *perm, int64_t n, int32_t *iperm, hipStream_t s);
// rl[p] = length of the row in sorted position p (0 for p >= n), p < np
hipError_t build_sorted_len(const int32_t *len, const int32_t *perm, int64_t n, int64_t np, int32_t *rl,
                            hipStream_t s);
// x windows of groups of gc consecutive chunks: segment count per group
// (nseg: ngroups + 1 int64, the last set to 0), the largest window (*maxwin,
// zeroed by the caller), flag bit 1 when a group holds more than kXwMaxSlots
// slots; then the segments and the window position of every slot.
hipError_t build_xw_count(const int32_t *col, const int64_t *cs, int64_t nchunks, int gc, int64_t *nseg,
                          uint32_t *flags, int32_t *maxwin, int32_t *maxseg, hipStream_t s);
hipError_t build_xw_fill(const int32_t *col, const int64_t *cs, int64_t nchunks, int gc, const int64_t *segoff,
                         int32_t *seg, uint16_t *lcol, hipStream_t s);
// out[p] = in[perm[p]] (scatter = false) or out[perm[p]] = in[p] (scatter = true).
hipError_t permute_vector(const void *in, void *out, const int32_t *perm, int64_t n, int elem_bytes, bool scatter,
                          hipStream_t s);
hipError_t launch_crs(const int64_t *rpt, const int32_t *col, const double *val, const double *x, double *y,
                      int64_t n, int L, hipStream_t s);

// Bandwidth probes.
hipError_t probe_read(const void *a, size_t bytes, double *sink, hipStream_t s);
hipError_t probe_copy(const void *a, void *b, size_t bytes, hipStream_t s);
hipError_t probe_write(void *a, size_t bytes, hipStream_t s);
// Four random rows of row_bytes read per row written in order, over an input
// of the largest power-of-two row count that fits in bytes and an output of
// as many rows; returns the rows moved (read and written).
int64_t probe_rows_write(const void *a, void *out, size_t bytes, int row_bytes, hipStream_t s, hipError_t *err);
// Launches 2^27 random 8-byte gathers over the largest power-of-two prefix
// of a (bytes); returns the gather count.
int64_t probe_gather(const void *a, size_t bytes, double *sink, hipStream_t s, hipError_t *err);
// Launches random whole-row reads (rows of row_bytes = 128, 256 or 512 bytes)
// over the largest power-of-two number of rows that fits in bytes; returns
// the row count.
int64_t probe_rows(const void *a, size_t bytes, int row_bytes, double *sink, hipStream_t s, hipError_t *err);

}  // namespace sell

// The handle.
struct sell_matrix {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  int32_t C = 0;
  int64_t sigma = 1;
  sell::Geom g{};
  int64_t nchunks = 0, padded = 0;
  int64_t max_len = 0;
  double beta = 1.0, zeta = 0.0;
  sell_dtype vdt = SELL_F64, xdt = SELL_F64, adt = SELL_F64;
  int combo = 0;
  int32_t unroll = 8;
  int32_t seg_cols = 0;
  int32_t ktile = 0;
  int32_t kmax = 32;
  bool sym = false;  // column indices permuted too: x and y live in sorted order
  int device = 0;

  int32_t *perm = nullptr;
  int32_t *rl = nullptr;   // row_lengths: length of every row in sorted order (N_c * C)
  int32_t *cl = nullptr;
  int64_t *cs = nullptr;
  int32_t *col = nullptr;
  void *val = nullptr;

  int64_t nitems = 0;
  int64_t nunits = 0;
  sell::Unit *units = nullptr;  // nullptr when no chunk is split
  // the single-vector product's units: the same, with each run of 64 / C
  // chunks of width 0 or 1 as one unit (nseg 0; C <= 32); nullptr: units
  sell::Unit *units1 = nullptr;
  int64_t nunits1 = 0;
  int64_t nsplit = 0;
  int64_t nsegs = 0;                  // total segments of split items
  sell::SplitDesc *splits = nullptr;  // per split id
  void *partial = nullptr;            // nsegs * rpw * next_pow2(kmax) doubles

  uint16_t *lcol = nullptr;     // x window mode: window position of every slot
  int64_t *xsegoff = nullptr;   // ngroups + 1 segment offsets
  int32_t *xseg = nullptr;      // per segment: start column, window position, length
  int64_t nxseg = 0;
  int32_t xwin_max = 0;         // largest window, in x elements
  int32_t xseg_max = 0;         // most segments of one window
  int32_t xw_gc = 0;            // chunks per window group

  std::vector<int32_t> h_cl;    // host copy of the chunk widths (batch planning)

  sell_allocator alloc{};
  bool custom_alloc = false;
  std::vector<std::pair<void *, size_t>> owned;
  int64_t device_bytes = 0;
};
