// Host side of the SELL-C-sigma library: argument checking, device memory,
// the construction pipeline, work planning for long chunks, the batched
// launch with its hipGraph, the autotuner and the probes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "batch_plan.h"
#include "sell_internal.h"

using sell::Geom;

namespace {

thread_local std::string g_err;

sell_status fail(sell_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

sell_status hip_fail(const char *what, hipError_t e) {
  return fail(SELL_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define SELL_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(#call, e_);    \
  } while (0)

int combo_of(sell_dtype v, sell_dtype a) {
  if (v == SELL_F64 && a == SELL_F64) return sell::COMBO_F64_F64;
  if (v == SELL_F32 && a == SELL_F32) return sell::COMBO_F32_F32;
  if (v == SELL_F32 && a == SELL_F64) return sell::COMBO_F32_F64;
  if (v == SELL_BF16 && a == SELL_F32) return sell::COMBO_BF16_F32;
  if (v == SELL_BF16 && a == SELL_F64) return sell::COMBO_BF16_F64;
  return -1;
}

size_t dtype_size(sell_dtype d) { return d == SELL_F64 ? 8 : d == SELL_F32 ? 4 : 2; }

bool valid_C(int C) { return C >= 1 && C <= 128 && (C & (C - 1)) == 0; }

int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

struct DeviceInfo {
  int cus = 256;
  size_t lds_per_block = 64 << 10;  // shared memory one workgroup may use
};

DeviceInfo device_info() {
  DeviceInfo d;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) d.cus = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      d.lds_per_block = (size_t)v;
  }
  return d;
}

// Dynamic LDS of the x-window product with gc chunks (waves) per workgroup:
// the window, then the segment table with room for one entry per thread.
size_t xw_lds_bytes(int64_t maxwin, int64_t maxseg, size_t xsz, int gc) {
  return (((size_t)maxwin * xsz + 7) & ~(size_t)7) + 8 * (size_t)std::max<int64_t>(maxseg, 64 * (int64_t)gc);
}

// Device memory through the caller's allocator or hipMalloc.
struct Mem {
  sell_allocator alloc{};
  bool custom = false;
  void *get(size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (custom) {
      p = alloc.alloc(bytes, alloc.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    return p;
  }
  void put(void *p) {
    if (!p) return;
    if (custom) alloc.free(p, alloc.ctx);
    else (void)hipFree(p);
  }
};

// Temporary device buffers released at scope exit.
struct Temp {
  Mem mem;
  std::vector<void *> ptrs;
  explicit Temp(const Mem &m) : mem(m) {}
  void *get(size_t bytes) {
    void *p = mem.get(bytes);
    if (p) ptrs.push_back(p);
    return p;
  }
  ~Temp() {
    for (void *p : ptrs) mem.put(p);
  }
};

// Two timing events, destroyed at scope exit (also when creating the second
// one failed).
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t create() {
    const hipError_t e = hipEventCreate(&a);
    return e != hipSuccess ? e : hipEventCreate(&b);
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

void *owned_alloc(sell_matrix *h, const Mem &mem, size_t bytes) {
  Mem m = mem;
  void *p = m.get(bytes);
  if (p) {
    h->owned.push_back({p, bytes});
    h->device_bytes += (int64_t)(bytes ? bytes : 256);
  }
  return p;
}

void free_owned(sell_matrix *h) {
  Mem m;
  m.alloc = h->alloc;
  m.custom = h->custom_alloc;
  for (auto &pr : h->owned) m.put(pr.first);
  h->owned.clear();
}

// Work of one matrix: per item (row slice) its width in chunk columns, and
// the number of wave steps all items take together.
struct ItemCols {
  std::vector<int32_t> cols;  // per item
  int64_t total_steps = 0;
  int32_t max = 0;
};

ItemCols item_cols(const std::vector<int32_t> &cl, const Geom &g) {
  ItemCols r;
  r.cols.resize(cl.size() * (size_t)g.wpc);
  for (size_t c = 0; c < cl.size(); ++c) {
    for (int h = 0; h < g.wpc; ++h) r.cols[c * g.wpc + h] = cl[c];
    r.total_steps += (int64_t)((cl[c] + g.T - 1) / g.T) * g.wpc;
    r.max = std::max(r.max, cl[c]);
  }
  return r;
}

// Slots per lane when the caller leaves it open: two for FP64 values (one
// 16-byte access) unless rows are short, one for FP32 and BF16 values.
// Measured: FP64 with V = 2 is faster on the 27-point stencil (26.7 nonzeros
// per row) and on long rows, V = 1 on the power-law matrix (4.2 per row),
// whose many one- and two-column chunks leave most lanes of a 4-column step
// idle.
int default_vec(int C, sell_dtype v, int64_t nnz, int64_t nrows) {
  int V = v == SELL_F64 && nnz >= 8 * nrows ? 2 : 1;
  if (C > 64) return 1;
  while (V > C) V >>= 1;
  return V;
}

int32_t round_seg(int64_t cols) {
  int64_t a = sell::kSegAlign;
  int64_t s = (cols + a - 1) / a * a;
  if (s < a) s = a;
  if (s > (1 << 30)) s = 1 << 30;
  return (int32_t)s;
}

// Automatic segment width: long enough that a unit amortises its fixed
// cost (at least 64 wave steps), short enough that no unit is much longer
// than an average wave's share of the whole product (resident waves:
// CUs x 32). Converted from wave steps to chunk columns.
int32_t auto_seg_cols(int64_t total_steps, int T, int cus) {
  int64_t resident = (int64_t)cus * 32;
  int64_t steps = total_steps / (2 * resident);
  if (steps < 64) steps = 64;
  return round_seg(steps * T);
}

}  // namespace

// ===========================================================================
// Construction
// ===========================================================================
namespace {

// The construction; with layout_only the handle stops after the row order,
// chunk widths and offsets (no values, no column indices, no work plan) --
// enough for beta and the model's byte count.
sell_status build_impl(const sell_crs *A, int32_t C, int64_t sigma, const sell_build_opts *opts, void *stream,
                       sell_handle *out, bool layout_only) {
  if (!A || !out) return fail(SELL_ERR_INVALID_ARG, "sell_build: null argument");
  *out = nullptr;
  if (A->nrows < 0 || A->ncols < 0 || A->nnz < 0) return fail(SELL_ERR_INVALID_ARG, "sell_build: negative size");
  if (A->nrows >= (int64_t)1 << 31 || A->ncols >= (int64_t)1 << 31)
    return fail(SELL_ERR_UNSUPPORTED, "sell_build: nrows and ncols must be below 2^31");
  if (!A->rpt || (A->nnz > 0 && (!A->col || !A->val)))
    return fail(SELL_ERR_INVALID_ARG, "sell_build: null CRS array");
  if (!valid_C(C)) return fail(SELL_ERR_UNSUPPORTED, "sell_build: C must be a power of two in [1, 128]");
  if (sigma < 1) return fail(SELL_ERR_INVALID_ARG, "sell_build: sigma must be >= 1");
  sell_build_opts o{};
  if (opts) o = *opts;
  else {
    o.val_dtype = SELL_F64;
    o.acc_dtype = SELL_F64;
  }
  const int combo = combo_of(o.val_dtype, o.acc_dtype);
  if (combo < 0) return fail(SELL_ERR_UNSUPPORTED, "sell_build: unsupported (value, accumulation) dtype pair");
  if (o.unroll != 0 && o.unroll != 4 && o.unroll != 8 && o.unroll != 16)
    return fail(SELL_ERR_UNSUPPORTED, "sell_build: unroll must be 0, 4, 8 or 16");
  if (o.vec != 0 && o.vec != 1 && o.vec != 2 && o.vec != 4)
    return fail(SELL_ERR_UNSUPPORTED, "sell_build: vec must be 0, 1, 2 or 4");
  if (o.vec > 1 && (C > 64 || o.vec > C))
    return fail(SELL_ERR_UNSUPPORTED, "sell_build: vec > 1 needs C <= 64 and vec <= C");
  if (o.ktile < 0 || o.ktile > 64 || (o.ktile & (o.ktile - 1)) != 0)
    return fail(SELL_ERR_UNSUPPORTED, "sell_build: ktile must be 0 or a power of two <= 64");
  if (o.kmax < 0) return fail(SELL_ERR_INVALID_ARG, "sell_build: kmax must be >= 0");
  if (o.permute_columns && A->nrows != A->ncols)
    return fail(SELL_ERR_UNSUPPORTED, "sell_build: permute_columns needs a square matrix");
  if (o.alloc && (!o.alloc->alloc || !o.alloc->free))
    return fail(SELL_ERR_INVALID_ARG, "sell_build: allocator needs alloc and free");
  if (o.xwindow < -1 || o.xwindow > 1) return fail(SELL_ERR_INVALID_ARG, "sell_build: xwindow must be -1, 0 or 1");
  if (o.xwindow_chunks != 0 && o.xwindow_chunks != sell::kXwChunks && o.xwindow_chunks != sell::kXwChunksWide)
    return fail(SELL_ERR_INVALID_ARG, "sell_build: xwindow_chunks must be 0, 4 or 8");
  if (o.row_lengths != 0 && o.row_lengths != 1) return fail(SELL_ERR_INVALID_ARG, "sell_build: row_lengths must be 0 or 1");
  if (o.row_lengths && (C < 8 || C > 64)) return fail(SELL_ERR_UNSUPPORTED, "sell_build: row_lengths needs C in 8..64");

  hipStream_t s = static_cast<hipStream_t>(stream);
  std::unique_ptr<sell_matrix> h(new sell_matrix());
  h->nrows = A->nrows;
  h->ncols = A->ncols;
  h->nnz = A->nnz;
  h->C = C;
  h->sigma = sigma;
  h->g = sell::geom_of(C, o.vec ? o.vec : default_vec(C, o.val_dtype, A->nnz, A->nrows));
  h->vdt = o.val_dtype;
  h->adt = o.acc_dtype;
  h->xdt = o.val_dtype == SELL_F64 ? SELL_F64 : SELL_F32;
  h->combo = combo;
  h->unroll = std::min(o.unroll ? o.unroll : 8, 8);  // 16 only for the x-window kernel, set below
  h->ktile = o.ktile;
  h->kmax = o.kmax ? o.kmax : 32;
  h->sym = o.permute_columns != 0;
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
  Mem mem;
  if (o.alloc) {
    mem.alloc = *o.alloc;
    mem.custom = true;
    h->alloc = *o.alloc;
    h->custom_alloc = true;
  }
  struct Guard {
    sell_matrix *h;
    bool armed = true;
    ~Guard() {
      if (armed && h) free_owned(h);
    }
  } guard{h.get()};

  const int64_t n = A->nrows;
  const int64_t nc = (n + C - 1) / C;
  h->nchunks = nc;
  Temp tmp(mem);

  // small counters: flags (u32), maxlen (i32), sumsq (u64)
  struct Small {
    uint32_t flags;
    int32_t maxlen;
    unsigned long long sumsq;
    int64_t padded;
  };
  Small *dsmall = static_cast<Small *>(tmp.get(sizeof(Small)));
  int32_t *len = static_cast<int32_t *>(tmp.get(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1)));
  if (!dsmall || !len) return fail(SELL_ERR_OOM, "sell_build: temporary allocation failed");
  SELL_HIP(hipMemsetAsync(dsmall, 0, sizeof(Small), s));
  SELL_HIP(sell::build_rowlen(A->rpt, n, A->nnz, len, &dsmall->flags, &dsmall->sumsq, &dsmall->maxlen, s));
  SELL_HIP(sell::build_colcheck(A->col, A->nnz, A->ncols, &dsmall->flags, s));

  // sigma-window sort
  int64_t sig = std::min<int64_t>(sigma, std::max<int64_t>(n, 1));
  if (sig > 1 && n > 1) {
    h->perm = static_cast<int32_t *>(owned_alloc(h.get(), mem, sizeof(int32_t) * (size_t)n));
    uint64_t *ka = nullptr, *kb = nullptr;
    if (sig > 4096) {
      ka = static_cast<uint64_t *>(tmp.get(sizeof(uint64_t) * (size_t)n));
      kb = static_cast<uint64_t *>(tmp.get(sizeof(uint64_t) * (size_t)n));
      if (!ka || !kb) return fail(SELL_ERR_OOM, "sell_build: sort buffers");
    }
    if (!h->perm) return fail(SELL_ERR_OOM, "sell_build: perm");
    SELL_HIP(sell::build_sort(len, n, sig, ka, kb, h->perm, s));
  }

  // chunk widths and offsets
  h->cl = static_cast<int32_t *>(owned_alloc(h.get(), mem, sizeof(int32_t) * (size_t)std::max<int64_t>(nc, 1)));
  h->cs = static_cast<int64_t *>(owned_alloc(h.get(), mem, sizeof(int64_t) * (size_t)(nc + 1)));
  int64_t *scan_tmp = static_cast<int64_t *>(tmp.get(sizeof(int64_t) * (size_t)sell::scan_tmp_elems(nc + 1)));
  if (!h->cl || !h->cs || !scan_tmp) return fail(SELL_ERR_OOM, "sell_build: chunk arrays");
  SELL_HIP(sell::build_chunkwidth(len, h->perm, n, C, nc, h->cl, h->cs, s));
  SELL_HIP(sell::build_scan(h->cs, h->cs, nc + 1, scan_tmp, s));
  SELL_HIP(hipMemcpyAsync(&dsmall->padded, h->cs + nc, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  Small hs{};
  SELL_HIP(hipMemcpyAsync(&hs, dsmall, sizeof(Small), hipMemcpyDeviceToHost, s));
  SELL_HIP(hipStreamSynchronize(s));
  if (hs.flags) {
    std::string why;
    if (hs.flags & 1u) why += " rpt[0] != 0;";
    if (hs.flags & 2u) why += " rpt decreases;";
    if (hs.flags & 8u) why += " rpt[nrows] != nnz;";
    if (hs.flags & 16u) why += " a row is longer than 2^31-1;";
    if (hs.flags & 4u) why += " column index outside [0, ncols);";
    return fail(SELL_ERR_BAD_CRS, "sell_build: malformed CRS:" + why);
  }
  h->padded = hs.padded;
  h->max_len = hs.maxlen;
  h->beta = h->padded == 0 ? 1.0 : (double)h->nnz / (double)h->padded;
  if (n > 0 && h->nnz > 0) {
    long double mean = (long double)h->nnz / (long double)n;
    long double var = (long double)hs.sumsq / (long double)n - mean * mean;
    if (var < 0) var = 0;
    h->zeta = (double)(std::sqrt((double)var) / (double)mean);
  }

  if (layout_only) {
    SELL_HIP(hipStreamSynchronize(s));
    h->nunits = h->nitems = nc * h->g.wpc;
    guard.armed = false;
    *out = h.release();
    return SELL_OK;
  }

  // padded column-major arrays
  if (h->padded > 0) {
    h->col = static_cast<int32_t *>(owned_alloc(h.get(), mem, sizeof(int32_t) * (size_t)h->padded));
    h->val = owned_alloc(h.get(), mem, dtype_size(h->vdt) * (size_t)h->padded);
    if (!h->col || !h->val) return fail(SELL_ERR_OOM, "sell_build: padded arrays");
    int32_t *iperm = nullptr;
    if (h->sym && h->perm) {
      iperm = static_cast<int32_t *>(tmp.get(sizeof(int32_t) * (size_t)n));
      if (!iperm) return fail(SELL_ERR_OOM, "sell_build: inverse permutation");
      SELL_HIP(sell::build_invert(h->perm, n, iperm, s));
    }
    SELL_HIP(sell::build_fill(A->rpt, A->col, A->val, n, C, h->perm, len, h->cs, nc, h->padded, iperm, h->col,
                              h->val, (int)h->vdt, s));
  }
  // length of every row in sorted order, for the product whose lanes stop at
  // their rows' ends
  if (o.row_lengths) {
    h->rl = static_cast<int32_t *>(owned_alloc(h.get(), mem, sizeof(int32_t) * (size_t)std::max<int64_t>(nc * C, 1)));
    if (!h->rl) return fail(SELL_ERR_OOM, "sell_build: row lengths");
    SELL_HIP(sell::build_sorted_len(len, h->perm, n, nc * C, h->rl, s));
  }

  // host copy of the chunk widths, then the work plan
  h->h_cl.resize((size_t)nc);
  if (nc > 0) SELL_HIP(hipMemcpyAsync(h->h_cl.data(), h->cl, sizeof(int32_t) * (size_t)nc, hipMemcpyDeviceToHost, s));
  SELL_HIP(hipStreamSynchronize(s));

  const Geom &g = h->g;
  h->nitems = nc * g.wpc;
  ItemCols st = item_cols(h->h_cl, g);
  DeviceInfo di = device_info();
  int32_t S = o.seg_cols > 0 ? round_seg(o.seg_cols) : auto_seg_cols(st.total_steps, g.T, di.cus);
  h->seg_cols = S;
  if (o.seg_cols >= 0 && st.max > S) {
    std::vector<sell::Unit> units;
    std::vector<sell::SplitDesc> splits;
    int64_t off = 0;
    // split items first: they are the longest work, so they start earliest
    for (int64_t it = 0; it < h->nitems; ++it) {
      int32_t w = st.cols[(size_t)it];
      if (w <= S) continue;
      int32_t nseg = (w + S - 1) / S;
      int32_t sid = (int32_t)splits.size();
      splits.push_back({(int32_t)it, nseg, off});
      off += (int64_t)nseg * g.rpw;
      for (int32_t q = 0; q < nseg; ++q) units.push_back({(int32_t)it, q, nseg, sid});
    }
    for (int64_t it = 0; it < h->nitems; ++it)
      if (st.cols[(size_t)it] <= S) units.push_back({(int32_t)it, 0, 1, 0});
    h->nunits = (int64_t)units.size();
    h->nsplit = (int64_t)splits.size();
    h->nsegs = off / g.rpw;
    const int64_t kcap = next_pow2(h->kmax);
    h->units = static_cast<sell::Unit *>(owned_alloc(h.get(), mem, sizeof(sell::Unit) * units.size()));
    h->splits = static_cast<sell::SplitDesc *>(owned_alloc(h.get(), mem, sizeof(sell::SplitDesc) * splits.size()));
    h->partial = owned_alloc(h.get(), mem, sizeof(double) * (size_t)(off * kcap));
    if (!h->units || !h->splits || !h->partial) return fail(SELL_ERR_OOM, "sell_build: work plan");
    SELL_HIP(hipMemcpyAsync(h->units, units.data(), sizeof(sell::Unit) * units.size(), hipMemcpyHostToDevice, s));
    SELL_HIP(hipMemcpyAsync(h->splits, splits.data(), sizeof(sell::SplitDesc) * splits.size(),
                            hipMemcpyHostToDevice, s));
    // the single-vector product's list: runs of 64 / C whole chunks at most
    // 64 / C columns wide become one unit each (one wave covers all their rows)
    if (C >= 8 && C <= 32) {
      const size_t grp = (size_t)(64 / C);
      const int32_t wmax = 64 / C;
      size_t nwhole = 0;
      for (int64_t it = 0; it < h->nitems; ++it) nwhole += st.cols[(size_t)it] <= S;
      std::vector<sell::Unit> u1(units.begin(), units.end() - (ptrdiff_t)nwhole);  // the split segments
      int64_t ngroups = 0;
      for (size_t it = 0; it < (size_t)h->nitems; ++it) {
        const int32_t w = st.cols[it];
        if (w > S) continue;
        if (w <= wmax && it + grp <= (size_t)h->nitems) {
          size_t e = it + 1;
          while (e < it + grp && st.cols[e] <= wmax) ++e;
          if (e == it + grp) {
            u1.push_back({(int32_t)it, 0, 0, 0});
            ++ngroups;
            it = e - 1;
            continue;
          }
        }
        u1.push_back({(int32_t)it, 0, 1, 0});
      }
      if (ngroups > 0) {
        h->units1 = static_cast<sell::Unit *>(owned_alloc(h.get(), mem, sizeof(sell::Unit) * u1.size()));
        if (!h->units1) return fail(SELL_ERR_OOM, "sell_build: work plan");
        h->nunits1 = (int64_t)u1.size();
        SELL_HIP(hipMemcpyAsync(h->units1, u1.data(), sizeof(sell::Unit) * u1.size(), hipMemcpyHostToDevice, s));
        SELL_HIP(hipStreamSynchronize(s));  // u1 ends with this scope
      }
    }
    SELL_HIP(hipStreamSynchronize(s));
  } else {
    h->nunits = h->nitems;
  }

  // x windows for LDS staging: when they fit (xwindow 0) or required (1)
  if (o.xwindow >= 0) {
    const int V = g.V;
    const int64_t ngroups_all = (nc + sell::kXwChunks - 1) / sell::kXwChunks;
    const bool shape_ok = C >= 8 && C <= 64 && (V == 1 || V == 2 || (V == 4 && C >= 16 && h->vdt != SELL_F64)) &&
                          !h->units && h->padded > 0;
    // automatic mode skips small matrices: with fewer than two workgroups per
    // CU the product is latency-bound and the staging round trip only adds
    // to it (the 128^2 Laplacian: 2.4 us per call without, 3.1 with)
    const bool big_enough = o.xwindow == 1 || ngroups_all >= 2 * (int64_t)di.cus;
    if (!shape_ok || !big_enough) {
      if (o.xwindow == 1)
        return fail(SELL_ERR_UNSUPPORTED,
                    "sell_build: the x window needs C in 8..64, vec 1 or 2 (or 4 with FP32/BF16 values and C >= 16) "
                    "and no split chunks");
    } else {
      // at C = 32, groups of kXwChunksWide chunks when their windows fit
      // (fewer workgroups stage the x lines that neighbouring chunks share;
      // measured on the 27-point stencil, 160^3: FP64 +1 %, FP32 +3 to 6 %,
      // BF16 +5 to 8 %), else of kXwChunks (at C = 16 the wide groups ran
      // 4 to 15 % slower, at C = 64 they exceed the slot limit of a group
      // and, with a limit twice as large, ran no faster); an explicit
      // xwindow_chunks builds that size only
      struct XwSmall {
        uint32_t flags;
        int32_t maxwin;
        int32_t maxseg;
        int32_t pad;
        int64_t nseg;
      };
      const size_t xsz = h->xdt == SELL_F64 ? 8 : 4;
      XwSmall *dxs = static_cast<XwSmall *>(tmp.get(sizeof(XwSmall)));
      const int64_t ngroups_max = (nc + sell::kXwChunks - 1) / sell::kXwChunks;
      int64_t *cnt = static_cast<int64_t *>(tmp.get(sizeof(int64_t) * (size_t)(ngroups_max + 1)));
      int64_t *offs = static_cast<int64_t *>(tmp.get(sizeof(int64_t) * (size_t)(ngroups_max + 1)));
      int64_t *stmp =
          static_cast<int64_t *>(tmp.get(sizeof(int64_t) * (size_t)sell::scan_tmp_elems(ngroups_max + 1)));
      if (!dxs || !cnt || !offs || !stmp) return fail(SELL_ERR_OOM, "sell_build: x window temporaries");
      int gcs[2] = {sell::kXwChunksWide, sell::kXwChunks};
      int ngc = 2;
      if (o.xwindow_chunks != 0) {
        gcs[0] = o.xwindow_chunks;
        ngc = 1;
      }
      XwSmall xs{};
      int gc = 0;
      int64_t ngroups = 0;
      for (int i = 0; i < ngc && gc == 0; ++i) {
        ngroups = (nc + gcs[i] - 1) / gcs[i];
        // the automatic choice keeps two workgroups per compute unit
        if (ngc > 1 && i + 1 < ngc && (C != 32 || (o.xwindow != 1 && ngroups < 2 * (int64_t)di.cus))) continue;
        SELL_HIP(hipMemsetAsync(dxs, 0, sizeof(XwSmall), s));
        SELL_HIP(sell::build_xw_count(h->col, h->cs, nc, gcs[i], cnt, &dxs->flags, &dxs->maxwin, &dxs->maxseg, s));
        SELL_HIP(sell::build_scan(cnt, offs, ngroups + 1, stmp, s));
        SELL_HIP(hipMemcpyAsync(&dxs->nseg, offs + ngroups, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        SELL_HIP(hipMemcpyAsync(&xs, dxs, sizeof(XwSmall), hipMemcpyDeviceToHost, s));
        SELL_HIP(hipStreamSynchronize(s));
        // window budget per wave of the workgroup: 4 KiB (16 KiB when required)
        const size_t budget = (o.xwindow == 1 ? (size_t)16 << 10 : (size_t)4 << 10) * (size_t)gcs[i];
        if (!xs.flags && (size_t)xs.maxwin * xsz <= budget && xs.maxseg <= sell::kXwMaxSeg &&
            xw_lds_bytes(xs.maxwin, xs.maxseg, xsz, gcs[i]) <= di.lds_per_block)
          gc = gcs[i];
      }
      if (gc == 0) {
        if (o.xwindow == 1)
          return fail(SELL_ERR_UNSUPPORTED,
                      "sell_build: x window too large (more than 8192 slots or 1024 column runs per group, "
                      "window over 16 KiB per chunk of the group, or more LDS than a workgroup may use)");
      } else {
        h->xsegoff = static_cast<int64_t *>(owned_alloc(h.get(), mem, sizeof(int64_t) * (size_t)(ngroups + 1)));
        h->xseg = static_cast<int32_t *>(owned_alloc(h.get(), mem, sizeof(int32_t) * 3 * (size_t)xs.nseg));
        h->lcol = static_cast<uint16_t *>(owned_alloc(h.get(), mem, sizeof(uint16_t) * (size_t)h->padded));
        if (!h->xsegoff || !h->xseg || !h->lcol) return fail(SELL_ERR_OOM, "sell_build: x window arrays");
        SELL_HIP(hipMemcpyAsync(h->xsegoff, offs, sizeof(int64_t) * (size_t)(ngroups + 1), hipMemcpyDeviceToDevice,
                                s));
        SELL_HIP(sell::build_xw_fill(h->col, h->cs, nc, gc, h->xsegoff, h->xseg, h->lcol, s));
        SELL_HIP(hipStreamSynchronize(s));
        h->xw_gc = gc;
        h->nxseg = xs.nseg;
        h->xwin_max = xs.maxwin;
        h->xseg_max = xs.maxseg;
        // with the window, FP32/BF16 values run faster with two slots per
        // lane (measured on the 27-point stencil: BF16 at C = 64 2,524 ->
        // 2,615 GF/s); the work plan (one item per chunk, nothing split)
        // does not depend on it
        if (o.vec == 0 && h->vdt != SELL_F64 && g.V == 1) h->g = sell::geom_of(C, 2);
        // with two slots per lane the window kernel keeps eight wave steps
        // in flight by default (measured on the 27-point stencil at C = 32:
        // FP64 1,186 -> 1,228 GF/s, BF16 2,170 -> 2,389; neutral at C = 64)
        if (h->g.V >= 2 && (o.unroll == 0 || o.unroll == 16)) h->unroll = 16;
      }
    }
  }
  guard.armed = false;
  *out = h.release();
  return SELL_OK;
}

}  // namespace

extern "C" sell_status sell_build(const sell_crs *A, int32_t C, int64_t sigma, const sell_build_opts *opts,
                                  void *stream, sell_handle *out) {
  return build_impl(A, C, sigma, opts, stream, out, false);
}

// ===========================================================================
// Products
// ===========================================================================
namespace {

sell::SpmvArgs args_of(const sell_matrix *h, const void *x, void *y) {
  sell::SpmvArgs a{};
  a.val = h->val;
  a.col = h->col;
  a.cs = h->cs;
  a.cl = h->cl;
  a.perm = h->sym ? nullptr : h->perm;  // symmetric mode: y is written in sorted order
  a.x = x;
  a.y = y;
  a.nrows = h->nrows;
  a.nwork = h->units ? h->nunits : h->nitems;
  a.units = h->units;
  a.splits = h->splits;
  a.nsplit = h->units ? h->nsplit : 0;
  a.partial = h->partial;
  a.seg_cols = h->seg_cols;
  a.k = 1;
  a.kt = 1;
  return a;
}

}  // namespace

namespace {

// The product on handle h; `partial` (non-null) replaces the handle's
// partial-sum buffer for the segment sums of split chunks.
sell_status spmv_run(sell_handle h, const void *x, void *y, void *stream, void *partial, const char *who) {
  if (!h) return fail(SELL_ERR_INVALID_ARG, std::string(who) + ": null handle");
  if ((h->nrows > 0 && !y) || (h->ncols > 0 && !x))
    return fail(SELL_ERR_INVALID_ARG, std::string(who) + ": null vector");
  if (h->nrows == 0) return SELL_OK;
  sell::SpmvArgs a = args_of(h, x, y);
  if (partial) a.partial = partial;
  a.rl = h->rl;  // row_lengths: each row's lanes stop at its end
  if (h->units1) {  // whole chunks of width 0 or 1 grouped 64 / C per wave
    a.units = h->units1;
    a.nwork = h->nunits1;
  }
  // padding-heavy layouts skip the gathers of their zero slots; near-dense
  // chunks skip the per-slot test
  const bool skip_zero = h->beta < 0.9;
  hipError_t e;
  if (h->lcol) {  // x windows staged in LDS
    const sell::XwArgs w{h->lcol, h->xsegoff, h->xseg, h->xwin_max, h->xw_gc};
    const size_t lds = xw_lds_bytes(h->xwin_max, h->xseg_max, h->xdt == SELL_F64 ? 8 : 4, h->xw_gc);
    e = sell::launch_spmv_xw(h->combo, h->C, h->g.V, h->unroll / h->g.V, a, w, lds, static_cast<hipStream_t>(stream));
  } else {
    e = sell::launch_spmv(h->combo, h->C, h->unroll / h->g.V, h->g.V, skip_zero, a, static_cast<hipStream_t>(stream));
  }
  if (e != hipSuccess) return hip_fail((std::string(who) + " launch").c_str(), e);
  return SELL_OK;
}

}  // namespace

extern "C" sell_status sell_spmv(sell_handle h, const void *x, void *y, void *stream) {
  return spmv_run(h, x, y, stream, nullptr, "sell_spmv");
}


namespace {

// Right-hand sides per lane (KV) for the block kernel: a power of two <= 8
// that divides k (aligned vector gathers), with the pass width G*KV not
// above the next power of two of k.
int choose_kv(const sell_matrix *h, int k, int ktile) {
  const int G = 64 / h->g.rpw;
  int want;
  if (ktile > 0) want = std::max(1, ktile / G);
  else want = (int)std::max<int64_t>(1, std::min<int64_t>(next_pow2(k), 16) / G);
  int kv = 1;
  while (kv * 2 <= want && kv * 2 <= 8 && k % (kv * 2) == 0) kv *= 2;
  return kv;
}

}  // namespace

namespace {

// Doubles of partial sums a block product of width k needs on handle h with
// passes of width kt (the one-pass row kernels: kt = k).
int64_t partial_doubles(const sell_matrix *h, int64_t k, int64_t kt) {
  if (!h->units || h->nsplit == 0) return 0;
  const int64_t ntiles = (k + kt - 1) / kt;
  return h->nsegs * (int64_t)h->g.rpw * ntiles * kt;
}

// The block product on handle h. scratch == nullptr: the handle's
// partial-sum buffer (sized at build for kmax); else a buffer of
// scratch_bytes bytes for the segment sums of split chunks.
sell_status spmmv_run(sell_handle h, const void *X, void *Y, int32_t k, void *stream, void *scratch,
                      size_t scratch_bytes, const char *who) {
  const std::string w = who;
  if (!h) return fail(SELL_ERR_INVALID_ARG, w + ": null handle");
  if (k < 1) return fail(SELL_ERR_INVALID_ARG, w + ": k must be >= 1");
  if ((h->nrows > 0 && !Y) || (h->ncols > 0 && !X)) return fail(SELL_ERR_INVALID_ARG, w + ": null block");
  if (h->combo != sell::COMBO_F64_F64) return fail(SELL_ERR_UNSUPPORTED, w + ": FP64 handles only");
  if (h->nrows == 0) return SELL_OK;
  auto too_big = [&](int64_t doubles) {
    return fail(SELL_ERR_UNSUPPORTED, w + ": the segment sums of split chunks need " +
                                          std::to_string(doubles * (int64_t)sizeof(double)) +
                                          " bytes of scratch, more than its " + std::to_string(scratch_bytes));
  };
  if (k == 1) {
    if (scratch && partial_doubles(h, 1, 1) * (int64_t)sizeof(double) > (int64_t)scratch_bytes)
      return too_big(partial_doubles(h, 1, 1));
    return spmv_run(h, X, Y, stream, scratch, who);
  }
  if (h->C < 8) return fail(SELL_ERR_UNSUPPORTED, w + ": C must be >= 8 for k > 1");
  if (!scratch && h->units && k > h->kmax) return fail(SELL_ERR_INVALID_ARG, w + ": k exceeds the kmax given at build");
  // With the automatic pass width, k = 32 and 64 run in one pass with 8
  // lanes per row and k = 16 with 4: each lane reads its share of a row of X
  // with two or four accesses of 16 bytes (X and Y aligned to 16 bytes).
  // Measured on the power-law 1M matrix at beta = 0.98 (sigma = n) / 0.14
  // (sigma = 1024), GF/s, with the right-hand sides as 16-byte pairs and the
  // columns in flight of k_spmmv_rows: k = 16 4 lanes 1,124-1,132 / 420,
  // 8 lanes 1,100 / 366 (before the pairs), pass kernel 756 / 405-407; k = 32
  // 8 lanes 1,214 / 505, 4 lanes 1,203, 16 lanes 1,131 / 410 (before the
  // pairs), pass kernel 862 / 402; k = 64 8 lanes 1,296 / 677, 16 lanes
  // 1,229 / 564, pass kernel 913 / 421; k = 8 4 lanes 626, 8 lanes 457 / 191,
  // pass kernel 686 / 293.
  {
    const int lpr = (k == 64 || k == 32) ? 8 : k == 16 ? 4 : 0;
    if (h->ktile == 0 && lpr > 0 && h->C >= 16 &&
        ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) % 16) == 0) {
      if (scratch && partial_doubles(h, k, k) * (int64_t)sizeof(double) > (int64_t)scratch_bytes)
        return too_big(partial_doubles(h, k, k));
      sell::SpmvArgs a = args_of(h, X, Y);
      if (scratch) a.partial = scratch;
      a.k = k;
      a.kt = k;
      hipError_t e = sell::launch_spmmv_rows(h->C, lpr, a, static_cast<hipStream_t>(stream));
      if (e != hipSuccess) return hip_fail((w + " launch").c_str(), e);
      return SELL_OK;
    }
  }
  int kv = choose_kv(h, k, h->ktile);
  // the gathers of KV contiguous right-hand sides and the stores of a lane's
  // KV results are vector accesses: keep them aligned (rows of X and Y are k
  // doubles apart, k % kv == 0 by choose_kv)
  while (kv > 1 && ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) % (sizeof(double) * kv)) != 0)
    kv >>= 1;
  const int KT = (64 / h->g.rpw) * kv;
  const int64_t ntiles = (k + KT - 1) / KT;
  if (!scratch && h->units && ntiles * KT > next_pow2(h->kmax))
    return fail(SELL_ERR_UNSUPPORTED, w + ": pass width exceeds the partial-sum buffer");
  if (scratch && partial_doubles(h, k, KT) * (int64_t)sizeof(double) > (int64_t)scratch_bytes)
    return too_big(partial_doubles(h, k, KT));
  sell::SpmvArgs a = args_of(h, X, Y);
  if (scratch) a.partial = scratch;
  a.k = k;
  a.kt = KT;
  hipError_t e = sell::launch_spmmv(h->C, kv, a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail((w + " launch").c_str(), e);
  return SELL_OK;
}

// Scratch of sell_spmmv_noalloc: the segment sums of split chunks, in a
// statically allocated device array (every GPU the library runs on holds its
// own copy until the process ends). Host code reaches it only through the
// device address hipGetSymbolAddress returns for the current device; the
// array's name in host code is a host-side stand-in, not that address.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of the scratch array, looked up once per
// device (with that device current) and kept.
sell_status scratch_for_current_device(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail("sell_spmmv_noalloc: hipGetDevice", e);
  if (dev < 0 || dev >= kMaxDevices) return fail(SELL_ERR_UNSUPPORTED, "sell_spmmv_noalloc: device index too large");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail("sell_spmmv_noalloc: hipGetSymbolAddress(scratch)", e);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SELL_OK;
}

}  // namespace

extern "C" sell_status sell_spmmv(sell_handle h, const void *X, void *Y, int32_t k, void *stream) {
  return spmmv_run(h, X, Y, k, stream, nullptr, 0, "sell_spmmv");
}

extern "C" sell_status sell_spmmv_noalloc(sell_handle h, const void *X, void *Y, int32_t k, void *stream) {
  if (!h) return fail(SELL_ERR_INVALID_ARG, "sell_spmmv_noalloc: null handle");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail("sell_spmmv_noalloc: hipGetDevice", e);
  if (dev != h->device)
    return fail(SELL_ERR_INVALID_ARG, "sell_spmmv_noalloc: the handle's device must be the current device");
  void *p = nullptr;
  sell_status st = scratch_for_current_device(&p);
  if (st != SELL_OK) return st;
  return spmmv_run(h, X, Y, k, stream, p, kScratchBytes, "sell_spmmv_noalloc");
}

// ===========================================================================
// Inspection
// ===========================================================================
extern "C" sell_status sell_info(sell_handle h, sell_info_t *info) {
  if (!h || !info) return fail(SELL_ERR_INVALID_ARG, "sell_info: null argument");
  sell_info_t r{};
  r.nrows = h->nrows;
  r.ncols = h->ncols;
  r.nnz = h->nnz;
  r.C = h->C;
  r.sigma = h->sigma;
  r.nchunks = h->nchunks;
  r.padded = h->padded;
  r.beta = h->beta;
  r.zeta = h->zeta;
  r.max_row_len = h->max_len;
  r.val_dtype = h->vdt;
  r.x_dtype = h->xdt;
  r.acc_dtype = h->adt;
  r.lanes_per_row = h->g.T;
  r.unroll = h->unroll;
  r.vec = h->g.V;
  r.seg_cols = h->seg_cols;
  r.nunits = h->units ? h->nunits : h->nitems;
  r.nsplit = h->nsplit;
  r.has_perm = h->perm ? 1 : 0;
  r.permuted_columns = h->sym ? 1 : 0;
  r.device_bytes = h->device_bytes;
  r.xwindow = h->lcol ? 1 : 0;
  r.xwindow_max = h->xwin_max;
  r.xsegments = h->nxseg;
  r.xwindow_group_chunks = h->lcol ? h->xw_gc : 0;
  r.row_lengths = h->rl ? 1 : 0;
  *info = r;
  return SELL_OK;
}

extern "C" sell_status sell_export(sell_handle h, int32_t *perm, int32_t *cl, int64_t *cs, int32_t *col, void *val) {
  if (!h) return fail(SELL_ERR_INVALID_ARG, "sell_export: null handle");
  SELL_HIP(hipDeviceSynchronize());
  if (perm) {
    if (h->perm) SELL_HIP(hipMemcpy(perm, h->perm, sizeof(int32_t) * (size_t)h->nrows, hipMemcpyDeviceToHost));
    else
      for (int64_t i = 0; i < h->nrows; ++i) perm[i] = (int32_t)i;
  }
  if (cl && h->nchunks > 0) SELL_HIP(hipMemcpy(cl, h->cl, sizeof(int32_t) * (size_t)h->nchunks, hipMemcpyDeviceToHost));
  if (cs) SELL_HIP(hipMemcpy(cs, h->cs, sizeof(int64_t) * (size_t)(h->nchunks + 1), hipMemcpyDeviceToHost));
  if (col && h->padded > 0) SELL_HIP(hipMemcpy(col, h->col, sizeof(int32_t) * (size_t)h->padded, hipMemcpyDeviceToHost));
  if (val && h->padded > 0)
    SELL_HIP(hipMemcpy(val, h->val, dtype_size(h->vdt) * (size_t)h->padded, hipMemcpyDeviceToHost));
  return SELL_OK;
}

extern "C" sell_status sell_export_xwindow(sell_handle h, int64_t *segoff, int32_t *seg, uint16_t *lcol) {
  if (!h) return fail(SELL_ERR_INVALID_ARG, "sell_export_xwindow: null handle");
  if (!h->lcol) return fail(SELL_ERR_UNSUPPORTED, "sell_export_xwindow: the handle has no x window");
  SELL_HIP(hipDeviceSynchronize());
  const int64_t ngroups = (h->nchunks + h->xw_gc - 1) / h->xw_gc;
  if (segoff)
    SELL_HIP(hipMemcpy(segoff, h->xsegoff, sizeof(int64_t) * (size_t)(ngroups + 1), hipMemcpyDeviceToHost));
  if (seg && h->nxseg > 0)
    SELL_HIP(hipMemcpy(seg, h->xseg, sizeof(int32_t) * 3 * (size_t)h->nxseg, hipMemcpyDeviceToHost));
  if (lcol && h->padded > 0)
    SELL_HIP(hipMemcpy(lcol, h->lcol, sizeof(uint16_t) * (size_t)h->padded, hipMemcpyDeviceToHost));
  return SELL_OK;
}

extern "C" sell_status sell_destroy(sell_handle h) {
  if (!h) return SELL_OK;
  (void)hipDeviceSynchronize();
  free_owned(h);
  delete h;
  return SELL_OK;
}

// ===========================================================================
// Batched launch
// ===========================================================================
struct sell_batch_s {
  std::vector<sell_handle> hs;
  int combo = 0, C = 0, U = 8;
  Geom g{};
  int32_t seg_cols = 0;
  int64_t nunits = 0, nsplit = 0;
  bool persistent = false;
  int32_t nwaves = 0;  // persistent form only
  sell::BatchMat *mats = nullptr;
  sell::BUnit *units = nullptr;
  int32_t *slice = nullptr;  // persistent form only
  sell::BSplitDesc *splits = nullptr;
  void *partial = nullptr;
  std::vector<sell::BatchMat> host_mats;
  bool bound = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<void *> owned;
};

namespace {

void batch_free(sell_batch_s *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (void *p : b->owned) (void)hipFree(p);
  b->owned.clear();
}

void *batch_alloc(sell_batch_s *b, size_t bytes) {
  void *p = nullptr;
  if (hipMalloc(&p, bytes ? bytes : 256) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  b->owned.push_back(p);
  return p;
}

}  // namespace

namespace {

sell_status batch_create_impl(const sell_handle *hs, int32_t count, bool persistent, sell_batch *out) {
  if (!hs || !out || count < 1) return fail(SELL_ERR_INVALID_ARG, "sell_batch_create: bad arguments");
  *out = nullptr;
  for (int32_t b = 0; b < count; ++b)
    if (!hs[b]) return fail(SELL_ERR_INVALID_ARG, "sell_batch_create: null handle");
  const sell_handle h0 = hs[0];
  for (int32_t b = 1; b < count; ++b)
    if (hs[b]->C != h0->C || hs[b]->combo != h0->combo)
      return fail(SELL_ERR_UNSUPPORTED, "sell_batch_create: all matrices must share C and dtypes");
  std::unique_ptr<sell_batch_s> B(new sell_batch_s());
  struct Guard {
    sell_batch_s *b;
    bool armed = true;
    ~Guard() {
      if (armed) batch_free(b);
    }
  } guard{B.get()};
  B->hs.assign(hs, hs + count);
  B->combo = h0->combo;
  B->C = h0->C;
  // the batched kernel: one slot per lane, 4 or 8 in flight, both forms.
  // Measured on 64 power-law matrices (sigma = n_b / 1024, us): with the
  // persistent waves' units in consecutive equal-cost slices, 4 in flight
  // (50 instead of 70 VGPRs: eight waves per SIMD instead of seven) gave
  // 172 -> 167 at sigma = n_b; with each unit dealt to the least-loaded
  // wave, 8 gives 128.0 -> 123.9 / 265.4 -> 268.3
  B->U = std::min(h0->unroll, 8);
  B->g = sell::geom_of(h0->C, 1);  // the batched kernel loads one slot per lane
  const Geom &g = B->g;

  // work of every matrix, one segment width for the whole batch
  std::vector<ItemCols> st(count);
  int64_t total = 0;
  for (int32_t b = 0; b < count; ++b) {
    st[b] = item_cols(hs[b]->h_cl, g);
    total += st[b].total_steps;
  }
  DeviceInfo di = device_info();
  const int32_t S = auto_seg_cols(total, g.T, di.cus);
  B->seg_cols = S;
  // work units of every matrix: the segments of its split chunks, then its
  // whole chunks; cost estimate of a unit: its wave steps plus a fixed charge
  std::vector<sell::BUnit> all;
  std::vector<sell::BSplitDesc> splits;
  std::vector<int32_t> umat;
  std::vector<int64_t> ucost;
  std::vector<uint8_t> usplit;
  const int64_t kFixed = 4;
  int64_t off = 0;
  for (int32_t b = 0; b < count; ++b) {
    const ItemCols &s = st[b];
    for (size_t it = 0; it < s.cols.size(); ++it) {
      const int32_t w = s.cols[it];
      if (w <= S) continue;
      const int32_t nseg = (w + S - 1) / S;
      const int32_t sid = (int32_t)splits.size();
      splits.push_back({b, (int32_t)it, nseg, 0, off});
      off += (int64_t)nseg * g.rpw;
      for (int32_t q = 0; q < nseg; ++q) {
        all.push_back({b, (int32_t)it, q, nseg, sid, {0, 0, 0}});
        const int64_t cols = std::min<int64_t>(S, (int64_t)w - (int64_t)q * S);
        umat.push_back(b);
        ucost.push_back((cols + g.T - 1) / g.T + kFixed);
        usplit.push_back(1);
      }
    }
    // whole chunks; with C in 8..32 each run of 64 / C consecutive chunks at
    // most 64 / C columns wide is one unit (nseg 0: one wave covers all their
    // rows)
    const size_t grp = B->C >= 8 && B->C <= 32 ? (size_t)(64 / B->C) : 0;
    const int32_t wmax = (int32_t)grp;
    for (size_t it = 0; it < s.cols.size(); ++it) {
      const int32_t w = s.cols[it];
      if (w > S) continue;
      if (grp && w <= wmax && it + grp <= s.cols.size()) {
        size_t e = it + 1;
        while (e < it + grp && s.cols[e] <= wmax) ++e;
        if (e == it + grp) {
          all.push_back({b, (int32_t)it, 0, 0, 0, {0, 0, 0}});
          umat.push_back(b);
          ucost.push_back(1 + kFixed);
          usplit.push_back(0);
          it = e - 1;
          continue;
        }
      }
      all.push_back({b, (int32_t)it, 0, 1, 0, {0, 0, 0}});
      umat.push_back(b);
      ucost.push_back((w + g.T - 1) / g.T + kFixed);
      usplit.push_back(0);
    }
  }
  B->nsplit = (int64_t)splits.size();

  // placement on the XCDs: each matrix (or piece of a large one) on one XCD,
  // so that its x stays in that XCD's L2 (batch_plan.h). One unit per wave
  // (filler slots where an XCD's queue is shorter), or the persistent form's
  // list of units per resident wave (each unit to the least-loaded wave of
  // its XCD).
  int64_t nwaves = 0;
  if (persistent) {
    const int wpcu = std::max(1, sell::batch_waves_per_cu(B->combo, B->C, B->U));
    const int64_t per_round = (int64_t)sell::kBatchPersistentWaves * sell::kXcds;
    nwaves = std::min<int64_t>((int64_t)di.cus * wpcu, (int64_t)all.size());
    nwaves = std::max<int64_t>(per_round, (nwaves + per_round - 1) / per_round * per_round);
  }
  const sell::XcdPlan plan = sell::plan_xcd(umat, ucost, usplit, count,
                                            persistent ? sell::kBatchPersistentWaves : sell::kWavesPerBlock,
                                            sell::kXcds, nwaves);
  std::vector<sell::BUnit> units(plan.order.size());
  for (size_t i = 0; i < plan.order.size(); ++i)
    units[i] = plan.order[i] < 0 ? sell::BUnit{-1, 0, 0, 1, 0, {0, 0, 0}} : all[(size_t)plan.order[i]];
  B->nunits = (int64_t)units.size();
  if (B->nunits >= ((int64_t)1 << 31)) return fail(SELL_ERR_UNSUPPORTED, "sell_batch_create: too many work units");
  std::vector<int32_t> slice = plan.slice;
  if (persistent) {
    B->persistent = true;
    B->nwaves = (int32_t)nwaves;
  }

  B->mats = static_cast<sell::BatchMat *>(batch_alloc(B.get(), sizeof(sell::BatchMat) * (size_t)count));
  B->units = static_cast<sell::BUnit *>(batch_alloc(B.get(), sizeof(sell::BUnit) * std::max<size_t>(1, units.size())));
  B->splits = static_cast<sell::BSplitDesc *>(
      batch_alloc(B.get(), sizeof(sell::BSplitDesc) * std::max<size_t>(1, splits.size())));
  B->partial = batch_alloc(B.get(), sizeof(double) * (size_t)std::max<int64_t>(1, off));
  if (persistent) B->slice = static_cast<int32_t *>(batch_alloc(B.get(), sizeof(int32_t) * slice.size()));
  if (!B->mats || !B->units || !B->splits || !B->partial || (persistent && !B->slice))
    return fail(SELL_ERR_OOM, "sell_batch_create: allocation failed");
  if (persistent)
    SELL_HIP(hipMemcpy(B->slice, slice.data(), sizeof(int32_t) * slice.size(), hipMemcpyHostToDevice));
  if (!units.empty())
    SELL_HIP(hipMemcpy(B->units, units.data(), sizeof(sell::BUnit) * units.size(), hipMemcpyHostToDevice));
  if (!splits.empty())
    SELL_HIP(hipMemcpy(B->splits, splits.data(), sizeof(sell::BSplitDesc) * splits.size(), hipMemcpyHostToDevice));
  B->host_mats.resize((size_t)count);
  for (int32_t b = 0; b < count; ++b) {
    sell::BatchMat &m = B->host_mats[(size_t)b];
    m.val = hs[b]->val;
    m.col = hs[b]->col;
    m.cs = hs[b]->cs;
    m.cl = hs[b]->cl;
    m.perm = hs[b]->sym ? nullptr : hs[b]->perm;
    m.x = nullptr;
    m.y = nullptr;
    m.nrows = hs[b]->nrows;
  }

  // capture the batched launch once
  sell::BatchArgs a{};
  a.mats = B->mats;
  a.units = B->units;
  a.nunits = B->nunits;
  a.slice = B->slice;
  a.nwaves = B->nwaves;
  a.splits = B->splits;
  a.nsplit = B->nsplit;
  a.partial = B->partial;
  a.seg_cols = B->seg_cols;
  hipStream_t cap = nullptr;
  SELL_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = sell::launch_batch(B->combo, B->C, B->U, a, cap);
    e = hipStreamEndCapture(cap, &B->graph);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess) return hip_fail("sell_batch_create: graph capture", e);
  guard.armed = false;
  *out = B.release();
  return SELL_OK;
}

}  // namespace

extern "C" sell_status sell_batch_create(const sell_handle *hs, int32_t count, sell_batch *out) {
  return batch_create_impl(hs, count, false, out);
}

extern "C" sell_status sell_batch_create_persistent(const sell_handle *hs, int32_t count, sell_batch *out) {
  return batch_create_impl(hs, count, true, out);
}

extern "C" sell_status sell_batch_spmv(sell_batch b, const void *const *xs, void *const *ys, void *stream) {
  if (!b || !xs || !ys) return fail(SELL_ERR_INVALID_ARG, "sell_batch_spmv: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  bool changed = !b->bound;
  for (size_t i = 0; i < b->hs.size(); ++i) {
    if ((b->hs[i]->nrows > 0 && !ys[i]) || (b->hs[i]->ncols > 0 && !xs[i]))
      return fail(SELL_ERR_INVALID_ARG, "sell_batch_spmv: null vector");
    if (b->host_mats[i].x != xs[i] || b->host_mats[i].y != ys[i]) changed = true;
  }
  if (changed) {
    // earlier launches of this batch, on any stream, may still read the table
    SELL_HIP(hipDeviceSynchronize());
    for (size_t i = 0; i < b->hs.size(); ++i) {
      b->host_mats[i].x = xs[i];
      b->host_mats[i].y = ys[i];
    }
    SELL_HIP(hipMemcpy(b->mats, b->host_mats.data(), sizeof(sell::BatchMat) * b->host_mats.size(),
                       hipMemcpyHostToDevice));
    b->bound = true;
  }
  SELL_HIP(hipGraphLaunch(b->exec, s));
  return SELL_OK;
}

extern "C" sell_status sell_batch_destroy(sell_batch b) {
  if (!b) return SELL_OK;
  (void)hipDeviceSynchronize();
  batch_free(b);
  delete b;
  return SELL_OK;
}

// ===========================================================================
// Sorted-order helpers and the CRS comparison kernels
// ===========================================================================
extern "C" sell_status sell_permute(sell_handle h, const void *x, void *xp, void *stream) {
  if (!h || ((!x || !xp) && h->nrows > 0)) return fail(SELL_ERR_INVALID_ARG, "sell_permute: null argument");
  if (h->nrows != h->ncols) return fail(SELL_ERR_UNSUPPORTED, "sell_permute: square matrices only");
  hipError_t e = sell::permute_vector(x, xp, h->perm, h->nrows, (int)dtype_size(h->xdt), false,
                                      static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail("sell_permute", e);
  return SELL_OK;
}

extern "C" sell_status sell_unpermute(sell_handle h, const void *yp, void *y, void *stream) {
  if (!h || ((!y || !yp) && h->nrows > 0)) return fail(SELL_ERR_INVALID_ARG, "sell_unpermute: null argument");
  hipError_t e = sell::permute_vector(yp, y, h->perm, h->nrows, (int)dtype_size(h->adt), true,
                                      static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail("sell_unpermute", e);
  return SELL_OK;
}

extern "C" sell_status sell_crs_spmv(const sell_crs *A, int32_t lanes_per_row, const double *x, double *y,
                                     void *stream) {
  if (!A || (A->nrows > 0 && (!A->rpt || !y)) || (A->nnz > 0 && (!A->col || !A->val || !x)))
    return fail(SELL_ERR_INVALID_ARG, "sell_crs_spmv: null argument");
  if (A->nrows < 0) return fail(SELL_ERR_INVALID_ARG, "sell_crs_spmv: negative size");
  int L = lanes_per_row;
  if (L == 0) {  // about half a wave step per row: the row length rounded down to a power of two
    double nnzr = A->nrows > 0 ? (double)A->nnz / (double)A->nrows : 1.0;
    L = 1;
    while (L < 64 && 2.0 * L <= nnzr) L *= 2;
  }
  if (L < 1 || L > 64 || (L & (L - 1)) != 0)
    return fail(SELL_ERR_UNSUPPORTED, "sell_crs_spmv: lanes_per_row must be 0 or a power of two <= 64");
  hipError_t e = sell::launch_crs(A->rpt, A->col, A->val, x, y, A->nrows, L, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail("sell_crs_spmv", e);
  return SELL_OK;
}

// ===========================================================================
// Autotuner
// ===========================================================================
extern "C" sell_status sell_autotune(const sell_crs *A, int32_t k, const sell_tune_space *space, void *stream,
                                     sell_tuned *best) {
  if (!A || !best || k < 1) return fail(SELL_ERR_INVALID_ARG, "sell_autotune: bad arguments");
  const int32_t defC[] = {16, 32, 64, 128};
  const int64_t defS[] = {1};
  const int32_t defU[] = {4, 8, 16};
  const int32_t defK[] = {0};
  sell_tune_space sp{};
  if (space) sp = *space;
  const int32_t *Cs = sp.nC > 0 ? sp.C : defC;
  int nC = sp.nC > 0 ? sp.nC : 4;
  const int64_t *Ss = sp.nsigma > 0 ? sp.sigma : defS;
  int nS = sp.nsigma > 0 ? sp.nsigma : 1;
  const int32_t *Us = sp.nunroll > 0 ? sp.unroll : defU;
  int nU = sp.nunroll > 0 ? sp.nunroll : 3;
  const int32_t *Ks = sp.nktile > 0 ? sp.ktile : defK;
  int nK = sp.nktile > 0 ? sp.nktile : 1;
  const int reps = sp.reps > 0 ? sp.reps : 20;
  const int32_t defV[] = {0}, defSeg[] = {0};
  const int32_t *Vs = sp.nvec > 0 ? sp.vec : defV;
  int nV = sp.nvec > 0 ? sp.nvec : 1;
  const int32_t *Gs = sp.nseg_cols > 0 ? sp.seg_cols : defSeg;
  int nG = sp.nseg_cols > 0 ? sp.nseg_cols : 1;
  const int32_t defX[] = {0};
  const int32_t *Xs = sp.nxwindow > 0 ? sp.xwindow : defX;
  int nX = sp.nxwindow > 0 ? sp.nxwindow : 1;
  const int32_t *Ws = sp.nxwindow_chunks > 0 ? sp.xwindow_chunks : defX;
  int nW = sp.nxwindow_chunks > 0 ? sp.nxwindow_chunks : 1;
  const int32_t *Rs = sp.nrow_lengths > 0 ? sp.row_lengths : defX;
  int nR = sp.nrow_lengths > 0 ? sp.nrow_lengths : 1;
  sell_build_opts o{};
  o.val_dtype = sp.val_dtype;
  o.acc_dtype = sp.acc_dtype;
  if (combo_of(o.val_dtype, o.acc_dtype) < 0) return fail(SELL_ERR_UNSUPPORTED, "sell_autotune: dtype pair");
  o.kmax = std::max(32, k);
  hipStream_t s = static_cast<hipStream_t>(stream);

  const size_t xs = (o.val_dtype == SELL_F64 ? 8 : 4), ys = (o.acc_dtype == SELL_F64 ? 8 : 4);
  Temp tmp(Mem{});
  void *x = tmp.get(xs * (size_t)std::max<int64_t>(1, A->ncols) * (size_t)k);
  void *y = tmp.get(ys * (size_t)std::max<int64_t>(1, A->nrows) * (size_t)k);
  if (!x || !y) return fail(SELL_ERR_OOM, "sell_autotune: vectors");
  SELL_HIP(hipMemsetAsync(x, 0, xs * (size_t)std::max<int64_t>(1, A->ncols) * (size_t)k, s));
  EventPair ev;
  SELL_HIP(ev.create());
  hipEvent_t e0 = ev.a, e1 = ev.b;

  // Model-guided search: rank every (C, sigma) by the bytes the code-balance
  // model assigns one product (padded matrix, x once, y, permutation, chunk
  // metadata -- Sect. 4 with the ideal alpha), from a layout-only build, and
  // time only the best space.model_guided of them.
  std::vector<std::pair<int, int>> order;
  int predicted = 0;
  if (sp.model_guided > 0) {
    std::vector<std::pair<double, std::pair<int, int>>> ranked;
    const double sv = (double)dtype_size(o.val_dtype), sx = (double)xs, sy = (double)ys;
    for (int ic = 0; ic < nC; ++ic)
      for (int is = 0; is < nS; ++is) {
        sell_handle h = nullptr;
        sell_status st = build_impl(A, Cs[ic], Ss[is], &o, stream, &h, true);
        if (st == SELL_ERR_UNSUPPORTED || st == SELL_ERR_INVALID_ARG) continue;
        if (st != SELL_OK) return st;
        const double kk = (double)k;
        double bytes = (sv + 4.0) * (double)h->padded + sx * kk * (double)A->ncols + sy * kk * (double)A->nrows +
                       (h->perm ? 4.0 * (double)A->nrows : 0.0) + 12.0 * (double)h->nchunks;
        ranked.push_back({bytes, {ic, is}});
        ++predicted;
        sell_destroy(h);
      }
    std::stable_sort(ranked.begin(), ranked.end(),
                     [](const std::pair<double, std::pair<int, int>> &a, const std::pair<double, std::pair<int, int>> &b) {
                       return a.first < b.first;
                     });
    for (size_t q = 0; q < ranked.size() && (int)q < sp.model_guided; ++q) order.push_back(ranked[q].second);
  } else {
    for (int ic = 0; ic < nC; ++ic)
      for (int is = 0; is < nS; ++is) order.push_back({ic, is});
  }

  sell_tuned r{};
  r.gflops = -1.0;
  int cands = 0;
  for (const auto &cand : order) {
    for (int iv = 0; iv < nV * nG * nX * nW * nR; ++iv) {
      const int ic = cand.first, is = cand.second;
      // slots per lane, split width, x path, window workgroup size and row
      // lengths are build parameters: one build each
      o.vec = Vs[iv % nV];
      o.seg_cols = Gs[(iv / nV) % nG];
      o.xwindow = Xs[(iv / (nV * nG)) % nX];
      o.xwindow_chunks = Ws[(iv / (nV * nG * nX)) % nW];
      o.row_lengths = Rs[iv / (nV * nG * nX * nW)];
      // row lengths need C in 8..64 and serve the single-vector product only
      if (o.row_lengths && (Cs[ic] < 8 || Cs[ic] > 64 || k > 1)) continue;
      sell_handle h = nullptr;
      sell_status st = sell_build(A, Cs[ic], Ss[is], &o, stream, &h);
      if (st == SELL_ERR_UNSUPPORTED || st == SELL_ERR_INVALID_ARG) continue;
      if (st != SELL_OK) return st;
      // without a window the size does not change the product: time it for
      // the first size of the list only
      if (!h->lcol && (iv / (nV * nG * nX)) % nW > 0) {
        sell_destroy(h);
        continue;
      }
      // the window product does not read the row lengths: nothing to time
      if (h->lcol && h->rl) {
        sell_destroy(h);
        continue;
      }
      for (int iu = 0; iu < nU; ++iu) {
        if (Us[iu] != 4 && Us[iu] != 8 && Us[iu] != 16) continue;
        // sixteen slots in flight: only the window kernel with two or four per lane
        if (Us[iu] == 16 && !(h->lcol && h->g.V >= 2)) continue;
        for (int ik = 0; ik < (k > 1 ? nK : 1); ++ik) {
          h->unroll = std::max(Us[iu], h->g.V);
          h->ktile = k > 1 ? Ks[ik] : 0;
          auto call = [&]() { return k > 1 ? sell_spmmv(h, x, y, k, stream) : sell_spmv(h, x, y, stream); };
          sell_status cs = SELL_OK;
          for (int w = 0; w < 3 && cs == SELL_OK; ++w) cs = call();
          if (cs != SELL_OK) continue;
          (void)hipEventRecord(e0, s);
          for (int q = 0; q < reps; ++q) call();
          (void)hipEventRecord(e1, s);
          if (hipEventSynchronize(e1) != hipSuccess) {
            sell_destroy(h);
            return hip_fail("sell_autotune: timing", hipGetLastError());
          }
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          double t = (double)ms * 1e-3 / reps;
          double gf = t > 0 ? 2.0 * (double)A->nnz * k / t * 1e-9 : 0.0;
          ++cands;
          if (gf > r.gflops) {
            r.C = Cs[ic];
            r.sigma = Ss[is];
            r.vec = h->g.V;
            r.seg_cols = h->seg_cols;
            r.unroll = Us[iu];
            r.ktile = h->ktile;
            r.xwindow = h->lcol ? 1 : 0;
            r.xwindow_chunks = h->lcol ? h->xw_gc : 0;
            r.row_lengths = h->rl ? 1 : 0;
            r.gflops = gf;
            r.us_per_call = t * 1e6;
            r.beta = h->beta;
          }
        }
      }
      sell_destroy(h);
    }
  }
  r.candidates = cands;
  r.predicted = predicted;
  if (cands == 0) return fail(SELL_ERR_UNSUPPORTED, "sell_autotune: no configuration could be measured");
  *best = r;
  return SELL_OK;
}

extern "C" sell_status sell_batch_autotune(const sell_crs *As, int32_t count, const sell_tune_space *space,
                                           void *stream, sell_batch_tuned *best, int64_t *sigma_out) {
  if (!As || count < 1 || !best || !sigma_out) return fail(SELL_ERR_INVALID_ARG, "sell_batch_autotune: bad arguments");
  const int32_t defC[] = {16, 32, 64};
  const int64_t defS[] = {1, 1024, (int64_t)1 << 40};
  sell_tune_space sp{};
  if (space) sp = *space;
  const int32_t *Cs = sp.nC > 0 ? sp.C : defC;
  const int nC = sp.nC > 0 ? sp.nC : 3;
  const int64_t *Ss = sp.nsigma > 0 ? sp.sigma : defS;
  const int nS = sp.nsigma > 0 ? sp.nsigma : 3;
  const int reps = sp.reps > 0 ? sp.reps : 20;
  sell_build_opts o{};
  o.val_dtype = sp.val_dtype;
  o.acc_dtype = sp.acc_dtype;
  if (combo_of(o.val_dtype, o.acc_dtype) < 0) return fail(SELL_ERR_UNSUPPORTED, "sell_batch_autotune: dtype pair");
  hipStream_t s = static_cast<hipStream_t>(stream);

  // one x and one y per matrix, carved from two buffers (offsets rounded to
  // 32 elements)
  const size_t xs = o.val_dtype == SELL_F64 ? 8 : 4, ys = o.acc_dtype == SELL_F64 ? 8 : 4;
  std::vector<size_t> xoff(count), yoff(count);
  size_t xtot = 0, ytot = 0;
  int64_t nnz = 0;
  for (int32_t b = 0; b < count; ++b) {
    xoff[b] = xtot;
    yoff[b] = ytot;
    xtot += (size_t)(std::max<int64_t>(As[b].ncols, 1) + 31) / 32 * 32;
    ytot += (size_t)(std::max<int64_t>(As[b].nrows, 1) + 31) / 32 * 32;
    nnz += As[b].nnz;
  }
  Temp tmp(Mem{});
  char *x = static_cast<char *>(tmp.get(xs * xtot));
  char *y = static_cast<char *>(tmp.get(ys * ytot));
  if (!x || !y) return fail(SELL_ERR_OOM, "sell_batch_autotune: vectors");
  SELL_HIP(hipMemsetAsync(x, 0, xs * xtot, s));
  std::vector<const void *> xp(count);
  std::vector<void *> yp(count);
  for (int32_t b = 0; b < count; ++b) {
    xp[b] = x + xs * xoff[b];
    yp[b] = y + ys * yoff[b];
  }
  EventPair ev;
  SELL_HIP(ev.create());
  hipEvent_t e0 = ev.a, e1 = ev.b;
  // handles and batch of one candidate, released on every exit
  struct Trial {
    std::vector<sell_handle> hs;
    sell_batch bt = nullptr;
    void clear() {
      if (bt) sell_batch_destroy(bt);
      bt = nullptr;
      for (sell_handle h : hs) sell_destroy(h);
      hs.clear();
    }
    ~Trial() { clear(); }
  } trial;

  const double sv = (double)dtype_size(o.val_dtype);
  sell_batch_tuned r{};
  r.gflops = -1.0;
  std::vector<int64_t> sig(count), best_sig(count);
  for (int ic = 0; ic < nC; ++ic) {
    const int32_t C = Cs[ic];
    bool ok = true;
    for (int32_t b = 0; b < count && ok; ++b) {
      double best_bytes = -1.0;
      for (int is = 0; is < nS; ++is) {
        sell_handle h = nullptr;
        sell_status st = build_impl(&As[b], C, Ss[is], &o, stream, &h, true);
        if (st == SELL_ERR_UNSUPPORTED || st == SELL_ERR_INVALID_ARG) continue;
        if (st != SELL_OK) return st;
        const double bytes = (sv + 4.0) * (double)h->padded + (h->perm ? 4.0 * (double)h->nrows : 0.0);
        if (best_bytes < 0 || bytes < best_bytes) {
          best_bytes = bytes;
          sig[b] = Ss[is];
        }
        sell_destroy(h);
      }
      if (best_bytes < 0) ok = false;
    }
    if (!ok) continue;
    trial.hs.assign(count, nullptr);
    for (int32_t b = 0; b < count; ++b) {
      sell_status st = sell_build(&As[b], C, sig[b], &o, stream, &trial.hs[b]);
      if (st != SELL_OK) return st;
    }
    sell_status st = sell_batch_create(trial.hs.data(), count, &trial.bt);
    if (st != SELL_OK) return st;
    for (int w = 0; w < 3 && st == SELL_OK; ++w) st = sell_batch_spmv(trial.bt, xp.data(), yp.data(), stream);
    if (st != SELL_OK) return st;
    (void)hipEventRecord(e0, s);
    for (int q = 0; q < reps; ++q) (void)sell_batch_spmv(trial.bt, xp.data(), yp.data(), stream);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) return hip_fail("sell_batch_autotune: timing", hipGetLastError());
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double t = (double)ms * 1e-3 / reps;
    const double gf = t > 0 ? 2.0 * (double)nnz / t * 1e-9 : 0.0;
    ++r.candidates;
    if (gf > r.gflops) {
      r.C = C;
      r.gflops = gf;
      r.us_per_call = t * 1e6;
      best_sig = sig;
    }
    trial.clear();
  }
  if (r.candidates == 0) return fail(SELL_ERR_UNSUPPORTED, "sell_batch_autotune: no C suits every matrix");
  for (int32_t b = 0; b < count; ++b) sigma_out[b] = best_sig[b];
  *best = r;
  return SELL_OK;
}

// ===========================================================================
// Bandwidth probes
// ===========================================================================
extern "C" sell_status sell_probe_bandwidth(int32_t kind, size_t bytes, int32_t reps, void *stream, double *gbs) {
  if (!gbs || reps < 1 || kind < 0 || kind > 9 || bytes < (1u << 20))
    return fail(SELL_ERR_INVALID_ARG, "sell_probe_bandwidth: bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  bytes = bytes / 64 * 64;
  Temp tmp(Mem{});
  const size_t abytes = kind == 1 ? bytes / 2 : bytes;
  // second buffer: the copy's target, or the output rows of kinds 7-9
  const size_t bbytes = kind == 1 ? bytes / 2 : kind >= 7 ? bytes : 0;
  void *a = tmp.get(abytes);
  void *b = bbytes ? tmp.get(bbytes) : nullptr;
  double *sink = static_cast<double *>(tmp.get(sizeof(double) * 256 * 16));
  if (!a || !sink || (bbytes && !b)) return fail(SELL_ERR_OOM, "sell_probe_bandwidth: buffers");
  SELL_HIP(hipMemsetAsync(a, 0, abytes, s));
  int64_t moved = (int64_t)bytes;  // bytes counted per pass
  auto run = [&]() {
    if (kind == 0) return sell::probe_read(a, bytes, sink, s);
    if (kind == 1) return sell::probe_copy(a, b, bytes / 2, s);
    if (kind == 6) return sell::probe_write(a, bytes, s);
    hipError_t e = hipSuccess;
    if (kind == 2) {
      moved = sell::probe_gather(a, bytes, sink, s, &e) * (int64_t)sizeof(double);
    } else if (kind >= 7) {
      const int row_bytes = 128 << (kind - 7);  // kinds 7, 8, 9: rows of 128, 256, 512 bytes
      moved = sell::probe_rows_write(a, b, bytes, row_bytes, s, &e) * (int64_t)row_bytes;
    } else {
      const int row_bytes = 128 << (kind - 3);  // kinds 3, 4, 5: rows of 128, 256, 512 bytes
      moved = sell::probe_rows(a, bytes, row_bytes, sink, s, &e) * (int64_t)row_bytes;
    }
    return e;
  };
  SELL_HIP(run());
  EventPair ev;
  SELL_HIP(ev.create());
  hipEvent_t e0 = ev.a, e1 = ev.b;
  double total_ms = 0.0;
  hipError_t err = hipSuccess;
  for (int r = 0; r < reps && err == hipSuccess; ++r) {
    (void)hipEventRecord(e0, s);
    err = run();
    (void)hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    total_ms += ms;
  }
  if (err != hipSuccess) return hip_fail("sell_probe_bandwidth", err);
  *gbs = (double)moved * reps / (total_ms * 1e-3) * 1e-9;
  return SELL_OK;
}

extern "C" const char *sell_status_string(sell_status s) {
  switch (s) {
    case SELL_OK: return "SELL_OK";
    case SELL_ERR_INVALID_ARG: return "SELL_ERR_INVALID_ARG";
    case SELL_ERR_BAD_CRS: return "SELL_ERR_BAD_CRS";
    case SELL_ERR_OOM: return "SELL_ERR_OOM";
    case SELL_ERR_UNSUPPORTED: return "SELL_ERR_UNSUPPORTED";
    case SELL_ERR_HIP: return "SELL_ERR_HIP";
  }
  return "SELL_ERR_UNKNOWN";
}

extern "C" const char *sell_last_error(void) { return g_err.c_str(); }
