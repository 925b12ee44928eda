// SELL-C-sigma spMVM kernels for gfx950 (64-lane wavefronts).
//
// The product y = A x follows Listing "SELL-4-sigma spMVM kernel" of
// Kreutzer et al. (arXiv:1307.6209), generalised to any C: chunk i holds
// cl[i] columns of C values stored column by column from cs[i]; lane r of a
// chunk accumulates val[cs[i] + j*C + r] * x[col[...]] over j, and the sum is
// stored at y[perm[i*C + r]].
//
// Mapping onto a wavefront. A wave owns rpw = min(C, 64) rows of one chunk
// (C = 128 uses two waves per chunk). When C < 64 the T = 64 / C lanes of a
// row split its columns: lane l = t*C + r takes columns j = t, t+T, ... so
// one wave step loads the 64 consecutive slots cs + s*64 + l -- fully
// coalesced streaming of val and col with no gaps, whatever C is. The T
// partial sums of a row are then added across lanes (the multiple-threads-
// per-row scheme the paper discusses for GPUs, Sects. 3.4 and 5.2, done
// inside one wavefront). val and col are read once, with non-temporal
// loads, so that the x vector keeps the caches; x is gathered through
// L2/MALL. Consecutive workgroups take consecutive chunks: all XCDs stream
// neighbouring parts of the matrix at the same time (measured faster than
// giving each XCD a contiguous range of its own, which keeps x in one L2
// but spreads the streams over eight distant regions).
//
// Long chunks. A chunk wider than seg_cols columns is cut into
// segments that run on different waves; each segment stores its row sums in
// a partial buffer and a second, small kernel adds them in segment order and
// writes y. The result does not depend on the order the waves ran in, and no
// cross-wave synchronisation (with its cache write-back and invalidation) is
// needed inside the product kernel.
#pragma once

#include "sell_internal.h"

#include <type_traits>

namespace sell {
namespace dev {

template <int COMBO>
struct Types;
template <>
struct Types<COMBO_F64_F64> {
  using V = double;
  using X = double;
  using A = double;
};
template <>
struct Types<COMBO_F32_F32> {
  using V = float;
  using X = float;
  using A = float;
};
template <>
struct Types<COMBO_F32_F64> {
  using V = float;
  using X = float;
  using A = double;
};
template <>
struct Types<COMBO_BF16_F32> {
  using V = uint16_t;
  using X = float;
  using A = float;
};
template <>
struct Types<COMBO_BF16_F64> {
  using V = uint16_t;
  using X = float;
  using A = double;
};

// Streaming (non-temporal) loads of N consecutive elements; N > 1 uses one
// vector access, so the base must be aligned to N elements.
template <int N, typename T>
__device__ __forceinline__ void ld_stream(const T *p, T (&out)[N]) {
  if constexpr (N == 1) {
    out[0] = __builtin_nontemporal_load(p);
  } else {
    typedef T vt __attribute__((ext_vector_type(N)));
    const vt v = __builtin_nontemporal_load(reinterpret_cast<const vt *>(p));
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = v[i];
  }
}

__device__ __forceinline__ double ld_val(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ int32_t ld_col(const int32_t *p) { return __builtin_nontemporal_load(p); }

// Stored value -> arithmetic type (bfloat16 -> binary32 is exact).
__device__ __forceinline__ double cvt(double v) { return v; }
__device__ __forceinline__ float cvt(float v) { return v; }
__device__ __forceinline__ float cvt(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float cvt(uint32_t b) { return __uint_as_float(b << 16); }  // bfloat16 bits held in 32

__device__ __forceinline__ double fmac(double v, double x, double acc) { return __builtin_fma(v, x, acc); }
__device__ __forceinline__ double fmac(float v, float x, double acc) {
  return __builtin_fma((double)v, (double)x, acc);  // the product is exact in double
}
__device__ __forceinline__ float fmac(float v, float x, float acc) { return __builtin_fmaf(v, x, acc); }

// Loads wave steps s0 .. s0+U-1 of one lane at slot offset off0 + step *
// stride of the arrays ci_base and v_base; ok[u] says which steps hold a
// column of the chunk (step below se, column t + step*T below cl), and the
// lanes of a partial step past the chunk load slot 0 instead (callers skip
// the slots with ok[u] false; the arrays must hold a slot). Steps past the
// chunk (a condition uniform over the wave; on short chunks most of a
// batch) are skipped by a branch, except where one lane holds two 16-bit
// elements in a word: around such a load a branch makes the compiler unpack
// the word inside it and wait for each load before issuing the next. Values
// narrower than 32 bits are returned widened (R), so that the compiler does
// not pack the values of several steps into shared registers either.
//
// lim (<= cl) limits the loads only: a lane whose step lies at or past lim
// loads slot 0 instead (the caller then zeroes what it loaded).
template <int U, int VV, typename I, typename V, typename R>
__device__ __forceinline__ void ld_batch(const I *ci_base, const V *v_base, int64_t off0, int64_t stride, int s0,
                                         int se, int T, int t, int cl, int lim, bool (&ok)[U], I (&ci)[U][VV],
                                         R (&raw)[U][VV]) {
  constexpr bool kSkip = VV == 1 || (sizeof(I) >= 4 && sizeof(V) >= 4);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int ss = s0 + u;
    ok[u] = ss < se && ss * T + t < cl;
    if (!kSkip || ss < se) {
      const int64_t o = ok[u] && ss * T + t < lim ? off0 + (int64_t)ss * stride : 0;
      ld_stream<VV>(ci_base + o, ci[u]);
      V r[VV];
      ld_stream<VV>(v_base + o, r);
#pragma unroll
      for (int v = 0; v < VV; ++v) raw[u][v] = (R)r[v];
    }
  }
}

// An empty statement that takes v in a register and may change it: the
// compiler can no longer fold the conversions of v that follow into the
// blocks that loaded it (a load in a per-step branch followed there by a
// conversion makes the step wait for its own load before the next issues).
template <typename T>
__device__ __forceinline__ void opaque(T &v) {
  asm volatile("" : "+v"(v));
}


// One work unit: rows [h*rpw, (h+1)*rpw) of chunk `chunk`, chunk columns
// [seg*seg_cols, ...) of it (all of them when nseg == 1).
//
// Lane l holds the VV consecutive slots VV*l .. VV*l+VV-1 of every wave step
// (64*VV consecutive slots = T chunk columns of RPW rows): rows
// rl0 .. rl0+VV-1 with rl0 = (VV*l) % RPW, column offset t = (VV*l) / RPW.
// With ZS (1 or 2), slots holding value 0 (padding) skip the gather; that
// pays on padding-heavy layouts and costs a compare per slot on dense ones.
// With ZS == 2 the lane also holds the lengths of its rows (rlp, in sorted
// order) and loads nothing past them -- the GPU form of the kernel in which
// each row's lane runs only to the row's own length (Sect. 3.4): a step past
// all of a lane's rows loads slot 0 (one line every lane shares) and the
// slots past a row's end are zeroed, so the arithmetic -- padding multiplies
// zero by zero -- and the result are those of the plain product.
template <int COMBO, int C, int U, int VV, int ZS>
__device__ __forceinline__ void spmv_unit(const void *__restrict__ valv, const int32_t *__restrict__ col,
                                          const int64_t *__restrict__ cs, const int32_t *__restrict__ clp,
                                          const int32_t *__restrict__ perm, const void *__restrict__ xv,
                                          void *__restrict__ yv, int64_t nrows, int32_t item, int32_t seg,
                                          int32_t nseg, int64_t poff, void *__restrict__ partial,
                                          int32_t seg_cols, int lane, const int32_t *__restrict__ rlp = nullptr) {
  constexpr bool RL = ZS == 2;
  using V = typename Types<COMBO>::V;
  using X = typename Types<COMBO>::X;
  using A = typename Types<COMBO>::A;
  constexpr int RPW = C < 64 ? C : 64;
  static_assert(VV == 1 || C <= 64, "several slots per lane need C <= 64");
  static_assert(RPW % VV == 0, "VV must divide the rows of an item");
  constexpr int T = 64 * VV / RPW;          // chunk columns per wave step
  constexpr int WPC = C > 64 ? C / 64 : 1;
  constexpr int LPC = RPW / VV;             // lanes covering one chunk column
  constexpr int64_t STRIDE = (int64_t)T * C;  // slots between two steps of a lane

  const int64_t chunk = item / WPC;
  const int h = item - (int)(chunk * WPC);
  const int rl0 = (VV * lane) % RPW, t = (VV * lane) / RPW;
  const int64_t base = cs[chunk];
  const int cl = clp[chunk];
  int jb = 0, je = cl;
  if (nseg > 1) {
    jb = seg * seg_cols;
    je = jb + seg_cols < cl ? jb + seg_cols : cl;
  }
  const int sb = jb / T, se = (je + T - 1) / T;
  const int full = je / T;  // steps below this one hold a real column in every lane
  const int64_t off0 = base + (int64_t)t * C + h * RPW + rl0;
  const int32_t *cp = col + off0;
  const V *vp = static_cast<const V *>(valv) + off0;
  const X *x = static_cast<const X *>(xv);
  // ZS == 2: the lengths of the lane's rows and the longest of them
  int rlen[VV];
  int lmax = je;
  if constexpr (RL) {
    lmax = 0;
#pragma unroll
    for (int v = 0; v < VV; ++v) {
      rlen[v] = rlp[chunk * C + h * RPW + rl0 + v];
      lmax = rlen[v] > lmax ? rlen[v] : lmax;
    }
  }

  A acc[VV];
#pragma unroll
  for (int v = 0; v < VV; ++v) acc[v] = 0;
  int s = sb;
  for (; s + U <= full; s += U) {
    int32_t ci[U][VV];
    V raw[U][VV];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (RL) {
        const bool live = (s + u) * T + t < lmax;
        ld_stream<VV>(live ? cp + (int64_t)(s + u) * STRIDE : col, ci[u]);
        ld_stream<VV>(live ? vp + (int64_t)(s + u) * STRIDE : static_cast<const V *>(valv), raw[u]);
      } else {
        ld_stream<VV>(cp + (int64_t)(s + u) * STRIDE, ci[u]);
        ld_stream<VV>(vp + (int64_t)(s + u) * STRIDE, raw[u]);
      }
    }
    if constexpr (RL) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < VV; ++v)
          if ((s + u) * T + t >= rlen[v]) {
            raw[u][v] = 0;
            ci[u][v] = 0;
          }
    }
    X xg[U][VV];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < VV; ++v) xg[u][v] = (!ZS || raw[u][v] != 0) ? x[ci[u][v]] : (X)0;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < VV; ++v) acc[v] = fmac(cvt(raw[u][v]), xg[u][v], acc[v]);
  }
  if (s < se) {  // at most U steps remain; the last one may be partial
    int32_t ci[U][VV];
    // one 16-bit value per lane is held in 32 bits (cvt takes either)
    using R = typename std::conditional<sizeof(V) < 4 && VV == 1, uint32_t, V>::type;
    R raw[U][VV];
    bool ok[U];
    ld_batch<U, VV>(col, static_cast<const V *>(valv), off0, STRIDE, s, se, T, t, je, lmax, ok, ci, raw);
    if constexpr (RL) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < VV; ++v)
          if ((s + u) * T + t >= rlen[v]) {
            raw[u][v] = 0;
            ci[u][v] = 0;
          }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < VV; ++v) {
        opaque(ci[u][v]);
        opaque(raw[u][v]);
      }
    X xg[U][VV];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < VV; ++v) xg[u][v] = (ok[u] && (!ZS || raw[u][v] != 0)) ? x[ci[u][v]] : (X)0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ok[u]) {
#pragma unroll
        for (int v = 0; v < VV; ++v) acc[v] = fmac(cvt(raw[u][v]), xg[u][v], acc[v]);
      }
  }
  // add the T partial sums of each row: lanes l, l + LPC, l + 2*LPC, ...
#pragma unroll
  for (int off = 32; off >= LPC; off >>= 1)
#pragma unroll
    for (int v = 0; v < VV; ++v) acc[v] += __shfl_xor(acc[v], off);

  A *y = static_cast<A *>(yv);
  const int64_t p0 = chunk * C + h * RPW + rl0;
  if (t != 0) return;
  if (nseg == 1) {
    if constexpr (VV > 1) {
      if (!perm && p0 + VV <= nrows &&
          (reinterpret_cast<uintptr_t>(y + p0) & (VV * sizeof(A) - 1)) == 0) {  // VV consecutive rows: one store
        typedef A avt __attribute__((ext_vector_type(VV)));
        avt o;
#pragma unroll
        for (int v = 0; v < VV; ++v) o[v] = acc[v];
        __builtin_nontemporal_store(o, reinterpret_cast<avt *>(y + p0));
        return;
      }
    }
#pragma unroll
    for (int v = 0; v < VV; ++v) {
      const int64_t p = p0 + v;
      if (p < nrows) __builtin_nontemporal_store(acc[v], y + (perm ? (int64_t)perm[p] : p));
    }
    return;
  }
  // segment of a split row slice: leave the sums for the combining kernel
  A *part = static_cast<A *>(partial) + poff + (int64_t)seg * RPW + rl0;
#pragma unroll
  for (int v = 0; v < VV; ++v) part[v] = acc[v];
}

// Raw buffer loads over the slots of one chunk. The descriptor (uniform over
// the wave) covers exactly the chunk's bytes; a load at an offset past them
// returns zero and touches no memory, so the partial last step of a chunk,
// steps past its end and empty chunks need neither a branch nor a substitute
// address. Loads are streaming (non-temporal).
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const T *p, int64_t slots) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(p), (short)0, (int)(slots * (int64_t)sizeof(T)),
                                           0x00020000);
}

constexpr int kBufStream = 2;  // cache policy: non-temporal

template <int N, typename T>
__device__ __forceinline__ void ld_buf(__amdgpu_buffer_rsrc_t r, uint32_t slot, T (&out)[N]) {
  constexpr int B = N * (int)sizeof(T);
  const uint32_t off = slot * (uint32_t)sizeof(T);
  if constexpr (B == 2) {
    const unsigned short v = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, kBufStream);
    __builtin_memcpy(out, &v, 2);
  } else if constexpr (B == 4) {
    const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kBufStream);
    __builtin_memcpy(out, &v, 4);
  } else if constexpr (B == 8) {
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kBufStream);
    __builtin_memcpy(out, &v, 8);
  } else {
    static_assert(B == 16, "2, 4, 8 or 16 bytes per lane");
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kBufStream);
    __builtin_memcpy(out, &v, 16);
  }
}

// Product with the x window in LDS. Workgroup g (GC waves, one chunk each) first issues its first U wave steps of val and of the 16-bit window
// positions, then stages its window -- every element with one load, its
// segment found by binary search -- and after the barrier runs the steps of
// spmv_unit (same lanes, same order of the multiply-adds, same cross-lane
// sum: the result equals the global-index product bit for bit) with x read
// from LDS.
constexpr int64_t kXcdTile = 16;  // groups of chunks per XCD tile

template <int COMBO, int C, int VV, int U, int GC>
__global__ void __launch_bounds__(64 * GC) k_spmv_xw(SpmvArgs a, XwArgs xa) {
  using V = typename Types<COMBO>::V;
  using X = typename Types<COMBO>::X;
  using A = typename Types<COMBO>::A;
  static_assert(C <= 64 && C % VV == 0, "one wave covers a chunk");
  constexpr int T = 64 * VV / C;           // chunk columns per wave step
  constexpr int LPC = C / VV;              // lanes covering one chunk column
  constexpr int64_t STRIDE = (int64_t)T * C;
  extern __shared__ unsigned char xw_lds[];
  X *xw = reinterpret_cast<X *>(xw_lds);

  // Workgroup b runs on XCD b mod 8. Consecutive groups of chunks share
  // most of their x lines, so each XCD takes tiles of kXcdTile consecutive
  // groups (the last, partial round of tiles keeps the plain order): the
  // staging loads find more of their lines in that XCD's L2.
  int64_t g = blockIdx.x;
  {
    const int64_t nb = gridDim.x, xcd = g % 8, i = g / 8;
    if (g < nb / (8 * kXcdTile) * (8 * kXcdTile))
      g = (i / kXcdTile) * 8 * kXcdTile + xcd * kXcdTile + i % kXcdTile;
  }
  const int lane = threadIdx.x & 63;
  // the wave's chunk, marked uniform so that its descriptors are scalar
  const int64_t chunk = g * GC + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const bool live = chunk < a.nwork;
  const int64_t base = live ? a.cs[chunk] : 0;
  const int cl = live ? a.cl[chunk] : 0;
  const int rl0 = (VV * lane) % C, t = (VV * lane) / C;
  // slot of step s of this lane within the chunk: s * STRIDE + lo0
  const uint32_t lo0 = (uint32_t)(t * C + rl0);
  const __amdgpu_buffer_rsrc_t rc = chunk_rsrc(xa.lcol + base, (int64_t)C * cl);
  const __amdgpu_buffer_rsrc_t rv = chunk_rsrc(static_cast<const V *>(a.val) + base, (int64_t)C * cl);
  const int full = cl / T, se = (cl + T - 1) / T;

  // The group's segment table (start column, window position) goes to LDS
  // behind the window, which has room for at least one entry per thread.
  // This thread's first entry is loaded ahead of the matrix steps and stored
  // unconditionally (threads past the table store a copy of entry 0 that is
  // never read), so that the store waits for that load only and the load
  // cannot move behind the matrix steps (a table entry always exists: the
  // layout holds a slot).
  int2 *segt = reinterpret_cast<int2 *>(xw_lds + (((size_t)xa.wcap * sizeof(X) + 7) & ~(size_t)7));
  const int64_t s0 = xa.segoff[g];
  const int ns = (int)(xa.segoff[g + 1] - s0);
  const int64_t e0 = (int)threadIdx.x < ns ? s0 + threadIdx.x : 0;
  const int2 seg0 = make_int2(xa.seg[3 * e0], xa.seg[3 * e0 + 1]);
  // steps 0 .. U-1; ok: the step holds a column of the chunk in this lane
  uint16_t ci[U][VV];
  V raw[U][VV];
  bool ok[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    ok[u] = u * T + t < cl;
    ld_buf<VV>(rc, lo0 + (uint32_t)(u * STRIDE), ci[u]);
    ld_buf<VV>(rv, lo0 + (uint32_t)(u * STRIDE), raw[u]);
  }
  // stage the window: every window element with one load, its segment found
  // by binary search in LDS
  {
    const X *x = static_cast<const X *>(a.x);
    segt[threadIdx.x] = seg0;
    for (int k = threadIdx.x + 64 * GC; k < ns; k += 64 * GC)
      segt[k] = make_int2(xa.seg[3 * (s0 + k)], xa.seg[3 * (s0 + k) + 1]);
    const int nwin = ns > 0 ? xa.seg[3 * (s0 + ns - 1) + 1] + xa.seg[3 * (s0 + ns - 1) + 2] : 0;
    __syncthreads();
    constexpr int K = 8;
    for (int b = 0; b < nwin; b += 64 * GC * K) {
      X tmp[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = b + k * 64 * GC + (int)threadIdx.x;
        tmp[k] = (X)0;
        if (i < nwin) {
          int lo = 0, hi = ns - 1;  // last segment with position <= i
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (segt[mid].y <= i) lo = mid;
            else hi = mid - 1;
          }
          tmp[k] = x[segt[lo].x + (i - segt[lo].y)];
        }
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = b + k * 64 * GC + (int)threadIdx.x;
        if (i < nwin) xw[i] = tmp[k];
      }
    }
  }
  __syncthreads();
  if (!live) return;

  A acc[VV];
#pragma unroll
  for (int v = 0; v < VV; ++v) acc[v] = 0;
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (ok[u]) {
#pragma unroll
      for (int v = 0; v < VV; ++v) acc[v] = fmac(cvt(raw[u][v]), xw[ci[u][v]], acc[v]);
    }
  int s = U;
  for (; s + U <= full; s += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ld_buf<VV>(rc, lo0 + (uint32_t)((s + u) * STRIDE), ci[u]);
      ld_buf<VV>(rv, lo0 + (uint32_t)((s + u) * STRIDE), raw[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < VV; ++v) acc[v] = fmac(cvt(raw[u][v]), xw[ci[u][v]], acc[v]);
  }
  if (s < se) {  // at most U steps remain, loaded together; the last may be partial
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = (s + u) * T + t < cl;
      ld_buf<VV>(rc, lo0 + (uint32_t)((s + u) * STRIDE), ci[u]);
      ld_buf<VV>(rv, lo0 + (uint32_t)((s + u) * STRIDE), raw[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ok[u]) {
#pragma unroll
        for (int v = 0; v < VV; ++v) acc[v] = fmac(cvt(raw[u][v]), xw[ci[u][v]], acc[v]);
      }
  }
#pragma unroll
  for (int off = 32; off >= LPC; off >>= 1)
#pragma unroll
    for (int v = 0; v < VV; ++v) acc[v] += __shfl_xor(acc[v], off);
  if (t != 0) return;
  A *y = static_cast<A *>(a.y);
  const int64_t p0 = chunk * C + rl0;
  if constexpr (VV > 1) {
    if (!a.perm && p0 + VV <= a.nrows && (reinterpret_cast<uintptr_t>(y + p0) & (VV * sizeof(A) - 1)) == 0) {
      typedef A avt __attribute__((ext_vector_type(VV)));
      avt o;
#pragma unroll
      for (int v = 0; v < VV; ++v) o[v] = acc[v];
      __builtin_nontemporal_store(o, reinterpret_cast<avt *>(y + p0));
      return;
    }
  }
#pragma unroll
  for (int v = 0; v < VV; ++v) {
    const int64_t p = p0 + v;
    if (p < a.nrows) __builtin_nontemporal_store(acc[v], y + (a.perm ? (int64_t)a.perm[p] : p));
  }
}

// Adds the segment sums of split row slices in segment order and writes y.
// One wave per split slice.
template <int COMBO, int C>
__device__ __forceinline__ void combine_split(const SplitDesc d, const int32_t *__restrict__ perm,
                                              const void *__restrict__ partial, void *__restrict__ yv,
                                              int64_t nrows, int lane) {
  using A = typename Types<COMBO>::A;
  constexpr int RPW = C < 64 ? C : 64;
  constexpr int WPC = C > 64 ? C / 64 : 1;
  if (lane >= RPW) return;
  const int64_t chunk = d.item / WPC;
  const int h = d.item - (int)(chunk * WPC);
  const int64_t p = chunk * C + h * RPW + lane;
  if (p >= nrows) return;
  const A *part = static_cast<const A *>(partial) + d.poff + lane;
  // sixteen loads in flight, added in order; the last round reads +0 past
  // the last segment (adding +0 leaves every sum but -0 unchanged, and -0
  // only turns into +0), so that it too is one round trip
  A sum = 0;
  for (int q = 0; q < d.nseg; q += 16) {
    A t[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = q + e < d.nseg ? part[(int64_t)(q + e) * RPW] : (A)0;
#pragma unroll
    for (int e = 0; e < 16; ++e) sum += t[e];
  }
  const int64_t row = perm ? (int64_t)perm[p] : p;
  static_cast<A *>(yv)[row] = sum;
}

template <int COMBO, int C>
__global__ void __launch_bounds__(64 * kWavesPerBlock) k_combine(SpmvArgs a) {
  const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (w >= a.nsplit) return;
  combine_split<COMBO, C>(a.splits[w], a.perm, a.partial, a.y, a.nrows, threadIdx.x & 63);
}

// A group of G = 64 / C consecutive chunks (C in 8..32), each at most
// T = 64 / C columns wide -- one wave step of the one-slot-per-lane kernel --
// as one work unit: one wave covers all their rows, lane l holding row l % C
// of chunk item + l / C and its (at most T) products. The products are
// added as the T lanes of a row add them in spmv_unit with one slot per lane
// (a butterfly over lane offsets 32, 16, ..., C with the missing columns as
// +0), so the result is the same bit for bit; slots holding 0 skip the
// gather.
template <int COMBO, int C, bool RL = false>
__device__ __forceinline__ void spmv_group(const void *__restrict__ valv, const int32_t *__restrict__ col,
                                           const int64_t *__restrict__ cs, const int32_t *__restrict__ clp,
                                           const int32_t *__restrict__ perm, const void *__restrict__ xv,
                                           void *__restrict__ yv, int64_t nrows, int32_t item, int lane,
                                           const int32_t *__restrict__ rlp = nullptr) {
  using V = typename Types<COMBO>::V;
  using X = typename Types<COMBO>::X;
  using A = typename Types<COMBO>::A;
  constexpr int T = 64 / C;
  static_assert(C >= 8 && C <= 32, "two to eight chunks per wave");
  const int32_t c = item + lane / C;
  const int r = lane % C;
  const int64_t p = (int64_t)c * C + r;
  // RL: only the row's own slots are loaded (the rest stay zero, as padding)
  const int w = RL ? rlp[p] : clp[c];
  const int64_t base = cs[c] + r;
  V v[T];
  int32_t ci[T];
#pragma unroll
  for (int j = 0; j < T; ++j) {
    v[j] = 0;
    ci[j] = 0;
    if (j < w) {
      v[j] = __builtin_nontemporal_load(static_cast<const V *>(valv) + base + (int64_t)j * C);
      ci[j] = __builtin_nontemporal_load(col + base + (int64_t)j * C);
    }
  }
  A s[T];
#pragma unroll
  for (int j = 0; j < T; ++j) s[j] = v[j] != 0 ? fmac(cvt(v[j]), static_cast<const X *>(xv)[ci[j]], (A)0) : (A)0;
#pragma unroll
  for (int d = T / 2; d >= 1; d >>= 1)
#pragma unroll
    for (int t = 0; t < d; ++t) s[t] = s[t] + s[t + d];
  if (p < nrows) __builtin_nontemporal_store(s[0], static_cast<A *>(yv) + (perm ? (int64_t)perm[p] : p));
}

template <int COMBO, int C, int U, int VV, int ZS>
__global__ void __launch_bounds__(64 * kWavesPerBlock) k_spmv(SpmvArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (w >= a.nwork) return;
  int32_t item, seg = 0, nseg = 1;
  int64_t poff = 0;
  if (a.units) {
    const Unit u = a.units[w];
    item = u.item;
    seg = u.seg;
    nseg = u.nseg;
    if (nseg > 1) poff = a.splits[u.sid].poff;
    if constexpr (C >= 8 && C <= 32) {
      if (nseg == 0) {  // a group of short chunks
        spmv_group<COMBO, C, ZS == 2>(a.val, a.col, a.cs, a.cl, a.perm, a.x, a.y, a.nrows, item, lane, a.rl);
        return;
      }
    }
  } else {
    item = (int32_t)w;
  }
  spmv_unit<COMBO, C, U, VV, ZS>(a.val, a.col, a.cs, a.cl, a.perm, a.x, a.y, a.nrows, item, seg, nseg, poff,
                                 a.partial, a.seg_cols, lane, a.rl);
}

// Batched form: one launch over the concatenated work units of all
// matrices. Default: one unit per wave (the hardware dispatcher balances the
// uneven matrices). Persistent form (slice != nullptr): a grid of resident
// waves, wave w running units [slice[w], slice[w+1]) back to back.
template <int COMBO, int C, int U>
__global__ void __launch_bounds__(64 * kWavesPerBlock) k_batch(BatchArgs a) {
  const int lane = threadIdx.x & 63;
  // the wave index is uniform over the wave: the unit and matrix
  // descriptors are then read through the scalar cache (94 -> 70 VGPRs at
  // C = 32, eight slots in flight)
  const int64_t w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  int64_t q0, q1;
  if (a.slice) {
    if (w >= a.nwaves) return;
    q0 = a.slice[w];
    q1 = a.slice[w + 1];
  } else {
    if (w >= a.nunits) return;
    q0 = w;
    q1 = w + 1;
  }
  for (int64_t q = q0; q < q1; ++q) {
    const BUnit u = a.units[q];
    if (u.mat < 0) continue;  // grid filler
    const BatchMat m = a.mats[u.mat];
    if constexpr (C >= 8 && C <= 32) {
      if (u.nseg == 0) {  // a group of short chunks
        spmv_group<COMBO, C>(m.val, m.col, m.cs, m.cl, m.perm, m.x, m.y, m.nrows, u.item, lane);
        continue;
      }
    }
    const int64_t poff = u.nseg > 1 ? a.splits[u.sid].poff : 0;
    spmv_unit<COMBO, C, U, 1, true>(m.val, m.col, m.cs, m.cl, m.perm, m.x, m.y, m.nrows, u.item, u.seg, u.nseg,
                                    poff, a.partial, a.seg_cols, lane);
  }
}

template <int COMBO, int C>
__global__ void __launch_bounds__(64 * kWavesPerBlock) k_batch_combine(BatchArgs a) {
  const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (w >= a.nsplit) return;
  const BSplitDesc b = a.splits[w];
  const BatchMat m = a.mats[b.mat];
  combine_split<COMBO, C>(SplitDesc{b.item, b.nseg, b.poff}, m.perm, a.partial, m.y, m.nrows, threadIdx.x & 63);
}

// ---------------------------------------------------------------------------
// Block form Y = A X (FP64), X row-major ncols x k. A wave owns rpw rows of a
// chunk and KT = G*KV right-hand sides (G = 64 / rpw lanes per row, KV
// contiguous right-hand sides per lane; lane = r*G + g). Every matrix entry
// is loaded once per pass and multiplies KT contiguous values of X.
// blockIdx.y selects the pass (right-hand sides [y*KT, (y+1)*KT)).
// ---------------------------------------------------------------------------
template <int KV>
struct DVec {
  typedef double type __attribute__((ext_vector_type(KV)));
};
template <>
struct DVec<1> {
  typedef double type;
};

template <int KV>
__device__ __forceinline__ double vget(const typename DVec<KV>::type &v, int i) {
  return v[i];
}
template <>
__device__ __forceinline__ double vget<1>(const double &v, int) {
  return v;
}

template <int C, int KV>
__global__ void __launch_bounds__(64 * kWavesPerBlock) k_spmmv(SpmvArgs a) {
  constexpr int RPW = C < 64 ? C : 64;
  constexpr int G = 64 / RPW;
  constexpr int WPC = C > 64 ? C / 64 : 1;
  constexpr int KT = G * KV;
  // chunk columns in flight: twelve for one or two right-hand sides per
  // lane, eight for four, four for eight. Measured on the power-law 1M
  // matrix, GF/s at sigma = n / 1024, against 8 / KV (two for KV >= 4):
  // k = 4 337 / 186 -> 375 / 199, k = 8 462 / 256 -> 684 / 292, k = 16
  // (KV = 8, sigma = 1024) 386 -> 406; with the masked last round below,
  // twelve against eight for KV <= 2: k = 2 213 -> 225, k = 4 391 -> 409
  // (210 -> 214); sixteen 234 / 112 and 401 / 207; for KV = 4 (k = 8) four
  // 579, six 639, eight 680.
  constexpr int U = KV >= 8 ? 4 : KV >= 4 ? 8 : 12;
  using VecT = typename DVec<KV>::type;

  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (w >= a.nwork) return;
  int32_t item, seg = 0, nseg = 1;
  int64_t poff = 0;
  if (a.units) {
    const Unit u = a.units[w];
    item = u.item;
    seg = u.seg;
    nseg = u.nseg;
    if (nseg > 1) poff = a.splits[u.sid].poff;
  } else {
    item = (int32_t)w;
  }
  const int k = a.k;
  const int tile = blockIdx.y;
  const int rl = lane / G, g = lane % G;
  const int v0 = tile * KT + g * KV;  // first right-hand side of this lane
  const bool active = v0 < k;          // k % KV == 0: a lane's KV values are all in range or all out

  const int64_t chunk = item / WPC;
  const int h = item - (int)(chunk * WPC);
  const int r = h * RPW + rl;
  const int64_t base = a.cs[chunk];
  const int cl = a.cl[chunk];
  int jb = 0, je = cl;
  if (nseg > 1) {
    jb = seg * a.seg_cols;
    je = jb + a.seg_cols < cl ? jb + a.seg_cols : cl;
  }
  const int32_t *cp = a.col + base + r;
  const double *vp = static_cast<const double *>(a.val) + base + r;
  const double *X = static_cast<const double *>(a.x);

  double acc[KV];
#pragma unroll
  for (int v = 0; v < KV; ++v) acc[v] = 0.0;
  int j = jb;
  for (; j + U <= je; j += U) {
    int32_t ci[U];
    double vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ci[u] = ld_col(cp + (int64_t)(j + u) * C);
      vv[u] = ld_val(vp + (int64_t)(j + u) * C);
    }
    if (active) {
      // padding slots hold value 0: their lanes skip the gather
      VecT xg[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        xg[u] = vv[u] != 0.0 ? *reinterpret_cast<const VecT *>(X + (int64_t)ci[u] * k + v0) : VecT{};
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < KV; ++v) acc[v] = __builtin_fma(vv[u], vget<KV>(xg[u], v), acc[v]);
    }
  }
  // the last je - j < U columns as one more masked round (columns past the
  // end read as padding), all their gathers in flight together
  if (j < je) {
    int32_t ci[U];
    double vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ci[u] = 0;
      vv[u] = 0.0;
      if (j + u < je) {
        ci[u] = ld_col(cp + (int64_t)(j + u) * C);
        vv[u] = ld_val(vp + (int64_t)(j + u) * C);
      }
    }
    if (active) {
      VecT xg[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        xg[u] = vv[u] != 0.0 ? *reinterpret_cast<const VecT *>(X + (int64_t)ci[u] * k + v0) : VecT{};
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < KV; ++v) acc[v] = __builtin_fma(vv[u], vget<KV>(xg[u], v), acc[v]);
    }
  }

  double *Y = static_cast<double *>(a.y);
  const int64_t p = chunk * C + r;
  if (nseg == 1) {
    if (active && p < a.nrows) {
      const int64_t row = a.perm ? (int64_t)a.perm[p] : p;
      // the KV results of a lane are contiguous and aligned (k % KV == 0,
      // Y aligned to KV doubles): one vector store for KV <= 4 (measured
      // faster there, slower for KV = 8 than eight single stores)
      if constexpr (KV > 1 && KV <= 4) {
        VecT o;
        __builtin_memcpy(&o, acc, sizeof(o));
        __builtin_nontemporal_store(o, reinterpret_cast<VecT *>(Y + row * k + v0));
      } else {
#pragma unroll
        for (int v = 0; v < KV; ++v) __builtin_nontemporal_store(acc[v], Y + row * k + v0 + v);
      }
    }
    return;
  }
  // segment of a split row slice: the sums of pass `tile` go to
  // partial[(poff*ntiles + tile*nseg*RPW + seg*RPW + rl)*KT + g*KV + v]
  if (active) {
    double *mine = static_cast<double *>(a.partial) +
                   ((poff * gridDim.y + (int64_t)tile * nseg * RPW + (int64_t)seg * RPW + rl) * KT + g * KV);
#pragma unroll
    for (int v = 0; v < KV; ++v) mine[v] = acc[v];
  }
}

// The KV right-hand sides of a lane of the one-pass block kernel, as 16-byte
// pairs: pair p of lane q of a row holds right-hand sides p*2*LPR + 2q and
// the next, so that one 16-byte access of the LPR lanes of a row covers
// 32*LPR contiguous bytes of it (KV contiguous values per lane would make
// each 16-byte access cover every other 16 bytes of a span twice as long).
// p points at the lane's first pair.
template <int LPR, int KV>
__device__ __forceinline__ typename DVec<KV>::type ld_rhs(const double *p) {
  typedef double P2 __attribute__((ext_vector_type(2)));
  typename DVec<KV>::type r;
#pragma unroll
  for (int q = 0; q < KV / 2; ++q) {
    const P2 t = *reinterpret_cast<const P2 *>(p + q * 2 * LPR);
    r[2 * q] = t[0];
    r[2 * q + 1] = t[1];
  }
  return r;
}

template <int LPR, int KV>
__device__ __forceinline__ void st_rhs(const typename DVec<KV>::type &o, double *p, bool nontemporal) {
  typedef double P2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int q = 0; q < KV / 2; ++q) {
    P2 t;
    t[0] = o[2 * q];
    t[1] = o[2 * q + 1];
    if (nontemporal) __builtin_nontemporal_store(t, reinterpret_cast<P2 *>(p + q * 2 * LPR));
    else *reinterpret_cast<P2 *>(p + q * 2 * LPR) = t;
  }
}

// Block form for k = LPR * KV right-hand sides: LPR lanes share a row (4 or
// 8; 16 measured slower), lane q of a row holding the KV/2 pairs of right-hand sides
// p*2*LPR + 2q, p*2*LPR + 2q + 1 (ld_rhs), so the k values of one row of X
// are read by KV/2 accesses of LPR lanes, each over 32*LPR contiguous bytes,
// and a wave covers 64/LPR rows per access. Work units and the partial-sum layout are
// those of k_spmmv with a single pass of width k; each unit (rpw rows of a
// chunk) is shared by rpw/16 waves of 16 rows each, which walk the unit's
// chunk columns with U columns in flight; each slot is read once. Per row
// the products are added in column order, as in k_spmmv.
template <int C, int LPR, int KV>
__global__ void __launch_bounds__(64 * kWavesPerBlock) k_spmmv_rows(SpmvArgs a) {
  constexpr int RPW = C < 64 ? C : 64;
  constexpr int WPC = C > 64 ? C / 64 : 1;
  constexpr int SUB = RPW / 16;          // waves per unit
  constexpr int RPA = 64 / LPR;          // rows per access
  constexpr int RB = 16 / RPA;           // accesses (rows of a lane group) per wave
  // chunk columns in flight: four with 8 lanes per row and two right-hand
  // sides per lane (k = 16), three with 16 lanes per row (k = 32), two with
  // 16 lanes and four right-hand sides per lane, three with 8 lanes and four
  // or eight. Measured on the power-law 1M matrix at sigma = n: k = 16 two
  // columns 845 GF/s, four 1,055; k = 32 two 996, three 1,099, four 1,008
  // (137 VGPRs, 3 waves per SIMD); k = 64 with 16 lanes per row one 1,015,
  // two 1,142; with 8 lanes per row one 1,167, two 1,299, three 1,288, four
  // 1,228 (sigma = 1024: 607, 585, 677, 574); k = 32 with 8 lanes per row
  // three 1,214 (sigma = 1024: two 488, three 506, four 486); k = 16 with 4
  // lanes per row three 1,061, four 1,124-1,132, six 1,113, eight 1,039;
  // otherwise neutral on the sigma = 1024 layout.
  constexpr int U = KV >= 8 ? 3 : KV >= 4 ? (LPR == 4 ? 4 : LPR == 8 ? 3 : 2) : (LPR == 16 ? 3 : 8 / RB);
  static_assert(RPW % 16 == 0, "blocks of 16 rows");
  using VecT = typename DVec<KV>::type;

  const int lane = threadIdx.x & 63;
  const int64_t wv = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t w = wv / SUB;
  const int rb = (int)(wv - w * SUB) * 16;  // first row of this wave within the unit
  if (w >= a.nwork) return;
  int32_t item, seg = 0, nseg = 1;
  int64_t poff = 0;
  if (a.units) {
    const Unit u = a.units[w];
    item = u.item;
    seg = u.seg;
    nseg = u.nseg;
    if (nseg > 1) poff = a.splits[u.sid].poff;
  } else {
    item = (int32_t)w;
  }
  const int k = a.k;  // LPR * KV
  const int gq = lane / LPR, v0 = 2 * (lane % LPR);  // first right-hand side of this lane
  const int64_t chunk = item / WPC;
  const int h = item - (int)(chunk * WPC);
  const int64_t base = a.cs[chunk];
  const int cl = a.cl[chunk];
  int jb = 0, je = cl;
  if (nseg > 1) {
    jb = seg * a.seg_cols;
    je = jb + a.seg_cols < cl ? jb + a.seg_cols : cl;
  }
  const int32_t *colc = a.col + base + h * RPW + rb + gq;
  const double *valc = static_cast<const double *>(a.val) + base + h * RPW + rb + gq;
  const double *X = static_cast<const double *>(a.x);
  double *Y = static_cast<double *>(a.y);

  double acc[RB][KV];
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int v = 0; v < KV; ++v) acc[m][v] = 0.0;
  int j = jb;
  for (; j + U <= je; j += U) {
    int32_t ci[U][RB];
    double vv[U][RB];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < RB; ++m) {
        const int64_t o = (int64_t)(j + u) * C + RPA * m;
        ci[u][m] = ld_col(colc + o);
        vv[u][m] = ld_val(valc + o);
      }
    // padding slots hold value 0: their rows skip the gather
    VecT xg[U][RB];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < RB; ++m)
        xg[u][m] = vv[u][m] != 0.0 ? ld_rhs<LPR, KV>(X + (int64_t)ci[u][m] * k + v0) : VecT{};
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < RB; ++m)
#pragma unroll
        for (int v = 0; v < KV; ++v) acc[m][v] = __builtin_fma(vv[u][m], vget<KV>(xg[u][m], v), acc[m][v]);
  }
  // the last je - j < U columns: one more round of the same shape, columns
  // past the end read as padding (value 0, no gather), so that all their
  // rows of X are in flight together (per column and per row group, a
  // gather inside a branch with its multiply-add waited for each row in
  // turn: most chunks of a power-law layout sorted by length are one to
  // three columns wide, so most rows took that path)
  if (j < je) {
    int32_t ci[U][RB];
    double vv[U][RB];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < RB; ++m) {
        const int64_t o = (int64_t)(j + u) * C + RPA * m;
        ci[u][m] = 0;
        vv[u][m] = 0.0;
        if (j + u < je) {
          ci[u][m] = ld_col(colc + o);
          vv[u][m] = ld_val(valc + o);
        }
      }
    VecT xg[U][RB];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < RB; ++m)
        xg[u][m] = vv[u][m] != 0.0 ? ld_rhs<LPR, KV>(X + (int64_t)ci[u][m] * k + v0) : VecT{};
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < RB; ++m)
#pragma unroll
        for (int v = 0; v < KV; ++v) acc[m][v] = __builtin_fma(vv[u][m], vget<KV>(xg[u][m], v), acc[m][v]);
  }
#pragma unroll
  for (int m = 0; m < RB; ++m) {
    const int rl = rb + gq + RPA * m;
    VecT o;
    __builtin_memcpy(&o, acc[m], sizeof(o));
    if (nseg == 1) {
      const int64_t p = chunk * C + h * RPW + rl;
      if (p < a.nrows) {
        const int64_t row = a.perm ? (int64_t)a.perm[p] : p;
        st_rhs<LPR, KV>(o, Y + row * k + v0, true);
      }
    } else {
      // partial[(poff + seg*RPW + rl)*k + v]: the layout of k_spmmv with one
      // pass of width k
      double *mine = static_cast<double *>(a.partial) + ((poff + (int64_t)seg * RPW + rl) * k + v0);
      st_rhs<LPR, KV>(o, mine, false);
    }
  }
}

// Block form: add the segment sums of split row slices. Block (w, tile, z):
// split slice w, pass tile, z-th part of the slice's (row, right-hand side)
// elements; one thread per element where the grid covers them all, the
// segment sums added in segment order with sixteen loads in flight (the
// longest slices have tens of segments, and each round trip to them is a
// separate latency: the combining is latency-bound).
template <int C>
__global__ void __launch_bounds__(512) k_combine_mm(SpmvArgs a) {
  constexpr int RPW = C < 64 ? C : 64;
  constexpr int WPC = C > 64 ? C / 64 : 1;
  const SplitDesc d = a.splits[blockIdx.x];
  const int tile = blockIdx.y, ntiles = gridDim.y, KT = a.kt, k = a.k;
  const int64_t chunk = d.item / WPC;
  const int h = d.item - (int)(chunk * WPC);
  const double *base = static_cast<const double *>(a.partial) + (d.poff * ntiles + (int64_t)tile * d.nseg * RPW) * KT;
  double *Y = static_cast<double *>(a.y);
  // blockIdx.z: which part of the slice's elements this block adds
  for (int e = blockIdx.z * blockDim.x + threadIdx.x; e < RPW * KT; e += gridDim.z * blockDim.x) {
    const int rl = e / KT, vl = e - rl * KT;
    const int v = tile * KT + vl;
    const int64_t p = chunk * C + h * RPW + rl;
    if (v >= k || p >= a.nrows) continue;
    const double *src = base + (int64_t)rl * KT + vl;
    const int64_t step = (int64_t)RPW * KT;  // between the sums of two segments
    double sum = 0.0;
    for (int q = 0; q < d.nseg; q += 16) {  // +0 past the last segment, as in combine_split
      double t[16];
#pragma unroll
      for (int e8 = 0; e8 < 16; ++e8) t[e8] = q + e8 < d.nseg ? src[(int64_t)(q + e8) * step] : 0.0;
#pragma unroll
      for (int e8 = 0; e8 < 16; ++e8) sum += t[e8];
    }
    const int64_t row = a.perm ? (int64_t)a.perm[p] : p;
    Y[row * k + v] = sum;
  }
}

}  // namespace dev
}  // namespace sell

namespace sell {
namespace dev {

// Host-side launchers for one dtype combination; every supported
// (C, U, VV) is instantiated. U*VV (slots in flight per lane) is 4 or 8.
#define SELL_FOR_EACH_CUV(X)                                                                                         \
  X(1, 4, 1) X(1, 8, 1) X(2, 4, 1) X(2, 8, 1) X(4, 4, 1) X(4, 8, 1) X(8, 4, 1) X(8, 8, 1) X(16, 4, 1) X(16, 8, 1) \
      X(32, 4, 1) X(32, 8, 1) X(64, 4, 1) X(64, 8, 1) X(128, 4, 1) X(128, 8, 1) X(2, 2, 2) X(2, 4, 2) X(4, 2, 2)   \
          X(4, 4, 2) X(8, 2, 2) X(8, 4, 2) X(16, 2, 2) X(16, 4, 2) X(32, 2, 2) X(32, 4, 2) X(64, 2, 2) X(64, 4, 2) \
              X(4, 1, 4) X(4, 2, 4) X(8, 1, 4) X(8, 2, 4) X(16, 1, 4) X(16, 2, 4) X(32, 1, 4) X(32, 2, 4)          \
                  X(64, 1, 4) X(64, 2, 4)

#define SELL_FOR_EACH_CU(X) \
  X(1, 4) X(1, 8) X(2, 4) X(2, 8) X(4, 4) X(4, 8) X(8, 4) X(8, 8) X(16, 4) X(16, 8) X(32, 4) X(32, 8) X(64, 4) \
      X(64, 8) X(128, 4) X(128, 8)

// ZS: 0 plain, 1 zero slots skip their gather, 2 also the row lengths
// (SpmvArgs::rl); mode 2 exists for C in 8..64 and the default pairs of
// steps in flight and slots per lane only.
#define SELL_FOR_EACH_CUV_RL(X)                                                                               \
  X(8, 4, 1) X(8, 8, 1) X(16, 4, 1) X(16, 8, 1) X(32, 4, 1) X(32, 8, 1) X(64, 4, 1) X(64, 8, 1) X(8, 2, 2)   \
      X(8, 4, 2) X(16, 2, 2) X(16, 4, 2) X(32, 2, 2) X(32, 4, 2) X(64, 2, 2) X(64, 4, 2) X(8, 1, 4)           \
          X(8, 2, 4) X(16, 1, 4) X(16, 2, 4) X(32, 1, 4) X(32, 2, 4) X(64, 1, 4) X(64, 2, 4)

template <int COMBO, int ZS>
hipError_t launch_spmv_zs(int C, int U, int VV, const SpmvArgs &a, hipStream_t s) {
  if (a.nwork <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((a.nwork + kWavesPerBlock - 1) / kWavesPerBlock);
#define SELL_L(CC, UU, VVV)                                                                                  \
  if (C == CC && U == UU && VV == VVV) {                                                                    \
    hipLaunchKernelGGL((k_spmv<COMBO, CC, UU, VVV, ZS>), dim3(nb), dim3(64 * kWavesPerBlock), 0, s, a);     \
    hipError_t e_ = hipGetLastError();                                                                       \
    if (e_ != hipSuccess || a.nsplit == 0) return e_;                                                        \
    const unsigned nbc = (unsigned)((a.nsplit + kWavesPerBlock - 1) / kWavesPerBlock);                        \
    hipLaunchKernelGGL((k_combine<COMBO, CC>), dim3(nbc), dim3(64 * kWavesPerBlock), 0, s, a);               \
    return hipGetLastError();                                                                                \
  }
  if constexpr (ZS == 2) {
    SELL_FOR_EACH_CUV_RL(SELL_L)
  } else {
    SELL_FOR_EACH_CUV(SELL_L)
  }
#undef SELL_L
  return hipErrorInvalidValue;
}

template <int COMBO>
hipError_t launch_spmv_t(int C, int U, int VV, bool skip_zero, const SpmvArgs &a, hipStream_t s) {
  if (a.rl) return launch_spmv_zs<COMBO, 2>(C, U, VV, a, s);
  return skip_zero ? launch_spmv_zs<COMBO, 1>(C, U, VV, a, s) : launch_spmv_zs<COMBO, 0>(C, U, VV, a, s);
}

// C in {8, 16, 32, 64}; V slots per lane (1, 2, or 4 for FP32/BF16 values,
// C >= 16), U wave steps in flight (U * V = 4, 8 or 16); w.gc chunks per
// workgroup: kXwChunks or kXwChunksWide.
template <int COMBO, int GC>
hipError_t launch_spmv_xw_g(int C, int VV, int U, const SpmvArgs &a, const XwArgs &w, size_t lds, hipStream_t s) {
  const unsigned nb = (unsigned)((a.nwork + GC - 1) / GC);
#define SELL_L(CC, VVV, UU)                                                                                    \
  if (C == CC && VV == VVV && U == UU) {                                                                       \
    hipLaunchKernelGGL((k_spmv_xw<COMBO, CC, VVV, UU, GC>), dim3(nb), dim3(64 * GC), lds, s, a, w);           \
    return hipGetLastError();                                                                                  \
  }
  SELL_L(8, 1, 4) SELL_L(16, 1, 4) SELL_L(32, 1, 4) SELL_L(64, 1, 4)
  SELL_L(8, 1, 8) SELL_L(16, 1, 8) SELL_L(32, 1, 8) SELL_L(64, 1, 8)
  SELL_L(8, 2, 2) SELL_L(16, 2, 2) SELL_L(32, 2, 2) SELL_L(64, 2, 2)
  SELL_L(8, 2, 4) SELL_L(16, 2, 4) SELL_L(32, 2, 4) SELL_L(64, 2, 4)
  SELL_L(8, 2, 8) SELL_L(16, 2, 8) SELL_L(32, 2, 8) SELL_L(64, 2, 8)
  // four slots per lane: FP32/BF16 values (16 or 8 bytes per load)
  if constexpr (sizeof(typename Types<COMBO>::V) <= 4) {
    SELL_L(16, 4, 1) SELL_L(32, 4, 1) SELL_L(64, 4, 1)
    SELL_L(16, 4, 2) SELL_L(32, 4, 2) SELL_L(64, 4, 2)
    SELL_L(16, 4, 4) SELL_L(32, 4, 4) SELL_L(64, 4, 4)
  }
#undef SELL_L
  return hipErrorInvalidValue;
}

template <int COMBO>
hipError_t launch_spmv_xw_t(int C, int VV, int U, const SpmvArgs &a, const XwArgs &w, size_t lds, hipStream_t s) {
  if (a.nwork <= 0) return hipSuccess;
  if (w.gc == kXwChunks) return launch_spmv_xw_g<COMBO, kXwChunks>(C, VV, U, a, w, lds, s);
  if (w.gc == kXwChunksWide) return launch_spmv_xw_g<COMBO, kXwChunksWide>(C, VV, U, a, w, lds, s);
  return hipErrorInvalidValue;
}

template <int COMBO>
hipError_t launch_batch_t(int C, int U, const BatchArgs &a, hipStream_t s) {
  if (a.nunits <= 0) return hipSuccess;
  const int64_t waves = a.slice ? a.nwaves : a.nunits;
  const int wpb = a.slice ? kBatchPersistentWaves : kWavesPerBlock;
  const unsigned nb = (unsigned)((waves + wpb - 1) / wpb);
#define SELL_L(CC, UU)                                                                                     \
  if (C == CC && U == UU) {                                                                               \
    hipLaunchKernelGGL((k_batch<COMBO, CC, UU>), dim3(nb), dim3(64 * wpb), 0, s, a);           \
    hipError_t e_ = hipGetLastError();                                                                    \
    if (e_ != hipSuccess || a.nsplit == 0) return e_;                                                     \
    const unsigned nbc = (unsigned)((a.nsplit + kWavesPerBlock - 1) / kWavesPerBlock);                     \
    hipLaunchKernelGGL((k_batch_combine<COMBO, CC>), dim3(nbc), dim3(64 * kWavesPerBlock), 0, s, a);      \
    return hipGetLastError();                                                                             \
  }
  SELL_FOR_EACH_CU(SELL_L)
#undef SELL_L
  return hipErrorInvalidValue;
}

template <int COMBO>
int batch_waves_per_cu_t(int C, int U) {
  int blocks = 0;
#define SELL_L(CC, UU)                                                                                              \
  if (C == CC && U == UU) {                                                                                        \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<COMBO, CC, UU>, 64 * kBatchPersistentWaves,  \
                                                     0) != hipSuccess)                                             \
      blocks = 1;                                                                                                  \
    return blocks * kBatchPersistentWaves;                                                                                \
  }
  SELL_FOR_EACH_CU(SELL_L)
#undef SELL_L
  return kWavesPerBlock;
}

}  // namespace dev
}  // namespace sell
