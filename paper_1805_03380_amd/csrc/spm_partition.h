// Grouping elements by segment (the column of a triplet for assembly, the row of a stored
// element for the plan) without device-wide atomics.  Device-scope atomics on gfx950 are
// performed beyond the XCD-local L2 (and contended ones serialize there), so the grouping is
// a two-level partition whose counters all live in LDS, and no workgroup ever waits for
// another:
//   level 1  the segments are cut into CB coarse buckets of W = 2^b consecutive segments.
//            k_part_hist: each tile of T1 elements counts its elements per coarse bucket in
//            LDS and writes one column of a (bucket x tile) table;  k_rows_scan scans every
//            bucket's row of the table, and each scatter workgroup scans the bucket totals,
//            which gives every (bucket, tile) pair its output range;
//            k_part_scatter: each tile ranks its elements per bucket with LDS atomics and
//            writes (key, segment-within-bucket) into the bucket's range.
//   level 2  k_part_level2: one workgroup per coarse bucket counts its elements per segment
//            in LDS, scatters them into segment order and sorts every segment by key; the plan
//            writes its row index from there, the assembly folds the runs and compacts them
//            per bucket, and k_part_emit places the buckets' survivors.
// Keys carry a unique element index, so the grouping order inside a bucket never matters.
#pragma once

#include "spm_assemble.h"

namespace spm {

constexpr int kPartMaxBuckets = 16384;  // coarse buckets per level (LDS counters, <= 64 KB)

// Workgroups go to the chip's 8 XCDs in turn (workgroup i to XCD i mod 8), each XCD with an
// L2 of its own.  xcd_tile hands the workgroups of one XCD consecutive logical tiles, so that
// neighbouring columns of a (bucket x tile) table, written or read by neighbouring tiles,
// meet in one L2 instead of eight.  A bijection of [0, n); results never depend on it.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n) {
  const int64_t q = n / kXcds, r = n % kXcds;
  const int64_t x = b % kXcds;
  return x * q + (x < r ? x : r) + b / kXcds;
}
constexpr int kPartMaxWidth = 4096;     // segments per coarse bucket (LDS counters)

// Element sources.  elem() reports kElemOk (seg and key set), kElemBad (an index out of
// range: skipped and reported in the status) or kElemSkip (an unused position: skipped
// silently); a bool source's true / false read as ok / bad.
constexpr int kElemBad = 0;
constexpr int kElemOk = 1;
constexpr int kElemSkip = 2;

struct PartSrcCoo {  // assembly: segment = column, key = row << 32 | input position
  const int32_t* row;
  const int32_t* col;
  int32_t n_rows, n_cols;
  int64_t n;
  __device__ __forceinline__ int64_t count() const { return n; }
  __device__ __forceinline__ bool elem(int64_t e, uint32_t& seg, uint64_t& key) const {
    const int32_t r = row[e], c = col[e];
    if ((uint32_t)r < (uint32_t)n_rows && (uint32_t)c < (uint32_t)n_cols) {
      seg = (uint32_t)c;
      key = ((uint64_t)(uint32_t)r << 32) | (uint32_t)e;
      return true;
    }
    return false;
  }
};

struct PartSrcCsc {  // plan: segment = row, key = column << 32 | CSC slot
  const int32_t* row_idx;
  const int32_t* colarr;   // column of every slot (k_expand_columns)
  const int32_t* col_ptr;  // col_ptr[n_cols] = number of stored elements
  int64_t n_rows, n_cols, cap;
  __device__ __forceinline__ int64_t count() const {
    const int64_t raw = col_ptr[n_cols];
    return raw < 0 ? 0 : (raw > cap ? cap : raw);
  }
  __device__ __forceinline__ bool elem(int64_t p, uint32_t& seg, uint64_t& key) const {
    const int32_t r = row_idx[p];
    if (r >= 0 && (int64_t)r < n_rows) {
      seg = (uint32_t)r;
      key = ((uint64_t)(uint32_t)colarr[p] << 32) | (uint32_t)p;
      return true;
    }
    return false;
  }
};

// Status without a cleared word: every workgroup of a checking kernel writes its own flag
// word (kFlagShape | kFlagIndex bits, 0 if clean) and k_rows_scan folds them into info[1],
// an invalid shape taking precedence over an out-of-range index.
constexpr uint32_t kFlagShape = 1u;
constexpr uint32_t kFlagIndex = 2u;

// Column of every stored slot of a CSC, plus the offset checks the plan needs (monotone,
// col_ptr[0] = 0, nnz <= capacity; row indices are checked by k_part_hist, which reads them
// anyway); flags[blockIdx.x] receives the workgroup's findings.  A workgroup takes chunks of
// NT columns (grid-stride) and stages their offsets in LDS.  A column of at most kShort slots
// is written by its own thread; longer ones are queued and each is then written by the whole
// workgroup, so long columns do not serialise one thread.  Offsets are clamped to [0, nnz]:
// a malformed col_ptr can only produce wrong columns (and a status), never an access out of
// range.
template <int NT>
__global__ __launch_bounds__(NT) void k_expand_columns(const int32_t* __restrict__ col_ptr,
                                                       int64_t n_cols, int64_t nnz_cap,
                                                       int32_t* __restrict__ colarr,
                                                       int32_t* __restrict__ info,
                                                       uint32_t* __restrict__ flags) {
  constexpr int64_t kShort = 32;
  __shared__ uint32_t s_flag;
  __shared__ int64_t s_cp[NT + 1];
  __shared__ int32_t s_long[NT];
  __shared__ int32_t s_nlong;
  if (threadIdx.x == 0) s_flag = 0;
  const int64_t raw = col_ptr[n_cols];
  const int64_t nnz = raw < 0 ? 0 : (raw > nnz_cap ? nnz_cap : raw);
  bool bad_shape = false;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (col_ptr[0] != 0 || raw < 0 || raw > nnz_cap) bad_shape = true;
    info[0] = (int32_t)nnz;
  }
  for (int64_t c0 = (int64_t)blockIdx.x * NT; c0 < n_cols; c0 += (int64_t)gridDim.x * NT) {
    const int nc = (int)((n_cols - c0) < NT ? (n_cols - c0) : NT);
    __syncthreads();  // the previous chunk is done with s_cp and s_long
    if (threadIdx.x == 0) s_nlong = 0;
    for (int j = threadIdx.x; j <= nc; j += NT) {
      const int64_t v = col_ptr[c0 + j];
      s_cp[j] = v < 0 ? 0 : (v > nnz ? nnz : v);
      if (j < nc && v > (int64_t)col_ptr[c0 + j + 1]) bad_shape = true;
    }
    __syncthreads();
    if (threadIdx.x < nc) {
      const int j = threadIdx.x;
      const int64_t p0 = s_cp[j], p1 = s_cp[j + 1];
      if (p1 - p0 <= kShort) {
        for (int64_t p = p0; p < p1; ++p) colarr[p] = (int32_t)(c0 + j);
      } else {
        s_long[atomicAdd(&s_nlong, 1)] = j;
      }
    }
    __syncthreads();
    for (int q = 0; q < s_nlong; ++q) {
      const int j = s_long[q];
      const int64_t p1 = s_cp[j + 1];
      for (int64_t p = s_cp[j] + threadIdx.x; p < p1; p += NT) colarr[p] = (int32_t)(c0 + j);
    }
  }
  if (bad_shape) atomicOr(&s_flag, kFlagShape);
  __syncthreads();
  if (threadIdx.x == 0) flags[blockIdx.x] = s_flag;
}

// Level 1a: per-tile coarse-bucket counts -> table[cb * ntiles + t].
// zero0 / zero1 (nullable): the counts of the big-bucket lists that k_rows_scan fills next;
// workgroup 0 clears them.
// Two-pass level 1 (below): the tile's counts per super-bucket (buckets >> sg) for each of its
// SH equal sub-tiles, subcnt[(t * SH + h) * SB + s]; SH == 0 for none.
struct SubCounts {
  uint32_t* subcnt;
  int sg;     // log2(buckets per super-bucket)
  int SH;     // sub-tiles per tile (a power of two), 0: not counted
  int32_t SB;
};
constexpr int kSubMax = 8;  // sub-tiles per tile at most

template <int NT, typename SRC>
__global__ __launch_bounds__(NT) void k_part_hist(SRC src, int b, int32_t CB, int64_t ntiles,
                                                  int64_t T1, uint32_t* __restrict__ table,
                                                  uint32_t* __restrict__ flags,
                                                  uint32_t* __restrict__ zero0,
                                                  uint32_t* __restrict__ zero1, SubCounts sc) {
  __shared__ uint32_t s_flag;
  __shared__ uint32_t s_sub[kSubMax * 128];
  extern __shared__ uint32_t h[];  // CB counters (dynamic LDS, 4*CB bytes)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (zero0) *zero0 = 0;
    if (zero1) *zero1 = 0;
  }
  const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t n = src.count();
  for (int i = threadIdx.x; i < CB; i += NT) h[i] = 0;
  const int nsub = sc.SH * sc.SB;
  for (int i = threadIdx.x; i < nsub; i += NT) s_sub[i] = 0;
  const int sub_shift = sc.SH > 0 ? 63 - __clzll((unsigned long long)(T1 / sc.SH)) : 0;
  if (threadIdx.x == 0) s_flag = 0;
  __syncthreads();
  bool bad = false;
  const int64_t base = t * T1;
  const int64_t end = (base + T1 < n) ? base + T1 : n;
  constexpr int U = 4;  // elements in flight per thread
  for (int64_t e0 = base + threadIdx.x; e0 < end; e0 += (int64_t)NT * U) {
    uint32_t seg[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + (int64_t)u * NT;
      uint64_t key;
      ok[u] = false;
      if (e < end) {
        const int st = (int)src.elem(e, seg[u], key);
        ok[u] = st == kElemOk;
        bad |= st == kElemBad;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ok[u]) {
        atomicAdd(&h[seg[u] >> b], 1u);
        if (nsub) {
          const int64_t e = e0 + (int64_t)u * NT;
          const int hh = (int)((e - base) >> sub_shift);
          atomicAdd(&s_sub[hh * sc.SB + (seg[u] >> (b + sc.sg))], 1u);
        }
      }
    }
  }
  if (bad) s_flag = kFlagIndex;
  __syncthreads();
  for (int i = threadIdx.x; i < CB; i += NT) table[(int64_t)i * ntiles + t] = h[i];
  for (int i = threadIdx.x; i < nsub; i += NT) sc.subcnt[t * nsub + i] = s_sub[i];
  if (flags && threadIdx.x == 0) flags[t] = s_flag;
}

// One element in a coarse bucket is one 16-byte record, so the scatter issues a single
// store per element (the scatter is bound by the number of scattered stores, not bytes):
// x, y = low and high word of the key, z = segment within the bucket, w = the value's low
// word (all of a float32 or bfloat16 value; a float64 value's high word goes to bvhi).
template <typename VT> struct ValWords;
template <> struct ValWords<float> {
  static constexpr bool kHi = false;
  __device__ __forceinline__ static uint32_t lo(float v) { return __float_as_uint(v); }
  __device__ __forceinline__ static uint32_t hi(float) { return 0u; }
  __device__ __forceinline__ static float make(uint32_t l, uint32_t) { return __uint_as_float(l); }
};
template <> struct ValWords<double> {
  static constexpr bool kHi = true;
  __device__ __forceinline__ static uint32_t lo(double v) { return (uint32_t)__double2loint(v); }
  __device__ __forceinline__ static uint32_t hi(double v) { return (uint32_t)__double2hiint(v); }
  __device__ __forceinline__ static double make(uint32_t l, uint32_t h) {
    return __hiloint2double((int)h, (int)l);
  }
};
template <> struct ValWords<bf16_t> {
  static constexpr bool kHi = false;
  __device__ __forceinline__ static uint32_t lo(bf16_t v) { return (uint32_t)v; }
  __device__ __forceinline__ static uint32_t hi(bf16_t) { return 0u; }
  __device__ __forceinline__ static bf16_t make(uint32_t l, uint32_t) { return (bf16_t)l; }
};
__device__ __forceinline__ uint64_t rec_key(const uint4& r) {
  return ((uint64_t)r.y << 32) | r.x;
}

// Cursors of one tile: cur[i] = bstart[i] + rowoff[i * ld + col] for the n buckets, where
// bstart is the exclusive scan of the bucket totals btot (scanned in LDS by every workgroup;
// the one with `writer` also stores bstart[0..n], bstart[n] = total).  The first RB * NT
// totals and table entries are loaded into registers before the scan starts.
template <int NT>
__device__ __forceinline__ void bucket_cursors(uint32_t* cur, int64_t n,
                                               const uint32_t* __restrict__ btot,
                                               const uint32_t* __restrict__ rowoff, int64_t ld,
                                               int64_t col, bool writer,
                                               int32_t* __restrict__ bstart, uint32_t* s_w) {
  constexpr int RB = NT >= 1024 ? 2 : 4;
  uint32_t bt[RB], ro[RB];
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const int64_t i = threadIdx.x + (int64_t)k * NT;
    bt[k] = 0;
    ro[k] = 0;
    if (i < n) {
      bt[k] = btot[i];
      ro[k] = rowoff[i * ld + col];
    }
  }
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const int64_t i = threadIdx.x + (int64_t)k * NT;
    if (i < n) cur[i] = bt[k];
  }
  for (int64_t i = threadIdx.x + (int64_t)RB * NT; i < n; i += NT) cur[i] = btot[i];
  __syncthreads();
  wg_inclusive_scan_inplace<NT>(cur, n, s_w);
  __syncthreads();
  const uint32_t total = n > 0 ? cur[n - 1] : 0u;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const int64_t i = threadIdx.x + (int64_t)k * NT;
    if (i < n) {
      const uint32_t ex = cur[i] - bt[k];
      if (writer) bstart[i] = (int32_t)ex;
      cur[i] = ex + ro[k];
    }
  }
  for (int64_t i = threadIdx.x + (int64_t)RB * NT; i < n; i += NT) {
    const uint32_t ex = cur[i] - btot[i];
    if (writer) bstart[i] = (int32_t)ex;
    cur[i] = ex + rowoff[i * ld + col];
  }
  if (writer && threadIdx.x == 0) bstart[n] = (int32_t)total;
  __syncthreads();
}

// Level 1b: scatter the elements' records into the buckets.  The range of (bucket cb,
// tile t) starts at bstart[cb] + rowoff[cb * ntiles + t], where bstart is the exclusive scan
// of the bucket totals: every workgroup scans btot (a few KB) itself, and workgroup 0 also
// stores the scan (bstart[0..CB], bstart[CB] = total) for the kernels that follow.
// With vin != nullptr each element's value travels in its record: read here in input order,
// coalesced, instead of gathered one cache line per element later.
template <int NT, typename SRC, typename VT>
__global__ __launch_bounds__(NT) void k_part_scatter(SRC src, int b, int32_t CB, int64_t ntiles,
                                                     int64_t T1,
                                                     const uint32_t* __restrict__ rowoff,
                                                     const uint32_t* __restrict__ btot,
                                                     int32_t* __restrict__ bstart,
                                                     uint4* __restrict__ brec,
                                                     const VT* __restrict__ vin,
                                                     uint32_t* __restrict__ bvhi) {
  extern __shared__ uint32_t cur[];  // CB cursors (dynamic LDS, 4*CB bytes)
  __shared__ uint32_t s_w[NT / kWave + 1];
  const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t n = src.count();
  const uint32_t wmask = (1u << b) - 1u;
  const int64_t base = t * T1;
  const int64_t end = (base + T1 < n) ? base + T1 : n;
  constexpr int U = 4;
  const bool carry = vin != nullptr;
  // cur[i] = bstart[i] + rowoff[i][t]: the bucket totals are scanned in LDS
  for (int64_t i = threadIdx.x; i < CB; i += NT) cur[i] = btot[i];
  __syncthreads();
  wg_inclusive_scan_inplace<NT>(cur, CB, s_w);
  __syncthreads();
  const uint32_t total = CB > 0 ? cur[CB - 1] : 0u;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < CB; i += NT) {
    const uint32_t ex = cur[i] - btot[i];
    if (t == 0) bstart[i] = (int32_t)ex;
    cur[i] = ex + rowoff[i * ntiles + t];
  }
  if (t == 0 && threadIdx.x == 0) bstart[CB] = (int32_t)total;
  __syncthreads();
  for (int64_t e0 = base + threadIdx.x; e0 < end; e0 += (int64_t)NT * U) {
    uint32_t seg[U];
    uint64_t key[U];
    VT v[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + (int64_t)u * NT;
      ok[u] = (e < end) && (int)src.elem(e, seg[u], key[u]) == kElemOk;
      if (carry && e < end) v[u] = vin[e];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ok[u]) {
        const uint32_t pos = atomicAdd(&cur[seg[u] >> b], 1u);
        const uint32_t vlo = carry ? ValWords<VT>::lo(v[u]) : 0u;
        brec[pos] = make_uint4((uint32_t)key[u], (uint32_t)(key[u] >> 32), seg[u] & wmask, vlo);
        if (ValWords<VT>::kHi && carry) bvhi[pos] = ValWords<VT>::hi(v[u]);
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Level 1 in two passes, for many buckets.  With CB in the thousands a tile holds only a few
// elements of each bucket, so the single scatter above writes every record to a line of its
// own.  Instead the buckets are taken in super-buckets of 2^g consecutive buckets:
//   k_super_offsets  bstart of every bucket, and for every super-bucket s and tile t the
//                    offset sbro[s][t] = bstart[s 2^g] + sum of rowoff over s's buckets (the
//                    start of tile t's elements of s in super-bucket order; sbro[s][ntiles]
//                    is the end of s);
//   k_part_scatter_a each tile sorts chunks of its elements by super-bucket in LDS and
//                    writes them out as runs at sbro[s][t] onwards (irec);
//   k_part_scatter_b each (super-bucket, group of K tiles) reads its slice of irec, sorts
//                    chunks by bucket in LDS and writes runs at bstart[cb] + rowoff[cb][first
//                    tile of the group] onwards (brec, the same layout as the single scatter).
// Every bucket receives exactly its elements; their order inside a bucket differs from the
// single scatter's, which level 2 does not see (it sorts by the unique key).
// ------------------------------------------------------------------------------------------
constexpr int kSuperMax = 128;       // super-buckets (and buckets per super-bucket) at most
constexpr uint32_t kNoGroup = 0xffffffffu;

// One chunk of NT*U elements (element u of thread i; grp == kNoGroup for none) goes out in
// runs: a counting sort by group in LDS (stage, stage_g, and stage_hi for HI), then every
// staged record is written to cur[its group] + its position among the group's records, so
// neighbouring lanes write neighbouring addresses; cur advances by the group counts.
template <int NT, int U, bool HI>
__device__ __forceinline__ void staged_runs(const uint32_t (&grp)[U], const uint4 (&rec)[U],
                                            const uint32_t (&hi)[U], int ng, uint32_t* cnt,
                                            uint32_t* cur, uint4* stage, uint32_t* stage_hi,
                                            uint8_t* stage_g, uint4* __restrict__ out,
                                            uint32_t* __restrict__ out_hi) {
  static_assert(kSuperMax <= 2 * kWave, "one wave scans the group counts");
  for (int i = threadIdx.x; i <= ng; i += NT) cnt[i] = 0;
  __syncthreads();
  uint32_t rank[U];
#pragma unroll
  for (int u = 0; u < U; ++u) rank[u] = grp[u] != kNoGroup ? atomicAdd(&cnt[grp[u]], 1u) : 0u;
  __syncthreads();
  if (threadIdx.x < kWave) {  // cnt[g] = end of group g in the chunk (ng <= 2 * kWave)
    const int l = threadIdx.x;
    const uint32_t a = 2 * l < ng ? cnt[2 * l] : 0u;
    const uint32_t c = 2 * l + 1 < ng ? cnt[2 * l + 1] : 0u;
    const uint32_t incl = wave_incl_scan(a + c);
    if (2 * l < ng) cnt[2 * l] = incl - c;
    if (2 * l + 1 < ng) cnt[2 * l + 1] = incl;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (grp[u] != kNoGroup) {
      const uint32_t slot = (grp[u] ? cnt[grp[u] - 1] : 0u) + rank[u];
      stage[slot] = rec[u];
      stage_g[slot] = (uint8_t)grp[u];
      if (HI) stage_hi[slot] = hi[u];
    }
  }
  __syncthreads();
  const uint32_t m = ng > 0 ? cnt[ng - 1] : 0u;
  for (uint32_t i = threadIdx.x; i < m; i += NT) {
    const uint32_t gi = stage_g[i];
    const uint32_t dst = cur[gi] + (i - (gi ? cnt[gi - 1] : 0u));
    out[dst] = stage[i];
    if (HI) out_hi[dst] = stage_hi[i];
  }
  __syncthreads();
  for (int gi = threadIdx.x; gi < ng; gi += NT) cur[gi] += cnt[gi] - (gi ? cnt[gi - 1] : 0u);
  __syncthreads();
}

__host__ __device__ inline size_t staged_lds_bytes(int nt, int u, bool hi) {
  const size_t c = (size_t)nt * u;
  return c * 16 + (hi ? c * 4 : 0) + c;
}

// bstart of every bucket and the super-bucket offsets sbro[s][t] (t = 0 .. ntiles).  Workgroup
// (s, c) takes super-bucket s of G = 2^g buckets and tiles [64 c, 64 c + 64): each of its four
// waves sums a quarter of the buckets' rowoff entries for its lane's tile (independent loads,
// eight in flight), LDS adds the quarters.
template <int NT>
__global__ __launch_bounds__(NT) void k_super_offsets(const uint32_t* __restrict__ btot,
                                                      const uint32_t* __restrict__ rowoff,
                                                      int32_t CB, int g, int64_t ntiles,
                                                      int64_t nchunk,
                                                      int32_t* __restrict__ bstart,
                                                      uint32_t* __restrict__ sbro) {
  static_assert(NT == 4 * kWave && NT >= kSuperMax, "four waves; one thread per bucket");
  __shared__ uint32_t s_w[NT / kWave + 1];
  __shared__ uint32_t s_part[4][kWave];
  const int64_t s = blockIdx.x / nchunk, c = blockIdx.x % nchunk;
  const int64_t cb0 = s << g;
  const int64_t ng = min((int64_t)1 << g, (int64_t)CB - cb0);
  // the totals of the buckets before this super-bucket, eight loads in flight per thread
  uint32_t part = 0;
  {
    constexpr int U = 8;
    int64_t i = threadIdx.x;
    for (; i + (int64_t)(U - 1) * NT < cb0; i += (int64_t)NT * U) {
      uint32_t r[U];
#pragma unroll
      for (int k = 0; k < U; ++k) r[k] = btot[i + (int64_t)k * NT];
#pragma unroll
      for (int k = 0; k < U; ++k) part += r[k];
    }
    for (; i < cb0; i += NT) part += btot[i];
  }
  uint32_t base;
  (void)wg_excl_scan<NT>(part, s_w, &base);
  const uint32_t v = threadIdx.x < ng ? btot[cb0 + threadIdx.x] : 0u;
  uint32_t tot;
  const uint32_t ex = wg_excl_scan<NT>(v, s_w, &tot);
  if (c == 0) {
    if (threadIdx.x < ng) bstart[cb0 + threadIdx.x] = (int32_t)(base + ex);
    if (cb0 + ng == CB && threadIdx.x == 0) bstart[CB] = (int32_t)(base + tot);
  }
  const int64_t t = c * kWave + lane_id();
  const int q = wave_id();
  const int64_t j0 = (ng * q) / 4, j1 = (ng * (q + 1)) / 4;
  uint32_t sum = 0;
  if (t < ntiles) {
    int64_t j = j0;
    for (; j + 8 <= j1; j += 8) {
      uint32_t r[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) r[k] = rowoff[(cb0 + j + k) * ntiles + t];
#pragma unroll
      for (int k = 0; k < 8; ++k) sum += r[k];
    }
    for (; j < j1; ++j) sum += rowoff[(cb0 + j) * ntiles + t];
  }
  s_part[q][lane_id()] = sum;
  __syncthreads();
  if (q == 0 && t <= ntiles) {
    const uint32_t all = s_part[0][lane_id()] + s_part[1][lane_id()] + s_part[2][lane_id()] +
                         s_part[3][lane_id()];
    sbro[s * (ntiles + 1) + t] = base + (t < ntiles ? all : tot);
  }
}

// Pass A: tile t's elements into super-bucket order (record z = segment within the
// super-bucket: bucket within it above bit b, segment within the bucket below).
// Workgroup (t, h) takes sub-tile h of tile t (SH sub-tiles per tile); its cursor for
// super-bucket s starts after the s-elements of the sub-tiles before it (subcnt).
template <int NT, typename SRC, typename VT>
__global__ __launch_bounds__(NT) void k_part_scatter_a(SRC src, int b, int g, int32_t SB,
                                                       int64_t ntiles, int64_t T1, int SH,
                                                       const uint32_t* __restrict__ sbro,
                                                       const uint32_t* __restrict__ subcnt,
                                                       uint4* __restrict__ irec,
                                                       const VT* __restrict__ vin,
                                                       uint32_t* __restrict__ ivhi) {
  constexpr int U = 4;
  constexpr bool HI = ValWords<VT>::kHi;
  extern __shared__ __align__(16) unsigned char smem[];
  uint4* stage = reinterpret_cast<uint4*>(smem);
  uint32_t* stage_hi = reinterpret_cast<uint32_t*>(smem + (size_t)NT * U * 16);
  uint8_t* stage_g = smem + (size_t)NT * U * (HI ? 20 : 16);
  __shared__ uint32_t cnt[kSuperMax + 1], cur[kSuperMax];
  const int64_t th = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t t = th / SH, hh = th % SH;
  const int64_t n = src.count();
  for (int i = threadIdx.x; i < SB; i += NT) {
    uint32_t c = sbro[(int64_t)i * (ntiles + 1) + t];
    for (int64_t k = 0; k < hh; ++k) c += subcnt[(t * SH + k) * SB + i];
    cur[i] = c;
  }
  __syncthreads();
  const bool carry = vin != nullptr;
  const uint32_t zmask = (1u << (b + g)) - 1u;
  const int64_t sub = T1 / SH;
  const int64_t base = t * T1 + hh * sub;
  const int64_t end = (base + sub < n) ? base + sub : n;
  for (int64_t e0 = base; e0 < end; e0 += (int64_t)NT * U) {
    uint32_t grp[U], hi[U];
    uint4 rec[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + (int64_t)u * NT + threadIdx.x;
      uint32_t seg;
      uint64_t key;
      grp[u] = kNoGroup;
      hi[u] = 0u;
      rec[u] = make_uint4(0u, 0u, 0u, 0u);
      if (e < end && (int)src.elem(e, seg, key) == kElemOk) {
        const VT v = carry ? vin[e] : VT(0);
        grp[u] = seg >> (b + g);
        rec[u] = make_uint4((uint32_t)key, (uint32_t)(key >> 32), seg & zmask,
                            carry ? ValWords<VT>::lo(v) : 0u);
        if (HI && carry) hi[u] = ValWords<VT>::hi(v);
      }
    }
    staged_runs<NT, U, HI>(grp, rec, hi, SB, cnt, cur, stage, stage_hi, stage_g, irec, ivhi);
  }
}

// Pass B: the slice of super-bucket s that tiles [q K, q K + K) wrote, into its buckets.
template <int NT, typename VT>
__global__ __launch_bounds__(NT) void k_part_scatter_b(int b, int g, int32_t CB,
                                                       int64_t ntiles, int64_t K, int64_t nq,
                                                       const uint32_t* __restrict__ sbro,
                                                       const uint32_t* __restrict__ rowoff,
                                                       const int32_t* __restrict__ bstart,
                                                       const uint4* __restrict__ irec,
                                                       const uint32_t* __restrict__ ivhi,
                                                       uint4* __restrict__ brec,
                                                       uint32_t* __restrict__ bvhi) {
  constexpr int U = 4;
  constexpr bool HI = ValWords<VT>::kHi;
  extern __shared__ __align__(16) unsigned char smem[];
  uint4* stage = reinterpret_cast<uint4*>(smem);
  uint32_t* stage_hi = reinterpret_cast<uint32_t*>(smem + (size_t)NT * U * 16);
  uint8_t* stage_g = smem + (size_t)NT * U * (HI ? 20 : 16);
  __shared__ uint32_t cnt[kSuperMax + 1], cur[kSuperMax];
  const int64_t idx = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t s = idx / nq, q = idx % nq;
  const int64_t t0 = q * K;
  const int64_t t1 = t0 + K < ntiles ? t0 + K : ntiles;
  const int64_t cb0 = s << g;
  const int ng = (int)min((int64_t)1 << g, (int64_t)CB - cb0);
  const uint32_t lo = sbro[s * (ntiles + 1) + t0], hi_end = sbro[s * (ntiles + 1) + t1];
  for (int j = threadIdx.x; j < ng; j += NT)
    cur[j] = (uint32_t)bstart[cb0 + j] + rowoff[(cb0 + j) * ntiles + t0];
  __syncthreads();
  const uint32_t wmask = (1u << b) - 1u;
  for (int64_t e0 = lo; e0 < (int64_t)hi_end; e0 += (int64_t)NT * U) {
    uint32_t grp[U], hi[U];
    uint4 rec[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + (int64_t)u * NT + threadIdx.x;
      grp[u] = kNoGroup;
      hi[u] = 0u;
      rec[u] = make_uint4(0u, 0u, 0u, 0u);
      if (e < (int64_t)hi_end) {
        rec[u] = irec[e];
        grp[u] = rec[u].z >> b;
        if (grp[u] >= (uint32_t)ng) grp[u] = kNoGroup;  // never, for records pass A wrote
        rec[u].z &= wmask;
        if (HI) hi[u] = ivhi[e];
      }
    }
    staged_runs<NT, U, HI>(grp, rec, hi, ng, cnt, cur, stage, stage_hi, stage_g, brec, bvhi);
  }
}

// Per-bucket exclusive scan of one row of the (bucket x tile) table: rowoff[cb][t] = number of
// bucket-cb elements in tiles before t; btot[cb] = the bucket's total.  One workgroup per row.
// Workgroup 0 also folds the nflags status flags of the checking kernel into info[1].
// big (nullable): a bucket of more than big_cap elements is appended to the list
// big[1 .. 1 + big[0]) (big[0] cleared by k_part_hist); level 2 takes those in a launch of
// their own.  The list's order is arbitrary; every bucket's result is independent of it.
template <int NT>
__global__ __launch_bounds__(NT) void k_rows_scan(const uint32_t* __restrict__ table,
                                                  int64_t ntiles, uint32_t* __restrict__ rowoff,
                                                  uint32_t* __restrict__ btot,
                                                  const uint32_t* __restrict__ flags,
                                                  int64_t nflags, int32_t* __restrict__ info,
                                                  uint32_t big_cap, uint32_t* __restrict__ big) {
  __shared__ uint32_t s_w[NT / kWave + 1];
  __shared__ uint32_t s_flag;
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) s_flag = 0;
    __syncthreads();
    uint32_t f = 0;
    for (int64_t i = threadIdx.x; i < nflags; i += NT) f |= flags[i];
    if (f) atomicOr(&s_flag, f);
    __syncthreads();
    if (threadIdx.x == 0)
      info[1] = (s_flag & kFlagShape) ? kStEinval : ((s_flag & kFlagIndex) ? kStBounds : 0);
  }
  constexpr int IPT = 4;
  const int64_t cb = blockIdx.x;
  const uint32_t* in = table + cb * ntiles;
  uint32_t* out = rowoff + cb * ntiles;
  uint32_t carry = 0;
  for (int64_t base = 0; base < ntiles; base += (int64_t)NT * IPT) {
    uint32_t v[IPT];
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      const int64_t i = base + (int64_t)threadIdx.x * IPT + q;
      v[q] = i < ntiles ? in[i] : 0u;
      sum += v[q];
    }
    uint32_t tot;
    uint32_t run = carry + wg_excl_scan<NT>(sum, s_w, &tot);
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      const int64_t i = base + (int64_t)threadIdx.x * IPT + q;
      if (i < ntiles) out[i] = run;
      run += v[q];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    btot[cb] = carry;
    if (big && carry > big_cap) big[1 + atomicAdd(&big[0], 1u)] = (uint32_t)cb;
  }
}

// ------------------------------------------------------------------------------------------
// Level 2, fused with what follows it.  One workgroup per coarse bucket (bucket elements
// bstarts[cb] .. bstarts[cb+1]).
//   PLAN = true : writes row_ptr for the bucket's rows and col_t / perm of their elements.
//   PLAN = false: (assembly) folds every run of equal (column, row) left to right in input
//                 order in binary64, drops zero sums, and writes the survivors compacted
//                 within the bucket to temporaries (trow, tval at the bucket's own offset),
//                 the bucket-relative column offsets to col_rel and the survivor count to
//                 bkept[cb]; k_part_emit then places them.
// A bucket of at most CAP elements stays in LDS from load to output (fast path); a larger
// one goes through global staging: segment scatter, sort_segments, then fold_tile over
// blocks of CAP keys.
// Dynamic LDS: cnt[W*R+1] u32 | s_in[CAP] u64 | s_key[CAP] u64 | s_flag[CAP] u8
//              (part_level2_lds_bytes).  The fold's values s_val[CAP] f64 and survivor
//              prefix s_pre[CAP+1] u32 reuse s_key, which is dead once the bucket is sorted;
//              at b = 7 a workgroup takes about 39 KB, four per CU.
// In the fast path each segment is split into R = 2^lr sub-segments by the top bits of the
// key's high word (the row for assembly, the column for the plan: key_hi >> rshift < R), so
// the ranking runs over short sub-segments even when a segment is long; the sub-segments of
// a segment are in ascending key order, so the sorted result is the same.
// In the fast path every thread keeps the key, segment (and, folding, the value) of its
// elements i = tid + u*NT in registers from the first load to the ranking; the value gather
// is issued before the counting so that its latency overlaps the LDS work.
// ------------------------------------------------------------------------------------------
// Sub-segments per segment in the in-LDS path: R = 2^l2_sub_log2(b), so that W*R >= 1024.
__host__ __device__ inline int l2_sub_log2(int b) { return b >= 10 ? 0 : 10 - b; }

__host__ __device__ inline size_t part_level2_lds_bytes(int b, int cap) {
  const size_t w = ((size_t)1 << (b + l2_sub_log2(b))) + 1;
  size_t off = (w * 4 + 15) & ~(size_t)15;
  off += (size_t)cap * 8 * 2;
  off += (size_t)cap;
  return off;
}

// What one level-2 workgroup sees of its bucket.
struct L2Bucket {
  int64_t cb, bstart, bend, m, seg0, nW, nseg;
  bool last_bucket;
};

// Assembly fused with the plan: the bucket's survivors counted per row bucket (2^br rows),
// table2[rb * CB + cb] -- the (row bucket x column bucket) table the plan's partition is
// laid out from.  table2 == nullptr: not counted.  The counters live in s_in (CBr <= CAP * 2
// u32), which is dead once the survivors are out.
struct L2RowCount {
  uint32_t* table2;
  int br;
  int32_t CBr;
  int32_t CB;
};

template <int NT>
__device__ __forceinline__ void l2_clear_counts(const L2RowCount& rc, uint32_t* h) {
  for (int64_t i = threadIdx.x; i < rc.CBr; i += NT) h[i] = 0;
}
template <int NT>
__device__ __forceinline__ void l2_store_counts(const L2RowCount& rc, int64_t cb,
                                                const uint32_t* h) {
  for (int64_t i = threadIdx.x; i < rc.CBr; i += NT) rc.table2[i * rc.CB + cb] = h[i];
}

// LDS views of the dynamic shared memory (layout as in part_level2_lds_bytes).
template <int CAP>
struct L2Lds {
  uint32_t* cnt;
  uint64_t* s_in;
  uint64_t* s_key;
  uint8_t* s_flag;
  __device__ __forceinline__ L2Lds(unsigned char* smem, int b) {
    const size_t wcnt = ((size_t)1 << (b + l2_sub_log2(b))) + 1;
    size_t off = (wcnt * 4 + 15) & ~(size_t)15;
    cnt = reinterpret_cast<uint32_t*>(smem);
    s_in = reinterpret_cast<uint64_t*>(smem + off);
    off += (size_t)CAP * 8;
    s_key = reinterpret_cast<uint64_t*>(smem + off);
    off += (size_t)CAP * 8;
    s_flag = smem + off;
  }
};

// PLAN: row_ptr of the bucket's rows from the inclusive counts (cnt[j] = end of row j).
template <int NT>
__device__ __forceinline__ void l2_row_ptr(const L2Bucket& B, const uint32_t* cnt,
                                           int32_t* __restrict__ row_ptr) {
  for (int64_t j = threadIdx.x; j < B.nW; j += NT)
    row_ptr[B.seg0 + j] = (int32_t)(B.bstart + (j == 0 ? 0 : (int64_t)cnt[j - 1]));
  if (B.last_bucket && threadIdx.x == 0) row_ptr[B.nseg] = (int32_t)B.bend;
}

// Fast path (m <= CAP): the whole bucket stays in LDS from load to output.
template <int NT, int CAP, bool PLAN, typename VT>
__device__ __forceinline__ void l2_fast(const L2Bucket& B, const L2Lds<CAP>& L, uint32_t* s_w,
                                        int lr, int rshift, const uint4* __restrict__ brec,
                                        const uint32_t* __restrict__ bvhi,
                                        int32_t* __restrict__ row_ptr,
                                        int32_t* __restrict__ col_t, int32_t* __restrict__ perm,
                                        VT* __restrict__ val_plan,
                                        int32_t* __restrict__ col_rel,
                                        uint32_t* __restrict__ trow, double* __restrict__ tval,
                                        uint32_t* __restrict__ bkept, const L2RowCount& rc) {
  constexpr int IPT = CAP / NT;
  const int64_t m = B.m, nW = B.nW;
  const int64_t nS = nW << lr;  // sub-segments
  const uint32_t rmax = (1u << lr) - 1u;
  uint32_t* cnt = L.cnt;
  uint64_t* s_in = L.s_in;
  uint64_t* s_key = L.s_key;
  uint8_t* s_flag = L.s_flag;

  for (int64_t j = threadIdx.x; j <= nS; j += NT) cnt[j] = 0;
  uint64_t ky[IPT];
  uint32_t sg[IPT];
  VT vv[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int64_t i = threadIdx.x + (int64_t)u * NT;
    ky[u] = 0ull;
    sg[u] = 0xffffffffu;
    if (i < m) {
      const uint4 r = brec[B.bstart + i];
      ky[u] = rec_key(r);
      // clamped: a malformed CSC handed to the plan may carry any column word
      const uint32_t sub = min((uint32_t)(ky[u] >> 32) >> rshift, rmax);
      sg[u] = (r.z << lr) | sub;
      if (!PLAN || val_plan)
        vv[u] = ValWords<VT>::make(r.w, ValWords<VT>::kHi ? bvhi[B.bstart + i] : 0u);
    }
  }
  __syncthreads();  // cnt cleared
#pragma unroll
  for (int u = 0; u < IPT; ++u)
    if (sg[u] != 0xffffffffu) atomicAdd(&cnt[sg[u]], 1u);
  __syncthreads();
  wg_inclusive_scan_inplace<NT>(cnt, nS, s_w);  // cnt[s] = end of sub-segment s (relative)
  if (PLAN) {
    for (int64_t j = threadIdx.x; j < nW; j += NT)
      row_ptr[B.seg0 + j] = (int32_t)(B.bstart + (j == 0 ? 0 : (int64_t)cnt[(j << lr) - 1]));
    if (B.last_bucket && threadIdx.x == 0) row_ptr[B.nseg] = (int32_t)B.bend;
  }
  __syncthreads();

  // Group by sub-segment: each element takes the next free slot of its sub-segment.
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    if (sg[u] != 0xffffffffu) {
      const uint32_t pos = atomicSub(&cnt[sg[u]], 1u) - 1u;
      s_key[pos] = ky[u];
    }
  }
  for (int64_t i = threadIdx.x; i < m; i += NT) s_flag[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) cnt[nS] = (uint32_t)m;  // cnt[s] = start of sub-segment s
  __syncthreads();
  for (int64_t j = threadIdx.x; j < nW; j += NT) {  // flags mark segment starts
    const uint32_t lo = cnt[j << lr];
    if (lo < (uint32_t)m) s_flag[lo] = 1;
  }
  // Rank each element among the keys of its sub-segment (keys are unique, so the ranks are a
  // permutation): the bounds come from cnt, so the loads are independent and issued four at
  // a time.
  uint32_t dst[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    dst[u] = 0;
    if (sg[u] != 0xffffffffu) {
      const uint32_t lo = cnt[sg[u]], hi = cnt[sg[u] + 1];
      const uint64_t key = ky[u];
      uint32_t r = 0, q = lo;
      for (; q + 4 <= hi; q += 4) {
        const uint64_t k0 = s_key[q], k1 = s_key[q + 1], k2 = s_key[q + 2], k3 = s_key[q + 3];
        r += (uint32_t)(k0 < key) + (uint32_t)(k1 < key) + (uint32_t)(k2 < key) +
             (uint32_t)(k3 < key);
      }
      for (; q < hi; ++q) r += (uint32_t)(s_key[q] < key);
      dst[u] = lo + r;
      s_in[lo + r] = key;  // s_in now holds the bucket sorted by (segment, key)
    }
  }
  __syncthreads();
  if (PLAN) {
    for (int64_t i = threadIdx.x; i < m; i += NT) {
      const uint64_t key = s_in[i];
      col_t[B.bstart + i] = (int32_t)(key >> 32);
      perm[B.bstart + i] = (int32_t)(uint32_t)key;
    }
    if (val_plan) {  // the values follow their keys to the sorted slots (s_key is dead)
      double* s_pv = reinterpret_cast<double*>(s_key);
#pragma unroll
      for (int u = 0; u < IPT; ++u)
        if (sg[u] != 0xffffffffu) s_pv[dst[u]] = to_acc<double>(vv[u]);
      __syncthreads();
      for (int64_t i = threadIdx.x; i < m; i += NT) val_plan[B.bstart + i] = (VT)s_pv[i];
    }
    return;
  }
  // Fold.  Each element's value (loaded with its key) goes to its sorted position in s_val
  // (reusing s_key, dead after the ranking).  The thread owning a run's head folds the run
  // from LDS in key order (= input order within a run); the sum replaces the value at the
  // head, which no other thread reads.
  double* s_val = reinterpret_cast<double*>(s_key);
#pragma unroll
  for (int u = 0; u < IPT; ++u)
    if (sg[u] != 0xffffffffu) s_val[dst[u]] = to_acc<double>(vv[u]);
  __syncthreads();
  // Position i = u*NT + tid (u = 0..IPT-1): rounds of consecutive positions, so a wave's
  // ballot of survivors gives each lane its rank within the wave, and one scan of the
  // (round, wave) counts in position order gives the rest.  Survivors go out coalesced.
  constexpr int NWV = NT / kWave;
  __shared__ uint32_t s_cw[IPT * NWV + 1];
  uint64_t bal[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int64_t i = (int64_t)u * NT + threadIdx.x;
    bool keep = false;
    if (i < m) {
      const uint32_t row = key_row(s_in[i]);
      const bool head = s_flag[i] || key_row(s_in[i - 1]) != row;
      if (head) {
        double acc = s_val[i];
        for (int64_t j = i + 1; j < m && !s_flag[j]; ++j) {
          if (key_row(s_in[j]) != row) break;
          acc = acc + s_val[j];
        }
        s_val[i] = acc;
        keep = acc != 0.0;
      }
    }
    bal[u] = __ballot(keep);
    if (lane_id() == 0) s_cw[u * NWV + wave_id()] = (uint32_t)__popcll(bal[u]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int k = 0; k < IPT * NWV; ++k) {
      const uint32_t c = s_cw[k];
      s_cw[k] = run;
      run += c;
    }
    s_cw[IPT * NWV] = run;
  }
  __syncthreads();
  const uint32_t kept = s_cw[IPT * NWV];
  const uint64_t lt = (1ull << lane_id()) - 1ull;
  uint32_t rank[IPT];
  uint32_t orow[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int64_t i = (int64_t)u * NT + threadIdx.x;
    rank[u] = s_cw[u * NWV + wave_id()] + (uint32_t)__popcll(bal[u] & lt);
    orow[u] = 0;
    if ((bal[u] >> lane_id()) & 1ull) {
      orow[u] = key_row(s_in[i]);
      trow[B.bstart + rank[u]] = orow[u];
      tval[B.bstart + rank[u]] = s_val[i];
    }
  }
  __syncthreads();  // s_val is read; the survivor prefix s_pre takes its place
  uint32_t* s_pre = reinterpret_cast<uint32_t*>(s_key);
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int64_t i = (int64_t)u * NT + threadIdx.x;
    if (i < m) s_pre[i] = rank[u];
  }
  if (threadIdx.x == 0) s_pre[m] = kept;
  __syncthreads();
  for (int64_t j = threadIdx.x; j < nW; j += NT)
    col_rel[B.seg0 + j] = (int32_t)s_pre[cnt[j << lr]];
  if (threadIdx.x == 0) bkept[B.cb] = kept;
  if (rc.table2) {
    uint32_t* h = reinterpret_cast<uint32_t*>(s_in);  // s_in was last read before a barrier
    l2_clear_counts<NT>(rc, h);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < IPT; ++u)
      if ((bal[u] >> lane_id()) & 1ull) atomicAdd(&h[orow[u] >> rc.br], 1u);
    __syncthreads();
    l2_store_counts<NT>(rc, B.cb, h);
  }
}

// Slow path (m > CAP): segment scatter through global staging, sort_segments, then
// fold_tile over blocks of CAP keys.
template <int NT, int CAP, bool PLAN, typename VT>
__device__ __forceinline__ void l2_slow(const L2Bucket& B, const L2Lds<CAP>& L, uint32_t* s_w,
                                        int64_t* s_b, const uint4* __restrict__ brec,
                                        uint64_t* __restrict__ gkeys,
                                        uint64_t* __restrict__ scratch,
                                        int32_t* __restrict__ row_ptr,
                                        int32_t* __restrict__ col_t, int32_t* __restrict__ perm,
                                        const VT* __restrict__ val, VT* __restrict__ val_plan,
                                        int32_t* __restrict__ col_rel,
                                        uint32_t* __restrict__ trow, double* __restrict__ tval,
                                        uint32_t* __restrict__ bkept, const L2RowCount& rc) {
  constexpr int IPT = CAP / NT;
  constexpr int U = 8;
  const int64_t m = B.m, nW = B.nW, bstart = B.bstart, bend = B.bend;
  uint32_t* cnt = L.cnt;
  uint64_t* s_in = L.s_in;
  uint32_t* s_pre = reinterpret_cast<uint32_t*>(L.s_key);
  for (int64_t j = threadIdx.x; j <= nW; j += NT) cnt[j] = 0;
  __syncthreads();
  for (int64_t e0 = bstart + threadIdx.x; e0 < bend; e0 += (int64_t)NT * U) {
    uint32_t gs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + (int64_t)u * NT;
      gs[u] = (e < bend) ? brec[e].z : 0xffffffffu;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (gs[u] != 0xffffffffu) atomicAdd(&cnt[gs[u]], 1u);
  }
  __syncthreads();
  wg_inclusive_scan_inplace<NT>(cnt, nW, s_w);  // cnt[j] = end of segment j (relative)
  if (PLAN) l2_row_ptr<NT>(B, cnt, row_ptr);
  __syncthreads();
  uint64_t* gk = gkeys + bstart;
  for (int64_t e0 = bstart + threadIdx.x; e0 < bend; e0 += (int64_t)NT * U) {
    uint32_t gs[U];
    uint64_t gy[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + (int64_t)u * NT;
      gs[u] = 0xffffffffu;
      gy[u] = 0ull;
      if (e < bend) {
        const uint4 r = brec[e];
        gs[u] = r.z;
        gy[u] = rec_key(r);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (gs[u] != 0xffffffffu) {
        const uint32_t pos = atomicSub(&cnt[gs[u]], 1u) - 1u;
        gk[pos] = gy[u];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) cnt[nW] = (uint32_t)m;
  __syncthreads();
  sort_segments<NT, CAP, PLAN>(gk, cnt, 0, nW, scratch + bstart, PLAN ? col_t + bstart : col_t,
                               PLAN ? perm + bstart : perm, L.s_key,
                               reinterpret_cast<uint32_t*>(L.s_in), s_b);
  if (PLAN) {
    if (val_plan) {  // staged buckets gather their values (val in CSC order, slots < cap)
      __syncthreads();
      for (int64_t q = bstart + threadIdx.x; q < bend; q += NT) val_plan[q] = val[perm[q]];
    }
    return;
  }
  __syncthreads();
  // one pass over blocks of CAP sorted (tagged) keys: fold, compact into the temporaries
  uint32_t running = 0;
  for (int64_t base = 0; base < m; base += CAP) {
    const int nb = (int)((m - base) < CAP ? (m - base) : CAP);
    for (int i = threadIdx.x; i < nb; i += NT) s_in[i] = gk[base + i];
    __syncthreads();
    uint32_t rows[IPT];
    double sums[IPT];
    const uint32_t mask = fold_tile<NT, IPT, VT>(gk, s_in, base, nb, m, val, rows, sums);
    uint32_t blk;
    const uint32_t excl = wg_excl_scan<NT>((uint32_t)__popc(mask), s_w, &blk);
    {
      uint32_t run = excl;
#pragma unroll
      for (int s = 0; s < IPT; ++s) {
        const int li = threadIdx.x * IPT + s;
        if (li < nb) s_pre[li] = run;
        run += (mask >> s) & 1u;
      }
      if (threadIdx.x == 0) {
        s_pre[nb] = blk;
        const bool last = base + CAP >= m;
        s_b[1] = lower_bound(cnt, nW + 1, base);
        s_b[2] = last ? nW + 1 : lower_bound(cnt, nW + 1, base + CAP);
      }
    }
    __syncthreads();
    {
      int64_t o = bstart + running + excl;
#pragma unroll
      for (int s = 0; s < IPT; ++s) {
        if ((mask >> s) & 1u) {
          trow[o] = rows[s];
          tval[o] = sums[s];
          ++o;
        }
      }
    }
    for (int64_t j = s_b[1] + threadIdx.x; j < s_b[2]; j += NT) {
      if (j >= nW) continue;  // cnt[nW] = m marks the bucket end, not a column
      int64_t p = (int64_t)cnt[j] - base;
      if (p > nb) p = nb;
      col_rel[B.seg0 + j] = (int32_t)(running + s_pre[p]);
    }
    running += blk;
    __syncthreads();
  }
  if (threadIdx.x == 0) bkept[B.cb] = running;
  if (rc.table2) {
    // the survivors are back in trow (written by this workgroup before the last barrier)
    uint32_t* h = reinterpret_cast<uint32_t*>(s_in);
    l2_clear_counts<NT>(rc, h);
    __syncthreads();
    for (int64_t i = threadIdx.x; i < (int64_t)running; i += NT)
      atomicAdd(&h[trow[bstart + i] >> rc.br], 1u);
    __syncthreads();
    l2_store_counts<NT>(rc, B.cb, h);
  }
}

// Level 2 of bucket cb: the in-LDS path when it holds at most CAP elements, else the staged
// path.
template <int NT, int CAP, bool PLAN, typename VT>
__device__ __forceinline__ void l2_bucket(
    int64_t cb, int b, int64_t nseg, const int32_t* __restrict__ bstarts,
    const uint4* __restrict__ brec, const uint32_t* __restrict__ bvhi,
    uint64_t* __restrict__ gkeys, uint64_t* __restrict__ scratch, int32_t* __restrict__ row_ptr,
    int32_t* __restrict__ col_t, int32_t* __restrict__ perm, const VT* __restrict__ val,
    VT* __restrict__ val_plan, int32_t* __restrict__ col_rel, uint32_t* __restrict__ trow,
    double* __restrict__ tval, uint32_t* __restrict__ bkept, int rshift, const L2RowCount& rc,
    const L2Lds<CAP>& L, uint32_t* s_w, int64_t* s_b) {
  L2Bucket B;
  B.cb = cb;
  B.bstart = bstarts[B.cb];
  B.bend = bstarts[B.cb + 1];
  B.m = B.bend - B.bstart;
  B.seg0 = B.cb << b;
  B.nseg = nseg;
  const int64_t rem = nseg - B.seg0;
  B.nW = rem < ((int64_t)1 << b) ? rem : ((int64_t)1 << b);
  B.last_bucket = B.seg0 + B.nW >= nseg;
  if (B.m <= CAP)
    l2_fast<NT, CAP, PLAN, VT>(B, L, s_w, l2_sub_log2(b), rshift, brec, bvhi, row_ptr, col_t,
                               perm, val_plan, col_rel, trow, tval, bkept, rc);
  else
    l2_slow<NT, CAP, PLAN, VT>(B, L, s_w, s_b, brec, gkeys, scratch, row_ptr, col_t, perm,
                               val, val_plan, col_rel, trow, tval, bkept, rc);
}

// One workgroup per bucket.  big_skip != nullptr: buckets of more than CAP elements are left
// to k_part_level2_big (listed by k_rows_scan).
// Waves per SIMD asked of the compiler for level 2.  The 512-thread form (many buckets) at
// eight waves spills a few registers of the fold and still measured faster than at the six its
// 78 VGPRs allow (power-law workload: fold 254 against 288 µs, plan 164 against 186 µs).
template <int NT> constexpr int kL2Waves = NT >= 512 ? 8 : 4;
template <int NT, int CAP, bool PLAN, typename VT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kL2Waves<NT>))) void k_part_level2(
    int b, int64_t nseg, const int32_t* __restrict__ bstarts, const uint4* __restrict__ brec,
    const uint32_t* __restrict__ bvhi, uint64_t* __restrict__ gkeys,
    uint64_t* __restrict__ scratch, int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_t,
    int32_t* __restrict__ perm, const VT* __restrict__ val, VT* __restrict__ val_plan,
    int32_t* __restrict__ col_rel, uint32_t* __restrict__ trow, double* __restrict__ tval,
    uint32_t* __restrict__ bkept, int rshift, L2RowCount rc,
    const uint32_t* __restrict__ big_skip) {
  static_assert((CAP / NT) * NT == CAP, "CAP must be a multiple of the workgroup size");
  static_assert((CAP + 1) * 4 <= CAP * 8, "s_pre must fit in s_key");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_w[NT / kWave + 1];
  __shared__ int64_t s_b[3];
  const L2Lds<CAP> L(smem, b);
  const int64_t cb = xcd_tile(blockIdx.x, gridDim.x);
  if (big_skip && bstarts[cb + 1] - bstarts[cb] > CAP) return;
  l2_bucket<NT, CAP, PLAN, VT>(cb, b, nseg, bstarts, brec, bvhi, gkeys, scratch, row_ptr,
                               col_t, perm, val, val_plan, col_rel, trow, tval, bkept, rshift,
                               rc, L, s_w, s_b);
}

// The listed big buckets (big[1 .. 1 + big[0]), k_rows_scan), persistent workgroups each
// taking every gridDim-th entry, with the larger in-LDS capacity CAP (staged path beyond).
template <int NT, int CAP, bool PLAN, typename VT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_part_level2_big(
    int b, int64_t nseg, const int32_t* __restrict__ bstarts, const uint4* __restrict__ brec,
    const uint32_t* __restrict__ bvhi, uint64_t* __restrict__ gkeys,
    uint64_t* __restrict__ scratch, int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_t,
    int32_t* __restrict__ perm, const VT* __restrict__ val, VT* __restrict__ val_plan,
    int32_t* __restrict__ col_rel, uint32_t* __restrict__ trow, double* __restrict__ tval,
    uint32_t* __restrict__ bkept, int rshift, L2RowCount rc, const uint32_t* __restrict__ big,
    int32_t CB) {
  static_assert((CAP / NT) * NT == CAP, "CAP must be a multiple of the workgroup size");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_w[NT / kWave + 1];
  __shared__ int64_t s_b[3];
  const L2Lds<CAP> L(smem, b);
  const uint32_t nbig = min(big[0], (uint32_t)CB);
  for (uint32_t i = blockIdx.x; i < nbig; i += gridDim.x) {
    const uint32_t cb = big[1 + i];
    __syncthreads();  // the previous bucket is done with the LDS
    if (cb >= (uint32_t)CB) continue;
    l2_bucket<NT, CAP, PLAN, VT>(cb, b, nseg, bstarts, brec, bvhi, gkeys, scratch, row_ptr,
                                 col_t, perm, val, val_plan, col_rel, trow, tval, bkept,
                                 rshift, rc, L, s_w, s_b);
  }
}

// Values in plan order for the plans built without the partition: val_plan[q] =
// val[perm[q]] for q < nnz (nnz = col_ptr[n_cols] clamped to the capacity; a slot outside
// the capacity, possible only for a malformed CSC, is skipped).
template <int NT, typename VT>
__global__ __launch_bounds__(NT) void k_plan_values(const int32_t* __restrict__ col_ptr,
                                                    int64_t n_cols, int64_t nnz_cap,
                                                    const int32_t* __restrict__ perm,
                                                    const VT* __restrict__ val,
                                                    VT* __restrict__ val_plan) {
  const int64_t raw = col_ptr[n_cols];
  const int64_t nnz = raw < 0 ? 0 : (raw > nnz_cap ? nnz_cap : raw);
  for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < nnz;
       q += (int64_t)gridDim.x * NT) {
    const int32_t p = perm[q];
    if (p >= 0 && (int64_t)p < nnz_cap) val_plan[q] = val[p];
  }
}

// Exclusive scan of n counts by ONE workgroup: out[i] = sum in[0..i), out[n] = total.  Used
// for the survivor offsets when there are too many buckets for k_part_emit to reduce them
// per workgroup.  Each wave scans a segment of 64 * IPT counts in coalesced slices of 64;
// with NT * IPT >= n (the launch takes 1024 x 16 for up to 16384 buckets) the scan is one
// round of loads.
template <int NT, int IPT>
__global__ __launch_bounds__(NT) void k_small_scan(const uint32_t* __restrict__ in, int64_t n,
                                                   int32_t* __restrict__ out) {
  __shared__ uint32_t s_w[NT / kWave + 1];
  constexpr int64_t kSeg = (int64_t)kWave * IPT;  // counts per wave and round
  uint32_t carry = 0;
  for (int64_t base = 0; base < n; base += (int64_t)NT * IPT) {
    // wave w scans its segment in coalesced slices of 64, carrying the slice totals
    const int64_t seg = base + (int64_t)wave_id() * kSeg;
    uint32_t v[IPT];
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      const int64_t i = seg + (int64_t)q * kWave + lane_id();
      v[q] = i < n ? in[i] : 0u;
    }
    uint32_t wsum = 0;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      const uint32_t incl = wave_incl_scan(v[q]);
      const uint32_t x = v[q];
      v[q] = wsum + incl - x;  // exclusive within the wave's segment
      wsum += __shfl(incl, kWave - 1, kWave);
    }
    uint32_t tot;
    const uint32_t wpre = wg_excl_scan<NT>(lane_id() == 0 ? wsum : 0u, s_w, &tot);
    const uint32_t woff = carry + __shfl(wpre, 0, kWave);  // the waves before this one
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      const int64_t i = seg + (int64_t)q * kWave + lane_id();
      if (i < n) out[i] = (int32_t)(woff + v[q]);
    }
    carry += tot;
  }
  if (threadIdx.x == 0) out[n] = (int32_t)carry;
}

// Plan outputs of the fused assembly + plan: the survivors go out a second time as records
// of the plan's row partition (key = column << 32 | CSC slot, segment = row within its row
// bucket, value = the stored value), into row bucket rb at bstart2[rb] + rowoff2[rb][cb] +
// rank.  rowoff2 / btot2 come from k_rows_scan over the counts level 2 took (L2RowCount).
struct EmitPlan {
  int br;                   // log2(rows per row bucket)
  int32_t CBr;              // row buckets (<= kFuseMaxRowBuckets)
  const uint32_t* rowoff2;  // [CBr][CB]: offset of column bucket cb's survivors in row bucket rb
  const uint32_t* btot2;    // [CBr] survivors per row bucket
  int32_t* bstart2;         // [CBr + 1] written by workgroup 0 (exclusive scan of btot2)
  uint4* brec2;             // plan partition records
  uint32_t* bvhi2;          // high words of float64 values
  int32_t* plan_info;       // plan info[0] = nnz
};
constexpr int kFuseMaxRowBuckets = 4096;

// Place each bucket's survivors.  The bucket's output offset is the sum of the survivor
// counts of the buckets before it: boff[cb] when the caller scanned them (boff != nullptr,
// many buckets), else each workgroup reduces bkept[0..cb) itself (the last one also takes
// its own, giving nnz_out).  Moves the survivors from the temporaries to their final place
// (rounded once to the output type), turns the bucket-relative column offsets into col_ptr,
// and finishes col_ptr / info.  With ep.brec2 set (fused plan) every survivor also goes out
// as a plan partition record; its column is found by binary search over the bucket's column
// offsets (in LDS), and its rank among the column bucket's survivors of its row bucket comes
// from an LDS cursor per row bucket.  Dynamic LDS: 4 * (CBr + 2^b + 1) bytes when fused.
template <int NT>
__global__ __launch_bounds__(NT) void k_part_emit(int b, int32_t CB, int64_t nseg,
                                                  const int32_t* __restrict__ bstarts,
                                                  const uint32_t* __restrict__ bkept,
                                                  const int32_t* __restrict__ boff,
                                                  const uint32_t* __restrict__ trow,
                                                  const double* __restrict__ tval,
                                                  int32_t* __restrict__ col_ptr,
                                                  int32_t* __restrict__ row_idx,
                                                  void* __restrict__ val_out, int out_f64,
                                                  int32_t* __restrict__ info, EmitPlan ep) {
  __shared__ uint32_t s_w[NT / kWave + 1];
  // fused plan only (dynamic LDS): cur2[CBr] cursors | crel[W + 1] column starts in the bucket
  extern __shared__ uint32_t s_emit[];
  const int64_t cb = xcd_tile(blockIdx.x, gridDim.x);
  const bool last = cb == (int64_t)CB - 1;
  const int64_t kept = bkept[cb];
  const int64_t src0 = bstarts[cb];
  const int64_t seg0 = cb << b;
  const int64_t rem = nseg - seg0;
  const int64_t nW = rem < ((int64_t)1 << b) ? rem : ((int64_t)1 << b);
  constexpr int U = 4;  // elements in flight per thread
  uint32_t r[U];
  double v[U];
  auto load = [&](int64_t i0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * NT;
      r[u] = 0;
      v[u] = 0.0;
      if (i < kept) {
        r[u] = trow[src0 + i];
        v[u] = tval[src0 + i];
      }
    }
  };
  uint32_t* cur2 = s_emit;
  uint32_t* crel = s_emit + ep.CBr;
  if (ep.brec2) {
    // the first batch, the bucket's column starts and the table column are all requested
    // before the row-bucket totals are scanned
    load(threadIdx.x);
    for (int64_t j = threadIdx.x; j < nW; j += NT) crel[j] = (uint32_t)col_ptr[seg0 + j];
    if (threadIdx.x == 0) crel[nW] = (uint32_t)kept;
    bucket_cursors<NT>(cur2, ep.CBr, ep.btot2, ep.rowoff2, CB, cb, cb == 0, ep.bstart2, s_w);
  }
  int64_t dst0, total;
  if (boff) {
    dst0 = boff[cb];
    total = boff[CB];
  } else {
    const int64_t lim = last ? CB : cb;
    uint32_t part = 0;
    for (int64_t i = threadIdx.x; i < lim; i += NT) part += bkept[i];
    uint32_t tot;
    (void)wg_excl_scan<NT>(part, s_w, &tot);
    dst0 = last ? (int64_t)tot - kept : (int64_t)tot;
    total = tot;
  }
  if (ep.brec2) {
    const uint32_t wmask2 = (1u << ep.br) - 1u;
    const int lgw = 31 - __clz((int)nW);  // floor(log2(nW)), nW >= 1
    for (int64_t i0 = threadIdx.x; i0 < kept; i0 += (int64_t)NT * U) {
      if (i0 != threadIdx.x) load(i0);
      // column of each element: the last j with crel[j] <= i (branch-free binary search
      // over the bucket's nW column starts; crel[nW] = kept is never passed)
      int c[U];
#pragma unroll
      for (int u = 0; u < U; ++u) c[u] = 0;
      for (int step = 1 << lgw; step > 0; step >>= 1) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t i = (uint32_t)(i0 + (int64_t)u * NT);
          const int nx = c[u] + step;
          if (nx < (int)nW && crel[nx] <= i) c[u] = nx;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + (int64_t)u * NT;
        if (i < kept) {
          row_idx[dst0 + i] = (int32_t)r[u];
          if (out_f64) static_cast<double*>(val_out)[dst0 + i] = v[u];
          else static_cast<float*>(val_out)[dst0 + i] = (float)v[u];
          const uint32_t pos = atomicAdd(&cur2[r[u] >> ep.br], 1u);
          uint32_t vlo;
          if (out_f64) {
            vlo = (uint32_t)__double2loint(v[u]);
            ep.bvhi2[pos] = (uint32_t)__double2hiint(v[u]);
          } else {
            vlo = __float_as_uint((float)v[u]);
          }
          ep.brec2[pos] =
              make_uint4((uint32_t)(dst0 + i), (uint32_t)(seg0 + c[u]), r[u] & wmask2, vlo);
        }
      }
    }
  } else {
    for (int64_t i0 = threadIdx.x; i0 < kept; i0 += (int64_t)NT * U) {
      load(i0);  // U elements' loads in flight before any store
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + (int64_t)u * NT;
        if (i < kept) {
          row_idx[dst0 + i] = (int32_t)r[u];
          if (out_f64) static_cast<double*>(val_out)[dst0 + i] = v[u];
          else static_cast<float*>(val_out)[dst0 + i] = (float)v[u];
        }
      }
    }
  }
  // (the fused branch copied the bucket-relative offsets to LDS behind a barrier)
  for (int64_t j = threadIdx.x; j < nW; j += NT) col_ptr[seg0 + j] += (int32_t)dst0;
  if (last && threadIdx.x == 0) {
    col_ptr[nseg] = (int32_t)total;
    info[0] = (int32_t)total;
    if (ep.brec2) ep.plan_info[0] = (int32_t)total;
  }
}

}  // namespace spm
