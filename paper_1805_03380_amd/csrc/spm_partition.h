// Grouping elements by segment (the column of a triplet for assembly, the row of a stored
// element for the plan) without device-wide atomics.  Device-scope atomics on gfx950 are
// performed beyond the XCD-local L2 and cost far more than LDS atomics, so the grouping is a
// two-level partition whose counters all live in LDS:
//   level 1  the segments are cut into CB coarse buckets of W = 2^b consecutive segments.
//            k_part_hist: each tile of T1 elements counts its elements per coarse bucket in
//            LDS and writes one column of a (bucket x tile) table;  an exclusive scan of the
//            table (bucket-major) gives every (bucket, tile) pair its output range;
//            k_part_scatter: each tile ranks its elements per bucket with LDS atomics and
//            writes (key, segment-within-bucket) into the bucket's range.
//   level 2  k_part_sort: one workgroup per coarse bucket counts its elements per segment in
//            LDS, writes the segments' start offsets, scatters the keys into segment order and
//            sorts every segment by key (sort_segments: LDS rank sort, merge sort for segments
//            longer than an LDS chunk).
// Keys carry a unique element index, so the grouping order inside a bucket never matters.
#pragma once

#include "spm_assemble.h"

namespace spm {

constexpr int kPartMaxBuckets = 4096;   // coarse buckets per level (LDS counters)
constexpr int kPartMaxWidth = 4096;     // segments per coarse bucket (LDS counters)

// Element sources.  part_elem returns false for an element that is skipped (out of range).
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

// Column of every stored slot of a CSC, plus the checks the plan needs (monotone offsets,
// col_ptr[0] = 0, nnz <= capacity, rows in range).  One thread per column.
template <int NT>
__global__ __launch_bounds__(NT) void k_expand_columns(const int32_t* __restrict__ col_ptr,
                                                       const int32_t* __restrict__ row_idx,
                                                       int64_t n_rows, int64_t n_cols,
                                                       int64_t nnz_cap,
                                                       int32_t* __restrict__ colarr,
                                                       int32_t* __restrict__ info) {
  const int64_t raw = col_ptr[n_cols];
  const int64_t nnz = raw < 0 ? 0 : (raw > nnz_cap ? nnz_cap : raw);
  const int64_t gid = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * NT;
  bool bad_shape = false, bad_row = false;
  if (gid == 0) {
    if (col_ptr[0] != 0 || raw < 0 || raw > nnz_cap) bad_shape = true;
    info[0] = (int32_t)nnz;
  }
  for (int64_t c = gid; c < n_cols; c += stride) {
    int64_t p0 = col_ptr[c], p1 = col_ptr[c + 1];
    if (p0 > p1) bad_shape = true;
    p0 = p0 < 0 ? 0 : (p0 > nnz ? nnz : p0);
    p1 = p1 < p0 ? p0 : (p1 > nnz ? nnz : p1);
    for (int64_t p = p0; p < p1; ++p) {
      colarr[p] = (int32_t)c;
      const int32_t r = row_idx[p];
      if (r < 0 || (int64_t)r >= n_rows) bad_row = true;
    }
  }
  if (bad_shape) set_status(info, kStEinval);
  if (bad_row) set_status(info, kStBounds);
}

// Level 1a: per-tile coarse-bucket counts -> table[cb * ntiles + t].
template <int NT, typename SRC>
__global__ __launch_bounds__(NT) void k_part_hist(SRC src, int b, int32_t CB, int64_t ntiles,
                                                  int64_t T1, uint32_t* __restrict__ table,
                                                  int32_t* __restrict__ info) {
  __shared__ uint32_t h[kPartMaxBuckets];
  const int64_t t = blockIdx.x;
  const int64_t n = src.count();
  for (int i = threadIdx.x; i < CB; i += NT) h[i] = 0;
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
        ok[u] = src.elem(e, seg[u], key);
        bad |= !ok[u];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ok[u]) atomicAdd(&h[seg[u] >> b], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < CB; i += NT) table[(int64_t)i * ntiles + t] = h[i];
  if (bad && info) set_status(info, kStBounds);
}

// Level 1b: scatter (key, segment-within-bucket) into the buckets.
template <int NT, typename SRC>
__global__ __launch_bounds__(NT) void k_part_scatter(SRC src, int b, int32_t CB, int64_t ntiles,
                                                     int64_t T1, const int32_t* __restrict__ offs,
                                                     uint64_t* __restrict__ bkey,
                                                     uint32_t* __restrict__ bseg) {
  __shared__ uint32_t cur[kPartMaxBuckets];
  const int64_t t = blockIdx.x;
  const int64_t n = src.count();
  for (int i = threadIdx.x; i < CB; i += NT) cur[i] = (uint32_t)offs[(int64_t)i * ntiles + t];
  __syncthreads();
  const uint32_t wmask = (1u << b) - 1u;
  const int64_t base = t * T1;
  const int64_t end = (base + T1 < n) ? base + T1 : n;
  constexpr int U = 4;
  for (int64_t e0 = base + threadIdx.x; e0 < end; e0 += (int64_t)NT * U) {
    uint32_t seg[U];
    uint64_t key[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + (int64_t)u * NT;
      ok[u] = (e < end) ? src.elem(e, seg[u], key[u]) : false;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ok[u]) {
        const uint32_t pos = atomicAdd(&cur[seg[u] >> b], 1u);
        bkey[pos] = key[u];
        bseg[pos] = seg[u] & wmask;
      }
    }
  }
}

// Level 2: one workgroup per coarse bucket.  Writes segstart for the bucket's segments
// (and segstart[nseg] = total from the last bucket) and the segments' sorted keys into `out`
// (in place with kSegHead tags, or split into out_hi / out_lo when PLAN).
template <int NT, int CAP, bool PLAN>
__global__ __launch_bounds__(NT) void k_part_sort(int b, int32_t CB, int64_t ntiles,
                                                  int64_t nseg,
                                                  const int32_t* __restrict__ offs,
                                                  const uint64_t* __restrict__ bkey,
                                                  const uint32_t* __restrict__ bseg,
                                                  uint64_t* __restrict__ out,
                                                  uint64_t* __restrict__ scratch,
                                                  int32_t* __restrict__ segstart,
                                                  int32_t* __restrict__ out_hi,
                                                  int32_t* __restrict__ out_lo) {
  __shared__ uint32_t cnt[kPartMaxWidth + 1];
  __shared__ uint64_t s_key[CAP];
  __shared__ uint8_t s_flag[CAP];
  __shared__ uint32_t s_w[NT / kWave + 1];
  __shared__ int64_t s_b[1];
  const int64_t cb = blockIdx.x;
  const int64_t bstart = offs[cb * ntiles];
  const int64_t bend = offs[(cb + 1) * ntiles];  // offs has CB * ntiles + 1 entries
  const int64_t seg0 = cb << b;
  const int64_t rem = nseg - seg0;
  const int64_t nW = rem < ((int64_t)1 << b) ? rem : ((int64_t)1 << b);
  for (int64_t i = threadIdx.x; i <= nW; i += NT) cnt[i] = 0;
  __syncthreads();
  constexpr int U = 8;
  for (int64_t e0 = bstart + threadIdx.x; e0 < bend; e0 += (int64_t)NT * U) {
    uint32_t sg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + (int64_t)u * NT;
      sg[u] = (e < bend) ? bseg[e] : 0xffffffffu;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (sg[u] != 0xffffffffu) atomicAdd(&cnt[sg[u]], 1u);
  }
  __syncthreads();
  wg_inclusive_scan_inplace<NT>(cnt, nW, s_w);  // cnt[j] = end of segment j (relative)
  for (int64_t j = threadIdx.x; j < nW; j += NT)
    segstart[seg0 + j] = (int32_t)(bstart + (j == 0 ? 0 : (int64_t)cnt[j - 1]));
  if (cb == CB - 1 && threadIdx.x == 0) segstart[nseg] = (int32_t)bend;
  __syncthreads();
  uint64_t* obase = out + bstart;
  for (int64_t e0 = bstart + threadIdx.x; e0 < bend; e0 += (int64_t)NT * U) {
    uint32_t sg[U];
    uint64_t ky[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + (int64_t)u * NT;
      sg[u] = (e < bend) ? bseg[e] : 0xffffffffu;
      ky[u] = (e < bend) ? bkey[e] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (sg[u] != 0xffffffffu) {
        const uint32_t pos = atomicSub(&cnt[sg[u]], 1u) - 1u;
        obase[pos] = ky[u];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) cnt[nW] = (uint32_t)(bend - bstart);  // cnt[j] = start of segment j
  __syncthreads();
  sort_segments<NT, CAP, PLAN>(obase, cnt, 0, nW, scratch + bstart,
                               PLAN ? out_hi + bstart : out_hi, PLAN ? out_lo + bstart : out_lo,
                               s_key, s_flag, s_b);
}

}  // namespace spm
