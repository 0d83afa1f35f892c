// Batched path: launches that assemble, plan, multiply forward and backward many
// independent matrices.
//   k_batch       assembly and plan: persistent workgroups take whole matrices from a device
//                 queue (in the order the caller gives, largest first), keep the matrix's
//                 per-column / per-row counters in LDS and its keys in a per-workgroup slice
//                 of the workspace; each chunk of whole columns is sorted and folded in LDS
//                 in one pass, and values travel inside the keys when row and input position
//                 leave room for them;
//   k_batch_prefix, k_batch_tab, k_batch_flat
//                 forward over all rows and adjoint over all columns of all matrices, one
//                 grid each: the prefixes lay the rows (columns) out in schedule order, a
//                 table maps every chunk to the matrix holding its start, one record per
//                 matrix and direction carries what the products need, and every XCD takes a
//                 contiguous range of chunks in order, so its L2 holds a few matrices at a time;
//   k_batch_spmm  the same products one workgroup per matrix, when the workspace cannot hold
//                 the prefixes and tables the flat launches need.
// Every output is summed in the same order as by the per-matrix entry points (the same key
// order and binary64 fold, the same spmm_row / spmm_col_bwd device functions), so the results
// are bitwise equal to theirs.
#pragma once

#include "spm_partition.h"
#include "spm_spmm.h"
#include "spm.h"

namespace spm {

constexpr int kBatchMaxLdsDim = 8192;  // counters of up to this many columns / rows live in LDS
constexpr int kBatchCap = 2048;        // LDS sort chunk (keys)

struct BatchArgs {
  const spm_batch_item* items;
  const int32_t* order;
  int32_t batch;
  int64_t k;
  int G;
  const int32_t* row;
  const int32_t* col;
  const void* val;
  const void* X;
  const void* Gm;
  int32_t* col_ptr;
  int32_t* row_idx;
  float* val_out;
  int32_t* row_ptr;
  int32_t* col_t;
  int32_t* perm;
  float* Y;
  float* dX;
  float* dval;
  int32_t* info;
  int64_t max_dim;
  int64_t max_nnz;
  char* ws;           // per-worker slices
  size_t ws_stride;   // bytes per worker
  uint32_t* queue;    // [0]: grouping queue, [1]: products queue; zeroed before the launches
  int xal;            // X / G rows start on 4-element boundaries (vector loads allowed)
  int yal;            // Y / dX rows likewise (vector stores allowed)
};

// The item's sizes against the batch's limits (an item beyond them is skipped by both
// launches; the grouping launch reports SPM_EINVAL for it).
__device__ __forceinline__ bool batch_item_ok(const BatchArgs& a, const spm_batch_item& it) {
  return !(it.n_rows < 0 || it.n_cols < 0 || it.nnz_in < 0 || it.n_rows > a.max_dim ||
           it.n_cols > a.max_dim || it.nnz_in > a.max_nnz);
}

// Packed keys.  When a matrix's row and input position fit in 31 bits together, the key is
// (row << tb | position) << 32 | the value's bits: the sort orders it exactly as
// row << 32 | position (positions are unique), and the fold reads the value from the key
// instead of gathering it.  bit 63 stays free for kSegHead.
struct BatchKey {
  int tb;       // bits of the input position; -1: plain keys, values gathered by position
  __device__ __forceinline__ uint32_t row(uint64_t k) const {
    const uint32_t hi = (uint32_t)(k >> 32) & 0x7fffffffu;
    return tb < 0 ? hi : hi >> tb;
  }
};
__device__ __forceinline__ uint32_t vin_bits(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint32_t vin_bits(bf16_t v) { return (uint32_t)v; }
template <typename VIN> __device__ __forceinline__ float vin_value(uint32_t b);
template <> __device__ __forceinline__ float vin_value<float>(uint32_t b) { return __uint_as_float(b); }
template <> __device__ __forceinline__ float vin_value<bf16_t>(uint32_t b) {
  return to_acc<float>((bf16_t)(b & 0xffffu));
}
// The value of an element, binary32 (exact for f32 and bf16 input).
template <typename VIN>
__device__ __forceinline__ float batch_value(const BatchKey& bk, uint64_t k,
                                             const VIN* __restrict__ tval) {
  return bk.tb < 0 ? to_acc<float>(tval[(uint32_t)k]) : vin_value<VIN>((uint32_t)k);
}

// Columns [ca, cb) of one matrix, their keys (row << 32 | input position) at
// bucket[cnt[ca] .. cnt[cb]), at most kBatchCap of them: each column sorted by rank in LDS,
// then each run (one row of one column) folded left to right in binary64 from LDS; the
// survivors go to ri / vo (and their columns to slot_col) from `running` on, and the columns'
// offsets to cp.  Runs never leave the chunk: it holds whole columns.
template <int NT, typename VIN>
__device__ void batch_fold_chunk(const BatchKey bk, int64_t ca, int64_t cb, const uint32_t* cnt,
                                 const uint64_t* __restrict__ bucket,
                                 const VIN* __restrict__ tval, int32_t* __restrict__ ri,
                                 float* __restrict__ vo, int32_t* __restrict__ slot_col,
                                 int32_t* __restrict__ cp, uint32_t& running, uint64_t* s_key,
                                 float* s_val, int32_t* s_col, uint32_t* s_pre, uint32_t* s_w) {
  constexpr int IPT = kBatchCap / NT;
  constexpr int kLong = 64;  // longer columns get their bounds from the whole workgroup
  __shared__ int32_t s_long[kBatchCap / kLong + 1];
  __shared__ int32_t s_nlong;
  uint32_t* s_lohi = s_pre;  // bounds first, then the compaction prefix
  const int64_t e0 = cnt[ca];
  const int n = (int)((int64_t)cnt[cb] - e0);
  if (threadIdx.x == 0) s_nlong = 0;
  // keys and values, every load issued before the first use
  uint64_t kv[IPT];
  float vv[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int i = u * NT + threadIdx.x;
    kv[u] = i < n ? bucket[e0 + i] : 0ull;
  }
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int i = u * NT + threadIdx.x;
    vv[u] = i < n ? batch_value<VIN>(bk, kv[u], tval) : 0.0f;
    if (i < n) s_key[i] = kv[u];
  }
  __syncthreads();
  // bounds (lo | hi << 16, chunk-relative) and column of every element
  for (int64_t c = ca + threadIdx.x; c < cb; c += NT) {
    const int lo = (int)((int64_t)cnt[c] - e0), hi = (int)((int64_t)cnt[c + 1] - e0);
    if (hi - lo <= kLong) {
      for (int i = lo; i < hi; ++i) {
        s_lohi[i] = (uint32_t)lo | ((uint32_t)hi << 16);
        s_col[i] = (int32_t)c;
      }
    } else {
      s_long[atomicAdd(&s_nlong, 1)] = (int32_t)(c - ca);
    }
  }
  __syncthreads();
  for (int q = 0; q < s_nlong; ++q) {
    const int64_t c = ca + s_long[q];
    const int lo = (int)((int64_t)cnt[c] - e0), hi = (int)((int64_t)cnt[c + 1] - e0);
    for (int i = lo + threadIdx.x; i < hi; i += NT) {
      s_lohi[i] = (uint32_t)lo | ((uint32_t)hi << 16);
      s_col[i] = (int32_t)c;
    }
  }
  __syncthreads();
  // rank of each key in its column (keys are unique): its sorted slot
  int dst[IPT];
  int32_t dcol[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int i = u * NT + threadIdx.x;
    dst[u] = -1;
    dcol[u] = 0;
    if (i < n) {
      const uint32_t lh = s_lohi[i];
      const int lo = (int)(lh & 0xffffu), hi = (int)(lh >> 16);
      int r = 0, j = lo;
      for (; j + 4 <= hi; j += 4) {
        const uint64_t k0 = s_key[j], k1 = s_key[j + 1], k2 = s_key[j + 2], k3 = s_key[j + 3];
        r += (int)(k0 < kv[u]) + (int)(k1 < kv[u]) + (int)(k2 < kv[u]) + (int)(k3 < kv[u]);
      }
      for (; j < hi; ++j) r += (int)(s_key[j] < kv[u]);
      dst[u] = lo + r;
      dcol[u] = s_col[i];
      if (r == 0) kv[u] |= kSegHead;
    }
  }
  __syncthreads();  // every read of the unsorted chunk is done
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    if (dst[u] >= 0) {
      s_key[dst[u]] = kv[u];
      s_val[dst[u]] = vv[u];
      s_col[dst[u]] = dcol[u];
    }
  }
  __syncthreads();
  // fold: a run starts at a column's first key or where the row changes
  uint32_t rows[IPT];
  double sums[IPT];
  uint32_t mask = 0;
#pragma unroll
  for (int s = 0; s < IPT; ++s) {
    const int li = threadIdx.x * IPT + s;
    rows[s] = 0;
    sums[s] = 0.0;
    if (li < n) {
      const uint64_t key = s_key[li];
      const uint32_t row = bk.row(key);
      rows[s] = row;
      if ((key & kSegHead) || li == 0 || bk.row(s_key[li - 1]) != row) {
        double acc = (double)s_val[li];
        for (int j = li + 1; j < n; ++j) {
          const uint64_t k2 = s_key[j];
          if ((k2 & kSegHead) || bk.row(k2) != row) break;
          acc += (double)s_val[j];
        }
        sums[s] = acc;
        if (acc != 0.0) mask |= 1u << s;
      }
    }
  }
  int32_t cols[IPT];
#pragma unroll
  for (int s = 0; s < IPT; ++s) {
    const int li = threadIdx.x * IPT + s;
    cols[s] = s_col[li < n ? li : 0];
  }
  uint32_t blk_kept;
  const uint32_t excl = wg_excl_scan<NT>((uint32_t)__popc(mask), s_w, &blk_kept);
  {
    uint32_t run = excl;
#pragma unroll
    for (int s = 0; s < IPT; ++s) {
      const int li = threadIdx.x * IPT + s;
      if (li < n) s_pre[li] = run;
      run += (mask >> s) & 1u;
    }
    if (threadIdx.x == 0) s_pre[n] = blk_kept;
  }
  __syncthreads();
  {
    int64_t o = (int64_t)running + excl;
#pragma unroll
    for (int s = 0; s < IPT; ++s) {
      if ((mask >> s) & 1u) {
        ri[o] = (int32_t)rows[s];
        vo[o] = (float)sums[s];
        slot_col[o] = cols[s];
        ++o;
      }
    }
  }
  for (int64_t c = ca + threadIdx.x; c < cb; c += NT)
    cp[c] = (int32_t)(running + s_pre[(int64_t)cnt[c] - e0]);
  running += blk_kept;
  __syncthreads();
}

// One column c longer than kBatchCap: merge-sorted in global memory, then folded in blocks of
// kBatchCap keys (a run may continue past a block: read from memory).
template <int NT, typename VIN>
__device__ void batch_giant_column(const BatchKey bk, int64_t c, const uint32_t* cnt,
                                   uint64_t* __restrict__ bucket,
                                   uint64_t* __restrict__ scratch, const VIN* __restrict__ tval,
                                   int32_t* __restrict__ ri, float* __restrict__ vo,
                                   int32_t* __restrict__ slot_col, int32_t* __restrict__ cp,
                                   uint32_t& running, uint64_t* s_key, float* s_val,
                                   uint32_t* s_pre, uint32_t* s_w) {
  constexpr int IPT = kBatchCap / NT;
  constexpr int T = kBatchCap;
  const int64_t e0 = cnt[c], e1 = cnt[c + 1];
  giant_sort<NT, false>(bucket + e0, e1 - e0, scratch + e0, e0, (int32_t*)nullptr,
                        (int32_t*)nullptr, s_key);
  if (threadIdx.x == 0) cp[c] = (int32_t)running;
  for (int64_t base = e0; base < e1; base += T) {
    const int m = (int)((e1 - base) < T ? (e1 - base) : T);
    uint64_t kv[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int i = u * NT + threadIdx.x;
      kv[u] = i < m ? bucket[base + i] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int i = u * NT + threadIdx.x;
      if (i < m) {
        s_key[i] = kv[u];
        s_val[i] = batch_value<VIN>(bk, kv[u], tval);
      }
    }
    __syncthreads();
    uint32_t rows[IPT];
    double sums[IPT];
    uint32_t mask = 0;
#pragma unroll
    for (int s = 0; s < IPT; ++s) {
      const int li = threadIdx.x * IPT + s;
      rows[s] = 0;
      sums[s] = 0.0;
      if (li < m) {
        const uint64_t key = s_key[li];
        const uint32_t row = bk.row(key);
        const uint64_t pk = li > 0 ? s_key[li - 1] : (base > e0 ? bucket[base - 1] : 0ull);
        rows[s] = row;
        if ((key & kSegHead) || bk.row(pk) != row) {
          double acc = (double)s_val[li];
          int j = li + 1;
          for (; j < m; ++j) {
            const uint64_t k2 = s_key[j];
            if (bk.row(k2) != row) break;
            acc += (double)s_val[j];
          }
          if (j == m) {
            for (int64_t g = base + m; g < e1; ++g) {
              const uint64_t k2 = bucket[g];
              if (bk.row(k2) != row) break;
              acc += (double)batch_value<VIN>(bk, k2, tval);
            }
          }
          sums[s] = acc;
          if (acc != 0.0) mask |= 1u << s;
        }
      }
    }
    uint32_t blk_kept;
    const uint32_t excl = wg_excl_scan<NT>((uint32_t)__popc(mask), s_w, &blk_kept);
    int64_t o = (int64_t)running + excl;
#pragma unroll
    for (int s = 0; s < IPT; ++s) {
      if ((mask >> s) & 1u) {
        ri[o] = (int32_t)rows[s];
        vo[o] = (float)sums[s];
        slot_col[o] = (int32_t)c;
        ++o;
      }
    }
    running += blk_kept;
    __syncthreads();
  }
  (void)s_pre;
}

template <int NT, typename VIN>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_batch(BatchArgs a) {
  constexpr int kBatchFoldIPT = kBatchCap / NT;  // fold block = the sort chunk buffer
  constexpr int T = NT * kBatchFoldIPT;
  constexpr int U = 8;  // elements per thread whose loads are issued together
  __shared__ uint32_t s_cnt[kBatchMaxLdsDim + 1];
  __shared__ uint64_t s_key[kBatchCap];
  __shared__ uint32_t s_pre[T + 1];
  __shared__ int32_t s_col[T];  // column of each element of a fold chunk
  __shared__ float s_val[T];    // value of each element of a fold chunk (exact: f32 or bf16)
  __shared__ uint32_t s_w[NT / kWave + 1];
  __shared__ int64_t s_b[4];
  __shared__ int32_t s_item;
  __shared__ int32_t s_bad;

  char* wsw = a.ws + (size_t)blockIdx.x * a.ws_stride;
  uint64_t* bucket = reinterpret_cast<uint64_t*>(wsw);
  uint64_t* scratch = bucket + a.max_nnz;
  uint32_t* gcnt = reinterpret_cast<uint32_t*>(scratch + a.max_nnz);
  const VIN* vin = static_cast<const VIN*>(a.val);

  while (true) {
    if (threadIdx.x == 0) {
      const uint32_t q = atomicAdd(a.queue, 1u);
      int32_t m = -1;  // -1: queue drained
      if (q < (uint32_t)a.batch) {
        m = a.order[q];
        if (m < 0 || m >= a.batch) m = -2;  // not a matrix index: skipped
      }
      s_item = m;
      s_bad = 0;
    }
    __syncthreads();
    const int32_t b = s_item;
    if (b == -1) break;  // every workgroup leaves through here once the queue is drained
    if (b == -2) {
      __syncthreads();
      continue;
    }
    const spm_batch_item it = a.items[b];
    const int64_t n_r = it.n_rows, n_c = it.n_cols, nnz_in = it.nnz_in;
    if (!batch_item_ok(a, it)) {
      if (threadIdx.x == 0) {
        a.info[2 * (int64_t)b] = 0;
        a.info[2 * (int64_t)b + 1] = kStEinval;
      }
      __syncthreads();
      continue;
    }
    const int64_t to = it.trip_off;
    const int32_t* trow = a.row + to;
    const int32_t* tcol = a.col + to;
    const VIN* tval = vin + to;
    int32_t* cp = a.col_ptr + it.colptr_off;
    int32_t* ri = a.row_idx + to;
    float* vo = a.val_out + to;
    int32_t* rp = a.row_ptr + it.rowptr_off;
    int32_t* slot_col = a.col_t + to;  // column of each CSC slot, until the plan overwrites it
    BatchKey bk{-1};
    {
      int rb = 0, tb = 0;
      while (((int64_t)1 << rb) < n_r) ++rb;
      while (((int64_t)1 << tb) < nnz_in) ++tb;
      if (rb + tb <= 31) bk.tb = tb;
    }
    uint32_t* cnt = (n_r <= kBatchMaxLdsDim && n_c <= kBatchMaxLdsDim) ? s_cnt : gcnt;

    // ---- 1. column histogram (bounds-checked) -------------------------------------------
    for (int64_t i = threadIdx.x; i <= n_c; i += NT) cnt[i] = 0;
    __syncthreads();
    bool bad = false;
    for (int64_t t0 = threadIdx.x; t0 < nnz_in; t0 += (int64_t)NT * U) {
      int32_t r[U], c[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t t = t0 + (int64_t)u * NT;
        r[u] = t < nnz_in ? trow[t] : 0;
        c[u] = t < nnz_in ? tcol[t] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (t0 + (int64_t)u * NT < nnz_in) {
          if (r[u] >= 0 && r[u] < n_r && c[u] >= 0 && c[u] < n_c) atomicAdd(&cnt[c[u]], 1u);
          else bad = true;
        }
      }
    }
    if (bad) s_bad = 1;
    // ---- 2. inclusive scan: cnt[c] = end of column c -------------------------------------
    __syncthreads();
    wg_inclusive_scan_inplace<NT>(cnt, n_c, s_w);
    if (threadIdx.x == 0) cnt[n_c] = n_c > 0 ? cnt[n_c - 1] : 0u;
    __syncthreads();
    // ---- 3. scatter keys (row << 32 | position); counters end as column starts ------------
    for (int64_t t0 = threadIdx.x; t0 < nnz_in; t0 += (int64_t)NT * U) {
      int32_t r[U], c[U];
      uint32_t vb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t t = t0 + (int64_t)u * NT;
        r[u] = t < nnz_in ? trow[t] : -1;
        c[u] = t < nnz_in ? tcol[t] : -1;
        vb[u] = (bk.tb >= 0 && t < nnz_in) ? vin_bits(tval[t]) : 0u;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t t = t0 + (int64_t)u * NT;
        if (t < nnz_in && r[u] >= 0 && r[u] < n_r && c[u] >= 0 && c[u] < n_c) {
          const uint32_t pos = atomicSub(&cnt[c[u]], 1u) - 1u;
          bucket[pos] = bk.tb >= 0
                            ? ((uint64_t)(((uint32_t)r[u] << bk.tb) | (uint32_t)t) << 32) | vb[u]
                            : ((uint64_t)(uint32_t)r[u] << 32) | (uint32_t)t;
        }
      }
    }
    __syncthreads();
    const int64_t N = cnt[n_c];
    // ---- 4 + 5. per chunk of whole columns (at most kBatchCap keys): sort each column in
    // LDS, fold each run in binary64 from LDS, drop zeros, compact, column offsets.  A
    // column longer than kBatchCap is merge-sorted in global memory and folded in blocks.
    uint32_t running = 0;
    for (int64_t ca = 0; ca < n_c;) {
      if (threadIdx.x == 0) s_b[0] = ca + upper_bound(cnt + ca, n_c - ca + 1,
                                                       (int64_t)cnt[ca] + kBatchCap) - 1;
      __syncthreads();
      const int64_t cb = s_b[0];
      __syncthreads();
      if (cb == ca) {  // one giant column
        batch_giant_column<NT, VIN>(bk, ca, cnt, bucket, scratch, tval, ri, vo, slot_col, cp,
                                    running, s_key, s_val, s_pre, s_w);
        ca += 1;
      } else {
        batch_fold_chunk<NT, VIN>(bk, ca, cb, cnt, bucket, tval, ri, vo, slot_col, cp, running,
                                  s_key, s_val, s_col, s_pre, s_w);
        ca = cb;
      }
    }
    if (threadIdx.x == 0) cp[n_c] = (int32_t)running;
    const int64_t nnz = running;
    if (threadIdx.x == 0) {
      a.info[2 * (int64_t)b] = (int32_t)nnz;
      a.info[2 * (int64_t)b + 1] = s_bad ? kStBounds : 0;
    }
    __syncthreads();
    // ---- 6. plan: row counts, row starts, (col << 32 | slot) keys sorted per row -----------
    for (int64_t i = threadIdx.x; i <= n_r; i += NT) cnt[i] = 0;
    __syncthreads();
    for (int64_t p0 = threadIdx.x; p0 < nnz; p0 += (int64_t)NT * U) {
      int32_t r[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t p = p0 + (int64_t)u * NT;
        r[u] = p < nnz ? ri[p] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (p0 + (int64_t)u * NT < nnz) atomicAdd(&cnt[r[u]], 1u);
    }
    __syncthreads();
    wg_inclusive_scan_inplace<NT>(cnt, n_r, s_w);
    if (threadIdx.x == 0) cnt[n_r] = n_r > 0 ? cnt[n_r - 1] : 0u;
    __syncthreads();
    for (int64_t p0 = threadIdx.x; p0 < nnz; p0 += (int64_t)NT * U) {
      int32_t r[U], c[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t p = p0 + (int64_t)u * NT;
        r[u] = p < nnz ? ri[p] : 0;
        c[u] = p < nnz ? slot_col[p] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t p = p0 + (int64_t)u * NT;
        if (p < nnz) {
          const uint32_t pos = atomicSub(&cnt[r[u]], 1u) - 1u;
          bucket[pos] = ((uint64_t)(uint32_t)c[u] << 32) | (uint32_t)p;
        }
      }
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i <= n_r; i += NT) rp[i] = (int32_t)cnt[i];
    sort_segments<NT, kBatchCap, true>(bucket, cnt, 0, n_r, scratch, a.col_t + to, a.perm + to,
                                       s_key, s_pre, &s_b[0]);
    __syncthreads();
  }
}

// Forward and adjoint of every matrix, after k_batch.  nnz comes from info[2b], written by
// k_batch for the same matrix.  FULL (k == 4 * GW, aligned rows) is chosen on the host, so
// each instantiation holds only the registers of its own path.
template <int NT, typename XT, typename ACC, int GW, bool FULL>
__global__ __launch_bounds__(NT) void k_batch_spmm(BatchArgs a) {
  __shared__ int32_t s_item;
  const XT* Xa = static_cast<const XT*>(a.X);
  const XT* Ga = static_cast<const XT*>(a.Gm);
  const int lg = threadIdx.x & (GW - 1);
  const int64_t groups = NT / GW;
  const int64_t gid = threadIdx.x / GW;
  while (true) {
    if (threadIdx.x == 0) {
      const uint32_t q = atomicAdd(a.queue + 1, 1u);
      int32_t m = -1;  // -1: queue drained
      if (q < (uint32_t)a.batch) {
        m = a.order[q];
        if (m < 0 || m >= a.batch) m = -2;  // not a matrix index: skipped
      }
      s_item = m;
    }
    __syncthreads();
    const int32_t b = s_item;
    __syncthreads();  // every thread has read s_item before thread 0 takes the next one
    if (b == -1) break;  // every workgroup leaves through here once the queue is drained
    if (b == -2) continue;
    const spm_batch_item it = a.items[b];
    if (!batch_item_ok(a, it)) continue;
    const int64_t n_r = it.n_rows, n_c = it.n_cols;
    int64_t nnz = a.info[2 * (int64_t)b];
    nnz = nnz < 0 ? 0 : (nnz > it.nnz_in ? it.nnz_in : nnz);
    const int64_t to = it.trip_off;
    const int32_t* cp = a.col_ptr + it.colptr_off;
    const int32_t* ri = a.row_idx + to;
    const float* vo = a.val_out + to;
    const int32_t* rp = a.row_ptr + it.rowptr_off;
    const XT* Xb = Xa + it.x_off;
    const XT* Gb = Ga + it.g_off;
    // ---- forward Y = A.X --------------------------------------------------------------
    for (int64_t r = gid; r < n_r; r += groups) {
      if constexpr (FULL)
        spmm_row_full<float, XT, ACC, GW>(r, lg, n_c, nnz, rp, a.col_t + to, a.perm + to, vo,
                                          Xb, a.k, a.Y + it.g_off, a.k, false);
      else
        spmm_row<float, XT, ACC, GW, false>(r, lg, a.k, n_c, nnz, rp, a.col_t + to,
                                            a.perm + to, vo, Xb, a.k, a.xal != 0,
                                            a.Y + it.g_off, a.k, false, a.yal != 0);
    }
    // ---- adjoint dX, dval ---------------------------------------------------------------
    for (int64_t c = gid; c < n_c; c += groups) {
      const int64_t p0 = cp[c], p1 = cp[c + 1];
      if constexpr (FULL)
        spmm_col_bwd_full<float, XT, XT, ACC, GW>(c, p0, p1, lg, n_r, ri, vo, Gb, a.k, Xb, a.k,
                                              a.dX + it.x_off, a.k, false, a.dval + to, false);
      else
        spmm_col_bwd<float, XT, XT, ACC, GW, false>(c, p0, p1, lg, a.k, n_r, ri, vo, Gb, a.k,
                                                a.xal != 0, Xb, a.k, a.xal != 0,
                                                a.dX + it.x_off, a.k, false, a.yal != 0,
                                                a.dval + to, false);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Flat products.  Matrices of the batch run concurrently by the dozen on every XCD, so their
// dense rows come from MALL / HBM, not from one XCD's L2; the products are then best run as
// one grid over all rows (forward) or all columns (adjoint) of all matrices, at the
// occupancy of the single-matrix kernels.  k_batch_prefix lays out the rows and columns in
// schedule order; k_batch_flat hands out chunks of consecutive rows (columns).  Every row
// (column) is computed by the same device function as in the per-matrix kernels.
// ------------------------------------------------------------------------------------------

// Inclusive scan of one int64 per thread across the workgroup; s_w holds NT/64 + 1 words.
template <int NT>
__device__ __forceinline__ int64_t wg_incl_scan_i64(int64_t x, int64_t* s_w) {
  constexpr int NW = NT / kWave;
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) s_w[wave_id()] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int w = 0; w < NW; ++w) {
      const int64_t t = s_w[w];
      s_w[w] = run;
      run += t;
    }
    s_w[NW] = run;
  }
  __syncthreads();
  const int64_t r = x + s_w[wave_id()];
  __syncthreads();
  return r;
}

// rpre[q] / cpre[q] = rows / columns of the valid matrices order[0 .. q), q = 0 .. batch.
// One workgroup.
template <int NT>
__global__ __launch_bounds__(NT) void k_batch_prefix(BatchArgs a, int64_t* __restrict__ rpre,
                                                     int64_t* __restrict__ cpre) {
  __shared__ int64_t s_w[NT / kWave + 1];
  int64_t rc = 0, cc = 0;
  if (threadIdx.x == 0) {
    rpre[0] = 0;
    cpre[0] = 0;
  }
  for (int64_t base = 0; base < a.batch; base += NT) {
    const int64_t q = base + threadIdx.x;
    int64_t r = 0, c = 0;
    if (q < a.batch) {
      const int32_t m = a.order[q];
      if (m >= 0 && m < a.batch) {
        const spm_batch_item it = a.items[m];
        if (batch_item_ok(a, it)) {
          r = it.n_rows;
          c = it.n_cols;
        }
      }
    }
    const int64_t ri = wg_incl_scan_i64<NT>(r, s_w) + rc;
    const int64_t ci = wg_incl_scan_i64<NT>(c, s_w) + cc;
    if (q < a.batch) {
      rpre[q + 1] = ri;
      cpre[q + 1] = ci;
    }
    // carry: the last thread's inclusive value, shared through s_w
    if (threadIdx.x == NT - 1) {
      s_w[0] = ri;
      s_w[1] = ci;
    }
    __syncthreads();
    rc = s_w[0];
    cc = s_w[1];
    __syncthreads();
  }
}

// tab[t] = the schedule slot q whose rows (columns) hold the start of chunk t, that is
// pre[q] <= t * chunk < pre[q + 1], for both prefixes.  One thread per slot.
// What the products need of schedule slot q, in one 64-byte record per direction: the rows
// (forward) or columns (adjoint) of the schedule before it and through it, the matrix's
// offsets and sizes, and its nnz from the grouping launch.
struct BatchSlot {
  int64_t lo, hi;
  int64_t trip_off, ptr_off, x_off, g_off;
  int32_t n_r, n_c, nnz, q;
};
static_assert(sizeof(BatchSlot) == 64, "one record per 64 bytes");

// Also writes the slot records (rslot: rows and row_ptr, cslot: columns and col_ptr) and
// clears the per-XCD chunk counters of the two product launches (2 * kXcds words).
template <int NT>
__global__ __launch_bounds__(NT) void k_batch_tab(BatchArgs a, const int64_t* __restrict__ rpre,
                                                  const int64_t* __restrict__ cpre,
                                                  int64_t chunk, int64_t cap,
                                                  int32_t* __restrict__ rtab,
                                                  int32_t* __restrict__ ctab,
                                                  uint32_t* __restrict__ xcd_next,
                                                  BatchSlot* __restrict__ rslot,
                                                  BatchSlot* __restrict__ cslot) {
  const int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (q < 2 * kXcds) xcd_next[q] = 0;
  if (q >= a.batch) return;
  {
    BatchSlot r{}, c{};
    const int32_t m = a.order[q];
    if (m >= 0 && m < a.batch) {
      const spm_batch_item it = a.items[m];
      int64_t nnz = a.info[2 * (int64_t)m];
      nnz = nnz < 0 ? 0 : (nnz > it.nnz_in ? it.nnz_in : nnz);
      r.trip_off = c.trip_off = it.trip_off;
      r.x_off = c.x_off = it.x_off;
      r.g_off = c.g_off = it.g_off;
      r.n_r = c.n_r = it.n_rows;
      r.n_c = c.n_c = it.n_cols;
      r.nnz = c.nnz = (int32_t)nnz;
      r.ptr_off = it.rowptr_off;
      c.ptr_off = it.colptr_off;
    }
    r.lo = rpre[q];
    r.hi = rpre[q + 1];
    c.lo = cpre[q];
    c.hi = cpre[q + 1];
    r.q = c.q = (int32_t)q;
    rslot[q] = r;
    cslot[q] = c;
  }
  for (int side = 0; side < 2; ++side) {
    const int64_t* pre = side == 0 ? rpre : cpre;
    int32_t* tab = side == 0 ? rtab : ctab;
    const int64_t t0 = (pre[q] + chunk - 1) / chunk, t1 = (pre[q + 1] + chunk - 1) / chunk;
    for (int64_t t = t0; t < t1 && t < cap; ++t) tab[t] = (int32_t)q;
  }
}

// FWD: rows of all matrices (pre = rpre), forward product.  !FWD: columns (pre = cpre),
// adjoint.  A chunk is kPerGroup rows (columns) per group.  The chunks are cut into one
// contiguous range per XCD (workgroup b runs on XCD b mod 8), and the workgroups of an XCD
// take its chunks in order from a counter of its own: each XCD then has about (its
// workgroups x chunk) consecutive rows in flight, a few matrices whose dense rows stay in its
// L2.
constexpr int kBatchFlatPerGroup = 2;
template <int NT, typename XT, typename ACC, int GW, bool FULL, bool FWD>
__global__ __launch_bounds__(NT) void k_batch_flat(BatchArgs a, const int64_t* __restrict__ pre,
                                                   const int32_t* __restrict__ tab,
                                                   uint32_t* __restrict__ xcd_next,
                                                   const BatchSlot* __restrict__ slots) {
  constexpr int64_t kGroups = NT / GW;
  constexpr int64_t kChunk = kGroups * kBatchFlatPerGroup;
  __shared__ int64_t s_next;
  __shared__ BatchSlot s_slot[2];  // the record of the current chunk's start, and the next's
  const XT* Xa = static_cast<const XT*>(a.X);
  const XT* Ga = static_cast<const XT*>(a.Gm);
  const int lg = threadIdx.x & (GW - 1);
  const int64_t gid = threadIdx.x / GW;
  const int64_t total = pre[a.batch];
  const int64_t nchunks = (total + kChunk - 1) / kChunk;
  const int64_t x = blockIdx.x % kXcds;
  const int64_t c_lo = nchunks * x / kXcds, c_hi = nchunks * (x + 1) / kXcds;
  // thread 0 takes the next chunk and loads its slot record while the current one is computed
  auto fetch = [&](int buf) {
    const int64_t ch = c_lo + (int64_t)atomicAdd(&xcd_next[x], 1u);
    s_next = ch;
    if (ch < c_hi) {
      int64_t q = tab[ch];
      q = q < 0 ? 0 : (q >= a.batch ? a.batch - 1 : q);
      s_slot[buf] = slots[q];
    }
  };
  if (threadIdx.x == 0) fetch(0);
  __syncthreads();
  int64_t chunk = s_next;
  int buf = 0;
  while (chunk < c_hi) {  // the same for every thread of the workgroup
    __syncthreads();  // s_next and the other record were read before thread 0 rewrites them
    if (threadIdx.x == 0) fetch(buf ^ 1);
    for (int j = 0; j < kBatchFlatPerGroup; ++j) {
      const int64_t g = chunk * kChunk + (int64_t)j * kGroups + gid;
      if (g >= total) break;
      BatchSlot S = s_slot[buf];
      // a row past the record's matrix (the chunk runs into later ones): walk the records
      for (int64_t q = (int64_t)S.q + 1; g >= S.hi && q < a.batch; ++q) S = slots[q];
      if (g < S.lo || g >= S.hi) continue;  // (only for malformed schedules)
      const int64_t e = g - S.lo;  // row (column) within the matrix
      const int64_t to = S.trip_off;
      const int64_t nnz = S.nnz;
      const float* vo = a.val_out + to;
      const XT* Xb = Xa + S.x_off;
      if constexpr (FWD) {
        const int32_t* rp = a.row_ptr + S.ptr_off;
        if constexpr (FULL)
          spmm_row_full<float, XT, ACC, GW>(e, lg, S.n_c, nnz, rp, a.col_t + to, a.perm + to,
                                            vo, Xb, a.k, a.Y + S.g_off, a.k, false);
        else
          spmm_row<float, XT, ACC, GW, false>(e, lg, a.k, S.n_c, nnz, rp, a.col_t + to,
                                              a.perm + to, vo, Xb, a.k, a.xal != 0,
                                              a.Y + S.g_off, a.k, false, a.yal != 0);
      } else {
        const int32_t* cp = a.col_ptr + S.ptr_off;
        const int32_t* ri = a.row_idx + to;
        const XT* Gb = Ga + S.g_off;
        const int64_t p0 = cp[e], p1 = cp[e + 1];
        if constexpr (FULL)
          spmm_col_bwd_full<float, XT, XT, ACC, GW>(e, p0, p1, lg, S.n_r, ri, vo, Gb, a.k, Xb,
                                                a.k, a.dX + S.x_off, a.k, false, a.dval + to,
                                                false);
        else
          spmm_col_bwd<float, XT, XT, ACC, GW, false>(e, p0, p1, lg, a.k, S.n_r, ri, vo, Gb,
                                                  a.k, a.xal != 0, Xb, a.k, a.xal != 0,
                                                  a.dX + S.x_off, a.k, false, a.yal != 0,
                                                  a.dval + to, false);
      }
    }
    __syncthreads();
    chunk = s_next;
    buf ^= 1;
  }
}

}  // namespace spm
