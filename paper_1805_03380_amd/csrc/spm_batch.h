// Batched path: two persistent launches assemble, plan, multiply forward and backward many
// independent matrices.  In each, a workgroup takes whole matrices from a device queue (in
// the order the caller gives, largest first) and runs one matrix at a time.
//   k_batch       assembly and plan, with the matrix's per-column / per-row counters in LDS
//                 and its keys in a per-workgroup slice of the workspace (one matrix's
//                 working set stays in the L2 of the XCD that runs it);
//   k_batch_spmm  forward and adjoint.  It needs no LDS and few registers, so many more
//                 workgroups share a CU than the grouping phases allow, which hides the
//                 latency of the dense-row gathers.
// The phases call the same device functions as the per-matrix kernels (segment sort, fold,
// spmm_row, spmm_col_bwd), so the results are bitwise equal to the per-matrix entry points.
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

template <int NT, typename VIN>
__global__ __launch_bounds__(NT) void k_batch(BatchArgs a) {
  constexpr int kBatchFoldIPT = kBatchCap / NT;  // fold block = the sort chunk buffer
  constexpr int T = NT * kBatchFoldIPT;
  __shared__ uint32_t s_cnt[kBatchMaxLdsDim + 1];
  __shared__ uint64_t s_key[kBatchCap];
  __shared__ uint32_t s_pre[T + 1];
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
    uint32_t* cnt = (n_r <= kBatchMaxLdsDim && n_c <= kBatchMaxLdsDim) ? s_cnt : gcnt;

    // ---- 1. column histogram (bounds-checked) -------------------------------------------
    for (int64_t i = threadIdx.x; i <= n_c; i += NT) cnt[i] = 0;
    __syncthreads();
    bool bad = false;
    for (int64_t t = threadIdx.x; t < nnz_in; t += NT) {
      const int32_t r = trow[t], c = tcol[t];
      if (r >= 0 && r < n_r && c >= 0 && c < n_c) atomicAdd(&cnt[c], 1u);
      else bad = true;
    }
    if (bad) s_bad = 1;
    // ---- 2. inclusive scan: cnt[c] = end of column c -------------------------------------
    __syncthreads();
    wg_inclusive_scan_inplace<NT>(cnt, n_c, s_w);
    if (threadIdx.x == 0) cnt[n_c] = n_c > 0 ? cnt[n_c - 1] : 0u;
    __syncthreads();
    // ---- 3. scatter keys (row << 32 | position); counters end as column starts ------------
    for (int64_t t = threadIdx.x; t < nnz_in; t += NT) {
      const int32_t r = trow[t], c = tcol[t];
      if (r >= 0 && r < n_r && c >= 0 && c < n_c) {
        const uint32_t pos = atomicSub(&cnt[c], 1u) - 1u;
        bucket[pos] = ((uint64_t)(uint32_t)r << 32) | (uint32_t)t;
      }
    }
    __syncthreads();
    const int64_t N = cnt[n_c];
    // ---- 4. sort each column's keys --------------------------------------------------------
    sort_segments<NT, kBatchCap, false>(bucket, cnt, 0, n_c, scratch, (int32_t*)nullptr,
                                        (int32_t*)nullptr, s_key, s_pre, &s_b[0]);
    __syncthreads();
    // ---- 5. fold, drop zeros, compact, column offsets --------------------------------------
    uint32_t running = 0;
    for (int64_t base = 0; base < N || base == 0; base += T) {
      const int cntb = (int)((N - base) < T ? (N - base) : T);
      for (int li = threadIdx.x; li < cntb; li += NT) s_key[li] = bucket[base + li];
      __syncthreads();
      uint32_t rows[kBatchFoldIPT];
      double sums[kBatchFoldIPT];
      const uint32_t mask = fold_tile<NT, kBatchFoldIPT, VIN>(bucket, s_key, base, cntb, N, tval,
                                                               rows, sums);
      uint32_t blk_kept;
      const uint32_t excl = wg_excl_scan<NT>((uint32_t)__popc(mask), s_w, &blk_kept);
      {
        uint32_t run = excl;
#pragma unroll
        for (int s = 0; s < kBatchFoldIPT; ++s) {
          const int li = threadIdx.x * kBatchFoldIPT + s;
          if (li < cntb) s_pre[li] = run;
          run += (mask >> s) & 1u;
        }
        if (threadIdx.x == 0) {
          s_pre[cntb] = blk_kept;
          const bool last = base + T >= N;
          s_b[1] = lower_bound(cnt, n_c + 1, base);
          s_b[2] = last ? n_c + 1 : lower_bound(cnt, n_c + 1, base + T);
        }
      }
      __syncthreads();
      {
        int64_t o = (int64_t)running + excl;
#pragma unroll
        for (int s = 0; s < kBatchFoldIPT; ++s) {
          if ((mask >> s) & 1u) {
            ri[o] = (int32_t)rows[s];
            vo[o] = (float)sums[s];
            ++o;
          }
        }
      }
      for (int64_t c = s_b[1] + threadIdx.x; c < s_b[2]; c += NT) {
        int64_t p = (int64_t)cnt[c] - base;
        if (p > cntb) p = cntb;
        cp[c] = (int32_t)(running + s_pre[p]);
      }
      running += blk_kept;
      __syncthreads();
      if (base + T >= N) break;
    }
    const int64_t nnz = running;
    if (threadIdx.x == 0) {
      a.info[2 * (int64_t)b] = (int32_t)nnz;
      a.info[2 * (int64_t)b + 1] = s_bad ? kStBounds : 0;
    }
    __syncthreads();
    // ---- 6. plan: row counts, row starts, (col << 32 | slot) keys sorted per row -----------
    for (int64_t i = threadIdx.x; i <= n_r; i += NT) cnt[i] = 0;
    __syncthreads();
    for (int64_t p = threadIdx.x; p < nnz; p += NT) atomicAdd(&cnt[ri[p]], 1u);
    __syncthreads();
    wg_inclusive_scan_inplace<NT>(cnt, n_r, s_w);
    if (threadIdx.x == 0) cnt[n_r] = n_r > 0 ? cnt[n_r - 1] : 0u;
    __syncthreads();
    for (int64_t p0 = (int64_t)threadIdx.x * 4; p0 < nnz; p0 += (int64_t)NT * 4) {
      int64_t c = upper_bound(cp, n_c + 1, p0) - 1;
      const int64_t p1 = (p0 + 4 < nnz) ? p0 + 4 : nnz;
      for (int64_t p = p0; p < p1; ++p) {
        while (c + 1 < n_c && (int64_t)cp[c + 1] <= p) ++c;
        const int32_t r = ri[p];
        const uint32_t pos = atomicSub(&cnt[r], 1u) - 1u;
        bucket[pos] = ((uint64_t)c << 32) | (uint32_t)p;
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
        spmm_col_bwd_full<float, XT, ACC, GW>(c, p0, p1, lg, n_r, ri, vo, Gb, a.k, Xb, a.k,
                                              a.dX + it.x_off, a.k, false, a.dval + to, false);
      else
        spmm_col_bwd<float, XT, ACC, GW, false>(c, p0, p1, lg, a.k, n_r, ri, vo, Gb, a.k,
                                                a.xal != 0, Xb, a.k, a.xal != 0,
                                                a.dX + it.x_off, a.k, false, a.yal != 0,
                                                a.dval + to, false);
    }
  }
}

}  // namespace spm
