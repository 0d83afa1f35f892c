// Batched path: launches that assemble, plan, multiply forward and backward many
// independent matrices.
//   k_batch       assembly and plan: a persistent workgroup takes whole matrices from a
//                 device queue (in the order the caller gives, largest first) and keeps the
//                 matrix's per-column / per-row counters in LDS and its keys in a
//                 per-workgroup slice of the workspace;
//   k_batch_prefix, k_batch_flat
//                 forward over all rows and adjoint over all columns of all matrices, one
//                 grid each, at the occupancy of the single-matrix kernels;
//   k_batch_spmm  the same products one workgroup per matrix, when the workspace cannot hold
//                 the prefixes the flat launches need.
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
  static_assert(T == 8 * NT, "the column scan of a fold block takes 8 entries per thread");
  constexpr int U = 8;  // elements per thread whose loads are issued together
  __shared__ uint32_t s_cnt[kBatchMaxLdsDim + 1];
  __shared__ uint64_t s_key[kBatchCap];
  __shared__ uint32_t s_pre[T + 1];
  __shared__ int32_t s_col[T];  // column of each element of a fold block
  __shared__ float s_val[T];    // value of each element of a fold block (exact: f32 or bf16)
  __shared__ uint64_t s_prev;   // the key before the fold block
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
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t t = t0 + (int64_t)u * NT;
        r[u] = t < nnz_in ? trow[t] : -1;
        c[u] = t < nnz_in ? tcol[t] : -1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t t = t0 + (int64_t)u * NT;
        if (t < nnz_in && r[u] >= 0 && r[u] < n_r && c[u] >= 0 && c[u] < n_c) {
          const uint32_t pos = atomicSub(&cnt[c[u]], 1u) - 1u;
          bucket[pos] = ((uint64_t)(uint32_t)r[u] << 32) | (uint32_t)t;
        }
      }
    }
    __syncthreads();
    const int64_t N = cnt[n_c];
    // ---- 4. sort each column's keys --------------------------------------------------------
    sort_segments<NT, kBatchCap, false>(bucket, cnt, 0, n_c, scratch, (int32_t*)nullptr,
                                        (int32_t*)nullptr, s_key, s_pre, &s_b[0]);
    __syncthreads();
    // ---- 5. fold, drop zeros, compact, column offsets --------------------------------------
    // (the column of each element comes from a max-scan over the column starts in the block)
    uint32_t running = 0;
    for (int64_t base = 0; base < N || base == 0; base += T) {
      const int cntb = (int)((N - base) < T ? (N - base) : T);
      {
        uint64_t kv[kBatchFoldIPT];
#pragma unroll
        for (int u = 0; u < kBatchFoldIPT; ++u) {
          const int li = u * NT + threadIdx.x;
          kv[u] = li < cntb ? bucket[base + li] : 0ull;
        }
        // the values of the block's elements, gathered at once
        float vv[kBatchFoldIPT];
#pragma unroll
        for (int u = 0; u < kBatchFoldIPT; ++u) {
          const int li = u * NT + threadIdx.x;
          vv[u] = li < cntb ? to_acc<float>(tval[(uint32_t)kv[u]]) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kBatchFoldIPT; ++u) {
          const int li = u * NT + threadIdx.x;
          if (li < cntb) {
            s_key[li] = kv[u];
            s_val[li] = vv[u];
          }
          s_col[li] = -1;
        }
        if (threadIdx.x == 0) s_prev = base > 0 ? bucket[base - 1] : 0ull;
      }
      if (threadIdx.x == 0) {
        const bool last = base + T >= N;
        s_b[1] = lower_bound(cnt, n_c + 1, base);
        s_b[2] = last ? n_c + 1 : lower_bound(cnt, n_c + 1, base + T);
      }
      __syncthreads();
      for (int64_t c = s_b[1] + threadIdx.x; c < s_b[2] && c < n_c; c += NT) {
        const int64_t p = (int64_t)cnt[c] - base;
        if (p >= 0 && p < cntb) atomicMax(&s_col[p], (int32_t)c);
      }
      __syncthreads();
      wg_max_scan8<NT>(s_col, (int32_t)(s_b[1] > 0 ? s_b[1] - 1 : 0),
                       reinterpret_cast<int32_t*>(s_w));
      __syncthreads();
      // fold: a run starts at a column's first key or where the row changes; its head sums
      // the run left to right in binary64 (from LDS, then from memory past the block)
      uint32_t rows[kBatchFoldIPT];
      double sums[kBatchFoldIPT];
      uint32_t mask = 0;
#pragma unroll
      for (int s = 0; s < kBatchFoldIPT; ++s) {
        const int li = threadIdx.x * kBatchFoldIPT + s;
        rows[s] = 0;
        sums[s] = 0.0;
        if (li < cntb) {
          const uint64_t key = s_key[li];
          const uint32_t row = key_row(key);
          const uint64_t pk = li > 0 ? s_key[li - 1] : s_prev;
          rows[s] = row;
          if ((key & kSegHead) || key_row(pk) != row) {
            double acc = (double)s_val[li];
            int j = li + 1;
            for (; j < cntb; ++j) {
              const uint64_t k2 = s_key[j];
              if ((k2 & kSegHead) || key_row(k2) != row) break;
              acc += (double)s_val[j];
            }
            if (j == cntb) {
              for (int64_t g = base + cntb; g < N; ++g) {
                const uint64_t k2 = bucket[g];
                if ((k2 & kSegHead) || key_row(k2) != row) break;
                acc += to_acc<double>(tval[(uint32_t)k2]);
              }
            }
            sums[s] = acc;
            if (acc != 0.0) mask |= 1u << s;
          }
        }
      }
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
        if (threadIdx.x == 0) s_pre[cntb] = blk_kept;
      }
      __syncthreads();
      {
        int64_t o = (int64_t)running + excl;
#pragma unroll
        for (int s = 0; s < kBatchFoldIPT; ++s) {
          if ((mask >> s) & 1u) {
            ri[o] = (int32_t)rows[s];
            vo[o] = (float)sums[s];
            slot_col[o] = s_col[threadIdx.x * kBatchFoldIPT + s];
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
// Also clears the per-XCD chunk counters of the two product launches (2 * kXcds words).
template <int NT>
__global__ __launch_bounds__(NT) void k_batch_tab(BatchArgs a, const int64_t* __restrict__ rpre,
                                                  const int64_t* __restrict__ cpre,
                                                  int64_t chunk, int64_t cap,
                                                  int32_t* __restrict__ rtab,
                                                  int32_t* __restrict__ ctab,
                                                  uint32_t* __restrict__ xcd_next) {
  const int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (q < 2 * kXcds) xcd_next[q] = 0;
  if (q >= a.batch) return;
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
                                                   uint32_t* __restrict__ xcd_next) {
  constexpr int64_t kGroups = NT / GW;
  constexpr int64_t kChunk = kGroups * kBatchFlatPerGroup;
  __shared__ int64_t s_chunk;
  const XT* Xa = static_cast<const XT*>(a.X);
  const XT* Ga = static_cast<const XT*>(a.Gm);
  const int lg = threadIdx.x & (GW - 1);
  const int64_t gid = threadIdx.x / GW;
  const int64_t total = pre[a.batch];
  const int64_t nchunks = (total + kChunk - 1) / kChunk;
  const int64_t x = blockIdx.x % kXcds;
  const int64_t c_lo = nchunks * x / kXcds, c_hi = nchunks * (x + 1) / kXcds;
  while (true) {
    if (threadIdx.x == 0) s_chunk = c_lo + (int64_t)atomicAdd(&xcd_next[x], 1u);
    __syncthreads();
    const int64_t chunk = s_chunk;
    __syncthreads();  // s_chunk is read before thread 0 rewrites it
    if (chunk >= c_hi) break;  // the same for every thread of the workgroup
    int64_t q = tab[chunk];
    q = q < 0 ? 0 : (q >= a.batch ? a.batch - 1 : q);
    for (int j = 0; j < kBatchFlatPerGroup; ++j) {
      const int64_t g = chunk * kChunk + (int64_t)j * kGroups + gid;
      if (g >= total) break;
      while (q + 1 < a.batch && pre[q + 1] <= g) ++q;  // g < total = pre[batch]
      const spm_batch_item it = a.items[a.order[q]];
      int64_t nnz = a.info[2 * (int64_t)a.order[q]];
      nnz = nnz < 0 ? 0 : (nnz > it.nnz_in ? it.nnz_in : nnz);
      const int64_t e = g - pre[q];  // row (column) within the matrix
      const int64_t to = it.trip_off;
      const int64_t n_r = it.n_rows, n_c = it.n_cols;
      const float* vo = a.val_out + to;
      const XT* Xb = Xa + it.x_off;
      if constexpr (FWD) {
        const int32_t* rp = a.row_ptr + it.rowptr_off;
        if constexpr (FULL)
          spmm_row_full<float, XT, ACC, GW>(e, lg, n_c, nnz, rp, a.col_t + to, a.perm + to, vo,
                                            Xb, a.k, a.Y + it.g_off, a.k, false);
        else
          spmm_row<float, XT, ACC, GW, false>(e, lg, a.k, n_c, nnz, rp, a.col_t + to,
                                              a.perm + to, vo, Xb, a.k, a.xal != 0,
                                              a.Y + it.g_off, a.k, false, a.yal != 0);
      } else {
        const int32_t* cp = a.col_ptr + it.colptr_off;
        const int32_t* ri = a.row_idx + to;
        const XT* Gb = Ga + it.g_off;
        const int64_t p0 = cp[e], p1 = cp[e + 1];
        if constexpr (FULL)
          spmm_col_bwd_full<float, XT, XT, ACC, GW>(e, p0, p1, lg, n_r, ri, vo, Gb, a.k, Xb, a.k,
                                                a.dX + it.x_off, a.k, false, a.dval + to,
                                                false);
        else
          spmm_col_bwd<float, XT, XT, ACC, GW, false>(e, p0, p1, lg, a.k, n_r, ri, vo, Gb, a.k,
                                                  a.xal != 0, Xb, a.k, a.xal != 0,
                                                  a.dX + it.x_off, a.k, false, a.yal != 0,
                                                  a.dval + to, false);
      }
    }
  }
}

}  // namespace spm
