// COO -> CSC assembly and the row index ("plan") of a CSC pattern: gfx950 kernels.
//
// Assembly (Section 3.2 COO -> Section 3.1 CSC, duplicates accumulate as the += update of
// Fig. 1, locations ordered by the column-major index of Section 3.3):
//   k_col_hist    bounds check of every triplet, per-column triplet counts
//   k_scan_excl   exclusive scan of the counts -> start of each column's bucket
//   k_col_scatter each triplet's key (row << 32 | input position) into its column's bucket
//   k_segsort     each bucket sorted by key, i.e. by (row, input position); the smallest key
//                 of every bucket is tagged so that later passes see column boundaries
//   k_fold        runs of equal (column, row) folded left to right in input order in
//                 binary64, zero sums dropped, survivors compacted through a single-pass
//                 chained scan; also writes the column offsets and nnz_out
// Sorting by (row, input position) inside a column is what makes the fold order the input
// order, so the result does not depend on how the scatter's atomics interleave.
//
// Plan (structural transpose of the pattern, used by the forward product):
//   k_plan_hist, k_scan_excl, k_row_scatter, k_segsort (keys col << 32 | CSC slot).
#pragma once

#include "spm_device.h"

namespace spm {

constexpr uint64_t kSegHead = 1ull << 63;  // tag on the smallest key of each bucket
constexpr int32_t kStEinval = 1;
constexpr int32_t kStBounds = 2;

__device__ __forceinline__ void set_status(int32_t* info, int32_t code) {
  atomicCAS(info + 1, 0, code);  // the first error reported wins
}

__device__ __forceinline__ uint32_t key_row(uint64_t key) {
  return (uint32_t)(key >> 32) & 0x7fffffffu;
}

// ------------------------------------------------------------------------------------------
// Fill two regions with zeros (workspace counters / look-back states, and the info words).
// ------------------------------------------------------------------------------------------
__global__ void k_zero2(uint32_t* __restrict__ a, int64_t na, uint32_t* __restrict__ b,
                        int64_t nb) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na; i += stride) a[i] = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += stride) b[i] = 0;
}

// ------------------------------------------------------------------------------------------
// K1: bounds check + column histogram.  Four triplets per thread per sweep, coalesced.
// ------------------------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void k_col_hist(const int32_t* __restrict__ row,
                                                 const int32_t* __restrict__ col, int64_t nnz,
                                                 int32_t n_rows, int32_t n_cols,
                                                 uint32_t* __restrict__ colcnt,
                                                 int32_t* __restrict__ info) {
  constexpr int U = 4;
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * NT * U;
  for (int64_t base = (int64_t)blockIdx.x * NT * U; base < nnz; base += stride) {
    int32_t r[U], c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * NT + threadIdx.x;
      r[u] = (i < nnz) ? row[i] : 0;
      c[u] = (i < nnz) ? col[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * NT + threadIdx.x;
      if (i < nnz) {
        if ((uint32_t)r[u] < (uint32_t)n_rows && (uint32_t)c[u] < (uint32_t)n_cols)
          atomicAdd(&colcnt[c[u]], 1u);
        else
          bad = true;
      }
    }
  }
  if (bad) set_status(info, kStBounds);
}

// ------------------------------------------------------------------------------------------
// Single-pass exclusive scan of n uint32 counts: out[i] = sum in[0..i), out[n] = total.
// Tiles of NT*IPT, decoupled look-back across tiles.
// ------------------------------------------------------------------------------------------
template <int NT, int IPT>
__global__ __launch_bounds__(NT) void k_scan_excl(const uint32_t* __restrict__ in, int64_t n,
                                                  int32_t* __restrict__ out,
                                                  uint64_t* __restrict__ state,
                                                  uint32_t* __restrict__ ticket) {
  constexpr int T = NT * IPT;
  __shared__ uint32_t s_v[T];
  __shared__ uint32_t s_w[NT / kWave + 1];
  __shared__ int64_t s_t;
  __shared__ uint64_t s_off;
  if (threadIdx.x == 0) s_t = atomicAdd(ticket, 1u);
  __syncthreads();
  const int64_t t = s_t;
  const int64_t ntiles = n > 0 ? (n + T - 1) / T : 1;
  if (t >= ntiles) return;
  const int64_t base = t * T;
#pragma unroll
  for (int s = 0; s < IPT; ++s) {
    const int64_t i = base + s * NT + threadIdx.x;
    s_v[s * NT + threadIdx.x] = (i < n) ? in[i] : 0u;
  }
  __syncthreads();
  uint32_t v[IPT];
  uint32_t sum = 0;
#pragma unroll
  for (int s = 0; s < IPT; ++s) {
    v[s] = s_v[threadIdx.x * IPT + s];
    sum += v[s];
  }
  uint32_t total;
  const uint32_t excl = wg_excl_scan<NT>(sum, s_w, &total);
  if (threadIdx.x < kWave) {
    uint64_t prefix = 0;
    if (t == 0) {
      if (threadIdx.x == 0) lb_publish(state, kLbPre | total);
    } else {
      if (threadIdx.x == 0) lb_publish(state + t, kLbAgg | total);
      prefix = lookback_exclusive(state, t);
      if (threadIdx.x == 0) lb_publish(state + t, kLbPre | (prefix + total));
    }
    if (threadIdx.x == 0) s_off = prefix;
  }
  uint32_t run = excl;
#pragma unroll
  for (int s = 0; s < IPT; ++s) {
    s_v[threadIdx.x * IPT + s] = run;
    run += v[s];
  }
  __syncthreads();
  const uint64_t off = s_off;
#pragma unroll
  for (int s = 0; s < IPT; ++s) {
    const int64_t i = base + s * NT + threadIdx.x;
    if (i < n) out[i] = (int32_t)(off + s_v[s * NT + threadIdx.x]);
  }
  if (t == ntiles - 1 && threadIdx.x == 0) out[n] = (int32_t)(off + total);
}

// ------------------------------------------------------------------------------------------
// first[t] = the first index c in [0, n] with starts[c] >= t*T, for every tile t with
// t*T <= starts[n].  One thread per c writes the tiles whose boundary falls in
// (starts[c-1], starts[c]]; this replaces per-tile binary searches (chains of dependent
// global loads) in the sort and fold kernels.
// ------------------------------------------------------------------------------------------
__global__ void k_tile_first(const int32_t* __restrict__ starts, int64_t n, int64_t T,
                             int64_t max_tiles, int32_t* __restrict__ first) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= n; c += stride) {
    const int64_t lo = (c == 0) ? -1 : (int64_t)starts[c - 1];
    const int64_t hi = starts[c];
    int64_t t = (lo < 0) ? 0 : lo / T + 1;
    int64_t t_end = hi / T;
    if (t_end > max_tiles) t_end = max_tiles;
    for (; t <= t_end; ++t) first[t] = (int32_t)c;
  }
}

// ------------------------------------------------------------------------------------------
// K2: scatter each in-range triplet's key into its column's bucket.  The per-column counter
// counts down, so it is zero again afterwards; slot order inside a bucket is arbitrary and
// is fixed by the sort that follows.
// ------------------------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void k_col_scatter(const int32_t* __restrict__ row,
                                                    const int32_t* __restrict__ col,
                                                    int64_t nnz, int32_t n_rows,
                                                    int32_t n_cols,
                                                    const int32_t* __restrict__ colstart,
                                                    uint32_t* __restrict__ cursor,
                                                    uint64_t* __restrict__ bucket) {
  constexpr int U = 4;
  const int64_t stride = (int64_t)gridDim.x * NT * U;
  for (int64_t base = (int64_t)blockIdx.x * NT * U; base < nnz; base += stride) {
    int32_t r[U], c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * NT + threadIdx.x;
      r[u] = (i < nnz) ? row[i] : -1;
      c[u] = (i < nnz) ? col[i] : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * NT + threadIdx.x;
      if (i < nnz && (uint32_t)r[u] < (uint32_t)n_rows && (uint32_t)c[u] < (uint32_t)n_cols) {
        const uint32_t slot = atomicSub(&cursor[c[u]], 1u) - 1u;
        bucket[(int64_t)colstart[c[u]] + slot] = ((uint64_t)(uint32_t)r[u] << 32) | (uint32_t)i;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Segment sorting.  Keys are unique within a segment (they carry an input position or a
// CSC slot), so every correct sort gives the same result.
//   chunk_sort : segments [a, b) whose elements fit in LDS (<= CAP); each element's rank in
//                its segment is counted against the segment's keys in LDS, with the segment's
//                bounds recorded per element first (s_lohi, CAP words) so that the loads are
//                independent.
//   giant_sort : one segment longer than CAP, merge-sorted by the workgroup in global
//                memory (runs of NT by rank, then merge-path merges), ping-ponging with
//                `tmp`.
// PLAN = false writes the sorted keys back in place, tagging the smallest with kSegHead;
// PLAN = true writes the key halves to out_hi / out_lo instead.
// ------------------------------------------------------------------------------------------
template <int NT, int CAP, bool PLAN, typename ST>
__device__ void chunk_sort(uint64_t* __restrict__ keys, const ST* starts, int64_t a, int64_t b,
                           int32_t* __restrict__ out_hi, int32_t* __restrict__ out_lo,
                           uint64_t* s_key, uint32_t* s_lohi) {
  static_assert(CAP <= 65535, "segment bounds are packed as two 16-bit halves");
  constexpr int kLong = 64;  // longer segments get their bounds from the whole workgroup
  __shared__ int32_t s_long[CAP / kLong + 1];
  __shared__ int32_t s_nlong;
  const int64_t e0 = starts[a];
  const int cnt = (int)((int64_t)starts[b] - e0);
  if (threadIdx.x == 0) s_nlong = 0;
  constexpr int U = (CAP + NT - 1) / NT < 8 ? (CAP + NT - 1) / NT : 8;  // one pass for CAP <= 8 NT
  for (int i0 = threadIdx.x; i0 < cnt; i0 += NT * U) {
    uint64_t kv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * NT;
      kv[u] = (i < cnt) ? keys[e0 + i] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * NT;
      if (i < cnt) s_key[i] = kv[u];
    }
  }
  __syncthreads();
  // bounds of every element's segment, packed lo | hi << 16 (chunk-relative): one thread per
  // short segment, the whole workgroup per long one
  for (int64_t s = a + threadIdx.x; s < b; s += NT) {
    const int lo = (int)((int64_t)starts[s] - e0), hi = (int)((int64_t)starts[s + 1] - e0);
    if (hi - lo <= kLong) {
      for (int i = lo; i < hi; ++i) s_lohi[i] = (uint32_t)lo | ((uint32_t)hi << 16);
    } else {
      s_long[atomicAdd(&s_nlong, 1)] = (int32_t)(s - a);
    }
  }
  __syncthreads();
  for (int q = 0; q < s_nlong; ++q) {
    const int64_t s = a + s_long[q];
    const int lo = (int)((int64_t)starts[s] - e0), hi = (int)((int64_t)starts[s + 1] - e0);
    for (int i = lo + threadIdx.x; i < hi; i += NT)
      s_lohi[i] = (uint32_t)lo | ((uint32_t)hi << 16);
  }
  __syncthreads();
  // rank of each key in its segment (keys are unique): the bounds are known, so the loads are
  // independent and issued four at a time
  for (int i = threadIdx.x; i < cnt; i += NT) {
    const uint64_t key = s_key[i];
    const uint32_t lh = s_lohi[i];
    const int lo = (int)(lh & 0xffffu), hi = (int)(lh >> 16);
    int r = 0, j = lo;
    for (; j + 4 <= hi; j += 4) {
      const uint64_t k0 = s_key[j], k1 = s_key[j + 1], k2 = s_key[j + 2], k3 = s_key[j + 3];
      r += (int)(k0 < key) + (int)(k1 < key) + (int)(k2 < key) + (int)(k3 < key);
    }
    for (; j < hi; ++j) r += (int)(s_key[j] < key);
    const int64_t pos = e0 + lo + r;
    if (PLAN) {
      out_hi[pos] = (int32_t)(key >> 32);
      out_lo[pos] = (int32_t)(uint32_t)key;
    } else {
      keys[pos] = key | (r == 0 ? kSegHead : 0ull);
    }
  }
  __syncthreads();
}

template <int NT, bool PLAN>
__device__ void giant_sort(uint64_t* __restrict__ a, int64_t n, uint64_t* __restrict__ tmp,
                           int64_t out_base, int32_t* __restrict__ out_hi,
                           int32_t* __restrict__ out_lo, uint64_t* s_key) {
  // runs of NT elements, each sorted by rank into tmp
  for (int64_t r0 = 0; r0 < n; r0 += NT) {
    const int m = (int)((n - r0) < NT ? (n - r0) : NT);
    if ((int)threadIdx.x < m) s_key[threadIdx.x] = a[r0 + threadIdx.x];
    __syncthreads();
    if ((int)threadIdx.x < m) {
      const uint64_t key = s_key[threadIdx.x];
      int r = 0;
      for (int j = 0; j < m; ++j) r += (s_key[j] < key) ? 1 : 0;
      tmp[r0 + r] = key;
    }
    __syncthreads();
  }
  uint64_t* src = tmp;
  uint64_t* dst = a;
  constexpr int IPT = 8;
  for (int64_t w = NT; w < n; w <<= 1) {
    for (int64_t lo = 0; lo < n; lo += 2 * w) {
      const int64_t mid = (lo + w < n) ? lo + w : n;
      const int64_t hi = (lo + 2 * w < n) ? lo + 2 * w : n;
      const uint64_t* A = src + lo;
      const uint64_t* B = src + mid;
      const int64_t la = mid - lo, lb = hi - mid, tot = la + lb;
      for (int64_t d0 = 0; d0 < tot; d0 += (int64_t)NT * IPT) {
        const int64_t d = d0 + (int64_t)threadIdx.x * IPT;
        if (d < tot) {
          int64_t x = d - lb > 0 ? d - lb : 0;
          int64_t y = d < la ? d : la;
          while (x < y) {  // merge path: how many of the first d outputs come from A
            const int64_t m = (x + y) >> 1;
            if (A[m] < B[d - 1 - m]) x = m + 1; else y = m;
          }
          int64_t i = x, j = d - x;
          const int64_t end = (d + IPT < tot) ? d + IPT : tot;
          for (int64_t o = d; o < end; ++o) {
            const bool take_a = (i < la) && (j >= lb || A[i] < B[j]);
            dst[lo + o] = take_a ? A[i++] : B[j++];
          }
        }
      }
    }
    __syncthreads();
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    const uint64_t key = src[i];
    if (PLAN) {
      out_hi[out_base + i] = (int32_t)(key >> 32);
      out_lo[out_base + i] = (int32_t)(uint32_t)key;
    } else {
      a[i] = key | (i == 0 ? kSegHead : 0ull);
    }
  }
  __syncthreads();
}

// Sort segments [a, b_end) of `keys` (segment s = [starts[s], starts[s+1])) with one
// workgroup: consecutive segments are packed into LDS chunks of at most CAP elements; a
// segment longer than CAP is merge-sorted on its own.  `s_b` is 1 int64 of LDS.
template <int NT, int CAP, bool PLAN, typename ST>
__device__ void sort_segments(uint64_t* __restrict__ keys, const ST* starts, int64_t a,
                              int64_t b_end, uint64_t* __restrict__ scratch,
                              int32_t* __restrict__ out_hi, int32_t* __restrict__ out_lo,
                              uint64_t* s_key, uint32_t* s_lohi, int64_t* s_b) {
  while (a < b_end) {
    if (threadIdx.x == 0) {
      const int64_t e0 = starts[a];
      *s_b = a + upper_bound(starts + a, b_end - a + 1, e0 + CAP) - 1;
    }
    __syncthreads();
    const int64_t b = *s_b;
    __syncthreads();
    if (b == a) {
      const int64_t e0 = starts[a];
      const int64_t n = (int64_t)starts[a + 1] - e0;
      giant_sort<NT, PLAN>(keys + e0, n, scratch + e0, e0, out_hi, out_lo, s_key);
      a += 1;
    } else {
      chunk_sort<NT, CAP, PLAN>(keys, starts, a, b, out_hi, out_lo, s_key, s_lohi);
      a = b;
    }
  }
}

// Tile t of the segment sort owns the segments that begin in [t*T, (t+1)*T) (the last tile
// also owns every later one).
template <int NT, int CAP, bool PLAN>
__global__ __launch_bounds__(NT) void k_segsort(uint64_t* __restrict__ keys,
                                                const int32_t* __restrict__ starts,
                                                int64_t nseg, int64_t T,
                                                const int32_t* __restrict__ first,
                                                uint64_t* __restrict__ scratch,
                                                int32_t* __restrict__ out_hi,
                                                int32_t* __restrict__ out_lo) {
  __shared__ uint64_t s_key[CAP];
  __shared__ uint32_t s_lohi[CAP];
  __shared__ int64_t s_b[3];
  const int64_t N = starts[nseg];
  const int64_t ntiles = N > 0 ? (N + T - 1) / T : 1;
  const int64_t t = blockIdx.x;
  if (t >= ntiles) return;
  int64_t a = first[t];
  int64_t b_end = (t == ntiles - 1) ? nseg : (int64_t)first[t + 1];
  if (a > nseg) a = nseg;
  if (b_end > nseg) b_end = nseg;
  sort_segments<NT, CAP, PLAN>(keys, starts, a, b_end, scratch, out_hi, out_lo, s_key, s_lohi,
                               &s_b[2]);
}

// ------------------------------------------------------------------------------------------
// Fold one tile of the sorted, tagged keys.  Element i heads a run when it starts a column
// bucket or its row differs from element i-1's; the head folds its run left to right in
// binary64 (the run is in input order) and survives iff the sum is not 0.0.  Outputs the
// per-thread survivor mask (blocked layout: thread owns IPT consecutive elements).
// ------------------------------------------------------------------------------------------
template <int NT, int IPT, typename VT>
__device__ __forceinline__ uint32_t fold_tile(const uint64_t* __restrict__ keys,
                                              const uint64_t* s_k, int64_t base, int cnt,
                                              int64_t N, const VT* __restrict__ val,
                                              uint32_t (&rows)[IPT], double (&sums)[IPT]) {
  // head flags and the first value of every run are gathered for all IPT elements at once
  // (independent loads in flight), then each head folds the rest of its run in order.
  bool head[IPT];
#pragma unroll
  for (int s = 0; s < IPT; ++s) {
    const int li = threadIdx.x * IPT + s;
    head[s] = false;
    rows[s] = 0;
    sums[s] = 0.0;
    if (li < cnt) {
      const uint64_t key = s_k[li];
      const uint32_t row = key_row(key);
      bool h = (key & kSegHead) != 0;
      if (!h) {
        const uint64_t pk = (li > 0) ? s_k[li - 1] : keys[base - 1];
        h = key_row(pk) != row;
      }
      head[s] = h;
      rows[s] = row;
      if (h) sums[s] = to_acc<double>(val[(uint32_t)key]);
    }
  }
  uint32_t mask = 0;
#pragma unroll
  for (int s = 0; s < IPT; ++s) {
    if (head[s]) {
      const int li = threadIdx.x * IPT + s;
      double acc = sums[s];
      for (int64_t j = base + li + 1; j < N; ++j) {
        const uint64_t k2 = (j < base + cnt) ? s_k[j - base] : keys[j];
        if ((k2 & kSegHead) || key_row(k2) != rows[s]) break;
        acc = acc + to_acc<double>(val[(uint32_t)k2]);
      }
      sums[s] = acc;
      if (acc != 0.0) mask |= 1u << s;
    }
  }
  return mask;
}

// K3b + K4: fold, drop zeros, compact through a chained scan over tiles, column offsets.
template <int NT, int IPT, typename VT>
__global__ __launch_bounds__(NT) void k_fold(const uint64_t* __restrict__ keys,
                                             const int32_t* __restrict__ colstart,
                                             int64_t n_cols, const VT* __restrict__ val,
                                             int32_t* __restrict__ col_ptr,
                                             int32_t* __restrict__ row_idx,
                                             void* __restrict__ val_out, int out_f64,
                                             int32_t* __restrict__ info,
                                             const int32_t* __restrict__ first,
                                             uint64_t* __restrict__ state,
                                             uint32_t* __restrict__ ticket) {
  constexpr int T = NT * IPT;
  __shared__ uint64_t s_k[T];
  __shared__ uint32_t s_pre[T + 1];
  __shared__ uint32_t s_w[NT / kWave + 1];
  __shared__ int64_t s_t;
  __shared__ uint64_t s_off;
  __shared__ int64_t s_c[2];

  if (threadIdx.x == 0) s_t = atomicAdd(ticket, 1u);
  __syncthreads();
  const int64_t t = s_t;
  const int64_t N = colstart[n_cols];
  const int64_t ntiles = N > 0 ? (N + T - 1) / T : 1;
  if (t >= ntiles) return;
  const int64_t base = t * T;
  const int cnt = (int)((N - base) < T ? (N - base) : T);
#pragma unroll
  for (int s = 0; s < IPT; ++s) {
    const int li = s * NT + threadIdx.x;
    if (li < cnt) s_k[li] = keys[base + li];
  }
  __syncthreads();

  uint32_t rows[IPT];
  double sums[IPT];
  const uint32_t mask = fold_tile<NT, IPT, VT>(keys, s_k, base, cnt, N, val, rows, sums);
  uint32_t tile_kept;
  const uint32_t excl = wg_excl_scan<NT>((uint32_t)__popc(mask), s_w, &tile_kept);
  {
    uint32_t run = excl;
#pragma unroll
    for (int s = 0; s < IPT; ++s) {
      const int li = threadIdx.x * IPT + s;
      if (li < cnt) s_pre[li] = run;
      run += (mask >> s) & 1u;
    }
    if (threadIdx.x == 0) s_pre[cnt] = tile_kept;
  }
  if (threadIdx.x < kWave) {
    uint64_t prefix = 0;
    if (t == 0) {
      if (threadIdx.x == 0) lb_publish(state, kLbPre | tile_kept);
    } else {
      if (threadIdx.x == 0) lb_publish(state + t, kLbAgg | tile_kept);
      prefix = lookback_exclusive(state, t);
      if (threadIdx.x == 0) lb_publish(state + t, kLbPre | (prefix + tile_kept));
    }
    if (threadIdx.x == 0) {
      s_off = prefix;
      s_c[0] = first[t];
      s_c[1] = (t == ntiles - 1) ? n_cols + 1 : (int64_t)first[t + 1];
    }
  }
  __syncthreads();
  const int64_t off = (int64_t)s_off;
  {
    int64_t o = off + excl;
#pragma unroll
    for (int s = 0; s < IPT; ++s) {
      if ((mask >> s) & 1u) {
        row_idx[o] = (int32_t)rows[s];
        if (out_f64) static_cast<double*>(val_out)[o] = sums[s];
        else static_cast<float*>(val_out)[o] = (float)sums[s];
        ++o;
      }
    }
  }
  for (int64_t c = s_c[0] + threadIdx.x; c < s_c[1]; c += NT) {
    int64_t p = (int64_t)colstart[c] - base;
    if (p > cnt) p = cnt;
    col_ptr[c] = (int32_t)(off + s_pre[p]);
  }
  if (t == ntiles - 1 && threadIdx.x == 0) info[0] = (int32_t)(off + tile_kept);
}

// ------------------------------------------------------------------------------------------
// Plan: check the CSC, count stored elements per row.
// ------------------------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void k_plan_hist(const int32_t* __restrict__ col_ptr,
                                                  const int32_t* __restrict__ row_idx,
                                                  int64_t n_rows, int64_t n_cols,
                                                  int64_t nnz_cap, uint32_t* __restrict__ rowcnt,
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
  for (int64_t c = gid; c < n_cols; c += stride)
    if (col_ptr[c] > col_ptr[c + 1]) bad_shape = true;
  for (int64_t p = gid; p < nnz; p += stride) {
    const int32_t r = row_idx[p];
    if ((uint64_t)(uint32_t)r < (uint64_t)n_rows && r >= 0) atomicAdd(&rowcnt[r], 1u);
    else bad_row = true;
  }
  if (bad_shape) set_status(info, kStEinval);
  if (bad_row) set_status(info, kStBounds);
}

// Scatter (col << 32 | slot) of every stored element into its row's bucket: one thread per
// column walks that column's slots.
template <int NT>
__global__ __launch_bounds__(NT) void k_row_scatter(const int32_t* __restrict__ col_ptr,
                                                    const int32_t* __restrict__ row_idx,
                                                    int64_t n_rows, int64_t n_cols,
                                                    int64_t nnz_cap,
                                                    const int32_t* __restrict__ row_ptr,
                                                    uint32_t* __restrict__ cursor,
                                                    uint64_t* __restrict__ bucket) {
  const int64_t raw = col_ptr[n_cols];
  const int64_t nnz = raw < 0 ? 0 : (raw > nnz_cap ? nnz_cap : raw);
  const int64_t stride = (int64_t)gridDim.x * NT;
  for (int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x; c < n_cols; c += stride) {
    int64_t p0 = col_ptr[c], p1 = col_ptr[c + 1];
    p0 = p0 < 0 ? 0 : (p0 > nnz ? nnz : p0);
    p1 = p1 < p0 ? p0 : (p1 > nnz ? nnz : p1);
    for (int64_t p = p0; p < p1; ++p) {
      const int32_t r = row_idx[p];
      if (r >= 0 && (int64_t)r < n_rows) {
        const uint32_t slot = atomicSub(&cursor[r], 1u) - 1u;
        bucket[(int64_t)row_ptr[r] + slot] = ((uint64_t)c << 32) | (uint32_t)p;
      }
    }
  }
}

}  // namespace spm
