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

// Level 1b: scatter (key, segment-within-bucket) into the buckets.  The range of (bucket cb,
// tile t) starts at bstart[cb] + rowoff[cb * ntiles + t], where bstart is the exclusive scan
// of the bucket totals: every workgroup scans btot (a few KB) itself, and workgroup 0 also
// stores the scan (bstart[0..CB], bstart[CB] = total) for the kernels that follow.
template <int NT, typename SRC>
__global__ __launch_bounds__(NT) void k_part_scatter(SRC src, int b, int32_t CB, int64_t ntiles,
                                                     int64_t T1,
                                                     const uint32_t* __restrict__ rowoff,
                                                     const uint32_t* __restrict__ btot,
                                                     int32_t* __restrict__ bstart,
                                                     uint64_t* __restrict__ bkey,
                                                     uint32_t* __restrict__ bseg) {
  __shared__ uint32_t cur[kPartMaxBuckets];
  __shared__ uint32_t s_w[NT / kWave + 1];
  const int64_t t = blockIdx.x;
  const int64_t n = src.count();
  {
    constexpr int IPT = kPartMaxBuckets / NT;
    uint32_t v[IPT];
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      const int i = threadIdx.x * IPT + q;
      v[q] = i < CB ? btot[i] : 0u;
      sum += v[q];
    }
    uint32_t tot;
    uint32_t run = wg_excl_scan<NT>(sum, s_w, &tot);
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      const int i = threadIdx.x * IPT + q;
      if (i < CB) {
        cur[i] = run + rowoff[(int64_t)i * ntiles + t];
        if (t == 0) bstart[i] = (int32_t)run;
      }
      run += v[q];
    }
    if (t == 0 && threadIdx.x == 0) bstart[CB] = (int32_t)tot;
  }
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

// Per-bucket exclusive scan of one row of the (bucket x tile) table: rowoff[cb][t] = number of
// bucket-cb elements in tiles before t; btot[cb] = the bucket's total.  One workgroup per row.
template <int NT>
__global__ __launch_bounds__(NT) void k_rows_scan(const uint32_t* __restrict__ table,
                                                  int64_t ntiles, uint32_t* __restrict__ rowoff,
                                                  uint32_t* __restrict__ btot) {
  __shared__ uint32_t s_w[NT / kWave + 1];
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
  if (threadIdx.x == 0) btot[cb] = carry;
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
// Dynamic LDS: cnt[W+1] u32 | s_in[CAP] u64 | s_key[CAP] u64 | s_seg[CAP] u16 |
//              s_flag[CAP] u8   (part_level2_lds_bytes).  The fold's survivor prefix
//              s_pre[CAP+1] u32 reuses s_key, which is dead once the bucket is sorted; at
//              b = 7 this keeps a workgroup under 40 KB, four per CU.
// ------------------------------------------------------------------------------------------
__host__ __device__ inline size_t part_level2_lds_bytes(int b, int cap) {
  const size_t w = ((size_t)1 << b) + 1;
  size_t off = (w * 4 + 15) & ~(size_t)15;
  off += (size_t)cap * 8 * 2;
  off += (((size_t)cap * 2) + 15) & ~(size_t)15;
  off += (size_t)cap;
  return off;
}

template <int NT, int CAP, bool PLAN, typename VT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_part_level2(
    int b, int64_t nseg, const int32_t* __restrict__ bstarts, const uint64_t* __restrict__ bkey,
    const uint32_t* __restrict__ bseg, uint64_t* __restrict__ gkeys,
    uint64_t* __restrict__ scratch, int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_t,
    int32_t* __restrict__ perm, const VT* __restrict__ val, int32_t* __restrict__ col_rel,
    uint32_t* __restrict__ trow, double* __restrict__ tval, uint32_t* __restrict__ bkept) {
  constexpr int IPT = CAP / NT;
  static_assert(IPT * NT == CAP, "CAP must be a multiple of the workgroup size");
  extern __shared__ __align__(16) unsigned char smem[];
  const size_t wcnt = ((size_t)1 << b) + 1;
  uint32_t* cnt = reinterpret_cast<uint32_t*>(smem);
  size_t off = (wcnt * 4 + 15) & ~(size_t)15;
  uint64_t* s_in = reinterpret_cast<uint64_t*>(smem + off);
  off += (size_t)CAP * 8;
  uint64_t* s_key = reinterpret_cast<uint64_t*>(smem + off);
  uint32_t* s_pre = reinterpret_cast<uint32_t*>(smem + off);  // aliases s_key (see above)
  static_assert((CAP + 1) * 4 <= CAP * 8, "s_pre must fit in s_key");
  off += (size_t)CAP * 8;
  uint16_t* s_seg = reinterpret_cast<uint16_t*>(smem + off);
  off += (((size_t)CAP * 2) + 15) & ~(size_t)15;
  uint8_t* s_flag = smem + off;
  __shared__ uint32_t s_w[NT / kWave + 1];
  __shared__ int64_t s_b[3];

  const int64_t cb = blockIdx.x;
  const int64_t bstart = bstarts[cb];
  const int64_t bend = bstarts[cb + 1];
  const int64_t m = bend - bstart;
  const int64_t seg0 = cb << b;
  const int64_t rem = nseg - seg0;
  const int64_t nW = rem < ((int64_t)1 << b) ? rem : ((int64_t)1 << b);
  const bool last_bucket = seg0 + nW >= nseg;
  constexpr int U = 8;

  for (int64_t j = threadIdx.x; j <= nW; j += NT) cnt[j] = 0;
  const bool fast = m <= CAP;
  if (fast) {
    for (int64_t i0 = threadIdx.x; i0 < m; i0 += (int64_t)NT * U) {
      uint64_t ky[U];
      uint32_t sg[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + (int64_t)u * NT;
        ky[u] = i < m ? bkey[bstart + i] : 0ull;
        sg[u] = i < m ? bseg[bstart + i] : 0u;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + (int64_t)u * NT;
        if (i < m) {
          s_in[i] = ky[u];
          s_seg[i] = (uint16_t)sg[u];
        }
      }
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < m; i += NT) atomicAdd(&cnt[s_seg[i]], 1u);
  } else {
    __syncthreads();
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
  }
  __syncthreads();
  wg_inclusive_scan_inplace<NT>(cnt, nW, s_w);  // cnt[j] = end of segment j (relative)
  if (PLAN) {
    for (int64_t j = threadIdx.x; j < nW; j += NT)
      row_ptr[seg0 + j] = (int32_t)(bstart + (j == 0 ? 0 : (int64_t)cnt[j - 1]));
    if (last_bucket && threadIdx.x == 0) row_ptr[nseg] = (int32_t)bend;
  }
  __syncthreads();

  if (fast) {
    // ---- everything in LDS ----------------------------------------------------------------
    // Group by segment: each element (load order) takes the next free slot of its segment;
    // the thread keeps the (key, segment) of its elements for the ranking.
    uint64_t ky[IPT];
    uint32_t sg[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int64_t i = threadIdx.x + (int64_t)u * NT;
      sg[u] = 0xffffffffu;
      ky[u] = 0;
      if (i < m) {
        sg[u] = s_seg[i];
        ky[u] = s_in[i];
        const uint32_t pos = atomicSub(&cnt[sg[u]], 1u) - 1u;
        s_key[pos] = ky[u];
      }
    }
    for (int64_t i = threadIdx.x; i < m; i += NT) s_flag[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) cnt[nW] = (uint32_t)m;  // cnt[j] = start of segment j
    __syncthreads();
    for (int64_t j = threadIdx.x; j < nW; j += NT) {
      const uint32_t lo = cnt[j];
      if (lo < (uint32_t)m) s_flag[lo] = 1;
    }
    // Rank each element among the keys of its segment (keys are unique, so the ranks are a
    // permutation): the segment's bounds come from cnt, so the loads are independent and
    // issued four at a time.
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
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
        s_in[lo + r] = key;  // s_in now holds the bucket sorted by (segment, key)
      }
    }
    __syncthreads();
    if (PLAN) {
      for (int64_t i = threadIdx.x; i < m; i += NT) {
        const uint64_t key = s_in[i];
        col_t[bstart + i] = (int32_t)(key >> 32);
        perm[bstart + i] = (int32_t)(uint32_t)key;
      }
      return;
    }
    // Fold.  Every element's value is gathered once, all of a thread's loads in flight, into
    // LDS (s_val reuses s_key, dead after the ranking); then each thread takes IPT
    // consecutive positions and folds every run that starts there, from LDS, in key order
    // (= input order within a run).
    double* s_val = reinterpret_cast<double*>(s_key);
    static_assert(sizeof(double) <= sizeof(uint64_t), "s_val must fit in s_key");
    {
      VT v[IPT];
#pragma unroll
      for (int u = 0; u < IPT; ++u) {
        const int64_t i = threadIdx.x + (int64_t)u * NT;
        if (i < m) v[u] = val[(uint32_t)s_in[i]];
      }
#pragma unroll
      for (int u = 0; u < IPT; ++u) {
        const int64_t i = threadIdx.x + (int64_t)u * NT;
        if (i < m) s_val[i] = to_acc<double>(v[u]);
      }
    }
    __syncthreads();
    uint32_t rows[IPT];
    double sums[IPT];
    uint32_t mask = 0;
#pragma unroll
    for (int s = 0; s < IPT; ++s) {
      const int64_t li = (int64_t)threadIdx.x * IPT + s;
      rows[s] = 0;
      sums[s] = 0.0;
      if (li < m) {
        const uint64_t key = s_in[li];
        rows[s] = key_row(key);
        const bool head = s_flag[li] || key_row(s_in[li - 1]) != rows[s];
        if (head) {
          double acc = s_val[li];
          for (int64_t j = li + 1; j < m && !s_flag[j]; ++j) {
            if (key_row(s_in[j]) != rows[s]) break;
            acc = acc + s_val[j];
          }
          sums[s] = acc;
          if (acc != 0.0) mask |= 1u << s;
        }
      }
    }
    uint32_t kept;
    const uint32_t excl = wg_excl_scan<NT>((uint32_t)__popc(mask), s_w, &kept);
    {
      uint32_t run = excl;
#pragma unroll
      for (int s = 0; s < IPT; ++s) {
        const int64_t li = (int64_t)threadIdx.x * IPT + s;
        if (li < m) s_pre[li] = run;
        run += (mask >> s) & 1u;
      }
      if (threadIdx.x == 0) s_pre[m] = kept;
    }
    __syncthreads();
    {
      int64_t o = bstart + excl;
#pragma unroll
      for (int s = 0; s < IPT; ++s) {
        if ((mask >> s) & 1u) {
          trow[o] = rows[s];
          tval[o] = sums[s];
          ++o;
        }
      }
    }
    for (int64_t j = threadIdx.x; j < nW; j += NT) col_rel[seg0 + j] = (int32_t)s_pre[cnt[j]];
    if (threadIdx.x == 0) bkept[cb] = kept;
    return;
  }

  // ---- large bucket: global staging ---------------------------------------------------------
  uint64_t* gk = gkeys + bstart;
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
        gk[pos] = ky[u];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) cnt[nW] = (uint32_t)m;
  __syncthreads();
  sort_segments<NT, CAP, PLAN>(gk, cnt, 0, nW, scratch + bstart, PLAN ? col_t + bstart : col_t,
                               PLAN ? perm + bstart : perm, s_key, s_flag, &s_b[0]);
  if (PLAN) return;
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
      col_rel[seg0 + j] = (int32_t)(running + s_pre[p]);
    }
    running += blk;
    __syncthreads();
  }
  if (threadIdx.x == 0) bkept[cb] = running;
}

// Place each bucket's survivors: the bucket's output offset is the sum of the survivor
// counts of the buckets before it (each workgroup reduces bkept[0..cb) itself; the last one
// also takes its own, giving nnz_out).  Moves the survivors from the temporaries to their
// final place (rounded once to the output type), turns the bucket-relative column offsets
// into col_ptr, and finishes col_ptr / info.
template <int NT>
__global__ __launch_bounds__(NT) void k_part_emit(int b, int32_t CB, int64_t nseg,
                                                  const int32_t* __restrict__ bstarts,
                                                  const uint32_t* __restrict__ bkept,
                                                  const uint32_t* __restrict__ trow,
                                                  const double* __restrict__ tval,
                                                  int32_t* __restrict__ col_ptr,
                                                  int32_t* __restrict__ row_idx,
                                                  void* __restrict__ val_out, int out_f64,
                                                  int32_t* __restrict__ info) {
  __shared__ uint32_t s_w[NT / kWave + 1];
  const int64_t cb = blockIdx.x;
  const bool last = cb == (int64_t)CB - 1;
  const int64_t lim = last ? CB : cb;
  uint32_t part = 0;
  for (int64_t i = threadIdx.x; i < lim; i += NT) part += bkept[i];
  uint32_t tot;
  (void)wg_excl_scan<NT>(part, s_w, &tot);
  const int64_t src0 = bstarts[cb];
  const int64_t kept = bkept[cb];
  const int64_t dst0 = last ? (int64_t)tot - kept : (int64_t)tot;
  for (int64_t i = threadIdx.x; i < kept; i += NT) {
    row_idx[dst0 + i] = (int32_t)trow[src0 + i];
    if (out_f64) static_cast<double*>(val_out)[dst0 + i] = tval[src0 + i];
    else static_cast<float*>(val_out)[dst0 + i] = (float)tval[src0 + i];
  }
  const int64_t seg0 = cb << b;
  const int64_t rem = nseg - seg0;
  const int64_t nW = rem < ((int64_t)1 << b) ? rem : ((int64_t)1 << b);
  for (int64_t j = threadIdx.x; j < nW; j += NT) col_ptr[seg0 + j] += (int32_t)dst0;
  if (last && threadIdx.x == 0) {
    col_ptr[nseg] = (int32_t)tot;
    info[0] = (int32_t)tot;
  }
}

}  // namespace spm
