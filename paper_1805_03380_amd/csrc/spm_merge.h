// Sum A + B of two CSCs by a direct merge of their sorted columns: one lane per column walks
// both row lists once to count the stored results, an exclusive scan turns the counts into
// the column offsets, and a second walk writes rows and values.  A location stored in both
// holds A's value plus B's in binary64 (rounded once to the output type); a result that
// compares equal to 0.0 is not stored.  This is the same arithmetic as the insertion path
// (existing value first, then the one new value), so both forms give the same bits; the merge
// reads each operand twice and never re-sorts, which pays off for short columns.
#pragma once

#include "spm_device.h"

namespace spm {

constexpr uint32_t kMergeShape = 1u;   // offsets not starting at 0, decreasing or beyond cap
constexpr uint32_t kMergeOrder = 2u;   // rows not strictly increasing down a column
constexpr uint32_t kMergeBounds = 4u;  // a stored row outside the matrix

// One operand's column: [p, pe) after the offset checks (empty when they fail).
__device__ __forceinline__ bool merge_span(const int32_t* __restrict__ cp, int64_t c,
                                           int64_t cap, int64_t& p, int64_t& pe) {
  p = cp[c];
  pe = cp[c + 1];
  const bool ok = p >= 0 && p <= pe && pe <= cap && (c != 0 || p == 0);
  if (!ok) p = pe = 0;
  return ok;
}

// Walks column c of A and B in row order; for each stored result calls emit(row, value).
// Rows outside the matrix are skipped; every irregularity is reported in `flags`.
template <typename VT, typename Emit>
__device__ __forceinline__ void merge_column(int64_t c, int64_t n_rows, int64_t a_cap,
                                             const int32_t* __restrict__ a_cp,
                                             const int32_t* __restrict__ a_ri,
                                             const VT* __restrict__ a_v, int64_t b_cap,
                                             const int32_t* __restrict__ b_cp,
                                             const int32_t* __restrict__ b_ri,
                                             const VT* __restrict__ b_v, uint32_t& flags,
                                             Emit emit) {
  int64_t p, pe, q, qe;
  if (!merge_span(a_cp, c, a_cap, p, pe)) flags |= kMergeShape;
  if (!merge_span(b_cp, c, b_cap, q, qe)) flags |= kMergeShape;
  int32_t a_prev = -1, b_prev = -1;
  while (p < pe || q < qe) {
    const int32_t ra = p < pe ? a_ri[p] : INT32_MAX;
    const int32_t rb = q < qe ? b_ri[q] : INT32_MAX;
    int32_t r;
    double v;
    if (ra < rb) {
      r = ra;
      v = (double)a_v[p];
      if (ra <= a_prev) flags |= kMergeOrder;
      a_prev = ra;
      ++p;
    } else if (rb < ra) {
      r = rb;
      v = (double)b_v[q];
      if (rb <= b_prev) flags |= kMergeOrder;
      b_prev = rb;
      ++q;
    } else {  // stored in both: A's value first
      r = ra;
      v = (double)a_v[p] + (double)b_v[q];
      if (ra <= a_prev || rb <= b_prev) flags |= kMergeOrder;
      a_prev = ra;
      b_prev = rb;
      ++p;
      ++q;
    }
    if (r < 0 || (int64_t)r >= n_rows) {
      flags |= kMergeBounds;
      continue;
    }
    if (v != 0.0) emit(r, v);
  }
}

template <int NT, typename VT>
__global__ __launch_bounds__(NT) void k_add_count(
    int64_t n_rows, int64_t n_cols, int64_t a_cap, const int32_t* __restrict__ a_cp,
    const int32_t* __restrict__ a_ri, const VT* __restrict__ a_v, int64_t b_cap,
    const int32_t* __restrict__ b_cp, const int32_t* __restrict__ b_ri,
    const VT* __restrict__ b_v, uint32_t* __restrict__ counts, uint32_t* __restrict__ flag) {
  uint32_t flags = 0;
  for (int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x; c < n_cols;
       c += (int64_t)gridDim.x * NT) {
    uint32_t n = 0;
    merge_column<VT>(c, n_rows, a_cap, a_cp, a_ri, a_v, b_cap, b_cp, b_ri, b_v, flags,
                     [&](int32_t, double) { ++n; });
    counts[c] = n;
  }
  if (flags) atomicOr(flag, flags);
}

template <int NT, typename VT>
__global__ __launch_bounds__(NT) void k_add_write(
    int64_t n_rows, int64_t n_cols, int64_t a_cap, const int32_t* __restrict__ a_cp,
    const int32_t* __restrict__ a_ri, const VT* __restrict__ a_v, int64_t b_cap,
    const int32_t* __restrict__ b_cp, const int32_t* __restrict__ b_ri,
    const VT* __restrict__ b_v, const int32_t* __restrict__ col_ptr,
    int32_t* __restrict__ row_idx, void* __restrict__ val_out, int out_f64, int64_t out_cap) {
  // A malformed pair of CSCs (offsets that pass each column's own checks but overlap between
  // columns) can make the counts total more than the outputs hold, and the int32 scan of such
  // counts can wrap: every store is therefore checked against [0, out_cap).  The count pass
  // has already reported the malformed input.
  for (int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x; c < n_cols;
       c += (int64_t)gridDim.x * NT) {
    int64_t o = col_ptr[c];
    uint32_t flags = 0;  // already reported by the count pass
    merge_column<VT>(c, n_rows, a_cap, a_cp, a_ri, a_v, b_cap, b_cp, b_ri, b_v, flags,
                     [&](int32_t r, double v) {
                       if (o >= 0 && o < out_cap) {
                         row_idx[o] = r;
                         if (out_f64) static_cast<double*>(val_out)[o] = v;
                         else static_cast<float*>(val_out)[o] = (float)v;
                       }
                       ++o;
                     });
  }
}

// info[0] = stored count, info[1] = status (a malformed CSC before a row out of range).
__global__ void k_add_finish(int64_t n_cols, const int32_t* __restrict__ col_ptr,
                             const uint32_t* __restrict__ flag, int32_t* __restrict__ info,
                             int32_t st_inval, int32_t st_bounds) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    info[0] = col_ptr[n_cols];
    const uint32_t f = *flag;
    info[1] = (f & (kMergeShape | kMergeOrder)) ? st_inval : ((f & kMergeBounds) ? st_bounds : 0);
  }
}

}  // namespace spm
