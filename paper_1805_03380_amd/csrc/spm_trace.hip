// trace(A^T B) of two CSC matrices of one shape, without forming A^T or the product
// (Section 2's example of an expression evaluated from its parts; Table 1).
//
// Entry (j, j) of A^T B is the dot product of column j of A with column j of B, so the trace
// is the sum, over locations stored in both matrices, of A[i,j] * B[i,j]: a sorted-list
// intersection per column followed by a reduction.  The work is HBM-bound (both index
// arrays are read once; values only where rows match), so the kernel is built around
// coalesced column reads and cached binary searches, not matrix cores.
//
// Reduction order (fixed by the data and two constants, never by the launch shape):
//   - element j of A's column (its offset from the column start) belongs to virtual lane
//     j mod 64; each virtual lane adds its matched products in increasing j;
//   - the 64 virtual lanes of a column combine by halving, v[i] += v[i + s] for
//     s = 32, 16, ..., 1, giving the column's dot product;
//   - chunks of kTraceChunk consecutive columns add their dot products in column order;
//   - the chunk sums combine in a fixed two-level order (kTraceFinishNT strided sequences,
//     then halving).
// A group of GW lanes (16, 32 or 64) walks one column at a time and keeps 64 / GW virtual
// lanes per physical lane, so every group width gives the same bits.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "spm.h"
#include "spm_range.h"

namespace spm {

constexpr int kTraceChunk = 16;      // columns per workgroup (one partial sum each)
constexpr int kTraceVL = 64;         // virtual lanes per column
constexpr int kTraceFinishNT = 256;  // threads of the single finishing workgroup
constexpr int kTraceU = 8;           // A elements per lane in flight (a multiple of 64 / GW)
constexpr int kTraceUB = 8;          // B rows per lane in flight
constexpr int kTraceBmRows = 16384;  // largest row count of the bitmap form (at most 3 KiB of
                                     // LDS per column)
constexpr int kTraceLdsPerLane = 19; // B rows per lane of the LDS slice (1216 at 64 lanes: two
                                     // workgroups of 16 columns fit in 160 KiB)

constexpr uint32_t kFlagInval = 1u;   // a malformed CSC (offsets, or rows not increasing)
constexpr uint32_t kFlagBounds = 2u;  // a stored row outside the matrix

template <typename VT>
__device__ __forceinline__ double widen_val(VT v) {
  return (double)v;
}

// First position in b[lo, hi) whose row is not below r (hi if none).
__device__ __forceinline__ int64_t lower_row(const int32_t* __restrict__ b, int64_t lo,
                                             int64_t hi, int32_t r) {
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (b[mid] < r) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Sum of v over the GW lanes of a group by halving strides below GW (lane 0 holds it).
template <int GW>
__device__ __forceinline__ double group_halving(double v) {
#pragma unroll
  for (int s = GW / 2; s >= 1; s >>= 1) v += __shfl_down(v, s, GW);
  return v;
}

template <int GW>
__device__ __forceinline__ uint32_t group_sum_u32(uint32_t v) {
#pragma unroll
  for (int s = GW / 2; s >= 1; s >>= 1) v += __shfl_down(v, s, GW);
  return v;
}

// Lower bound of r in the sorted rows b[lo, lo + n): a fixed number of halving steps for the
// whole group (n is the same for every lane), so the lanes stay converged.
__device__ __forceinline__ int lower_row_fixed(const int32_t* __restrict__ b, int n, int32_t r) {
  int lo = 0;
  int step = 1;
  while (step <= n / 2) step <<= 1;
  for (; step > 0; step >>= 1)
    if (lo + step <= n && b[lo + step - 1] < r) lo += step;
  return lo;
}

// Rows of one column, read U per lane at a time (element j = j0 + u GW + lg), checked
// to lie in the matrix and to increase strictly (the previous element's row comes from the
// neighbouring lane, or from the last lane's previous read).
template <int GW, int U>
__device__ __forceinline__ void check_rows(const int32_t (&r)[U], int j0, int n, int lg,
                                           int64_t n_rows, int32_t& prev, uint32_t& flags) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = j0 + u * GW + lg;
    const int32_t up = __shfl_up(r[u], 1, GW);
    const int32_t before = lg == 0 ? prev : up;
    prev = __shfl(r[u], GW - 1, GW);
    if (j < n) {
      if (r[u] < 0 || (int64_t)r[u] >= n_rows) flags |= kFlagBounds;
      if (j > 0 && before >= r[u]) flags |= kFlagInval;
    }
  }
}

// Exclusive prefix sum over the GW lanes of a group.
template <int GW>
__device__ __forceinline__ uint32_t group_excl_scan(uint32_t x, int lg) {
  uint32_t incl = x;
#pragma unroll
  for (int d = 1; d < GW; d <<= 1) {
    const uint32_t t = __shfl_up(incl, d, GW);
    if (lg >= d) incl += t;
  }
  return incl - x;
}

// One workgroup per chunk of kTraceChunk columns, one group of GW lanes per column.  Per
// column, B's rows are read once (coalesced) and checked, then made searchable in LDS:
//   BM (n_rows <= kTraceBmRows): a bitmap of B's rows with the set-bit count before each
//     32-row word, so that a row's presence and its position in B's column (the rank) take
//     two LDS reads and a popcount;
//   otherwise: B's rows themselves (when they fit the group's slice of kTraceLdsPerLane * GW
//     rows; a longer column is searched in global memory), looked up by binary search.
// A's rows are then read in batches of kTraceU per lane, checked, and looked up; a match adds
// A's value times B's value (binary64) to the lane's accumulator of that element's virtual
// lane.  Writes the chunk's sum, matched count and status flags at index blockIdx.x.
template <typename VT, int GW, bool BM>
__global__ __launch_bounds__(kTraceChunk * GW) void k_trace_atb(
    int64_t n_rows, int64_t n_cols, int64_t a_cap, const int32_t* __restrict__ a_col_ptr,
    const int32_t* __restrict__ a_row_idx, const VT* __restrict__ a_val, int64_t b_cap,
    const int32_t* __restrict__ b_col_ptr, const int32_t* __restrict__ b_row_idx,
    const VT* __restrict__ b_val, double* __restrict__ part_sum,
    uint32_t* __restrict__ part_hits, uint32_t* __restrict__ part_flags, int slice) {
  constexpr int A = kTraceVL / GW;              // virtual lanes per physical lane
  constexpr int CAP = kTraceLdsPerLane * GW;    // B rows per LDS slice (search form)
  static_assert(kTraceU % A == 0, "a batch of GW * kTraceU elements spans whole virtual rounds");
  extern __shared__ __align__(16) unsigned char s_raw[];  // kTraceChunk slices of `slice` bytes
  __shared__ double s_col[kTraceChunk];
  __shared__ uint32_t s_hits[kTraceChunk];
  __shared__ uint32_t s_flags;
  const int lg = threadIdx.x % GW;
  const int ci = threadIdx.x / GW;
  const int nw = (int)((n_rows + 31) >> 5);  // bitmap words (bitmap form)
  // search form: up to CAP of B's rows; bitmap form: nw words, then nw 16-bit ranks
  int32_t* sb = reinterpret_cast<int32_t*>(s_raw + ci * slice);
  uint32_t* bm = reinterpret_cast<uint32_t*>(s_raw + ci * slice);
  uint16_t* pre = reinterpret_cast<uint16_t*>(s_raw + ci * slice + nw * 4);
  const int64_t c = (int64_t)blockIdx.x * kTraceChunk + ci;
  if (threadIdx.x == 0) s_flags = 0;
  uint32_t flags = 0;
  int64_t pa0 = 0, pa1 = 0, pb0 = 0, pb1 = 0;
  if (c < n_cols) {
    pa0 = a_col_ptr[c];
    pa1 = a_col_ptr[c + 1];
    pb0 = b_col_ptr[c];
    pb1 = b_col_ptr[c + 1];
    bool ok = pa0 >= 0 && pa0 <= pa1 && pa1 <= a_cap && pb0 >= 0 && pb0 <= pb1 && pb1 <= b_cap;
    if (c == 0 && (pa0 != 0 || pb0 != 0)) ok = false;
    if (!ok) {
      flags |= kFlagInval;
      pa0 = pa1 = pb0 = pb1 = 0;
    }
  }
  const int nb = (int)(pb1 - pb0), na = (int)(pa1 - pa0);
  const bool lds = BM || nb <= CAP;
  const int32_t* bcol = b_row_idx + pb0;
  const int32_t* acol = a_row_idx + pa0;
  if (BM) {
    for (int w = lg; w < nw; w += GW) bm[w] = 0u;
    __syncthreads();
  }
  // B's rows: checked once, kTraceUB loads in flight per lane, then into LDS
  int32_t prev = INT32_MIN;
  for (int q0 = 0; q0 < nb; q0 += GW * kTraceUB) {
    int32_t rb[kTraceUB];
#pragma unroll
    for (int u = 0; u < kTraceUB; ++u) {
      const int q = q0 + u * GW + lg;
      rb[u] = q < nb ? bcol[q] : INT32_MAX;
    }
    check_rows<GW, kTraceUB>(rb, q0, nb, lg, n_rows, prev, flags);
#pragma unroll
    for (int u = 0; u < kTraceUB; ++u) {
      const int q = q0 + u * GW + lg;
      if (q < nb) {
        if (BM) {
          if (rb[u] >= 0 && (int64_t)rb[u] < n_rows)
            atomicOr(&bm[rb[u] >> 5], 1u << (rb[u] & 31));
        } else if (lds) {
          sb[q] = rb[u];
        }
      }
    }
  }
  __syncthreads();  // B in LDS (and s_flags cleared) before any lookup
  if (BM) {
    // rank of each word: set bits in the words before it (a run of words per lane)
    const int per = (nw + GW - 1) / GW;
    const int w0 = lg * per;
    uint32_t run = 0;
    for (int k = 0; k < per; ++k)
      if (w0 + k < nw) run += __popc(bm[w0 + k]);
    uint32_t before = group_excl_scan<GW>(run, lg);
    for (int k = 0; k < per; ++k)
      if (w0 + k < nw) {
        pre[w0 + k] = (uint16_t)before;
        before += __popc(bm[w0 + k]);
      }
    __syncthreads();
  }
  const int32_t* sc = lds ? sb : bcol;  // where the searches read B's rows (search form)
  double acc[A];
#pragma unroll
  for (int u = 0; u < A; ++u) acc[u] = 0.0;
  uint32_t hits = 0;
  prev = INT32_MIN;
  // A's rows in batches of kTraceU per lane.  A batch starts at a multiple of GW * kTraceU,
  // a multiple of 64, so element j's virtual lane j mod 64 is this lane's accumulator u mod A.
  for (int j0 = 0; j0 < na; j0 += GW * kTraceU) {
    int32_t r[kTraceU];
#pragma unroll
    for (int u = 0; u < kTraceU; ++u) {
      const int j = j0 + u * GW + lg;
      r[u] = j < na ? acol[j] : INT32_MAX;
    }
    check_rows<GW, kTraceU>(r, j0, na, lg, n_rows, prev, flags);
    int32_t qb[kTraceU];  // B position of a match (offset from pb0), or -1
#pragma unroll
    for (int u = 0; u < kTraceU; ++u) {
      qb[u] = -1;
      if (j0 + u * GW + lg < na) {
        if (BM) {
          if (r[u] >= 0 && (int64_t)r[u] < n_rows) {
            const uint32_t word = bm[r[u] >> 5];
            const uint32_t bit = (uint32_t)r[u] & 31u;
            if ((word >> bit) & 1u)
              qb[u] = (int32_t)pre[r[u] >> 5] + __popc(word & ((1u << bit) - 1u));
          }
        } else {
          const int lo = lower_row_fixed(sc, nb, r[u]);
          if (lo < nb && sc[lo] == r[u]) qb[u] = lo;
        }
      }
    }
    double av[kTraceU], bv[kTraceU];
#pragma unroll
    for (int u = 0; u < kTraceU; ++u) {
      av[u] = qb[u] >= 0 ? widen_val(a_val[pa0 + j0 + u * GW + lg]) : 0.0;
      bv[u] = qb[u] >= 0 ? widen_val(b_val[pb0 + qb[u]]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kTraceU; ++u)
      if (qb[u] >= 0) {
        acc[u % A] += av[u] * bv[u];
        ++hits;
      }
  }
  // halving over the 64 virtual lanes: strides >= GW inside the lane, the rest across lanes
#pragma unroll
  for (int s = A / 2; s >= 1; s >>= 1) {
#pragma unroll
    for (int u = 0; u < s; ++u) acc[u] += acc[u + s];
  }
  const double col = group_halving<GW>(acc[0]);
  hits = group_sum_u32<GW>(hits);
  if (lg == 0) {
    s_col[ci] = col;
    s_hits[ci] = hits;
  }
  if (flags) atomicOr(&s_flags, flags);
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    uint32_t h = 0;
    for (int k = 0; k < kTraceChunk; ++k) {
      sum += s_col[k];
      h += s_hits[k];
    }
    part_sum[blockIdx.x] = sum;
    part_hits[blockIdx.x] = h;
    part_flags[blockIdx.x] = s_flags;
  }
}

// One workgroup: thread t adds chunk sums t, t + NT, t + 2 NT, ... in order, then the NT
// partial sums combine by halving.  Writes out[0], info[0] (matched count), info[1] (status).
__global__ __launch_bounds__(kTraceFinishNT) void k_trace_finish(
    int64_t n_chunks, const double* __restrict__ part_sum, const uint32_t* __restrict__ part_hits,
    const uint32_t* __restrict__ part_flags, double* __restrict__ out,
    int32_t* __restrict__ info) {
  __shared__ double s_sum[kTraceFinishNT];
  __shared__ unsigned long long s_hits[kTraceFinishNT];
  __shared__ uint32_t s_flags;
  const int t = threadIdx.x;
  if (t == 0) s_flags = 0;
  __syncthreads();
  double sum = 0.0;
  unsigned long long hits = 0;
  uint32_t flags = 0;
  for (int64_t i = t; i < n_chunks; i += kTraceFinishNT) {
    sum += part_sum[i];
    hits += part_hits[i];
    flags |= part_flags[i];
  }
  s_sum[t] = sum;
  s_hits[t] = hits;
  if (flags) atomicOr(&s_flags, flags);
  __syncthreads();
  for (int s = kTraceFinishNT / 2; s >= 1; s >>= 1) {
    if (t < s) {
      s_sum[t] += s_sum[t + s];
      s_hits[t] += s_hits[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = s_sum[0];
    info[0] = (int32_t)(s_hits[0] > (unsigned long long)INT32_MAX ? INT32_MAX : s_hits[0]);
    info[1] = (s_flags & kFlagInval) ? (int32_t)SPM_EINVAL
              : (s_flags & kFlagBounds) ? (int32_t)SPM_EBOUNDS
                                        : (int32_t)SPM_OK;
  }
}

}  // namespace spm

namespace {

using namespace spm;

bool fits_i32(int64_t x) { return x >= 0 && x <= INT32_MAX; }
bool aligned256(const void* p) { return ((uintptr_t)p & 255) == 0; }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t trace_chunks(int64_t n_cols) { return (n_cols + kTraceChunk - 1) / kTraceChunk; }

// Workspace: chunk sums (binary64), matched counts and flags (uint32 each), 256-byte carved.
size_t trace_ws_bytes(int64_t n_cols, size_t* off_hits, size_t* off_flags) {
  const size_t m = (size_t)trace_chunks(n_cols);
  size_t off = align256(sizeof(double) * (m ? m : 1));
  *off_hits = off;
  off += align256(sizeof(uint32_t) * (m ? m : 1));
  *off_flags = off;
  off += align256(sizeof(uint32_t) * (m ? m : 1));
  return off;
}

// Group width from the longer operand's average column length (capacity-based): enough lanes
// to cover a typical column, at least 16 so that short columns still fill the chunk.
// The bitmap costs nw words of set-up per column: worth it once B's columns are long enough
// (average from the capacity) to make binary searches the larger cost.
bool trace_bitmap(int64_t n_rows, int64_t n_cols, int64_t b_cap) {
  const int64_t nw = (n_rows + 31) >> 5;
  return n_rows <= kTraceBmRows && 4 * (b_cap / (n_cols > 0 ? n_cols : 1)) >= nw;
}

// Lanes per column.  Sorted-row form: enough lanes for the LDS slice (19 GW rows) to hold a
// typical column.  Bitmap form: a lookup is cheap, so fewer lanes per column and more columns
// in flight win (measured on 10,000-row matrices: 16 lanes at about 100 elements per column,
// 32 at about 1,000).
int trace_group_width(int64_t n_rows, int64_t n_cols, int64_t a_cap, int64_t b_cap) {
  spm_tuning tu;
  if (spm_tuning_get(&tu) == SPM_OK && tu.trace_group_width != 0) return tu.trace_group_width;
  const int64_t cap = a_cap > b_cap ? a_cap : b_cap;
  const int64_t avg = n_cols > 0 ? cap / n_cols : 0;
  if (trace_bitmap(n_rows, n_cols, b_cap)) {
    if (avg >= 4096) return 64;
    if (avg >= 256) return 32;
    return 16;
  }
  if (avg >= 48) return 64;
  if (avg >= 12) return 32;
  return 16;
}

template <typename VT, int GW>
void launch_trace_gw(int64_t n_rows, int64_t n_cols, int64_t a_cap, const int32_t* a_cp,
                     const int32_t* a_ri, const VT* av, int64_t b_cap, const int32_t* b_cp,
                     const int32_t* b_ri, const VT* bv, double* ps, uint32_t* ph, uint32_t* pf,
                     hipStream_t s) {
  const dim3 grid((unsigned)trace_chunks(n_cols)), block(kTraceChunk * GW);
  const int nw = (int)((n_rows + 31) >> 5);
  if (trace_bitmap(n_rows, n_cols, b_cap)) {
    const int slice = (nw * 6 + 15) & ~15;  // nw words and nw 16-bit ranks, 16-byte aligned
    k_trace_atb<VT, GW, true><<<grid, block, (size_t)kTraceChunk * slice, s>>>(
        n_rows, n_cols, a_cap, a_cp, a_ri, av, b_cap, b_cp, b_ri, bv, ps, ph, pf, slice);
  } else {
    const int slice = kTraceLdsPerLane * GW * 4;
    k_trace_atb<VT, GW, false><<<grid, block, (size_t)kTraceChunk * slice, s>>>(
        n_rows, n_cols, a_cap, a_cp, a_ri, av, b_cap, b_cp, b_ri, bv, ps, ph, pf, slice);
  }
}

template <typename VT>
void launch_trace(int gw, int64_t n_rows, int64_t n_cols, int64_t a_cap, const int32_t* a_cp,
                  const int32_t* a_ri, const void* a_v, int64_t b_cap, const int32_t* b_cp,
                  const int32_t* b_ri, const void* b_v, double* ps, uint32_t* ph, uint32_t* pf,
                  hipStream_t s) {
  const VT* av = static_cast<const VT*>(a_v);
  const VT* bv = static_cast<const VT*>(b_v);
  if (gw == 64)
    launch_trace_gw<VT, 64>(n_rows, n_cols, a_cap, a_cp, a_ri, av, b_cap, b_cp, b_ri, bv, ps,
                            ph, pf, s);
  else if (gw == 32)
    launch_trace_gw<VT, 32>(n_rows, n_cols, a_cap, a_cp, a_ri, av, b_cap, b_cp, b_ri, bv, ps,
                            ph, pf, s);
  else
    launch_trace_gw<VT, 16>(n_rows, n_cols, a_cap, a_cp, a_ri, av, b_cap, b_cp, b_ri, bv, ps,
                            ph, pf, s);
}

}  // namespace

extern "C" {

spm_status spm_csc_trace_atb_workspace(int64_t n_cols, size_t* ws_bytes) {
  if (!ws_bytes || n_cols < 0) return SPM_EINVAL;
  if (!fits_i32(n_cols) || n_cols == INT32_MAX) return SPM_EOVERFLOW;
  size_t oh, of;
  *ws_bytes = trace_ws_bytes(n_cols, &oh, &of);
  return SPM_OK;
}

spm_status spm_csc_trace_atb(int64_t n_rows, int64_t n_cols, int64_t a_cap,
                             const int32_t* a_col_ptr, const int32_t* a_row_idx,
                             const void* a_val, int64_t b_cap, const int32_t* b_col_ptr,
                             const int32_t* b_row_idx, const void* b_val, spm_dtype val_type,
                             double* out, int32_t* info, void* ws, size_t ws_bytes,
                             void* stream) {
  SPM_RANGE("spm_csc_trace_atb");
  if (n_rows < 0 || n_cols < 0 || a_cap < 0 || b_cap < 0) return SPM_EINVAL;
  if (!fits_i32(n_rows) || !fits_i32(n_cols) || !fits_i32(a_cap) || !fits_i32(b_cap) ||
      n_rows == INT32_MAX || n_cols == INT32_MAX)
    return SPM_EOVERFLOW;
  if (val_type != SPM_F64 && val_type != SPM_F32) return SPM_EDTYPE;
  if (!a_col_ptr || !b_col_ptr || !out || !info || !ws) return SPM_EINVAL;
  if ((a_cap > 0 && (!a_row_idx || !a_val)) || (b_cap > 0 && (!b_row_idx || !b_val)))
    return SPM_EINVAL;
  if (!aligned256(ws)) return SPM_EINVAL;
  size_t oh, of;
  if (ws_bytes < trace_ws_bytes(n_cols, &oh, &of)) return SPM_EWORKSPACE;
  // One workgroup of kTraceChunk * gw lanes per chunk of columns: the launch's lane count
  // must stay below 2^32.  The lane count per column does not enter the summation order, so
  // a huge n_cols takes narrower groups first; beyond 16-lane groups the shape is rejected.
  int gw = n_cols > 0 ? trace_group_width(n_rows, n_cols, a_cap, b_cap) : 16;
  const uint64_t lanes_per_gw = (uint64_t)trace_chunks(n_cols) * kTraceChunk;
  while (gw > 16 && lanes_per_gw * (uint64_t)gw > 0xFFFFFFFFull) gw >>= 1;
  if (lanes_per_gw * (uint64_t)gw > 0xFFFFFFFFull) return SPM_EOVERFLOW;
  char* w = static_cast<char*>(ws);
  double* ps = reinterpret_cast<double*>(w);
  uint32_t* ph = reinterpret_cast<uint32_t*>(w + oh);
  uint32_t* pf = reinterpret_cast<uint32_t*>(w + of);
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  if (n_cols > 0) {
    if (val_type == SPM_F64)
      launch_trace<double>(gw, n_rows, n_cols, a_cap, a_col_ptr, a_row_idx, a_val, b_cap,
                           b_col_ptr, b_row_idx, b_val, ps, ph, pf, s);
    else
      launch_trace<float>(gw, n_rows, n_cols, a_cap, a_col_ptr, a_row_idx, a_val, b_cap,
                          b_col_ptr, b_row_idx, b_val, ps, ph, pf, s);
  }
  k_trace_finish<<<dim3(1), dim3(kTraceFinishNT), 0, s>>>(trace_chunks(n_cols), ps, ph, pf,
                                                          out, info);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPM_OK : SPM_EHIP;
}

}  // extern "C"
