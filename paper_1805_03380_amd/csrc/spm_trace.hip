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

namespace spm {

constexpr int kTraceNT = 256;        // threads per workgroup of the column kernel
constexpr int kTraceChunk = 16;      // columns per workgroup (one partial sum each)
constexpr int kTraceVL = 64;         // virtual lanes per column
constexpr int kTraceFinishNT = 256;  // threads of the single finishing workgroup

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

// One workgroup per chunk of kTraceChunk columns; groups of GW lanes walk its columns.
// Writes the chunk's sum, matched count and status flags at index blockIdx.x.
template <typename VT, int GW>
__global__ __launch_bounds__(kTraceNT) void k_trace_atb(
    int64_t n_rows, int64_t n_cols, int64_t a_cap, const int32_t* __restrict__ a_col_ptr,
    const int32_t* __restrict__ a_row_idx, const VT* __restrict__ a_val, int64_t b_cap,
    const int32_t* __restrict__ b_col_ptr, const int32_t* __restrict__ b_row_idx,
    const VT* __restrict__ b_val, double* __restrict__ part_sum,
    uint32_t* __restrict__ part_hits, uint32_t* __restrict__ part_flags) {
  constexpr int G = kTraceNT / GW;  // columns in flight per workgroup
  constexpr int A = kTraceVL / GW;  // virtual lanes per physical lane
  static_assert(G <= kTraceChunk && kTraceChunk % G == 0, "groups tile the chunk");
  __shared__ double s_col[kTraceChunk];
  __shared__ uint32_t s_hits[kTraceChunk];
  __shared__ uint32_t s_flags;
  const int lg = threadIdx.x % GW;
  const int g = threadIdx.x / GW;
  const int64_t c0 = (int64_t)blockIdx.x * kTraceChunk;
  if (threadIdx.x == 0) s_flags = 0;
  __syncthreads();
  uint32_t flags = 0;
  for (int ci = g; ci < kTraceChunk; ci += G) {
    const int64_t c = c0 + ci;
    double acc[A];
#pragma unroll
    for (int a = 0; a < A; ++a) acc[a] = 0.0;
    uint32_t hits = 0;
    if (c < n_cols) {
      const int64_t pa0 = a_col_ptr[c], pa1 = a_col_ptr[c + 1];
      const int64_t pb0 = b_col_ptr[c], pb1 = b_col_ptr[c + 1];
      bool ok = pa0 >= 0 && pa0 <= pa1 && pa1 <= a_cap && pb0 >= 0 && pb0 <= pb1 &&
                pb1 <= b_cap;
      if (c == 0 && (pa0 != 0 || pb0 != 0)) ok = false;
      if (!ok) {
        flags |= kFlagInval;
      } else {
        // B's column: rows inside the matrix and strictly increasing
        for (int64_t q = pb0 + lg; q < pb1; q += GW) {
          const int32_t rb = b_row_idx[q];
          if (rb < 0 || (int64_t)rb >= n_rows) flags |= kFlagBounds;
          if (q > pb0 && b_row_idx[q - 1] >= rb) flags |= kFlagInval;
        }
        // A's column: element j = p - pa0 goes to virtual lane j mod 64, which is this
        // lane's accumulator (j / GW) mod A
        int a = 0;
        for (int64_t p = pa0 + lg; p < pa1; p += GW) {
          const int32_t r = a_row_idx[p];
          if (r < 0 || (int64_t)r >= n_rows) flags |= kFlagBounds;
          if (p > pa0 && a_row_idx[p - 1] >= r) flags |= kFlagInval;
          const int64_t q = lower_row(b_row_idx, pb0, pb1, r);
          if (q < pb1 && b_row_idx[q] == r) {
            const double prod = widen_val(a_val[p]) * widen_val(b_val[q]);
#pragma unroll
            for (int u = 0; u < A; ++u)
              if (u == a) acc[u] += prod;
            ++hits;
          }
          a = (a + 1 == A) ? 0 : a + 1;
        }
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
  }
  if (flags) atomicOr(&s_flags, flags);
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    uint32_t h = 0;
    for (int ci = 0; ci < kTraceChunk; ++ci) {
      sum += s_col[ci];
      h += s_hits[ci];
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
int trace_group_width(int64_t n_cols, int64_t a_cap, int64_t b_cap) {
  spm_tuning tu;
  if (spm_tuning_get(&tu) == SPM_OK && tu.trace_group_width != 0) return tu.trace_group_width;
  const int64_t cap = a_cap > b_cap ? a_cap : b_cap;
  const int64_t avg = n_cols > 0 ? cap / n_cols : 0;
  if (avg >= 48) return 64;
  if (avg >= 12) return 32;
  return 16;
}

template <typename VT>
void launch_trace(int gw, int64_t n_rows, int64_t n_cols, int64_t a_cap, const int32_t* a_cp,
                  const int32_t* a_ri, const void* a_v, int64_t b_cap, const int32_t* b_cp,
                  const int32_t* b_ri, const void* b_v, double* ps, uint32_t* ph, uint32_t* pf,
                  hipStream_t s) {
  const dim3 grid((unsigned)trace_chunks(n_cols)), block(kTraceNT);
  const VT* av = static_cast<const VT*>(a_v);
  const VT* bv = static_cast<const VT*>(b_v);
  if (gw == 64)
    k_trace_atb<VT, 64><<<grid, block, 0, s>>>(n_rows, n_cols, a_cap, a_cp, a_ri, av, b_cap,
                                               b_cp, b_ri, bv, ps, ph, pf);
  else if (gw == 32)
    k_trace_atb<VT, 32><<<grid, block, 0, s>>>(n_rows, n_cols, a_cap, a_cp, a_ri, av, b_cap,
                                               b_cp, b_ri, bv, ps, ph, pf);
  else
    k_trace_atb<VT, 16><<<grid, block, 0, s>>>(n_rows, n_cols, a_cap, a_cp, a_ri, av, b_cap,
                                               b_cp, b_ri, bv, ps, ph, pf);
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
  char* w = static_cast<char*>(ws);
  double* ps = reinterpret_cast<double*>(w);
  uint32_t* ph = reinterpret_cast<uint32_t*>(w + oh);
  uint32_t* pf = reinterpret_cast<uint32_t*>(w + of);
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  if (n_cols > 0) {
    const int gw = trace_group_width(n_cols, a_cap, b_cap);
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
