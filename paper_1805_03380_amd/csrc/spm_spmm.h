// CSC sparse x dense products on gfx950: the forward product Y = A.X through the plan (row
// index) of A's pattern, and the fused adjoint (dX = A^T.G, dval = G.X^T on A's pattern) by a
// walk down each CSC column.  Bandwidth-bound (about 0.5 flop per byte): no matrix cores;
// every nonzero's dense row is read as coalesced 16-byte vectors by a group of lanes.
//
// Result ordering does not depend on the launch shape:
//   * a group of G lanes serves one output row (forward) or one column (adjoint), each lane
//     owning 4 consecutive dense columns; G depends on k alone (group_width);
//   * every Y / dX element is ONE accumulator updated with fma in ascending column (forward)
//     or ascending row (adjoint) order, starting from 0;
//   * dval[p]: each lane folds its 4-element pieces with fma in ascending j, then the group's
//     lane partials are combined by a fixed tree (group_sum).
// The batched kernel calls the same device functions, so its results are bitwise equal.
#pragma once

#include <type_traits>

#include "spm_device.h"

namespace spm {

// Lanes per row: next power of two >= ceil(k/4), capped at one wavefront.
__host__ __device__ inline int group_width(int64_t k) {
  int64_t need = (k + 3) / 4;
  int g = 1;
  while (g < need && g < kWave) g <<= 1;
  return g;
}

// Accumulator type of a product over operands of element types VT, GT, XT: binary64 when
// any operand is binary64, else binary32 when any is bfloat16, else binary64.
template <typename VT, typename GT, typename XT>
struct AccOf {
  static constexpr bool any64 = std::is_same<VT, double>::value ||
                                std::is_same<GT, double>::value ||
                                std::is_same<XT, double>::value;
  static constexpr bool any16 = std::is_same<VT, bf16_t>::value ||
                                std::is_same<GT, bf16_t>::value ||
                                std::is_same<XT, bf16_t>::value;
  using type = typename std::conditional<!any64 && any16, float, double>::type;
};

template <typename ACC>
__device__ __forceinline__ ACC fma_acc(ACC a, ACC b, ACC c);
template <>
__device__ __forceinline__ double fma_acc<double>(double a, double b, double c) {
  return __fma_rn(a, b, c);
}
template <>
__device__ __forceinline__ float fma_acc<float>(float a, float b, float c) {
  return __fmaf_rn(a, b, c);
}

// ------------------------------------------------------------------------------------------
// Sum of one value over the GW lanes of an aligned lane group (GW a power of two <= 64),
// returned in every lane of the group.  Within a 16-lane DPP row the steps are: swap
// neighbours, swap pairs, mirror each half-row, mirror the row (each step adds the lane's
// partner, so after step s all lanes of a 2^s block hold that block's sum); across rows an
// xor exchange.  The tree is fixed by GW alone.
// ------------------------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL, typename T> __device__ __forceinline__ T dpp_mov(T x);
template <> __device__ __forceinline__ float dpp_mov<0xB1, float>(float x) { return dpp_f32<0xB1>(x); }
template <> __device__ __forceinline__ float dpp_mov<0x4E, float>(float x) { return dpp_f32<0x4E>(x); }
template <> __device__ __forceinline__ float dpp_mov<0x141, float>(float x) { return dpp_f32<0x141>(x); }
template <> __device__ __forceinline__ float dpp_mov<0x140, float>(float x) { return dpp_f32<0x140>(x); }
template <> __device__ __forceinline__ double dpp_mov<0xB1, double>(double x) { return dpp_f64<0xB1>(x); }
template <> __device__ __forceinline__ double dpp_mov<0x4E, double>(double x) { return dpp_f64<0x4E>(x); }
template <> __device__ __forceinline__ double dpp_mov<0x141, double>(double x) { return dpp_f64<0x141>(x); }
template <> __device__ __forceinline__ double dpp_mov<0x140, double>(double x) { return dpp_f64<0x140>(x); }

template <int GW, typename ACC>
__device__ __forceinline__ ACC group_sum(ACC d) {
  if (GW >= 2) d += dpp_mov<0xB1, ACC>(d);   // quad_perm [1,0,3,2]
  if (GW >= 4) d += dpp_mov<0x4E, ACC>(d);   // quad_perm [2,3,0,1]
  if (GW >= 8) d += dpp_mov<0x141, ACC>(d);  // row_half_mirror
  if (GW >= 16) d += dpp_mov<0x140, ACC>(d); // row_mirror
  if (GW >= 32) d += __shfl_xor(d, 16, kWave);
  if (GW >= 64) d += __shfl_xor(d, 32, kWave);
  return d;
}

// One exchange step of the lane tree: the partner lane differs in lane bit B (and, for the
// mirrors, in the bits below it).
template <int B, typename ACC>
__device__ __forceinline__ ACC exch(ACC x) {
  if constexpr (B == 0) return dpp_mov<0xB1, ACC>(x);        // quad_perm [1,0,3,2]
  else if constexpr (B == 1) return dpp_mov<0x4E, ACC>(x);   // quad_perm [2,3,0,1]
  else if constexpr (B == 2) return dpp_mov<0x141, ACC>(x);  // row_half_mirror
  else if constexpr (B == 3) return dpp_mov<0x140, ACC>(x);  // row_mirror
  else if constexpr (B == 4) return __shfl_xor(x, 16, kWave);
  else return __shfl_xor(x, 32, kWave);
}

template <int B, typename ACC>
__device__ __forceinline__ ACC exch_sum_down(ACC f) {
  if constexpr (B >= 0) {
    f += exch<B, ACC>(f);
    return exch_sum_down<B - 1, ACC>(f);
  } else {
    return f;
  }
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// Sums of four values d[0..3] over the GW >= 4 lanes of a group, transposed: the exchanges on
// the two highest lane bits A and B each keep half of the values (bit A picks {0,1} or
// {2,3}, bit B one of the pair), the remaining exchanges carry one value, so lane lg ends
// with the group sum of value v = 2*bit_A + bit_B after log2(GW) + 1 exchanges instead of
// 4*log2(GW).  The tree is fixed by GW alone; lanes whose bits below B are zero hold one of
// the four sums each.
template <int GW, typename ACC>
__device__ __forceinline__ ACC group_sum4(const ACC (&d)[4], int lg, int& v) {
  static_assert(GW >= 4 && GW <= 64, "four values need at least four lanes");
  constexpr int A = ilog2(GW) - 1, B = ilog2(GW) - 2;
  const bool ba = (lg >> A) & 1, bb = (lg >> B) & 1;
  const ACC e0 = (ba ? d[2] : d[0]) + exch<A, ACC>(ba ? d[0] : d[2]);
  const ACC e1 = (ba ? d[3] : d[1]) + exch<A, ACC>(ba ? d[1] : d[3]);
  const ACC f = (bb ? e1 : e0) + exch<B, ACC>(bb ? e0 : e1);
  v = 2 * (int)ba + (int)bb;
  return exch_sum_down<B - 1, ACC>(f);
}

// ------------------------------------------------------------------------------------------
// Forward: Y[r, :] for one row r by the GW lanes of a group (lane lg).  Each lane owns the
// 4-element pieces j0 = (m*GW + lg)*4; for every piece it walks the row's stored elements in
// ascending column order, U at a time (their indices, values and dense pieces all in flight
// before the fma chain consumes them).  FULL: k == 4*GW with aligned rows (one vector piece
// per lane, no tail handling).  A plan entry whose column or slot is out of range (only
// possible for a plan not built from a valid CSC) contributes nothing and is not followed.
// ------------------------------------------------------------------------------------------
constexpr int kU = 4;

// One aligned 4-element vector of row `r` (always a valid row), widened; the caller zeroes
// the contribution of invalid entries with selects, so the loop has no divergent branches.
template <typename ACC>
__device__ __forceinline__ void vload4(const float* __restrict__ p, ACC (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = (ACC)v.x; o[1] = (ACC)v.y; o[2] = (ACC)v.z; o[3] = (ACC)v.w;
}
template <typename ACC>
__device__ __forceinline__ void vload4(const double* __restrict__ p, ACC (&o)[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0];
  const double2 b = reinterpret_cast<const double2*>(p)[1];
  o[0] = (ACC)a.x; o[1] = (ACC)a.y; o[2] = (ACC)b.x; o[3] = (ACC)b.y;
}
template <typename ACC>
__device__ __forceinline__ void vload4(const bf16_t* __restrict__ p, ACC (&o)[4]) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  o[0] = (ACC)__uint_as_float(v.x << 16);
  o[1] = (ACC)__uint_as_float(v.x & 0xffff0000u);
  o[2] = (ACC)__uint_as_float(v.y << 16);
  o[3] = (ACC)__uint_as_float(v.y & 0xffff0000u);
}

// Forward, full aligned pieces (k == 4*GW): lane lg owns columns [4 lg, 4 lg + 4).  PV: the
// values are in plan order (val[q], read contiguously) instead of CSC order (val[perm[q]]).
template <typename VT, typename XT, typename ACC, int GW, bool PV = false>
__device__ __forceinline__ void spmm_row_full(int64_t r, int lg, int64_t n_cols, int64_t nnz_cap,
                                              const int32_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col_t,
                                              const int32_t* __restrict__ perm,
                                              const VT* __restrict__ val,
                                              const XT* __restrict__ X, int64_t ldx,
                                              void* __restrict__ Y, int64_t ldy, bool y_f64) {
  int64_t q0 = row_ptr[r], q1 = row_ptr[r + 1];
  q0 = q0 < 0 ? 0 : (q0 > nnz_cap ? nnz_cap : q0);
  q1 = q1 < q0 ? q0 : (q1 > nnz_cap ? nnz_cap : q1);
  const XT* Xl = X + (int64_t)lg * 4;
  ACC acc[4] = {(ACC)0, (ACC)0, (ACC)0, (ACC)0};
  int64_t q = q0;
  for (; q + kU <= q1; q += kU) {
    int32_t c[kU], pp[kU];
    bool ok[kU];
    ACC v[kU];
    ACC x[kU][4];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      c[u] = col_t[q + u];
      pp[u] = PV ? (int32_t)(q + u) : perm[q + u];
      ok[u] = (uint32_t)c[u] < (uint64_t)n_cols && (uint32_t)pp[u] < (uint64_t)nnz_cap;
      c[u] = ok[u] ? c[u] : 0;
      pp[u] = ok[u] ? pp[u] : 0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = to_acc<ACC>(val[pp[u]]);
#pragma unroll
    for (int u = 0; u < kU; ++u) vload4<ACC>(Xl + (int64_t)c[u] * ldx, x[u]);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const ACC t = fma_acc<ACC>(v[u], x[u][e], acc[e]);
        acc[e] = ok[u] ? t : acc[e];
      }
    }
  }
  for (; q < q1; ++q) {
    int32_t c = col_t[q], pq = PV ? (int32_t)q : perm[q];
    const bool ok = (uint32_t)c < (uint64_t)n_cols && (uint32_t)pq < (uint64_t)nnz_cap;
    c = ok ? c : 0;
    pq = ok ? pq : 0;
    const ACC v = to_acc<ACC>(val[pq]);
    ACC x[4];
    vload4<ACC>(Xl + (int64_t)c * ldx, x);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const ACC t = fma_acc<ACC>(v, x[e], acc[e]);
      acc[e] = ok ? t : acc[e];
    }
  }
  store_n<ACC>(Y, r * ldy + (int64_t)lg * 4, 4, y_f64, true, acc);
}

// Adjoint, full aligned pieces (k == 4*GW).  G (GT) and X (XT) have element types of their
// own: a binary64 G is read as binary64, never narrowed to X's type.
template <typename VT, typename GT, typename XT, typename ACC, int GW>
__device__ __forceinline__ void spmm_col_bwd_full(int64_t c, int64_t p0, int64_t p1, int lg,
                                                  int64_t n_rows,
                                                  const int32_t* __restrict__ row_idx,
                                                  const VT* __restrict__ val,
                                                  const GT* __restrict__ Gm, int64_t ldg,
                                                  const XT* __restrict__ X, int64_t ldx,
                                                  void* __restrict__ dX, int64_t lddx,
                                                  bool dx_f64, void* __restrict__ dval,
                                                  bool dv_f64) {
  static_assert(kU == 4, "the dvalues store selects among four sums");
  const GT* Gl = Gm + (int64_t)lg * 4;
  ACC x[4];
  vload4<ACC>(X + c * ldx + (int64_t)lg * 4, x);
  ACC dx[4] = {(ACC)0, (ACC)0, (ACC)0, (ACC)0};
  int64_t p = p0;
  for (; p + kU <= p1; p += kU) {
    int32_t r[kU];
    bool ok[kU];
    ACC v[kU];
    ACC g[kU][4];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      r[u] = row_idx[p + u];
      ok[u] = r[u] >= 0 && (int64_t)r[u] < n_rows;
      r[u] = ok[u] ? r[u] : 0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = to_acc<ACC>(val[p + u]);
#pragma unroll
    for (int u = 0; u < kU; ++u) vload4<ACC>(Gl + (int64_t)r[u] * ldg, g[u]);
    ACC d[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        g[u][e] = ok[u] ? g[u][e] : (ACC)0;
        dx[e] = fma_acc<ACC>(v[u], g[u][e], dx[e]);
      }
      d[u] = (ACC)0;
#pragma unroll
      for (int e = 0; e < 4; ++e) d[u] = fma_acc<ACC>(g[u][e], x[e], d[u]);
    }
    if (dval) {
      if constexpr (GW >= kU) {
        // the kU group sums together (group_sum4); the lanes holding them store the kU
        // consecutive dvalues with one store instruction
        int vi;
        const ACC dv = group_sum4<GW, ACC>(d, lg, vi);
        if ((lg & ((GW / kU) - 1)) == 0) {
          if (dv_f64) static_cast<double*>(dval)[p + vi] = (double)dv;
          else static_cast<float*>(dval)[p + vi] = (float)dv;
        }
      } else {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const ACC su = group_sum<GW, ACC>(d[u]);
          if (lg == 0) {
            if (dv_f64) static_cast<double*>(dval)[p + u] = (double)su;
            else static_cast<float*>(dval)[p + u] = (float)su;
          }
        }
      }
    }
  }
  for (; p < p1; ++p) {
    int32_t r = row_idx[p];
    const bool ok = r >= 0 && (int64_t)r < n_rows;
    r = ok ? r : 0;
    const ACC v = to_acc<ACC>(val[p]);
    ACC g[4];
    vload4<ACC>(Gl + (int64_t)r * ldg, g);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      g[e] = ok ? g[e] : (ACC)0;
      dx[e] = fma_acc<ACC>(v, g[e], dx[e]);
    }
    if (dval) {
      ACC d = (ACC)0;
#pragma unroll
      for (int e = 0; e < 4; ++e) d = fma_acc<ACC>(g[e], x[e], d);
      d = group_sum<GW, ACC>(d);
      if (lg == 0) {
        if (dv_f64) static_cast<double*>(dval)[p] = (double)d;
        else static_cast<float*>(dval)[p] = (float)d;
      }
    }
  }
  if (dX) store_n<ACC>(dX, c * lddx + (int64_t)lg * 4, 4, dx_f64, true, dx);
}

template <typename VT, typename XT, typename ACC, int GW, bool FULL>
__device__ __forceinline__ void spmm_row(int64_t r, int lg, int64_t k, int64_t n_cols,
                                         int64_t nnz_cap,
                                         const int32_t* __restrict__ row_ptr,
                                         const int32_t* __restrict__ col_t,
                                         const int32_t* __restrict__ perm,
                                         const VT* __restrict__ val, const XT* __restrict__ X,
                                         int64_t ldx, bool xal, void* __restrict__ Y,
                                         int64_t ldy, bool y_f64, bool yal) {
  int64_t q0 = row_ptr[r], q1 = row_ptr[r + 1];
  q0 = q0 < 0 ? 0 : (q0 > nnz_cap ? nnz_cap : q0);
  q1 = q1 < q0 ? q0 : (q1 > nnz_cap ? nnz_cap : q1);
  const int nch = FULL ? 1 : (int)((k + 4 * GW - 1) / (4 * GW));
  for (int m = 0; m < nch; ++m) {
    const int64_t j0 = ((int64_t)m * GW + lg) * 4;
    const int avail = FULL ? 4 : (int)((k - j0) < 0 ? 0 : ((k - j0) < 4 ? (k - j0) : 4));
    if (!FULL && avail <= 0) break;
    const bool al = FULL ? true : xal;
    ACC acc[4] = {(ACC)0, (ACC)0, (ACC)0, (ACC)0};
    int64_t q = q0;
    for (; q + kU <= q1; q += kU) {
      int32_t c[kU], pp[kU];
      bool ok[kU];
      ACC v[kU];
      ACC x[kU][4];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        c[u] = col_t[q + u];
        pp[u] = perm ? perm[q + u] : (int32_t)(q + u);
        ok[u] = (uint32_t)c[u] < (uint64_t)n_cols && (uint32_t)pp[u] < (uint64_t)nnz_cap;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) v[u] = ok[u] ? to_acc<ACC>(val[pp[u]]) : (ACC)0;
#pragma unroll
      for (int u = 0; u < kU; ++u)
        load4<ACC>(X + (int64_t)(ok[u] ? c[u] : 0) * ldx + j0, ok[u] ? avail : 0, al, x[u]);
#pragma unroll
      for (int u = 0; u < kU; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = fma_acc<ACC>(v[u], x[u][e], acc[e]);
    }
    for (; q < q1; ++q) {
      const int32_t c = col_t[q], pq = perm ? perm[q] : (int32_t)q;
      const bool ok = (uint32_t)c < (uint64_t)n_cols && (uint32_t)pq < (uint64_t)nnz_cap;
      const ACC v = ok ? to_acc<ACC>(val[pq]) : (ACC)0;
      ACC x[4];
      load4<ACC>(X + (int64_t)(ok ? c : 0) * ldx + j0, ok ? avail : 0, al, x);
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] = fma_acc<ACC>(v, x[e], acc[e]);
    }
    store_n<ACC>(Y, r * ldy + j0, avail, y_f64, FULL ? true : yal, acc);
  }
}

// ------------------------------------------------------------------------------------------
// Adjoint for one column c by the GW lanes of a group (p range already clamped): X[c, piece]
// is loaded once per piece; for every stored element p (ascending row) the lane's G-row piece
// updates dX with one fma chain per output and contributes a 4-term partial (fma, ascending j)
// to dval[p]; the group sums the partials with group_sum and its first lane stores dval[p].
// When k > 4*GW a lane owns several pieces; its dval partial then runs over its pieces in
// order before the group sum.
// ------------------------------------------------------------------------------------------
template <typename VT, typename GT, typename XT, typename ACC, int GW, bool FULL>
__device__ __forceinline__ void spmm_col_bwd(int64_t c, int64_t p0, int64_t p1, int lg,
                                             int64_t k, int64_t n_rows,
                                             const int32_t* __restrict__ row_idx,
                                             const VT* __restrict__ val,
                                             const GT* __restrict__ Gm, int64_t ldg, bool gal,
                                             const XT* __restrict__ X, int64_t ldx, bool xal,
                                             void* __restrict__ dX, int64_t lddx, bool dx_f64,
                                             bool dxal, void* __restrict__ dval, bool dv_f64) {
  const int nch = FULL ? 1 : (int)((k + 4 * GW - 1) / (4 * GW));
  if (nch == 1) {
    const int64_t j0 = (int64_t)lg * 4;
    const int avail = FULL ? 4 : (int)((k - j0) < 0 ? 0 : ((k - j0) < 4 ? (k - j0) : 4));
    const bool gl = FULL ? true : gal;
    ACC x[4];
    load4<ACC>(X + c * ldx + j0, avail, FULL ? true : xal, x);
    ACC dx[4] = {(ACC)0, (ACC)0, (ACC)0, (ACC)0};
    int64_t p = p0;
    for (; p + kU <= p1; p += kU) {
      int32_t r[kU];
      ACC v[kU];
      ACC g[kU][4];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        r[u] = row_idx[p + u];
        if (r[u] < 0 || (int64_t)r[u] >= n_rows) r[u] = -1;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) v[u] = to_acc<ACC>(val[p + u]);
#pragma unroll
      for (int u = 0; u < kU; ++u)
        load4<ACC>(Gm + (int64_t)(r[u] < 0 ? 0 : r[u]) * ldg + j0, r[u] < 0 ? 0 : avail, gl,
                   g[u]);
#pragma unroll
      for (int u = 0; u < kU; ++u) {
#pragma unroll
        for (int e = 0; e < 4; ++e) dx[e] = fma_acc<ACC>(v[u], g[u][e], dx[e]);
        if (dval) {
          ACC d = (ACC)0;
#pragma unroll
          for (int e = 0; e < 4; ++e) d = fma_acc<ACC>(g[u][e], x[e], d);
          d = group_sum<GW, ACC>(d);
          if (lg == 0) {
            if (dv_f64) static_cast<double*>(dval)[p + u] = (double)d;
            else static_cast<float*>(dval)[p + u] = (float)d;
          }
        }
      }
    }
    for (; p < p1; ++p) {
      int32_t r = row_idx[p];
      if (r < 0 || (int64_t)r >= n_rows) r = -1;
      const ACC v = to_acc<ACC>(val[p]);
      ACC g[4];
      load4<ACC>(Gm + (int64_t)(r < 0 ? 0 : r) * ldg + j0, r < 0 ? 0 : avail, gl, g);
#pragma unroll
      for (int e = 0; e < 4; ++e) dx[e] = fma_acc<ACC>(v, g[e], dx[e]);
      if (dval) {
        ACC d = (ACC)0;
#pragma unroll
        for (int e = 0; e < 4; ++e) d = fma_acc<ACC>(g[e], x[e], d);
        d = group_sum<GW, ACC>(d);
        if (lg == 0) {
          if (dv_f64) static_cast<double*>(dval)[p] = (double)d;
          else static_cast<float*>(dval)[p] = (float)d;
        }
      }
    }
    if (dX && avail > 0)
      store_n<ACC>(dX, c * lddx + j0, avail, dx_f64, FULL ? true : dxal, dx);
    return;
  }
  // several 4-element pieces per lane
  if (dX) {
    for (int m = 0; m < nch; ++m) {
      const int64_t j0 = ((int64_t)m * GW + lg) * 4;
      if (j0 >= k) break;
      const int avail = (int)((k - j0) < 4 ? (k - j0) : 4);
      ACC dx[4] = {(ACC)0, (ACC)0, (ACC)0, (ACC)0};
      for (int64_t p = p0; p < p1; ++p) {
        const int32_t r = row_idx[p];
        if (r < 0 || (int64_t)r >= n_rows) continue;
        const ACC v = to_acc<ACC>(val[p]);
        ACC g[4];
        load4<ACC>(Gm + (int64_t)r * ldg + j0, avail, gal, g);
#pragma unroll
        for (int e = 0; e < 4; ++e) dx[e] = fma_acc<ACC>(v, g[e], dx[e]);
      }
      store_n<ACC>(dX, c * lddx + j0, avail, dx_f64, dxal, dx);
    }
  }
  if (dval) {
    for (int64_t p = p0; p < p1; ++p) {
      int32_t r = row_idx[p];
      if (r < 0 || (int64_t)r >= n_rows) r = -1;
      ACC d = (ACC)0;
      for (int m = 0; m < nch; ++m) {
        const int64_t j0 = ((int64_t)m * GW + lg) * 4;
        const int avail = (r < 0 || j0 >= k) ? 0 : (int)((k - j0) < 4 ? (k - j0) : 4);
        ACC g[4], x[4];
        load4<ACC>(Gm + (int64_t)(r < 0 ? 0 : r) * ldg + (avail ? j0 : 0), avail, gal, g);
        load4<ACC>(X + c * ldx + (avail ? j0 : 0), avail, xal, x);
#pragma unroll
        for (int e = 0; e < 4; ++e) d = fma_acc<ACC>(g[e], x[e], d);
      }
      d = group_sum<GW, ACC>(d);
      if (lg == 0) {
        if (dv_f64) static_cast<double*>(dval)[p] = (double)d;
        else static_cast<float*>(dval)[p] = (float)d;
      }
    }
  }
}

// perm == nullptr (general path) or PV (full path): values in plan order.
template <typename VT, typename XT, typename ACC, int GW, bool FULL, bool PV>
__global__ __launch_bounds__(256) void k_spmm_fwd(int64_t n_rows, int64_t n_cols, int64_t nnz_cap,
                                                  int64_t k, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col_t,
                                                  const int32_t* __restrict__ perm,
                                                  const VT* __restrict__ val,
                                                  const XT* __restrict__ X, int64_t ldx,
                                                  int xal, void* __restrict__ Y, int64_t ldy,
                                                  int y_f64, int yal) {
  const int lg = threadIdx.x & (GW - 1);
  const int64_t groups_per_block = blockDim.x / GW;
  const int64_t ngroups = (int64_t)gridDim.x * groups_per_block;
  for (int64_t r = (int64_t)blockIdx.x * groups_per_block + threadIdx.x / GW; r < n_rows;
       r += ngroups)
    if constexpr (FULL)
      spmm_row_full<VT, XT, ACC, GW, PV>(r, lg, n_cols, nnz_cap, row_ptr, col_t, perm, val, X,
                                         ldx, Y, ldy, y_f64 != 0);
    else
      spmm_row<VT, XT, ACC, GW, false>(r, lg, k, n_cols, nnz_cap, row_ptr, col_t, perm, val, X,
                                       ldx, xal != 0, Y, ldy, y_f64 != 0, yal != 0);
}

// Waves per SIMD asked of the compiler for the adjoint (1: no request).  At 32 lanes per
// column (k = 128) six waves, with a few spilled registers, measured faster than the five the
// compiler picks on its own (power-law workload: 1.64 against 1.67 ms; seven and eight waves
// spill more and took 2.9 and 3.8 ms).  At 16 lanes a request lost (66 against 52 µs).
template <int GW> constexpr int kBwdWaves = GW == 32 ? 6 : 1;
template <typename VT, typename GT, typename XT, typename ACC, int GW, bool FULL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kBwdWaves<GW>))) void k_spmm_bwd(int64_t n_rows, int64_t n_cols, int64_t nnz_cap,
                                                  int64_t k, const int32_t* __restrict__ col_ptr,
                                                  const int32_t* __restrict__ row_idx,
                                                  const VT* __restrict__ val,
                                                  const GT* __restrict__ Gm, int64_t ldg, int gal,
                                                  const XT* __restrict__ X, int64_t ldx, int xal,
                                                  void* __restrict__ dX, int64_t lddx, int dx_f64,
                                                  int dxal, void* __restrict__ dval, int dv_f64) {
  const int lg = threadIdx.x & (GW - 1);
  const int64_t groups_per_block = blockDim.x / GW;
  const int64_t ngroups = (int64_t)gridDim.x * groups_per_block;
  const int64_t raw = col_ptr[n_cols];
  const int64_t nnz = raw < 0 ? 0 : (raw > nnz_cap ? nnz_cap : raw);
  for (int64_t c = (int64_t)blockIdx.x * groups_per_block + threadIdx.x / GW; c < n_cols;
       c += ngroups) {
    int64_t p0 = col_ptr[c], p1 = col_ptr[c + 1];
    p0 = p0 < 0 ? 0 : (p0 > nnz ? nnz : p0);
    p1 = p1 < p0 ? p0 : (p1 > nnz ? nnz : p1);
    if constexpr (FULL)
      spmm_col_bwd_full<VT, GT, XT, ACC, GW>(c, p0, p1, lg, n_rows, row_idx, val, Gm, ldg, X, ldx,
                                         dX, lddx, dx_f64 != 0, dval, dv_f64 != 0);
    else
      spmm_col_bwd<VT, GT, XT, ACC, GW, false>(c, p0, p1, lg, k, n_rows, row_idx, val, Gm, ldg,
                                           gal != 0, X, ldx, xal != 0, dX, lddx, dx_f64 != 0,
                                           dxal != 0, dval, dv_f64 != 0);
  }
}

}  // namespace spm
