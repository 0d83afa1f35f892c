// Gradient with respect to each input triplet's value, for assembly followed by Y = A.X and a
// loss with dL/dY = G.  Assembly makes A[r,c] the sum of the values of the triplets at (r, c)
// (Fig. 1's +=; a zero sum is only not stored), so every triplet at (r, c) has
//     dL/dv_t = sum_j G[r,j] * X[c,j],
// duplicates share it, a location that summed to zero still has it, and a triplet outside the
// matrix (skipped by assembly) has 0.  This is an SDDMM over the triplet list: one gather of
// a G row and an X row per triplet, bandwidth-bound, no matrix cores.
//
// Summation order, as for the adjoint's dvalues: each lane of a group of GW lanes
// (group_width(k)) owns the 4-element pieces (m GW + lane) * 4 and folds them with fma in
// ascending m, then ascending element; the group's lane partials combine by group_sum's fixed
// tree.  It depends on k alone, never on the launch shape.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "spm.h"
#include "spm_range.h"
#include "spm_spmm.h"

namespace spm {

constexpr int kTgNT = 256;  // threads per workgroup
constexpr int kTgU = 4;     // triplets per group in flight

template <typename GT, typename XT, typename ACC, int GW>
__global__ __launch_bounds__(kTgNT) void k_triplet_grad(
    int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k, const int32_t* __restrict__ row,
    const int32_t* __restrict__ col, const GT* __restrict__ Gm, int64_t ldg, bool gal,
    const XT* __restrict__ X, int64_t ldx, bool xal, void* __restrict__ dv, bool dv_f64) {
  constexpr int NG = kTgNT / GW;  // groups per workgroup
  const int lg = threadIdx.x % GW;
  const int nch = (int)((k + 4 * GW - 1) / (4 * GW));
  const int64_t stride = (int64_t)gridDim.x * NG * kTgU;
  for (int64_t t0 = ((int64_t)blockIdx.x * NG + threadIdx.x / GW) * kTgU; t0 < nnz_in;
       t0 += stride) {
    int32_t r[kTgU], c[kTgU];
    bool ok[kTgU];
#pragma unroll
    for (int u = 0; u < kTgU; ++u) {
      const int64_t t = t0 + u;
      r[u] = t < nnz_in ? row[t] : -1;
      c[u] = t < nnz_in ? col[t] : -1;
      ok[u] = r[u] >= 0 && c[u] >= 0 && (int64_t)r[u] < n_rows && (int64_t)c[u] < n_cols;
    }
    ACC d[kTgU];
#pragma unroll
    for (int u = 0; u < kTgU; ++u) d[u] = (ACC)0;
    for (int m = 0; m < nch; ++m) {
      const int64_t j0 = ((int64_t)m * GW + lg) * 4;
      ACC g[kTgU][4], x[kTgU][4];
#pragma unroll
      for (int u = 0; u < kTgU; ++u) {
        const int avail = (!ok[u] || j0 >= k) ? 0 : (int)((k - j0) < 4 ? (k - j0) : 4);
        const int64_t off = avail ? j0 : 0;
        load4<ACC>(Gm + (int64_t)(ok[u] ? r[u] : 0) * ldg + off, avail, gal, g[u]);
        load4<ACC>(X + (int64_t)(ok[u] ? c[u] : 0) * ldx + off, avail, xal, x[u]);
      }
#pragma unroll
      for (int u = 0; u < kTgU; ++u) {
#pragma unroll
        for (int e = 0; e < 4; ++e) d[u] = fma_acc<ACC>(g[u][e], x[u][e], d[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < kTgU; ++u) {
      const ACC s = group_sum<GW, ACC>(d[u]);
      const int64_t t = t0 + u;
      if (lg == 0 && t < nnz_in) {
        if (dv_f64) static_cast<double*>(dv)[t] = (double)s;
        else static_cast<float*>(dv)[t] = (float)s;
      }
    }
  }
}

// The same gradients, read from the adjoint's dvalues where the triplet's location is stored
// in the assembled CSC (col_ptr, row_idx of capacity nnz_cap, rows increasing down each
// column).  One lane per triplet: a binary search in the triplet's column finds its slot p
// and dv[t] = dval[p], bit for bit; a triplet outside the matrix gets 0.  A triplet whose
// location was dropped (its values summed to zero) has no slot: the wave then computes the
// dot product above for it, on its first GW lanes (the same lane pieces and group_sum tree),
// one such triplet at a time.
template <typename GT, typename XT, typename ACC, int GW, typename DT>
__global__ __launch_bounds__(kTgNT) void k_triplet_grad_csc(
    int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k, const int32_t* __restrict__ row,
    const int32_t* __restrict__ col, int64_t nnz_cap, const int32_t* __restrict__ col_ptr,
    const int32_t* __restrict__ row_idx, const DT* __restrict__ dval,
    const GT* __restrict__ Gm, int64_t ldg, bool gal, const XT* __restrict__ X, int64_t ldx,
    bool xal, void* __restrict__ dv, bool dv_f64) {
  const int lane = threadIdx.x % kWave;
  const int nch = (int)((k + 4 * GW - 1) / (4 * GW));
  const int64_t stride = (int64_t)gridDim.x * kTgNT;
  for (int64_t base = (int64_t)blockIdx.x * kTgNT + (threadIdx.x - lane); base < nnz_in;
       base += stride) {
    const int64_t t = base + lane;
    const bool live = t < nnz_in;
    const int32_t r = live ? row[t] : -1;
    const int32_t c = live ? col[t] : -1;
    const bool ok = r >= 0 && c >= 0 && (int64_t)r < n_rows && (int64_t)c < n_cols;
    int64_t lo = ok ? col_ptr[c] : 0;
    int64_t hi = ok ? col_ptr[c + 1] : 0;
    lo = lo < 0 ? 0 : (lo > nnz_cap ? nnz_cap : lo);
    hi = hi < lo ? lo : (hi > nnz_cap ? nnz_cap : hi);
    // [lo, hi) shrinks to the one slot whose row can equal r: rows before lo are below r,
    // and once hi has moved, the slot before hi holds a row not below r
    while (hi - lo > 1) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (row_idx[mid - 1] < r) lo = mid;
      else hi = mid;
    }
    const bool hit = ok && lo < hi && row_idx[lo] == r;
    if (live && (hit || !ok)) {
      const double v = hit ? (double)dval[lo] : 0.0;
      if (dv_f64) static_cast<double*>(dv)[t] = v;
      else static_cast<float*>(dv)[t] = (float)v;
    }
    // dropped locations: the dot product, one triplet at a time on lanes 0 .. GW-1
    uint64_t miss = __ballot(live && ok && !hit);
    while (miss) {
      const int j = __ffsll((unsigned long long)miss) - 1;
      miss &= miss - 1;
      const int32_t rj = __shfl(r, j, kWave);
      const int32_t cj = __shfl(c, j, kWave);
      if (lane < GW) {
        ACC d = (ACC)0;
        for (int m = 0; m < nch; ++m) {
          const int64_t j0 = ((int64_t)m * GW + lane) * 4;
          const int avail = j0 >= k ? 0 : (int)((k - j0) < 4 ? (k - j0) : 4);
          const int64_t off = avail ? j0 : 0;
          ACC g[4], x[4];
          load4<ACC>(Gm + (int64_t)rj * ldg + off, avail, gal, g);
          load4<ACC>(X + (int64_t)cj * ldx + off, avail, xal, x);
#pragma unroll
          for (int e = 0; e < 4; ++e) d = fma_acc<ACC>(g[e], x[e], d);
        }
        d = group_sum<GW, ACC>(d);
        if (lane == 0) {
          if (dv_f64) static_cast<double*>(dv)[base + j] = (double)d;
          else static_cast<float*>(dv)[base + j] = (float)d;
        }
      }
    }
  }
}

}  // namespace spm

namespace {

using namespace spm;

bool fits_i32(int64_t x) { return x >= 0 && x <= INT32_MAX; }
bool aligned_to(const void* p, size_t a) { return ((uintptr_t)p & (a - 1)) == 0; }
size_t dsize(spm_dtype t) { return t == SPM_F64 ? 8 : t == SPM_F32 ? 4 : 2; }

int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

template <typename GT, typename XT, typename ACC, int GW>
void launch_tg(int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k, const int32_t* row,
               const int32_t* col, const void* Gm, int64_t ldg, bool gal, const void* X,
               int64_t ldx, bool xal, void* dv, bool dv_f64, hipStream_t s) {
  const int64_t per_block = (int64_t)(kTgNT / GW) * kTgU;
  int64_t grid = (nnz_in + per_block - 1) / per_block;
  const int64_t cap = (int64_t)device_cus() * 32;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  k_triplet_grad<GT, XT, ACC, GW><<<dim3((unsigned)grid), dim3(kTgNT), 0, s>>>(
      n_rows, n_cols, nnz_in, k, row, col, static_cast<const GT*>(Gm), ldg, gal,
      static_cast<const XT*>(X), ldx, xal, dv, dv_f64);
}

template <typename GT, typename XT, typename ACC>
void launch_tg_gw(int gw, int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k,
                  const int32_t* row, const int32_t* col, const void* Gm, int64_t ldg, bool gal,
                  const void* X, int64_t ldx, bool xal, void* dv, bool dv_f64, hipStream_t s) {
#define SPM_TG(W)                                                                            \
  launch_tg<GT, XT, ACC, W>(n_rows, n_cols, nnz_in, k, row, col, Gm, ldg, gal, X, ldx, xal, dv, \
                        dv_f64, s)
  switch (gw) {
    case 1: SPM_TG(1); break;
    case 2: SPM_TG(2); break;
    case 4: SPM_TG(4); break;
    case 8: SPM_TG(8); break;
    case 16: SPM_TG(16); break;
    case 32: SPM_TG(32); break;
    default: SPM_TG(64); break;
  }
#undef SPM_TG
}

template <typename GT, typename XT, typename ACC, int GW>
void launch_tg_csc(int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k, const int32_t* row,
                   const int32_t* col, int64_t nnz_cap, const int32_t* col_ptr,
                   const int32_t* row_idx, const void* dval, bool dval_f64, const void* Gm,
                   int64_t ldg, bool gal, const void* X, int64_t ldx, bool xal, void* dv,
                   bool dv_f64, hipStream_t s) {
  int64_t grid = (nnz_in + kTgNT - 1) / kTgNT;  // one lane per triplet
  const int64_t cap = (int64_t)device_cus() * 32;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  const GT* g = static_cast<const GT*>(Gm);
  const XT* x = static_cast<const XT*>(X);
  if (dval_f64)
    k_triplet_grad_csc<GT, XT, ACC, GW, double><<<dim3((unsigned)grid), dim3(kTgNT), 0, s>>>(
        n_rows, n_cols, nnz_in, k, row, col, nnz_cap, col_ptr, row_idx,
        static_cast<const double*>(dval), g, ldg, gal, x, ldx, xal, dv, dv_f64);
  else
    k_triplet_grad_csc<GT, XT, ACC, GW, float><<<dim3((unsigned)grid), dim3(kTgNT), 0, s>>>(
        n_rows, n_cols, nnz_in, k, row, col, nnz_cap, col_ptr, row_idx,
        static_cast<const float*>(dval), g, ldg, gal, x, ldx, xal, dv, dv_f64);
}

template <typename GT, typename XT, typename ACC>
void launch_tg_csc_gw(int gw, int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k,
                      const int32_t* row, const int32_t* col, int64_t nnz_cap,
                      const int32_t* col_ptr, const int32_t* row_idx, const void* dval,
                      bool dval_f64, const void* Gm, int64_t ldg, bool gal, const void* X,
                      int64_t ldx, bool xal, void* dv, bool dv_f64, hipStream_t s) {
#define SPM_TGC(W)                                                                          \
  launch_tg_csc<GT, XT, ACC, W>(n_rows, n_cols, nnz_in, k, row, col, nnz_cap, col_ptr, row_idx, \
                            dval, dval_f64, Gm, ldg, gal, X, ldx, xal, dv, dv_f64, s)
  switch (gw) {
    case 1: SPM_TGC(1); break;
    case 2: SPM_TGC(2); break;
    case 4: SPM_TGC(4); break;
    case 8: SPM_TGC(8); break;
    case 16: SPM_TGC(16); break;
    case 32: SPM_TGC(32); break;
    default: SPM_TGC(64); break;
  }
#undef SPM_TGC
}

// Element-type dispatch of G and X: each has a type of its own.  The accumulator follows the
// adjoint's rule over the values, G and X (AccOf): binary32 only when bfloat16 is involved and
// binary64 is not.
template <template <typename, typename, typename> class F, typename... A>
void dispatch_gx(spm_dtype vt, spm_dtype gt, spm_dtype xt, A&&... args) {
  auto with_x = [&](auto g_tag) {
    using GT = decltype(g_tag);
    auto go = [&](auto x_tag) {
      using XT = decltype(x_tag);
      if (vt == SPM_F64) F<GT, XT, double>::run(args...);
      else F<GT, XT, typename AccOf<float, GT, XT>::type>::run(args...);
    };
    if (xt == SPM_F64) go(double{});
    else if (xt == SPM_F32) go(float{});
    else go(bf16_t{});
  };
  if (gt == SPM_F64) with_x(double{});
  else if (gt == SPM_F32) with_x(float{});
  else with_x(bf16_t{});
}

template <typename GT, typename XT, typename ACC>
struct RunTg {
  template <typename... A>
  static void run(A&&... args) { launch_tg_gw<GT, XT, ACC>(args...); }
};

template <typename GT, typename XT, typename ACC>
struct RunTgCsc {
  template <typename... A>
  static void run(A&&... args) { launch_tg_csc_gw<GT, XT, ACC>(args...); }
};

}  // namespace

extern "C" {

spm_status spm_coo_triplet_grad(int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k,
                                const int32_t* row, const int32_t* col, spm_dtype val_type,
                                const void* Gm, int64_t ldg, spm_dtype g_type, const void* X,
                                int64_t ldx, spm_dtype x_type, void* dv, spm_dtype dv_type,
                                void* stream) {
  SPM_RANGE("spm_coo_triplet_grad");
  if (n_rows < 0 || n_cols < 0 || nnz_in < 0) return SPM_EINVAL;
  if (!fits_i32(n_rows) || !fits_i32(n_cols) || !fits_i32(nnz_in) || n_rows == INT32_MAX ||
      n_cols == INT32_MAX)
    return SPM_EOVERFLOW;
  if (k < 1 || ldg < k || ldx < k) return SPM_EINVAL;
  if (!fits_i32(k)) return SPM_EOVERFLOW;
  if (val_type != SPM_F64 && val_type != SPM_F32) return SPM_EDTYPE;
  if (g_type != SPM_F64 && g_type != SPM_F32 && g_type != SPM_BF16) return SPM_EDTYPE;
  if (x_type != SPM_F64 && x_type != SPM_F32 && x_type != SPM_BF16) return SPM_EDTYPE;
  if (dv_type != SPM_F64 && dv_type != SPM_F32) return SPM_EDTYPE;
  if (nnz_in > 0 && (!row || !col || !dv)) return SPM_EINVAL;
  if ((n_rows > 0 && !Gm) || (n_cols > 0 && !X)) return SPM_EINVAL;
  if (nnz_in == 0) return SPM_OK;
  const int gw = group_width(k);
  const bool gal = aligned_to(Gm, 4 * dsize(g_type)) && (ldg % 4) == 0;
  const bool xal = aligned_to(X, 4 * dsize(x_type)) && (ldx % 4) == 0;
  const bool f64 = dv_type == SPM_F64;
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  dispatch_gx<RunTg>(val_type, g_type, x_type, gw, n_rows, n_cols, nnz_in, k, row, col, Gm, ldg,
                     gal, X, ldx, xal, dv, f64, s);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPM_OK : SPM_EHIP;
}

spm_status spm_coo_triplet_grad_csc(int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k,
                                    const int32_t* row, const int32_t* col, int64_t nnz_cap,
                                    const int32_t* col_ptr, const int32_t* row_idx,
                                    const void* dval, spm_dtype dval_type, spm_dtype val_type,
                                    const void* Gm, int64_t ldg, spm_dtype g_type,
                                    const void* X, int64_t ldx, spm_dtype x_type, void* dv,
                                    spm_dtype dv_type, void* stream) {
  SPM_RANGE("spm_coo_triplet_grad_csc");
  if (n_rows < 0 || n_cols < 0 || nnz_in < 0 || nnz_cap < 0) return SPM_EINVAL;
  if (!fits_i32(n_rows) || !fits_i32(n_cols) || !fits_i32(nnz_in) || !fits_i32(nnz_cap) ||
      n_rows == INT32_MAX || n_cols == INT32_MAX)
    return SPM_EOVERFLOW;
  if (k < 1 || ldg < k || ldx < k) return SPM_EINVAL;
  if (!fits_i32(k)) return SPM_EOVERFLOW;
  if (val_type != SPM_F64 && val_type != SPM_F32) return SPM_EDTYPE;
  if (dval_type != SPM_F64 && dval_type != SPM_F32) return SPM_EDTYPE;
  if (g_type != SPM_F64 && g_type != SPM_F32 && g_type != SPM_BF16) return SPM_EDTYPE;
  if (x_type != SPM_F64 && x_type != SPM_F32 && x_type != SPM_BF16) return SPM_EDTYPE;
  if (dv_type != SPM_F64 && dv_type != SPM_F32) return SPM_EDTYPE;
  if (nnz_in > 0 && (!row || !col || !dv || !col_ptr)) return SPM_EINVAL;
  if (nnz_cap > 0 && (!row_idx || !dval)) return SPM_EINVAL;
  if ((n_rows > 0 && !Gm) || (n_cols > 0 && !X)) return SPM_EINVAL;
  if (nnz_in == 0) return SPM_OK;
  const int gw = group_width(k);
  const bool gal = aligned_to(Gm, 4 * dsize(g_type)) && (ldg % 4) == 0;
  const bool xal = aligned_to(X, 4 * dsize(x_type)) && (ldx % 4) == 0;
  const bool f64 = dv_type == SPM_F64, d64 = dval_type == SPM_F64;
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  dispatch_gx<RunTgCsc>(val_type, g_type, x_type, gw, n_rows, n_cols, nnz_in, k, row, col,
                        nnz_cap, col_ptr, row_idx, dval, d64, Gm, ldg, gal, X, ldx, xal, dv, f64,
                        s);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPM_OK : SPM_EHIP;
}

}  // extern "C"
