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
#include "spm_spmm.h"

namespace spm {

constexpr int kTgNT = 256;  // threads per workgroup
constexpr int kTgU = 4;     // triplets per group in flight

template <typename XT, typename ACC, int GW>
__global__ __launch_bounds__(kTgNT) void k_triplet_grad(
    int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k, const int32_t* __restrict__ row,
    const int32_t* __restrict__ col, const XT* __restrict__ Gm, int64_t ldg, bool gal,
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

template <typename XT, typename ACC, int GW>
void launch_tg(int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k, const int32_t* row,
               const int32_t* col, const void* Gm, int64_t ldg, bool gal, const void* X,
               int64_t ldx, bool xal, void* dv, bool dv_f64, hipStream_t s) {
  const int64_t per_block = (int64_t)(kTgNT / GW) * kTgU;
  int64_t grid = (nnz_in + per_block - 1) / per_block;
  const int64_t cap = (int64_t)device_cus() * 32;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  k_triplet_grad<XT, ACC, GW><<<dim3((unsigned)grid), dim3(kTgNT), 0, s>>>(
      n_rows, n_cols, nnz_in, k, row, col, static_cast<const XT*>(Gm), ldg, gal,
      static_cast<const XT*>(X), ldx, xal, dv, dv_f64);
}

template <typename XT, typename ACC>
void launch_tg_gw(int gw, int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k,
                  const int32_t* row, const int32_t* col, const void* Gm, int64_t ldg, bool gal,
                  const void* X, int64_t ldx, bool xal, void* dv, bool dv_f64, hipStream_t s) {
#define SPM_TG(W)                                                                            \
  launch_tg<XT, ACC, W>(n_rows, n_cols, nnz_in, k, row, col, Gm, ldg, gal, X, ldx, xal, dv, \
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

}  // namespace

extern "C" {

spm_status spm_coo_triplet_grad(int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k,
                                const int32_t* row, const int32_t* col, spm_dtype val_type,
                                const void* Gm, int64_t ldg, const void* X, int64_t ldx,
                                spm_dtype x_type, void* dv, spm_dtype dv_type, void* stream) {
  if (n_rows < 0 || n_cols < 0 || nnz_in < 0) return SPM_EINVAL;
  if (!fits_i32(n_rows) || !fits_i32(n_cols) || !fits_i32(nnz_in) || n_rows == INT32_MAX ||
      n_cols == INT32_MAX)
    return SPM_EOVERFLOW;
  if (k < 1 || ldg < k || ldx < k) return SPM_EINVAL;
  if (!fits_i32(k)) return SPM_EOVERFLOW;
  if (val_type != SPM_F64 && val_type != SPM_F32) return SPM_EDTYPE;
  if (x_type != SPM_F64 && x_type != SPM_F32 && x_type != SPM_BF16) return SPM_EDTYPE;
  if (dv_type != SPM_F64 && dv_type != SPM_F32) return SPM_EDTYPE;
  if (nnz_in > 0 && (!row || !col || !dv)) return SPM_EINVAL;
  if ((n_rows > 0 && !Gm) || (n_cols > 0 && !X)) return SPM_EINVAL;
  if (nnz_in == 0) return SPM_OK;
  const int gw = group_width(k);
  const bool gal = aligned_to(Gm, 4 * dsize(x_type)) && (ldg % 4) == 0;
  const bool xal = aligned_to(X, 4 * dsize(x_type)) && (ldx % 4) == 0;
  const bool f64 = dv_type == SPM_F64;
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  // accumulation as in the adjoint: binary32 for bfloat16 operands with binary32 values
  if (x_type == SPM_F64)
    launch_tg_gw<double, double>(gw, n_rows, n_cols, nnz_in, k, row, col, Gm, ldg, gal, X, ldx,
                                 xal, dv, f64, s);
  else if (x_type == SPM_F32)
    launch_tg_gw<float, double>(gw, n_rows, n_cols, nnz_in, k, row, col, Gm, ldg, gal, X, ldx,
                                xal, dv, f64, s);
  else if (val_type == SPM_F64)
    launch_tg_gw<bf16_t, double>(gw, n_rows, n_cols, nnz_in, k, row, col, Gm, ldg, gal, X, ldx,
                                 xal, dv, f64, s);
  else
    launch_tg_gw<bf16_t, float>(gw, n_rows, n_cols, nnz_in, k, row, col, Gm, ldg, gal, X, ldx,
                                xal, dv, f64, s);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPM_OK : SPM_EHIP;
}

}  // extern "C"
