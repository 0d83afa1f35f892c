// Calls every host-side size query and every host-side argument check of libspm.so (the
// paths that return before anything touches the device), for a host-only build of the library
// under AddressSanitizer and UndefinedBehaviorSanitizer.  Pointers below are never
// dereferenced: each call fails validation first, or only computes sizes.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "spm.h"

namespace {
int g_fail = 0;
void expect(int got, int want, const char* what) {
  if (got != want) {
    std::fprintf(stderr, "FAIL %s: status %d, expected %d\n", what, got, want);
    ++g_fail;
  }
}
}  // namespace

int main() {
  void* fake = reinterpret_cast<void*>(0x1000);
  int32_t* fi = static_cast<int32_t*>(fake);
  void* ws = reinterpret_cast<void*>(0x100000);
  const size_t big = (size_t)1 << 40;
  size_t a = 0, b = 0;
  // size queries over many shapes, including the two-level and two-pass layouts
  const int64_t shapes[][3] = {{0, 0, 0},         {1, 1, 1},          {10, 10, 100},
                               {1000, 3, 50000},  {3, 1000, 50000},   {100000, 100000, 1000000},
                               {200000, 150000, 6000000}, {1000000, 1000000, 20000000},
                               {2000000000, 5, 7}};
  for (const auto& s : shapes) {
    expect(spm_coo_to_csc_workspace(s[0], s[1], s[2], &a), SPM_OK, "asm workspace");
    expect(spm_coo_to_csc_plan_size(s[0], s[1], s[2], &a, &b), SPM_OK, "fused sizes");
    expect(spm_csc_plan_size(s[0], s[1], s[2], &a, &b), SPM_OK, "plan sizes");
    expect(spm_csc_transpose_workspace(s[0], s[1], s[2], &a), SPM_OK, "transpose workspace");
    expect(spm_csc_insert_workspace(s[0], s[1], s[2], s[2] / 2, &a), SPM_OK, "insert ws");
    expect(spm_csc_add_workspace(s[0], s[1], s[2], s[2] / 3, &a), SPM_OK, "add workspace");
    expect(spm_csc_trace_atb_workspace(s[1], &a), SPM_OK, "trace workspace");
  }
  expect(spm_coo_to_csc_workspace(-1, 1, 1, &a), SPM_EINVAL, "negative rows");
  expect(spm_coo_to_csc_workspace(1, 1, (int64_t)1 << 31, &a), SPM_EOVERFLOW, "too many");
  expect(spm_coo_to_csc_workspace(1, 1, 1, nullptr), SPM_EINVAL, "null out");
  expect(spm_batch_workspace(8192, 131072, 0, &a), SPM_OK, "batch workspace");
  expect(spm_batch_workspace(-1, 1, 0, &a), SPM_EINVAL, "batch workspace negative");
  // entry points rejecting their arguments on the host
  expect(spm_coo_to_csc(-1, 4, 8, fi, fi, fake, SPM_F64, fi, fi, fake, SPM_F64, fi, ws, big,
                        nullptr), SPM_EINVAL, "asm negative");
  expect(spm_coo_to_csc(4, 4, 8, fi, fi, fake, (spm_dtype)7, fi, fi, fake, SPM_F64, fi, ws, big,
                        nullptr), SPM_EDTYPE, "asm dtype");
  expect(spm_coo_to_csc(4, 4, 8, nullptr, fi, fake, SPM_F64, fi, fi, fake, SPM_F64, fi, ws, big,
                        nullptr), SPM_EINVAL, "asm null row");
  expect(spm_coo_to_csc(4, 4, 8, fi, fi, fake, SPM_F64, fi, fi, fake, SPM_F64, fi, ws, 16,
                        nullptr), SPM_EWORKSPACE, "asm workspace small");
  expect(spm_coo_to_csc_plan(4, 4, 8, fi, fi, fake, SPM_F64, fi, fi, fake, SPM_F64, fi, nullptr,
                             big, nullptr, fi, ws, big, nullptr), SPM_EINVAL, "fused no plan");
  expect(spm_coo_to_csc_plan_noalloc(200000, 200000, 5000000, fi, fi, fake, SPM_F32, fi, fi,
                                     fake, SPM_F32, fi, fake, big, nullptr, fi, nullptr),
         SPM_EWORKSPACE, "noalloc beyond the scratch");
  expect(spm_csc_plan_build(4, 4, 8, fi, fi, nullptr, SPM_F32, fake, 16, nullptr, fi, ws, big,
                            nullptr), SPM_EWORKSPACE, "plan buffer small");
  expect(spm_csc_spmm(4, 4, 8, 0, fake, fake, SPM_F32, SPM_ORDER_CSC, fake, 4, SPM_F32, fake, 4,
                      SPM_F32, nullptr), SPM_EINVAL, "spmm k = 0");
  expect(spm_csc_spmm(4, 4, 8, 4, fake, fake, SPM_BF16, SPM_ORDER_CSC, fake, 4, SPM_F32, fake,
                      4, SPM_F32, nullptr), SPM_EDTYPE, "spmm bf16 values");
  expect(spm_csc_spmm_backward(4, 4, 8, 4, nullptr, fi, fake, SPM_F32, fake, 4, SPM_F64, fake,
                               4, SPM_F32, fake, 4, SPM_F32, fake, SPM_F64, nullptr),
         SPM_EINVAL, "adjoint null col_ptr");
  expect(spm_csc_spmm_backward(4, 4, 8, 4, fi, fi, fake, SPM_F32, fake, 4, (spm_dtype)9, fake,
                               4, SPM_F32, fake, 4, SPM_F32, fake, SPM_F64, nullptr),
         SPM_EDTYPE, "adjoint G dtype");
  expect(spm_csc_insert(4, 4, 8, fi, fi, fake, 8, fi, fi, fake, SPM_F64, fi, fi, fake, SPM_F64,
                        fi, ws, 16, nullptr), SPM_EWORKSPACE, "insert workspace small");
  expect(spm_csc_add(4, 0, 8, fi, fi, fake, 8, fi, fi, fake, SPM_F64, fi, fi, fake, SPM_F64, fi,
                     ws, big, nullptr), SPM_EINVAL, "add no columns");
  expect(spm_csc_transpose(4, 4, 8, fi, fi, fake, SPM_BF16, fi, fi, fake, fi, ws, big, nullptr),
         SPM_EDTYPE, "transpose dtype");
  expect(spm_csc_trace_atb(4, ((int64_t)1 << 28) + 16, 8, fi, fi, fake, 8, fi, fi, fake, SPM_F64,
                           static_cast<double*>(fake), fi, ws, big, nullptr),
         SPM_EOVERFLOW, "trace too many columns");
  expect(spm_coo_triplet_grad(4, 4, 8, 0, fi, fi, SPM_F32, fake, 4, SPM_F32, fake, 4, SPM_F32,
                              fake, SPM_F32, nullptr), SPM_EINVAL, "triplet grad k = 0");
  expect(spm_coo_triplet_grad_csc(4, 4, 8, 4, fi, fi, -1, fi, fi, fake, SPM_F64, SPM_F32, fake,
                                  4, SPM_F64, fake, 4, SPM_F32, fake, SPM_F32, nullptr),
         SPM_EINVAL, "triplet grad csc negative capacity");
  // host-only batch schedule on a real host array
  std::vector<spm_batch_item> items(5);
  std::vector<int32_t> order(5);
  for (int i = 0; i < 5; ++i) items[i] = spm_batch_item{64 * (i + 1), 64 * (i + 1), 1024 * i, 0,
                                                         0, 0, 0, 0, 0};
  expect(spm_batch_schedule(items.data(), 5, 32, order.data()), SPM_OK, "batch schedule");
  expect(spm_batch_schedule(items.data(), -1, 32, order.data()), SPM_EINVAL, "schedule neg");
  // tuning round trip and rejection
  spm_tuning t{};
  expect(spm_tuning_get(&t), SPM_OK, "tuning get");
  spm_tuning bad = t;
  bad.spmm_block = 100;
  expect(spm_tuning_set(&bad), SPM_EINVAL, "tuning rejects");
  expect(spm_tuning_set(&t), SPM_OK, "tuning set");
  for (int s = -1; s < 9; ++s)
    if (!spm_status_string(s)) ++g_fail;
  if (!spm_version()) ++g_fail;
  if (g_fail) return 1;
  std::printf("abi driver: clean\n");
  return 0;
}
