// Host side of libspm.so: argument validation, workspace layout, launch sequencing.
// Every entry point is declared (and documented) in include/spm.h.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>

#include "spm.h"
#include "spm_range.h"
#include "spm_assemble.h"
#include "spm_spmm.h"
#include "spm_batch.h"
#include "spm_mergepath.h"
#include <algorithm>
#include <vector>


namespace {

using namespace spm;

constexpr int kNT = 256;          // threads per workgroup of the assembly / plan kernels
constexpr int kScanIPT = 8;       // scan tile = 2048 counts
constexpr int kFoldIPT = 8;       // fold tile = 2048 keys
constexpr int kSortT = 2048;      // segment-sort tile (segments starting in a tile)
constexpr int kSortCap = 4096;    // LDS capacity of one sort chunk (keys)

constexpr int64_t kScanTile = (int64_t)kNT * kScanIPT;
constexpr int64_t kFoldTile = (int64_t)kNT * kFoldIPT;
static_assert(kFoldTile == kSortT, "sort and fold tiles share one tile -> first-segment table");

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Sequential carving of a 256-byte aligned workspace.
struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t at = off;
    off += align256(bytes);
    return at;
  }
};

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Tuning in effect for a call: the calling thread's selection (spm_tuning_select) if it made
// one, else the process-wide values (spm_tuning_set).  Named tunings live in a registry.
spm_tuning g_tuning = {256, 64, 2, 2048, 512, 0, 0, 0};
std::mutex g_tuning_mu;
std::map<std::string, spm_tuning> g_tuning_named;
thread_local bool t_tuning_on = false;
thread_local spm_tuning t_tuning;

spm_tuning tuning() {
  if (t_tuning_on) return t_tuning;
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  return g_tuning;
}

int cu_count() {
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

// Largest dynamic LDS a workgroup may request on the current device (cached per device).
int max_lds_per_block() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        n <= 0)
      n = 65536;
    cached[dev] = n;
  }
  return cached[dev];
}

int grid_for(int64_t work_items, int64_t per_block, int cap) {
  int64_t g = ceil_div(work_items, per_block);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

bool fits_i32(int64_t x) { return x >= 0 && x <= INT32_MAX; }
bool aligned(const void* p, size_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

spm_status launch_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPM_OK : SPM_EHIP;
}

// ------------------------------------------------------------------------------------------
// Two-level partition parameters (spm_partition.h).  b = log2(segments per coarse bucket):
// at least what keeps the number of buckets within the level-1 LDS counters, and an expected
// bucket size of at most min(part_bucket_target, 3/4 of kPartCap) when the sizes allow it.
// Returns ok = false when no b <= 12 fits (more than about kPartMaxBuckets * kPartMaxWidth
// segments); then the atomic-histogram path is used.
// ------------------------------------------------------------------------------------------
constexpr int kPartNT = 1024;  // level-1 workgroup (hist, scatter): long per-bucket runs
constexpr int kPartCap = 2048;  // bucket size kept entirely in LDS by the fused level 2
// Up to this many buckets k_part_emit reduces the survivor counts of the buckets before it
// per workgroup; beyond it one k_small_scan launch computes them.
constexpr int kEmitReduceMax = 1024;
// k_small_scan's shape: one round of loads for up to kPartMaxBuckets counts
constexpr int kSmallScanNT = 1024;
constexpr int kSmallScanIPT = 16;
static_assert(kSmallScanNT * kSmallScanIPT >= kPartMaxBuckets, "one round of the small scan");

// Level 2 splits each segment into R = 2^l2_sub_log2(b) sub-ranges of the key's high word
// (values in [0, key_range)): the shift that maps that range onto [0, R).
int sub_shift(int64_t key_range, int b) {
  int bits = 0;
  while (((int64_t)1 << bits) < key_range) ++bits;
  const int lr = l2_sub_log2(b);
  return bits > lr ? bits - lr : 0;
}

struct PartParams {
  bool ok;
  int b;
  int32_t CB;
  int64_t ntiles;
  int64_t T1;  // level-1 tile: elements per workgroup
};

int ceil_log2(int64_t x) {
  int b = 0;
  while (((int64_t)1 << b) < x) ++b;
  return b;
}
int floor_log2(int64_t x) {
  int b = 0;
  while (((int64_t)2 << b) <= x) ++b;
  return b;
}

PartParams part_params(int64_t nseg, int64_t n) {
  PartParams P{false, 0, 0, 1, 1024};
  if (nseg <= 0) return P;
  const spm_tuning tu = tuning();
  // level-1 kernels keep one LDS counter per bucket (plus under 1 KB of static LDS, and the
  // histogram's sub-tile counters)
  const int64_t max_buckets = std::min<int64_t>(
      kPartMaxBuckets, ((int64_t)max_lds_per_block() - 1024 - 4 * kSubMax * 128) / 4);
  const int bmin = ceil_log2(ceil_div(nseg, max_buckets));
  // floor_log2 puts the expected bucket size in (target/2, target]; keep it at most 3/4 of
  // the in-LDS capacity so that ordinary fluctuations stay on the in-LDS path
  const int64_t target = std::min<int64_t>(tu.part_bucket_target, kPartCap * 3 / 4);
  const int btarget = n > 0 ? floor_log2(std::max<int64_t>(1, nseg * target / n)) : 12;
  int b = std::max(bmin, btarget);
  if (b > 12) b = 12;
  if (b < bmin) return P;
  P.ok = true;
  P.b = b;
  P.CB = (int32_t)ceil_div(nseg, (int64_t)1 << b);
  // level-1 tiles: at least 1024 elements, at most part_max_tiles tiles (the bucket x tile
  // table stays below kPartMaxBuckets * part_max_tiles entries)
  int64_t T1 = 1024;
  while (ceil_div(n, T1) > tu.part_max_tiles) T1 <<= 1;
  P.T1 = T1;
  P.ntiles = std::max<int64_t>(1, ceil_div(n, T1));
  return P;
}

// Level 1 in two passes (spm_partition.h) once there are this many buckets: a tile then
// holds only a few elements per bucket, and the single scatter's records would each go to a
// line of their own.  Super-buckets of 2^kSuperLog2 buckets; pass-B workgroups take K
// consecutive tiles' slices of a super-bucket, about one LDS chunk each.
constexpr int32_t kSplitMinBuckets = 4096;
constexpr int kSuperLog2 = 7;
static_assert((1 << kSuperLog2) <= kSuperMax, "buckets per super-bucket");
static_assert(kPartMaxBuckets <= kSuperMax << kSuperLog2, "super-buckets per partition");
constexpr int kSplitNT = 512;  // threads of a pass-A / pass-B workgroup
constexpr int kSplitU = 4;     // elements per thread of a chunk

struct SplitParams {
  bool on;
  int g;
  int32_t SB;
  int SH;           // pass-A sub-tiles per tile
  int64_t K, nq;    // pass B: tiles per slice, slices per super-bucket
  int64_t nchunk;   // k_super_offsets: workgroups per super-bucket (64 tiles each)
};

SplitParams split_params(const PartParams& P) {
  SplitParams S{false, kSuperLog2, 0, 0, 1, 1, 1};
  if (!P.ok || P.CB < kSplitMinBuckets) return S;
  if (staged_lds_bytes(kSplitNT, kSplitU, true) + 2048 > (size_t)max_lds_per_block()) return S;
  S.on = true;
  S.SB = (int32_t)ceil_div(P.CB, (int64_t)1 << S.g);
  const int64_t chunk = (int64_t)kSplitNT * kSplitU;
  // pass A: enough workgroups to fill the chip several times over, each at least a chunk
  S.SH = 1;
  while (S.SH < kSubMax && P.ntiles * S.SH < 4 * (int64_t)cu_count() &&
         P.T1 / (2 * S.SH) >= chunk)
    S.SH *= 2;
  // pass B: a slice of about 85 % of a chunk, so that one chunk nearly always covers it
  const int64_t K = (chunk * S.SB * 85) / (100 * P.T1);
  S.K = std::min<int64_t>(std::max<int64_t>(K, 1), P.ntiles);
  S.nq = ceil_div(P.ntiles, S.K);
  S.nchunk = ceil_div(P.ntiles + 1, (int64_t)kWave);
  return S;
}

// ------------------------------------------------------------------------------------------
// Assembly workspace layout.  The first region (counters, look-back states, tickets) is
// zeroed by one kernel at the start of every call.
// ------------------------------------------------------------------------------------------
struct AsmLayout {
  PartParams pp;
  // zeroed at the start of every call (only the fallback path needs these)
  size_t colcnt, scan_state, fold_state, tickets, zero_bytes;
  // fallback path
  size_t colstart, first;
  // shared
  size_t bucket, scratch;
  // partition path
  size_t table, rowoff, btot, bstart, brec, bvhi, trow, tval, bkept, boff, flags, big;
  size_t sbro, subcnt;  // two-pass level 1 (its records go to bucket + scratch)
  SplitParams sp;
  size_t total;
  int64_t fold_tiles;
};

AsmLayout asm_layout(int64_t n_cols, int64_t nnz_in) {
  AsmLayout L;
  Carve c;
  L.pp = part_params(n_cols, nnz_in);
  const bool ok = L.pp.ok;
  const int64_t tab = ok ? (int64_t)L.pp.CB * L.pp.ntiles : 0;
  const int64_t cb = ok ? L.pp.CB : 0;
  const int64_t nP = ok ? nnz_in : 0;  // per-element partition arrays
  const int64_t nF = ok ? 0 : n_cols;  // fallback-only arrays
  const int64_t scan_tiles = (!ok && n_cols > 0) ? ceil_div(n_cols, kScanTile) : 1;
  L.fold_tiles = nnz_in > 0 ? ceil_div(nnz_in, kFoldTile) : 1;
  L.colcnt = c.take(sizeof(uint32_t) * (size_t)nF);
  L.scan_state = c.take(sizeof(uint64_t) * (size_t)(ok ? 0 : scan_tiles));
  L.fold_state = c.take(sizeof(uint64_t) * (size_t)(ok ? 0 : L.fold_tiles));
  L.tickets = c.take(sizeof(uint32_t) * 4);
  L.zero_bytes = c.off;
  L.colstart = c.take(sizeof(int32_t) * (size_t)(ok ? 0 : n_cols + 1));
  L.first = c.take(sizeof(int32_t) * (size_t)(ok ? 0 : L.fold_tiles + 1));
  L.bucket = c.take(sizeof(uint64_t) * (size_t)nnz_in);
  L.scratch = c.take(sizeof(uint64_t) * (size_t)nnz_in);
  L.table = c.take(sizeof(uint32_t) * (size_t)tab);
  L.rowoff = c.take(sizeof(uint32_t) * (size_t)tab);
  L.btot = c.take(sizeof(uint32_t) * (size_t)cb);
  L.bstart = c.take(sizeof(int32_t) * (size_t)(cb + 1));
  L.brec = c.take(16 * (size_t)nP);               // bucket records (key, segment, value word)
  L.bvhi = c.take(sizeof(uint32_t) * (size_t)nP);  // high words of float64 values
  L.trow = c.take(sizeof(uint32_t) * (size_t)nP);
  L.tval = c.take(sizeof(double) * (size_t)nP);
  L.bkept = c.take(sizeof(uint32_t) * (size_t)cb);
  L.boff = c.take(sizeof(int32_t) * (size_t)(cb > kEmitReduceMax ? cb + 1 : 0));
  L.flags = c.take(sizeof(uint32_t) * (size_t)(ok ? L.pp.ntiles : 0));
  L.big = c.take(sizeof(uint32_t) * (size_t)(cb + 1));  // big-bucket list (count, buckets)
  L.sp = split_params(L.pp);
  L.sbro = c.take(sizeof(uint32_t) * (size_t)(L.sp.on ? L.sp.SB * (L.pp.ntiles + 1) : 0));
  L.subcnt = c.take(sizeof(uint32_t) *
                    (size_t)(L.sp.on ? L.sp.SB * L.sp.SH * L.pp.ntiles : 0));
  L.total = c.off;
  return L;
}

struct PlanLayout {
  PartParams pp;
  size_t rowcnt, scan_state, tickets, zero_bytes, first, bucket, scratch;
  size_t colarr, table, rowoff, btot, bstart, brec, bvhi, flags, big, total;
  size_t sbro, subcnt, ivhi;  // two-pass level 1 (records in bucket + scratch)
  SplitParams sp;
  int64_t sort_tiles;
};

// Workgroups of k_expand_columns (one thread per column, grid-stride beyond the cap); a
// fixed cap keeps the workspace size independent of the device.
constexpr int kExpandMaxGroups = 4096;
int expand_grid(int64_t n_cols) { return grid_for(n_cols > 0 ? n_cols : 1, kNT, kExpandMaxGroups); }

PlanLayout plan_ws_layout(int64_t n_rows, int64_t n_cols, int64_t nnz_cap) {
  PlanLayout L;
  Carve c;
  L.pp = part_params(n_rows, nnz_cap);
  const bool ok = L.pp.ok;
  const int64_t tab = ok ? (int64_t)L.pp.CB * L.pp.ntiles : 0;
  const int64_t cb = ok ? L.pp.CB : 0;
  const int64_t nP = ok ? nnz_cap : 0;
  const int64_t scan_tiles = (!ok && n_rows > 0) ? ceil_div(n_rows, kScanTile) : 1;
  L.sort_tiles = nnz_cap > 0 ? ceil_div(nnz_cap, kSortT) : 1;
  L.rowcnt = c.take(sizeof(uint32_t) * (size_t)(ok ? 0 : n_rows));
  L.scan_state = c.take(sizeof(uint64_t) * (size_t)(ok ? 0 : scan_tiles));
  L.tickets = c.take(sizeof(uint32_t) * 4);
  L.zero_bytes = c.off;
  L.first = c.take(sizeof(int32_t) * (size_t)(ok ? 0 : L.sort_tiles + 1));
  L.bucket = c.take(sizeof(uint64_t) * (size_t)nnz_cap);
  L.scratch = c.take(sizeof(uint64_t) * (size_t)nnz_cap);
  L.colarr = c.take(sizeof(int32_t) * (size_t)nP);
  L.table = c.take(sizeof(uint32_t) * (size_t)tab);
  L.rowoff = c.take(sizeof(uint32_t) * (size_t)tab);
  L.btot = c.take(sizeof(uint32_t) * (size_t)cb);
  L.bstart = c.take(sizeof(int32_t) * (size_t)(cb + 1));
  L.brec = c.take(16 * (size_t)nP);
  L.bvhi = c.take(sizeof(uint32_t) * (size_t)nP);  // high words of float64 values
  // status flags: one per k_expand_columns workgroup, then one per k_part_hist tile
  L.flags = c.take(sizeof(uint32_t) * (size_t)(ok ? expand_grid(n_cols) + L.pp.ntiles : 0));
  L.big = c.take(sizeof(uint32_t) * (size_t)(cb + 1));  // big-bucket list (count, buckets)
  L.sp = split_params(L.pp);
  L.sbro = c.take(sizeof(uint32_t) * (size_t)(L.sp.on ? L.sp.SB * (L.pp.ntiles + 1) : 0));
  L.subcnt = c.take(sizeof(uint32_t) *
                    (size_t)(L.sp.on ? L.sp.SB * L.sp.SH * L.pp.ntiles : 0));
  L.ivhi = c.take(sizeof(uint32_t) * (size_t)(L.sp.on ? nP : 0));
  L.total = c.off;
  return L;
}

struct PlanParts {
  size_t row_ptr, col_t, perm, total;
};

PlanParts plan_parts(int64_t n_rows, int64_t nnz_cap) {
  PlanParts P;
  Carve c;
  P.row_ptr = c.take(sizeof(int32_t) * (size_t)(n_rows + 1));
  P.col_t = c.take(sizeof(int32_t) * (size_t)nnz_cap);
  P.perm = c.take(sizeof(int32_t) * (size_t)nnz_cap);
  P.total = c.off;
  return P;
}

// Fused assembly + plan (spm_coo_to_csc_plan).  The assembly's survivors are counted per
// (row bucket, column bucket) and the emit writes them a second time as records of the
// plan's row partition, so the plan needs no column expansion, histogram or scatter of its
// own.  Applies when the row partition exists with at most kFuseMaxRowBuckets buckets and
// the (row bucket x column bucket) table stays small; otherwise the two builds run one after
// the other on the same workspace.  The plan's records reuse the assembly's record buffers
// (dead once the assembly's level 2 has run); its level 2 reuses the staging buffers.
constexpr int64_t kFuseMaxTable = (int64_t)1 << 22;  // entries of the fused table
static_assert(kFuseMaxRowBuckets <= 2 * kPartCap, "row-bucket counters live in level 2's s_in");

struct FuseLayout {
  AsmLayout A;
  PartParams Q;  // plan partition by row (capacity nnz_in)
  bool fused;
  size_t table2, rowoff2, btot2, bstart2, big2, total;
};

FuseLayout fuse_layout(int64_t n_rows, int64_t n_cols, int64_t nnz_in) {
  FuseLayout F;
  F.A = asm_layout(n_cols, nnz_in);
  F.Q = part_params(n_rows, nnz_in);
  F.fused = F.A.pp.ok && F.Q.ok && nnz_in > 0 && F.Q.CB <= kFuseMaxRowBuckets &&
            (int64_t)F.Q.CB * F.A.pp.CB <= kFuseMaxTable;
  if (!F.fused) {
    F.table2 = F.rowoff2 = F.btot2 = F.bstart2 = F.big2 = 0;
    F.total = std::max(F.A.total, plan_ws_layout(n_rows, n_cols, nnz_in).total);
    return F;
  }
  Carve c;
  c.off = F.A.total;
  const size_t tab = (size_t)F.Q.CB * (size_t)F.A.pp.CB;
  F.table2 = c.take(sizeof(uint32_t) * tab);
  F.rowoff2 = c.take(sizeof(uint32_t) * tab);
  F.btot2 = c.take(sizeof(uint32_t) * (size_t)F.Q.CB);
  F.bstart2 = c.take(sizeof(int32_t) * ((size_t)F.Q.CB + 1));
  F.big2 = c.take(sizeof(uint32_t) * ((size_t)F.Q.CB + 1));
  F.total = c.off;
  return F;
}

// What the assembly's partition path needs to also build the plan.
struct FuseCtx {
  const FuseLayout* F;
  int64_t n_rows;
  const PlanParts* P;
  char* plan;
  void* val_plan;  // optional, of the output type
  int32_t* plan_info;
};

// Level 2 over every bucket.  Buckets of at most kPartCap elements go through the first launch,
// one workgroup each (small LDS, four per CU).  When the device's LDS allows, buckets above
// that (listed by k_rows_scan in big) go through a second, persistent launch with an in-LDS
// capacity of kPartBigCap and 512 threads, so that power-law buckets of up to twice the usual
// size stay off the staged path.  big == nullptr: one launch, larger buckets staged.
constexpr int kPartBigNT = 512;
constexpr int kPartBigCap = 4096;

// Partitions of fewer buckets keep the one launch (a big bucket is rare there, and the second
// launch would cost more than staging it).
constexpr int32_t kBigMinBuckets = 2048;

bool level2_big_ok(int b, int32_t CB) {
  return CB >= kBigMinBuckets &&
         part_level2_lds_bytes(b, kPartBigCap) + 2048 <= (size_t)max_lds_per_block();
}

constexpr int kL2WideMinBucketsPerCu = 16;

template <bool PLAN, typename VT>
void launch_level2(int b, int32_t CB, int64_t nseg, const int32_t* bstart, const uint4* brec,
                   const uint32_t* bvhi, uint64_t* bucket, uint64_t* scratch, int32_t* row_ptr,
                   int32_t* col_t, int32_t* perm, const VT* val, VT* val_plan, int32_t* col_rel,
                   uint32_t* trow, double* tval, uint32_t* bkept, int rshift,
                   const L2RowCount& rc, const uint32_t* big, hipStream_t s) {
  // With many buckets (several rounds of workgroups) 512-thread workgroups put more waves on
  // each CU than LDS allows 256-thread ones (each thread's share of a bucket halves, and so do
  // its registers); with one round, four buckets per CU at a time finish sooner.
  if ((int64_t)CB > (int64_t)cu_count() * kL2WideMinBucketsPerCu)
    k_part_level2<2 * kNT, kPartCap, PLAN, VT>
        <<<dim3((unsigned)CB), dim3(2 * kNT), part_level2_lds_bytes(b, kPartCap), s>>>(
            b, nseg, bstart, brec, bvhi, bucket, scratch, row_ptr, col_t, perm, val, val_plan,
            col_rel, trow, tval, bkept, rshift, rc, big);
  else
    k_part_level2<kNT, kPartCap, PLAN, VT>
        <<<dim3((unsigned)CB), dim3(kNT), part_level2_lds_bytes(b, kPartCap), s>>>(
            b, nseg, bstart, brec, bvhi, bucket, scratch, row_ptr, col_t, perm, val, val_plan,
            col_rel, trow, tval, bkept, rshift, rc, big);
  if (big) {
    const int grid = (int)std::min<int64_t>(CB, (int64_t)cu_count() * 2);
    k_part_level2_big<kPartBigNT, kPartBigCap, PLAN, VT>
        <<<dim3((unsigned)grid), dim3(kPartBigNT), part_level2_lds_bytes(b, kPartBigCap), s>>>(
            b, nseg, bstart, brec, bvhi, bucket, scratch, row_ptr, col_t, perm, val, val_plan,
            col_rel, trow, tval, bkept, rshift, rc, big, CB);
  }
}

// Level 1's scatter into the buckets' records (brec, bvhi) and bstart: one pass, or the two
// passes of spm_partition.h through irec / ivhi (16 and 4 bytes per element) and sbro.
template <typename SRC, typename VT>
void launch_scatter(const SRC& src, const PartParams& P, const SplitParams& S,
                    const uint32_t* rowoff, const uint32_t* btot, int32_t* bstart, uint4* brec,
                    const VT* vin, uint32_t* bvhi, uint4* irec, uint32_t* ivhi, uint32_t* sbro,
                    const uint32_t* subcnt, hipStream_t s) {
  if (!S.on) {
    k_part_scatter<kPartNT, SRC, VT>
        <<<dim3((unsigned)P.ntiles), dim3(kPartNT), 4 * (size_t)P.CB, s>>>(
            src, P.b, P.CB, P.ntiles, P.T1, rowoff, btot, bstart, brec, vin, bvhi);
    return;
  }
  k_super_offsets<kNT><<<dim3((unsigned)(S.SB * S.nchunk)), dim3(kNT), 0, s>>>(
      btot, rowoff, P.CB, S.g, P.ntiles, S.nchunk, bstart, sbro);
  const size_t lds = staged_lds_bytes(kSplitNT, kSplitU, ValWords<VT>::kHi);
  k_part_scatter_a<kSplitNT, SRC, VT>
      <<<dim3((unsigned)(P.ntiles * S.SH)), dim3(kSplitNT), lds, s>>>(
          src, P.b, S.g, S.SB, P.ntiles, P.T1, S.SH, sbro, subcnt, irec, vin, ivhi);
  k_part_scatter_b<kSplitNT, VT>
      <<<dim3((unsigned)(S.SB * S.nq)), dim3(kSplitNT), lds, s>>>(
          P.b, S.g, P.CB, P.ntiles, S.K, S.nq, sbro, rowoff, bstart, irec, ivhi, brec, bvhi);
}

// The histogram's sub-tile counts for the two-pass level 1 (none when it is off).
SubCounts sub_counts(const SplitParams& S, char* w, size_t off) {
  return S.on ? SubCounts{reinterpret_cast<uint32_t*>(w + off), S.g, S.SH, S.SB}
              : SubCounts{nullptr, 0, 0, 0};
}

spm_status assemble_impl(int64_t n_rows, int64_t n_cols, int64_t nnz_in, const int32_t* row,
                         const int32_t* col, const void* val, spm_dtype val_type,
                         int32_t* col_ptr, int32_t* row_idx, void* val_out, spm_dtype out_type,
                         int32_t* info, char* w, const AsmLayout& L, hipStream_t s,
                         const FuseCtx* fz);

spm_status check_dims(int64_t n_rows, int64_t n_cols, int64_t nnz) {
  if (n_rows < 0 || n_cols < 0 || nnz < 0) return SPM_EINVAL;
  if (!fits_i32(n_rows) || !fits_i32(n_cols) || !fits_i32(nnz) || n_cols == INT32_MAX ||
      n_rows == INT32_MAX)
    return SPM_EOVERFLOW;
  return SPM_OK;
}

template <int NT, int IPT>
void launch_scan(const uint32_t* in, int64_t n, int32_t* out, uint64_t* state, uint32_t* ticket,
                 hipStream_t s) {
  const int64_t tiles = n > 0 ? ceil_div(n, (int64_t)NT * IPT) : 1;
  k_scan_excl<NT, IPT><<<dim3((unsigned)tiles), dim3(NT), 0, s>>>(
      in, n, out, state, ticket);
}

template <typename VT>
void launch_fold(const uint64_t* keys, const int32_t* colstart, int64_t n_cols, const VT* val,
                 int32_t* col_ptr, int32_t* row_idx, void* val_out, int out_f64, int32_t* info,
                 const int32_t* first, uint64_t* state, uint32_t* ticket, int64_t tiles,
                 hipStream_t s) {
  k_fold<kNT, kFoldIPT, VT><<<dim3((unsigned)tiles), dim3(kNT), 0, s>>>(
      keys, colstart, n_cols, val, col_ptr, row_idx, val_out, out_f64, info, first, state,
      ticket);
}

// ------------------------------------------------------------------------------------------
// SpMM dispatch over element types.
// ------------------------------------------------------------------------------------------
// The lane-group width is a compile-time parameter of the product kernels; it depends on k
// alone (group_width), never on tuning, so results do not depend on the launch shape.
#define SPM_GW_SWITCH(G, CALL) \
  switch (G) {                 \
    case 1: CALL(1); break;    \
    case 2: CALL(2); break;    \
    case 4: CALL(4); break;    \
    case 8: CALL(8); break;    \
    case 16: CALL(16); break;  \
    case 32: CALL(32); break;  \
    default: CALL(64); break;  \
  }

// FULL kernels (k == 4 * group width, aligned rows: no tail handling) are built for the
// widths of the common dense widths k = 32, 64, 128; every other case runs the general kernel,
// which computes the same values in the same order.
template <typename VT, typename XT, typename ACC>
void launch_fwd_t(int64_t n_rows, int64_t n_cols, int64_t nnz_cap, int64_t k, int G, bool full,
                  bool pv, const int32_t* row_ptr, const int32_t* col_t,
                  const int32_t* perm, const void* val, const void* X, int64_t ldx, int xal,
                  void* Y, int64_t ldy, int y_f64, int yal, int grid, int block, hipStream_t s) {
  // plan-order values: the full kernels take them as a template flag, the general kernel
  // as perm == nullptr
  const int32_t* gperm = pv ? nullptr : perm;
#define SPM_CALL_F(GW, F, PV, PERM)                                                            \
  k_spmm_fwd<VT, XT, ACC, GW, F, PV><<<dim3(grid), dim3(block), 0, s>>>(                       \
      n_rows, n_cols, nnz_cap, k, row_ptr, col_t, PERM, static_cast<const VT*>(val),           \
      static_cast<const XT*>(X), ldx, xal, Y, ldy, y_f64, yal)
#define SPM_CALL_FULL(GW)                                                                      \
  do {                                                                                         \
    if (pv) SPM_CALL_F(GW, true, true, perm);                                                  \
    else SPM_CALL_F(GW, true, false, perm);                                                    \
  } while (0)
#define SPM_CALL(GW) SPM_CALL_F(GW, false, false, gperm)
  if (full && G == 8) SPM_CALL_FULL(8);
  else if (full && G == 16) SPM_CALL_FULL(16);
  else if (full && G == 32) SPM_CALL_FULL(32);
  else SPM_GW_SWITCH(G, SPM_CALL)
#undef SPM_CALL
#undef SPM_CALL_FULL
#undef SPM_CALL_F
}

template <typename VT, typename GT, typename XT, typename ACC>
void launch_bwd_t(int64_t n_rows, int64_t n_cols, int64_t nnz_cap, int64_t k, int G, bool full,
                  const int32_t* col_ptr, const int32_t* row_idx, const void* val, const void* Gm,
                  int64_t ldg, int gal, const void* X, int64_t ldx, int xal, void* dX,
                  int64_t lddx, int dx_f64, int dxal, void* dval, int dv_f64, int grid,
                  int block, hipStream_t s) {
#define SPM_CALL_F(GW, F)                                                                      \
  k_spmm_bwd<VT, GT, XT, ACC, GW, F><<<dim3(grid), dim3(block), 0, s>>>(                       \
      n_rows, n_cols, nnz_cap, k, col_ptr, row_idx, static_cast<const VT*>(val),               \
      static_cast<const GT*>(Gm), ldg, gal, static_cast<const XT*>(X), ldx, xal, dX, lddx,     \
      dx_f64, dxal, dval, dv_f64)
#define SPM_CALL(GW) SPM_CALL_F(GW, false)
  if (full && G == 8) SPM_CALL_F(8, true);
  else if (full && G == 16) SPM_CALL_F(16, true);
  else if (full && G == 32) SPM_CALL_F(32, true);
  else SPM_GW_SWITCH(G, SPM_CALL)
#undef SPM_CALL
#undef SPM_CALL_F
}

size_t dsize(spm_dtype t) { return t == SPM_F64 ? 8 : (t == SPM_F32 ? 4 : 2); }

// binary32 accumulation only when bfloat16 is involved and binary64 is not.
bool acc_is_f32(spm_dtype vt, spm_dtype xt) { return xt == SPM_BF16 && vt != SPM_F64; }

int spmm_grid(int64_t groups, int G, int block) {
  const spm_tuning tu = tuning();
  const int64_t per_block = block / G;
  int64_t want = ceil_div(groups, per_block);
  int64_t cap = (int64_t)cu_count() * tu.spmm_blocks_per_cu;
  if (want > cap) want = cap;
  if (want < 1) want = 1;
  return (int)want;
}

}  // namespace

// ============================================================================================
// C ABI
// ============================================================================================
extern "C" {

const char* spm_status_string(int status) {
  switch (status) {
    case SPM_OK: return "ok";
    case SPM_EINVAL: return "invalid argument";
    case SPM_EBOUNDS: return "triplet index out of range";
    case SPM_EOVERFLOW: return "size does not fit in int32";
    case SPM_EWORKSPACE: return "workspace too small";
    case SPM_EDTYPE: return "unsupported element type";
    case SPM_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* spm_version(void) { return "0.1.0 gfx950"; }

spm_status spm_coo_to_csc_workspace(int64_t n_rows, int64_t n_cols, int64_t nnz_in,
                                    size_t* ws_bytes) {
  if (!ws_bytes) return SPM_EINVAL;
  spm_status st = check_dims(n_rows, n_cols, nnz_in);
  if (st != SPM_OK) return st;
  *ws_bytes = asm_layout(n_cols, nnz_in).total;
  return SPM_OK;
}

spm_status spm_coo_to_csc(int64_t n_rows, int64_t n_cols, int64_t nnz_in, const int32_t* row,
                          const int32_t* col, const void* val, spm_dtype val_type,
                          int32_t* col_ptr, int32_t* row_idx, void* val_out, spm_dtype out_type,
                          int32_t* info, void* ws, size_t ws_bytes, void* stream) {
  SPM_RANGE("spm_coo_to_csc");
  spm_status st = check_dims(n_rows, n_cols, nnz_in);
  if (st != SPM_OK) return st;
  if (val_type != SPM_F64 && val_type != SPM_F32 && val_type != SPM_BF16) return SPM_EDTYPE;
  if (out_type != SPM_F64 && out_type != SPM_F32) return SPM_EDTYPE;
  if (!col_ptr || !info || !ws) return SPM_EINVAL;
  if (nnz_in > 0 && (!row || !col || !val || !row_idx || !val_out)) return SPM_EINVAL;
  if (!aligned(ws, 256)) return SPM_EINVAL;
  const AsmLayout L = asm_layout(n_cols, nnz_in);
  if (ws_bytes < L.total) return SPM_EWORKSPACE;
  return assemble_impl(n_rows, n_cols, nnz_in, row, col, val, val_type, col_ptr, row_idx,
                       val_out, out_type, info, static_cast<char*>(ws), L,
                       static_cast<hipStream_t>(stream), nullptr);
}

spm_status spm_csc_plan_size(int64_t n_rows, int64_t n_cols, int64_t nnz_cap, size_t* plan_bytes,
                             size_t* ws_bytes) {
  if (!plan_bytes || !ws_bytes) return SPM_EINVAL;
  spm_status st = check_dims(n_rows, n_cols, nnz_cap);
  if (st != SPM_OK) return st;
  *plan_bytes = plan_parts(n_rows, nnz_cap).total;
  *ws_bytes = plan_ws_layout(n_rows, n_cols, nnz_cap).total;
  return SPM_OK;
}

}  // extern "C"

namespace {

// Assembly on a validated argument set.  With fz != nullptr (fused plan, partition path
// only) the survivors also feed the plan's row partition and the plan's level 2 runs last.
spm_status assemble_impl(int64_t n_rows, int64_t n_cols, int64_t nnz_in, const int32_t* row,
                         const int32_t* col, const void* val, spm_dtype val_type,
                         int32_t* col_ptr, int32_t* row_idx, void* val_out, spm_dtype out_type,
                         int32_t* info, char* w, const AsmLayout& L, hipStream_t s,
                         const FuseCtx* fz) {
  uint32_t* colcnt = reinterpret_cast<uint32_t*>(w + L.colcnt);
  uint64_t* scan_state = reinterpret_cast<uint64_t*>(w + L.scan_state);
  uint64_t* fold_state = reinterpret_cast<uint64_t*>(w + L.fold_state);
  uint32_t* tickets = reinterpret_cast<uint32_t*>(w + L.tickets);
  int32_t* colstart = reinterpret_cast<int32_t*>(w + L.colstart);
  int32_t* first = reinterpret_cast<int32_t*>(w + L.first);
  uint64_t* bucket = reinterpret_cast<uint64_t*>(w + L.bucket);
  uint64_t* scratch = reinterpret_cast<uint64_t*>(w + L.scratch);

  (void)hipGetLastError();
  const int cap = cu_count() * 16;
  if (L.pp.ok) {
    // two-level partition by column: no device-wide atomics, no inter-workgroup waiting
    const PartParams& P = L.pp;
    uint32_t* table = reinterpret_cast<uint32_t*>(w + L.table);
    uint32_t* rowoff = reinterpret_cast<uint32_t*>(w + L.rowoff);
    uint32_t* btot = reinterpret_cast<uint32_t*>(w + L.btot);
    int32_t* bstart = reinterpret_cast<int32_t*>(w + L.bstart);
    uint4* brec = reinterpret_cast<uint4*>(w + L.brec);
    uint32_t* bvhi = reinterpret_cast<uint32_t*>(w + L.bvhi);
    uint32_t* trow = reinterpret_cast<uint32_t*>(w + L.trow);
    double* tval = reinterpret_cast<double*>(w + L.tval);
    uint32_t* bkept = reinterpret_cast<uint32_t*>(w + L.bkept);
    PartSrcCoo src{row, col, (int32_t)n_rows, (int32_t)n_cols, nnz_in};
    uint32_t* flags = reinterpret_cast<uint32_t*>(w + L.flags);
    uint32_t* big = level2_big_ok(P.b, P.CB) ? reinterpret_cast<uint32_t*>(w + L.big) : nullptr;
    uint32_t* big2 = (fz && level2_big_ok(fz->F->Q.b, fz->F->Q.CB))
                         ? reinterpret_cast<uint32_t*>(w + fz->F->big2) : nullptr;
    k_part_hist<kPartNT, PartSrcCoo>
        <<<dim3((unsigned)P.ntiles), dim3(kPartNT), 4 * (size_t)P.CB, s>>>(
            src, P.b, P.CB, P.ntiles, P.T1, table, flags, big, big2,
            sub_counts(L.sp, w, L.subcnt));
    k_rows_scan<kNT><<<dim3((unsigned)P.CB), dim3(kNT), 0, s>>>(
        (const uint32_t*)table, P.ntiles, rowoff, btot, (const uint32_t*)flags, P.ntiles, info,
        (uint32_t)kPartCap, big);
    // fused plan: level 2 also counts the survivors per (row bucket, column bucket)
    const L2RowCount rc = fz ? L2RowCount{reinterpret_cast<uint32_t*>(w + fz->F->table2),
                                          fz->F->Q.b, fz->F->Q.CB, P.CB}
                             : L2RowCount{nullptr, 0, 0, 0};
#define SPM_L2(VT)                                                                             \
  do {                                                                                         \
  launch_scatter<PartSrcCoo, VT>(src, P, L.sp, rowoff, btot, bstart, brec,                    \
                                 static_cast<const VT*>(val), bvhi,                            \
                                 reinterpret_cast<uint4*>(bucket), trow,                       \
                                 reinterpret_cast<uint32_t*>(w + L.sbro),                      \
                                 reinterpret_cast<const uint32_t*>(w + L.subcnt), s);          \
  launch_level2<false, VT>(P.b, P.CB, n_cols, (const int32_t*)bstart, (const uint4*)brec,     \
                           (const uint32_t*)bvhi, bucket, scratch, (int32_t*)nullptr,          \
                           (int32_t*)nullptr, (int32_t*)nullptr, static_cast<const VT*>(val),  \
                           (VT*)nullptr, col_ptr, trow, tval, bkept, sub_shift(n_rows, P.b),   \
                           rc, big, s);                                                        \
  } while (0)
    if (val_type == SPM_F64) SPM_L2(double);
    else if (val_type == SPM_F32) SPM_L2(float);
    else SPM_L2(bf16_t);
#undef SPM_L2
    int32_t* boff = nullptr;
    if (P.CB > kEmitReduceMax) {
      boff = reinterpret_cast<int32_t*>(w + L.boff);
      k_small_scan<kSmallScanNT, kSmallScanIPT><<<dim3(1), dim3(kSmallScanNT), 0, s>>>(
          (const uint32_t*)bkept, (int64_t)P.CB, boff);
    }
    EmitPlan ep{0, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    size_t emit_lds = 0;
    if (fz) {
      const FuseLayout& F = *fz->F;
      const PartParams& Q = F.Q;
      uint32_t* table2 = reinterpret_cast<uint32_t*>(w + F.table2);
      uint32_t* rowoff2 = reinterpret_cast<uint32_t*>(w + F.rowoff2);
      uint32_t* btot2 = reinterpret_cast<uint32_t*>(w + F.btot2);
      int32_t* bstart2 = reinterpret_cast<int32_t*>(w + F.bstart2);
      // the column buckets are the tiles of the plan's level 1; no status flags to fold
      k_rows_scan<kNT><<<dim3((unsigned)Q.CB), dim3(kNT), 0, s>>>(
          (const uint32_t*)table2, (int64_t)P.CB, rowoff2, btot2, (const uint32_t*)nullptr,
          (int64_t)0, fz->plan_info, (uint32_t)kPartCap, big2);
      ep = EmitPlan{Q.b, Q.CB, rowoff2, btot2, bstart2, brec, bvhi, fz->plan_info};
      emit_lds = 4 * ((size_t)Q.CB + ((size_t)1 << P.b) + 1);
    }
    k_part_emit<kNT><<<dim3((unsigned)P.CB), dim3(kNT), emit_lds, s>>>(
        P.b, P.CB, n_cols, (const int32_t*)bstart, (const uint32_t*)bkept, (const int32_t*)boff,
        (const uint32_t*)trow, (const double*)tval, col_ptr, row_idx, val_out,
        out_type == SPM_F64 ? 1 : 0, info, ep);
    if (fz) {
      const PartParams& Q = fz->F->Q;
      const PlanParts& PP = *fz->P;
      int32_t* row_ptr = reinterpret_cast<int32_t*>(fz->plan + PP.row_ptr);
      int32_t* col_t = reinterpret_cast<int32_t*>(fz->plan + PP.col_t);
      int32_t* perm = reinterpret_cast<int32_t*>(fz->plan + PP.perm);
      const int32_t* bstart2 = reinterpret_cast<const int32_t*>(w + fz->F->bstart2);
#define SPM_PL2(VT)                                                                            \
  launch_level2<true, VT>(Q.b, Q.CB, n_rows, bstart2, (const uint4*)brec,                      \
                          (const uint32_t*)bvhi, bucket, scratch, row_ptr, col_t, perm,        \
                          static_cast<const VT*>(val_out), static_cast<VT*>(fz->val_plan),     \
                          (int32_t*)nullptr, (uint32_t*)nullptr, (double*)nullptr,             \
                          (uint32_t*)nullptr, sub_shift(n_cols, Q.b),                          \
                          L2RowCount{nullptr, 0, 0, 0}, big2, s)
      if (out_type == SPM_F64) SPM_PL2(double);
      else SPM_PL2(float);
#undef SPM_PL2
    }
    return launch_status();
  } else {
    // one counter per column in global memory (shapes with more columns than the partition
    // covers, and n_cols = 0); counters, look-back states and info start at zero
    k_zero2<<<dim3(grid_for((int64_t)(L.zero_bytes / 4), kNT * 4, cap)), dim3(kNT), 0, s>>>(
        reinterpret_cast<uint32_t*>(w), (int64_t)(L.zero_bytes / 4),
        reinterpret_cast<uint32_t*>(info), (int64_t)2);
    if (nnz_in > 0)
      k_col_hist<kNT><<<dim3(grid_for(nnz_in, kNT * 4, cap)), dim3(kNT), 0, s>>>(
          row, col, nnz_in, (int32_t)n_rows, (int32_t)n_cols, colcnt, info);
    launch_scan<kNT, kScanIPT>(colcnt, n_cols, colstart, scan_state, tickets + 0, s);
    k_tile_first<<<dim3(grid_for(n_cols + 1, kNT, cap)), dim3(kNT), 0, s>>>(
        (const int32_t*)colstart, n_cols, (int64_t)kFoldTile, L.fold_tiles, first);
    if (nnz_in > 0) {
      k_col_scatter<kNT><<<dim3(grid_for(nnz_in, kNT * 4, cap)), dim3(kNT), 0, s>>>(
          row, col, nnz_in, (int32_t)n_rows, (int32_t)n_cols, colstart, colcnt, bucket);
      k_segsort<kNT, kSortCap, false>
          <<<dim3((unsigned)ceil_div(nnz_in, kSortT)), dim3(kNT), 0, s>>>(
              bucket, colstart, n_cols, (int64_t)kSortT, (const int32_t*)first, scratch,
              (int32_t*)nullptr, (int32_t*)nullptr);
    }
  }
  const int out_f64 = out_type == SPM_F64 ? 1 : 0;
  switch (val_type) {
    case SPM_F64:
      launch_fold<double>(bucket, colstart, n_cols, static_cast<const double*>(val), col_ptr,
                          row_idx, val_out, out_f64, info, first, fold_state, tickets + 1,
                          L.fold_tiles, s);
      break;
    case SPM_F32:
      launch_fold<float>(bucket, colstart, n_cols, static_cast<const float*>(val), col_ptr,
                         row_idx, val_out, out_f64, info, first, fold_state, tickets + 1,
                         L.fold_tiles, s);
      break;
    default:
      launch_fold<bf16_t>(bucket, colstart, n_cols, static_cast<const bf16_t*>(val), col_ptr,
                          row_idx, val_out, out_f64, info, first, fold_state, tickets + 1,
                          L.fold_tiles, s);
      break;
  }
  return launch_status();
}

// Plan build for one value type VT (the type of the optional values carried to plan order),
// into row_ptr[n_rows+1], col_t[nnz_cap], perm[nnz_cap] wherever they are.
template <typename VT>
void plan_build_into(int64_t n_rows, int64_t n_cols, int64_t nnz_cap, const int32_t* col_ptr,
                     const int32_t* row_idx, const VT* val, VT* val_plan, int32_t* row_ptr,
                     int32_t* col_t, int32_t* perm, int32_t* info, char* w,
                     const PlanLayout& L, hipStream_t s) {
  uint64_t* scan_state = reinterpret_cast<uint64_t*>(w + L.scan_state);
  uint32_t* tickets = reinterpret_cast<uint32_t*>(w + L.tickets);
  uint64_t* bucket = reinterpret_cast<uint64_t*>(w + L.bucket);
  uint64_t* scratch = reinterpret_cast<uint64_t*>(w + L.scratch);
  const int cap = cu_count() * 16;
  if (L.pp.ok) {
    // two-level partition by row: no device-wide atomics, no inter-workgroup waiting; the
    // values (if any) travel in the partition records
    const PartParams& Q = L.pp;
    int32_t* colarr = reinterpret_cast<int32_t*>(w + L.colarr);
    uint32_t* table = reinterpret_cast<uint32_t*>(w + L.table);
    uint32_t* rowoff = reinterpret_cast<uint32_t*>(w + L.rowoff);
    uint32_t* btot = reinterpret_cast<uint32_t*>(w + L.btot);
    int32_t* bstart = reinterpret_cast<int32_t*>(w + L.bstart);
    uint4* brec = reinterpret_cast<uint4*>(w + L.brec);
    uint32_t* bvhi = reinterpret_cast<uint32_t*>(w + L.bvhi);
    uint32_t* flags = reinterpret_cast<uint32_t*>(w + L.flags);
    k_expand_columns<kNT><<<dim3(expand_grid(n_cols)), dim3(kNT), 0, s>>>(
        col_ptr, n_cols, nnz_cap, colarr, info, flags);
    PartSrcCsc src{row_idx, colarr, col_ptr, n_rows, n_cols, nnz_cap};
    uint32_t* big = level2_big_ok(Q.b, Q.CB) ? reinterpret_cast<uint32_t*>(w + L.big) : nullptr;
    k_part_hist<kPartNT, PartSrcCsc>
        <<<dim3((unsigned)Q.ntiles), dim3(kPartNT), 4 * (size_t)Q.CB, s>>>(
            src, Q.b, Q.CB, Q.ntiles, Q.T1, table, flags + expand_grid(n_cols), big,
            (uint32_t*)nullptr, sub_counts(L.sp, w, L.subcnt));
    k_rows_scan<kNT><<<dim3((unsigned)Q.CB), dim3(kNT), 0, s>>>(
        (const uint32_t*)table, Q.ntiles, rowoff, btot, (const uint32_t*)flags,
        (int64_t)expand_grid(n_cols) + Q.ntiles, info, (uint32_t)kPartCap, big);
    launch_scatter<PartSrcCsc, VT>(src, Q, L.sp, rowoff, btot, bstart, brec,
                                   val_plan ? val : (const VT*)nullptr, bvhi,
                                   reinterpret_cast<uint4*>(bucket),
                                   reinterpret_cast<uint32_t*>(w + L.ivhi),
                                   reinterpret_cast<uint32_t*>(w + L.sbro),
                                   reinterpret_cast<const uint32_t*>(w + L.subcnt), s);
    launch_level2<true, VT>(Q.b, Q.CB, n_rows, (const int32_t*)bstart, (const uint4*)brec,
                            (const uint32_t*)bvhi, bucket, scratch, row_ptr, col_t, perm, val,
                            val_plan, (int32_t*)nullptr, (uint32_t*)nullptr, (double*)nullptr,
                            (uint32_t*)nullptr, sub_shift(n_cols, Q.b),
                            L2RowCount{nullptr, 0, 0, 0}, big, s);
  } else {
    k_zero2<<<dim3(grid_for((int64_t)(L.zero_bytes / 4), kNT * 4, cap)), dim3(kNT), 0, s>>>(
        reinterpret_cast<uint32_t*>(w), (int64_t)(L.zero_bytes / 4),
        reinterpret_cast<uint32_t*>(info), (int64_t)2);
    uint32_t* rowcnt = reinterpret_cast<uint32_t*>(w + L.rowcnt);
    int32_t* first = reinterpret_cast<int32_t*>(w + L.first);
    k_plan_hist<kNT>
        <<<dim3(grid_for(nnz_cap > n_cols ? nnz_cap : n_cols, kNT, cap)), dim3(kNT), 0, s>>>(
            col_ptr, row_idx, n_rows, n_cols, nnz_cap, rowcnt, info);
    launch_scan<kNT, kScanIPT>(rowcnt, n_rows, row_ptr, scan_state, tickets, s);
    if (nnz_cap > 0 && n_cols > 0) {
      k_row_scatter<kNT><<<dim3(grid_for(n_cols, kNT, cap)), dim3(kNT), 0, s>>>(
          col_ptr, row_idx, n_rows, n_cols, nnz_cap, row_ptr, rowcnt, bucket);
      k_tile_first<<<dim3(grid_for(n_rows + 1, kNT, cap)), dim3(kNT), 0, s>>>(
          (const int32_t*)row_ptr, n_rows, (int64_t)kSortT, L.sort_tiles, first);
      k_segsort<kNT, kSortCap, true><<<dim3((unsigned)L.sort_tiles), dim3(kNT), 0, s>>>(
          bucket, row_ptr, n_rows, (int64_t)kSortT, (const int32_t*)first, scratch, col_t, perm);
      if (val_plan)
        k_plan_values<kNT, VT><<<dim3(grid_for(nnz_cap, kNT * 4, cap)), dim3(kNT), 0, s>>>(
            col_ptr, n_cols, nnz_cap, perm, val, val_plan);
    }
  }
}

// Plan build into one plan buffer (layout of include/spm.h).
template <typename VT>
void plan_build_t(int64_t n_rows, int64_t n_cols, int64_t nnz_cap, const int32_t* col_ptr,
                  const int32_t* row_idx, const VT* val, VT* val_plan, char* pl, int32_t* info,
                  char* w, const PlanParts& P, const PlanLayout& L, hipStream_t s) {
  plan_build_into<VT>(n_rows, n_cols, nnz_cap, col_ptr, row_idx, val, val_plan,
                      reinterpret_cast<int32_t*>(pl + P.row_ptr),
                      reinterpret_cast<int32_t*>(pl + P.col_t),
                      reinterpret_cast<int32_t*>(pl + P.perm), info, w, L, s);
}

// Transpose: the plan build writes the row index of A, which is the CSC of A^T, straight
// into the caller's arrays; the CSC slot of each element (perm) goes to the workspace, after
// the plan build's own layout.
size_t transpose_ws_bytes(int64_t n_rows, int64_t n_cols, int64_t nnz_cap, size_t* perm_off) {
  const PlanLayout L = plan_ws_layout(n_rows, n_cols, nnz_cap);
  Carve c;
  c.off = L.total;
  *perm_off = c.take(sizeof(int32_t) * (size_t)nnz_cap);
  return c.off;
}

// Merge path (spm_mergepath.h): one look-back state per workgroup tile of kNT * kMergeE merged
// positions, the column of each tile's start (and of position M), the tile ticket.  k_merge_cols
// writes the columns and clears the rest at the start of every call.
struct MpLayout {
  size_t scan_state, tile_col, ticket, end;
  int64_t ntiles;
};

void mp_carve(Carve& c, int64_t m_cap, MpLayout& M) {
  M.ntiles = std::max<int64_t>(1, ceil_div(m_cap, (int64_t)kNT * kMergeE));
  M.scan_state = c.take(sizeof(uint64_t) * (size_t)M.ntiles);
  M.tile_col = c.take(sizeof(int32_t) * (size_t)(M.ntiles + 1));
  M.ticket = c.take(sizeof(uint32_t) * 4);
  M.end = c.off;
}

// Workgroups of kernel k (kNT threads each) that fit on the current device at once, 0 if
// unknown (cached per device; one cache per kernel type).
template <typename K>
int64_t resident_blocks(K k) {
  static int64_t cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cached[dev] == 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k),
                                                     kNT, 0) != hipSuccess)
      per_cu = 0;
    cached[dev] = per_cu > 0 ? (int64_t)per_cu * cu_count() : -1;
  }
  return cached[dev] > 0 ? cached[dev] : 0;
}

// The merge of the two lists into (col_ptr, row_idx, val_out).  info_clear: info when nothing
// was reported before in this call (its info[1] is cleared), else null (info[1] keeps the
// earlier report unless the merge finds worse).
template <typename VA, typename VB>
void mp_run(const MergeLists& ML, const VA* a_v, const VB* b_v, int32_t* col_ptr,
            int32_t* row_idx, void* val_out, int out_f64, int64_t out_cap, int32_t* info,
            int32_t* info_clear, char* w, const MpLayout& M, hipStream_t s) {
  uint64_t* state = reinterpret_cast<uint64_t*>(w + M.scan_state);
  int32_t* tile_col = reinterpret_cast<int32_t*>(w + M.tile_col);
  uint32_t* ticket = reinterpret_cast<uint32_t*>(w + M.ticket);
  const int64_t seg = (int64_t)kNT * kMergeE;
  const int64_t cblocks = std::min<int64_t>(ceil_div(ML.n_cols + 1, (int64_t)kNT), 1 << 16);
  k_merge_cols<kNT><<<dim3((unsigned)cblocks), dim3(kNT), 0, s>>>(ML, seg, M.ntiles, tile_col,
                                                                   state, ticket, info_clear);
  const int by_ticket = M.ntiles > resident_blocks(k_merge<kNT, VA, VB>) ? 1 : 0;
  k_merge<kNT, VA, VB><<<dim3((unsigned)M.ntiles), dim3(kNT), 0, s>>>(
      ML, a_v, b_v, (const int32_t*)tile_col, col_ptr, row_idx, val_out, out_f64, out_cap,
      state, ticket, by_ticket, info, (int32_t)SPM_EINVAL, (int32_t)SPM_EBOUNDS);
}

// Batch insertion (Section 3.1: the new elements sorted, then merged with the existing
// arrays): the new triplets alone go through the partition by column, with level 2 in its
// sorting form (no fold): per column their rows in increasing order, equal rows in input
// order, with their values (b_cp, b_ri, b_v; b_perm is the input position, unused); then the
// merge path folds every location, the existing value first.
struct InsertLayout {
  PartParams pp;
  SplitParams sp;
  size_t table, rowoff, btot, bstart, brec, bvhi, flags, big, bucket, scratch, ivhi, sbro,
      subcnt;
  size_t b_cp, b_ri, b_perm, b_v;
  MpLayout mp;
  size_t total;
};

InsertLayout insert_layout(int64_t n_cols, int64_t cap_a, int64_t nnz_t) {
  InsertLayout L;
  Carve c;
  L.pp = part_params(n_cols, nnz_t);
  L.sp = split_params(L.pp);
  const bool ok = L.pp.ok;
  const int64_t tab = ok ? (int64_t)L.pp.CB * L.pp.ntiles : 0;
  const int64_t cb = ok ? L.pp.CB : 0;
  const size_t nt = (size_t)nnz_t;
  mp_carve(c, cap_a + nnz_t, L.mp);
  L.table = c.take(sizeof(uint32_t) * (size_t)tab);
  L.rowoff = c.take(sizeof(uint32_t) * (size_t)tab);
  L.btot = c.take(sizeof(uint32_t) * (size_t)cb);
  L.bstart = c.take(sizeof(int32_t) * (size_t)(cb + 1));
  L.brec = c.take(16 * nt);
  L.bvhi = c.take(sizeof(uint32_t) * nt);
  L.flags = c.take(sizeof(uint32_t) * (size_t)(ok ? L.pp.ntiles : 0));
  L.big = c.take(sizeof(uint32_t) * (size_t)(cb + 1));
  L.bucket = c.take(sizeof(uint64_t) * nt);  // bucket and scratch back to back: also the
  L.scratch = c.take(sizeof(uint64_t) * nt);  // two-pass level 1's records
  L.ivhi = c.take(sizeof(uint32_t) * (L.sp.on ? nt : 0));
  L.sbro = c.take(sizeof(uint32_t) * (size_t)(L.sp.on ? L.sp.SB * (L.pp.ntiles + 1) : 0));
  L.subcnt = c.take(sizeof(uint32_t) *
                    (size_t)(L.sp.on ? L.sp.SB * L.sp.SH * L.pp.ntiles : 0));
  L.b_cp = c.take(sizeof(int32_t) * (size_t)(n_cols + 1));
  L.b_ri = c.take(sizeof(int32_t) * nt);
  L.b_perm = c.take(sizeof(int32_t) * nt);
  L.b_v = c.take(sizeof(double) * nt);
  L.total = c.off;
  return L;
}

template <typename VT>
void insert_t(int64_t n_rows, int64_t n_cols, int64_t cap_a, const int32_t* a_col_ptr,
              const int32_t* a_row_idx, const VT* a_val, int64_t nnz_t, const int32_t* row,
              const int32_t* col, const VT* val, int32_t* col_ptr, int32_t* row_idx,
              void* val_out, int out_f64, int32_t* info, char* w, const InsertLayout& L,
              hipStream_t s) {
  const PartParams& P = L.pp;
  uint32_t* table = reinterpret_cast<uint32_t*>(w + L.table);
  uint32_t* rowoff = reinterpret_cast<uint32_t*>(w + L.rowoff);
  uint32_t* btot = reinterpret_cast<uint32_t*>(w + L.btot);
  int32_t* bstart = reinterpret_cast<int32_t*>(w + L.bstart);
  uint4* brec = reinterpret_cast<uint4*>(w + L.brec);
  uint32_t* bvhi = reinterpret_cast<uint32_t*>(w + L.bvhi);
  uint32_t* flags = reinterpret_cast<uint32_t*>(w + L.flags);
  uint64_t* bucket = reinterpret_cast<uint64_t*>(w + L.bucket);
  uint64_t* scratch = reinterpret_cast<uint64_t*>(w + L.scratch);
  int32_t* b_cp = reinterpret_cast<int32_t*>(w + L.b_cp);
  int32_t* b_ri = reinterpret_cast<int32_t*>(w + L.b_ri);
  int32_t* b_perm = reinterpret_cast<int32_t*>(w + L.b_perm);
  VT* b_v = reinterpret_cast<VT*>(w + L.b_v);
  uint32_t* big = level2_big_ok(P.b, P.CB) ? reinterpret_cast<uint32_t*>(w + L.big) : nullptr;
  // the new triplets sorted by (column, row, input position); out-of-range ones are skipped
  // and reported in info[1] (k_rows_scan)
  PartSrcCoo src{row, col, (int32_t)n_rows, (int32_t)n_cols, nnz_t};
  k_part_hist<kPartNT, PartSrcCoo>
      <<<dim3((unsigned)P.ntiles), dim3(kPartNT), 4 * (size_t)P.CB, s>>>(
          src, P.b, P.CB, P.ntiles, P.T1, table, flags, big, (uint32_t*)nullptr,
          sub_counts(L.sp, w, L.subcnt));
  k_rows_scan<kNT><<<dim3((unsigned)P.CB), dim3(kNT), 0, s>>>(
      (const uint32_t*)table, P.ntiles, rowoff, btot, (const uint32_t*)flags, P.ntiles, info,
      (uint32_t)kPartCap, big);
  launch_scatter<PartSrcCoo, VT>(src, P, L.sp, rowoff, btot, bstart, brec, val, bvhi,
                                 reinterpret_cast<uint4*>(bucket),
                                 reinterpret_cast<uint32_t*>(w + L.ivhi),
                                 reinterpret_cast<uint32_t*>(w + L.sbro),
                                 reinterpret_cast<const uint32_t*>(w + L.subcnt), s);
  launch_level2<true, VT>(P.b, P.CB, n_cols, (const int32_t*)bstart, (const uint4*)brec,
                          (const uint32_t*)bvhi, bucket, scratch, b_cp, b_ri, b_perm, val, b_v,
                          (int32_t*)nullptr, (uint32_t*)nullptr, (double*)nullptr,
                          (uint32_t*)nullptr, sub_shift(n_rows, P.b),
                          L2RowCount{nullptr, 0, 0, 0}, big, s);
  const MergeLists ML{a_col_ptr, a_row_idx, cap_a, b_cp, b_ri, nnz_t, n_rows, n_cols, false};
  mp_run<VT, VT>(ML, a_val, b_v, col_ptr, row_idx, val_out, out_f64, cap_a + nnz_t, info,
                 (int32_t*)nullptr, w, L.mp, s);
}

}  // namespace

extern "C" {

spm_status spm_csc_plan_build(int64_t n_rows, int64_t n_cols, int64_t nnz_cap,
                              const int32_t* col_ptr, const int32_t* row_idx, const void* val,
                              spm_dtype val_type, void* plan, size_t plan_bytes,
                              void* val_plan, int32_t* info, void* ws, size_t ws_bytes,
                              void* stream) {
  SPM_RANGE("spm_csc_plan_build");
  spm_status st = check_dims(n_rows, n_cols, nnz_cap);
  if (st != SPM_OK) return st;
  if (!col_ptr || !plan || !info || !ws) return SPM_EINVAL;
  if (nnz_cap > 0 && !row_idx) return SPM_EINVAL;
  if ((val == nullptr) != (val_plan == nullptr)) return SPM_EINVAL;
  if (val && val_type != SPM_F64 && val_type != SPM_F32) return SPM_EDTYPE;
  if (!aligned(ws, 256) || !aligned(plan, 256)) return SPM_EINVAL;
  const PlanParts P = plan_parts(n_rows, nnz_cap);
  const PlanLayout L = plan_ws_layout(n_rows, n_cols, nnz_cap);
  if (plan_bytes < P.total || ws_bytes < L.total) return SPM_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  if (val && val_type == SPM_F64)
    plan_build_t<double>(n_rows, n_cols, nnz_cap, col_ptr, row_idx,
                         static_cast<const double*>(val), static_cast<double*>(val_plan),
                         static_cast<char*>(plan), info, static_cast<char*>(ws), P, L, s);
  else
    plan_build_t<float>(n_rows, n_cols, nnz_cap, col_ptr, row_idx,
                        static_cast<const float*>(val), static_cast<float*>(val_plan),
                        static_cast<char*>(plan), info, static_cast<char*>(ws), P, L, s);
  return launch_status();
}

spm_status spm_coo_to_csc_plan_size(int64_t n_rows, int64_t n_cols, int64_t nnz_in,
                                    size_t* plan_bytes, size_t* ws_bytes) {
  if (!plan_bytes || !ws_bytes) return SPM_EINVAL;
  spm_status st = check_dims(n_rows, n_cols, nnz_in);
  if (st != SPM_OK) return st;
  *plan_bytes = plan_parts(n_rows, nnz_in).total;
  *ws_bytes = fuse_layout(n_rows, n_cols, nnz_in).total;
  return SPM_OK;
}

spm_status spm_coo_to_csc_plan(int64_t n_rows, int64_t n_cols, int64_t nnz_in,
                               const int32_t* row, const int32_t* col, const void* val,
                               spm_dtype val_type, int32_t* col_ptr, int32_t* row_idx,
                               void* val_out, spm_dtype out_type, int32_t* info, void* plan,
                               size_t plan_bytes, void* val_plan, int32_t* plan_info, void* ws,
                               size_t ws_bytes, void* stream) {
  SPM_RANGE("spm_coo_to_csc_plan");
  spm_status st = check_dims(n_rows, n_cols, nnz_in);
  if (st != SPM_OK) return st;
  if (val_type != SPM_F64 && val_type != SPM_F32 && val_type != SPM_BF16) return SPM_EDTYPE;
  if (out_type != SPM_F64 && out_type != SPM_F32) return SPM_EDTYPE;
  if (!col_ptr || !info || !plan || !plan_info || !ws) return SPM_EINVAL;
  if (nnz_in > 0 && (!row || !col || !val || !row_idx || !val_out)) return SPM_EINVAL;
  if (!aligned(ws, 256) || !aligned(plan, 256)) return SPM_EINVAL;
  const PlanParts P = plan_parts(n_rows, nnz_in);
  const FuseLayout F = fuse_layout(n_rows, n_cols, nnz_in);
  if (plan_bytes < P.total || ws_bytes < F.total) return SPM_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (F.fused) {
    const FuseCtx fz{&F, n_rows, &P, static_cast<char*>(plan), val_plan, plan_info};
    return assemble_impl(n_rows, n_cols, nnz_in, row, col, val, val_type, col_ptr, row_idx,
                         val_out, out_type, info, w, F.A, s, &fz);
  }
  // the two builds one after the other on the same workspace
  st = assemble_impl(n_rows, n_cols, nnz_in, row, col, val, val_type, col_ptr, row_idx,
                     val_out, out_type, info, w, F.A, s, nullptr);
  if (st != SPM_OK) return st;
  const PlanLayout PL = plan_ws_layout(n_rows, n_cols, nnz_in);
  (void)hipGetLastError();
  if (out_type == SPM_F64)
    plan_build_t<double>(n_rows, n_cols, nnz_in, col_ptr, row_idx,
                         static_cast<const double*>(val_out), static_cast<double*>(val_plan),
                         static_cast<char*>(plan), plan_info, w, P, PL, s);
  else
    plan_build_t<float>(n_rows, n_cols, nnz_in, col_ptr, row_idx,
                        static_cast<const float*>(val_out), static_cast<float*>(val_plan),
                        static_cast<char*>(plan), plan_info, w, P, PL, s);
  return launch_status();
}

spm_status spm_csc_transpose_workspace(int64_t n_rows, int64_t n_cols, int64_t nnz_cap,
                                       size_t* ws_bytes) {
  if (!ws_bytes) return SPM_EINVAL;
  spm_status st = check_dims(n_rows, n_cols, nnz_cap);
  if (st != SPM_OK) return st;
  size_t perm_off;
  *ws_bytes = transpose_ws_bytes(n_rows, n_cols, nnz_cap, &perm_off);
  return SPM_OK;
}

spm_status spm_csc_transpose(int64_t n_rows, int64_t n_cols, int64_t nnz_cap,
                             const int32_t* col_ptr, const int32_t* row_idx, const void* val,
                             spm_dtype val_type, int32_t* t_col_ptr, int32_t* t_row_idx,
                             void* t_val, int32_t* info, void* ws, size_t ws_bytes,
                             void* stream) {
  SPM_RANGE("spm_csc_transpose");
  spm_status st = check_dims(n_rows, n_cols, nnz_cap);
  if (st != SPM_OK) return st;
  if (val_type != SPM_F64 && val_type != SPM_F32) return SPM_EDTYPE;
  if (!col_ptr || !t_col_ptr || !info || !ws) return SPM_EINVAL;
  if (nnz_cap > 0 && (!row_idx || !val || !t_row_idx || !t_val)) return SPM_EINVAL;
  if (!aligned(ws, 256)) return SPM_EINVAL;
  size_t perm_off;
  if (ws_bytes < transpose_ws_bytes(n_rows, n_cols, nnz_cap, &perm_off))
    return SPM_EWORKSPACE;
  const PlanLayout L = plan_ws_layout(n_rows, n_cols, nnz_cap);
  char* w = static_cast<char*>(ws);
  int32_t* perm = reinterpret_cast<int32_t*>(w + perm_off);
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  // a CSC with no stored element still needs its (all-zero) offsets; the plan build writes
  // them, and carries the values only when there are some
  if (val_type == SPM_F64)
    plan_build_into<double>(n_rows, n_cols, nnz_cap, col_ptr, row_idx,
                            nnz_cap ? static_cast<const double*>(val) : nullptr,
                            nnz_cap ? static_cast<double*>(t_val) : nullptr, t_col_ptr,
                            t_row_idx, perm, info, w, L, s);
  else
    plan_build_into<float>(n_rows, n_cols, nnz_cap, col_ptr, row_idx,
                           nnz_cap ? static_cast<const float*>(val) : nullptr,
                           nnz_cap ? static_cast<float*>(t_val) : nullptr, t_col_ptr,
                           t_row_idx, perm, info, w, L, s);
  return launch_status();
}

spm_status spm_csc_insert_workspace(int64_t n_rows, int64_t n_cols, int64_t cap_a,
                                    int64_t nnz_t, size_t* ws_bytes) {
  if (!ws_bytes || cap_a < 0 || nnz_t < 0) return SPM_EINVAL;
  spm_status st = check_dims(n_rows, n_cols, cap_a);
  if (st != SPM_OK) return st;
  if (!fits_i32(nnz_t) || !fits_i32(cap_a + nnz_t)) return SPM_EOVERFLOW;
  *ws_bytes = insert_layout(n_cols, cap_a, nnz_t).total;
  return SPM_OK;
}

spm_status spm_csc_insert(int64_t n_rows, int64_t n_cols, int64_t cap_a,
                          const int32_t* a_col_ptr, const int32_t* a_row_idx, const void* a_val,
                          int64_t nnz_t, const int32_t* row, const int32_t* col,
                          const void* val, spm_dtype val_type, int32_t* col_ptr,
                          int32_t* row_idx, void* val_out, spm_dtype out_type, int32_t* info,
                          void* ws, size_t ws_bytes, void* stream) {
  SPM_RANGE("spm_csc_insert");
  if (cap_a < 0 || nnz_t < 0) return SPM_EINVAL;
  spm_status st = check_dims(n_rows, n_cols, cap_a);
  if (st != SPM_OK) return st;
  if (!fits_i32(nnz_t) || !fits_i32(cap_a + nnz_t)) return SPM_EOVERFLOW;
  if (val_type != SPM_F64 && val_type != SPM_F32) return SPM_EDTYPE;
  if (out_type != SPM_F64 && out_type != SPM_F32) return SPM_EDTYPE;
  if (!a_col_ptr || !col_ptr || !info || !ws) return SPM_EINVAL;
  if (cap_a > 0 && (!a_row_idx || !a_val)) return SPM_EINVAL;
  if (nnz_t > 0 && (!row || !col || !val)) return SPM_EINVAL;
  if (cap_a + nnz_t > 0 && (!row_idx || !val_out)) return SPM_EINVAL;
  if (!aligned(ws, 256)) return SPM_EINVAL;
  const InsertLayout L = insert_layout(n_cols, cap_a, nnz_t);
  if (!L.pp.ok) return SPM_EINVAL;  // no columns, or more than the partition covers
  if (ws_bytes < L.total) return SPM_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  const int out_f64 = out_type == SPM_F64 ? 1 : 0;
  if (val_type == SPM_F64)
    insert_t<double>(n_rows, n_cols, cap_a, a_col_ptr, a_row_idx,
                     static_cast<const double*>(a_val), nnz_t, row, col,
                     static_cast<const double*>(val), col_ptr, row_idx, val_out, out_f64, info,
                     static_cast<char*>(ws), L, s);
  else
    insert_t<float>(n_rows, n_cols, cap_a, a_col_ptr, a_row_idx,
                    static_cast<const float*>(a_val), nnz_t, row, col,
                    static_cast<const float*>(val), col_ptr, row_idx, val_out, out_f64, info,
                    static_cast<char*>(ws), L, s);
  return launch_status();
}

}  // extern "C"


extern "C" {

spm_status spm_csc_add_workspace(int64_t n_rows, int64_t n_cols, int64_t a_cap, int64_t b_cap,
                                 size_t* ws_bytes) {
  if (!ws_bytes || a_cap < 0 || b_cap < 0) return SPM_EINVAL;
  spm_status st = check_dims(n_rows, n_cols, a_cap);
  if (st != SPM_OK) return st;
  if (!fits_i32(b_cap) || !fits_i32(a_cap + b_cap)) return SPM_EOVERFLOW;
  Carve c;
  MpLayout M;
  mp_carve(c, a_cap + b_cap, M);
  *ws_bytes = c.off;
  return SPM_OK;
}

spm_status spm_csc_add(int64_t n_rows, int64_t n_cols, int64_t a_cap, const int32_t* a_col_ptr,
                       const int32_t* a_row_idx, const void* a_val, int64_t b_cap,
                       const int32_t* b_col_ptr, const int32_t* b_row_idx, const void* b_val,
                       spm_dtype val_type, int32_t* col_ptr, int32_t* row_idx, void* val_out,
                       spm_dtype out_type, int32_t* info, void* ws, size_t ws_bytes,
                       void* stream) {
  SPM_RANGE("spm_csc_add");
  if (a_cap < 0 || b_cap < 0) return SPM_EINVAL;
  spm_status st = check_dims(n_rows, n_cols, a_cap);
  if (st != SPM_OK) return st;
  if (!fits_i32(b_cap) || !fits_i32(a_cap + b_cap)) return SPM_EOVERFLOW;
  if (val_type != SPM_F64 && val_type != SPM_F32) return SPM_EDTYPE;
  if (out_type != SPM_F64 && out_type != SPM_F32) return SPM_EDTYPE;
  if (!a_col_ptr || !b_col_ptr || !col_ptr || !info || !ws) return SPM_EINVAL;
  if (a_cap > 0 && (!a_row_idx || !a_val)) return SPM_EINVAL;
  if (b_cap > 0 && (!b_row_idx || !b_val)) return SPM_EINVAL;
  if (a_cap + b_cap > 0 && (!row_idx || !val_out)) return SPM_EINVAL;
  if (!aligned(ws, 256)) return SPM_EINVAL;
  if (n_cols == 0) return SPM_EINVAL;  // as for the insertion
  Carve c;
  MpLayout M;
  mp_carve(c, a_cap + b_cap, M);
  if (ws_bytes < c.off) return SPM_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int out_f64 = out_type == SPM_F64 ? 1 : 0;
  char* w = static_cast<char*>(ws);
  (void)hipGetLastError();
  const MergeLists ML{a_col_ptr, a_row_idx, a_cap, b_col_ptr, b_row_idx, b_cap,
                      n_rows,    n_cols,    true};
  if (val_type == SPM_F64)
    mp_run<double, double>(ML, static_cast<const double*>(a_val),
                           static_cast<const double*>(b_val), col_ptr, row_idx, val_out,
                           out_f64, a_cap + b_cap, info, info, w, M, s);
  else
    mp_run<float, float>(ML, static_cast<const float*>(a_val), static_cast<const float*>(b_val),
                         col_ptr, row_idx, val_out, out_f64, a_cap + b_cap, info, info, w, M,
                         s);
  return launch_status();
}

spm_status spm_csc_spmm(int64_t n_rows, int64_t n_cols, int64_t nnz_cap, int64_t k,
                        const void* plan, const void* val, spm_dtype val_type,
                        spm_val_order val_order, const void* X, int64_t ldx, spm_dtype x_type,
                        void* Y, int64_t ldy, spm_dtype y_type, void* stream) {
  SPM_RANGE("spm_csc_spmm");
  spm_status st = check_dims(n_rows, n_cols, nnz_cap);
  if (st != SPM_OK) return st;
  if (k < 1 || ldx < k || ldy < k) return SPM_EINVAL;
  if (!fits_i32(k) || (n_cols > 0 && ldx > INT64_MAX / n_cols) ||
      (n_rows > 0 && ldy > INT64_MAX / n_rows))
    return SPM_EOVERFLOW;
  if (val_type != SPM_F64 && val_type != SPM_F32) return SPM_EDTYPE;
  if (val_order != SPM_ORDER_CSC && val_order != SPM_ORDER_PLAN) return SPM_EINVAL;
  if (x_type != SPM_F64 && x_type != SPM_F32 && x_type != SPM_BF16) return SPM_EDTYPE;
  if (y_type != SPM_F64 && y_type != SPM_F32) return SPM_EDTYPE;
  if (!plan || !Y || (nnz_cap > 0 && !val) || (n_cols > 0 && !X)) return SPM_EINVAL;
  if (!aligned(plan, 256)) return SPM_EINVAL;
  if (n_rows == 0) return SPM_OK;
  const PlanParts P = plan_parts(n_rows, nnz_cap);
  const char* pl = static_cast<const char*>(plan);
  const int32_t* row_ptr = reinterpret_cast<const int32_t*>(pl + P.row_ptr);
  const int32_t* col_t = reinterpret_cast<const int32_t*>(pl + P.col_t);
  const int32_t* perm = reinterpret_cast<const int32_t*>(pl + P.perm);
  const int G = group_width(k);
  const spm_tuning tu = tuning();
  const int block = tu.spmm_block;
  const int grid = spmm_grid(n_rows, G, block);
  const int xal = (aligned(X, 4 * dsize(x_type)) && (ldx % 4) == 0) ? 1 : 0;
  const int yal = (aligned(Y, 4 * dsize(y_type)) && (ldy % 4) == 0) ? 1 : 0;
  const int y_f64 = y_type == SPM_F64;
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  const bool f32acc = acc_is_f32(val_type, x_type);
  // The full path loads a clamped (valid) dense row for out-of-range plan entries, so it
  // needs at least one dense row.
  const bool full = k == 4 * (int64_t)G && xal && yal && n_cols > 0;
#define SPM_FWD(VT, XT, ACC)                                                                  \
  launch_fwd_t<VT, XT, ACC>(n_rows, n_cols, nnz_cap, k, G, full, val_order == SPM_ORDER_PLAN,  \
                            row_ptr, col_t, perm, val, X, ldx, xal, Y, ldy, y_f64, yal, grid, \
                            block, s)
  if (val_type == SPM_F64) {
    if (x_type == SPM_F64) SPM_FWD(double, double, double);
    else if (x_type == SPM_F32) SPM_FWD(double, float, double);
    else SPM_FWD(double, bf16_t, double);
  } else {
    if (x_type == SPM_F64) SPM_FWD(float, double, double);
    else if (x_type == SPM_F32) SPM_FWD(float, float, double);
    else if (f32acc) SPM_FWD(float, bf16_t, float);
    else SPM_FWD(float, bf16_t, double);
  }
#undef SPM_FWD
  return launch_status();
}

spm_status spm_csc_spmm_backward(int64_t n_rows, int64_t n_cols, int64_t nnz_cap, int64_t k,
                                 const int32_t* col_ptr, const int32_t* row_idx, const void* val,
                                 spm_dtype val_type, const void* Gm, int64_t ldg,
                                 spm_dtype g_type, const void* X, int64_t ldx, spm_dtype x_type,
                                 void* dX, int64_t lddx, spm_dtype dx_type, void* dval,
                                 spm_dtype dval_type, void* stream) {
  SPM_RANGE("spm_csc_spmm_backward");
  spm_status st = check_dims(n_rows, n_cols, nnz_cap);
  if (st != SPM_OK) return st;
  if (k < 1 || ldg < k || ldx < k || (dX && lddx < k)) return SPM_EINVAL;
  if (!fits_i32(k)) return SPM_EOVERFLOW;
  if (val_type != SPM_F64 && val_type != SPM_F32) return SPM_EDTYPE;
  if (g_type != SPM_F64 && g_type != SPM_F32 && g_type != SPM_BF16) return SPM_EDTYPE;
  if (x_type != SPM_F64 && x_type != SPM_F32 && x_type != SPM_BF16) return SPM_EDTYPE;
  if (dX && dx_type != SPM_F64 && dx_type != SPM_F32) return SPM_EDTYPE;
  if (dval && dval_type != SPM_F64 && dval_type != SPM_F32) return SPM_EDTYPE;
  if (!col_ptr || (nnz_cap > 0 && (!row_idx || !val)) || (n_rows > 0 && !Gm) ||
      (n_cols > 0 && !X))
    return SPM_EINVAL;
  if (!dX && !dval) return SPM_OK;
  if (n_cols == 0) return SPM_OK;
  const int G = group_width(k);
  const spm_tuning tu = tuning();
  const int block = tu.spmm_block;
  const int grid = spmm_grid(n_cols, G, block);
  const int gal = (aligned(Gm, 4 * dsize(g_type)) && (ldg % 4) == 0) ? 1 : 0;
  const int xal = (aligned(X, 4 * dsize(x_type)) && (ldx % 4) == 0) ? 1 : 0;
  const int dxal = dX ? ((aligned(dX, 4 * dsize(dx_type)) && (lddx % 4) == 0) ? 1 : 0) : 0;
  const int dx_f64 = dx_type == SPM_F64;
  const int dv_f64 = dval_type == SPM_F64;
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  const bool full = k == 4 * (int64_t)G && gal && xal && (!dX || dxal) && n_rows > 0;
#define SPM_BWD(VT, GT, XT)                                                                   \
  launch_bwd_t<VT, GT, XT, typename AccOf<VT, GT, XT>::type>(                                 \
      n_rows, n_cols, nnz_cap, k, G, full, col_ptr, row_idx, val, Gm, ldg, gal, X, ldx, xal,  \
      dX, lddx, dx_f64, dxal, dval, dv_f64, grid, block, s)
#define SPM_BWD_X(VT, GT)                                         \
  do {                                                            \
    if (x_type == SPM_F64) SPM_BWD(VT, GT, double);               \
    else if (x_type == SPM_F32) SPM_BWD(VT, GT, float);           \
    else SPM_BWD(VT, GT, bf16_t);                                 \
  } while (0)
  // G's element type is dispatched on its own, never converted to X's.
  if (val_type == SPM_F64) {
    if (g_type == SPM_F64) SPM_BWD_X(double, double);
    else if (g_type == SPM_F32) SPM_BWD_X(double, float);
    else SPM_BWD_X(double, bf16_t);
  } else {
    if (g_type == SPM_F64) SPM_BWD_X(float, double);
    else if (g_type == SPM_F32) SPM_BWD_X(float, float);
    else SPM_BWD_X(float, bf16_t);
  }
#undef SPM_BWD_X
#undef SPM_BWD
  return launch_status();
}

spm_status spm_tuning_get(spm_tuning* out) {
  if (!out) return SPM_EINVAL;
  *out = tuning();
  return SPM_OK;
}

static spm_status tuning_valid(const spm_tuning* in) {
  if (!in) return SPM_EINVAL;
  auto pow2 = [](int32_t x) { return x > 0 && (x & (x - 1)) == 0; };
  if (in->spmm_block != 64 && in->spmm_block != 128 && in->spmm_block != 256) return SPM_EINVAL;
  if (in->spmm_blocks_per_cu < 1 || in->spmm_blocks_per_cu > 64) return SPM_EINVAL;
  if (in->batch_wg_per_cu < 1 || in->batch_wg_per_cu > 8) return SPM_EINVAL;
  if (in->batch_spmm_wg_per_cu < 0 || in->batch_spmm_wg_per_cu > 32) return SPM_EINVAL;
  if (in->trace_group_width != 0 && in->trace_group_width != 16 &&
      in->trace_group_width != 32 && in->trace_group_width != 64)
    return SPM_EINVAL;
  if (!pow2(in->part_bucket_target) || in->part_bucket_target < 256 ||
      in->part_bucket_target > 2048)
    return SPM_EINVAL;
  if (!pow2(in->part_max_tiles) || in->part_max_tiles < 64 || in->part_max_tiles > 4096)
    return SPM_EINVAL;
  return SPM_OK;
}

spm_status spm_tuning_set(const spm_tuning* in) {
  const spm_status st = tuning_valid(in);
  if (st != SPM_OK) return st;
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  g_tuning = *in;
  return SPM_OK;
}

spm_status spm_tuning_register(const char* key, const spm_tuning* in) {
  if (!key || !*key) return SPM_EINVAL;
  const spm_status st = tuning_valid(in);
  if (st != SPM_OK) return st;
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  g_tuning_named[key] = *in;
  return SPM_OK;
}

spm_status spm_tuning_select(const char* key) {
  if (!key) {
    t_tuning_on = false;
    return SPM_OK;
  }
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  const auto it = g_tuning_named.find(key);
  if (it == g_tuning_named.end()) return SPM_EINVAL;
  t_tuning = it->second;
  t_tuning_on = true;
  return SPM_OK;
}

spm_status spm_csc_plan_bytes(int64_t n_rows, int64_t n_cols, int64_t nnz_cap,
                              size_t* plan_bytes) {
  if (!plan_bytes) return SPM_EINVAL;
  size_t ws = 0;
  return spm_csc_plan_size(n_rows, n_cols, nnz_cap, plan_bytes, &ws);
}

}  // extern "C"

// ============================================================================================
// Batched path
// ============================================================================================
namespace {

size_t batch_stride(int64_t max_dim, int64_t max_nnz) {
  return align256(sizeof(uint64_t) * 2 * (size_t)max_nnz +
                  sizeof(uint32_t) * (size_t)(max_dim + 1));
}

int batch_workers(int32_t workers, int32_t batch) {
  const spm_tuning tu = tuning();
  int w = workers > 0 ? workers : cu_count() * tu.batch_wg_per_cu;
  if (batch > 0 && w > batch) w = batch;
  return w < 1 ? 1 : w;
}

// Threads of a grouping workgroup (its LDS, not its thread count, bounds the workgroups per
// CU, so more threads per workgroup mean more waves in flight).
constexpr int kBatchNT = 512;

// Persistent workgroups of the products launch: it holds no LDS and few registers, so
// several times the grouping launch's workgroups fit a CU.
constexpr int kBatchSpmmDefaultWgPerCu = 8;

int batch_spmm_workers(int32_t batch) {
  const spm_tuning tu = tuning();
  const int per_cu = tu.batch_spmm_wg_per_cu > 0 ? tu.batch_spmm_wg_per_cu
                                                 : kBatchSpmmDefaultWgPerCu;
  int w = cu_count() * per_cu;
  if (batch > 0 && w > batch) w = batch;
  return w < 1 ? 1 : w;
}

template <int NT, typename XT, typename ACC>
void launch_batch_spmm(const BatchArgs& a, int workers, hipStream_t s) {
  // the full path for k = 32, 64, 128 with aligned rows, as in the single-matrix launches
  const bool full = a.k == 4 * (int64_t)a.G && a.xal && a.yal;
#define SPM_CALL_F(GW, F) k_batch_spmm<NT, XT, ACC, GW, F><<<dim3(workers), dim3(NT), 0, s>>>(a)
#define SPM_CALL(GW) SPM_CALL_F(GW, false)
  if (full && a.G == 8) SPM_CALL_F(8, true);
  else if (full && a.G == 16) SPM_CALL_F(16, true);
  else if (full && a.G == 32) SPM_CALL_F(32, true);
  else SPM_GW_SWITCH(a.G, SPM_CALL)
#undef SPM_CALL
#undef SPM_CALL_F
}

// Flat products: the forward over all rows, then the adjoint over all columns.
template <int NT, typename XT, typename ACC>
void launch_batch_flat(const BatchArgs& a, const int64_t* rpre, const int64_t* cpre,
                       const int32_t* rtab, const int32_t* ctab, uint32_t* xcd_next,
                       const BatchSlot* rslot, const BatchSlot* cslot, int grid, hipStream_t s) {
  const bool full = a.k == 4 * (int64_t)a.G && a.xal && a.yal;
#define SPM_CALL_F(GW, F)                                                                      \
  do {                                                                                         \
    k_batch_flat<NT, XT, ACC, GW, F, true><<<dim3(grid), dim3(NT), 0, s>>>(a, rpre, rtab,      \
                                                                           xcd_next, rslot);   \
    k_batch_flat<NT, XT, ACC, GW, F, false><<<dim3(grid), dim3(NT), 0, s>>>(                   \
        a, cpre, ctab, xcd_next + kXcds, cslot);                                               \
  } while (0)
#define SPM_CALL(GW) SPM_CALL_F(GW, false)
  if (full && a.G == 8) SPM_CALL_F(8, true);
  else if (full && a.G == 16) SPM_CALL_F(16, true);
  else if (full && a.G == 32) SPM_CALL_F(32, true);
  else SPM_GW_SWITCH(a.G, SPM_CALL)
#undef SPM_CALL
#undef SPM_CALL_F
}

// Grouping launch, then the products: flat when the (now free) worker slices can hold the
// row and column prefixes, else one persistent workgroup per matrix.
template <int NT>
void launch_batch_nt(const BatchArgs& a, spm_dtype vt, spm_dtype xt, int workers,
                     int spmm_workers, size_t slices_bytes, hipStream_t s) {
  if (vt == SPM_F32) k_batch<kBatchNT, float><<<dim3(workers), dim3(kBatchNT), 0, s>>>(a);
  else k_batch<kBatchNT, bf16_t><<<dim3(workers), dim3(kBatchNT), 0, s>>>(a);
  // the flat products need the two prefixes and a chunk table per prefix (one entry per
  // chunk of NT / G rows or columns; at most batch * max_dim of those) in the freed slices
  const int64_t chunk = (int64_t)kBatchFlatPerGroup * (NT / (a.G > 0 ? a.G : 1));
  const int64_t tab_cap = ((int64_t)a.batch * a.max_dim + chunk - 1) / chunk + 1;
  const size_t pre_bytes = 2 * sizeof(int64_t) * ((size_t)a.batch + 1);
  const size_t tab_bytes = sizeof(int32_t) * (size_t)tab_cap;
  const size_t ctr_bytes = sizeof(uint32_t) * 2 * kXcds;
  const size_t slot_bytes = sizeof(BatchSlot) * (size_t)a.batch;
  const size_t need = pre_bytes + 2 * tab_bytes + ctr_bytes + 64 + 2 * slot_bytes;
  if (a.batch > 0 && slices_bytes >= need) {
    int64_t* rpre = reinterpret_cast<int64_t*>(a.ws);
    int64_t* cpre = rpre + a.batch + 1;
    int32_t* rtab = reinterpret_cast<int32_t*>(cpre + a.batch + 1);
    int32_t* ctab = rtab + tab_cap;
    uint32_t* xcd_next = reinterpret_cast<uint32_t*>(ctab + tab_cap);
    const size_t slot_at = (pre_bytes + 2 * tab_bytes + ctr_bytes + 63) & ~(size_t)63;
    BatchSlot* rslot = reinterpret_cast<BatchSlot*>(a.ws + slot_at);
    BatchSlot* cslot = rslot + a.batch;
    k_batch_prefix<NT><<<dim3(1), dim3(NT), 0, s>>>(a, rpre, cpre);
    const int64_t tab_blocks = ceil_div(std::max<int64_t>((int64_t)a.batch, 2 * kXcds), (int64_t)NT);
    k_batch_tab<NT><<<dim3((unsigned)tab_blocks), dim3(NT), 0, s>>>(a, rpre, cpre, chunk, tab_cap,
                                                                    rtab, ctab, xcd_next, rslot,
                                                                    cslot);
    const int grid = cu_count() * (tuning().batch_spmm_wg_per_cu > 0
                                       ? tuning().batch_spmm_wg_per_cu
                                       : kBatchSpmmDefaultWgPerCu);
    // values are assembled into binary32; bfloat16 dense operands accumulate in binary32
    if (xt == SPM_F32)
      launch_batch_flat<NT, float, double>(a, rpre, cpre, rtab, ctab, xcd_next, rslot, cslot,
                                           grid, s);
    else
      launch_batch_flat<NT, bf16_t, float>(a, rpre, cpre, rtab, ctab, xcd_next, rslot, cslot,
                                           grid, s);
    return;
  }
  if (xt == SPM_F32) launch_batch_spmm<NT, float, double>(a, spmm_workers, s);
  else launch_batch_spmm<NT, bf16_t, float>(a, spmm_workers, s);
}

}  // namespace

extern "C" {

spm_status spm_batch_workspace(int64_t max_dim, int64_t max_nnz_in, int32_t workers,
                               size_t* ws_bytes) {
  if (!ws_bytes || max_dim < 0 || max_nnz_in < 0 || workers < 0) return SPM_EINVAL;
  if (!fits_i32(max_dim) || !fits_i32(max_nnz_in) || max_dim == INT32_MAX) return SPM_EOVERFLOW;
  const int w = batch_workers(workers, 0);
  *ws_bytes = 256 + (size_t)w * batch_stride(max_dim, max_nnz_in);
  return SPM_OK;
}

spm_status spm_batch_schedule(const spm_batch_item* items, int32_t batch, int64_t k,
                              int32_t* order) {
  if (batch < 0 || (batch > 0 && (!items || !order)) || k < 1) return SPM_EINVAL;
  std::vector<int32_t> idx(batch);
  std::vector<double> cost(batch);
  for (int32_t b = 0; b < batch; ++b) {
    idx[b] = b;
    // assembly + plan work grows with the triplets, the products with nnz * k and (n_r+n_c)*k
    const double nnz = items[b].nnz_in > 0 ? items[b].nnz_in : 0;
    const double dim = (double)(items[b].n_rows > 0 ? items[b].n_rows : 0) +
                       (double)(items[b].n_cols > 0 ? items[b].n_cols : 0);
    cost[b] = nnz * (8.0 + 0.5 * (double)k) + dim * (double)k;
  }
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
  std::memcpy(order, idx.data(), sizeof(int32_t) * (size_t)batch);
  return SPM_OK;
}

spm_status spm_batch_run(int32_t batch, int64_t k, const spm_batch_item* items,
                         const int32_t* order, const int32_t* row, const int32_t* col,
                         const void* val, spm_dtype val_type, const void* X, const void* Gm,
                         spm_dtype x_type, int32_t* col_ptr, int32_t* row_idx, float* val_out,
                         int32_t* row_ptr, int32_t* col_t, int32_t* perm, float* Y, float* dX,
                         float* dval, int32_t* info, int64_t max_dim, int64_t max_nnz_in,
                         int32_t workers, void* ws, size_t ws_bytes, void* stream) {
  SPM_RANGE("spm_batch_run");
  if (batch < 0 || k < 1 || max_dim < 0 || max_nnz_in < 0 || workers < 0) return SPM_EINVAL;
  if (!fits_i32(k) || !fits_i32(max_dim) || !fits_i32(max_nnz_in) || max_dim == INT32_MAX)
    return SPM_EOVERFLOW;
  if (val_type != SPM_F32 && val_type != SPM_BF16) return SPM_EDTYPE;
  if (x_type != SPM_F32 && x_type != SPM_BF16) return SPM_EDTYPE;
  if (batch == 0) return SPM_OK;
  if (!items || !order || !row || !col || !val || !X || !Gm || !col_ptr || !row_idx ||
      !val_out || !row_ptr || !col_t || !perm || !Y || !dX || !dval || !info || !ws)
    return SPM_EINVAL;
  if (!aligned(ws, 256)) return SPM_EINVAL;
  const int w = batch_workers(workers, batch);
  const size_t stride = batch_stride(max_dim, max_nnz_in);
  if (ws_bytes < 256 + (size_t)w * stride) return SPM_EWORKSPACE;
  const spm_tuning tu = tuning();
  BatchArgs a;
  a.items = items;
  a.order = order;
  a.batch = batch;
  a.k = k;
  a.G = group_width(k);
  a.row = row;
  a.col = col;
  a.val = val;
  a.X = X;
  a.Gm = Gm;
  a.col_ptr = col_ptr;
  a.row_idx = row_idx;
  a.val_out = val_out;
  a.row_ptr = row_ptr;
  a.col_t = col_t;
  a.perm = perm;
  a.Y = Y;
  a.dX = dX;
  a.dval = dval;
  a.info = info;
  a.max_dim = max_dim;
  a.max_nnz = max_nnz_in;
  a.ws = static_cast<char*>(ws) + 256;
  a.ws_stride = stride;
  a.queue = static_cast<uint32_t*>(ws);
  a.xal = (k % 4 == 0 && aligned(X, 4 * dsize(x_type)) && aligned(Gm, 4 * dsize(x_type))) ? 1 : 0;
  a.yal = (k % 4 == 0 && aligned(Y, 16) && aligned(dX, 16)) ? 1 : 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  k_zero2<<<dim3(1), dim3(64), 0, s>>>(
      a.queue, (int64_t)2, (uint32_t*)nullptr, (int64_t)0);
  launch_batch_nt<256>(a, val_type, x_type, w, batch_spmm_workers(batch), (size_t)w * stride,
                       s);
  return launch_status();
}

spm_status spm_batch_coo_to_csc_spmm(int32_t batch, int64_t k, const spm_batch_item* items,
                                     const int32_t* order, const int32_t* row,
                                     const int32_t* col, const void* val, spm_dtype val_type,
                                     const void* X, const void* Gm, spm_dtype x_type,
                                     int32_t* col_ptr, int32_t* row_idx, float* val_out,
                                     int32_t* row_ptr, int32_t* col_t, int32_t* perm, float* Y,
                                     float* dX, float* dval, int32_t* info, int64_t max_dim,
                                     int64_t max_nnz_in, int32_t workers, void* ws,
                                     size_t ws_bytes, const char* tune_key, void* stream) {
  SPM_RANGE("spm_batch_coo_to_csc_spmm");
  // the named tuning for this call only: the thread's own selection is restored afterwards
  const bool had = t_tuning_on;
  const spm_tuning saved = t_tuning;
  if (tune_key) {
    const spm_status st = spm_tuning_select(tune_key);
    if (st != SPM_OK) return st;
  }
  const spm_status st = spm_batch_run(batch, k, items, order, row, col, val, val_type, X, Gm,
                                      x_type, col_ptr, row_idx, val_out, row_ptr, col_t, perm,
                                      Y, dX, dval, info, max_dim, max_nnz_in, workers, ws,
                                      ws_bytes, stream);
  t_tuning_on = had;
  t_tuning = saved;
  return st;
}

}  // extern "C"

// ============================================================================================
// Assembly and plan without allocation: the workspace is a fixed device array of the library.
// ============================================================================================
namespace {

constexpr size_t kNoallocScratchBytes = SPM_NOALLOC_SCRATCH_BYTES;

// The scratch array.  In host code its name is only a stand-in for the symbol: the device
// address comes from hipGetSymbolAddress, once per device (each GPU holds its own copy).
static __device__ __align__(256) unsigned char spm_noalloc_scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up on first use.
spm_status noalloc_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SPM_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(spm_noalloc_scratch)) != hipSuccess || !p)
      return SPM_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SPM_OK;
}

}  // namespace

extern "C" {

spm_status spm_coo_to_csc_plan_noalloc(int64_t n_rows, int64_t n_cols, int64_t nnz_in,
                                       const int32_t* row, const int32_t* col, const void* val,
                                       spm_dtype val_type, int32_t* col_ptr, int32_t* row_idx,
                                       void* val_out, spm_dtype out_type, int32_t* info,
                                       void* plan, size_t plan_bytes, void* val_plan,
                                       int32_t* plan_info, void* stream) {
  SPM_RANGE("spm_coo_to_csc_plan_noalloc");
  spm_status st = check_dims(n_rows, n_cols, nnz_in);
  if (st != SPM_OK) return st;
  if (fuse_layout(n_rows, n_cols, nnz_in).total > kNoallocScratchBytes) return SPM_EWORKSPACE;
  void* ws = nullptr;
  st = noalloc_scratch(&ws);
  if (st != SPM_OK) return st;
  return spm_coo_to_csc_plan(n_rows, n_cols, nnz_in, row, col, val, val_type, col_ptr, row_idx,
                             val_out, out_type, info, plan, plan_bytes, val_plan, plan_info, ws,
                             kNoallocScratchBytes, stream);
}

}  // extern "C"
