// Merge of two column-sorted element lists into one CSC, by merge path over the whole matrix.
// A is a CSC (rows strictly increasing down each column); B lists elements by column, rows
// non-decreasing, equal rows in the order their values are to be added (for batch insertion:
// the new triplets sorted by (column, row, input position); for the sum A + B: B's CSC).
// The merged sequence takes, within a column, A's element before B's on equal rows.  A run is
// the merged elements of one (column, row): at most one of A, then B's in order; it folds
// left to right in binary64 (Section 3.1's sort-then-merge insertion with Fig. 1's +=, the
// existing value first), and a fold that compares equal to 0.0 is not stored.
//
// Work is cut by position in the merged sequence, not by column, so a long column is shared
// by many workgroups.  Position d lies in the column c with mcp(c) <= d < mcp(c + 1),
// mcp(c) = acp(c) + bcp(c) (the columns' merged starts); inside the column a binary search on
// the diagonal (merge path) gives how many of the first d - mcp(c) merged elements are A's.
// k_merge_cols (one thread per column) records for every workgroup tile the column of its
// first position, and clears the per-call state.  k_merge, one workgroup per tile of
// NT * kMergeE positions: the merge-path splits at the tile's two ends (one wave each) give
// its slices of A and B; every element gets the key (column, row), its column from a max-scan
// over the column starts inside the slices; a merge-path split per thread over the keys and
// a serial merge of kMergeE steps give the tile's merged order; runs fold from their first
// position (a run continues into later threads' positions, and past the tile into B's next
// elements); the kept results take their offsets from a workgroup scan and a decoupled
// look-back over the tiles before, and go out in position order with the offsets of the
// columns that start in the tile.  The last tile also writes nnz, the status and the offsets
// of the columns that start at the very end (the status flags travel in the look-back words).
// The offsets of both lists are checked on the way (start at 0, non-decreasing, end within
// capacity; else SPM_EINVAL).  Every read goes through clamped offsets and bounded indices,
// and every store is checked against the output capacity, so malformed offsets give a wrong
// result, never an access out of range.
#pragma once

#include "spm_device.h"

namespace spm {

constexpr int kMergeE = 8;  // merged positions per thread

constexpr uint32_t kMpShape = 1u;   // offsets not starting at 0, decreasing or beyond capacity
constexpr uint32_t kMpOrder = 2u;   // rows of A not increasing down a column (or of B, for A + B)
constexpr uint32_t kMpBounds = 4u;  // a stored row of A (or B) outside the matrix

struct MergeLists {
  const int32_t* a_cp;
  const int32_t* a_ri;
  int64_t a_cap;
  const int32_t* b_cp;
  const int32_t* b_ri;
  int64_t b_cap;
  int64_t n_rows, n_cols;
  bool b_strict;  // B's rows must increase strictly down a column (a CSC)
};

// Offsets of one list clamped into [0, nnz] (only well-formed offsets reach the walk).
struct MergeView {
  const int32_t* cp;
  int64_t nnz;
  __device__ __forceinline__ int64_t at(int64_t c) const {
    const int64_t v = cp[c];
    return v < 0 ? 0 : (v > nnz ? nnz : v);
  }
};

__device__ __forceinline__ int64_t clamp_cap(int64_t v, int64_t cap) {
  return v < 0 ? 0 : (v > cap ? cap : v);
}

// Offsets of both lists well formed (grid-stride over the columns); flags what is not.
template <int NT>
__device__ __forceinline__ uint32_t merge_check(const MergeLists& L) {
  uint32_t f = 0;
  const int64_t stride = (int64_t)gridDim.x * NT;
  for (int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x; c <= L.n_cols; c += stride) {
    if (c == 0) {
      if (L.a_cp[0] != 0 || L.b_cp[0] != 0) f |= kMpShape;
      if (L.a_cp[L.n_cols] > L.a_cap || L.b_cp[L.n_cols] > L.b_cap) f |= kMpShape;
    }
    if (c < L.n_cols && (L.a_cp[c] > L.a_cp[c + 1] || L.b_cp[c] > L.b_cp[c + 1])) f |= kMpShape;
  }
  return f;
}

// Column starts of the tiles, and the per-call state.  One thread per column c: the first
// column to start at mcp(c) (mcp(c - 1) < mcp(c), or c = 0) is the first column whose merged
// start is at or after every position x in (mcp(c - 1), mcp(c)], so it records itself as
// tile_col[t] for every tile start x = t SEG in that interval below M, and as tile_col[ntiles]
// (the column of position M) when M lies there.  The same launch clears the look-back states,
// the ticket and, for a call with nothing reported before, info[1].
template <int NT>
__global__ __launch_bounds__(NT) void k_merge_cols(MergeLists L, int64_t seg, int64_t ntiles,
                                                   int32_t* __restrict__ tile_col,
                                                   uint64_t* __restrict__ state,
                                                   uint32_t* __restrict__ ticket,
                                                   int32_t* __restrict__ info_clear) {
  const MergeView A{L.a_cp, clamp_cap(L.a_cp[L.n_cols], L.a_cap)};
  const MergeView B{L.b_cp, clamp_cap(L.b_cp[L.n_cols], L.b_cap)};
  const int64_t M = A.nnz + B.nnz;
  const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * NT;
  for (int64_t q = g; q < ntiles; q += stride) state[q] = 0;
  if (g == 0) {
    *ticket = 0;
    if (info_clear) info_clear[1] = 0;
  }
  for (int64_t c = g; c <= L.n_cols; c += stride) {
    const int64_t mc = A.at(c) + B.at(c);
    const int64_t mp = c > 0 ? A.at(c - 1) + B.at(c - 1) : -1;
    if (mp >= mc) continue;  // not the first column to start at mc
    if (mp < M && M <= mc) tile_col[ntiles] = (int32_t)c;
    const int64_t top = mc < M ? mc : M - 1;  // tile starts in (mp, top]
    for (int64_t t = mp < 0 ? 0 : mp / seg + 1; t < ntiles && t * seg <= top; ++t)
      tile_col[t] = (int32_t)c;
  }
}

// Merge-path split at merged position d, found by one wave: d lies at the start of column cl
// (the first column whose merged start is at or after d) or inside column cl - 1.  Each round
// the 64 lanes probe 64 evenly spaced candidates of the interval that is left.
__device__ __forceinline__ void wave_split(const MergeLists& L, const MergeView& A,
                                           const MergeView& B, int64_t cl, int64_t d,
                                           int64_t& i, int64_t& j) {
  if (cl <= L.n_cols && A.at(cl) + B.at(cl) <= d) {  // d at the start of column cl
    i = A.at(cl);
    j = B.at(cl);
    return;
  }
  const int64_t c = cl > 0 ? cl - 1 : 0;
  if (c >= L.n_cols) {  // (malformed offsets only)
    i = A.nnz;
    j = B.nnz;
    return;
  }
  const int64_t a0 = A.at(c), a1 = max(a0, A.at(c + 1));
  const int64_t b0 = B.at(c), b1 = max(b0, B.at(c + 1));
  const int64_t na = a1 - a0, nb = b1 - b0;
  int64_t k = d - (a0 + b0);
  k = k < 0 ? 0 : (k > na + nb ? na + nb : k);
  int64_t lo = k - nb > 0 ? k - nb : 0, hi = k < na ? k : na;
  const int lane = lane_id();
  while (lo < hi) {  // first m in [lo, hi] where A's (a0 + m) no longer precedes B's (b0 + k - m - 1)
    const int64_t sp = hi - lo;
    const int64_t m = lo + (sp * lane) / kWave;
    const bool q = L.a_ri[a0 + m] <= L.b_ri[b0 + k - m - 1];
    const int cnt = __popcll(__ballot(q));
    if (cnt == 0) {
      hi = lo;
    } else {
      const int64_t nlo = lo + (sp * (cnt - 1)) / kWave + 1, nhi = lo + (sp * cnt) / kWave;
      lo = nlo;
      if (cnt < kWave) hi = nhi;
    }
  }
  i = a0 + lo;
  j = b0 + k - lo;
}

constexpr int kMergeFlagBits = 3;  // kMp* flags carried in the look-back words
constexpr int kMergeCntBits = 62 - kMergeFlagBits;
constexpr uint64_t kNoKey = ~0ull;

__device__ __forceinline__ uint64_t merge_key(int64_t col, int32_t row) {
  return ((uint64_t)(uint32_t)col << 32) | (uint32_t)row;
}

// Inclusive max-scan of two arrays of NT * 8 int32 (8 consecutive entries per thread), both
// seeded with `init`.  `s_w` needs 2 * NT / 64 words.
template <int NT>
__device__ __forceinline__ void wg_max_scan2(int32_t* a, int32_t* b, int32_t init,
                                             int32_t* s_w) {
  constexpr int NW = NT / kWave;
  int32_t va[8], vb[8];
  int32_t ma = init, mb = init;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    va[k] = a[threadIdx.x * 8 + k];
    vb[k] = b[threadIdx.x * 8 + k];
    ma = max(ma, va[k]);
    mb = max(mb, vb[k]);
  }
  int32_t ia = ma, ib = mb;  // inclusive over the wave
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int32_t ya = __shfl_up(ia, d, kWave), yb = __shfl_up(ib, d, kWave);
    if (lane_id() >= d) {
      ia = max(ia, ya);
      ib = max(ib, yb);
    }
  }
  if (lane_id() == kWave - 1) {
    s_w[wave_id()] = ia;
    s_w[NW + wave_id()] = ib;
  }
  __syncthreads();
  int32_t ea = init, eb = init;  // exclusive: earlier waves and earlier lanes
  for (int w = 0; w < wave_id(); ++w) {
    ea = max(ea, s_w[w]);
    eb = max(eb, s_w[NW + w]);
  }
  const int32_t pa = __shfl_up(ia, 1, kWave), pb = __shfl_up(ib, 1, kWave);
  if (lane_id() > 0) {
    ea = max(ea, pa);
    eb = max(eb, pb);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    ea = max(ea, va[k]);
    eb = max(eb, vb[k]);
    a[threadIdx.x * 8 + k] = ea;
    b[threadIdx.x * 8 + k] = eb;
  }
}

// One workgroup per tile of SEG = NT * 8 merged positions [W0, W1): the splits at both ends
// (one wave each) give the tile's slices A[iA0, iA1) and B[jB0, jB1).  The column of every
// element comes from a max-scan over the column starts that fall in the slices, so each
// element gets the key (column, row); a merge-path split per thread over the keys (A first on
// equal keys) and a serial merge of 8 steps give the tile's merged order.  A position starts
// a run when its key differs from the one before (at the tile start: the element before W0,
// when it lies in the same column); each run folds left to right, the thread of its first
// position continuing into the next threads' positions and, at the tile end, into B's
// elements after jB1.  The kept results get their offsets from a workgroup scan and the
// look-back, and are written in position order; then the offsets of the columns that start
// in the tile.
template <int NT, typename VA, typename VB>
__global__ __launch_bounds__(NT) void k_merge(MergeLists L, const VA* __restrict__ a_v,
                                              const VB* __restrict__ b_v,
                                              const int32_t* __restrict__ tile_col,
                                              int32_t* __restrict__ col_ptr,
                                              int32_t* __restrict__ row_idx,
                                              void* __restrict__ val_out, int out_f64,
                                              int64_t out_cap, uint64_t* __restrict__ state,
                                              uint32_t* __restrict__ ticket, int by_ticket,
                                              int32_t* __restrict__ info, int32_t st_inval,
                                              int32_t st_bounds) {
  constexpr int E = kMergeE;
  static_assert(E == 8, "wg_max_scan2 takes 8 entries per thread");
  constexpr int SEG = NT * E;
  // LDS, reused across phases: R1 keys of A, then merged keys; R2 keys of B, then the run
  // results; R3 / R4 the column scans of A / B, then merged sources / result rows
  __shared__ uint64_t s_r1[SEG], s_r2[SEG];
  __shared__ int32_t s_r3[SEG], s_r4[SEG];
  __shared__ uint32_t s_w[2 * (NT / kWave) + 1];
  __shared__ uint32_t s_toff[NT];
  __shared__ uint8_t s_kmask[NT];
  __shared__ int64_t s_t, s_split[4];
  __shared__ uint64_t s_pre, s_prevkey;
  __shared__ uint32_t s_flags;
  // The look-back waits only on earlier tiles.  When every workgroup of the grid fits on the
  // device at once, each of them gets a slot whatever the dispatch order, so the workgroup
  // index serves; otherwise tiles number themselves in the order they start (a ticket).
  if (threadIdx.x == 0) {
    s_t = by_ticket ? (int64_t)atomicAdd(ticket, 1u) : (int64_t)blockIdx.x;
    s_flags = 0;
  }
  __syncthreads();
  const int64_t t = s_t;
  const int64_t ntiles = gridDim.x;
  const MergeView A{L.a_cp, clamp_cap(L.a_cp[L.n_cols], L.a_cap)};
  const MergeView B{L.b_cp, clamp_cap(L.b_cp[L.n_cols], L.b_cap)};
  const int64_t M = A.nnz + B.nnz;
  const auto clamp_col = [&](int64_t c) -> int64_t {
    return c < 0 ? 0 : (c > L.n_cols + 1 ? L.n_cols + 1 : c);
  };
  const int64_t cM = clamp_col(tile_col[ntiles]);  // first column starting at M
  uint32_t flags = merge_check<NT>(L);
  const int64_t W0 = t * SEG;
  const int64_t W1 = W0 + SEG < M ? W0 + SEG : M;
  int64_t iA0 = 0, jB0 = 0, nA = 0, nB = 0, n = 0, c_first = 0, cl1 = 0;
  // per thread: its E consecutive positions of the merged tile
  uint64_t mk[E];
  int32_t ms[E];  // source: index into A's slice, or ~index into B's
  double mv[E];
  if (W0 < M) {  // the same for the whole workgroup
    // ---- the splits at W0 (wave 0) and W1 (wave 1) ----------------------------------------
    const int64_t cl0 = clamp_col(tile_col[t]);
    cl1 = W1 < M ? clamp_col(tile_col[t + 1]) : cM;
    if (threadIdx.x < 2 * kWave) {
      const bool at1 = threadIdx.x >= kWave;
      int64_t i, j;
      if (at1 && W1 == M) {
        i = A.nnz;
        j = B.nnz;
      } else {
        wave_split(L, A, B, at1 ? cl1 : cl0, at1 ? W1 : W0, i, j);
      }
      if (lane_id() == 0) {
        s_split[at1 ? 2 : 0] = i;
        s_split[at1 ? 3 : 1] = j;
      }
    }
    for (int q = threadIdx.x; q < SEG; q += NT) {
      s_r3[q] = -1;
      s_r4[q] = -1;
    }
    __syncthreads();
    iA0 = s_split[0];
    jB0 = s_split[1];
    nA = s_split[2] - iA0;
    nB = s_split[3] - jB0;
    nA = nA < 0 ? 0 : (nA > SEG ? SEG : nA);  // (malformed offsets only)
    nB = nB < 0 ? 0 : (nB > SEG - nA ? SEG - nA : nB);
    n = nA + nB;
    c_first = (cl0 <= L.n_cols && A.at(cl0) + B.at(cl0) <= W0) ? cl0 : (cl0 > 0 ? cl0 - 1 : 0);
    // ---- rows of the slices (every load issued before the first use) ----------------------
    int32_t ra[E], rb[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int64_t q = r * NT + threadIdx.x;
      ra[r] = q < nA ? L.a_ri[iA0 + q] : 0;
      rb[r] = q < nB ? L.b_ri[jB0 + q] : 0;
    }
    // the element before W0 when it lies in column c_first: the later of A[iA0 - 1], B[jB0 - 1]
    if (threadIdx.x == 0) {
      uint64_t pk = kNoKey;
      if (c_first < L.n_cols) {  // (every load issued at once)
        const int64_t a0 = A.at(c_first), b0 = B.at(c_first);
        const int64_t a1 = A.at(c_first + 1), b1 = B.at(c_first + 1);
        const int32_t pa = iA0 > 0 && iA0 - 1 < A.nnz ? L.a_ri[iA0 - 1] : 0;
        const int32_t pb = jB0 > 0 && jB0 - 1 < B.nnz ? L.b_ri[jB0 - 1] : 0;
        const int32_t fa = nA > 0 ? L.a_ri[iA0] : 0, fb = nB > 0 ? L.b_ri[jB0] : 0;
        const bool ha = iA0 > a0 && iA0 - 1 < A.nnz, hb = jB0 > b0 && jB0 - 1 < B.nnz;
        if (ha || hb) pk = merge_key(c_first, hb && (!ha || pb >= pa) ? pb : pa);
        // the pairs across the tile start
        if (ha && nA > 0 && fa <= pa && a1 > iA0) flags |= kMpOrder;
        if (L.b_strict && hb && nB > 0 && fb <= pb && b1 > jB0) flags |= kMpOrder;
      }
      s_prevkey = pk;
    }
    // ---- the column starts inside the slices, then the column of every element -----------
    for (int64_t c = c_first + 1 + threadIdx.x; c <= cl1 && c <= L.n_cols; c += NT) {
      const int64_t a = A.at(c) - iA0, b = B.at(c) - jB0;
      if (a >= 0 && a < nA) atomicMax(&s_r3[a], (int32_t)c);
      if (b >= 0 && b < nB) atomicMax(&s_r4[b], (int32_t)c);
    }
    __syncthreads();
    wg_max_scan2<NT>(s_r3, s_r4, (int32_t)c_first, reinterpret_cast<int32_t*>(s_w));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int q = r * NT + threadIdx.x;
      if (q < nA) {
        s_r1[q] = merge_key(s_r3[q], ra[r]);
        if (ra[r] < 0 || (int64_t)ra[r] >= L.n_rows) flags |= kMpBounds;
      }
      if (q < nB) {
        s_r2[q] = merge_key(s_r4[q], rb[r]);
        if (rb[r] < 0 || (int64_t)rb[r] >= L.n_rows) flags |= kMpBounds;
      }
    }
    __syncthreads();
    // rows increasing down a column (strictly for A, and for B when it is a CSC)
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int q = r * NT + threadIdx.x;
      if (q + 1 < nA && s_r3[q] == s_r3[q + 1] && ra[r] >= (int32_t)s_r1[q + 1])
        flags |= kMpOrder;
      if (L.b_strict && q + 1 < nB && s_r4[q] == s_r4[q + 1] && rb[r] >= (int32_t)s_r2[q + 1])
        flags |= kMpOrder;
    }
    // ---- merge path per thread over the keys, then a serial merge of E steps -------------
    const int64_t d = (int64_t)threadIdx.x * E;
    int64_t lo = d - nB > 0 ? d - nB : 0, hi = d < nA ? d : nA;
    if (d < n) {
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (s_r1[mid] <= s_r2[d - 1 - mid]) lo = mid + 1;
        else hi = mid;
      }
    }
    int64_t i = lo, j = d - lo;
    uint64_t ka = i < nA ? s_r1[i] : kNoKey, kb = j < nB ? s_r2[j] : kNoKey;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const bool take_a = i < nA && (j >= nB || ka <= kb);
      mk[k] = take_a ? ka : kb;
      ms[k] = take_a ? (int32_t)i : ~(int32_t)j;
      if (d + k < n) {
        if (take_a) {
          ++i;
          ka = i < nA ? s_r1[i] : kNoKey;
        } else {
          ++j;
          kb = j < nB ? s_r2[j] : kNoKey;
        }
      }
    }
    // values of the thread's positions (independent loads)
#pragma unroll
    for (int k = 0; k < E; ++k) {
      mv[k] = 0.0;
      if (d + k < n)
        mv[k] = ms[k] >= 0 ? (double)a_v[iA0 + ms[k]] : (double)b_v[jB0 + ~ms[k]];
    }
    __syncthreads();  // the slices' keys are dead: the merged tile goes to R1 / R3
#pragma unroll
    for (int k = 0; k < E; ++k) {
      if (d + k < n) {
        s_r1[d + k] = mk[k];
        s_r3[d + k] = ms[k];
      }
    }
    __syncthreads();
  }
  // ---- runs: heads, the fold, the kept results (R2 values, R4 rows) ------------------------
  const int64_t d = (int64_t)threadIdx.x * E;
  uint32_t kmask = 0;
  if (d < n) {
    uint64_t prev = d > 0 ? s_r1[d - 1] : s_prevkey;
    double cur = 0.0;
    int cur_k = -1;
    uint64_t cur_key = kNoKey;
    auto emit = [&]() {  // (no branch around the flag updates: they stay in registers)
      const int32_t r = (int32_t)(uint32_t)cur_key;
      const bool bad = r < 0 || (int64_t)r >= L.n_rows;
      const bool keep = !bad && cur != 0.0;
      flags |= bad ? kMpBounds : 0u;
      kmask |= keep ? (1u << cur_k) : 0u;
      if (keep) {
        s_r2[d + cur_k] = __double_as_longlong(cur);
        s_r4[d + cur_k] = r;
      }
    };
#pragma unroll
    for (int k = 0; k < E; ++k) {
      if (d + k < n) {
        if (mk[k] != prev) {
          if (cur_k >= 0) emit();
          cur = mv[k];
          cur_k = k;
          cur_key = mk[k];
        } else if (cur_k >= 0) {
          cur += mv[k];
        }
        prev = mk[k];
      }
    }
    if (cur_k >= 0) {  // the last run may continue past the thread's positions
      int64_t q = d + E;
      while (q < n && s_r1[q] == cur_key) {
        const int32_t sq = s_r3[q];
        cur += sq >= 0 ? (double)a_v[iA0 + sq] : (double)b_v[jB0 + ~sq];
        ++q;
      }
      if (q >= n && W1 < M) {  // ... and past the tile: B's elements after jB1
        const int64_t col = (int64_t)(cur_key >> 32);
        const int64_t bend = col < L.n_cols ? B.at(col + 1) : B.nnz;
        const int32_t row = (int32_t)(uint32_t)cur_key;
        for (int64_t y = jB0 + nB; y < bend && L.b_ri[y] == row; ++y) cur += (double)b_v[y];
      }
      emit();
    }
  }
  // ---- offsets: the workgroup's scan, then look-back; the tile's flags travel in its word --
  if (flags) atomicOr(&s_flags, flags);
  const uint32_t kept = (uint32_t)__popc(kmask);
  uint32_t total_wg;
  const uint32_t excl = wg_excl_scan<NT>(kept, s_w, &total_wg);
  s_toff[threadIdx.x] = excl;
  s_kmask[threadIdx.x] = (uint8_t)kmask;
  __syncthreads();
  const uint32_t wg_flags = s_flags;
  if (threadIdx.x < kWave) {
    const uint64_t own = (uint64_t)total_wg | ((uint64_t)wg_flags << kMergeCntBits);
    uint64_t prefix = 0;
    if (t == 0) {
      if (threadIdx.x == 0) lb_publish(state, kLbPre | own);
    } else {
      if (threadIdx.x == 0) lb_publish(state + t, kLbAgg | own);
      prefix = lookback_exclusive<kMergeFlagBits>(state, t);
      if (threadIdx.x == 0) {
        const uint64_t cnt = (prefix & ((1ull << kMergeCntBits) - 1)) + total_wg;
        const uint64_t fl = (prefix >> kMergeCntBits) | wg_flags;
        lb_publish(state + t, kLbPre | cnt | (fl << kMergeCntBits));
      }
    }
    if (threadIdx.x == 0) s_pre = prefix;
  }
  __syncthreads();
  const int64_t base = (int64_t)(s_pre & ((1ull << kMergeCntBits) - 1));
  // number of kept results before tile position p
  auto kept_before = [&](int64_t p) -> int64_t {
    const int64_t th = p / E;
    if (th >= NT) return total_wg;
    return (int64_t)s_toff[th] + __popc((uint32_t)s_kmask[th] & ((1u << (p % E)) - 1u));
  };
  // the results in position order: consecutive threads take consecutive positions
  for (int64_t p = threadIdx.x; p < n; p += NT) {
    const int64_t th = p / E, k = p % E;
    if ((s_kmask[th] >> k) & 1u) {
      const int64_t o = base + s_toff[th] + __popc((uint32_t)s_kmask[th] & ((1u << k) - 1u));
      if (o >= 0 && o < out_cap) {
        row_idx[o] = s_r4[p];
        const double v = __longlong_as_double((long long)s_r2[p]);
        if (out_f64) static_cast<double*>(val_out)[o] = v;
        else static_cast<float*>(val_out)[o] = (float)v;
      }
    }
  }
  // offsets of the columns that start in [W0, W1)
  if (n > 0) {
    for (int64_t c = c_first + threadIdx.x; c <= cl1 && c < L.n_cols; c += NT) {
      const int64_t m = A.at(c) + B.at(c) - W0;
      if (m >= 0 && m < n) col_ptr[c] = (int32_t)(base + kept_before(m));
    }
  }
  // the last tile: nnz, the status and the offsets of the columns that start at M
  if (t == ntiles - 1) {
    const int64_t total = base + total_wg;
    const uint32_t f = (uint32_t)(s_pre >> kMergeCntBits) | wg_flags;
    for (int64_t c = cM + threadIdx.x; c <= L.n_cols; c += NT) col_ptr[c] = (int32_t)total;
    if (threadIdx.x == 0) {
      info[0] = (int32_t)total;
      const int32_t prior = info[1];
      info[1] = (f & (kMpShape | kMpOrder)) ? st_inval : ((f & kMpBounds) ? st_bounds : prior);
    }
  }
}

}  // namespace spm
