// Device-side building blocks shared by the gfx950 kernels: element loads, wavefront and
// workgroup scans, the decoupled look-back of single-pass chained scans, binary searches.
// Wavefronts are 64 lanes wide (CDNA4); every helper below assumes blockDim.x is a multiple
// of 64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spm {

constexpr int kWave = 64;

// ------------------------------------------------------------------------------------------
// Element types.  bfloat16 is carried as its raw 16 bits; widening to binary32 is exact
// (append 16 zero bits) and binary32 -> binary64 is exact too.
// ------------------------------------------------------------------------------------------
typedef uint16_t bf16_t;

__device__ __forceinline__ float bf16_to_f32(bf16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}

template <typename ACC> __device__ __forceinline__ ACC widen(double x);
template <> __device__ __forceinline__ double widen<double>(double x) { return x; }
template <> __device__ __forceinline__ float widen<float>(double x) { return (float)x; }

template <typename ACC> __device__ __forceinline__ ACC to_acc(double x) { return (ACC)x; }
template <typename ACC> __device__ __forceinline__ ACC to_acc(float x) { return (ACC)x; }
template <typename ACC> __device__ __forceinline__ ACC to_acc(bf16_t x) {
  return (ACC)bf16_to_f32(x);
}

// Four consecutive elements starting at p (p is 4-element aligned when `aligned`), widened to
// ACC.  Elements at or beyond `avail` are returned as 0 and never read.
template <typename ACC, typename T>
__device__ __forceinline__ void load4(const T* __restrict__ p, int avail, bool aligned,
                                      ACC (&o)[4]);

template <typename ACC>
__device__ __forceinline__ void load4(const float* __restrict__ p, int avail, bool aligned,
                                      ACC (&o)[4]) {
  if (aligned && avail >= 4) {
    float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = (ACC)v.x; o[1] = (ACC)v.y; o[2] = (ACC)v.z; o[3] = (ACC)v.w;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = (e < avail) ? (ACC)p[e] : (ACC)0;
  }
}

template <typename ACC>
__device__ __forceinline__ void load4(const double* __restrict__ p, int avail, bool aligned,
                                      ACC (&o)[4]) {
  if (aligned && avail >= 4) {
    double2 a = reinterpret_cast<const double2*>(p)[0];
    double2 b = reinterpret_cast<const double2*>(p)[1];
    o[0] = (ACC)a.x; o[1] = (ACC)a.y; o[2] = (ACC)b.x; o[3] = (ACC)b.y;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = (e < avail) ? (ACC)p[e] : (ACC)0;
  }
}

template <typename ACC>
__device__ __forceinline__ void load4(const bf16_t* __restrict__ p, int avail, bool aligned,
                                      ACC (&o)[4]) {
  if (aligned && avail >= 4) {
    uint2 v = *reinterpret_cast<const uint2*>(p);
    o[0] = (ACC)__uint_as_float(v.x << 16);
    o[1] = (ACC)__uint_as_float(v.x & 0xffff0000u);
    o[2] = (ACC)__uint_as_float(v.y << 16);
    o[3] = (ACC)__uint_as_float(v.y & 0xffff0000u);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = (e < avail) ? (ACC)bf16_to_f32(p[e]) : (ACC)0;
  }
}

// Store n (<= 4) accumulated values rounded once to binary64 or binary32.
template <typename ACC>
__device__ __forceinline__ void store_n(void* base, int64_t idx, int n, bool f64, bool aligned,
                                        const ACC (&v)[4]) {
  if (f64) {
    double* d = static_cast<double*>(base) + idx;
    if (aligned && n == 4) {
      reinterpret_cast<double2*>(d)[0] = make_double2((double)v[0], (double)v[1]);
      reinterpret_cast<double2*>(d)[1] = make_double2((double)v[2], (double)v[3]);
    } else {
      for (int e = 0; e < n; ++e) d[e] = (double)v[e];
    }
  } else {
    float* f = static_cast<float*>(base) + idx;
    if (aligned && n == 4) {
      *reinterpret_cast<float4*>(f) = make_float4((float)v[0], (float)v[1], (float)v[2],
                                                  (float)v[3]);
    } else {
      for (int e = 0; e < n; ++e) f[e] = (float)v[e];
    }
  }
}

// ------------------------------------------------------------------------------------------
// Scans and reductions.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

__device__ __forceinline__ uint64_t wave_or_u64(uint64_t x) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) x |= __shfl_xor(x, d, kWave);
  return x;
}

// Exclusive scan of one value per thread across the workgroup (NT threads).  `lds` needs
// NT/64 + 1 words.  Returns the exclusive prefix; *total receives the workgroup sum.
template <int NT>
__device__ __forceinline__ uint32_t wg_excl_scan(uint32_t x, uint32_t* lds, uint32_t* total) {
  constexpr int NW = NT / kWave;
  const uint32_t incl = wave_incl_scan(x);
  if (lane_id() == kWave - 1) lds[wave_id()] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      uint32_t t = lds[w];
      lds[w] = run;
      run += t;
    }
    lds[NW] = run;
  }
  __syncthreads();
  const uint32_t excl = lds[wave_id()] + incl - x;
  *total = lds[NW];
  __syncthreads();
  return excl;
}

// In-place inclusive max-scan of a[0 .. 8 NT) seeded with `init` (8 consecutive entries per
// thread).  `s_w` needs NT/64 words.
template <int NT>
__device__ __forceinline__ void wg_max_scan8(int32_t* a, int32_t init, int32_t* s_w) {
  int32_t v[8];
  int32_t m = init;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[k] = a[threadIdx.x * 8 + k];
    m = max(m, v[k]);
  }
  int32_t inc = m;  // inclusive over the wave
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int32_t y = __shfl_up(inc, d, kWave);
    if (lane_id() >= d) inc = max(inc, y);
  }
  if (lane_id() == kWave - 1) s_w[wave_id()] = inc;
  __syncthreads();
  int32_t e = init;  // earlier waves, then earlier lanes
  for (int w = 0; w < wave_id(); ++w) e = max(e, s_w[w]);
  const int32_t p = __shfl_up(inc, 1, kWave);
  if (lane_id() > 0) e = max(e, p);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    e = max(e, v[k]);
    a[threadIdx.x * 8 + k] = e;
  }
}

// In-place inclusive scan of a[0..n) by the whole workgroup (blocked chunks with a carry).
template <int NT>
__device__ void wg_inclusive_scan_inplace(uint32_t* a, int64_t n, uint32_t* s_w) {
  constexpr int IPT = 8;
  uint32_t carry = 0;
  for (int64_t base = 0; base < n; base += (int64_t)NT * IPT) {
    uint32_t v[IPT];
    uint32_t sum = 0;
#pragma unroll
    for (int s = 0; s < IPT; ++s) {
      const int64_t i = base + (int64_t)threadIdx.x * IPT + s;
      v[s] = (i < n) ? a[i] : 0u;
      sum += v[s];
    }
    uint32_t total;
    const uint32_t excl = wg_excl_scan<NT>(sum, s_w, &total);
    uint32_t run = carry + excl;
#pragma unroll
    for (int s = 0; s < IPT; ++s) {
      const int64_t i = base + (int64_t)threadIdx.x * IPT + s;
      run += v[s];
      if (i < n) a[i] = run;
    }
    carry += total;
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------
// Decoupled look-back (single-pass chained scan; Merrill & Garland, "Single-pass Parallel
// Prefix Scan with Decoupled Look-back", 2016).  Each tile publishes one 64-bit word:
// bits 63..62 = state (0 none, 1 aggregate only, 2 inclusive prefix), bits 61..0 = value.
// Tiles take their index from an atomic ticket so that every predecessor has started.
// ------------------------------------------------------------------------------------------
constexpr uint64_t kLbAgg = 1ull << 62;
constexpr uint64_t kLbPre = 2ull << 62;
constexpr uint64_t kLbVal = (1ull << 62) - 1;

// The state and the value share one 64-bit word, so a reader never needs any other memory
// made visible by the writer: relaxed device-scope atomics suffice.  (Acquire / release at
// device scope would also write back / invalidate the XCD-local L2 on every access.)
__device__ __forceinline__ void lb_publish(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t lb_read(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by all 64 lanes of ONE wave of tile `tile` (> 0) after it published its aggregate.
// Returns the sum of every earlier tile.  Each pass reads a window of 4 states per lane
// (256 predecessors): device-coherent reads cross the XCD fabric, so fewer, wider passes
// shorten the chain.  Lane l holds the states of tiles base - 4l - q, q = 0..3 (q = 0 is the
// closest); the window is summed up to and including the closest inclusive prefix.
// With FB > 0 the top FB bits of a value are flags: those are OR-ed instead of summed (the
// count lives in the low 62 - FB bits).
template <int FB = 0>
__device__ inline uint64_t lookback_exclusive(const uint64_t* state, int64_t tile) {
  constexpr int Q = 4;
  constexpr int CB = 62 - FB;
  constexpr uint64_t kCnt = (1ull << CB) - 1;
  const int lane = lane_id();
  uint64_t excl = 0, fl = 0;
  int64_t base = tile - 1;
  while (base >= 0) {
    uint64_t v[Q];
    int firstp_q = Q;     // closest (smallest q) inclusive prefix in this lane, Q if none
    bool zero_before = false;  // a not-yet-published state closer than that prefix
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t i = base - (int64_t)lane * Q - q;
      v[q] = (i >= 0) ? lb_read(state + i) : kLbPre;
    }
#pragma unroll
    for (int q = Q - 1; q >= 0; --q) {
      if ((v[q] >> 62) == 2) firstp_q = q;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (q < firstp_q && (v[q] >> 62) == 0) zero_before = true;
    const uint64_t pm = __ballot(firstp_q < Q);
    const int first_lane = pm ? (__ffsll((unsigned long long)pm) - 1) : kWave;
    // lanes up to first_lane matter; in first_lane only states up to its prefix matter
    const bool relevant = lane <= first_lane;
    const uint64_t zm = __ballot(relevant && zero_before);
    if (zm) {  // a tile we depend on has not published yet: wait and re-read
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    uint64_t mine = 0, mf = 0;
    if (relevant) {
      const int qmax = (lane == first_lane) ? firstp_q : Q - 1;
#pragma unroll
      for (int q = 0; q < Q; ++q)
        if (q <= qmax) {
          mine += v[q] & kCnt;
          if (FB > 0) mf |= (v[q] & kLbVal) >> CB;
        }
    }
    excl += wave_sum_u64(mine);
    if (FB > 0) fl |= wave_or_u64(mf);
    if (pm) break;
    base -= (int64_t)kWave * Q;
  }
  return FB > 0 ? (excl | (fl << CB)) : excl;
}

// ------------------------------------------------------------------------------------------
// Searches over non-decreasing int32 arrays (any address space via generic pointers).
// ------------------------------------------------------------------------------------------
// First i in [0, n) with a[i] >= x, or n.
template <typename T>
__device__ __forceinline__ int64_t lower_bound(const T* a, int64_t n, int64_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// First i in [0, n) with a[i] > x, or n.
template <typename T>
__device__ __forceinline__ int64_t upper_bound(const T* a, int64_t n, int64_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

}  // namespace spm
