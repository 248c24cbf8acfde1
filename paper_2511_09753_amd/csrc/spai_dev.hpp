// spai_dev.hpp — device building blocks shared by the libspai kernels (gfx950, wave64).
//
// Every per-column kernel runs one 64-lane wavefront per workgroup, so a workgroup
// barrier is a wave barrier: the LDS scratch of one column belongs to one wave and
// __syncthreads() orders its LDS traffic at negligible cost.
//
// Floating-point contraction is disabled for the whole library (-ffp-contract=off):
// the mirrored computations (R(j,k) from column k and R^T(k,j) from the neighbour
// columns of M) must round identically for the symmetrized iterate to be exactly
// symmetric.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <limits.h>

#define SPAI_WAVE 64

namespace spai {

struct Csr {                 // A on the device (symmetric: row k == column k)
  int64_t n = 0, nnz = 0;
  const int64_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const double* val = nullptr;   // float64 values
  const float* val32 = nullptr;  // float32 copy (mixed precision), or null
};

template <typename T>
struct Cols {                // padded column-compressed matrix: column j occupies
  int64_t* beg = nullptr;    // idx/val[beg[j] .. beg[j] + len[j]), rows ascending
  int32_t* len = nullptr;
  int32_t* idx = nullptr;
  T* val = nullptr;
  int64_t cap = 0;           // capacity of idx/val
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & (SPAI_WAVE - 1); }

__device__ __forceinline__ unsigned long long lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// fixed-tree butterfly sum: every lane gets the bitwise-identical total
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, SPAI_WAVE);
  return v;
}
__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, SPAI_WAVE);
  return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, SPAI_WAVE);
  return v;
}
__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, SPAI_WAVE));
  return v;
}

// inclusive prefix sum over the wave
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < SPAI_WAVE; d <<= 1) {
    int t = __shfl_up(v, d, SPAI_WAVE);
    if (l >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ unsigned hash_key(int k) {
  unsigned x = (unsigned)k * 0x9E3779B1u;
  return x ^ (x >> 16);
}

// ---- LDS key set (open addressing, -1 = empty) -------------------------------
// The caller guarantees fewer distinct keys than slots, so probing terminates.
__device__ __forceinline__ void ks_clear(int* keys, int H) {
  for (int i = lane_id(); i < H; i += SPAI_WAVE) keys[i] = -1;
}
__device__ __forceinline__ void ks_insert(int* keys, int H, int key) {
  unsigned h = hash_key(key) & (unsigned)(H - 1);
  while (true) {
    int prev = atomicCAS(&keys[h], -1, key);
    if (prev == -1 || prev == key) return;
    h = (h + 1) & (unsigned)(H - 1);
  }
}

// Insert with a bound on the number of distinct keys: `cnt` counts the keys placed,
// and once it reaches `limit` further inserts are refused and `*over` is set.  With
// limit + 64 < H (at most 64 lanes insert at once) an empty slot always exists, so
// probing terminates.
__device__ __forceinline__ void ks_insert_bounded(int* keys, int H, int key, int* cnt, int limit,
                                                  int* over) {
  if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= limit) {
    *over = 1;
    return;
  }
  unsigned h = hash_key(key) & (unsigned)(H - 1);
  while (true) {
    int prev = atomicCAS(&keys[h], -1, key);
    if (prev == -1) {
      if (atomicAdd(cnt, 1) + 1 > limit) *over = 1;
      return;
    }
    if (prev == key) return;
    h = (h + 1) & (unsigned)(H - 1);
  }
}

__device__ __forceinline__ int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// ascending bitonic sort of a[0..S) (S a power of two) by one wave
__device__ inline void bitonic_sort_int(int* a, int S) {
  for (int k = 2; k <= S; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane_id(); i < S; i += SPAI_WAVE) {
        int ixj = i ^ j;
        if (ixj > i) {
          int x = a[i], y = a[ixj];
          bool asc = (i & k) == 0;
          if ((x > y) == asc) { a[i] = y; a[ixj] = x; }
        }
      }
      __syncthreads();
    }
  }
}

// Ascending bitonic sort of 64 * C keys held in registers: element c * 64 + lane is
// v[c].  Fully unrolled so every register index is a compile-time constant.
template <int C>
__device__ __forceinline__ void wave_bitonic(int (&v)[C]) {
  const int lane = lane_id();
  constexpr int S = 64 * C;
#pragma unroll
  for (int k = 2; k <= S; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int c2 = c ^ (j / 64);
          if (c2 > c) {
            const bool asc = (((c * 64 + lane) & k) == 0);
            const int a = v[c], b = v[c2];
            if ((a > b) == asc) { v[c] = b; v[c2] = a; }
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int i = c * 64 + lane;
          const int o = __shfl_xor(v[c], j, SPAI_WAVE);
          const bool asc = ((i & k) == 0);
          const bool lower = ((i & j) == 0);
          v[c] = (lower == asc) ? min(v[c], o) : max(v[c], o);
        }
      }
    }
  }
}

template <int C>
__device__ __forceinline__ void sort_in_registers(int* keys, int cnt) {
  int v[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int i = c * 64 + lane_id();
    v[c] = i < cnt ? keys[i] : INT_MAX;
  }
  wave_bitonic<C>(v);
#pragma unroll
  for (int c = 0; c < C; ++c) keys[c * 64 + lane_id()] = v[c];
}

// Sort the keys of the set in place: keys[0..cnt) ascending, returns cnt.  The
// compaction writes slot s to position <= s after the whole 64-slot chunk has been
// read, so it can run in place.  Up to 256 keys are sorted in registers with
// shuffles; larger sets by the LDS bitonic network.
__device__ inline int ks_sort_inplace(int* keys, int H) {
  int cnt = 0;
  for (int base = 0; base < H; base += SPAI_WAVE) {
    int k = keys[base + lane_id()];
    bool occ = k != -1;
    unsigned long long m = __ballot(occ);
    __syncthreads();
    if (occ) keys[cnt + __popcll(m & lanemask_lt())] = k;
    cnt += __popcll(m);
    __syncthreads();
  }
  if (cnt <= 1) return cnt;
  if (cnt <= 64 && H >= 64) {
    sort_in_registers<1>(keys, cnt);
  } else if (cnt <= 128 && H >= 128) {
    sort_in_registers<2>(keys, cnt);
  } else if (cnt <= 256 && H >= 256) {
    sort_in_registers<4>(keys, cnt);
  } else {
    int S = next_pow2(cnt);
    for (int i = cnt + lane_id(); i < S; i += SPAI_WAVE) keys[i] = INT_MAX;
    __syncthreads();
    bitonic_sort_int(keys, S);
  }
  __syncthreads();
  return cnt;
}

// Gather the keys of the set into out[0..cnt) in ascending order; returns cnt.
// out must hold next_pow2(cnt) ints (<= H).
__device__ inline int ks_sorted(int* keys, int H, int* out) {
  int cnt = 0;
  for (int base = 0; base < H; base += SPAI_WAVE) {
    int k = keys[base + lane_id()];
    bool occ = k != -1;
    unsigned long long m = __ballot(occ);
    if (occ) out[cnt + __popcll(m & lanemask_lt())] = k;
    cnt += __popcll(m);
  }
  int S = next_pow2(cnt > 0 ? cnt : 1);
  for (int i = cnt + lane_id(); i < S; i += SPAI_WAVE) out[i] = INT_MAX;
  __syncthreads();
  if (cnt > 1) bitonic_sort_int(out, S);
  return cnt;
}

// position of key in ascending a[0..n), or -1
__device__ __forceinline__ int bsearch_idx(const int* a, int n, int key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return (lo < n && a[lo] == key) ? lo : -1;
}

// first position p with a[p] > v in ascending a[0..n)
__device__ __forceinline__ int upper_bound_int(const int* a, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] <= v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <typename T> __device__ __forceinline__ double ld(const T* p) { return (double)(*p); }

// Columns of a grid-stride loop.  The columns are split into 8 contiguous ranges,
// one per XCD (workgroups are dealt round-robin over the 8 XCDs of the chip), so
// the neighbour columns a workgroup touches tend to be cached in its own XCD's L2.
// `unit` / `units` identify the wave (or workgroup) walking and how many there are.
struct ColumnWalk {
  int64_t begin, end, step;
  __device__ ColumnWalk(int64_t n, int64_t unit, int64_t units) {
    const int64_t nx = (units >= 8) ? 8 : 1;
    const int64_t per = units / nx;        // walkers per XCD
    const int64_t x = unit % nx;           // XCD of this walker
    const int64_t loc = unit / nx;
    const int64_t chunk = (n + nx - 1) / nx;
    step = per;
    end = (x + 1) * chunk < n ? (x + 1) * chunk : n;
    begin = (loc < per) ? x * chunk + loc : end;   // surplus walkers get no columns
  }
};

}  // namespace spai
