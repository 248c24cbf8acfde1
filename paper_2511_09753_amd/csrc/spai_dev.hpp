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
  // ELL copy, used when eshift >= 0: row u occupies slots [u << eshift, (u + 1) << eshift)
  // (width a power of two >= 8), its entries first in ascending column order, then
  // padding with column -1 and value 0.  Row u's address needs no row-pointer load.
  int eshift = -1;
  const int32_t* ecol = nullptr;
  const double* eval = nullptr;   // float64 values, or null
  const float* eval32 = nullptr;  // float32 values (mixed precision), or null
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
// lane l's value of a 64-bit per-lane register, as a wave-uniform value (l constant)
__device__ __forceinline__ int64_t wave_read64(int64_t v, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(uint64_t)v, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
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

// ---- ordered key set (history independent) -----------------------------------
// A key k is stored as its Fibonacci hash h(k) = k * kHashMul (mod 2^32), a bijection
// on 32-bit words, so k = h * kHashInv recovers it.  The home slot is the top bits of
// h, and an insert walks forward from home keeping the smaller hash in every slot it
// passes (an atomic min that carries the displaced, larger value on).  With no wrap
// around (the table ends in an overflow area instead), the final contents do not
// depend on the order of the inserts: occupied slots, read in slot order, list the
// keys sorted by h (Amble and Knuth's ordered hash tables).  The kernels sum over the
// keys in that order, so results are deterministic without sorting the keys.
constexpr unsigned kHashMul = 0x9E3779B1u;
constexpr unsigned kHashInv = 0x0E8B2F51u;   // kHashMul * kHashInv = 1 (mod 2^32)
constexpr unsigned kOhEmpty = 0xFFFFFFFFu;   // no row index hashes to it (its preimage is > 2^31)
constexpr int kOhOver = 64;                  // overflow slots after the H home slots

__device__ __forceinline__ unsigned ohash(int k) { return (unsigned)k * kHashMul; }
__device__ __forceinline__ int ounhash(unsigned h) { return (int)(h * kHashInv); }

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

// Insert up to U keys per lane (a negative key inserts nothing), every lane's CASes in
// flight together, then linear probing for the few that collide.  Returns the number
// of slots this lane claimed.  The caller keeps the table below full (see
// ks_insert_rows), so every probe sequence ends at a free slot or at its own key.
template <int U>
__device__ __forceinline__ int ks_insert_batch(int* keys, int H, const int (&key)[U]) {
  unsigned h[U];
  bool pend[U];
  int claimed = 0;
#pragma unroll
  for (int c = 0; c < U; ++c) {
    pend[c] = key[c] >= 0;
    h[c] = hash_key(key[c]) & (unsigned)(H - 1);
  }
  while (true) {
    int prev[U];
#pragma unroll
    for (int c = 0; c < U; ++c) prev[c] = pend[c] ? atomicCAS(&keys[h[c]], -1, key[c]) : key[c];
    bool any = false;
#pragma unroll
    for (int c = 0; c < U; ++c) {
      if (!pend[c]) continue;
      if (prev[c] == -1) {
        ++claimed;
        pend[c] = false;
      } else if (prev[c] == key[c]) {
        pend[c] = false;
      } else {
        h[c] = (h[c] + 1) & (unsigned)(H - 1);
        any = true;
      }
    }
    if (!any) break;
  }
  return claimed;
}

// ---- LDS position map: row index -> positions of that row in up to two lists ------
// keys[slot] (-1 = empty) and pos[slot], two 16-bit list positions (0xFFFF = absent).
// The caller sizes the map (a power of two) at least twice the number of keys, so
// probing terminates.
constexpr unsigned kNoPos = 0xFFFFu;

__device__ __forceinline__ void lm_clear(int* keys, unsigned* pos, int hs) {
  for (int i = lane_id(); i < hs; i += SPAI_WAVE) {
    keys[i] = -1;
    pos[i] = 0xFFFFFFFFu;
  }
}

// record that row `key` sits at position e of list `half` (0 or 1)
__device__ __forceinline__ void lm_put(int* keys, unsigned* pos, int hs, int key, int half, int e) {
  unsigned h = hash_key(key) & (unsigned)(hs - 1);
  while (true) {
    const int prev = atomicCAS(&keys[h], -1, key);
    if (prev == -1 || prev == key) break;
    h = (h + 1) & (unsigned)(hs - 1);
  }
  atomicAnd(&pos[h], half ? (((unsigned)e << 16) | 0xFFFFu) : (0xFFFF0000u | (unsigned)e));
}

// position words of U rows (a negative row is absent); the U first probes (key and
// position word of the home slot) are issued together
template <int U>
__device__ __forceinline__ void lm_find(const int* keys, const unsigned* pos, int hs,
                                        const int (&key)[U], unsigned (&pw)[U]) {
  unsigned h[U];
  int k[U];
#pragma unroll
  for (int c = 0; c < U; ++c) {
    h[c] = hash_key(key[c]) & (unsigned)(hs - 1);
    k[c] = keys[h[c]];
    pw[c] = pos[h[c]];
  }
#pragma unroll
  for (int c = 0; c < U; ++c) {
    while (k[c] != key[c] && k[c] != -1) {
      h[c] = (h[c] + 1) & (unsigned)(hs - 1);
      k[c] = keys[h[c]];
      pw[c] = pos[h[c]];
    }
    if (k[c] != key[c] || key[c] < 0) pw[c] = 0xFFFFFFFFu;
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
// shuffles; larger sets by the LDS bitonic network.  by_hash: order by the Fibonacci
// hash ohash(k) instead of k (the order the ordered key set yields; h ^ 2^31 orders
// as a signed int like h as unsigned, and the INT_MAX padding is the empty word).
__device__ inline int ks_sort_inplace(int* keys, int H, bool by_hash = false) {
  int cnt = 0;
  for (int base = 0; base < H; base += SPAI_WAVE) {
    int k = keys[base + lane_id()];
    bool occ = k != -1;
    unsigned long long m = __ballot(occ);
    __syncthreads();
    if (occ) keys[cnt + __popcll(m & lanemask_lt())] = by_hash ? (int)(ohash(k) ^ 0x80000000u) : k;
    cnt += __popcll(m);
    __syncthreads();
  }
  if (by_hash && cnt == 1) {
    if (lane_id() == 0) keys[0] = ounhash((unsigned)keys[0] ^ 0x80000000u);
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
  if (by_hash) {
    for (int i = lane_id(); i < cnt; i += SPAI_WAVE)
      keys[i] = ounhash((unsigned)keys[i] ^ 0x80000000u);
    __syncthreads();
  }
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

// U lower-bound searches in lock-step: lookup c looks for key[c] in the ascending list
// a[base[c] .. base[c] + len[c]) and gets its index there in pos[c], or -1.  All U
// lookups take the same power-of-two steps, so each step issues U independent LDS
// reads instead of U dependent chains.
template <int U>
__device__ __forceinline__ void search_lockstep(const int* a, const int (&base)[U],
                                                const int (&len)[U], const int (&key)[U],
                                                int (&pos)[U]) {
  int mx = 0;
#pragma unroll
  for (int c = 0; c < U; ++c) mx = max(mx, len[c]);
  int lo[U];
#pragma unroll
  for (int c = 0; c < U; ++c) lo[c] = 0;
  for (int step = mx ? (1 << (31 - __clz(mx))) : 0; step > 0; step >>= 1) {
#pragma unroll
    for (int c = 0; c < U; ++c) {
      const int m = lo[c] + step;
      if (m <= len[c] && a[base[c] + m - 1] < key[c]) lo[c] = m;
    }
  }
#pragma unroll
  for (int c = 0; c < U; ++c) pos[c] = (lo[c] < len[c] && a[base[c] + lo[c]] == key[c]) ? lo[c] : -1;
}

// the same with every lookup in one list a[0..n)
template <int U>
__device__ __forceinline__ void search_lockstep1(const int* a, int n, const int (&key)[U],
                                                 int (&pos)[U]) {
  int lo[U];
#pragma unroll
  for (int c = 0; c < U; ++c) lo[c] = 0;
  for (int step = n ? (1 << (31 - __clz(n))) : 0; step > 0; step >>= 1) {
#pragma unroll
    for (int c = 0; c < U; ++c) {
      const int m = lo[c] + step;
      if (m <= n && a[m - 1] < key[c]) lo[c] = m;
    }
  }
#pragma unroll
  for (int c = 0; c < U; ++c) pos[c] = (lo[c] < n && a[lo[c]] == key[c]) ? lo[c] : -1;
}

// the same for two lists a[b0 .. b0 + n0) and a[b1 .. b1 + n1) searched for the same keys
template <int U>
__device__ __forceinline__ void search_lockstep2(const int* a, int b0, int n0, int b1, int n1,
                                                 const int (&key)[U], int (&p0)[U],
                                                 int (&p1)[U]) {
  int l0[U], l1[U];
#pragma unroll
  for (int c = 0; c < U; ++c) l0[c] = l1[c] = 0;
  const int mx = max(n0, n1);
  for (int step = mx ? (1 << (31 - __clz(mx))) : 0; step > 0; step >>= 1) {
#pragma unroll
    for (int c = 0; c < U; ++c) {
      const int m0 = l0[c] + step, m1 = l1[c] + step;
      const bool g0 = m0 <= n0 && a[b0 + m0 - 1] < key[c];
      const bool g1 = m1 <= n1 && a[b1 + m1 - 1] < key[c];
      if (g0) l0[c] = m0;
      if (g1) l1[c] = m1;
    }
  }
#pragma unroll
  for (int c = 0; c < U; ++c) {
    p0[c] = (l0[c] < n0 && a[b0 + l0[c]] == key[c]) ? l0[c] : -1;
    p1[c] = (l1[c] < n1 && a[b1 + l1[c]] == key[c]) ? l1[c] : -1;
  }
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

// Insert up to U keys per lane (negative: none) into T[0 .. H + kOhOver), H = 2^(32 - shift).
// A walk moves one slot per step and starts at a home slot below H, so capping the
// walks at kOhOver steps keeps every probe inside the table.  Returns false (on every
// lane) if a walk needed more steps; the caller then gives the column to a larger tile.
template <int U>
__device__ __forceinline__ bool oh_insert_batch(unsigned* T, int shift, const int (&key)[U]) {
  // The walk state is updated with selects, not branches: only the atomic itself sits
  // under a condition, so the wave runs one short loop (until no lane has a key in
  // flight) instead of a branch per key and step.  A walk that found an empty slot
  // gets max(empty, v) = empty, so placed, already present and not started all end as
  // the empty word, which no key hashes to.
  unsigned v[U];
  int s[U];
#pragma unroll
  for (int c = 0; c < U; ++c) {
    v[c] = key[c] >= 0 ? ohash(key[c]) : kOhEmpty;
    s[c] = key[c] >= 0 ? (int)(v[c] >> shift) : 0;
  }
  for (int step = 0; step < kOhOver; ++step) {
    unsigned old[U];
#pragma unroll
    for (int c = 0; c < U; ++c) {
      old[c] = kOhEmpty;
      if (v[c] != kOhEmpty) old[c] = atomicMin(&T[s[c]], v[c]);
    }
    bool live = false;
#pragma unroll
    for (int c = 0; c < U; ++c) {
      v[c] = old[c] == v[c] ? kOhEmpty : max(old[c], v[c]);   // walk on with the larger
      s[c] += 1;
      live = live || v[c] != kOhEmpty;
    }
    if (__ballot(live) == 0ull) return true;
  }
  return false;
}

// Compact the occupied slots of T[0 .. end) in place into keys (decoded), in slot order;
// returns the count.  One wave; each 64-slot chunk is read before it is written.
__device__ __forceinline__ int oh_compact(unsigned* T, int end) {
  int cnt = 0;
  for (int base = 0; base < end; base += SPAI_WAVE) {
    const unsigned x = T[base + lane_id()];
    const bool occ = x != kOhEmpty;
    const unsigned long long m = __ballot(occ);
    if (occ) ((int*)T)[cnt + __popcll(m & lanemask_lt())] = ounhash(x);
    cnt += __popcll(m);
  }
  return cnt;
}

// Sum of six values over the wave as a fixed transpose tree: the first three halving
// steps exchange half of the live values (six padded to eight), the last three add the
// single remaining value; every step pairs lanes by xor, so the order of the additions
// is fixed.  Returns the six sums in s[0..5] on every lane.
__device__ __forceinline__ void wave_sum6(double (&v)[6]) {
  const int lane = lane_id();
  double a[8] = {v[0], v[1], v[2], v[3], v[4], v[5], 0.0, 0.0};
  // xor 32: lanes < 32 keep values 0-3, lanes >= 32 keep 4-7
  const bool up32 = (lane & 32) != 0;
  double b[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double send = up32 ? a[c] : a[c + 4];
    const double keep = up32 ? a[c + 4] : a[c];
    b[c] = keep + __shfl_xor(send, 32, SPAI_WAVE);
  }
  // xor 16: keep two of the four
  const bool up16 = (lane & 16) != 0;
  double d[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const double send = up16 ? b[c] : b[c + 2];
    const double keep = up16 ? b[c + 2] : b[c];
    d[c] = keep + __shfl_xor(send, 16, SPAI_WAVE);
  }
  // xor 8: keep one of the two
  const bool up8 = (lane & 8) != 0;
  double e;
  {
    const double send = up8 ? d[0] : d[1];
    const double keep = up8 ? d[1] : d[0];
    e = keep + __shfl_xor(send, 8, SPAI_WAVE);
  }
#pragma unroll
  for (int dd = 4; dd >= 1; dd >>= 1) e += __shfl_xor(e, dd, SPAI_WAVE);
  // value q = 4 (lane bit 5) + 2 (bit 4) + (bit 3) lives in lane 8 q (and its group)
#pragma unroll
  for (int q = 0; q < 6; ++q) v[q] = __shfl(e, 8 * q, SPAI_WAVE);
}

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
