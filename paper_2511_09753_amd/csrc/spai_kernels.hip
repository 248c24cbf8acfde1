// spai_kernels.hip — HIP kernels of the global SPAI iterations for gfx950.
//
// Method: Venkovic & Anzt, MR (Algorithm 1), CG with matrix iterates (Algorithm 3),
// LOMR (Theorem 4.2, Algorithm 4), hard thresholding (Section 6.1), explicit residual
// (Section 6.2) and the main-iterate drop steps of Appendix A.
//
// Storage: every iterate is column-compressed with padded columns (see Cols): column
// j is an independent unit of f(M) = sum_j ||e_j - A m_j||^2 (Section 2), so each
// per-column kernel gives one column to one 64-lane wavefront and keeps that column's
// working set (input lists, hash set of output rows, sorted keys) in LDS.  A is
// symmetric, so row k of A is also column k.
//
// Determinism: no floating-point atomics.  Every output value is a sum taken in a
// fixed order (ascending row index of A's row, or of the key set), every per-column
// Frobenius partial is a fixed-tree wave sum, and the cross-column reductions run
// in a fixed order (launch_reduce).  The set of keys in the LDS hash is independent
// of insertion order and is sorted before use.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "spai_dev.hpp"
#include "spai_kern.hpp"

namespace spai {

static_assert(offsetof(DevState, rawM) == offsetof(DevState, thrM) + 2 * sizeof(double) &&
                  offsetof(DevState, rawP) == offsetof(DevState, thrP) + 2 * sizeof(double),
              "the selection writes the raw key two doubles after its threshold");

__device__ __forceinline__ double aval(const Csr& A, int64_t q) {
  return A.val32 ? (double)A.val32[q] : A.val[q];
}

// 8-byte aligned carve-up of the dynamic LDS of a per-column kernel
// (offsets only, no integer round trip of the pointer, so the compiler still sees
// LDS addresses and emits ds_* instructions rather than flat ones)
struct Carve {
  char* base;
  unsigned off = 0;
  __device__ explicit Carve(char* b) : base(b) {}
  template <typename U> __device__ U* take(int count) {
    off = (off + 7u) & ~7u;
    U* r = (U*)(base + off);
    off += (unsigned)(sizeof(U) * (unsigned)count);
    return r;
  }
  template <typename U> __device__ U* take16(int count) {   // 16-byte aligned
    off = (off + 15u) & ~15u;
    U* r = (U*)(base + off);
    off += (unsigned)(sizeof(U) * (unsigned)count);
    return r;
  }
};

// ---- lean resident tier helpers (A in ELL) -----------------------------------------
// Byte-table map of a column's lists (up to 128 entries, two lists with unique rows in
// each): a table of kBtCells 16-bit cells maps the hash of a row to 1 + its position in
// list 0 (low byte) and in list 1 (high byte), 0 meaning none.  Each list's entries sit
// in ent[] behind a sentinel entry (a row no lookup asks for, value 0), so the byte is
// the entry's index in its list's block as it stands.  The hash multiplier is picked per
// column among kBtMuls odd constants so that no two rows of one list share a cell; a
// lookup is then one cell read plus one entry read per list, with no probing and no
// branches.
constexpr int kBtCells = 1024;
constexpr int kBtMuls = 16;
constexpr int kBtNone = -2;           // the sentinel's row (ELL padding asks for -1)

// odd 24-bit multipliers (a column retries with the next one while two of its rows
// share a cell)
__device__ __forceinline__ unsigned bt_mul(int a) {
  switch (a & 15) {
    case 0: return 0x9E3779u;
    case 1: return 0x85EBCBu;
    case 2: return 0xC2B2AFu;
    case 3: return 0x27D4EBu;
    case 4: return 0x165667u;
    case 5: return 0xD3A265u;
    case 6: return 0xFD7047u;
    case 7: return 0xB55A4Fu;
    case 8: return 0x7FEB35u;
    case 9: return 0x846CA7u;
    case 10: return 0x2C1B3Du;
    case 11: return 0x297A2Du;
    case 12: return 0xA136ABu;
    case 13: return 0x9E6C63u;
    case 14: return 0x1B8735u;
    default: return 0xCC9E2Du;
  }
}

template <typename T>
struct BtEnt {
  int row;
  T val;
};

// multiplicative hash on 24-bit words: the top 10 of the low 24 bits of row * m, from
// one full-rate 24-bit multiply.  A cluster of nearby rows (a column of a matrix with
// local couplings) spreads over the cells almost like a linear map, so the first
// multiplier seldom clashes.  Rows equal in their low 24 bits share a cell under every
// multiplier; a column holding two such rows goes to the next tier.
// (The multiply is written out: left to itself the compiler sees that only the low 24
// bits of the operands matter, drops the 24-bit form and emits the quarter-rate 32-bit
// multiply instead.)
__device__ __forceinline__ unsigned bt_cell(int row, unsigned m) {
  unsigned p;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(p) : "v"(row), "v"(m));
  return (p >> 14) & (unsigned)(kBtCells - 1);
}

// a value masked to zero in the iterate's type, then widened: the opaque copy keeps the
// compiler from widening first and masking both halves of the double
template <typename T>
__device__ __forceinline__ double bt_masked(bool h, T x) {
  T y = h ? x : (T)0;
  if constexpr (sizeof(T) == 4) asm("" : "+v"(y));
  return (double)y;
}

// Each lane holds up to K entries (row < 0: none), entry k of list lst[k] at position
// pos[k].  Writes 1 + pos into the entry's byte and keeps the first multiplier under
// which every byte reads back as written; returns its index, or -1 (nothing left written).
// (S bytes per cell: one per list)
template <int K, int S = 2>
__device__ __forceinline__ int bt_build(unsigned char* cb, const int (&row)[K], const int (&lst)[K],
                                        const int (&pos)[K]) {
  for (int a = 0; a < kBtMuls; ++a) {
    const unsigned m = bt_mul(a);
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (row[k] >= 0) cb[S * bt_cell(row[k], m) + lst[k]] = (unsigned char)(pos[k] + 1);
    __syncthreads();
    bool clash = false;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (row[k] >= 0 && cb[S * bt_cell(row[k], m) + lst[k]] != (unsigned char)(pos[k] + 1))
        clash = true;
    if (__ballot(clash) == 0ull) return a;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (row[k] >= 0) cb[S * bt_cell(row[k], m) + lst[k]] = 0;
    __syncthreads();
  }
  return -1;
}

template <int K, int S = 2>
__device__ __forceinline__ void bt_clear(unsigned char* cb, const int (&row)[K], const int (&lst)[K],
                                         unsigned m) {
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (row[k] >= 0) cb[S * bt_cell(row[k], m) + lst[k]] = 0;
}

// row w in list 0 (block e0: sentinel, then its entries) and list 1 (block e1): hit
// flags and values (the value is 0 where the byte is 0: the sentinel's)
template <typename T>
__device__ __forceinline__ void bt_find(const unsigned short* cell, unsigned m,
                                        const BtEnt<T>* e0, const BtEnt<T>* e1, int w, bool& h0,
                                        T& x0, bool& h1, T& x1) {
  const unsigned v = cell[bt_cell(w, m)];
  const BtEnt<T> a = e0[v & 0xFFu];
  const BtEnt<T> b = e1[v >> 8];
  h0 = a.row == w;
  h1 = b.row == w;
  x0 = a.val;
  x1 = b.val;
}

// the same for a map of one list (a byte per cell)
template <typename T>
__device__ __forceinline__ void bt_find1(const unsigned char* cell, unsigned m,
                                         const BtEnt<T>* e0, int w, bool& h0, T& x0) {
  const unsigned v = cell[bt_cell(w, m)];
  const BtEnt<T> a = e0[v];
  h0 = a.row == w;
  x0 = a.val;
}

// the eight column indices of ELL row `row` from slot c (all -1 for row < 0)
__device__ __forceinline__ void ell_cols8(const Csr& A, int row, int c, int (&cols)[8]) {
  if (row >= 0) {
    const int64_t q = ((int64_t)row << A.eshift) + c;
    const int4 a = *(const int4*)(A.ecol + q);
    const int4 b = *(const int4*)(A.ecol + q + 4);
    cols[0] = a.x; cols[1] = a.y; cols[2] = a.z; cols[3] = a.w;
    cols[4] = b.x; cols[5] = b.y; cols[6] = b.z; cols[7] = b.w;
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) cols[k] = -1;
  }
}

__device__ __forceinline__ int log2_pow2(int x) { return 31 - __clz(x); }

// eight ELL slots of A from q (a multiple of 8) with their values in the iterate's type
// (float32 copy on the mixed path, float64 otherwise): 16-byte loads, no conversion
template <typename T>
__device__ __forceinline__ void ell_chunk(const Csr& A, int64_t q, int (&cols)[8], T (&vals)[8]) {
  const int4 a = *(const int4*)(A.ecol + q);
  const int4 b = *(const int4*)(A.ecol + q + 4);
  cols[0] = a.x; cols[1] = a.y; cols[2] = a.z; cols[3] = a.w;
  cols[4] = b.x; cols[5] = b.y; cols[6] = b.z; cols[7] = b.w;
  if constexpr (sizeof(T) == 4) {
    const float4 u = *(const float4*)(A.eval32 + q);
    const float4 v = *(const float4*)(A.eval32 + q + 4);
    vals[0] = u.x; vals[1] = u.y; vals[2] = u.z; vals[3] = u.w;
    vals[4] = v.x; vals[5] = v.y; vals[6] = v.z; vals[7] = v.w;
  } else {
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
      const double2 v = *(const double2*)(A.eval + q + k);
      vals[k] = v.x;
      vals[k + 1] = v.y;
    }
  }
}

// CSR only: degree prefix of the rows rows[0..cnt): pre[e] = sum_{f<=e} deg(rows[f]),
// and the row starts rs[e] = rowptr[rows[e]].  Returns the total.
__device__ inline int degree_prefix(const Csr& A, const int* rows, int cnt, int* pre,
                                    int64_t* rs) {
  const int lane = lane_id();
  int run = 0;
  for (int base = 0; base < cnt; base += SPAI_WAVE) {
    const int e = base + lane;
    int d = 0;
    if (e < cnt) {
      const int l = rows[e];
      const int64_t q0 = A.rowptr[l];
      d = (int)(A.rowptr[l + 1] - q0);
      rs[e] = q0;
    }
    const int inc = wave_incl_scan(d);
    if (e < cnt) pre[e] = run + inc;
    run += __shfl(inc, SPAI_WAVE - 1, SPAI_WAVE);
  }
  return run;
}

// Insert into the key set the column index of every nonzero of the rows rows[0..cnt)
// of A, four products per lane per batch, the loads of a batch in flight together.
// In ELL the products are the cnt << eshift slots (padding skipped); in CSR they are
// numbered through the degree prefix (pre, rs, total from degree_prefix).  `have` is
// the number of distinct keys already in the set; after every batch the count (a wave
// sum of the slots claimed) is compared with `limit`, and insertion stops once it is
// exceeded.  With limit + 256 < H the table is never full, so probing terminates.
// Returns the distinct count (> limit: the set outgrew the tile).
__device__ inline int insert_products(const Csr& A, const int* rows, int cnt, const int* pre,
                                      const int64_t* rs, int total, int* keys, int H, int have,
                                      int limit) {
  constexpr int U = 4;
  const bool ell = A.eshift >= 0;
  const int sh = A.eshift;
  const int wm = ell ? (1 << sh) - 1 : 0;
  const int tot = ell ? (cnt << sh) : total;
  int count = have;
  for (int p0 = 0; p0 < tot; p0 += SPAI_WAVE * U) {
    int cols[U];
#pragma unroll
    for (int c = 0; c < U; ++c) {
      const int p = p0 + c * SPAI_WAVE + lane_id();
      cols[c] = -1;
      if (p < tot) {
        if (ell) {
          cols[c] = A.ecol[((int64_t)rows[p >> sh] << sh) + (p & wm)];
        } else {
          const int e = upper_bound_int(pre, cnt, p);
          const int before = e ? pre[e - 1] : 0;
          cols[c] = A.col[rs[e] + (p - before)];
        }
      }
    }
    count += wave_sum_int(ks_insert_batch<U>(keys, H, cols));
    if (count > limit) break;
  }
  return count;
}

// Eight entries of A's row storage from slot q (q < qe; the row ends at qe), loaded
// together: cols[k] = -1 where there is no entry.  ELL chunks are aligned 32-byte
// pieces of the padded row.
__device__ __forceinline__ void load_chunk(const Csr& A, int64_t q, int64_t qe, int (&cols)[8],
                                           double (&vals)[8]) {
  if (A.eshift >= 0) {
    const int4 c0 = *(const int4*)(A.ecol + q);
    const int4 c1 = *(const int4*)(A.ecol + q + 4);
    cols[0] = c0.x; cols[1] = c0.y; cols[2] = c0.z; cols[3] = c0.w;
    cols[4] = c1.x; cols[5] = c1.y; cols[6] = c1.z; cols[7] = c1.w;
    if (A.eval32) {
      const float4 v0 = *(const float4*)(A.eval32 + q);
      const float4 v1 = *(const float4*)(A.eval32 + q + 4);
      vals[0] = v0.x; vals[1] = v0.y; vals[2] = v0.z; vals[3] = v0.w;
      vals[4] = v1.x; vals[5] = v1.y; vals[6] = v1.z; vals[7] = v1.w;
    } else {
#pragma unroll
      for (int k = 0; k < 8; k += 2) {
        const double2 v = *(const double2*)(A.eval + q + k);
        vals[k] = v.x;
        vals[k + 1] = v.y;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cols[k] = -1;
      vals[k] = 0.0;
      if (q + k < qe) {
        cols[k] = A.col[q + k];
        vals[k] = aval(A, q + k);
      }
    }
  }
}

__device__ __forceinline__ void row_span(const Csr& A, int u, int64_t& q0, int64_t& q1) {
  if (A.eshift >= 0) {
    q0 = (int64_t)u << A.eshift;
    q1 = q0 + ((int64_t)1 << A.eshift);
  } else {
    q0 = A.rowptr[u];
    q1 = A.rowptr[u + 1];
  }
}

// Pull over the rows of A selected by sorted keys[0..nu): G keys per lane at a time,
// their first 8-entry chunks loaded together before any is used.  Row u is visited in
// ascending column order, chunk by chunk: init(c, t) before key keys[t] (slot c),
// chunk(c, cols, vals) per chunk (column -1: no entry), done(c, t) after it.
template <int G, typename FI, typename FC, typename FD>
__device__ __forceinline__ void pull_rows(const Csr& A, const int* keys, int nu, FI init,
                                          FC chunk, FD done) {
  const int lane = lane_id();
  for (int t0 = 0; t0 < nu; t0 += SPAI_WAVE * G) {
    int tt[G];
    int64_t qa[G], qb[G];
    int cols[G][8];
    double vals[G][8];
#pragma unroll
    for (int c = 0; c < G; ++c) {
      tt[c] = t0 + c * SPAI_WAVE + lane;
      qa[c] = qb[c] = 0;
      if (tt[c] < nu) row_span(A, keys[tt[c]], qa[c], qb[c]);
    }
#pragma unroll
    for (int c = 0; c < G; ++c) {
#pragma unroll
      for (int k = 0; k < 8; ++k) cols[c][k] = -1;
      if (qa[c] < qb[c]) load_chunk(A, qa[c], qb[c], cols[c], vals[c]);
    }
#pragma unroll
    for (int c = 0; c < G; ++c) {
      if (tt[c] >= nu) continue;
      init(c, tt[c]);
      chunk(c, cols[c], vals[c]);
      for (int64_t q = qa[c] + 8; q < qb[c] && cols[c][7] >= 0; q += 8) {
        load_chunk(A, q, qb[c], cols[c], vals[c]);
        chunk(c, cols[c], vals[c]);
      }
      done(c, tt[c]);
    }
  }
}

// a column that does not fit its tile: hand it to the next tier, or flag it after the last
__device__ inline void defer_column(int tier, BigList big, DevState* st, int64_t j) {
  if (lane_id() == 0) {
    if (tier == 0) big.list[atomicAdd(big.count, 1)] = (int)j;
    else if (tier == 1) big.list2[atomicAdd(big.count2, 1)] = (int)j;
    else atomicOr(&st->err, 1);
  }
}

// Barrier of a per-column kernel.  In the huge tier the working set is device memory
// and its hash tables are updated with atomics, which are performed in L2: the fence
// (device scope, so the acquire side invalidates L1) keeps later plain loads from
// reading stale L1 lines.
template <bool GS>
__device__ __forceinline__ void tile_sync() {
  if constexpr (GS) __threadfence();
  __syncthreads();
}

// working-set base of a per-column kernel: dynamic LDS, or (GS, the huge tier) this
// workgroup's slice of the device-memory scratch
template <bool GS>
__device__ __forceinline__ char* tile_base(char* smem, const BigList& big) {
  if constexpr (GS) return big.scratch + (int64_t)blockIdx.x * big.scratch_stride;
  else return smem;
}

// ============================================================================
// small utilities: exclusive scan, fixed-order reductions
// ============================================================================

// counters are cleared by a kernel, never by a memset node, so that the
// iteration sequence can be captured in a HIP graph
// the deferred-column counters of a tiered launch, both zeroed by one launch
__global__ void k_zero_counts(int* a, int* b) {
  *a = 0;
  *b = 0;
}

// clear the drop record (a kernel, not a memset node: the iteration may be captured)
__global__ void k_rec_clear(DevState* st, int next) {
  const int64_t total = (int64_t)st->rec_cap * kRec;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x)
    st->rec[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rec_i = -1;
    st->rec_next = next;
    st->floorM = st->floorP = 0.0;     // a restarted or restored run starts without floors
    st->belowM = st->belowP = 0;
    st->redo = 0;
  }
}
void launch_rec_clear(DevState* st, int next, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_clear, dim3(64), dim3(256), 0, s, st, next);
}

// the floor-free second pass: masked unless the first pass's floors were too high
__global__ void k_redo_begin(DevState* st) {
  st->saved_active = st->iter_active;
  st->iter_active = st->iter_active && st->redo;
  if (st->redo) {
    st->floorM = st->floorP = 0.0;
    st->belowM = st->belowP = 0;
  }
}
__global__ void k_redo_end(DevState* st) { st->iter_active = st->saved_active; }
// next iteration's floors: a fraction of this iteration's cuts (none without a cut)
__device__ void floor_next_body(DevState* st, int doM, int doP, double frac) {
  if (doM) {
    st->floorM = (st->rawM > 0.0 && isfinite(st->rawM)) ? frac * st->rawM : 0.0;
    st->belowM = 0;
  }
  if (doP) {
    st->floorP = (st->rawP > 0.0 && isfinite(st->rawP)) ? frac * st->rawP : 0.0;
    st->belowP = 0;
  }
  st->redo = 0;
}
void launch_redo_begin(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_redo_begin, dim3(1), dim3(1), 0, s, st);
}
void launch_redo_end(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_redo_end, dim3(1), dim3(1), 0, s, st);
}

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int64_t block_excl_scan_i64(int64_t v, int64_t* sh, int64_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < (int)blockDim.x; d <<= 1) {
    int64_t add = (t >= d) ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int64_t incl = sh[t];
  *total = sh[blockDim.x - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int64_t* in, int64_t* out,
                                                             int64_t n, int64_t* tile_sums) {
  __shared__ int64_t sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t loc[kScanItems];
  int64_t run = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t g = base + i;
    const int64_t v = g < n ? in[g] : 0;
    loc[i] = run;
    run += v;
  }
  int64_t tot;
  const int64_t off = block_excl_scan_i64(run, sh, &tot);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t g = base + i;
    if (g < n) out[g] = off + loc[i];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_sums(int64_t* tile_sums, int64_t ntiles,
                                                    int64_t* total) {
  __shared__ int64_t sh[1024];
  const int per = (int)((ntiles + 1023) / 1024);
  const int64_t b = (int64_t)threadIdx.x * per;
  int64_t run = 0;
  for (int i = 0; i < per; ++i)
    if (b + i < ntiles) run += tile_sums[b + i];
  int64_t tot;
  const int64_t off = block_excl_scan_i64(run, sh, &tot);
  int64_t acc = off;
  for (int i = 0; i < per; ++i)
    if (b + i < ntiles) {
      const int64_t v = tile_sums[b + i];
      tile_sums[b + i] = acc;
      acc += v;
    }
  if (threadIdx.x == 0 && total) *total = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int64_t* out, int64_t n,
                                                           const int64_t* tile_off) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int64_t add = tile_off[blockIdx.x];
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
    const int64_t g = base + i;
    if (g < n) out[g] += add;
  }
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void launch_scan(const int64_t* in, int64_t* out, int64_t* total, int64_t n, int64_t* tmp,
                 hipStream_t s) {
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in, out, n,
                     tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, tmp, ntiles, total);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, out, n, tmp);
}

// ---- fixed-order reduction of per-column partials ---------------------------
constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;

// one block per chunk of columns (single segment) or per segment (batched)
__global__ __launch_bounds__(kRedThreads) void k_reduce_chunks(const double* colpart, int nd,
                                                               int64_t n, int64_t chunk,
                                                               const int64_t* seg_beg,
                                                               double* out) {
  __shared__ double sh[kRedThreads];
  int64_t lo, hi;
  if (seg_beg) {
    lo = seg_beg[blockIdx.x];
    hi = seg_beg[blockIdx.x + 1];
  } else {
    lo = (int64_t)blockIdx.x * chunk;
    hi = lo + chunk < n ? lo + chunk : n;
  }
  // up to kRedNd partials per column summed together: a column's partials are adjacent, and
  // four columns' loads are in flight before any is added; each partial's sum takes the
  // columns in the order of one pass per partial (the results are those of that pass)
  constexpr int kRedNd = 8, kRedU = 4;
  double acc[kRedNd];
  const int nd0 = nd < kRedNd ? nd : kRedNd;
#pragma unroll
  for (int d = 0; d < kRedNd; ++d) acc[d] = 0.0;
  {
    int64_t j = lo + threadIdx.x;
    for (; j + (kRedU - 1) * kRedThreads < hi; j += kRedU * kRedThreads) {
      double v[kRedU][kRedNd];
#pragma unroll
      for (int u = 0; u < kRedU; ++u)
#pragma unroll
        for (int d = 0; d < kRedNd; ++d)
          if (d < nd0) v[u][d] = colpart[(j + u * kRedThreads) * nd + d];
#pragma unroll
      for (int u = 0; u < kRedU; ++u)
#pragma unroll
        for (int d = 0; d < kRedNd; ++d)
          if (d < nd0) acc[d] += v[u][d];
    }
    for (; j < hi; j += kRedThreads)
#pragma unroll
      for (int d = 0; d < kRedNd; ++d)
        if (d < nd0) acc[d] += colpart[j * nd + d];
  }
  for (int d = 0; d < nd; ++d) {
    double a = 0.0;
    if (d < kRedNd) {
#pragma unroll
      for (int e = 0; e < kRedNd; ++e)
        if (e == d) a = acc[e];
    } else {
      for (int64_t j = lo + threadIdx.x; j < hi; j += kRedThreads) a += colpart[j * nd + d];
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)blockIdx.x * nd + d] = sh[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double* part, int nd,
                                                              int nparts, double* out) {
  __shared__ double sh[kRedThreads];
  for (int d = 0; d < nd; ++d) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kRedThreads) acc += part[(int64_t)b * nd + d];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[d] = sh[0];
    __syncthreads();
  }
}

void launch_reduce(const double* colpart, int nd, int64_t n, const Seg& seg,
                   const int64_t* seg_beg, double* red, double* blockpart, hipStream_t s) {
  if (seg.nseg > 1) {
    hipLaunchKernelGGL(k_reduce_chunks, dim3(seg.nseg), dim3(kRedThreads), 0, s, colpart, nd, n,
                       (int64_t)0, seg_beg, red);
    return;
  }
  const int64_t chunk = (n + kRedBlocks - 1) / kRedBlocks;
  const int nb = (int)((n + chunk - 1) / chunk);
  hipLaunchKernelGGL(k_reduce_chunks, dim3(nb), dim3(kRedThreads), 0, s, colpart, nd, n, chunk,
                     (const int64_t*)nullptr, blockpart);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, s, blockpart, nd, nb, red);
}

// ============================================================================
// setup: traces, M_0 = c I
// ============================================================================

// per row k: a_kk and sum_l a_kl^2 (tr A and tr A^2 = ||A||_F^2 for symmetric A)
__global__ void k_trace_parts(Csr A, double* colpart) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= A.n) return;
  double d = 0.0, s2 = 0.0;
  for (int64_t q = A.rowptr[k]; q < A.rowptr[k + 1]; ++q) {
    const double v = A.val[q];
    if (A.col[q] == k) d = v;
    s2 += v * v;
  }
  colpart[2 * k] = d;
  colpart[2 * k + 1] = s2;
}

void launch_trace_parts(const Csr& A, double* colpart, hipStream_t s) {
  hipLaunchKernelGGL(k_trace_parts, dim3((unsigned)((A.n + 255) / 256)), dim3(256), 0, s, A,
                     colpart);
}

// c = tr A / tr A^2 per segment; segment bookkeeping
__global__ void k_init_state(Seg seg, const double* red_tr, const int64_t* seg_beg, int64_t n,
                             double* cvec, int method, DevState* st) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < seg.nseg) {
    SegState& g = seg.st[s];
    cvec[s] = red_tr[2 * s] / red_tr[2 * s + 1];
    const int64_t ns = seg_beg ? seg_beg[s + 1] - seg_beg[s] : n;
    g.inv_sqrt_n = 1.0 / sqrt((double)ns);
    g.rr = 0.0;
    g.last_resid = 0.0;
    for (int d = 0; d < kND; ++d) g.dots[d] = 0.0;
    g.coef[0] = g.coef[1] = g.coef[2] = g.coef[3] = 0.0;
    g.step1 = g.step2 = 0.0;
    g.iters = 0;
    g.stop = 0;
    g.status = 0;
    g.first = (method == kLOMR) ? 1 : 0;
    g.mr_fallbacks = 0;
  }
  if (s == 0) {
    st->any_active = 1;
    st->err = 0;
    st->curM = 0;
    st->curP = 0;
    st->iter_active = 1;
  }
}

void launch_init_state(const Seg& seg, const double* red_tr, const int64_t* seg_beg, int64_t n,
                       double* cvec, int method, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3((seg.nseg + 255) / 256), dim3(256), 0, s, seg, red_tr,
                     seg_beg, n, cvec, method, st);
}

template <typename T>
__global__ void k_init_m(int64_t n, Cols<T> M, const double* cvec, Seg seg) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  M.beg[j] = j;
  M.len[j] = 1;
  M.idx[j] = (int32_t)j;
  M.val[j] = (T)cvec[seg.segof(j)];
}

template <typename T>
void launch_init_m(int64_t n, Cols<T> M, const double* cvec, const Seg& seg, hipStream_t s) {
  hipLaunchKernelGGL(k_init_m<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, M, cvec,
                     seg);
}

template <typename T>
__global__ void k_zero_cols(int64_t n, Cols<T> X) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  X.beg[j] = 0;
  X.len[j] = 0;
}

template <typename T>
void launch_zero_cols(int64_t n, Cols<T> X, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_cols<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, X);
}

// ============================================================================
// R = I - A M (explicit residual, Section 6.2) with ||r_j||^2 per column
// ============================================================================

// upper bound of nnz(r_j): 1 + sum_{l in supp(m_j)} deg(l).  Eight lanes per column read
// its entries together (two per lane in flight) and add their degrees with shuffles: an
// integer sum, the same in any order.
constexpr int kBoundLanes = 8;
template <typename T>
__global__ __launch_bounds__(256) void k_bound_resid(Csr A, Pair<T> Mp, int64_t* ub, int64_t n,
                                                     const DevState* st) {
  if (!st->any_active) return;
  const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kBoundLanes;
  const int g = threadIdx.x % kBoundLanes;
  const Cols<T> M = Mp.now();
  long long s = 0;
  if (j < n) {
    const int64_t b = M.beg[j];
    const int lm = M.len[j];
    int e = g;
    for (; e + kBoundLanes < lm; e += 2 * kBoundLanes) {
      const int l0 = M.idx[b + e], l1 = M.idx[b + e + kBoundLanes];
      s += (A.rowptr[l0 + 1] - A.rowptr[l0]) + (A.rowptr[l1 + 1] - A.rowptr[l1]);
    }
    if (e < lm) {
      const int l = M.idx[b + e];
      s += A.rowptr[l + 1] - A.rowptr[l];
    }
  }
#pragma unroll
  for (int d = 1; d < kBoundLanes; d <<= 1) s += __shfl_xor(s, d, SPAI_WAVE);   // all lanes
  if (j < n && g == 0) ub[j] = 1 + s;
}

template <typename T>
void launch_bound_resid(const Csr& A, Pair<T> M, int64_t* ub, int64_t n, const DevState* st,
                        hipStream_t s) {
  const int64_t threads = n * kBoundLanes;
  hipLaunchKernelGGL(k_bound_resid<T>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, A,
                     M, ub, n, st);
}

// five waves per SIMD: measured faster than the compiler's own choice (four) for this
// kernel, with no spills
template <typename T, bool GS>
__global__ __launch_bounds__(SPAI_WAVE) __attribute__((amdgpu_waves_per_eu(5, 5))) void k_resid(Csr A, Pair<T> Mp, Cols<T> R,
                                                     const int64_t* off, const int64_t* total,
                                                     double* colnorm, int weighted, double* colrz,
                                                     BigList big, DevState* st, int tier, int L,
                                                     int H) {
  if (!st->any_active) return;
  extern __shared__ char smem[];
  const bool ell = A.eshift >= 0;
  Carve cv(tile_base<GS>(smem, big));
  int* s_mi = cv.take<int>(L);
  int* s_keys = cv.take<int>(H);         // hash set, then the sorted keys
  double* s_mv = cv.take<double>(L);
  int* s_mk = cv.take<int>(2 * L);       // position map of m_j's rows
  unsigned* s_mp = cv.take<unsigned>(2 * L);
  int* s_pre = ell ? nullptr : cv.take<int>(L);           // CSR: degree prefix
  int64_t* s_rs = ell ? nullptr : cv.take<int64_t>(L);    // CSR: row starts
  const int lane = lane_id();
  const Cols<T> M = Mp.now();
  const bool overflow = *total > R.cap;
  const int limit = H / 2 - 1;
  unsigned long long outcnt = 0;

  auto body = [&](int64_t j) {
    const int64_t mb = M.beg[j];
    const int lm = M.len[j];
    if (lm > L) {
      defer_column(tier, big, st, j);
      return;
    }
    if (overflow) {
      if (lane == 0) atomicOr(&st->err, 2);
      return;
    }
    const int hs = next_pow2(max(2 * lm, 64));
    ks_clear(s_keys, H);
    lm_clear(s_mk, s_mp, hs);
    tile_sync<GS>();
    for (int e = lane; e < lm; e += SPAI_WAVE) {
      const int i = M.idx[mb + e];
      s_mi[e] = i;
      s_mv[e] = (double)M.val[mb + e];
      lm_put(s_mk, s_mp, hs, i, 0, e);
    }
    tile_sync<GS>();
    int tot = 0;
    if (!ell) {
      tot = degree_prefix(A, s_mi, lm, s_pre, s_rs);
      tile_sync<GS>();
    }
    int kd[1] = {lane == 0 ? (int)j : -1};
    int nk = wave_sum_int(ks_insert_batch<1>(s_keys, H, kd));
    nk = insert_products(A, s_mi, lm, s_pre, s_rs, tot, s_keys, H, nk, limit);
    tile_sync<GS>();
    if (nk > limit) {               // more distinct rows than the tile holds
      defer_column(tier, big, st, j);
      tile_sync<GS>();
      return;
    }
    const int nu = ks_sort_inplace(s_keys, H);
    tile_sync<GS>();
    const int64_t ob = off[j];
    double acc = 0.0, acc_rz = 0.0;
    double sum[1];
    double diag[1];             // a_uu of the pulled row (the Pi weight is 1 / a_uu)
    int key[1];
    pull_rows<1>(
        A, s_keys, nu,
        [&](int c, int t) {
          sum[c] = 0.0;
          diag[c] = 0.0;
          key[c] = s_keys[t];
        },
        [&](int c, const int (&cols)[8], const double (&vals)[8]) {
          unsigned pw[8];
          lm_find<8>(s_mk, s_mp, hs, cols, pw);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const unsigned e = pw[k] & kNoPos;
            if (e != kNoPos) sum[c] += vals[k] * s_mv[e];
            if (cols[k] == key[c]) diag[c] = vals[k];
          }
        },
        [&](int c, int t) {
          const int u = key[c];
          const double r = ((u == (int)j) ? 1.0 : 0.0) - sum[c];
          const T rt = (T)r;
          T out = rt;
          if (weighted) {                   // Z = Pi R, Pi = D_A^{-1}
            const double pi = 1.0 / diag[c];
            out = (T)(pi * r);
            acc_rz += (double)rt * (double)out;
          }
          R.idx[ob + t] = u;
          R.val[ob + t] = out;
          acc += (double)rt * (double)rt;
        });
    acc = wave_sum(acc);
    if (weighted) acc_rz = wave_sum(acc_rz);
    if (lane == 0) {
      colnorm[j] = acc;
      if (weighted) colrz[j] = acc_rz;
      R.beg[j] = ob;
      R.len[j] = nu;
    }
    outcnt += (unsigned long long)nu;
    tile_sync<GS>();
  };

  if (tier == 0) {
    ColumnWalk w(A.n, blockIdx.x, gridDim.x);
    for (int64_t j = w.begin; j < w.end; j += w.step) body(j);
  } else if (tier == 1) {
    const int cnt = *big.count;
    for (int t = blockIdx.x; t < cnt; t += gridDim.x) body(big.list[t]);
  } else {
    const int cnt = *big.count2;
    for (int t = blockIdx.x; t < cnt; t += gridDim.x) body(big.list2[t]);
  }
  if (lane == 0 && tier == 0 && blockIdx.x < kCntSlots) st->cnt[6 * kCntSlots + blockIdx.x] += outcnt;
  if (lane == 0 && tier >= 1 && outcnt) atomicAdd(&st->cnt[6 * kCntSlots + kCntSlots - 1], outcnt);
}

// Lean resident tier of the residual (A in ELL): the same arithmetic and summation
// order as k_resid, with far fewer instructions per column.  Each lane holds one entry
// of m_j (up to L <= 128 entries, two per lane), enters it in the byte-table map and
// inserts the columns of its ELL row straight from 16-byte loads into the ordered key
// set, sized from the column's bound ub_j = off[j+1] - off[j]; the keys are then sorted
// by row (the stored order of R) and each pulled over A's row with branch-free lookups.
// A column that does not fit (list, key set, sort) goes to the next tier.  WT: the
// Pi-weighted form (weighted != 0), fixed at compile time so that the unweighted pull
// carries no diagonal tracking.
template <typename T, bool WT>
__global__ __launch_bounds__(SPAI_WAVE) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 5))) void k_resid_lean(Csr A, Pair<T> Mp, Cols<T> R,
                                                          const int64_t* off,
                                                          const int64_t* total, double* colnorm,
                                                          int weighted, double* colrz,
                                                          BigList big, DevState* st, int L,
                                                          int H) {
  if (!st->any_active) return;
  weighted = WT ? 1 : 0;
  // the map at fixed LDS addresses (their offsets fold into the reads), the key set behind
  __shared__ __align__(16) unsigned char cell[kBtCells];   // one list: a byte per cell
  __shared__ __align__(16) BtEnt<T> ent[128 + 1];
  extern __shared__ char smem[];
  Carve cv(smem);
  const int Lc = min(L, 128);             // two list entries per lane
  unsigned* kt = cv.take<unsigned>(max(H + kOhOver, 256));
  int* keys = (int*)kt;
  const int lane = lane_id();
  for (int i = lane; i < kBtCells / 4; i += SPAI_WAVE) ((unsigned*)cell)[i] = 0u;
  if (lane == 0) ent[0] = BtEnt<T>{kBtNone, (T)0};    // list 0's sentinel
  __syncthreads();
  const Cols<T> M = Mp.now();
  const int64_t ntot = *total;
  const bool overflow = ntot > R.cap;
  const int W = 1 << A.eshift;
  unsigned long long outcnt = 0;
  ColumnWalk w(A.n, blockIdx.x, gridDim.x);
  for (int64_t j = w.begin; j < w.end; j += w.step) {
    // the column's descriptors, all loaded before the first is used (one wait)
    const int lm = M.len[j];
    const int64_t mb = M.beg[j];
    const int64_t ob = off[j];
    const int64_t oe = j + 1 < A.n ? off[j + 1] : ntot;
    if (lm > Lc) {
      defer_column(0, big, st, j);
      continue;
    }
    if (overflow) {
      if (lane == 0) atomicOr(&st->err, 2);
      continue;
    }
    const int64_t ub = oe - ob;                  // >= distinct rows of r_j
    const int Hc = next_pow2((int)min<int64_t>(max<int64_t>(ub, 64), (int64_t)H));
    const int ksh = 32 - log2_pow2(Hc);
    const int kend = Hc + kOhOver;
    // both slots' loads unconditional (entry 0 where a lane has none), so they are in
    // flight together before the first LDS store waits on one
    int row[2], lst[2] = {0, 0}, pos[2];
    T val[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = lane + k * SPAI_WAVE;
      pos[k] = e;
      const int64_t q = e < lm ? mb + e : 0;
      row[k] = __builtin_nontemporal_load(&M.idx[q]);   // read once here (see R below)
      val[k] = __builtin_nontemporal_load(&M.val[q]);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = lane + k * SPAI_WAVE;
      if (e < lm) ent[e + 1] = BtEnt<T>{row[k], val[k]};
      else row[k] = -1;
    }
    for (int i = lane; i < kend; i += SPAI_WAVE) kt[i] = kOhEmpty;
    const int a = bt_build<2, 1>(cell, row, lst, pos);
    if (a < 0) {
      defer_column(0, big, st, j);
      continue;
    }
    const unsigned mul = bt_mul(a);
    bool ok = true;
    const int npass = lm > SPAI_WAVE ? 2 : 1;      // entries per lane in use
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k >= npass) break;
      int rr = row[k];
      for (int c = 0; c < W; c += 8) {
        int cols[8];
        ell_cols8(A, rr, c, cols);
        const int c0[4] = {cols[0], cols[1], cols[2], cols[3]};
        const int c1[4] = {cols[4], cols[5], cols[6], cols[7]};
        ok = oh_insert_batch<4>(kt, ksh, c0) && ok;
        ok = oh_insert_batch<4>(kt, ksh, c1) && ok;
        if (cols[7] < 0) rr = -1;                  // the row ended in this chunk
      }
    }
    {
      const int kd[1] = {lane == 0 ? (int)j : -1};
      ok = oh_insert_batch<1>(kt, ksh, kd) && ok;
    }
    const bool bad = __ballot(!ok) != 0ull;
    __syncthreads();
    int nu = bad ? 0 : oh_compact(kt, kend);
    __syncthreads();
    if (bad || nu > 256) {                         // key set or register sort too small
      bt_clear<2, 1>(cell, row, lst, mul);
      __syncthreads();
      defer_column(0, big, st, j);
      continue;
    }
    // rows ascending (the stored order of R)
    if (nu <= 64) sort_in_registers<1>(keys, nu);
    else if (nu <= 128) sort_in_registers<2>(keys, nu);
    else sort_in_registers<4>(keys, nu);
    __syncthreads();
    double acc = 0.0, acc_rz = 0.0;
    for (int t0 = 0; t0 < nu; t0 += SPAI_WAVE) {
      const int t = t0 + lane;
      if (t < nu) {
        const int u = keys[t];
        const int64_t q0 = (int64_t)u << A.eshift;
        double sum = 0.0, diag = 0.0;
        for (int c = 0; c < W; c += 8) {
          int cols[8];
          T vals[8];
          ell_chunk<T>(A, q0 + c, cols, vals);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            bool h0;
            T x0;
            bt_find1<T>(cell, mul, ent, cols[k], h0, x0);
            // a masked product adds +-0 to a sum that is never -0: bitwise the skip
            sum += (double)vals[k] * bt_masked<T>(h0, x0);
            if (weighted && cols[k] == u) diag = (double)vals[k];
          }
          if (cols[7] < 0) break;
        }
        const double r = ((u == (int)j) ? 1.0 : 0.0) - sum;
        const T rt = (T)r;
        T out = rt;
        if (weighted) {                   // Z = Pi R, Pi = D_A^{-1}
          const double pi = 1.0 / diag;
          out = (T)(pi * r);
          acc_rz += (double)rt * (double)out;
        }
        // stored nontemporally: R is read again only in the next iteration, and the
        // column's own entries of M are loaded so, which keeps the rows of A this kernel
        // gathers in the caches
        __builtin_nontemporal_store(u, &R.idx[ob + t]);
        __builtin_nontemporal_store(out, &R.val[ob + t]);
        acc += (double)rt * (double)rt;
      }
    }
    acc = wave_sum(acc);
    if (weighted) acc_rz = wave_sum(acc_rz);
    if (lane == 0) {
      colnorm[j] = acc;
      if (weighted) colrz[j] = acc_rz;
      R.beg[j] = ob;
      R.len[j] = nu;
    }
    outcnt += (unsigned long long)nu;
    bt_clear<2, 1>(cell, row, lst, mul);
    __syncthreads();
  }
  if (lane == 0 && blockIdx.x < kCntSlots) st->cnt[6 * kCntSlots + blockIdx.x] += outcnt;
}

// resident workgroups of the lean residual per compute unit at most: at 96^3 the mixed
// path took 1.44 ms with 21 and 1.86 ms with the 24 its LDS allows
constexpr int kResidLeanPerCu = 21;

template <typename T>
static size_t resid_lean_lds(Tile t) {   // dynamic part (the map is static)
  return (size_t)std::max(t.H + kOhOver, 256) * 4 + 64;
}

static size_t resid_lds(Tile t, bool ell) {
  return (size_t)t.L * 4 + (size_t)t.H * 4 + (size_t)t.L * 8 + (size_t)t.L * 16 +
         (ell ? 0 : (size_t)t.L * 12) + 64;
}

int g_grid_cols = 2048;   // fallback persistent grid of the per-column kernels

// Persistent grid for a per-column kernel: as many one-wave workgroups as can be
// resident at once given its LDS tile (queried once per kernel and tile), rounded
// down to a multiple of the 8 XCDs.
template <typename K>
static int resident_grid(K kernel, size_t lds, int threads = SPAI_WAVE) {
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_pair((const void*)kernel, lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int dev = 0, cus = 0, per = 0;
  int grid = g_grid_cols;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, lds) == hipSuccess &&
      per > 0 && cus > 0) {
    // The query counts a workgroup's static and dynamic LDS but not the 512-byte granule
    // the hardware allocates it in: with 8,528 bytes it reports 19 workgroups per compute
    // unit where 18 fit, and the 19th starts only once another has finished (1.5x the
    // time of a persistent kernel).  Cap by the rounded size.
    hipFuncAttributes fa;
    int lds_cu = 0;
    if (hipFuncGetAttributes(&fa, (const void*)kernel) == hipSuccess &&
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
            hipSuccess &&
        lds_cu > 0) {
      const size_t need = (fa.sharedSizeBytes + lds + 511) / 512 * 512;
      if (need > 0) per = std::max(1, std::min<int>(per, (int)((size_t)lds_cu / need)));
    } else {
      (void)hipGetLastError();
    }
    grid = std::max(8, (per * cus) / 8 * 8);
  } else {
    (void)hipGetLastError();
  }
  cache[key] = grid;
  return grid;
}

// `per` workgroups per compute unit of the current device
static int per_cu_grid(int per) {
  static std::mutex mu;
  static int cus = 0;
  std::lock_guard<std::mutex> lock(mu);
  if (cus <= 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0) {
      (void)hipGetLastError();
      cus = 0;
      return g_grid_cols;
    }
  }
  return per * cus;
}


template <typename T>
void launch_resid(const Csr& A, Pair<T> M, Cols<T> R, const int64_t* off, const int64_t* total,
                  double* colnorm, int weighted, double* colrz, BigList big, DevState* st,
                  Tile small, Tile large, Tile huge, hipStream_t s) {
  const bool ell = A.eshift >= 0;
  hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(1), 0, s, big.count, big.count2);
  if (ell) {
    auto go = [&](auto KR) {
      hipLaunchKernelGGL((KR),
                         dim3(std::min(resident_grid(KR, resid_lean_lds<T>(small)),
                                       per_cu_grid(kResidLeanPerCu))),
                         dim3(SPAI_WAVE), resid_lean_lds<T>(small), s, A, M, R, off, total, colnorm,
                         weighted, colrz, big, st, small.L, small.H);
    };
    if (weighted) go(k_resid_lean<T, true>);
    else go(k_resid_lean<T, false>);
  } else
    hipLaunchKernelGGL((k_resid<T, false>),
                       dim3(resident_grid(k_resid<T, false>, resid_lds(small, ell))),
                       dim3(SPAI_WAVE), resid_lds(small, ell), s, A, M, R, off, total, colnorm,
                       weighted, colrz, big, st, 0, small.L, small.H);
  hipLaunchKernelGGL((k_resid<T, false>), dim3(256), dim3(SPAI_WAVE), resid_lds(large, ell), s, A, M,
                     R, off, total, colnorm, weighted, colrz, big, st, 1, large.L, large.H);
  hipLaunchKernelGGL((k_resid<T, true>), dim3(big.grid2), dim3(SPAI_WAVE), 0, s, A, M, R, off, total,
                     colnorm, weighted, colrz, big, st, 2, huge.L, huge.H);
}

// LDS of the lean tiers' static map (cells, entries with two sentinels, FP64 values)
constexpr size_t kLeanMapBytes = (size_t)kBtCells * 2 + (size_t)130 * sizeof(BtEnt<double>);

size_t resid_tile_bytes(Tile t, bool ell) {
  return ell ? std::max(resid_lds(t, ell), kLeanMapBytes + resid_lean_lds<double>(t))
             : resid_lds(t, ell);
}

// ============================================================================
// SpGEMM fused with Frobenius dots: A r_j and A p_j in LDS, never stored
// ============================================================================

template <typename T, bool GS>
__device__ __forceinline__ void dots_body(Csr A, Cols<T> R, Pair<T> Pp, int useR, int useP,
                                          int weighted, double* colpart, BigList big,
                                          DevState* st, int tier, int L, int H) {
  if (!st->any_active || !st->iter_active) return;
  extern __shared__ char smem[];
  const bool ell = A.eshift >= 0;
  Carve cv(tile_base<GS>(smem, big));
  int* s_li = cv.take<int>(L);           // r_j rows, then p_j rows
  int* s_keys = cv.take<int>(H);
  double* s_lv = cv.take<double>(L);
  int* s_mk = cv.take<int>(2 * L);       // position map: row -> (place in r_j, in p_j)
  unsigned* s_mp = cv.take<unsigned>(2 * L);
  int* s_pre = ell ? nullptr : cv.take<int>(L);
  int64_t* s_rs = ell ? nullptr : cv.take<int64_t>(L);
  const int lane = lane_id();
  const Cols<T> P = Pp.now();
  const int limit = H / 2 - 1;

  auto body = [&](int64_t j) {
    const int lr = useR ? R.len[j] : 0;
    const int lp = useP ? P.len[j] : 0;
    if (lr + lp > L) {
      defer_column(tier, big, st, j);
      return;
    }
    const int64_t rb = useR ? R.beg[j] : 0;
    const int64_t pb = useP ? P.beg[j] : 0;
    const int hs = next_pow2(max(2 * (lr + lp), 64));
    ks_clear(s_keys, H);
    lm_clear(s_mk, s_mp, hs);
    tile_sync<GS>();
    for (int e = lane; e < lr + lp; e += SPAI_WAVE) {   // both lists in one pass
      int i;
      double v;
      if (e < lr) {
        i = R.idx[rb + e];
        v = (double)R.val[rb + e];
      } else {
        i = P.idx[pb + e - lr];
        v = (double)P.val[pb + e - lr];
      }
      s_li[e] = i;
      s_lv[e] = v;
      lm_put(s_mk, s_mp, hs, i, e < lr ? 0 : 1, e < lr ? e : e - lr);
    }
    tile_sync<GS>();
    int tot = 0;
    if (!ell) {
      tot = degree_prefix(A, s_li, lr + lp, s_pre, s_rs);
      tile_sync<GS>();
    }
    const int nk = insert_products(A, s_li, lr + lp, s_pre, s_rs, tot, s_keys, H, 0, limit);
    tile_sync<GS>();
    if (nk > limit) {
      defer_column(tier, big, st, j);
      tile_sync<GS>();
      return;
    }
    const int nu = ks_sort_inplace(s_keys, H, true);   // ordered by ohash, as the lean tier
    tile_sync<GS>();
    const int* ri = s_li;
    const double* rv = s_lv;
    const int* pi = s_li + lr;
    const double* pv = s_lv + lr;
    double d0 = 0, d1 = 0, d2 = 0, d3 = 0, d4 = 0, d5 = 0;
    double ar[1], ap[1], diag[1];
    int key[1];
    pull_rows<1>(
        A, s_keys, nu,
        [&](int c, int t) {
          ar[c] = 0.0;
          ap[c] = 0.0;
          diag[c] = 0.0;
          key[c] = s_keys[t];
        },
        [&](int c, const int (&cols)[8], const double (&vals)[8]) {
          unsigned pw[8];
          lm_find<8>(s_mk, s_mp, hs, cols, pw);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const unsigned e0 = pw[k] & kNoPos, e1 = pw[k] >> 16;
            // fused multiply-add of the masked value: bitwise the lean tier's sum
            ar[c] = fma(vals[k], e0 != kNoPos ? rv[e0] : 0.0, ar[c]);
            ap[c] = fma(vals[k], e1 != kNoPos ? pv[e1] : 0.0, ap[c]);
            if (cols[k] == key[c]) diag[c] = vals[k];
          }
        },
        [&](int c, int t) {
          const int kk[1] = {key[c]};
          unsigned pw[1];
          lm_find<1>(s_mk, s_mp, hs, kk, pw);
          const unsigned e0 = pw[0] & kNoPos, e1 = pw[0] >> 16;
          const double ru = e0 != kNoPos ? rv[e0] : 0.0;
          const double pu = e1 != kNoPos ? pv[e1] : 0.0;
          d0 += ru * ar[c];
          d3 += ru * ap[c];
          d5 += pu * ap[c];
          if (weighted) {            // (AZ, Pi AZ), (AZ, Pi AP), (AP, Pi AP), Pi = D_A^{-1}
            const double pi = 1.0 / diag[c];
            d1 += ar[c] * (pi * ar[c]);
            d2 += ar[c] * (pi * ap[c]);
            d4 += ap[c] * (pi * ap[c]);
          } else {
            d1 += ar[c] * ar[c];
            d2 += ar[c] * ap[c];
            d4 += ap[c] * ap[c];
          }
        });
    (void)ri;
    (void)pi;
    double dd[6] = {d0, d1, d2, d3, d4, d5};
    wave_sum6(dd);
    if (lane == 0) {
      double* o = colpart + j * kND;
      o[0] = dd[0]; o[1] = dd[1]; o[2] = dd[2]; o[3] = dd[3]; o[4] = dd[4]; o[5] = dd[5];
    }
    tile_sync<GS>();
  };

  if (tier == 0) {
    ColumnWalk w(A.n, blockIdx.x, gridDim.x);
    for (int64_t j = w.begin; j < w.end; j += w.step) body(j);
  } else if (tier == 1) {
    const int cnt = *big.count;
    for (int t = blockIdx.x; t < cnt; t += gridDim.x) body(big.list[t]);
  } else {
    const int cnt = *big.count2;
    for (int t = blockIdx.x; t < cnt; t += gridDim.x) body(big.list2[t]);
  }
}

template <typename T, bool GS>
__global__ __launch_bounds__(SPAI_WAVE) void k_dots(Csr A, Cols<T> R, Pair<T> Pp, int useR,
                                                    int useP, int weighted, double* colpart,
                                                    BigList big, DevState* st, int tier, int L,
                                                    int H) {
  dots_body<T, GS>(A, R, Pp, useR, useP, weighted, colpart, big, st, tier, L, H);
}

// The resident tier with registers capped at five waves per SIMD (spills): slower on
// large columns, faster on small ones; a tuning candidate like k_update_w5.
template <typename T>
__global__ __launch_bounds__(SPAI_WAVE) __attribute__((amdgpu_waves_per_eu(5, 5))) void k_dots_w5(
    Csr A, Cols<T> R, Pair<T> Pp, int useR, int useP, int weighted, double* colpart, BigList big,
    DevState* st, int tier, int L, int H) {
  dots_body<T, false>(A, R, Pp, useR, useP, weighted, colpart, big, st, tier, L, H);
}

// Lean resident tier of the dots (A in ELL).  Each lane holds up to two entries of
// r_j | p_j (L <= 128 in all), enters them in the byte-table map and inserts the columns
// of their ELL rows into the ordered key set straight from 16-byte loads.  The ordered
// set needs no count (a walk off its end sends the column to the next tier) and no sort:
// its slots read in order list the rows of A r_j and A p_j sorted by ohash, the order
// every tier sums in.  Per row u, one pass over A's row gives (A r)_u, (A p)_u, r_u, p_u
// (the diagonal entry's lookup) and a_uu, with the same arithmetic as dots_body.
// Registers are capped for five waves per SIMD (no spills at that cap).  WT: the
// Pi-weighted form, fixed at compile time (as in k_resid_lean).
template <typename T, bool WT>
__global__ __launch_bounds__(SPAI_WAVE) __attribute__((amdgpu_waves_per_eu(5))) void k_dots_lean(Csr A, Cols<T> R, Pair<T> Pp, int useR,
                                                         int useP, int weighted,
                                                         double* colpart, BigList big,
                                                         DevState* st, int L, int H) {
  if (!st->any_active || !st->iter_active) return;
  weighted = WT ? 1 : 0;
  // the map at fixed LDS addresses (their offsets fold into the reads), the key set behind
  __shared__ __align__(16) unsigned short cell[kBtCells];
  __shared__ __align__(16) BtEnt<T> ent[128 + 2];   // two sentinels
  extern __shared__ char smem[];
  Carve cv(smem);
  const int Lc = min(L, 128);
  unsigned* kt = cv.take<unsigned>(H + kOhOver);
  const int lane = lane_id();
  for (int i = lane; i < kBtCells / 2; i += SPAI_WAVE) ((unsigned*)cell)[i] = 0u;
  if (lane == 0) ent[0] = BtEnt<T>{kBtNone, (T)0};    // list 0's sentinel
  __syncthreads();
  const Cols<T> P = Pp.now();
  const int W = 1 << A.eshift;
  ColumnWalk w(A.n, blockIdx.x, gridDim.x);
  for (int64_t j = w.begin; j < w.end; j += w.step) {
    // the column's descriptors, all loaded before the first is used (one wait; both
    // lists have their n descriptors whether in use or not)
    const int lr0 = R.len[j], lp0 = P.len[j];
    const int64_t rb = R.beg[j], pb = P.beg[j];
    const int lr = useR ? lr0 : 0;
    const int lp = useP ? lp0 : 0;
    const int le = lr + lp;
    if (le > Lc) {
      defer_column(0, big, st, j);
      continue;
    }
    const int Hc = min(H, max(128, next_pow2(max(le * W / 2, 1))));   // home slots
    const int ksh = 32 - log2_pow2(Hc);
    const int kend = Hc + kOhOver;
    // both slots' loads unconditional, from the list the lane's entry lies in (entry 0
    // of R where a lane has none), so they are in flight together before the first LDS
    // store waits on one
    int row[2], lst[2], pos[2];
    T val[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = lane + k * SPAI_WAVE;
      const bool isr = e < lr;
      lst[k] = isr ? 0 : 1;
      pos[k] = isr ? e : e - lr;
      const int* ip = (isr || e >= le) ? R.idx : P.idx;
      const T* vp = (isr || e >= le) ? R.val : P.val;
      const int64_t q = isr ? rb + e : (e < le ? pb + (e - lr) : 0);
      row[k] = ip[q];
      val[k] = vp[q];
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = lane + k * SPAI_WAVE;
      if (e < le) ent[e + 1 + (e >= lr)] = BtEnt<T>{row[k], val[k]};
      else row[k] = -1;
    }
    if (lane == 0) ent[lr + 1] = BtEnt<T>{kBtNone, (T)0};   // list 1's sentinel
    const BtEnt<T>* ent1 = ent + lr + 1;
    for (int i = lane; i < kend; i += SPAI_WAVE) kt[i] = kOhEmpty;
    const int a = bt_build<2>((unsigned char*)cell, row, lst, pos);
    if (a < 0) {
      defer_column(0, big, st, j);
      continue;
    }
    const unsigned mul = bt_mul(a);
    bool ok = true;
    const int npass = le > SPAI_WAVE ? 2 : 1;      // entries per lane in use
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k >= npass) break;
      int rr = row[k];
      for (int c = 0; c < W; c += 8) {
        int cols[8];
        ell_cols8(A, rr, c, cols);
        const int c0[4] = {cols[0], cols[1], cols[2], cols[3]};
        const int c1[4] = {cols[4], cols[5], cols[6], cols[7]};
        ok = oh_insert_batch<4>(kt, ksh, c0) && ok;
        ok = oh_insert_batch<4>(kt, ksh, c1) && ok;
        if (cols[7] < 0) rr = -1;
      }
    }
    const bool bad = __ballot(!ok) != 0ull;
    __syncthreads();
    if (bad) {
      bt_clear<2>((unsigned char*)cell, row, lst, mul);
      __syncthreads();
      defer_column(0, big, st, j);
      continue;
    }
    const int nu = oh_compact(kt, kend);
    __syncthreads();
    const int* keys = (const int*)kt;
    double d[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // KP keys per lane per pass (t, t + 64, ...; two on the float path, whose registers
    // allow it), all their rows of A loaded before any is used; each key's sum runs over
    // its row as with one key per pass and the partials take the keys in the same order
    constexpr int KP = sizeof(T) == 4 ? 2 : 1;
    for (int t0 = 0; t0 < nu; t0 += KP * SPAI_WAVE) {
      int uk[KP];
      bool live[KP], has[KP];
      double ar[KP], ap[KP], dg[KP];
#pragma unroll
      for (int h = 0; h < KP; ++h) {
        ar[h] = 0.0;
        ap[h] = 0.0;
        dg[h] = 0.0;
        const int t = t0 + h * SPAI_WAVE + lane;
        uk[h] = t < nu ? keys[t] : -1;
        live[h] = uk[h] >= 0;
        has[h] = live[h];
      }
      for (int c = 0; c < W; c += 8) {
        int cols[KP][8];
        T vals[KP][8];
#pragma unroll
        for (int h = 0; h < KP; ++h)               // a lane without a key reads row 0
          ell_chunk<T>(A, ((int64_t)(live[h] ? uk[h] : 0) << A.eshift) + c, cols[h], vals[h]);
#pragma unroll
        for (int h = 0; h < KP; ++h) {
          if (!live[h]) continue;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            bool h0, h1;
            T x0, x1;
            bt_find<T>(cell, mul, ent, ent1, cols[h][k], h0, x0, h1, x1);
            const double av = (double)vals[h][k];
            ar[h] = fma(av, bt_masked<T>(h0, x0), ar[h]);
            ap[h] = fma(av, bt_masked<T>(h1, x1), ap[h]);
            if (weighted && cols[h][k] == uk[h]) dg[h] = av;
          }
          if (cols[h][7] < 0) live[h] = false;     // the row ended in this chunk
        }
        bool any = false;
#pragma unroll
        for (int h = 0; h < KP; ++h) any = any || live[h];
        if (!any) break;
      }
#pragma unroll
      for (int h = 0; h < KP; ++h) {
        if (!has[h]) continue;
        double ru, pu;                 // u's own entries in r_j and p_j
        {
          bool h0, h1;
          T x0, x1;
          bt_find<T>(cell, mul, ent, ent1, uk[h], h0, x0, h1, x1);
          ru = h0 ? (double)x0 : 0.0;
          pu = h1 ? (double)x1 : 0.0;
        }
        d[0] += ru * ar[h];
        d[3] += ru * ap[h];
        d[5] += pu * ap[h];
        if (weighted) {            // (AZ, Pi AZ), (AZ, Pi AP), (AP, Pi AP), Pi = D_A^{-1}
          const double pi = 1.0 / dg[h];
          d[1] += ar[h] * (pi * ar[h]);
          d[2] += ar[h] * (pi * ap[h]);
          d[4] += ap[h] * (pi * ap[h]);
        } else {
          d[1] += ar[h] * ar[h];
          d[2] += ar[h] * ap[h];
          d[4] += ap[h] * ap[h];
        }
      }
    }
    wave_sum6(d);
    if (lane == 0) {
      double* o = colpart + j * kND;
      o[0] = d[0]; o[1] = d[1]; o[2] = d[2]; o[3] = d[3]; o[4] = d[4]; o[5] = d[5];
    }
    bt_clear<2>((unsigned char*)cell, row, lst, mul);
    __syncthreads();
  }
}

template <typename T>
static size_t dots_lean_lds(Tile t) {    // dynamic part (the map is static)
  return (size_t)(t.H + kOhOver) * 4 + 64;
}

static size_t dots_lds(Tile t, bool ell) {
  return (size_t)t.L * 4 + (size_t)t.H * 4 + (size_t)t.L * 8 + (size_t)t.L * 16 +
         (ell ? 0 : (size_t)t.L * 12) + 64;
}

template <typename T>
void launch_dots(const Csr& A, Cols<T> R, Pair<T> P, int useR, int useP, int weighted,
                 double* colpart, BigList big, DevState* st, Tile small, Tile large, Tile huge,
                 hipStream_t s) {
  const bool ell = A.eshift >= 0;
  hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(1), 0, s, big.count, big.count2);
  if (small.waves == 1 && ell) {
    auto go = [&](auto KD) {
      hipLaunchKernelGGL((KD), dim3(resident_grid(KD, dots_lean_lds<T>(small))),
                         dim3(SPAI_WAVE), dots_lean_lds<T>(small), s, A, R, P, useR, useP, weighted,
                         colpart, big, st, small.L, small.H);
    };
    if (weighted) go(k_dots_lean<T, true>);
    else go(k_dots_lean<T, false>);
  } else if (small.waves == 5)
    hipLaunchKernelGGL((k_dots_w5<T>), dim3(resident_grid(k_dots_w5<T>, dots_lds(small, ell))),
                       dim3(SPAI_WAVE), dots_lds(small, ell), s, A, R, P, useR, useP, weighted,
                       colpart, big, st, 0, small.L, small.H);
  else
    hipLaunchKernelGGL((k_dots<T, false>),
                       dim3(resident_grid(k_dots<T, false>, dots_lds(small, ell))),
                       dim3(SPAI_WAVE), dots_lds(small, ell), s, A, R, P, useR, useP, weighted,
                       colpart, big, st, 0, small.L, small.H);
  hipLaunchKernelGGL((k_dots<T, false>), dim3(256), dim3(SPAI_WAVE), dots_lds(large, ell), s, A, R, P,
                     useR, useP, weighted, colpart, big, st, 1, large.L, large.H);
  hipLaunchKernelGGL((k_dots<T, true>), dim3(big.grid2), dim3(SPAI_WAVE), 0, s, A, R, P, useR, useP,
                     weighted, colpart, big, st, 2, huge.L, huge.H);
}

size_t dots_tile_bytes(Tile t, bool ell) {
  return (t.waves == 1 && ell) ? kLeanMapBytes + dots_lean_lds<double>(t) : dots_lds(t, ell);
}

// ============================================================================
// implicit residual update R_{i+1} = R_i - c A X_i (Algorithms 1, 3, 4 as printed,
// Section 6.2: valid only while nothing is dropped)
// ============================================================================
//
// X is R_i itself (MR, c = alpha), P_i (CG, c = alpha) or the new direction P_i =
// delta R_i + gamma P_{i-1} (LOMR, c = 1).  In the Pi-weighted forms the direction
// lists hold Z = Pi R, so R_i comes from its own buffer and Z_{i+1} is written beside
// R_{i+1}.  Output column j: supp(r_j) united with the rows reached from supp(x_j)
// through A, values r_uj - c sum_l a_ul x_lj (l ascending), written at off[j].

struct ImplSrc {
  int xsrc;      // 0: X is the direction-list buffer given as Xr, 1: X is P.now()
  int cidx;      // coefficient index into the segment's coef[], -1: c = 1
};

template <typename T>
__global__ void k_bound_impl(Csr A, Cols<T> Rin, Cols<T> Xr, Pair<T> Pp, ImplSrc src, int64_t* ub,
                             int64_t n, const DevState* st) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (!st->any_active || !st->iter_active) return;
  const Cols<T> X = src.xsrc ? Pp.now() : Xr;
  const int64_t b = X.beg[j];
  const int lx = X.len[j];
  int64_t s = Rin.len[j];
  for (int e = 0; e < lx; ++e) {
    const int l = X.idx[b + e];
    s += A.rowptr[l + 1] - A.rowptr[l];
  }
  ub[j] = s;
}

template <typename T>
void launch_bound_impl(const Csr& A, Cols<T> Rin, Cols<T> Xr, Pair<T> P, int xsrc, int64_t* ub,
                       int64_t n, const DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_bound_impl<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, Rin,
                     Xr, P, ImplSrc{xsrc, 0}, ub, n, st);
}

template <typename T, bool GS>
__global__ __launch_bounds__(SPAI_WAVE) void k_resid_impl(Csr A, Cols<T> Rin, Cols<T> Xr,
                                                          Pair<T> Pp, ImplSrc src, Seg seg,
                                                          const int64_t* off,
                                                          const int64_t* total, Cols<T> Rout,
                                                          Cols<T> Zout, int weighted,
                                                          double* colnorm, double* colrz,
                                                          BigList big, DevState* st, int tier,
                                                          int L, int H) {
  if (!st->any_active || !st->iter_active) return;
  extern __shared__ char smem[];
  const bool ell = A.eshift >= 0;
  Carve cv(tile_base<GS>(smem, big));
  int* s_li = cv.take<int>(L);           // r_j rows, then x_j rows
  int* s_keys = cv.take<int>(H);
  double* s_lv = cv.take<double>(L);
  int* s_mk = cv.take<int>(2 * L);       // position map: row -> (place in r_j, in x_j)
  unsigned* s_mp = cv.take<unsigned>(2 * L);
  int* s_pre = ell ? nullptr : cv.take<int>(L);
  int64_t* s_rs = ell ? nullptr : cv.take<int64_t>(L);
  const int lane = lane_id();
  const Cols<T> X = src.xsrc ? Pp.now() : Xr;
  const bool overflow = *total > Rout.cap;
  const int limit = H / 2 - 1;

  auto body = [&](int64_t j) {
    const int lr = Rin.len[j];
    const int lx = X.len[j];
    if (lr + lx > L) {
      defer_column(tier, big, st, j);
      return;
    }
    if (overflow) {
      if (lane == 0) atomicOr(&st->err, 2);
      return;
    }
    const SegState& g = seg.st[seg.segof(j)];
    // a stopped matrix of a batch keeps its residual
    const double c = g.stop ? 0.0 : (src.cidx < 0 ? 1.0 : g.coef[src.cidx]);
    const int64_t rb = Rin.beg[j];
    const int64_t xb = X.beg[j];
    const int hs = next_pow2(max(2 * (lr + lx), 64));
    ks_clear(s_keys, H);
    lm_clear(s_mk, s_mp, hs);
    tile_sync<GS>();
    for (int e = lane; e < lr + lx; e += SPAI_WAVE) {
      int i;
      double v;
      if (e < lr) {
        i = Rin.idx[rb + e];
        v = (double)Rin.val[rb + e];
      } else {
        i = X.idx[xb + e - lr];
        v = (double)X.val[xb + e - lr];
      }
      s_li[e] = i;
      s_lv[e] = v;
      lm_put(s_mk, s_mp, hs, i, e < lr ? 0 : 1, e < lr ? e : e - lr);
    }
    tile_sync<GS>();
    int nk = 0;
    for (int b0 = 0; b0 < lr; b0 += SPAI_WAVE) {           // supp(r_j)
      const int kd[1] = {b0 + lane < lr ? s_li[b0 + lane] : -1};
      nk += wave_sum_int(ks_insert_batch<1>(s_keys, H, kd));
    }
    int tot = 0;
    if (!ell) {
      tot = degree_prefix(A, s_li + lr, lx, s_pre, s_rs);
      tile_sync<GS>();
    }
    if (nk <= limit)
      nk = insert_products(A, s_li + lr, lx, s_pre, s_rs, tot, s_keys, H, nk, limit);
    tile_sync<GS>();
    if (nk > limit) {
      defer_column(tier, big, st, j);
      tile_sync<GS>();
      return;
    }
    const int nu = ks_sort_inplace(s_keys, H);
    tile_sync<GS>();
    const double* rv = s_lv;
    const double* xv = s_lv + lr;
    const int64_t ob = off[j];
    double acc = 0.0, acc_rz = 0.0;
    double ax[1], diag[1];
    int key[1];
    pull_rows<1>(
        A, s_keys, nu,
        [&](int cc, int t) {
          ax[cc] = 0.0;
          diag[cc] = 0.0;
          key[cc] = s_keys[t];
        },
        [&](int cc, const int (&cols)[8], const double (&vals)[8]) {
          unsigned pw[8];
          lm_find<8>(s_mk, s_mp, hs, cols, pw);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const unsigned e1 = pw[k] >> 16;
            if (e1 != kNoPos) ax[cc] += vals[k] * xv[e1];
            if (cols[k] == key[cc]) diag[cc] = vals[k];
          }
        },
        [&](int cc, int t) {
          const int kk[1] = {key[cc]};
          unsigned pw[1];
          lm_find<1>(s_mk, s_mp, hs, kk, pw);
          const unsigned e0 = pw[0] & kNoPos;
          const double ru = e0 != kNoPos ? rv[e0] : 0.0;
          const double r = ru - c * ax[cc];
          const T rt = (T)r;
          Rout.idx[ob + t] = key[cc];
          Rout.val[ob + t] = rt;
          acc += (double)rt * (double)rt;
          if (weighted) {                   // Z = Pi R, Pi = D_A^{-1}
            const T zt = (T)((1.0 / diag[cc]) * r);
            Zout.idx[ob + t] = key[cc];
            Zout.val[ob + t] = zt;
            acc_rz += (double)rt * (double)zt;
          }
        });
    acc = wave_sum(acc);
    if (weighted) acc_rz = wave_sum(acc_rz);
    if (lane == 0) {
      colnorm[j] = acc;
      Rout.beg[j] = ob;
      Rout.len[j] = nu;
      if (weighted) {
        colrz[j] = acc_rz;
        Zout.beg[j] = ob;
        Zout.len[j] = nu;
      }
    }
    tile_sync<GS>();
  };

  if (tier == 0) {
    ColumnWalk w(A.n, blockIdx.x, gridDim.x);
    for (int64_t j = w.begin; j < w.end; j += w.step) body(j);
  } else if (tier == 1) {
    const int cnt = *big.count;
    for (int t = blockIdx.x; t < cnt; t += gridDim.x) body(big.list[t]);
  } else {
    const int cnt = *big.count2;
    for (int t = blockIdx.x; t < cnt; t += gridDim.x) body(big.list2[t]);
  }
}

template <typename T>
void launch_resid_impl(const Csr& A, Cols<T> Rin, Cols<T> Xr, Pair<T> P, int xsrc, int cidx,
                       const Seg& seg, const int64_t* off, const int64_t* total, Cols<T> Rout,
                       Cols<T> Zout, int weighted, double* colnorm, double* colrz, BigList big,
                       DevState* st, Tile small, Tile large, Tile huge, hipStream_t s) {
  const bool ell = A.eshift >= 0;
  const ImplSrc src{xsrc, cidx};
  hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(1), 0, s, big.count, big.count2);
  hipLaunchKernelGGL((k_resid_impl<T, false>),
                     dim3(resident_grid(k_resid_impl<T, false>, dots_lds(small, ell))),
                     dim3(SPAI_WAVE), dots_lds(small, ell), s, A, Rin, Xr, P, src, seg, off, total,
                     Rout, Zout, weighted, colnorm, colrz, big, st, 0, small.L, small.H);
  hipLaunchKernelGGL((k_resid_impl<T, false>), dim3(256), dim3(SPAI_WAVE), dots_lds(large, ell), s,
                     A, Rin, Xr, P, src, seg, off, total, Rout, Zout, weighted, colnorm, colrz, big,
                     st, 1, large.L, large.H);
  hipLaunchKernelGGL((k_resid_impl<T, true>), dim3(big.grid2), dim3(SPAI_WAVE), 0, s, A, Rin, Xr,
                     P, src, seg, off, total, Rout, Zout, weighted, colnorm, colrz, big, st, 2,
                     huge.L, huge.H);
}

// dst := src for column lists laid out at the same offsets (entries [0, *total))
template <typename T>
__global__ void k_copy_cols(Cols<T> src, Cols<T> dst, int64_t n, const int64_t* total,
                            const DevState* st) {
  if (!st->any_active || !st->iter_active) return;
  // an overflowing total was flagged by the producer, which then wrote nothing
  const int64_t tot = min(*total, min(src.cap, dst.cap));
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot || q < n; q += stride) {
    if (q < n) {
      dst.beg[q] = src.beg[q];
      dst.len[q] = src.len[q];
    }
    if (q < tot) {
      dst.idx[q] = src.idx[q];
      dst.val[q] = src.val[q];
    }
  }
}

template <typename T>
void launch_copy_cols(Cols<T> src, Cols<T> dst, int64_t n, const int64_t* total,
                      const DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_cols<T>, dim3(2048), dim3(256), 0, s, src, dst, n, total, st);
}

// ============================================================================
// merge (SpGEAM) + symmetrize + small-entry drop + per-column thresholds
// ============================================================================
//
// Column j of the candidates:
//   x  = (m_j + a1 X1(:,j)) + a2 X2(:,j)           (M_i + alpha R_i, M_i + alpha P_i or
//                                                   M_i + delta R_i + gamma P_{i-1})
//   y  = (m_j + a1 X1^T(:,j)) + a2 X2^T(:,j)       (row j of the same sum)
//   M candidate = (x + y) / 2                      (Appendix A step 1)
//   P candidate = c1 R(:,j) + c2 P(:,j), and the same from R^T, P^T for P^T.
// R^T(:,j) = e_j - M a_j is recomputed from the neighbour columns m_l, l in N(j):
// with M and A exactly symmetric and both sums taken over l ascending, it equals
// the transposed R bitwise, so the symmetrized M is exactly symmetric and the P^T
// candidates are exactly the transposed P candidates.

// upper bound of the union of the lists of column j
template <typename T>
__global__ void k_bound_update(Csr A, Pair<T> Mp, Cols<T> R, Pair<T> Pp, Pair<T> PTp, UpdMode md,
                               int64_t* ub, int64_t n, const DevState* st) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (!st->any_active || !st->iter_active) return;
  const Cols<T> M = Mp.now();
  const Cols<T> P = Pp.now();
  const Cols<T> PT = PTp.now();
  const bool needR = (md.doM && (md.x1 == 1 || md.x2 == 1)) || (md.doP && md.pR);
  const bool needP = (md.doM && (md.x1 == 2 || md.x2 == 2)) || (md.doP && md.pP);
  const bool mirror = md.sym != 0;   // R^T, P^T serve only the symmetrization
  int64_t s = 1;
  if (md.doM) s += M.len[j];
  if (needR) s += R.len[j];
  if (needP) s += P.len[j];
  if (needP && mirror) s += PT.len[j];
  if (needR && mirror)
    for (int64_t q = A.rowptr[j]; q < A.rowptr[j + 1]; ++q) s += M.len[A.col[q]];
  ub[j] = s;
}

template <typename T>
void launch_bound_update(const Csr& A, Pair<T> M, Cols<T> R, Pair<T> P, Pair<T> PT, UpdMode md,
                         int64_t* ub, int64_t n, const DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_bound_update<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, M,
                     R, P, PT, md, ub, n, st);
}

// (b+1)-th largest magnitude of a candidate column in global memory (0 if it has at
// most b entries), skipping the entry with row `skip`; the same on all lanes.
// Up to 64 candidates: one per lane, loaded once, the others' magnitudes broadcast from
// their lanes (the same comparisons in the same order as the general loop below).
template <typename T>
__device__ inline double kth_largest_cols(const int32_t* idx, const T* val, int cnt, int skip,
                                          int b) {
  if (cnt <= SPAI_WAVE) {
    const int lane = lane_id();
    const bool have = lane < cnt;
    const bool use = have && idx[lane] != skip;
    const double x = have ? fabs((double)val[lane]) : 0.0;
    const unsigned long long um = __ballot(use);
    double t = 0.0;
    if (__popcll(um) > b) {
      int r = 0;
      for (int f = 0; f < cnt; ++f) {
        const double y = __shfl(x, f, SPAI_WAVE);
        if ((um >> f) & 1ull) r += (y > x) || (y == x && f < lane);
      }
      if (use && r == b) t = x;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) t = fmax(t, __shfl_xor(t, d, SPAI_WAVE));
    return t;
  }
  int m = 0;
  for (int e = lane_id(); e < cnt; e += SPAI_WAVE) m += idx[e] != skip;
  m = wave_sum_int(m);
  double t = 0.0;
  if (m > b) {
    for (int e = lane_id(); e < cnt; e += SPAI_WAVE) {
      if (idx[e] == skip) continue;
      const double x = fabs((double)val[e]);
      int r = 0;
      for (int f = 0; f < cnt; ++f) {
        if (idx[f] == skip) continue;
        const double y = fabs((double)val[f]);
        r += (y > x) || (y == x && f < e);
      }
      if (r == b) t = x;
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) t = fmax(t, __shfl_xor(t, d, SPAI_WAVE));
  return t;
}

template <typename T, bool GS>
__device__ __forceinline__ void update_body(Csr A, Pair<T> Mp, Cols<T> R, Pair<T> Pp,
                                            Pair<T> PTp, UpdMode md, const int64_t* off,
                                            const int64_t* total, const int32_t* kcol,
                                            double* tM, double* tP, BigList big, Seg seg,
                                            DevState* st, int tier, int L, int H, int DG) {
  if (!st->any_active || !st->iter_active) return;
  extern __shared__ char smem[];
  Carve cv(tile_base<GS>(smem, big));
  int* s_li = cv.take<int>(L);
  int* s_keys = cv.take<int>(H);        // hash set, then the sorted keys
  int* s_nbcol = cv.take<int>(DG);
  int* s_nboff = cv.take<int>(DG + 1);
  double* s_lv = cv.take<double>(L);
  double* s_nbval = cv.take<double>(DG);
  // small tile: the neighbour columns m_l sit in LDS; large tile: they stay in global
  // memory and are searched in place (s_nbbeg / s_nboff hold their start and length)
  const bool nb_lds = tier == 0;
  int64_t* s_nbbeg = cv.take<int64_t>(DG);
  const int lane = lane_id();

  const Cols<T> M = Mp.now();
  const Cols<T> Mo = Mp.nxt();
  const Cols<T> P = Pp.now();
  const Cols<T> Po = Pp.nxt();
  const Cols<T> PT = PTp.now();
  const Cols<T> PTo = PTp.nxt();
  const bool needR = (md.doM && (md.x1 == 1 || md.x2 == 1)) || (md.doP && md.pR);
  const bool needP = (md.doM && (md.x1 == 2 || md.x2 == 2)) || (md.doP && md.pP);
  const bool mirror = md.sym != 0;   // R^T, P^T serve only the symmetrization
  const bool needRT = needR && mirror;
  const bool needPT = needP && mirror;
  const bool overflow = *total > Mo.cap || (md.doP && (*total > Po.cap || *total > PTo.cap));

  const bool ell = A.eshift >= 0;
  const int limit = H / 2 - 1;

  auto body = [&](int64_t j) {
    const SegState& g = seg.st[seg.segof(j)];
    const double a1 = g.coef[0], a2 = g.coef[1], c1 = g.coef[2], c2 = g.coef[3];
    // ---- own lists: m_j | r_j | p_j | pT_j
    const int lm = md.doM ? M.len[j] : 0;
    const int lr = needR ? R.len[j] : 0;
    const int lp = needP ? P.len[j] : 0;
    const int lpt = needPT ? PT.len[j] : 0;
    const int64_t mb = md.doM ? M.beg[j] : 0;
    const int64_t rb = lr ? R.beg[j] : 0;
    const int64_t pb = lp ? P.beg[j] : 0;
    const int64_t ptb = lpt ? PT.beg[j] : 0;
    const int om = 0, orr = lm, op = lm + lr, opt = lm + lr + lp, onb = lm + lr + lp + lpt;
    // ---- neighbours l in N(j) (row j of A, for R^T): l, a_jl, where m_l sits, and the
    // offsets s_nboff of their entries after the own lists
    int64_t qa = 0;
    int deg = 0;
    if (needRT) {
      if (ell) {
        qa = (int64_t)j << A.eshift;
        const int c = lane < (1 << A.eshift) ? A.ecol[qa + lane] : -1;
        deg = __popcll(__ballot(c >= 0));
      } else {
        qa = A.rowptr[j];
        deg = (int)(A.rowptr[j + 1] - qa);
      }
    }
    if (deg > DG) {
      defer_column(tier, big, st, j);
      return;
    }
    int run = 0;
    double ajj = 0.0;                 // a_jj (Pi-weighted variants: Pi_jj = 1 / a_jj)
    for (int base = 0; base < deg; base += SPAI_WAVE) {
      const int t = base + lane;
      int len = 0;
      int l = -1;
      double av = 0.0;
      if (t < deg) {
        if (ell) {
          l = A.ecol[qa + t];
          av = A.eval32 ? (double)A.eval32[qa + t] : A.eval[qa + t];
        } else {
          l = A.col[qa + t];
          av = aval(A, qa + t);
        }
        len = M.len[l];
        s_nbcol[t] = l;
        s_nbval[t] = av;
        s_nbbeg[t] = M.beg[l];
      }
      const unsigned long long dj = __ballot(l == (int)j);
      if (dj) ajj = __shfl(av, __ffsll((long long)dj) - 1, SPAI_WAVE);
      const int inc = wave_incl_scan(len);
      if (t < deg) s_nboff[t] = onb + run + inc - len;
      run += __shfl(inc, SPAI_WAVE - 1, SPAI_WAVE);
    }
    if (lane == 0) s_nboff[deg] = onb + run;
    const int ltot = onb + (nb_lds ? run : 0);
    if (ltot > L) {
      defer_column(tier, big, st, j);
      return;
    }
    if (overflow) {
      if (lane == 0) atomicOr(&st->err, 2);
      return;
    }
    ks_clear(s_keys, H);
    tile_sync<GS>();
    // ---- every list entry held in LDS, in one flattened gather (four per lane in flight)
    {
      constexpr int U = 4;
      for (int x0 = 0; x0 < ltot; x0 += SPAI_WAVE * U) {
        int ix[U];
        T vx[U];
        int dst[U];
#pragma unroll
        for (int c = 0; c < U; ++c) {
          const int pos = x0 + c * SPAI_WAVE + lane;
          dst[c] = -1;
          if (pos < ltot) {
            if (pos < orr) {
              ix[c] = M.idx[mb + pos];
              vx[c] = M.val[mb + pos];
            } else if (pos < op) {
              ix[c] = R.idx[rb + (pos - orr)];
              vx[c] = R.val[rb + (pos - orr)];
            } else if (pos < opt) {
              ix[c] = P.idx[pb + (pos - op)];
              vx[c] = P.val[pb + (pos - op)];
            } else if (pos < onb) {
              ix[c] = PT.idx[ptb + (pos - opt)];
              vx[c] = PT.val[ptb + (pos - opt)];
            } else {
              const int t = upper_bound_int(s_nboff + 1, deg, pos);
              const int64_t src = s_nbbeg[t] + (pos - s_nboff[t]);
              ix[c] = M.idx[src];
              vx[c] = M.val[src];
            }
            dst[c] = pos;
          }
        }
#pragma unroll
        for (int c = 0; c < U; ++c)
          if (dst[c] >= 0) {
            s_li[dst[c]] = ix[c];
            s_lv[dst[c]] = (double)vx[c];
          }
      }
    }
    tile_sync<GS>();
    // ---- key union (at most limit distinct keys)
    int kd[1] = {lane == 0 ? (int)j : -1};
    int nkeys = wave_sum_int(ks_insert_batch<1>(s_keys, H, kd));
    for (int x0 = 0; x0 < ltot && nkeys <= limit; x0 += SPAI_WAVE * 4) {
      int kk[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int pos = x0 + c * SPAI_WAVE + lane;
        kk[c] = pos < ltot ? s_li[pos] : -1;
      }
      nkeys += wave_sum_int(ks_insert_batch<4>(s_keys, H, kk));
    }
    if (!nb_lds)
      for (int t = 0; t < deg && nkeys <= limit; ++t) {
        const int64_t b0 = s_nbbeg[t];
        const int len = s_nboff[t + 1] - s_nboff[t];
        for (int x0 = 0; x0 < len && nkeys <= limit; x0 += SPAI_WAVE * 4) {
          int kk[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int e = x0 + c * SPAI_WAVE + lane;
            kk[c] = e < len ? M.idx[b0 + e] : -1;
          }
          nkeys += wave_sum_int(ks_insert_batch<4>(s_keys, H, kk));
        }
      }
    tile_sync<GS>();
    if (nkeys > limit) {
      defer_column(tier, big, st, j);
      tile_sync<GS>();
      return;
    }
    const int nk = ks_sort_inplace(s_keys, H);
    tile_sync<GS>();
    // ---- values, candidates
    const int64_t ob = off[j];
    int cntM = 0, cntMo = 0, cntP = 0, cntPT = 0;
    for (int base = 0; base < nk; base += SPAI_WAVE) {
      const int t = base + lane;
      const bool valid = t < nk;
      const int k = valid ? s_keys[t] : -1;
      double mv = 0.0, rv = 0.0, rtv = 0.0, pv = 0.0, ptv = 0.0;
      {
        const int ob4[4] = {om, orr, op, opt}, ln4[4] = {lm, lr, lp, lpt}, k4[4] = {k, k, k, k};
        int p4[4];
        search_lockstep<4>(s_li, ob4, ln4, k4, p4);
        if (p4[0] >= 0) mv = s_lv[om + p4[0]];
        if (p4[1] >= 0) rv = s_lv[orr + p4[1]];
        if (p4[2] >= 0) pv = s_lv[op + p4[2]];
        if (p4[3] >= 0) ptv = s_lv[opt + p4[3]];
      }
      if (needRT) {
        double sum = 0.0;
        for (int t0 = 0; t0 < deg; t0 += 8) {
          int b8[8], n8[8], k8[8], p8[8];
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const int t2 = t0 + c;
            b8[c] = t2 < deg ? s_nboff[t2] : 0;
            n8[c] = t2 < deg ? s_nboff[t2 + 1] - b8[c] : 0;
            k8[c] = k;
          }
          if (nb_lds) {
            search_lockstep<8>(s_li, b8, n8, k8, p8);
#pragma unroll
            for (int c = 0; c < 8; ++c)
              if (p8[c] >= 0) sum += s_nbval[t0 + c] * s_lv[b8[c] + p8[c]];
          } else {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
              if (t0 + c >= deg) continue;
              const int64_t b0 = s_nbbeg[t0 + c];
              const int e = bsearch_idx(M.idx + b0, n8[c], k);
              if (e >= 0) sum += s_nbval[t0 + c] * (double)M.val[b0 + e];
            }
          }
        }
        const double rj = ((k == (int)j) ? 1.0 : 0.0) - sum;
        rtv = md.weighted ? (double)(T)((1.0 / ajj) * rj) : (double)(T)rj;   // Z^T = Pi R^T
      }
      // M candidate
      bool keepM = false, offM = false;
      T mt = (T)0;
      if (md.doM) {
        const double v1 = md.x1 == 1 ? rv : (md.x1 == 2 ? pv : 0.0);
        const double v2 = md.x2 == 1 ? rv : (md.x2 == 2 ? pv : 0.0);
        const double x = (mv + a1 * v1) + a2 * v2;
        double sv = x;
        if (md.sym) {
          const double w1 = md.x1 == 1 ? rtv : (md.x1 == 2 ? ptv : 0.0);
          const double w2 = md.x2 == 1 ? rtv : (md.x2 == 2 ? ptv : 0.0);
          const double y = (mv + a1 * w1) + a2 * w2;
          sv = (x + y) * 0.5;
        }
        mt = (T)sv;
        const double sd = (double)mt;
        keepM = valid && sd != 0.0 && (k == (int)j || fabs(sd) >= md.u);
        offM = keepM && k != (int)j;
      }
      // P and P^T candidates
      bool keepP = false, keepPT = false;
      T pt = (T)0, ptt = (T)0;
      if (md.doP) {
        const double x = (md.pR ? c1 * rv : 0.0) + (md.pP ? c2 * pv : 0.0);
        const double y = (md.pR ? c1 * rtv : 0.0) + (md.pP ? c2 * ptv : 0.0);
        pt = (T)x;
        ptt = (T)y;
        keepP = valid && (double)pt != 0.0;
        keepPT = valid && (double)ptt != 0.0;
      }
      const unsigned long long bm = __ballot(keepM);
      const unsigned long long bmo = __ballot(offM);
      const unsigned long long bp = __ballot(keepP);
      const unsigned long long bpt = __ballot(keepPT);
      const unsigned long long lt = lanemask_lt();
      if (keepM) {
        const int64_t pos = ob + cntM + __popcll(bm & lt);
        Mo.idx[pos] = k;
        Mo.val[pos] = mt;
      }
      if (keepP) {
        const int64_t pos = ob + cntP + __popcll(bp & lt);
        Po.idx[pos] = k;
        Po.val[pos] = pt;
      }
      if (keepPT) {
        const int64_t pos = ob + cntPT + __popcll(bpt & lt);
        PTo.idx[pos] = k;
        PTo.val[pos] = ptt;
      }
      cntM += __popcll(bm);
      cntMo += __popcll(bmo);
      cntP += __popcll(bp);
      cntPT += __popcll(bpt);
    }
    tile_sync<GS>();
    if (lane == 0) {
      if (md.doM) { Mo.beg[j] = ob; Mo.len[j] = cntM; }
      if (md.doP) {
        Po.beg[j] = ob; Po.len[j] = cntP;
        PTo.beg[j] = ob; PTo.len[j] = cntPT;
      }
    }
    if (md.colcap) {
      // thresholds from the candidates this wave has just written (L1/L2 resident)
      const int k = kcol[j];
      __threadfence_block();
      tile_sync<GS>();
      if (md.doM) {
        const double t = kth_largest_cols(Mo.idx + ob, Mo.val + ob, cntM, (int)j, k - 1);
        if (lane == 0) tM[j] = t;
      }
      if (md.doP) {
        const double t = kth_largest_cols(Po.idx + ob, Po.val + ob, cntP, -1, k);
        if (lane == 0) tP[j] = t;
      }
    }
    tile_sync<GS>();
  };

  if (tier == 0) {
    ColumnWalk w(A.n, blockIdx.x, gridDim.x);
    for (int64_t j = w.begin; j < w.end; j += w.step) body(j);
  } else if (tier == 1) {
    const int cnt = *big.count;
    for (int t = blockIdx.x; t < cnt; t += gridDim.x) body(big.list[t]);
  } else {
    const int cnt = *big.count2;
    for (int t = blockIdx.x; t < cnt; t += gridDim.x) body(big.list2[t]);
  }
}

template <typename T, bool GS>
__global__ __launch_bounds__(SPAI_WAVE) void k_update(Csr A, Pair<T> Mp, Cols<T> R, Pair<T> Pp,
                                                      Pair<T> PTp, UpdMode md, const int64_t* off,
                                                      const int64_t* total, const int32_t* kcol,
                                                      double* tM, double* tP, BigList big,
                                                      Seg seg, DevState* st, int tier, int L,
                                                      int H, int DG) {
  update_body<T, GS>(A, Mp, R, Pp, PTp, md, off, total, kcol, tM, tP, big, seg, st, tier, L, H,
                     DG);
}

// The same resident tier with registers capped at five waves per SIMD (a few spills):
// slower on large columns, faster where columns are small and more columns in flight
// pay; the register allocation does not change the arithmetic, so the tile autotuner
// may pick either.
template <typename T>
__global__ __launch_bounds__(SPAI_WAVE) __attribute__((amdgpu_waves_per_eu(5, 5))) void k_update_w5(
    Csr A, Pair<T> Mp, Cols<T> R, Pair<T> Pp, Pair<T> PTp, UpdMode md, const int64_t* off,
    const int64_t* total, const int32_t* kcol, double* tM, double* tP, BigList big, Seg seg,
    DevState* st, int tier, int L, int H, int DG) {
  update_body<T, false>(A, Mp, R, Pp, PTp, md, off, total, kcol, tM, tP, big, seg, st, tier, L, H,
                        DG);
}

// Lean resident tier of the update (A in ELL).  Same
// candidates and the same arithmetic as update_body, built without searches: every row
// of the column's own lists (m_j, r_j, p_j, p^T_j, up to 192 entries, three per lane) and
// of its neighbour columns m_l, l in N(j) (up to 256 entries together, laid out flat over
// the lanes), goes into the ordered key set; the keys are sorted by row and a byte table maps a row's hash to its
// rank; the own lists' values are then scattered to dense per-rank arrays and the
// neighbour products a_jl m_l(k) added to a per-rank sum neighbour by neighbour in
// ascending l (one round per neighbour, so each sum runs in the order update_body uses),
// and each lane forms the candidates of its keys.
constexpr int kUpdLeanKeys = 128;
constexpr int kUpdLeanOwn = 192;   // own-list entries (whatever the tile's L)
constexpr int kUpdLeanNbr = 256;   // entries of the neighbour columns together

// SECOND: the same kernel under another name for the floor-free second pass (masked
// unless needed), so that profiles keep the two apart.  LM: a mode fixed at compile time,
// so that its flags take no registers and its branches fold -- 1: the symmetrized LOMR
// step under a global cap (M + a1 R + a2 P, and P from R and P), 2: the symmetrized MR
// step (M + a1 R, no P; either cap); 0: every mode, read from md.
// Registers capped for six waves per SIMD on the float path (2% faster at 96^3; the
// float64 path spills there and keeps five).
template <typename T, bool FLAT, bool SECOND, int LM>
__global__ __launch_bounds__(SPAI_WAVE) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 5))) void k_update_lean(
    Csr A, Pair<T> Mp, Cols<T> R, Pair<T> Pp, Pair<T> PTp, UpdMode mdin, const int64_t* off,
    const int64_t* total, const int32_t* kcol, double* tM, double* tP, BigList big, Seg seg,
    DevState* st, int L, int H) {
  if (!st->any_active || !st->iter_active) return;
  UpdMode md = mdin;
  if constexpr (LM == 1) {
    md.doM = 1;
    md.x1 = 1;
    md.x2 = 2;
    md.doP = 1;
    md.pR = 1;
    md.pP = 1;
    md.sym = 1;
    md.colcap = 0;
  } else if constexpr (LM == 2) {
    md.doM = 1;
    md.x1 = 1;
    md.x2 = 0;
    md.doP = 0;
    md.sym = 1;
  }
  // the fixed-size arrays at fixed LDS addresses (their offsets fold into the accesses),
  // the key set behind
  __shared__ __align__(16) unsigned char cb[kBtCells];        // 1 + rank of a row's hash
  __shared__ __align__(16) T dv[4 * kUpdLeanKeys];            // m, r, p, p^T by rank
  __shared__ __align__(16) double rta[kUpdLeanKeys];          // sum_l a_jl m_l(k) by rank
  extern __shared__ char smem[];
  Carve cv(smem);
  unsigned* kt = cv.take<unsigned>(max(H + kOhOver, kUpdLeanKeys));
  int* keys = (int*)kt;
  const int lane = lane_id();
  for (int i = lane; i < kBtCells / 4; i += SPAI_WAVE) ((unsigned*)cb)[i] = 0u;
  __syncthreads();
  const Cols<T> M = Mp.now();
  const Cols<T> Mo = Mp.nxt();
  const Cols<T> P = Pp.now();
  const Cols<T> Po = Pp.nxt();
  const Cols<T> PT = PTp.now();
  const Cols<T> PTo = PTp.nxt();
  const bool needR = (md.doM && (md.x1 == 1 || md.x2 == 1)) || (md.doP && md.pR);
  const bool needP = (md.doM && (md.x1 == 2 || md.x2 == 2)) || (md.doP && md.pP);
  const bool mirror = md.sym != 0;
  const bool needRT = needR && mirror;
  const bool needPT = needP && mirror;
  const int64_t ntot = *total;
  const bool overflow = ntot > Mo.cap || (md.doP && (ntot > Po.cap || ntot > PTo.cap));
  const T* eval = sizeof(T) == 4 ? (const T*)A.eval32 : (const T*)A.eval;
  const int W = 1 << A.eshift;                   // ELL width of A (at most 64)
  // A column's descriptors are loaded one column ahead, one value per lane (lanes 0-3
  // the lengths of m_j, r_j, p_j, p^T_j, lanes 4-7 their starts, lanes 8 and 9 the
  // column's candidate range off[j] .. off[j+1]) together with row j of A (lanes 0-7:
  // neighbour l and a_jl), and each neighbour column's length and start once those
  // have arrived: a column's first loads are then its entries, and its descriptors
  // arrive while the column before it is computed.
  struct Pre {
    int64_t d = 0;
    int nl = -1;
    T av = (T)0;
    int nlen = 0;
    int64_t nbeg = 0;
  };
  auto pre1 = [&](int64_t jj, Pre& p) {
    p = Pre{};
    if (lane < 4) {
      const int* lp = lane == 0 ? M.len : lane == 1 ? R.len : lane == 2 ? P.len : PT.len;
      p.d = lp[jj];
    } else if (lane < 8) {
      const int64_t* bp = lane == 4 ? M.beg : lane == 5 ? R.beg : lane == 6 ? P.beg : PT.beg;
      p.d = bp[jj];
    } else if (lane == 8) {
      p.d = off[jj];
    } else if (lane == 9) {
      p.d = jj + 1 < A.n ? off[jj + 1] : ntot;
    }
    if (needRT && lane < W) {
      p.nl = A.ecol[(jj << A.eshift) + lane];
      p.av = eval[(jj << A.eshift) + lane];
    }
  };
  auto pre2 = [&](Pre& p) {
    if (p.nl >= 0) {
      p.nlen = M.len[p.nl];
      p.nbeg = M.beg[p.nl];
    }
  };
  __shared__ unsigned below[2];                   // candidates left out below the floors
  const double fM = st->floorM, fP = st->floorP;  // 0 unless a global cap set them
  if (lane < 2) below[lane] = 0u;
  __syncthreads();
  ColumnWalk w(A.n, blockIdx.x, gridDim.x);
  Pre cur, nxt;
  if (w.begin < w.end) {
    pre1(w.begin, cur);
    pre2(cur);
  }
  for (int64_t j = w.begin; j < w.end; j += w.step, cur = nxt) {
    const int lm = md.doM ? (int)wave_read64(cur.d, 0) : 0;
    const int lr = needR ? (int)wave_read64(cur.d, 1) : 0;
    const int lp = needP ? (int)wave_read64(cur.d, 2) : 0;
    const int lpt = needPT ? (int)wave_read64(cur.d, 3) : 0;
    const int lown = lm + lr + lp + lpt;
    const int64_t bm = wave_read64(cur.d, 4), br = wave_read64(cur.d, 5);
    const int64_t bp = wave_read64(cur.d, 6), bpt = wave_read64(cur.d, 7);
    const int64_t ob = wave_read64(cur.d, 8);
    const int64_t ub = wave_read64(cur.d, 9) - ob;               // entries of all lists + 1
    const int nl = cur.nl;                                       // neighbour l in N(j)
    const double av = (double)cur.av;
    const int nlen = cur.nlen;
    const int64_t nbeg = cur.nbeg;
    const int64_t jn = j + w.step;
    if (jn < w.end) pre1(jn, nxt);
    // own entries, up to three per lane (list 0 m, 1 r, 2 p, 3 p^T; an entry's list
    // follows from its place e), one unconditional load per slot from the list the
    // lane's entry lies in (entry 0 of m where it has none; bit k of ovalid says which
    // are real), so all of them are in flight together (a column whose lists hold
    // more is deferred below)
    int orow[kUpdLeanOwn / SPAI_WAVE];
    T oval[kUpdLeanOwn / SPAI_WAVE];
    unsigned ovalid = 0u;
    const bool fits = lown <= kUpdLeanOwn;
#pragma unroll
    for (int k = 0; k < kUpdLeanOwn / SPAI_WAVE; ++k) {
      const int e = lane + k * SPAI_WAVE;
      const bool v = fits && e < lown;
      const int lst = (e >= lm) + (e >= lm + lr) + (e >= lm + lr + lp);
      const int* ip = lst == 0 ? M.idx : lst == 1 ? R.idx : lst == 2 ? P.idx : PT.idx;
      const T* vp = lst == 0 ? M.val : lst == 1 ? R.val : lst == 2 ? P.val : PT.val;
      const int64_t q0 = lst == 0 ? bm + e : lst == 1 ? br + (e - lm)
                       : lst == 2 ? bp + (e - lm - lr) : bpt + (e - lm - lr - lp);
      const int64_t q = v ? q0 : 0;
      orow[k] = (v ? ip : M.idx)[q];
      oval[k] = (v ? vp : M.val)[q];
      ovalid |= (v ? 1u : 0u) << k;
    }
    const unsigned long long nm = __ballot(nl >= 0);
    const int deg = __popcll(nm);                 // entries first, so lanes 0 .. deg-1
    // neighbour entries.  FLAT (A's ELL rows wider than 8): laid out flat over the lanes,
    // entry e of the concatenated neighbour columns m_l (in row j's order) in lane e mod
    // 64, slot e / 64, its neighbour t found by a binary search over the lanes' exclusive
    // prefix of the lengths.  Else (rows of at most 8): entry `lane` of each of the eight
    // neighbour columns in slot t.  The loads are unconditional (entry 0 of m where a
    // slot has none; ntag is -1 there), so no conversion or select waits on one before
    // all are in flight.
    constexpr int NS = kUpdLeanNbr / SPAI_WAVE;   // neighbour slots per lane
    int nrow[NS], ntag[NS];                       // ntag: slot k's neighbour, or -1
    T nval[NS];
    int ne;                                       // entries of all neighbour columns
    if constexpr (FLAT) {                         // up to 64 neighbours: binary search
      const int nincl = wave_incl_scan(nlen);     // lengths are 0 on lanes >= deg
      const int npre = nincl - nlen;
      ne = __builtin_amdgcn_readlane(nincl, SPAI_WAVE - 1);
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int e = lane + k * SPAI_WAVE;
        int t = 0;                                // the last neighbour starting at or before e
#pragma unroll
        for (int step = SPAI_WAVE / 2; step >= 1; step >>= 1) {
          const int c = t + step;
          const int pc = __shfl(npre, c < deg ? c : 0, SPAI_WAVE);   // every lane shuffles
          if (c < deg && pc <= e) t = c;
        }
        const bool v = e < ne;
        // both shuffles on every lane (a shuffle from a lane left out of a branch is
        // undefined), then the select
        const int64_t bt = __shfl(nbeg, t, SPAI_WAVE);
        const int pt = __shfl(npre, t, SPAI_WAVE);
        const int64_t q = v ? bt + (e - pt) : 0;
        nrow[k] = M.idx[q];
        nval[k] = M.val[q];
        ntag[k] = v ? t : -1;
      }
    } else {                                      // at most 8 neighbours: scalar prefix sums
      int pre[8];
      int acc = 0;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        pre[c] = acc;
        acc += __builtin_amdgcn_readlane(nlen, c);
      }
      ne = acc;
      // lane c's neighbour start less its first flat index, so that entry e of neighbour t
      // sits at nrel[t] + e
      int mypre = 0;
#pragma unroll
      for (int c = 1; c < 8; ++c) mypre = lane == c ? pre[c] : mypre;
      const int64_t nrel = nbeg - (int64_t)mypre;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int e = lane + k * SPAI_WAVE;
        // the last neighbour starting at or before e: the prefix is non-decreasing and
        // equals ne from neighbour deg on, so for e < ne it is the count of c >= 1 with
        // pre[c] <= e
        int t = 0;
#pragma unroll
        for (int c = 1; c < 8; ++c) t += pre[c] <= e ? 1 : 0;
        const bool v = e < ne;
        const int64_t bt = __shfl(nrel, t, SPAI_WAVE);   // on every lane
        const int64_t q = v ? bt + e : 0;
        nrow[k] = M.idx[q];
        nval[k] = M.val[q];
        ntag[k] = v ? t : -1;
      }
    }
    const bool nfits = ne <= kUpdLeanNbr;
    auto slot_nbr = [&](int k) -> int { return ntag[k]; };   // the neighbour of slot k, or -1
    if (jn < w.end) pre2(nxt);
    if (!fits || !nfits) {
      defer_column(0, big, st, j);
      continue;
    }
    if (overflow) {
      if (lane == 0) atomicOr(&st->err, 2);
      continue;
    }
    const unsigned long long dj = __ballot(nl == (int)j);
    const double ajj = dj ? __shfl(av, __ffsll((long long)dj) - 1, SPAI_WAVE) : 0.0;
    const int Hc = next_pow2((int)min<int64_t>(max<int64_t>(ub, 64), (int64_t)H));
    const int ksh = 32 - log2_pow2(Hc);
    const int kend = Hc + kOhOver;
    for (int i = lane; i < kend; i += SPAI_WAVE) kt[i] = kOhEmpty;
    // the diagonal key first: the table is empty, so it sits at its home slot (the
    // slots of an ordered table do not depend on the order of the inserts)
    if (lane == 0) kt[ohash((int)j) >> ksh] = ohash((int)j);
    __syncthreads();
    int okey[kUpdLeanOwn / SPAI_WAVE];
#pragma unroll
    for (int k = 0; k < kUpdLeanOwn / SPAI_WAVE; ++k) okey[k] = (ovalid >> k) & 1u ? orow[k] : -1;
    bool ok = oh_insert_batch<kUpdLeanOwn / SPAI_WAVE>(kt, ksh, okey);
#pragma unroll
    for (int k0 = 0; k0 < NS; k0 += 4) {           // batches of four keys per lane
      int nk[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) nk[k] = slot_nbr(k0 + k) >= 0 ? nrow[k0 + k] : -1;
      ok = oh_insert_batch<4>(kt, ksh, nk) && ok;
    }
    const bool bad = __ballot(!ok) != 0ull;
    __syncthreads();
    const int nk = bad ? 0 : oh_compact(kt, kend);
    __syncthreads();
    if (bad || nk > kUpdLeanKeys) {
      defer_column(0, big, st, j);
      continue;
    }
    if (nk <= 64) sort_in_registers<1>(keys, nk);
    else sort_in_registers<2>(keys, nk);
    __syncthreads();
    int krow[2], klst[2] = {0, 0}, kpos[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      kpos[k] = lane + k * SPAI_WAVE;
      krow[k] = kpos[k] < nk ? keys[kpos[k]] : -1;
    }
    const int a = bt_build<2, 1>(cb, krow, klst, kpos);
    if (a < 0) {
      defer_column(0, big, st, j);
      continue;
    }
    const unsigned mul = bt_mul(a);
    // dense per-rank values (zero where a list has no entry)
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (kpos[k] < nk) {
#pragma unroll
        for (int q = 0; q < 4; ++q) dv[q * kUpdLeanKeys + kpos[k]] = (T)0;
        rta[kpos[k]] = 0.0;
      }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kUpdLeanOwn / SPAI_WAVE; ++k)
      if ((ovalid >> k) & 1u) {
        const int e = lane + k * SPAI_WAVE;
        const int lst = (e >= lm) + (e >= lm + lr) + (e >= lm + lr + lp);
        dv[lst * kUpdLeanKeys + (int)cb[bt_cell(orow[k], mul)] - 1] = oval[k];
      }
    // neighbour products in ascending l: one round per neighbour, distinct ranks inside
    for (int t = 0; t < deg; ++t) {
      const double a_t = __shfl(av, t, SPAI_WAVE);
      // the entries of m_t: distinct rows, so distinct ranks (a lane's slots too)
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (slot_nbr(k) == t) {
          const int rk = (int)cb[bt_cell(nrow[k], mul)] - 1;
          rta[rk] += a_t * (double)nval[k];
        }
    }
    __syncthreads();
    // the matrix's step sizes, read only now: a load at the top of the column would
    // make the column's first wait also wait for it
    const SegState& g = seg.st[seg.segof(j)];
    const double a1 = g.coef[0], a2 = g.coef[1], c1 = g.coef[2], c2 = g.coef[3];
    int cntM = 0, cntP = 0, cntPT = 0;
    for (int base = 0; base < nk; base += SPAI_WAVE) {
      const int t = base + lane;
      const bool valid = t < nk;
      const int k = valid ? keys[t] : -1;
      double mv = 0.0, rv = 0.0, pv = 0.0, ptv = 0.0, rtv = 0.0;
      if (valid) {
        mv = (double)dv[t];
        rv = (double)dv[kUpdLeanKeys + t];
        pv = (double)dv[2 * kUpdLeanKeys + t];
        ptv = (double)dv[3 * kUpdLeanKeys + t];
      }
      if (needRT) {
        const double rj = ((k == (int)j) ? 1.0 : 0.0) - (valid ? rta[t] : 0.0);
        rtv = md.weighted ? (double)(T)((1.0 / ajj) * rj) : (double)(T)rj;   // Z^T = Pi R^T
      }
      bool keepM = false;
      T mt = (T)0;
      if (md.doM) {
        const double v1 = md.x1 == 1 ? rv : (md.x1 == 2 ? pv : 0.0);
        const double v2 = md.x2 == 1 ? rv : (md.x2 == 2 ? pv : 0.0);
        const double x = (mv + a1 * v1) + a2 * v2;
        double sv = x;
        if (md.sym) {
          const double w1 = md.x1 == 1 ? rtv : (md.x1 == 2 ? ptv : 0.0);
          const double w2 = md.x2 == 1 ? rtv : (md.x2 == 2 ? ptv : 0.0);
          const double y = (mv + a1 * w1) + a2 * w2;
          sv = (x + y) * 0.5;
        }
        mt = (T)sv;
        const double sd = (double)mt;
        keepM = valid && sd != 0.0 && (k == (int)j || fabs(sd) >= md.u);
      }
      bool keepP = false, keepPT = false;
      T pt = (T)0, ptt = (T)0;
      if (md.doP) {
        const double x = (md.pR ? c1 * rv : 0.0) + (md.pP ? c2 * pv : 0.0);
        const double y = (md.pR ? c1 * rtv : 0.0) + (md.pP ? c2 * ptv : 0.0);
        pt = (T)x;
        ptt = (T)y;
        keepP = valid && (double)pt != 0.0;
        keepPT = valid && (double)ptt != 0.0;
      }
      // candidates below the floor are not written (the diagonal always is); they are
      // counted, and the selection checks that its cut clears the floor
      const bool wM = keepM && (k == (int)j || fabs((double)mt) >= fM);
      const bool wP = keepP && fabs((double)pt) >= fP;
      const bool wPT = keepPT && fabs((double)ptt) >= fP;
      {
        const unsigned bM = (unsigned)__popcll(__ballot(keepM && !wM));
        const unsigned bP = (unsigned)__popcll(__ballot(keepP && !wP));
        if (lane == 0 && (bM | bP)) {
          below[0] += bM;
          below[1] += bP;
        }
      }
      keepM = wM;
      keepP = wP;
      keepPT = wPT;
      const unsigned long long bm = __ballot(keepM);
      const unsigned long long bp = __ballot(keepP);
      const unsigned long long bpt = __ballot(keepPT);
      const unsigned long long lt = lanemask_lt();
      if (keepM) {
        const int64_t q = ob + cntM + __popcll(bm & lt);
        Mo.idx[q] = k;
        Mo.val[q] = mt;
      }
      if (keepP) {
        const int64_t q = ob + cntP + __popcll(bp & lt);
        Po.idx[q] = k;
        Po.val[q] = pt;
      }
      if (keepPT) {
        const int64_t q = ob + cntPT + __popcll(bpt & lt);
        PTo.idx[q] = k;
        PTo.val[q] = ptt;
      }
      cntM += __popcll(bm);
      cntP += __popcll(bp);
      cntPT += __popcll(bpt);
    }
    if (lane == 0) {
      if (md.doM) { Mo.beg[j] = ob; Mo.len[j] = cntM; }
      if (md.doP) {
        Po.beg[j] = ob; Po.len[j] = cntP;
        PTo.beg[j] = ob; PTo.len[j] = cntPT;
      }
    }
    if (md.colcap) {
      // thresholds from the candidates this wave has just written (L1/L2 resident)
      const int kc = kcol[j];
      __threadfence_block();
      __syncthreads();
      if (md.doM) {
        const double t = kth_largest_cols(Mo.idx + ob, Mo.val + ob, cntM, (int)j, kc - 1);
        if (lane == 0) tM[j] = t;
      }
      if (md.doP) {
        const double t = kth_largest_cols(Po.idx + ob, Po.val + ob, cntP, -1, kc);
        if (lane == 0) tP[j] = t;
      }
    }
    bt_clear<2, 1>(cb, krow, klst, mul);
    __syncthreads();
  }
  __syncthreads();
  if (lane == 0) {
    if (below[0]) atomicAdd(&st->belowM, (unsigned long long)below[0]);
    if (below[1]) atomicAdd(&st->belowP, (unsigned long long)below[1]);
  }
}

template <typename T>   // the lean update's static arrays
static size_t update_lean_lds() {
  return (size_t)kBtCells + (size_t)4 * kUpdLeanKeys * sizeof(T) + (size_t)kUpdLeanKeys * 8;
}

static int update_deg(Tile t) { return t.DG ? t.DG : (t.L >= 2048 ? 256 : 64); }

static size_t update_lds(Tile t, bool) {
  const int DG = update_deg(t);
  return (size_t)t.L * 4 + (size_t)t.H * 4 + (size_t)DG * 4 * 2 + 4 + 8 + (size_t)t.L * 8 +
         (size_t)DG * 8 * 2 + 96;
}

size_t update_tile_bytes(Tile t) {
  return t.waves == 1
             ? update_lean_lds<double>() + (size_t)std::max(t.H + kOhOver, kUpdLeanKeys) * 4 + 64
             : update_lds(t, false);
}

template <typename T>
void launch_update(const Csr& A, Pair<T> M, Cols<T> R, Pair<T> P, Pair<T> PT, UpdMode md,
                   const int64_t* off, const int64_t* total, const int32_t* kcol, double* tM,
                   double* tP, BigList big, const Seg& seg, DevState* st, Tile small, Tile large,
                   Tile huge, hipStream_t s, bool second) {
  hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(1), 0, s, big.count, big.count2);
  if (small.waves == 1 && A.eshift >= 0) {
    const size_t lds = (size_t)std::max(small.H + kOhOver, kUpdLeanKeys) * 4 + 64;   // dynamic part
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(resident_grid(kern, lds)), dim3(SPAI_WAVE), lds, s, A, M, R,
                         P, PT, md, off, total, kcol, tM, tP, big, seg, st, small.L, small.H);
    };
    // ELL rows wider than 8: neighbour entries laid out flat
    const bool lomr = md.doM == 1 && md.x1 == 1 && md.x2 == 2 && md.doP == 1 && md.pR == 1 &&
                      md.pP == 1 && md.sym == 1 && md.colcap == 0;
    const bool mr = md.doM == 1 && md.x1 == 1 && md.x2 == 0 && md.doP == 0 && md.sym == 1;
    auto pick = [&](auto lmc) {
      constexpr int L2 = decltype(lmc)::value;
      if (A.eshift > 3)
        second ? go(k_update_lean<T, true, true, L2>) : go(k_update_lean<T, true, false, L2>);
      else
        second ? go(k_update_lean<T, false, true, L2>) : go(k_update_lean<T, false, false, L2>);
    };
    if (lomr) pick(std::integral_constant<int, 1>{});
    else if (mr) pick(std::integral_constant<int, 2>{});
    else pick(std::integral_constant<int, 0>{});
  } else if (small.waves == 5)
    hipLaunchKernelGGL((k_update_w5<T>),
                       dim3(resident_grid(k_update_w5<T>, update_lds(small, true))),
                       dim3(SPAI_WAVE), update_lds(small, true), s, A, M, R, P, PT, md, off,
                       total, kcol, tM, tP, big, seg, st, 0, small.L, small.H, update_deg(small));
  else
    hipLaunchKernelGGL((k_update<T, false>),
                       dim3(resident_grid(k_update<T, false>, update_lds(small, true))),
                       dim3(SPAI_WAVE), update_lds(small, true), s, A, M, R, P, PT, md, off,
                       total, kcol, tM, tP, big, seg, st, 0, small.L, small.H, update_deg(small));
  hipLaunchKernelGGL((k_update<T, false>), dim3(256), dim3(SPAI_WAVE), update_lds(large, false), s,
                     A, M, R, P, PT, md, off, total, kcol, tM, tP, big, seg, st, 1, large.L,
                     large.H, update_deg(large));
  hipLaunchKernelGGL((k_update<T, true>), dim3(big.grid2), dim3(SPAI_WAVE), 0, s, A, M, R, P, PT,
                     md, off, total, kcol, tM, tP, big, seg, st, 2, huge.L, huge.H,
                     update_deg(huge));
}

// ============================================================================
// global cap: exact (b+1)-th largest candidate magnitude by radix selection on the
// bits of |x| (positive doubles order like their bit patterns)
// ============================================================================

constexpr int kSelThreads = 256;

__device__ __forceinline__ unsigned long long mag_key(double v) {
  return (unsigned long long)__double_as_longlong(fabs(v));
}

// signed doubles (the heuristic drop scores) as keys that order like the values: the
// sign bit flipped for v >= 0, every bit flipped for v < 0
__device__ __forceinline__ unsigned long long ord_key(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  return (u >> 63) ? ~u : (u | (1ull << 63));
}

__device__ __forceinline__ double ord_value(unsigned long long k) {
  return __longlong_as_double((long long)((k >> 63) ? (k & ~(1ull << 63)) : ~k));
}

// ---- grouped walk over the entries of 64 consecutive columns ----------------------
// A one-wave workgroup takes columns j0 .. j0+63 at once: lane c holds column j0 + c's
// start cb and length cl (loaded together) and ex, the exclusive prefix of the
// lengths, so the T entries of the group form one flat range.  Entry x belongs to the
// column c with ex[c] <= x < ex[c] + cl[c], found by a six-step shuffle search, and
// kGU entries per lane are loaded per batch, all in flight together.  This replaces
// two dependent loads per column (descriptor, then entries) by about one per group.
// The compaction takes eight entries per lane per batch (measured 11% faster than
// four at 96^3), the selection passes four (eight was 3% slower there).
constexpr int kGU = 4;
constexpr int kGUc = 8;

struct Group64 {
  int64_t j0, cb;
  int cl, ex, T;
};

template <typename T>
__device__ __forceinline__ Group64 group_load(const Cols<T>& X, int64_t j0, int64_t n) {
  Group64 g;
  g.j0 = j0;
  const int64_t j = j0 + lane_id();
  g.cb = 0;
  g.cl = 0;
  if (j < n) {
    g.cb = X.beg[j];
    g.cl = X.len[j];
  }
  const int inc = wave_incl_scan(g.cl);
  g.ex = inc - g.cl;
  g.T = __shfl(inc, SPAI_WAVE - 1, SPAI_WAVE);
  return g;
}

// group column of flat entry x (< T): the last c with ex[c] <= x.  The shuffles read
// other lanes' registers, so every lane of the wave must execute this (and group_src)
// together, outside any lane-dependent branch.
__device__ __forceinline__ int group_col(const Group64& g, int x) {
  int c = 0;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1)
    if (__shfl(g.ex, c + step, SPAI_WAVE) <= x) c += step;
  return c;
}

__device__ __forceinline__ int64_t group_src(const Group64& g, int c, int x) {
  return __shfl(g.cb, c, SPAI_WAVE) + (int64_t)(x - __shfl(g.ex, c, SPAI_WAVE));
}

// histogram of the top key bits (63..52; for magnitudes bit 63 is 0) of the candidates,
// counting diagonal entries apart.  SC: the keys are the signed scores sc[] stored beside
// the candidates instead of their magnitudes.  Four waves per workgroup share one LDS
// histogram, each walking its own 64-column groups: the histogram's LDS no longer limits
// the waves in flight (one wave per histogram allowed five per SIMD, 7% slower).
template <typename T, bool SC>
__global__ __launch_bounds__(4 * SPAI_WAVE) void k_sel_hist_exp(Pair<T> Xp, const double* sc,
                                                            int excl_diag,
                                                            unsigned long long* hist, int64_t n,
                                                            DevState* st) {
  if (!st->any_active || !st->iter_active) return;
  constexpr int NB = SC ? 4096 : 2048;
  __shared__ unsigned int h[NB];
  const int lane = lane_id();
  const int wv = threadIdx.x / SPAI_WAVE;
  for (int i = threadIdx.x; i < NB; i += 4 * SPAI_WAVE) h[i] = 0;
  __syncthreads();
  const Cols<T> X = Xp.nxt();
  long long diag = 0;
  const int64_t ng = (n + 63) / 64;
  for (int64_t gi = (int64_t)blockIdx.x * 4 + wv; gi < ng; gi += (int64_t)gridDim.x * 4) {
    const Group64 g = group_load(X, gi * 64, n);
    for (int x0 = 0; x0 < g.T; x0 += SPAI_WAVE * kGU) {
      int col[kGU], idx[kGU];
      T val[kGU];
      double sv[kGU];
#pragma unroll
      for (int u = 0; u < kGU; ++u) {
        const int x = x0 + u * SPAI_WAVE + lane;
        const int xc = min(x, g.T - 1);            // all lanes shuffle together
        const int c = group_col(g, xc);
        const int64_t src = group_src(g, c, xc);
        sv[u] = 0.0;
        col[u] = -1;
        idx[u] = -1;
        val[u] = (T)0;
        if (x < g.T) {
          col[u] = c;
          if (excl_diag) idx[u] = X.idx[src];
          if constexpr (SC) sv[u] = sc[src]; else val[u] = X.val[src];
        }
      }
#pragma unroll
      for (int u = 0; u < kGU; ++u) {
        if (col[u] < 0) continue;
        if (excl_diag && idx[u] == (int)(g.j0 + col[u])) {
          ++diag;
          continue;
        }
        const unsigned long long key = SC ? ord_key(sv[u]) : mag_key((double)val[u]);
        atomicAdd(&h[(int)(key >> 52)], 1u);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NB; i += 4 * SPAI_WAVE)
    if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
  diag = wave_sum_ll(diag);
  if (lane == 0 && diag) atomicAdd((unsigned long long*)&st->sel_diag, (unsigned long long)diag);
}

// Find, with one 1024-thread block, the bin i holding the rank-th largest key of a
// histogram counted from the top bin down: *bin = i, *above = keys in bins above i.
// Each thread owns nbins / 1024 consecutive bins (thread 0 the highest).
__device__ inline void find_bin_desc(const unsigned long long* hist, int nbins, long long rank,
                                     long long* total, int* bin, long long* above) {
  __shared__ int64_t sh[1024];
  __shared__ int s_bin;
  __shared__ long long s_above, s_total;
  const int t = threadIdx.x;
  const int per = nbins / 1024;
  const int hi = nbins - 1 - t * per;            // this thread's bins: hi, hi-1, ..., hi-per+1
  long long loc = 0;
  for (int k = 0; k < per; ++k) loc += (long long)hist[hi - k];
  int64_t tot;
  const int64_t before = block_excl_scan_i64(loc, sh, &tot);
  if (t == 0) { s_total = tot; s_bin = -1; s_above = 0; }
  __syncthreads();
  if (rank >= 1 && before < rank && before + loc >= rank) {
    long long acc = before;
    for (int k = 0; k < per; ++k) {
      const long long c = (long long)hist[hi - k];
      if (acc + c >= rank) { s_bin = hi - k; s_above = acc; break; }
      acc += c;
    }
  }
  __syncthreads();
  *total = s_total;
  *bin = s_bin;
  *above = s_above;
}

// find the exponent bin of the (b+1)-th largest; b = m - (diagonal count if excluded)
__global__ __launch_bounds__(1024) void k_sel_find_exp(unsigned long long* hist,
                                                       int excl_diag, int64_t m, int signed_keys,
                                                       double* thr, DevState* st) {
  if (!st->any_active || !st->iter_active) return;
  const long long b = m - (excl_diag ? st->sel_diag : 0);
  long long total, above;
  int bin;
  const int nb = signed_keys ? 4096 : 2048;
  find_bin_desc(hist, nb, b + 1, &total, &bin, &above);
  // every read of the histogram is done (the search ends on a barrier): clear it for the
  // first pass over the collected keys (the bins above nb were never written)
  for (int i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0;
  if (threadIdx.x != 0) return;
  st->sel_count = 0;
  if (b < 0) {                      // cap below the diagonal count: keep only the diagonal
    st->sel_done = 1;
    *thr = INFINITY;
    thr[2] = INFINITY;
    return;
  }
  if (total <= b) {                  // |supp| within the cap: nothing to drop
    st->sel_done = 1;
    *thr = signed_keys ? -INFINITY : 0.0;
    thr[2] = *thr;
    // candidates left out below a floor would have to be kept: run again without it
    const bool isM = thr == &st->thrM;
    if ((isM ? st->belowM : st->belowP) > 0) st->redo = 1;
    return;
  }
  st->sel_prefix = (unsigned long long)bin << 52;
  st->sel_rank = (b + 1) - above;
  st->sel_done = 0;
}

// keys whose exponent bin is the selected one, staged in LDS (one stage per one-wave
// workgroup) and flushed to the global buffer with one atomic reservation per flush
constexpr int kStage = 1024;
template <typename T, bool SC>
__global__ __launch_bounds__(SPAI_WAVE) void k_sel_collect(Pair<T> Xp, const double* sc,
                                                           int excl_diag,
                                                           unsigned long long* selbuf,
                                                           int64_t n, DevState* st) {
  if (!st->any_active || !st->iter_active || st->sel_done) return;
  __shared__ unsigned long long stage[kStage];
  const Cols<T> X = Xp.nxt();
  const unsigned long long want = st->sel_prefix >> 52;
  const int lane = lane_id();
  int cnt = 0;                                    // staged keys (wave-uniform)
  auto flush = [&]() {
    __syncthreads();
    unsigned long long base = 0;
    if (lane == 0 && cnt) base = atomicAdd(&st->sel_count, (unsigned long long)cnt);
    base = __shfl(base, 0, SPAI_WAVE);
    for (int i = lane; i < cnt; i += SPAI_WAVE) selbuf[base + i] = stage[i];
    __syncthreads();
    cnt = 0;
  };
  const int64_t ng = (n + 63) / 64;
  for (int64_t gi = blockIdx.x; gi < ng; gi += gridDim.x) {
    const Group64 g = group_load(X, gi * 64, n);
    for (int x0 = 0; x0 < g.T; x0 += SPAI_WAVE * kGU) {
      if (cnt > kStage - SPAI_WAVE * kGU) flush();
      int idx[kGU];
      T val[kGU];
      double sv[kGU];
      bool ok[kGU];
      int col[kGU];
#pragma unroll
      for (int u = 0; u < kGU; ++u) {
        const int x = x0 + u * SPAI_WAVE + lane;
        const int xc = min(x, g.T - 1);            // all lanes shuffle together
        const int c = group_col(g, xc);
        const int64_t src = group_src(g, c, xc);
        ok[u] = x < g.T;
        idx[u] = -1;
        val[u] = (T)0;
        sv[u] = 0.0;
        col[u] = c;
        if (ok[u]) {
          if (excl_diag) idx[u] = X.idx[src];
          if constexpr (SC) sv[u] = sc[src]; else val[u] = X.val[src];
        }
      }
#pragma unroll
      for (int u = 0; u < kGU; ++u) {
        bool take = false;
        unsigned long long key = 0;
        if (ok[u] && !(excl_diag && idx[u] == (int)(g.j0 + col[u]))) {
          key = SC ? ord_key(sv[u]) : mag_key((double)val[u]);
          take = (key >> 52) == want;
        }
        const unsigned long long bal = __ballot(take);
        if (take) stage[cnt + __popcll(bal & lanemask_lt())] = key;
        cnt += __popcll(bal);
      }
    }
  }
  flush();
}

// histogram of 13 key bits at `shift` among the collected keys matching the prefix above
__global__ __launch_bounds__(kSelThreads) void k_sel_hist_buf(const unsigned long long* selbuf,
                                                              int shift,
                                                              unsigned long long* hist,
                                                              DevState* st) {
  if (!st->any_active || !st->iter_active || st->sel_done) return;
  __shared__ unsigned int h[8192];
  for (int i = threadIdx.x; i < 8192; i += kSelThreads) h[i] = 0;
  __syncthreads();
  const unsigned long long cnt = st->sel_count;
  const int hi = shift + 13;
  const unsigned long long pre = st->sel_prefix >> hi;
  for (unsigned long long i = (unsigned long long)blockIdx.x * kSelThreads + threadIdx.x; i < cnt;
       i += (unsigned long long)gridDim.x * kSelThreads) {
    const unsigned long long key = selbuf[i];
    if ((key >> hi) == pre) atomicAdd(&h[(int)((key >> shift) & 8191ull)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 8192; i += kSelThreads)
    if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

__global__ __launch_bounds__(1024) void k_sel_find_buf(unsigned long long* hist, int shift,
                                                       int last, double eta, int signed_keys,
                                                       double* thr, DevState* st) {
  if (!st->any_active || !st->iter_active || st->sel_done) return;
  const long long rank = st->sel_rank;
  long long total, above;
  int bin;
  find_bin_desc(hist, 8192, rank, &total, &bin, &above);
  for (int i = threadIdx.x; i < 8192; i += blockDim.x) hist[i] = 0;   // for the next pass
  if (threadIdx.x != 0) return;
  if (bin >= 0) {
    st->sel_prefix |= (unsigned long long)bin << shift;
    st->sel_rank = rank - above;
  }
  if (shift == last) {                 // the bits below hold no candidate's bit
    double t;
    if (signed_keys) {                 // keep score > t + eta |t|
      t = ord_value(st->sel_prefix);
      *thr = t + eta * fabs(t);
    } else {                           // keep |x| > t (1 + eta)
      t = __longlong_as_double((long long)st->sel_prefix);
      *thr = t * (1.0 + eta);
      // every candidate the cut keeps or counts in its tie band must have been written:
      // t (1 - eta) must clear the floor under which candidates were left out
      const bool isM = thr == &st->thrM;
      const double fl = isM ? st->floorM : st->floorP;
      if ((isM ? st->belowM : st->belowP) > 0 && t * (1.0 - eta) < fl) st->redo = 1;
    }
    thr[2] = t;                        // rawM / rawP, two doubles after thrM / thrP
    st->sel_done = 1;
  }
}

__global__ void k_sel_reset(unsigned long long* hist, int nbins, DevState* st) {
  for (int i = threadIdx.x; i < nbins; i += blockDim.x) hist[i] = 0;
  if (threadIdx.x == 0) {
    st->sel_diag = 0;
    st->sel_count = 0;
    st->sel_done = 0;
  }
}

template <typename T>
void launch_global_select(Pair<T> X, int exclude_diag, int64_t m, double eta, int which,
                          unsigned long long* hist, unsigned long long* selbuf, int64_t n,
                          DevState* st, hipStream_t s, const double* score) {
  double* thr = which == 0 ? &st->thrM : &st->thrP;
  const int sk = score ? 1 : 0;
  hipLaunchKernelGGL(k_sel_reset, dim3(1), dim3(1024), 0, s, hist, 8192, st);
  const int ng = (int)std::min<int64_t>((n + 63) / 64, 1 << 30);
  // the magnitude passes run below full occupancy, as the compaction does: 4 four-wave
  // histogram workgroups and 12 collecting waves per compute unit took 0.55 ms per
  // iteration at 96^3 against 0.62 ms at the occupancy limit
  if (score)
    hipLaunchKernelGGL(
        (k_sel_hist_exp<T, true>),
        dim3(std::min((ng + 3) / 4, resident_grid(k_sel_hist_exp<T, true>, 0, 4 * SPAI_WAVE))),
        dim3(4 * SPAI_WAVE), 0, s, X, score, exclude_diag, hist, n, st);
  else
    hipLaunchKernelGGL(
        (k_sel_hist_exp<T, false>),
        dim3(std::min({(ng + 3) / 4, resident_grid(k_sel_hist_exp<T, false>, 0, 4 * SPAI_WAVE),
                       per_cu_grid(4)})),
        dim3(4 * SPAI_WAVE), 0, s, X, score, exclude_diag, hist, n, st);
  hipLaunchKernelGGL(k_sel_find_exp, dim3(1), dim3(1024), 0, s, hist, exclude_diag, m, sk, thr,
                     st);
  if (score)
    hipLaunchKernelGGL((k_sel_collect<T, true>),
                       dim3(std::min(ng, resident_grid(k_sel_collect<T, true>, 0))),
                       dim3(SPAI_WAVE), 0, s, X, score, exclude_diag, selbuf, n, st);
  else
    hipLaunchKernelGGL((k_sel_collect<T, false>),
                       dim3(std::min({ng, resident_grid(k_sel_collect<T, false>, 0),
                                      per_cu_grid(12)})),
                       dim3(SPAI_WAVE), 0, s, X, score, exclude_diag, selbuf, n, st);
  // float candidates widened to double have zero in the low 29 mantissa bits, so the
  // passes over bits 0..25 would each select bin 0: they stop after bits 26..38
  const int last = (sizeof(T) == 4 && !score) ? 26 : 0;
  for (int shift = 39; shift >= last; shift -= 13) {
    hipLaunchKernelGGL(k_sel_hist_buf, dim3(256), dim3(kSelThreads), 0, s, selbuf, shift, hist,
                       st);
    hipLaunchKernelGGL(k_sel_find_buf, dim3(1), dim3(1024), 0, s, hist, shift, last, eta, sk,
                       thr, st);
  }
}

// ============================================================================
// heuristic drop score of Appendix A (global cap, optional)
// ============================================================================
//
// For the candidates M~ (symmetrized, small entries dropped) in M.nxt(): per entry
//   s_kl = m_kl^2 ||A e_k||^2 + 2 m_kl (A R~)_kl,   R~ = I - A M~,
// the change of ||R~||_F^2 from dropping that entry alone, and per symmetric pair
//   sigma_kl = s_kl + s_lk
// (the change from dropping the pair; its entries lie in different columns and do not
// couple).  Column l: r~_l = e_l - A m~_l is formed in LDS (keys sorted, values beside
// them), then each candidate row k pulls row k of A against it, which also gives
// ||A e_k||^2 = sum_t a_kt^2 (A symmetric).

template <typename T, bool GS>
__global__ __launch_bounds__(SPAI_WAVE) void k_score(Csr A, Pair<T> Mp, double* sc, BigList big,
                                                     DevState* st, int tier, int L, int H) {
  if (!st->any_active || !st->iter_active) return;
  extern __shared__ char smem[];
  const bool ell = A.eshift >= 0;
  Carve cv(tile_base<GS>(smem, big));
  int* s_mi = cv.take<int>(L);
  int* s_keys = cv.take<int>(H);         // hash set, then the sorted rows of r~_l
  double* s_mv = cv.take<double>(L);
  int* s_mk = cv.take<int>(2 * L);       // position map of m~_l's rows
  unsigned* s_mp = cv.take<unsigned>(2 * L);
  double* s_rv = cv.take<double>(H / 2); // r~_l values beside the sorted keys
  int* s_pre = ell ? nullptr : cv.take<int>(L);
  int64_t* s_rs = ell ? nullptr : cv.take<int64_t>(L);
  const int lane = lane_id();
  const Cols<T> Mc = Mp.nxt();
  const int limit = H / 2 - 1;

  auto body = [&](int64_t j) {
    const int64_t mb = Mc.beg[j];
    const int lm = Mc.len[j];
    if (lm > L) {
      defer_column(tier, big, st, j);
      return;
    }
    const int hs = next_pow2(max(2 * lm, 64));
    ks_clear(s_keys, H);
    lm_clear(s_mk, s_mp, hs);
    tile_sync<GS>();
    for (int e = lane; e < lm; e += SPAI_WAVE) {
      const int i = Mc.idx[mb + e];
      s_mi[e] = i;
      s_mv[e] = (double)Mc.val[mb + e];
      lm_put(s_mk, s_mp, hs, i, 0, e);
    }
    tile_sync<GS>();
    int tot = 0;
    if (!ell) {
      tot = degree_prefix(A, s_mi, lm, s_pre, s_rs);
      tile_sync<GS>();
    }
    int kd[1] = {lane == 0 ? (int)j : -1};
    int nk = wave_sum_int(ks_insert_batch<1>(s_keys, H, kd));
    nk = insert_products(A, s_mi, lm, s_pre, s_rs, tot, s_keys, H, nk, limit);
    tile_sync<GS>();
    if (nk > limit) {
      defer_column(tier, big, st, j);
      tile_sync<GS>();
      return;
    }
    const int nu = ks_sort_inplace(s_keys, H);
    tile_sync<GS>();
    double sum[1];
    int key[1];
    pull_rows<1>(
        A, s_keys, nu,
        [&](int c, int t) {
          sum[c] = 0.0;
          key[c] = s_keys[t];
        },
        [&](int c, const int (&cols)[8], const double (&vals)[8]) {
          unsigned pw[8];
          lm_find<8>(s_mk, s_mp, hs, cols, pw);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const unsigned e = pw[k] & kNoPos;
            if (e != kNoPos) sum[c] += vals[k] * s_mv[e];
          }
        },
        [&](int c, int t) { s_rv[t] = ((key[c] == (int)j) ? 1.0 : 0.0) - sum[c]; });
    tile_sync<GS>();
    // per candidate row k: (A r~_l)_k and ||A e_k||^2 from row k of A
    for (int e = lane; e < lm; e += SPAI_WAVE) {
      const int k = s_mi[e];
      const double m = s_mv[e];
      int64_t q0, q1;
      row_span(A, k, q0, q1);
      double ar = 0.0, n2 = 0.0;
      for (int64_t q = q0; q < q1; q += 8) {
        int cols[8];
        double vals[8];
        load_chunk(A, q, q1, cols, vals);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          if (cols[c] < 0) continue;
          n2 += vals[c] * vals[c];
          const int pos = bsearch_idx(s_keys, nu, cols[c]);
          if (pos >= 0) ar += vals[c] * s_rv[pos];
        }
        if (cols[7] < 0) break;
      }
      sc[mb + e] = (m * m) * n2 + (2.0 * m) * ar;
    }
    tile_sync<GS>();
  };

  if (tier == 0) {
    ColumnWalk w(A.n, blockIdx.x, gridDim.x);
    for (int64_t j = w.begin; j < w.end; j += w.step) body(j);
  } else if (tier == 1) {
    const int cnt = *big.count;
    for (int t = blockIdx.x; t < cnt; t += gridDim.x) body(big.list[t]);
  } else {
    const int cnt = *big.count2;
    for (int t = blockIdx.x; t < cnt; t += gridDim.x) body(big.list2[t]);
  }
}

static size_t score_lds(Tile t, bool ell) {
  return (size_t)t.L * 4 + (size_t)t.H * 4 + (size_t)t.L * 8 + (size_t)t.L * 16 +
         (size_t)(t.H / 2) * 8 + (ell ? 0 : (size_t)t.L * 12) + 128;
}

size_t score_tile_bytes(Tile t, bool ell) { return score_lds(t, ell); }

// sigma at entry (k, l) of the candidates: s_kl + s_lk, the partner found by binary
// search in column k (the candidates are exactly symmetric); the diagonal keeps s_kk
template <typename T>
__global__ __launch_bounds__(SPAI_WAVE) void k_score_pair(Pair<T> Mp, const double* sc,
                                                          double* sig, int64_t n,
                                                          DevState* st) {
  if (!st->any_active || !st->iter_active) return;
  const Cols<T> X = Mp.nxt();
  const int lane = lane_id();
  const int64_t ng = (n + 63) / 64;
  for (int64_t gi = blockIdx.x; gi < ng; gi += gridDim.x) {
    const Group64 g = group_load(X, gi * 64, n);
    for (int x0 = 0; x0 < g.T; x0 += SPAI_WAVE) {
      const int x = x0 + lane;
      const int xc = min(x, g.T - 1);              // all lanes shuffle together
      const int c = group_col(g, xc);
      const int64_t src = group_src(g, c, xc);
      if (x >= g.T) continue;
      const int l = (int)(g.j0 + c);
      const int k = X.idx[src];
      double v = sc[src];
      if (k != l) {
        const int64_t kb = X.beg[k];
        const int p = bsearch_idx(X.idx + kb, X.len[k], l);
        if (p >= 0) v = v + sc[kb + p];
        else atomicOr(&st->err, 4);              // not symmetric: cannot happen
      }
      sig[src] = v;
    }
  }
}

template <typename T>
void launch_score(const Csr& A, Pair<T> M, double* sc, double* sig, BigList big, DevState* st,
                  Tile small, Tile large, Tile huge, int64_t n, hipStream_t s) {
  const bool ell = A.eshift >= 0;
  hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(1), 0, s, big.count, big.count2);
  hipLaunchKernelGGL((k_score<T, false>), dim3(resident_grid(k_score<T, false>, score_lds(small, ell))),
                     dim3(SPAI_WAVE), score_lds(small, ell), s, A, M, sc, big, st, 0, small.L,
                     small.H);
  hipLaunchKernelGGL((k_score<T, false>), dim3(256), dim3(SPAI_WAVE), score_lds(large, ell), s, A,
                     M, sc, big, st, 1, large.L, large.H);
  hipLaunchKernelGGL((k_score<T, true>), dim3(big.grid2), dim3(SPAI_WAVE), 0, s, A, M, sc, big, st,
                     2, huge.L, huge.H);
  const int ng = (int)std::min<int64_t>((n + 63) / 64, 1 << 30);
  hipLaunchKernelGGL(k_score_pair<T>, dim3(std::min(ng, resident_grid(k_score_pair<T>, 0))),
                     dim3(SPAI_WAVE), 0, s, M, sc, sig, n, st);
}

// ============================================================================
// keep rule + in-place compaction
// ============================================================================

// Keep rule and in-place compaction, 64 columns per one-wave workgroup (grouped walk).
// Each round of 64 consecutive entries takes a ballot of the kept ones; a kept
// entry's place in its column is the column's running count (s_run, LDS) plus the
// kept entries before it in the same column segment of the round.  It moves only
// toward the column start, and a batch's entries are all loaded before any is written.
// SC: the keys are the scores stored beside the candidates (score non-null).
template <typename T, bool SC>
__global__ __launch_bounds__(SPAI_WAVE) void k_compact(Pair<T> Xp, int kind, int colcap, int sym,
                                                       int global, const double* tcol,
                                                       const double* gthr, double eta, int64_t n,
                                                       DevState* st, const double* score) {
  if (!st->any_active || !st->iter_active) return;
  __shared__ int s_run[SPAI_WAVE];
  const Cols<T> X = Xp.nxt();
  const int lane = lane_id();
  const double gt = global ? *gthr : 0.0;
  const double graw = global ? gthr[2] : 0.0;      // the cut before the tie factor
  const bool need_tk = colcap && ((kind == 0 && sym) || kind == 2);
  unsigned long long kept = 0, seen = 0, band = 0;
  const int64_t ng = (n + 63) / 64;
  for (int64_t gi = blockIdx.x; gi < ng; gi += gridDim.x) {
    const Group64 g = group_load(X, gi * 64, n);
    const int64_t jl = g.j0 + lane;
    const double tl = (colcap && jl < n) ? tcol[jl] : 0.0;   // this lane's column threshold
    s_run[lane] = 0;
    __syncthreads();
    // A batch's entries are loaded before the stores of the batch before it go out: one
    // counter tracks both loads and stores and completes in order, so the first use of
    // a batch loaded after those stores would also wait for them to be written.  It is
    // safe because entries only move toward their column's start: no store of a batch
    // reaches a later batch's entries.
    constexpr int NSV = SC ? kGUc : 1;               // score keys (none unless SC)
    int col[kGUc], idx[kGUc], ncol[kGUc], nidx[kGUc];
    T val[kGUc], nval[kGUc];
    double sv[NSV], nsv[NSV];
    auto load_batch = [&](int x0, int (&c_)[kGUc], int (&i_)[kGUc], T (&v_)[kGUc],
                          double (&s_)[NSV]) {
#pragma unroll
      for (int u = 0; u < kGUc; ++u) {
        const int x = x0 + u * SPAI_WAVE + lane;
        const int xc = min(x, g.T - 1);            // all lanes shuffle together
        const int c = group_col(g, xc);
        const int64_t src = group_src(g, c, xc);
        c_[u] = c;
        i_[u] = -1;
        v_[u] = (T)0;
        if constexpr (SC) s_[u] = 0.0;
        if (x < g.T) {
          i_[u] = X.idx[src];
          v_[u] = X.val[src];
          if constexpr (SC) s_[u] = score[src];
        }
      }
    };
    if (g.T > 0) load_batch(0, col, idx, val, sv);
    for (int x0 = 0; x0 < g.T; x0 += SPAI_WAVE * kGUc) {
      const bool more = x0 + SPAI_WAVE * kGUc < g.T;   // wave-uniform
      if (more) load_batch(x0 + SPAI_WAVE * kGUc, ncol, nidx, nval, nsv);
      double tk[kGUc];
#pragma unroll
      for (int u = 0; u < kGUc; ++u) tk[u] = 0.0;
      if (need_tk) {
#pragma unroll
        for (int u = 0; u < kGUc; ++u)
          if (idx[u] >= 0) tk[u] = tcol[idx[u]];
      }
#pragma unroll
      for (int u = 0; u < kGUc; ++u) {
        const int rb = x0 + u * SPAI_WAVE;           // flat index of lane 0's entry
        const int x = rb + lane;
        const bool ok = x < g.T;
        const int c = col[u];
        const int j = (int)(g.j0 + c);
        // every shuffle below runs on all lanes
        const double tcj = __shfl(tl, c, SPAI_WAVE);
        const int64_t cbc = __shfl(g.cb, c, SPAI_WAVE);
        const int exc = __shfl(g.ex, c, SPAI_WAVE);
        bool keep = false;
        if (ok) {
          const int k = idx[u];
          const double a = fabs((double)val[u]);
          if (kind == 0 && k == j) {
            keep = true;
          } else if (global) {
            double key = a;
            if constexpr (SC) key = sv[u];
            keep = key > gt;
            // dropped within the tie band of the cut (a relative eta below it)
            band += (!keep && key >= graw - eta * fabs(graw)) ? 1ull : 0ull;
          } else if (colcap) {
            double t = tcj;
            if (kind == 0 && sym) t = fmax(t, tk[u]);
            if (kind == 2) t = tk[u];
            keep = a > t * (1.0 + eta);
            band += (!keep && t > 0.0 && a >= t * (1.0 - eta)) ? 1ull : 0ull;
          } else {
            keep = true;
          }
        }
        const unsigned long long bal = __ballot(keep);
        const int seg0 = max(0, exc - rb);          // first lane of my column in this round
        const unsigned long long below = lanemask_lt() & ~((seg0 >= 64) ? ~0ull : ((1ull << seg0) - 1ull));
        const int before = __popcll(bal & below);
        const int base = s_run[c];
        if (keep) {
          const int64_t pos = cbc + base + before;
          X.idx[pos] = idx[u];
          X.val[pos] = val[u];
        }
        const int cn = __shfl_down(c, 1, SPAI_WAVE);
        const bool last = ok && (lane == SPAI_WAVE - 1 || x + 1 >= g.T || cn != c);
        __syncthreads();
        if (last) s_run[c] = base + before + (keep ? 1 : 0);
        __syncthreads();
      }
      if (more) {
#pragma unroll
        for (int u = 0; u < kGUc; ++u) {
          col[u] = ncol[u];
          idx[u] = nidx[u];
          val[u] = nval[u];
          if constexpr (SC) sv[u] = nsv[u];
        }
      }
    }
    if (jl < n) {
      X.len[jl] = s_run[lane];
      kept += (unsigned long long)s_run[lane];
      seen += (unsigned long long)g.cl;
    }
    __syncthreads();
  }
  kept = (unsigned long long)wave_sum_ll((long long)kept);
  seen = (unsigned long long)wave_sum_ll((long long)seen);
  band = (unsigned long long)wave_sum_ll((long long)band);
  if (lane == 0 && blockIdx.x < kCntSlots) {
    st->cnt[(3 + kind) * kCntSlots + blockIdx.x] += kept;
    st->cnt[kind * kCntSlots + blockIdx.x] += seen;
  }
  // the iteration's record (M and P; P^T mirrors P); integer sums, so the order of the
  // workgroups' atomics does not matter
  const int ri = st->rec_i;
  if (lane == 0 && kind < 2 && st->rec && ri >= 0 && ri < st->rec_cap) {
    unsigned long long* r = st->rec + (int64_t)ri * kRec + 3 * kind;
    // candidates: the ones written plus (once) those the update left out below a floor
    const unsigned long long below = blockIdx.x == 0 ? (kind == 0 ? st->belowM : st->belowP) : 0;
    atomicAdd(&r[0], kept);
    atomicAdd(&r[1], seen + below);
    atomicAdd(&r[2], band);
  }
}

template <typename T>
void launch_compact(Pair<T> X, int kind, int colcap, int sym, int global, const double* tcol,
                    double eta, int64_t n, DevState* st, hipStream_t s, const double* score) {
  const double* gthr = kind == 0 ? &st->thrM : &st->thrP;
  const int ng = (int)std::min<int64_t>((n + 63) / 64, 1 << 30);
  if (score)
    hipLaunchKernelGGL((k_compact<T, true>), dim3(std::min(ng, resident_grid(k_compact<T, true>, 0))),
                       dim3(SPAI_WAVE), 0, s, X, kind, colcap, sym, global, tcol, gthr, eta, n, st,
                       score);
  else   // two workgroups per SIMD: more waves in flight made the pass slower at 96^3
         // (0.52 ms at 8 per compute unit, 0.62 at 16, 0.66 at 4)
    hipLaunchKernelGGL((k_compact<T, false>),
                       dim3(std::min({ng, resident_grid(k_compact<T, false>, 0), per_cu_grid(8)})),
                       dim3(SPAI_WAVE), 0, s, X, kind, colcap, sym, global, tcol, gthr, eta, n, st,
                       score);
}

// ============================================================================
// scalar steps (one thread per segment)
// ============================================================================

// step sizes from the reduced dots; decides whether this iteration runs
__global__ void k_scal_step(int method, Seg seg, const double* red, DevState* st) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= seg.nseg) return;
  SegState& g = seg.st[s];
  if (s == 0) st->rec_i = st->rec_next++;   // the drops of this iteration go to this record
  const double* d = red + (int64_t)s * kND;
  for (int i = 0; i < kND; ++i) g.dots[i] = d[i];
  if (!g.stop) {
    if (method == kMR) {
      if (!(d[1] > 0.0)) {              // A R = 0: R = 0, converged
        g.stop = 1;
        g.status = 1;
      } else {
        const double alpha = d[0] / d[1];
        g.coef[0] = alpha; g.coef[1] = 0.0; g.coef[2] = 0.0; g.coef[3] = 0.0;
        g.step1 = alpha;
        g.step2 = 0.0;
      }
    } else if (method == kCG) {
      // rz = (R, Z)_F (Algorithm 7; = ||R||_F^2 unweighted, Algorithm 3)
      if (!(g.rz > 0.0)) {
        g.stop = 1;
        g.status = 1;
      } else if (!(d[5] > 0.0)) {       // (P, A P) <= 0: A is not SPD, or P = 0
        g.stop = 1;
        g.status = 3;
      } else {
        const double alpha = g.rz / d[5];
        g.coef[0] = alpha; g.coef[1] = 0.0;
        g.step1 = alpha;
      }
    } else {  // LOMR (Theorem 4.2)
      const double r_ar = d[0], ar_ar = d[1], ar_ap = d[2], r_ap = d[3], ap_ap = d[4];
      if (!(ar_ar > 0.0)) {
        g.stop = 1;
        g.status = 1;
      } else {
        double delta, gamma;
        if (g.first) {
          delta = r_ar / ar_ar;
          gamma = 1.0;
          g.first = 0;
        } else {
          const double c = ar_ar * ap_ap - ar_ap * ar_ap;
          if (!(c > 1e-14 * ar_ar * ap_ap)) {
            delta = r_ar / ar_ar;
            gamma = 0.0;
            g.mr_fallbacks += 1;
          } else {
            delta = (ap_ap * r_ar - ar_ap * r_ap) / c;
            gamma = (ar_ar * r_ap - ar_ap * r_ar) / c;
          }
        }
        g.coef[0] = delta; g.coef[1] = gamma; g.coef[2] = delta; g.coef[3] = gamma;
        g.step1 = delta;
        g.step2 = gamma;
      }
    }
  }
  if (g.stop) {                         // carry a stopped matrix through unchanged
    g.coef[0] = 0.0; g.coef[1] = 0.0; g.coef[2] = 0.0; g.coef[3] = 1.0;
  }
}

// any segment still running -> the iteration runs
__global__ void k_any_active(Seg seg, DevState* st) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < seg.nseg; s += blockDim.x)
    if (!seg.st[s].stop) atomicOr(&any, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    st->iter_active = any;
    st->any_active = any;
    st->nnz_m = 0;
    st->nnz_p = 0;
  }
}

void launch_scal_step(int method, const Seg& seg, const double* red, DevState* st,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_scal_step, dim3((seg.nseg + 255) / 256), dim3(256), 0, s, method, seg, red,
                     st);
  hipLaunchKernelGGL(k_any_active, dim3(1), dim3(256), 0, s, seg, st);
}

// after R_{i+1}: record ||R||, test the stopping rule, CG's beta
__global__ void k_scal_post(int method, Seg seg, const double* red, const double* red_rz,
                            double tol, double* hist, int hist_cap, int setup, DevState* st) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= seg.nseg) return;
  if (!st->iter_active) return;
  SegState& g = seg.st[s];
  const double rr_new = red[s];
  const double rz_new = red_rz ? red_rz[s] : rr_new;
  const double rn = sqrt(rr_new);
  if (setup) {                          // R_0: no iteration counted
    g.rr = rr_new;
    g.rz = rz_new;
    g.last_resid = rn;
    g.coef[0] = 0.0; g.coef[1] = 0.0; g.coef[2] = 1.0; g.coef[3] = 0.0;   // CG: P_0 = R_0
    if (tol > 0.0 && rn * g.inv_sqrt_n <= tol) { g.stop = 1; g.status = 1; }
    return;
  }
  if (g.stop) return;
  g.last_resid = rn;
  if (hist && g.iters < hist_cap) hist[(int64_t)s * hist_cap + g.iters] = rn;
  g.iters += 1;
  if (method == kCG) {
    const double beta = g.rz > 0.0 ? rz_new / g.rz : 0.0;
    g.coef[2] = 1.0;
    g.coef[3] = beta;
    g.step2 = beta;
  }
  g.rr = rr_new;
  g.rz = rz_new;
  if (tol > 0.0 && rn * g.inv_sqrt_n <= tol) {
    g.stop = 1;
    g.status = 1;
  }
}

void launch_scal_post(int method, const Seg& seg, const double* red, const double* red_rz,
                      double tol, double* hist, int hist_cap, int setup, DevState* st,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_scal_post, dim3((seg.nseg + 255) / 256), dim3(256), 0, s, method, seg, red,
                     red_rz, tol, hist, hist_cap, setup, st);
}

// the end of a drop in one launch: the new M (doM) and P (doP) become current, and with
// floors the next iteration's floors are set
__global__ void k_drop_finish(DevState* st, int doM, int doP, int floors, double frac) {
  if (!st->iter_active) return;
  if (doM) st->curM ^= 1;
  if (doP) st->curP ^= 1;
  if (floors) floor_next_body(st, doM, doP, frac);
}

void launch_drop_finish(DevState* st, int doM, int doP, int floors, double frac, hipStream_t s) {
  hipLaunchKernelGGL(k_drop_finish, dim3(1), dim3(1), 0, s, st, doM, doP, floors, frac);
}

// ---- explicit instantiations
#define SPAI_INST(T)                                                                               \
  template void launch_init_m<T>(int64_t, Cols<T>, const double*, const Seg&, hipStream_t);       \
  template void launch_zero_cols<T>(int64_t, Cols<T>, hipStream_t);                               \
  template void launch_bound_resid<T>(const Csr&, Pair<T>, int64_t*, int64_t, const DevState*,    \
                                      hipStream_t);                                               \
  template void launch_resid<T>(const Csr&, Pair<T>, Cols<T>, const int64_t*, const int64_t*,    \
                                double*, int, double*, BigList, DevState*, Tile, Tile, Tile,      \
                                hipStream_t);                                                     \
  template void launch_dots<T>(const Csr&, Cols<T>, Pair<T>, int, int, int, double*, BigList,     \
                               DevState*, Tile, Tile, Tile, hipStream_t);                         \
  template void launch_bound_impl<T>(const Csr&, Cols<T>, Cols<T>, Pair<T>, int, int64_t*,       \
                                     int64_t, const DevState*, hipStream_t);                      \
  template void launch_resid_impl<T>(const Csr&, Cols<T>, Cols<T>, Pair<T>, int, int, const Seg&, \
                                     const int64_t*, const int64_t*, Cols<T>, Cols<T>, int,       \
                                     double*, double*, BigList, DevState*, Tile, Tile, Tile,      \
                                     hipStream_t);                                                \
  template void launch_copy_cols<T>(Cols<T>, Cols<T>, int64_t, const int64_t*, const DevState*,   \
                                    hipStream_t);                                                 \
  template void launch_bound_update<T>(const Csr&, Pair<T>, Cols<T>, Pair<T>, Pair<T>, UpdMode,   \
                                       int64_t*, int64_t, const DevState*, hipStream_t);          \
  template void launch_update<T>(const Csr&, Pair<T>, Cols<T>, Pair<T>, Pair<T>, UpdMode,         \
                                 const int64_t*, const int64_t*, const int32_t*, double*,         \
                                 double*, BigList, const Seg&, DevState*, Tile, Tile, Tile,       \
                                 hipStream_t, bool);                                              \
  template void launch_global_select<T>(Pair<T>, int, int64_t, double, int, unsigned long long*,  \
                                        unsigned long long*, int64_t, DevState*, hipStream_t,     \
                                        const double*);                                           \
  template void launch_compact<T>(Pair<T>, int, int, int, int, const double*, double, int64_t,    \
                                  DevState*, hipStream_t, const double*);                         \
  template void launch_score<T>(const Csr&, Pair<T>, double*, double*, BigList, DevState*, Tile,  \
                                Tile, Tile, int64_t, hipStream_t);

SPAI_INST(double)
SPAI_INST(float)

}  // namespace spai
