// spai_pcg.hip — preconditioned CG with the SPAI as preconditioner (z = M r), many
// right-hand sides at once (the vector solves of Section 7, Experiments 04 and 06).
//
// Every right-hand side runs its own textbook recurrence in float64; the block of
// vectors is row-major (n x nrhs, the nrhs values of a row contiguous), so one
// wavefront reads the 64 values of a row of X as one coalesced 512-byte line and the
// SpMM gathers whole rows (with at most 32 right-hand sides, pow2(nrhs) lanes share a
// row instead).  Frobenius-free per-RHS dots are reduced per workgroup in
// a fixed order and then across workgroups in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "spai.h"
#include "spai_dev.hpp"
#include "spai_host.hpp"

namespace spai {
namespace {

constexpr int kThreads = 256;
constexpr int kGrid = 2048;

using Mat = PcgMat;
typedef double d2v __attribute__((ext_vector_type(2)));   // for nontemporal 16-byte stores

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// a wave-uniform 64-bit value moved to scalar registers
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (int64_t)(unsigned)lo;
}

enum { kLayEll = 0, kLayPad = 1, kLayCsr = 2 };

template <int LAY>
__device__ __forceinline__ int64_t row_lo(const Mat& A, int64_t i) {
  if (LAY == kLayEll) return i << A.eshift;
  if (LAY == kLayPad) return A.beg[i];
  return A.rowptr[i];
}
template <int LAY>
__device__ __forceinline__ int64_t row_hi(const Mat& A, int64_t i) {
  if (LAY == kLayEll) return (i + 1) << A.eshift;
  if (LAY == kLayPad) return A.beg[i] + A.len[i];
  return A.rowptr[i + 1];
}
template <typename VT>
__device__ __forceinline__ VT entry_val(const Mat& A, int64_t q) {
  if constexpr (sizeof(VT) == 4) return A.val32[q];
  else return A.val[q];
}
__device__ __forceinline__ float readlane_val(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane_val(double v, int l) { return readlane_f64(v, l); }

// G gathers of one row, all issued before any is used: entry e0 + k of the row (held
// one per lane in cc) selects row col of X, whose 64-value piece starting at column c0
// is one 512-byte line; lane k's value sits at byte offset loff.  Entries past cnt
// repeat the last one, so every load is in bounds and there is no branch between them.
template <int G>
__device__ __forceinline__ void gather_row(const double* X, int nrhs, int c0, unsigned loff,
                                           int cc, int e0, int cnt, double (&xs)[G]) {
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const int e = min(e0 + k, cnt - 1);
    const int col = __builtin_amdgcn_readlane(cc, e);
    const char* xrow = (const char*)(X + ((int64_t)col * nrhs + c0));   // uniform base
    xs[k] = *(const double*)(xrow + loff);
  }
}

// y += v_e x_e over the entries e0 .. min(e0 + G, cnt) in order (v_e widened to float64);
// the gathered value of the entry in column `diag` (the row's own index) is kept in xd
template <int G, typename VT>
__device__ __forceinline__ void accumulate_row(double& y, VT cv, int cc, int e0, int cnt,
                                               const double (&xs)[G], int diag, double& xd,
                                               bool& found) {
#pragma unroll
  for (int k = 0; k < G; ++k)
    if (e0 + k < cnt) {
      y += (double)readlane_val(cv, e0 + k) * xs[k];
      if (__builtin_amdgcn_readlane(cc, e0 + k) == diag) {
        xd = xs[k];
        found = true;
      }
    }
}

// Y[:, c0:c0+64) = K X[:, c0:c0+64) and, when dot is set, per-block partials of
// sum_i X[i, r] Y[i, r] (X[i, :] taken from the row's own diagonal gather), stored
// transposed: part[r * gridDim.x + block].
// One wave per row at a time, lane r owning right-hand side c0 + r, so every gather is
// one 512-byte line of X.  The row's entries are loaded by the lanes together (one per
// lane) and broadcast with readlane, so the row's gathers (up to 16 in flight) wait on
// a single entry load; the next row's entries and the descriptor of the row after it
// are loaded while the current row's gathers are in flight.  Row i's sum runs over its
// entries in stored (ascending column) order.  The rows are split into eight
// contiguous ranges, one per XCD (workgroups are dealt round-robin over the XCDs), and
// each wave takes kRowsPerWave consecutive positions of its range.  The launch is not
// persistent: workgroups are dispatched in order as others finish, so the positions in
// flight stay within a few thousand of each other and the rows of X they gather stay in
// the XCD's L2 (a persistent grid whose waves walk the range with a fixed stride drifts
// apart and gathers rows again from beyond L2).
constexpr int kRowsPerWave = 16;

template <typename VT, int LAY>
__global__ __launch_bounds__(kThreads) void k_spmm_wave(Mat A, const double* X, double* Y,
                                                        int dot, int nrhs, int c0,
                                                        const int32_t* order, double* part) {
  if (A.gate && *A.gate == 0) return;                     // every right-hand side stopped
  if (A.ran && c0 == 0 && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(A.ran, 1);
  __shared__ double sh[kThreads];
  constexpr int WPB = kThreads / 64;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t xcd = blockIdx.x & 7, kb = blockIdx.x >> 3, nb = gridDim.x >> 3;
  const int64_t per = (A.n + 7) / 8;
  const int64_t r0 = xcd * per;
  const int64_t r1 = r0 + per < A.n ? r0 + per : A.n;
  (void)nb;
  const int64_t stride = 1;
  const bool on = c0 + lane < nrhs;
  const int64_t cofs = c0 + lane;
  const unsigned loff = on ? (unsigned)lane * 8u : 0u;   // idle lanes re-read column c0
  auto rowof = [&](int64_t k) -> int64_t { return order ? (int64_t)order[k] : k; };
  double acc = 0.0;
  int64_t k = r0 + (kb * WPB + wv) * kRowsPerWave;
  const int64_t kend = k + kRowsPerWave < r1 ? k + kRowsPerWave : r1;
  // position k: row i, its descriptor (a, b) and first 64 entries (ec, ev), one per lane;
  // position k + stride: row ni and descriptor (na, nbe); position k + 2 stride: row mi
  int64_t i = 0, ni = 0, mi = 0, a = 0, b = 0, na = 0, nbe = 0;
  int ec = -1;
  VT ev = 0;
  if (k < kend) {
    i = rowof(k);
    a = row_lo<LAY>(A, i);
    b = row_hi<LAY>(A, i);
    if (a + lane < b) {
      ec = A.col[a + lane];
      ev = entry_val<VT>(A, a + lane);
    }
  }
  if (k + stride < kend) {
    ni = rowof(k + stride);
    na = row_lo<LAY>(A, ni);
    nbe = row_hi<LAY>(A, ni);
  }
  if (k + 2 * stride < kend) mi = rowof(k + 2 * stride);
  for (; k < kend; k += stride) {
    const int64_t kn = k + stride;
    const int cnt = __popcll(__ballot(ec >= 0));   // ELL padding (column -1) sits last
    int nc = -1;
    VT nv = 0;
    int64_t ma = 0, mb = 0, li = 0;
    auto prefetch = [&]() {
      if (kn < kend && na + lane < nbe) {
        nc = A.col[na + lane];
        nv = entry_val<VT>(A, na + lane);
      }
      if (kn + stride < kend) {
        ma = row_lo<LAY>(A, mi);
        mb = row_hi<LAY>(A, mi);
      }
      if (kn + 2 * stride < kend) li = rowof(kn + 2 * stride);
    };
    // X[i, :] for the dot: the row's own (diagonal) gather
    const int diag = dot ? (int)i : -1;
    double xd = 0.0;
    bool found = false;
    double y = 0.0;
    if (cnt == 0) {
      prefetch();
    } else if (cnt <= 8) {
      double xs[8];
      gather_row<8>(X, nrhs, c0, loff, ec, 0, cnt, xs);
      prefetch();
      accumulate_row<8>(y, ev, ec, 0, cnt, xs, diag, xd, found);
    } else {
      double xs[16];
      gather_row<16>(X, nrhs, c0, loff, ec, 0, cnt, xs);
      prefetch();
      accumulate_row<16>(y, ev, ec, 0, cnt, xs, diag, xd, found);
      for (int e0 = 16; e0 < cnt; e0 += 16) {
        gather_row<16>(X, nrhs, c0, loff, ec, e0, cnt, xs);
        accumulate_row<16>(y, ev, ec, e0, cnt, xs, diag, xd, found);
      }
      for (int64_t q = a + 64; q < b; q += 64) {   // rows longer than 64 entries
        int cc = -1;
        VT cv = 0;
        if (q + lane < b) {
          cc = A.col[q + lane];
          cv = entry_val<VT>(A, q + lane);
        }
        const int cn = __popcll(__ballot(cc >= 0));
        if (cn == 0) break;
        for (int e0 = 0; e0 < cn; e0 += 16) {
          gather_row<16>(X, nrhs, c0, loff, cc, e0, cn, xs);
          accumulate_row<16>(y, cv, cc, e0, cn, xs, diag, xd, found);
        }
      }
    }
    if (on) {
      Y[i * nrhs + cofs] = y;
      if (dot) {
        // a row without a diagonal entry loads X[i, :] after all
        const double wv = found ? xd : X[i * nrhs + cofs];
        acc += wv * y;
      }
    }
    ec = nc;
    ev = nv;
    a = na;
    b = nbe;
    na = ma;
    nbe = mb;
    i = ni;
    ni = mi;
    mi = li;
  }
  if (!part) return;
  sh[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < 64 && c0 + (int)threadIdx.x < nrhs) {
    double sum = 0.0;
    for (int w = 0; w < WPB; ++w) sum += sh[w * 64 + threadIdx.x];
    part[(int64_t)(c0 + threadIdx.x) * gridDim.x + blockIdx.x] = sum;
  }
}

// The product for an even number of right-hand sides: two rows per wave at a time,
// lanes 0-31 the row at one position and lanes 32-63 the row at the next, lane l of a
// half owning right-hand sides c0 + 2 (l mod 32) and the one after, so every gather is
// one 16-byte load per lane and one load instruction serves two rows (half the
// address-unit work of k_spmm_wave per row).  A half's row entries are loaded 32 at a
// time (one per lane of the half) and broadcast with readlane; the gathers of both
// rows are issued in groups of four before any is used (groups of eight hold 100
// registers, five waves per SIMD, and the 64-right-hand-side solve at 96^3 took 6%
// longer than with four at six waves) -- of two for A in ELL, whose short rows do best
// with more, smaller groups (350 against 353 ms per solve) --, entries past a row's count
// repeating its last one so every load is in bounds.  Each row's sum runs over its
// entries in stored order, and the dot terms are added in position order, so the rows
// of Y and the dot partials are those of k_spmm_wave bit for bit.  Positions are
// dealt as in k_spmm_wave (eight XCD ranges, kRowsPerWave consecutive positions per
// wave, a non-persistent launch).
template <typename VT, int LAY>
__global__ __launch_bounds__(kThreads) void k_spmm_pair(Mat A, const double* X, double* Y,
                                                        int dot, int nrhs, int c0,
                                                        const int32_t* order, double* part) {
  if (A.gate && *A.gate == 0) return;                     // every right-hand side stopped
  if (A.ran && c0 == 0 && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(A.ran, 1);
  constexpr int G = LAY == kLayEll ? 2 : 4;
  __shared__ double sh[kThreads];
  constexpr int WPB = kThreads / 64;
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int hl = lane & 31;
  const int wv = threadIdx.x >> 6;
  const int64_t xcd = blockIdx.x & 7, kb = blockIdx.x >> 3;
  const int64_t per = (A.n + 7) / 8;
  const int64_t r0 = xcd * per;
  const int64_t r1 = r0 + per < A.n ? r0 + per : A.n;
  const bool on = c0 + 2 * hl < nrhs;
  const unsigned loff = on ? (unsigned)hl * 16u : 0u;   // idle lanes re-read column c0
  auto rowof = [&](int64_t k) -> int64_t { return order ? (int64_t)order[k] : k; };
  double acc0 = 0.0, acc1 = 0.0;
  const int64_t kbeg = r0 + (kb * WPB + wv) * kRowsPerWave;
  const int64_t kend = kbeg + kRowsPerWave < r1 ? kbeg + kRowsPerWave : r1;
  // this half's position k + half: row i, descriptor [a, b), first 32 entries (ec, ev)
  auto load_pos = [&](int64_t p, int64_t& i, int64_t& a, int64_t& b) {
    i = -1;
    a = 0;
    b = 0;
    if (p < kend) {
      i = rowof(p);
      a = row_lo<LAY>(A, i);
      b = row_hi<LAY>(A, i);
    }
  };
  auto load_ent = [&](int64_t a, int64_t b, int& cc, VT& cv) {
    cc = -1;
    cv = 0;
    if (a + hl < b) {
      cc = A.col[a + hl];
      cv = entry_val<VT>(A, a + hl);
    }
  };
  int64_t i, a, b, ni, na, nb;
  int ec, nec = -1;
  VT ev, nev = 0;
  load_pos(kbeg + half, i, a, b);
  load_ent(a, b, ec, ev);
  load_pos(kbeg + 2 + half, ni, na, nb);
  for (int64_t k = kbeg; k < kend; k += 2) {
    const bool has = i >= 0;
    double y0 = 0.0, y1 = 0.0;
    double2 xd = make_double2(0.0, 0.0);
    bool found = false;
    int64_t q0 = 0;                     // entries a + q0 .. a + q0 + 31 are in (ec, ev)
    bool first = true;
    for (;;) {
      const unsigned long long bal = __ballot(ec >= 0);   // ELL padding (column -1) last
      const int cA = __popcll(bal & 0xffffffffull), cB = __popcll(bal >> 32);
      const int cmax = cA > cB ? cA : cB;
      if (first) {                      // the next pair's entries while these are gathered
        load_ent(na, nb, nec, nev);
        first = false;
      }
      if (cmax == 0) break;
      const int cmine = half ? cB : cA;
      for (int e0 = 0; e0 < cmax; e0 += G) {
        double2 xs[G];
        int cs[G];
#pragma unroll
        for (int t = 0; t < G; ++t) {
          const int e = e0 + t;
          const int eA = cA ? min(e, cA - 1) : 0, eB = cB ? min(e, cB - 1) : 0;
          const int colA = __builtin_amdgcn_readlane(ec, eA);
          const int colB = __builtin_amdgcn_readlane(ec, 32 + eB);
          int col = half ? colB : colA;
          cs[t] = col;
          col = col < 0 ? 0 : col;
          const char* xrow = (const char*)(X + ((int64_t)col * nrhs + c0));
          xs[t] = *(const double2*)(xrow + loff);
        }
#pragma unroll
        for (int t = 0; t < G; ++t) {
          const int e = e0 + t;
          const VT vA = readlane_val(ev, e < 32 ? e : 31);
          const VT vB = readlane_val(ev, 32 + (e < 32 ? e : 31));
          if (e < cmine) {
            const double v = (double)(half ? vB : vA);
            y0 += v * xs[t].x;
            y1 += v * xs[t].y;
            if (cs[t] == (int)i) {
              xd = xs[t];
              found = true;
            }
          }
        }
      }
      // rows longer than 32 entries: the next 32 of each half's row
      q0 += 32;
      if (__ballot(a + q0 < b) == 0ull) break;   // every lane takes part in the ballot
      load_ent(a + q0, b, ec, ev);
    }
    double t0 = 0.0, t1 = 0.0;          // this row's terms of the dot
    if (has && on) {
      // stored nontemporally: the next kernel reads Y once
      d2v* yr = (d2v*)(Y + (i * nrhs + c0 + 2 * hl));
      d2v yv;
      yv.x = y0;
      yv.y = y1;
      __builtin_nontemporal_store(yv, yr);
      if (dot) {
        // a row without a diagonal entry loads X[i, :] after all
        const double2 w = found ? xd : *(const double2*)(X + (i * nrhs + c0 + 2 * hl));
        t0 = w.x * y0;
        t1 = w.y * y1;
      }
    }
    if (dot) {
      // both halves add the pair's terms in position order, as k_spmm_wave adds its
      // rows one after the other, so the partials equal that kernel's bit for bit
      const double o0 = __shfl_xor(t0, 32, SPAI_WAVE), o1 = __shfl_xor(t1, 32, SPAI_WAVE);
      const bool hasA = __shfl_xor((int)has, half ? 32 : 0, SPAI_WAVE) != 0;
      const bool hasB = __shfl_xor((int)has, half ? 0 : 32, SPAI_WAVE) != 0;
      if (on && hasA) {
        acc0 += half ? o0 : t0;
        acc1 += half ? o1 : t1;
      }
      if (on && hasB) {
        acc0 += half ? t0 : o0;
        acc1 += half ? t1 : o1;
      }
    }
    i = ni;
    a = na;
    b = nb;
    ec = nec;
    ev = nev;
    load_pos(k + 4 + half, ni, na, nb);
  }
  if (!part) return;
  // per right-hand side r = 2 (l mod 32) + s, wave w's sum (the same in both halves) at
  // sh[w 64 + r], reduced over the waves in order as in k_spmm_wave
  if (half == 0) {
    sh[wv * 64 + 2 * hl] = acc0;
    sh[wv * 64 + 2 * hl + 1] = acc1;
  }
  __syncthreads();
  if (threadIdx.x < 64 && c0 + (int)threadIdx.x < nrhs) {
    double sum = 0.0;
    for (int w = 0; w < WPB; ++w) sum += sh[w * 64 + threadIdx.x];
    part[(int64_t)(c0 + threadIdx.x) * gridDim.x + blockIdx.x] = sum;
  }
}

// The product for at most 32 right-hand sides.  A wave of k_spmm_wave would leave
// 64 - nrhs lanes idle; here R = pow2(nrhs) lanes share a row (lane r owns right-hand
// side r), so a workgroup has kThreads / R rows in flight, and each lane sums its row's
// entries in stored order, eight entries and their gathers issued together (the order
// of k_spmm_wave: the rows of Y are the same bit for bit).  Positions are dealt as in
// k_spmm_wave: eight contiguous XCD ranges, each workgroup a contiguous chunk of
// narrow_chunk(R) positions, its lanes taking them kThreads / R at a time.  With dot
// set, per-block partials of sum_i X[i, r] Y[i, r], stored transposed as there.
template <int R>
constexpr int narrow_rpt() { return R / 4 > 4 ? R / 4 : 4; }   // rows per lane
template <int R>
constexpr int narrow_chunk() { return (kThreads / R) * narrow_rpt<R>(); }

template <typename VT, int LAY, int R>
__global__ __launch_bounds__(kThreads) void k_spmm_narrow(Mat A, const double* X, double* Y,
                                                          int dot, int nrhs, int c0, int ld,
                                                          const int32_t* order, double* part) {
  static_assert(narrow_chunk<R>() >= (kThreads / 64) * kRowsPerWave,
                "no more workgroups than the partial buffer holds");
  if (A.gate && *A.gate == 0) return;                     // every right-hand side stopped
  if (A.ran && c0 == 0 && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(A.ran, 1);
  __shared__ double sh[kThreads];
  constexpr int G = kThreads / R;
  constexpr int RPT = narrow_rpt<R>();
  const int t = threadIdx.x;
  const int r = t % R, g = t / R;
  const int64_t xcd = blockIdx.x & 7, kb = blockIdx.x >> 3;
  const int64_t per = (A.n + 7) / 8;
  const int64_t r0 = xcd * per;
  const int64_t r1 = r0 + per < A.n ? r0 + per : A.n;
  const int64_t base = r0 + kb * (int64_t)narrow_chunk<R>();
  double acc = 0.0;
  // columns c0 .. c0 + nrhs of blocks whose rows are ld doubles apart (ld = nrhs, c0 = 0
  // for a whole block; a wide block is taken R columns at a time)
  X += c0;
  Y += c0;
  if (r < nrhs) {
    for (int j = 0; j < RPT; ++j) {
      const int64_t k = base + (int64_t)j * G + g;
      if (k >= r1) break;
      const int64_t i = order ? (int64_t)order[k] : k;
      const int64_t a = row_lo<LAY>(A, i), b = row_hi<LAY>(A, i);
      double y = 0.0, xd = 0.0;
      bool found = false;
      for (int64_t q0 = a; q0 < b; q0 += 8) {
        int cc[8];
        VT vv[8];
        double xx[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          cc[u] = -1;
          vv[u] = 0;
          if (q0 + u < b) {
            cc[u] = A.col[q0 + u];
            vv[u] = entry_val<VT>(A, q0 + u);
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) xx[u] = cc[u] >= 0 ? X[(int64_t)cc[u] * ld + r] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (cc[u] >= 0) {               // ELL padding (column -1) sits last
            y += (double)vv[u] * xx[u];
            if (cc[u] == (int)i) {
              xd = xx[u];
              found = true;
            }
          }
        if (cc[7] < 0) break;
      }
      Y[i * ld + r] = y;
      if (dot) {
        // a row without a diagonal entry loads X[i, r] after all
        const double wx = found ? xd : X[i * ld + r];
        acc += wx * y;
      }
    }
  }
  if (!part) return;
  sh[t] = acc;
  __syncthreads();
  if (t < R && t < nrhs) {
    double sum = 0.0;
    for (int w = 0; w < G; ++w) sum += sh[w * R + t];
    part[(int64_t)(c0 + t) * gridDim.x + blockIdx.x] = sum;
  }
}

// per-block partials of sum_i A[i, r] B[i, r] (B may be A), optionally of (B - C)
__global__ __launch_bounds__(kThreads) void k_dot_rows(const double* Xa, const double* Xb,
                                                       const double* Xc, int64_t n, int nrhs,
                                                       int c0, int cw, int R, double* part) {
  __shared__ double sh[kThreads];
  const int t = threadIdx.x;
  const int r = t % R;
  const int rows_per = kThreads / R;
  const int roff = t / R;
  double acc = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * rows_per; base < n; base += (int64_t)gridDim.x * rows_per) {
    const int64_t i = base + roff;
    if (i < n && r < cw) {
      const int64_t o = i * nrhs + c0 + r;
      double a = Xa[o];
      double b = Xb[o];
      if (Xc) {
        a = a - Xc[o];
        b = a;
      }
      acc += a * b;
    }
  }
  sh[t] = acc;
  __syncthreads();
  if (t < cw) {
    double s = 0.0;
    for (int k = t; k < kThreads; k += R) s += sh[k];
    part[(int64_t)blockIdx.x * nrhs + c0 + t] = s;
  }
}

// one workgroup per right-hand side: fixed strided partial sums, then a fixed tree
// sum_b p[b] over the workgroup in a fixed order (on thread 0)
__device__ double rows_sum(const double* p, int nblocks, double* sh) {
  // eight loads in flight per thread, added in the order of the plain loop
  double s = 0.0;
  int b = threadIdx.x;
  for (; b + 7 * kThreads < nblocks; b += 8 * kThreads) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[b + u * kThreads];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; b < nblocks; b += kThreads) s += p[b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

// sum_b part[b * nrhs + r] in a fixed order (on thread 0)
__device__ double parts_sum(const double* part, int nblocks, int nrhs, int r, double* sh) {
  double s = 0.0;
  int b = threadIdx.x;
  for (; b + 7 * kThreads < nblocks; b += 8 * kThreads) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(b + u * kThreads) * nrhs + r];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; b < nblocks; b += kThreads) s += part[(int64_t)b * nrhs + r];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

// out[r] = sum_b part[r * nblocks + b] in a fixed order (the products' transposed partials)
__global__ __launch_bounds__(kThreads) void k_reduce_rows(const double* part, int nblocks,
                                                          double* out) {
  __shared__ double sh[kThreads];
  const int r = blockIdx.x;
  const double v = rows_sum(part + (int64_t)r * nblocks, nblocks, sh);
  if (threadIdx.x == 0) out[r] = v;
}

__global__ __launch_bounds__(kThreads) void k_reduce_parts(const double* part, int nblocks,
                                                           int nrhs, double* out) {
  __shared__ double sh[kThreads];
  const int r = blockIdx.x;
  const double v = parts_sum(part, nblocks, nrhs, r, sh);
  if (threadIdx.x == 0) out[r] = v;
}

struct RhsState {
  double bnorm, rz, pq, rr, alpha, beta;
  double alpha_prev;                // the previous iteration's alpha (its x term may be pending)
  int active, iters, status, pad;   // status 0 running, 1 converged, 2 maxiter, 4 indefinite
};

__global__ void k_init_rhs(RhsState* S, const double* bb, int nrhs, int* nactive) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  S[r].bnorm = sqrt(bb[r]);
  S[r].iters = 0;
  S[r].alpha = S[r].beta = 0.0;
  if (S[r].bnorm == 0.0) {
    S[r].active = 0;
    S[r].status = 1;
  } else {
    S[r].active = 1;
    S[r].status = 0;
    atomicAdd(nactive, 1);
  }
}

__global__ void k_set_rz(RhsState* S, const double* rz, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrhs) S[r].rz = rz[r];
}

// alpha = (r, z) / (p, A p), with the indefiniteness checks of the recurrence
// alpha = (r, z) / (p, q) of one right-hand side; a non-positive (r, z) or (p, q) stops it
// as indefinite
__device__ void rhs_alpha(RhsState& g, double pq, int* nactive) {
  g.alpha_prev = g.alpha;
  g.alpha = 0.0;
  if (!g.active) return;
  g.pq = pq;
  if (!(g.rz > 0.0) || !(g.pq > 0.0)) {
    g.active = 0;
    g.status = 4;
    atomicSub(nactive, 1);
    return;
  }
  g.alpha = g.rz / g.pq;
  g.iters += 1;
}

// r -= alpha q (inactive right-hand sides have alpha = 0), fused with the per-block
// partials of ||r||^2 for every right-hand side; x is updated later, with p.  Blocks read
// for the last time before they are written again (q here, z and x in the p updates)
// are loaded nontemporally, and x and the new p are stored so, as are the products'
// outputs: they do not push out of the caches what a product gathers (the 64-right-hand-
// side solve at 96^3 339 -> 330 ms; r, which the next product gathers, gained nothing).
__global__ __launch_bounds__(kThreads) void k_axpy(double* __restrict__ rv,
                                                   const double* __restrict__ q,
                                                   const RhsState* __restrict__ S, int64_t n,
                                                   int nrhs, int R, double* __restrict__ part,
                                                   const int* __restrict__ gate) {
  if (*gate == 0) return;                                  // every right-hand side stopped
  __shared__ double sh[kThreads];
  const int t = threadIdx.x;
  const int r = t % R;
  const int rows_per = kThreads / R;
  const int roff = t / R;
  double acc = 0.0;
  if (r < nrhs) {
    const double a = S[r].alpha;
    for (int64_t base = (int64_t)blockIdx.x * rows_per; base < n; base += (int64_t)gridDim.x * rows_per) {
      const int64_t i = base + roff;
      if (i < n) {
        const int64_t o = i * nrhs + r;
        double rr = rv[o];
        if (a != 0.0) {
          rr = rr - a * __builtin_nontemporal_load(&q[o]);
          rv[o] = rr;
        }
        acc += rr * rr;
      }
    }
  }
  sh[t] = acc;
  __syncthreads();
  if (t < nrhs) {
    double s2 = 0.0;
    for (int k = t; k < kThreads; k += R) s2 += sh[k];
    part[(int64_t)blockIdx.x * nrhs + t] = s2;
  }
}

// convergence of one right-hand side on the recursive residual: ||r|| <= rtol ||b||
__device__ void rhs_conv(RhsState& g, double rr, double rtol, int* nactive) {
  if (!g.active) return;
  g.rr = rr;
  if (sqrt(g.rr) <= rtol * g.bnorm) {
    g.active = 0;
    g.status = 1;
    atomicSub(nactive, 1);
  }
}

__global__ void k_conv(RhsState* S, const double* rr, double rtol, int nrhs, int* nactive) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  rhs_conv(S[r], rr[r], rtol, nactive);
}

// beta = (r, z)_new / (r, z)_old of one right-hand side
__device__ void rhs_beta(RhsState& g, double rz_new) {
  g.beta = 0.0;
  if (!g.active) return;
  g.beta = rz_new / g.rz;
  g.rz = rz_new;
}

// The reductions of an iteration with the scalar step that consumes them (one launch
// instead of two; the same sums and the same step): step 0 alpha from (p, q), 1 beta from
// (r, z) -- both from the products' partials -- and convergence from ||r||^2 partials.
__global__ __launch_bounds__(kThreads) void k_reduce_rows_step(const double* part, int nblocks,
                                                               double* out, RhsState* S, int step,
                                                               int* nactive) {
  __shared__ double sh[kThreads];
  const int r = blockIdx.x;
  const double v = rows_sum(part + (int64_t)r * nblocks, nblocks, sh);
  if (threadIdx.x == 0) {
    out[r] = v;
    if (step == 0) rhs_alpha(S[r], v, nactive);
    else rhs_beta(S[r], v);
  }
}

__global__ __launch_bounds__(kThreads) void k_reduce_parts_conv(const double* part, int nblocks,
                                                                int nrhs, double* out,
                                                                RhsState* S, double rtol,
                                                                int* nactive) {
  __shared__ double sh[kThreads];
  const int r = blockIdx.x;
  const double v = parts_sum(part, nblocks, nrhs, r, sh);
  if (threadIdx.x == 0) {
    out[r] = v;
    rhs_conv(S[r], v, rtol, nactive);
  }
}

// The x update taken two iterations at a time (up to 64 right-hand sides): p alternates
// between two buffers, an even iteration only forms the next p, and the odd one after it
// adds both iterations' terms to x, first alpha_prev p_prev, then alpha p (the additions
// and their order are those of one update per iteration, so x is the same bit for bit).
// Reading x once per two iterations saves half a block pass per iteration.
//
// even iteration: pn = z + beta p for the running right-hand sides
__global__ __launch_bounds__(kThreads) void k_pupd_p(double* __restrict__ pn,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ z,
                                                     const RhsState* __restrict__ S, int64_t n,
                                                     int nrhs, int R) {
  const int t = threadIdx.x;
  const int r = t % R;
  const int rows_per = kThreads / R;
  const int roff = t / R;
  if (r >= nrhs || S[r].active == 0) return;
  const double b = S[r].beta;
  for (int64_t base = (int64_t)blockIdx.x * rows_per; base < n; base += (int64_t)gridDim.x * rows_per) {
    const int64_t i = base + roff;
    if (i < n) {
      const int64_t o = i * nrhs + r;
      __builtin_nontemporal_store(__builtin_nontemporal_load(&z[o]) + b * p[o], &pn[o]);
    }
  }
}

// odd iteration: x += alpha_prev pp, x += alpha p; then pp = z + beta p (pp holds the even
// iteration's p, read before it is overwritten)
__global__ __launch_bounds__(kThreads) void k_pupd_x2(double* __restrict__ pp,
                                                      const double* __restrict__ p,
                                                      double* __restrict__ x,
                                                      const double* __restrict__ z,
                                                      const RhsState* __restrict__ S, int64_t n,
                                                      int nrhs, int R) {
  const int t = threadIdx.x;
  const int r = t % R;
  const int rows_per = kThreads / R;
  const int roff = t / R;
  if (r >= nrhs) return;
  const double a0 = S[r].alpha_prev, a1 = S[r].alpha;
  const bool act = S[r].active != 0;
  const bool upx = a0 != 0.0 || a1 != 0.0;
  if (!upx && !act) return;
  const double b = S[r].beta;
  for (int64_t base = (int64_t)blockIdx.x * rows_per; base < n; base += (int64_t)gridDim.x * rows_per) {
    const int64_t i = base + roff;
    if (i < n) {
      const int64_t o = i * nrhs + r;
      const double po = p[o];
      if (upx) {
        double xv = __builtin_nontemporal_load(&x[o]);
        if (a0 != 0.0) xv = xv + a0 * pp[o];
        if (a1 != 0.0) xv = xv + a1 * po;
        __builtin_nontemporal_store(xv, &x[o]);
      }
      if (act) __builtin_nontemporal_store(__builtin_nontemporal_load(&z[o]) + b * po, &pp[o]);
    }
  }
}

// the pending x term of a solve that stopped after an even iteration: x += alpha p
__global__ __launch_bounds__(kThreads) void k_x_flush(double* __restrict__ x,
                                                      const double* __restrict__ p,
                                                      const RhsState* __restrict__ S, int64_t n,
                                                      int nrhs, int R) {
  const int t = threadIdx.x;
  const int r = t % R;
  const int rows_per = kThreads / R;
  const int roff = t / R;
  if (r >= nrhs) return;
  const double a = S[r].alpha;
  if (a == 0.0) return;
  for (int64_t base = (int64_t)blockIdx.x * rows_per; base < n; base += (int64_t)gridDim.x * rows_per) {
    const int64_t i = base + roff;
    if (i < n) {
      const int64_t o = i * nrhs + r;
      x[o] = x[o] + a * p[o];
    }
  }
}

// the same updates for more than 64 right-hand sides (flat indexing)
__global__ __launch_bounds__(kThreads) void k_axpy_wide(double* rv, const double* q,
                                                        const RhsState* S, int64_t n, int nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < tot; o += (int64_t)gridDim.x * kThreads) {
    const double a = S[o % nrhs].alpha;
    if (a != 0.0) rv[o] = rv[o] - a * q[o];
  }
}

__global__ __launch_bounds__(kThreads) void k_pupd_wide(double* p, double* x, const double* z,
                                                        const RhsState* S, int64_t n, int nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < tot; o += (int64_t)gridDim.x * kThreads) {
    const int r = (int)(o % nrhs);
    const double a = S[r].alpha;
    const double po = p[o];
    if (a != 0.0) x[o] = x[o] + a * po;
    if (S[r].active) p[o] = z[o] + S[r].beta * po;
  }
}

__global__ __launch_bounds__(kThreads) void k_copy(double* dst, const double* src, int64_t tot) {
  for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < tot; o += (int64_t)gridDim.x * kThreads)
    dst[o] = src[o];
}

__global__ __launch_bounds__(kThreads) void k_fill(double* dst, double v, int64_t tot) {
  for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < tot; o += (int64_t)gridDim.x * kThreads)
    dst[o] = v;
}

struct Solver {
  Mat A, M;
  Mat Ag, Mg;                        // A and M as the iterations use them (gated, counted)
  int* runs = nullptr;               // products that did their work, per kind: nactive + 1
  int runs_seen[2] = {0, 0};
  int ctr_host[3] = {0, 0, 0};       // the last host copy of nactive and runs
  int64_t n;
  int nrhs;
  hipStream_t s;
  double *x, *r, *z, *p, *q, *part, *tmp;
  double* p1 = nullptr;              // the second p buffer (up to 64 right-hand sides)
  const double* b;
  RhsState* S;
  int* nactive;
  const int32_t* order = nullptr;   // row visiting order of the products (null: natural)
  // workgroups of the x, p update: 5 per compute unit (20 waves; the 64-right-hand-side solve
  // at 96^3 took 352 ms, against 361 ms with the full 2048 and 363 ms with 3 per unit)
  int pupd_grid = kGrid;
  // optional timing of the products inside the iterations: HIP events recorded on the
  // solver's stream around each A p (kind 0) and M r (kind 1), read back per chunk
  PcgTiming* timing = nullptr;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kind;
  int ev_used = 0;

  // Y = K X with the per-RHS dots (X, Y) reduced into out and the scalar step `step` applied
  // to them in the same launch (0: alpha, 1: beta)
  void timed_spmm(int kind, const Mat& K, const double* X, double* Y, double* out, int step) {
    const bool rec = timing && ev_used + 2 <= (int)ev.size();
    if (rec) (void)hipEventRecord(ev[ev_used], s);
    if (K.val32) spmm_v<float>(K, X, Y, part);
    else spmm_v<double>(K, X, Y, part);
    if (rec) {
      (void)hipEventRecord(ev[ev_used + 1], s);
      ev_kind[ev_used / 2] = kind;
      ev_used += 2;
    }
    hipLaunchKernelGGL(k_reduce_rows_step, dim3(nrhs), dim3(kThreads), 0, s, part, spmm_grid, out,
                       S, step, nactive);
  }
  // after a synchronisation: add the recorded product times to the totals
  // (calls: the products that did their work; a product of a solve whose right-hand sides
  // have all stopped returns at once, and its few microseconds stay in the time)
  void collect_timing() {
    for (int i = 0; i + 1 < ev_used; i += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) {
        timing->ms[ev_kind[i / 2]] += ms;
      } else {
        (void)hipGetLastError();
      }
    }
    ev_used = 0;
    for (int k = 0; k < 2; ++k) {
      timing->calls[k] += ctr_host[1 + k] - runs_seen[k];
      runs_seen[k] = ctr_host[1 + k];
    }
  }

  static int pow2(int w) {
    int R = 1;
    while (R < w) R <<= 1;
    return R;
  }

  // workgroups of a product: 8 XCD ranges of ceil(n / 8) positions, kRowsPerWave
  // positions per wave, kThreads / 64 waves per workgroup (blocks of its partials)
  static int spmm_blocks(int64_t n) {
    const int64_t per = (n + 7) / 8, rows = (int64_t)(kThreads / 64) * kRowsPerWave;
    return (int)(8 * ((per + rows - 1) / rows));
  }
  int spmm_grid = 8;

  template <typename VT, int LAY, int R>
  void spmm_narrow(const Mat& K, const double* X, double* Y, double* pt, int c0 = 0,
                   int cw = 0) {
    const int64_t per = (n + 7) / 8;
    spmm_grid = (int)(8 * ((per + narrow_chunk<R>() - 1) / narrow_chunk<R>()));
    hipLaunchKernelGGL((k_spmm_narrow<VT, LAY, R>), dim3(spmm_grid), dim3(kThreads), 0, s, K, X,
                       Y, pt ? 1 : 0, cw ? cw : nrhs, c0, nrhs, order, pt);
  }
  template <typename VT, int LAY>
  void spmm_as(const Mat& K, const double* X, double* Y, double* pt) {
    switch (nrhs <= 32 ? pow2(nrhs) : 0) {   // few right-hand sides: rows share a wave
      case 1: return spmm_narrow<VT, LAY, 1>(K, X, Y, pt);
      case 2: return spmm_narrow<VT, LAY, 2>(K, X, Y, pt);
      case 4: return spmm_narrow<VT, LAY, 4>(K, X, Y, pt);
      case 8: return spmm_narrow<VT, LAY, 8>(K, X, Y, pt);
      case 16: return spmm_narrow<VT, LAY, 16>(K, X, Y, pt);
      case 32: return spmm_narrow<VT, LAY, 32>(K, X, Y, pt);
      default: break;
    }
    spmm_grid = spmm_blocks(n);
    for (int c0 = 0; c0 < nrhs; c0 += 64) {
      if (nrhs % 2 == 0)   // 16-byte gathers, two rows per wave
        hipLaunchKernelGGL((k_spmm_pair<VT, LAY>), dim3(spmm_grid), dim3(kThreads), 0, s, K, X,
                           Y, pt ? 1 : 0, nrhs, c0, order, pt);
      else
        hipLaunchKernelGGL((k_spmm_wave<VT, LAY>), dim3(spmm_grid), dim3(kThreads), 0, s, K, X,
                           Y, pt ? 1 : 0, nrhs, c0, order, pt);
    }
  }
  template <typename VT>
  void spmm_v(const Mat& K, const double* X, double* Y, double* pt) {
    if (K.eshift >= 0) spmm_as<VT, kLayEll>(K, X, Y, pt);
    else if (K.beg) spmm_as<VT, kLayPad>(K, X, Y, pt);
    else spmm_as<VT, kLayCsr>(K, X, Y, pt);
  }
  // Y = Mat X, and with out set the per-RHS dots (X, Y) reduced into out
  void spmm(const Mat& K, const double* X, double* Y, double* out) {
    if (K.val32) spmm_v<float>(K, X, Y, out ? part : nullptr);
    else spmm_v<double>(K, X, Y, out ? part : nullptr);
    if (out)
      hipLaunchKernelGGL(k_reduce_rows, dim3(nrhs), dim3(kThreads), 0, s, part, spmm_grid, out);
  }

  void dot(const double* Xa, const double* Xb, const double* Xc, double* out) {
    for (int c0 = 0; c0 < nrhs; c0 += 64) {
      const int cw = std::min(64, nrhs - c0);
      const int R = pow2(cw);
      hipLaunchKernelGGL(k_dot_rows, dim3(kGrid), dim3(kThreads), 0, s, Xa, Xb, Xc, n, nrhs, c0, cw, R,
                         part);
    }
    hipLaunchKernelGGL(k_reduce_parts, dim3(nrhs), dim3(kThreads), 0, s, part, kGrid, nrhs, out);
  }

  // one PCG iteration; each reduction applies the scalar step that consumes it.  odd:
  // the parity of the iteration's index (p in p1, and x updated for this and the previous)
  void iteration(double rtol, int odd) {
    const dim3 gs((nrhs + 63) / 64), bs(64);
    const bool two = nrhs <= 64;
    double* pc = two && odd ? p1 : p;                          // this iteration's p
    timed_spmm(0, Ag, pc, q, tmp, 0);                         // q = A p, (p, q), alpha
    if (nrhs <= 64) {                                            // r update fused with ||r||^2
      hipLaunchKernelGGL(k_axpy, dim3(kGrid), dim3(kThreads), 0, s, r, q, S, n, nrhs, pow2(nrhs),
                         part, nactive);
      hipLaunchKernelGGL(k_reduce_parts_conv, dim3(nrhs), dim3(kThreads), 0, s, part, kGrid, nrhs,
                         tmp, S, rtol, nactive);               // convergence test
    } else {
      hipLaunchKernelGGL(k_axpy_wide, dim3(kGrid), dim3(kThreads), 0, s, r, q, S, n, nrhs);
      dot(r, r, nullptr, tmp);
      hipLaunchKernelGGL(k_conv, gs, bs, 0, s, S, tmp, rtol, nrhs, nactive);
    }
    timed_spmm(1, Mg, r, z, tmp, 1);                          // z = M r, (r, z), beta
    if (two && !odd)                                             // p1 = z + beta p
      hipLaunchKernelGGL(k_pupd_p, dim3(pupd_grid), dim3(kThreads), 0, s, p1, p, z, S, n, nrhs,
                         pow2(nrhs));
    else if (two)                                                // x += both terms, p = z + beta p1
      hipLaunchKernelGGL(k_pupd_x2, dim3(pupd_grid), dim3(kThreads), 0, s, p, p1, x, z, S, n,
                         nrhs, pow2(nrhs));
    else
      hipLaunchKernelGGL(k_pupd_wide, dim3(kGrid), dim3(kThreads), 0, s, p, x, z, S, n, nrhs);
  }
};

int upload_csr(DevPool& pool, const HostCsr& h, bool f32, Mat& m, hipStream_t s) {
  int rc;
  int64_t* rp;
  int32_t* c;
  if ((rc = pool.alloc(&rp, h.n + 1)) || (rc = pool.alloc(&c, h.nnz))) return rc;
  HIPCHK(hipMemcpyAsync(rp, h.rowptr.data(), sizeof(int64_t) * (h.n + 1), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c, h.col.data(), sizeof(int32_t) * h.nnz, hipMemcpyHostToDevice, s));
  m = Mat{};
  m.n = h.n;
  m.rowptr = rp;
  m.col = c;
  if (f32) {
    std::vector<float> v(h.nnz);
    for (int64_t q = 0; q < h.nnz; ++q) v[q] = (float)h.val[q];
    float* d;
    if ((rc = pool.alloc(&d, h.nnz))) return rc;
    HIPCHK(hipMemcpyAsync(d, v.data(), sizeof(float) * h.nnz, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    m.val32 = d;
  } else {
    double* d;
    if ((rc = pool.alloc(&d, h.nnz))) return rc;
    HIPCHK(hipMemcpyAsync(d, h.val.data(), sizeof(double) * h.nnz, hipMemcpyHostToDevice, s));
    m.val = d;
  }
  return SPAI_OK;
}

}  // namespace
}  // namespace spai

using namespace spai;

namespace spai {

int pcg_run(const PcgMat& A, const PcgMat& M, int nrhs, const double* dB, double* dX, double rtol,
            int max_iter, int* iters, double* relres, const int32_t* order, hipStream_t s,
            PcgTiming* timing, PcgWork* work) {
  int rc;
  DevPool local;
  DevPool& pool = work ? work->pool : local;
  Solver S{};
  struct EvGuard {
    std::vector<hipEvent_t>* v;
    ~EvGuard() {
      for (hipEvent_t e : *v) (void)hipEventDestroy(e);
    }
  } evg{&S.ev};
  S.A = A;
  S.M = M;
  S.n = A.n;
  S.nrhs = nrhs;
  S.s = s;
  S.order = order;
  const int64_t tot = S.n * nrhs;
  // every block is initialised or written before it is read in each solve, so kept
  // blocks need no clearing beyond the state reset below
  if (work && work->n == S.n && work->nrhs == nrhs) {
    S.r = (double*)work->blk[0];
    S.z = (double*)work->blk[1];
    S.p = (double*)work->blk[2];
    S.p1 = (double*)work->blk[3];
    S.q = (double*)work->blk[4];
    S.part = (double*)work->blk[5];
    S.tmp = (double*)work->blk[6];
    S.S = (RhsState*)work->blk[7];
    S.nactive = (int*)work->blk[8];
  } else {
    if (work) {
      work->pool.release();
      work->n = -1;
    }
    if ((rc = pool.alloc(&S.r, tot)) || (rc = pool.alloc(&S.z, tot)) || (rc = pool.alloc(&S.p, tot)) ||
        (nrhs <= 64 && (rc = pool.alloc(&S.p1, tot))) ||
        (rc = pool.alloc(&S.q, tot)) ||
        (rc = pool.alloc(&S.part, (int64_t)std::max<int64_t>(kGrid, Solver::spmm_blocks(S.n)) * nrhs)) ||
        (rc = pool.alloc(&S.tmp, nrhs)) || (rc = pool.alloc(&S.S, nrhs)) || (rc = pool.alloc(&S.nactive, 3)))
      return rc;
    if (work) {
      void* const b[9] = {S.r, S.z, S.p, S.p1, S.q, S.part, S.tmp, S.S, S.nactive};
      for (int i = 0; i < 9; ++i) work->blk[i] = b[i];
      work->n = S.n;
      work->nrhs = nrhs;
    }
  }
  S.b = dB;
  S.x = dX;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
      S.pupd_grid = 5 * cus;
    else
      (void)hipGetLastError();
  }
  if (timing) {                         // two products per iteration, 8 iterations per chunk
    S.timing = timing;
    S.ev.resize(32, nullptr);
    S.ev_kind.resize(16, 0);
    for (auto& e : S.ev)
      if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        e = nullptr;
        S.timing = nullptr;
      }
  }
  if (S.timing) S.runs = S.nactive + 1;   // read with the active count in one copy
  S.Ag = S.A;
  S.Mg = S.M;
  S.Ag.gate = S.Mg.gate = S.nactive;
  S.Ag.ran = S.runs;
  S.Mg.ran = S.runs ? S.runs + 1 : nullptr;
  HIPCHK(hipMemsetAsync(S.nactive, 0, 3 * sizeof(int), s));
  HIPCHK(hipMemsetAsync(S.S, 0, sizeof(RhsState) * nrhs, s));
  const dim3 gs((nrhs + 63) / 64), bs(64);
  // x_0 = 0, r = b, z = M r, p = z
  hipLaunchKernelGGL(k_fill, dim3(kGrid), dim3(kThreads), 0, s, S.x, 0.0, tot);
  hipLaunchKernelGGL(k_copy, dim3(kGrid), dim3(kThreads), 0, s, S.r, dB, tot);
  S.dot(dB, dB, nullptr, S.tmp);
  hipLaunchKernelGGL(k_init_rhs, gs, bs, 0, s, S.S, S.tmp, nrhs, S.nactive);
  S.spmm(S.M, S.r, S.z, S.tmp);
  hipLaunchKernelGGL(k_set_rz, gs, bs, 0, s, S.S, S.tmp, nrhs);
  hipLaunchKernelGGL(k_copy, dim3(kGrid), dim3(kThreads), 0, s, S.p, S.z, tot);
  HIPCHK(hipGetLastError());
  // iterate in chunks, checking the running count between chunks.  On a stream of
  // its own (not the null stream) and without the per-product timing, a full chunk is
  // captured once as a HIP graph and replayed: every launch of an iteration has fixed
  // arguments, and converged right-hand sides are masked on the device.
  int it = 0;
  const int chunk = 8;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  struct GraphGuard {
    hipGraph_t* g;
    hipGraphExec_t* e;
    ~GraphGuard() {
      if (*e) (void)hipGraphExecDestroy(*e);
      if (*g) (void)hipGraphDestroy(*g);
    }
  } gguard{&graph, &gexec};
  bool use_graph = s != nullptr && !S.timing;
  while (it < max_iter) {
    HIPCHK(hipMemcpyAsync(S.ctr_host, S.nactive, (S.timing ? 3 : 1) * sizeof(int),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (S.timing) S.collect_timing();
    if (S.ctr_host[0] == 0) break;
    const int k = std::min(chunk, max_iter - it);
    if (use_graph && k == chunk && !gexec) {
      if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        for (int t = 0; t < k; ++t) S.iteration(rtol, (it + t) & 1);
        if (hipStreamEndCapture(s, &graph) != hipSuccess ||
            hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
          (void)hipGetLastError();
          if (graph) (void)hipGraphDestroy(graph);
          graph = nullptr;
          gexec = nullptr;
          return fail(SPAI_ERR_HIP, "pcg: capturing the iteration graph failed");
        }
      } else {
        (void)hipGetLastError();
        use_graph = false;
      }
    }
    if (use_graph && k == chunk && gexec) {
      HIPCHK(hipGraphLaunch(gexec, s));
    } else {
      for (int t = 0; t < k; ++t) S.iteration(rtol, (it + t) & 1);
    }
    HIPCHK(hipGetLastError());
    it += k;
  }
  if (nrhs <= 64 && (it & 1))      // the last iteration was even: its x term is pending
    hipLaunchKernelGGL(k_x_flush, dim3(S.pupd_grid), dim3(kThreads), 0, s, S.x, S.p, S.S, S.n, nrhs,
                       Solver::pow2(nrhs));
  // true residual ||b - A x|| / ||b||
  S.spmm(S.A, S.x, S.q, nullptr);
  S.dot(dB, dB, S.q, S.tmp);     // sum (b - Ax)^2
  std::vector<double> rr(nrhs);
  HIPCHK(hipMemcpyAsync(rr.data(), S.tmp, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
  std::vector<RhsState> hs(nrhs);
  HIPCHK(hipMemcpyAsync(hs.data(), S.S, sizeof(RhsState) * nrhs, hipMemcpyDeviceToHost, s));
  if (S.timing)
    HIPCHK(hipMemcpyAsync(S.ctr_host, S.nactive, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (S.timing) S.collect_timing();
  bool indef = false, unconv = false;
  for (int r = 0; r < nrhs; ++r) {
    if (iters) iters[r] = hs[r].iters;
    if (relres) relres[r] = hs[r].bnorm > 0.0 ? std::sqrt(rr[r]) / hs[r].bnorm : 0.0;
    if (hs[r].status == 4) indef = true;
    if (hs[r].status == 0) unconv = true;
  }
  if (indef) return PCG_INDEFINITE;
  if (unconv) return SPAI_MAXITER;
  return SPAI_OK;
}

}  // namespace spai

extern "C" int pcg_solve(const spai_csr_t* A, const spai_csr_t* M, int nrhs, const double* B,
                         double* X, double rtol, int max_iter, int* iters, double* relres,
                         const spai_opts_t* opts) {
  try {
    if (!A || !M || nrhs < 1 || !B || !X || !(rtol >= 0.0) || max_iter < 0)
      return fail(SPAI_ERR_ARG, "pcg_solve: bad arguments");
    int rc;
    HostCsr hA, hM;
    if ((rc = fetch_csr(A, hA)) || (rc = fetch_csr(M, hM))) return rc;
    if (hM.n != hA.n) return fail(SPAI_ERR_ARG, "pcg_solve: A and M differ in size");
    spai_opts_t o;
    spai_default_opts(&o);
    if (opts) o = *opts;
    hipStream_t s = (hipStream_t)o.stream;
    DevPool pool;
    Mat dA, dM;
    if ((rc = upload_csr(pool, hA, false, dA, s))) return rc;
    if ((rc = upload_csr(pool, hM, o.precision == SPAI_PREC_MIXED, dM, s))) return rc;
    const int64_t tot = hA.n * nrhs;
    const double* dB = B;
    double* dX = X;
    if (!A->on_device) {
      double *b2, *x2;
      if ((rc = pool.alloc(&b2, tot)) || (rc = pool.alloc(&x2, tot))) return rc;
      HIPCHK(hipMemcpyAsync(b2, B, sizeof(double) * tot, hipMemcpyHostToDevice, s));
      dB = b2;
      dX = x2;
    }
    std::vector<int32_t> ord;
    locality_order(hA, kBallRows, ord);
    int32_t* d_order;
    if ((rc = pool.alloc(&d_order, hA.n))) return rc;
    HIPCHK(hipMemcpyAsync(d_order, ord.data(), sizeof(int32_t) * hA.n, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    rc = pcg_run(dA, dM, nrhs, dB, dX, rtol, max_iter, iters, relres, d_order, s, nullptr);
    if (rc < 0) return rc;
    if (!A->on_device) {
      HIPCHK(hipMemcpyAsync(X, dX, sizeof(double) * tot, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    return rc;
  } catch (const std::bad_alloc&) {
    return fail(SPAI_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}
