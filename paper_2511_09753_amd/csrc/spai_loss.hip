// spai_loss.hip — f(M) = ||I - A M||_F^2 (Section 2) on fixed patterns and its adjoint.
//
// With R = I - A M:  df = -2 (R, dA M + A dM)_F, so
//   d f / d A = -2 R M^T   restricted to supp(A),
//   d f / d M = -2 A^T R   restricted to supp(M)   (= -2 A R of Section 2 for symmetric A).
// Neither A M nor R is stored: the row kernel rebuilds row i of R from the rows of M
// selected by A's row i (giving f and d f / d A), the column kernel rebuilds column j
// of R from column j of M (giving d f / d M).  Both keep one row/column per 64-lane
// wavefront in LDS and sum in fixed orders, so the results are deterministic.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "spai.h"
#include "spai_dev.hpp"
#include "spai_host.hpp"

namespace spai {
namespace {

// (offsets only, no integer round trip of the pointer, so the compiler still sees
// LDS addresses and emits ds_* instructions rather than flat ones)
struct Carve2 {
  char* base;
  unsigned off = 0;
  __device__ explicit Carve2(char* b) : base(b) {}
  template <typename U> __device__ U* take(int count) {
    off = (off + 7u) & ~7u;
    U* r = (U*)(base + off);
    off += (unsigned)(sizeof(U) * (unsigned)count);
    return r;
  }
};

struct Pat {                    // CSR pattern
  int64_t n;
  const int64_t* rowptr;
  const int32_t* col;
};

// position of (col[q], row(q)) for every stored entry q of a symmetric pattern; an
// entry without its mirror maps to itself and raises err bit 2
__global__ void k_transpose_map(Pat P, int64_t* tmap, int* err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n) return;
  for (int64_t q = P.rowptr[i]; q < P.rowptr[i + 1]; ++q) {
    const int32_t k = P.col[q];
    int64_t lo = P.rowptr[k], hi = P.rowptr[k + 1];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (P.col[mid] < (int32_t)i) lo = mid + 1; else hi = mid;
    }
    if (lo < P.rowptr[k + 1] && P.col[lo] == (int32_t)i) {
      tmap[q] = lo;
    } else {
      tmap[q] = q;
      atomicOr(err, 2);
    }
  }
}

template <typename T>
__global__ void k_gather(const T* src, const int64_t* map, T* dst, int64_t nnz) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nnz) dst[q] = src[map[q]];
}

__global__ void k_to_f32(const double* a, float* b, int64_t nnz) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nnz) b[q] = (float)a[q];
}

// row kernel: rowpart[i] = ||R(i,:)||^2 and, if gA, gA[q] = -2 dL (R M^T)(i, col q)
template <typename T>
__global__ __launch_bounds__(SPAI_WAVE) void k_loss_rows(Pat A, const T* Av, Pat M, const T* Mv,
                                                         double* rowpart, double* gA, double dL,
                                                         int* err, int L, int H, int DG) {
  extern __shared__ char smem[];
  Carve2 cv(smem);
  int* s_li = cv.take<int>(L);
  int* s_keys = cv.take<int>(H);
  int* s_sorted = cv.take<int>(H);
  int* s_off = cv.take<int>(DG + 1);
  double* s_lv = cv.take<double>(L);
  double* s_a = cv.take<double>(DG);
  double* s_rho = cv.take<double>(H / 2);
  const int lane = lane_id();
  ColumnWalk w(A.n, blockIdx.x, gridDim.x);
  for (int64_t i = w.begin; i < w.end; i += w.step) {
    const int64_t qa = A.rowptr[i];
    const int deg = (int)(A.rowptr[i + 1] - qa);
    int ltot = 0;
    for (int t = lane; t < deg; t += SPAI_WAVE) {
      const int l = A.col[qa + t];
      ltot += (int)(M.rowptr[l + 1] - M.rowptr[l]);
    }
    ltot = wave_sum_int(ltot);
    if (deg > DG || ltot > L || ltot + 2 >= H / 2) {
      if (lane == 0) atomicOr(err, 1);
      continue;
    }
    int run = 0;
    for (int base = 0; base < deg; base += SPAI_WAVE) {
      const int t = base + lane;
      int len = 0;
      if (t < deg) {
        const int l = A.col[qa + t];
        len = (int)(M.rowptr[l + 1] - M.rowptr[l]);
        s_a[t] = (double)Av[qa + t];
      }
      const int inc = wave_incl_scan(len);
      if (t < deg) s_off[t] = run + inc - len;
      run += __shfl(inc, SPAI_WAVE - 1, SPAI_WAVE);
    }
    if (lane == 0) s_off[deg] = run;
    __syncthreads();
    for (int t = 0; t < deg; ++t) {
      const int l = A.col[qa + t];
      const int64_t b = M.rowptr[l];
      const int len = s_off[t + 1] - s_off[t];
      for (int e = lane; e < len; e += SPAI_WAVE) {
        s_li[s_off[t] + e] = M.col[b + e];
        s_lv[s_off[t] + e] = (double)Mv[b + e];
      }
    }
    ks_clear(s_keys, H);
    __syncthreads();
    if (lane == 0) ks_insert(s_keys, H, (int)i);
    for (int e = lane; e < ltot; e += SPAI_WAVE) ks_insert(s_keys, H, s_li[e]);
    __syncthreads();
    const int nk = ks_sorted(s_keys, H, s_sorted);
    __syncthreads();
    double acc = 0.0;
    for (int t0 = lane; t0 < nk; t0 += SPAI_WAVE) {
      const int j = s_sorted[t0];
      double s = 0.0;
      for (int t = 0; t < deg; ++t) {
        const int o = s_off[t];
        const int e = bsearch_idx(s_li + o, s_off[t + 1] - o, j);
        if (e >= 0) s += s_a[t] * s_lv[o + e];
      }
      const double rho = ((j == (int)i) ? 1.0 : 0.0) - s;
      s_rho[t0] = rho;
      acc += rho * rho;
    }
    acc = wave_sum(acc);
    if (lane == 0) rowpart[i] = acc;
    __syncthreads();
    if (gA) {
      for (int t = 0; t < deg; ++t) {
        const int o = s_off[t];
        const int len = s_off[t + 1] - o;
        double g = 0.0;
        for (int e = lane; e < len; e += SPAI_WAVE) {
          const int pos = bsearch_idx(s_sorted, nk, s_li[o + e]);
          g += s_rho[pos] * s_lv[o + e];
        }
        g = wave_sum(g);
        if (lane == 0) gA[qa + t] = -2.0 * dL * g;
      }
    }
    __syncthreads();
  }
}

// column kernel: gM at (k, j) for k in supp(M(:, j)) = -2 dL sum_u A(u,k) R(u,j)
template <typename T>
__global__ __launch_bounds__(SPAI_WAVE) void k_loss_cols(Pat A, const T* Av, const T* Atv, Pat M,
                                                         const T* Mv, const int64_t* tmapM,
                                                         double* gM, double dL, int* err, int L,
                                                         int H) {
  extern __shared__ char smem[];
  Carve2 cv(smem);
  int* s_mi = cv.take<int>(L);
  int* s_pre = cv.take<int>(L);
  int* s_keys = cv.take<int>(H);
  int* s_sorted = cv.take<int>(H);
  double* s_mv = cv.take<double>(L);
  double* s_r = cv.take<double>(H / 2);
  const int lane = lane_id();
  ColumnWalk w(M.n, blockIdx.x, gridDim.x);
  for (int64_t j = w.begin; j < w.end; j += w.step) {
    const int64_t mb = M.rowptr[j];
    const int lm = (int)(M.rowptr[j + 1] - mb);     // column j of M = row j pattern (symmetric)
    if (lm > L) {
      if (lane == 0) atomicOr(err, 1);
      continue;
    }
    for (int e = lane; e < lm; e += SPAI_WAVE) {
      s_mi[e] = M.col[mb + e];
      s_mv[e] = (double)Mv[tmapM[mb + e]];          // M(l, j)
    }
    __syncthreads();
    // products: neighbours of every l in supp(m_j)
    int run = 0;
    for (int base = 0; base < lm; base += SPAI_WAVE) {
      const int e = base + lane;
      int d = 0;
      if (e < lm) {
        const int l = s_mi[e];
        d = (int)(A.rowptr[l + 1] - A.rowptr[l]);
      }
      const int inc = wave_incl_scan(d);
      if (e < lm) s_pre[e] = run + inc;
      run += __shfl(inc, SPAI_WAVE - 1, SPAI_WAVE);
    }
    if (run + 2 >= H / 2) {
      if (lane == 0) atomicOr(err, 1);
      __syncthreads();
      continue;
    }
    ks_clear(s_keys, H);
    __syncthreads();
    if (lane == 0) ks_insert(s_keys, H, (int)j);
    for (int p = lane; p < run; p += SPAI_WAVE) {
      const int e = upper_bound_int(s_pre, lm, p);
      const int before = e ? s_pre[e - 1] : 0;
      ks_insert(s_keys, H, A.col[A.rowptr[s_mi[e]] + (p - before)]);
    }
    __syncthreads();
    const int nu = ks_sorted(s_keys, H, s_sorted);
    __syncthreads();
    for (int t = lane; t < nu; t += SPAI_WAVE) {
      const int u = s_sorted[t];
      double s = 0.0;
      for (int64_t q = A.rowptr[u]; q < A.rowptr[u + 1]; ++q) {
        const int e = bsearch_idx(s_mi, lm, A.col[q]);
        if (e >= 0) s += (double)Av[q] * s_mv[e];
      }
      s_r[t] = ((u == (int)j) ? 1.0 : 0.0) - s;
    }
    __syncthreads();
    for (int e = lane; e < lm; e += SPAI_WAVE) {
      const int k = s_mi[e];
      double g = 0.0;
      for (int64_t q = A.rowptr[k]; q < A.rowptr[k + 1]; ++q) {
        const int pos = bsearch_idx(s_sorted, nu, A.col[q]);
        if (pos >= 0) g += (double)Atv[q] * s_r[pos];   // A(u, k) R(u, j), u = col q
      }
      gM[tmapM[mb + e]] = -2.0 * dL * g;
    }
    __syncthreads();
  }
}

__global__ void k_sum_parts(const double* part, int64_t n, double* out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_sum_chunks(const double* part, int64_t n, int64_t chunk, double* out) {
  __shared__ double sh[256];
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

constexpr int kGridRows = 2048;

size_t rows_lds(int L, int H, int DG) {
  return (size_t)L * 4 + (size_t)H * 8 + (size_t)(DG + 1) * 4 + (size_t)L * 8 + (size_t)DG * 8 +
         (size_t)(H / 2) * 8 + 64;
}
size_t cols_lds(int L, int H) { return (size_t)L * 8 + (size_t)H * 8 + (size_t)L * 8 + (size_t)(H / 2) * 8 + 64; }

struct LossCall {
  DevPool pool;
  Pat pA{}, pM{};
  const double* Av64 = nullptr;
  const double* Mv64 = nullptr;
  hipStream_t s = nullptr;
  int64_t nnzA = 0, nnzM = 0;
  int* err = nullptr;

  int load(const spai_csr_t* A, const spai_csr_t* M, const spai_opts_t* opts, bool check_pat) {
    int rc;
    if (!A || !M || A->n != M->n || A->n < 1) return fail(SPAI_ERR_ARG, "loss: bad shapes");
    spai_opts_t o;
    spai_default_opts(&o);
    if (opts) o = *opts;
    s = (hipStream_t)o.stream;
    nnzA = A->nnz;
    nnzM = M->nnz;
    if (check_pat || !A->on_device) {
      HostCsr hA, hM;
      if ((rc = fetch_csr(A, hA)) || (rc = fetch_csr(M, hM))) return rc;
      if (check_pat && ((rc = check_symmetric_pattern(hA)) || (rc = check_symmetric_pattern(hM))))
        return rc;
      if (!A->on_device) return upload(hA, hM);
    }
    if ((rc = pool.alloc(&err, 1))) return rc;
    HIPCHK(hipMemsetAsync(err, 0, sizeof(int), s));
    pA = Pat{A->n, A->rowptr, A->colind};
    pM = Pat{M->n, M->rowptr, M->colind};
    Av64 = A->val;
    Mv64 = M->val;
    return SPAI_OK;
  }

  int upload(const HostCsr& hA, const HostCsr& hM) {
    int rc;
    int64_t *ra, *rm;
    int32_t *ca, *cm;
    double *va, *vm;
    if ((rc = pool.alloc(&ra, hA.n + 1)) || (rc = pool.alloc(&ca, hA.nnz)) || (rc = pool.alloc(&va, hA.nnz)) ||
        (rc = pool.alloc(&rm, hM.n + 1)) || (rc = pool.alloc(&cm, hM.nnz)) || (rc = pool.alloc(&vm, hM.nnz)) ||
        (rc = pool.alloc(&err, 1)))
      return rc;
    HIPCHK(hipMemcpyAsync(ra, hA.rowptr.data(), 8 * (hA.n + 1), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ca, hA.col.data(), 4 * hA.nnz, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(va, hA.val.data(), 8 * hA.nnz, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(rm, hM.rowptr.data(), 8 * (hM.n + 1), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cm, hM.col.data(), 4 * hM.nnz, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(vm, hM.val.data(), 8 * hM.nnz, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(err, 0, sizeof(int), s));
    pA = Pat{hA.n, ra, ca};
    pM = Pat{hM.n, rm, cm};
    Av64 = va;
    Mv64 = vm;
    return SPAI_OK;
  }
};

template <typename T>
int run_rows(LossCall& c, const T* Av, const T* Mv, double* rowpart, double* gA, double dL) {
  const int L = 512, H = 1024, DG = 64;
  hipLaunchKernelGGL(k_loss_rows<T>, dim3(kGridRows), dim3(SPAI_WAVE), rows_lds(L, H, DG), c.s, c.pA,
                     Av, c.pM, Mv, rowpart, gA, dL, c.err, L, H, DG);
  HIPCHK(hipGetLastError());
  return SPAI_OK;
}

template <typename T>
int run_cols(LossCall& c, const T* Av, const T* Atv, const T* Mv, const int64_t* tmapM, double* gM,
             double dL) {
  const int L = 256, H = 1024;
  hipLaunchKernelGGL(k_loss_cols<T>, dim3(kGridRows), dim3(SPAI_WAVE), cols_lds(L, H), c.s, c.pA, Av,
                     Atv, c.pM, Mv, tmapM, gM, dL, c.err, L, H);
  HIPCHK(hipGetLastError());
  return SPAI_OK;
}

template <typename T>
int values(LossCall& c, const T** Av, const T** Mv) {
  if constexpr (sizeof(T) == 8) {
    *Av = (const T*)c.Av64;
    *Mv = (const T*)c.Mv64;
  } else {
    int rc;
    float *a, *m;
    if ((rc = c.pool.alloc(&a, c.nnzA)) || (rc = c.pool.alloc(&m, c.nnzM))) return rc;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((c.nnzA + 255) / 256)), dim3(256), 0, c.s, c.Av64, a, c.nnzA);
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((c.nnzM + 255) / 256)), dim3(256), 0, c.s, c.Mv64, m, c.nnzM);
    *Av = (const T*)a;
    *Mv = (const T*)m;
  }
  return SPAI_OK;
}

template <typename T>
int loss_fwd_t(LossCall& c, double* Lout) {
  int rc;
  const T *Av, *Mv;
  if ((rc = values<T>(c, &Av, &Mv))) return rc;
  double *rowpart, *chunks, *out;
  const int nch = 512;
  if ((rc = c.pool.alloc(&rowpart, c.pA.n)) || (rc = c.pool.alloc(&chunks, nch)) || (rc = c.pool.alloc(&out, 1)))
    return rc;
  if ((rc = run_rows<T>(c, Av, Mv, rowpart, nullptr, 1.0))) return rc;
  const int64_t chunk = (c.pA.n + nch - 1) / nch;
  const int nb = (int)((c.pA.n + chunk - 1) / chunk);
  hipLaunchKernelGGL(k_sum_chunks, dim3(nb), dim3(256), 0, c.s, rowpart, c.pA.n, chunk, chunks);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, c.s, chunks, (int64_t)nb, out);
  int herr = 0;
  HIPCHK(hipMemcpyAsync(Lout, out, sizeof(double), hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipMemcpyAsync(&herr, c.err, sizeof(int), hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipStreamSynchronize(c.s));
  if (herr) return fail(SPAI_ERR_CAPACITY, "loss: a row or column exceeded the per-column tile");
  return SPAI_OK;
}

template <typename T>
int loss_bwd_t(LossCall& c, double dL, double* gA, double* gM, bool host_out) {
  int rc;
  const T *Av, *Mv;
  if ((rc = values<T>(c, &Av, &Mv))) return rc;
  double *rowpart, *dgA = gA, *dgM = gM;
  if ((rc = c.pool.alloc(&rowpart, c.pA.n))) return rc;
  if (host_out) {
    if (gA && (rc = c.pool.alloc(&dgA, c.nnzA))) return rc;
    if (gM && (rc = c.pool.alloc(&dgM, c.nnzM))) return rc;
  }
  if (gA && (rc = run_rows<T>(c, Av, Mv, rowpart, dgA, dL))) return rc;
  if (gM) {
    int64_t *tA, *tM;
    T* Atv;
    if ((rc = c.pool.alloc(&tA, c.nnzA)) || (rc = c.pool.alloc(&tM, c.nnzM)) || (rc = c.pool.alloc(&Atv, c.nnzA)))
      return rc;
    hipLaunchKernelGGL(k_transpose_map, dim3((unsigned)((c.pA.n + 255) / 256)), dim3(256), 0, c.s, c.pA, tA, c.err);
    hipLaunchKernelGGL(k_transpose_map, dim3((unsigned)((c.pM.n + 255) / 256)), dim3(256), 0, c.s, c.pM, tM, c.err);
    hipLaunchKernelGGL(k_gather<T>, dim3((unsigned)((c.nnzA + 255) / 256)), dim3(256), 0, c.s, Av, tA, Atv, c.nnzA);
    if ((rc = run_cols<T>(c, Av, Atv, Mv, tM, dgM, dL))) return rc;
  }
  int herr = 0;
  HIPCHK(hipMemcpyAsync(&herr, c.err, sizeof(int), hipMemcpyDeviceToHost, c.s));
  if (host_out) {
    if (gA) HIPCHK(hipMemcpyAsync(gA, dgA, 8 * c.nnzA, hipMemcpyDeviceToHost, c.s));
    if (gM) HIPCHK(hipMemcpyAsync(gM, dgM, 8 * c.nnzM, hipMemcpyDeviceToHost, c.s));
  }
  HIPCHK(hipStreamSynchronize(c.s));
  if (herr & 2) return fail(SPAI_ERR_ARG, "loss: the pattern of A or M is not symmetric");
  if (herr) return fail(SPAI_ERR_CAPACITY, "loss: a row or column exceeded the per-column tile");
  return SPAI_OK;
}

// ---- allocation-free forward loss ---------------------------------------------------
// Scratch of spai_loss_fwd_noalloc: the per-row partial sums (at most kNoAllocRows rows)
// and the chunk sums of the fixed-order reduction, in a file-scope device array (each
// GPU holds its own copy until the process ends).  Host code never passes the array's
// name to a kernel: it takes the array's device address from hipGetSymbolAddress, once
// per device, and uses that address.
constexpr int64_t kNoAllocRows = (int64_t)1 << 21;
constexpr int kNoAllocChunks = 512;
__device__ __align__(256) double scratch[kNoAllocRows + kNoAllocChunks];

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;   // device -> address of its scratch array

int noalloc_scratch(double** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    it = g_scratch_ptr.emplace(dev, (double*)p).first;
  }
  *out = it->second;
  return SPAI_OK;
}

__global__ void k_zero_flag(int* p) { *p = 0; }

}  // namespace
}  // namespace spai

using namespace spai;

extern "C" int spai_loss_fwd(const spai_csr_t* A, const spai_csr_t* M, double* L,
                             const spai_opts_t* opts) {
  try {
    if (!L) return fail(SPAI_ERR_ARG, "loss: null output");
    LossCall c;
    int rc = c.load(A, M, opts, false);
    if (rc) return rc;
    const bool f32 = opts && opts->precision == SPAI_PREC_MIXED;
    return f32 ? loss_fwd_t<float>(c, L) : loss_fwd_t<double>(c, L);
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

extern "C" int spai_loss_bwd(const spai_csr_t* A, const spai_csr_t* M, double dL, double* gA,
                             double* gM, const spai_opts_t* opts) {
  try {
    LossCall c;
    int rc = c.load(A, M, opts, false);
    if (rc) return rc;
    const bool f32 = opts && opts->precision == SPAI_PREC_MIXED;
    const bool host_out = !A->on_device;
    return f32 ? loss_bwd_t<float>(c, dL, gA, gM, host_out) : loss_bwd_t<double>(c, dL, gA, gM, host_out);
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

extern "C" int spai_loss_fwd_noalloc(const spai_csr_t* A, const spai_csr_t* M, double* L, int* err,
                                     const spai_opts_t* opts) {
  try {
    if (!A || !M || !L || !err) return fail(SPAI_ERR_ARG, "loss_fwd_noalloc: null argument");
    if (A->n != M->n || A->n < 1) return fail(SPAI_ERR_ARG, "loss_fwd_noalloc: bad shapes");
    if (!A->on_device || !M->on_device)
      return fail(SPAI_ERR_ARG, "loss_fwd_noalloc: A and M must be on the device");
    if (A->n > kNoAllocRows)
      return fail(SPAI_ERR_ARG, "loss_fwd_noalloc: more than 2^21 rows (the scratch holds 2^21)");
    if (opts && opts->precision != SPAI_PREC_F64)
      return fail(SPAI_ERR_ARG, "loss_fwd_noalloc: float64 only (the float32 copies would need "
                                "scratch of the matrices' size)");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    double* scr = nullptr;
    int rc = noalloc_scratch(&scr);
    if (rc) return rc;
    double* rowpart = scr;
    double* chunks = scr + kNoAllocRows;
    const Pat pA{A->n, A->rowptr, A->colind}, pM{M->n, M->rowptr, M->colind};
    // the flag is cleared by a kernel (no memset node), so the call can be captured
    hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, s, err);
    const int Lt = 512, Ht = 1024, DG = 64;
    hipLaunchKernelGGL(k_loss_rows<double>, dim3(kGridRows), dim3(SPAI_WAVE),
                       rows_lds(Lt, Ht, DG), s, pA, A->val, pM, M->val, rowpart,
                       (double*)nullptr, 1.0, err, Lt, Ht, DG);
    const int64_t chunk = (A->n + kNoAllocChunks - 1) / kNoAllocChunks;
    const int nb = (int)((A->n + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_sum_chunks, dim3(nb), dim3(256), 0, s, rowpart, A->n, chunk, chunks);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, chunks, (int64_t)nb, L);
    HIPCHK(hipGetLastError());
    return SPAI_OK;
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}
