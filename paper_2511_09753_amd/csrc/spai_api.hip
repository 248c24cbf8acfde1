// spai_api.hip — C ABI and host driver of libspai (see include/spai.h).
//
// The driver validates A once, sizes every device pool for the worst case the cap
// allows (so an iteration never needs the host), and enqueues each iteration as a
// fixed sequence of kernels on the caller's stream.  All step sizes, stopping
// decisions and buffer parities live in device memory; the host synchronises only
// when it returns host results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "spai.h"
#include "spai_kern.hpp"
#include "spai_host.hpp"

using namespace spai;

namespace spai {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int fetch_csr(const spai_csr_t* A, HostCsr& h) {
  if (!A || A->n < 1 || A->nnz < 0 || !A->rowptr || (A->nnz > 0 && (!A->colind || !A->val)))
    return fail(SPAI_ERR_ARG, "CSR: bad shape or null pointer");
  if (A->n > INT32_MAX - 1) return fail(SPAI_ERR_ARG, "CSR: n exceeds the int32 index range");
  h.n = A->n;
  h.nnz = A->nnz;
  h.rowptr.resize(A->n + 1);
  h.col.resize(A->nnz);
  h.val.resize(A->nnz);
  if (A->on_device) {
    HIPCHK(hipMemcpy(h.rowptr.data(), A->rowptr, sizeof(int64_t) * (A->n + 1), hipMemcpyDeviceToHost));
    if (A->nnz) {
      HIPCHK(hipMemcpy(h.col.data(), A->colind, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(h.val.data(), A->val, sizeof(double) * A->nnz, hipMemcpyDeviceToHost));
    }
  } else {
    std::memcpy(h.rowptr.data(), A->rowptr, sizeof(int64_t) * (A->n + 1));
    if (A->nnz) {
      std::memcpy(h.col.data(), A->colind, sizeof(int32_t) * A->nnz);
      std::memcpy(h.val.data(), A->val, sizeof(double) * A->nnz);
    }
  }
  // structure
  if (h.rowptr[0] != 0 || h.rowptr[h.n] != h.nnz) return fail(SPAI_ERR_ARG, "CSR: bad row pointers");
  for (int64_t i = 0; i < h.n; ++i) {
    if (h.rowptr[i + 1] < h.rowptr[i]) return fail(SPAI_ERR_ARG, "CSR: row pointers decrease");
    for (int64_t q = h.rowptr[i]; q < h.rowptr[i + 1]; ++q) {
      const int32_t c = h.col[q];
      if (c < 0 || c >= h.n) return fail(SPAI_ERR_ARG, "CSR: column index out of range");
      if (q > h.rowptr[i] && c <= h.col[q - 1])
        return fail(SPAI_ERR_ARG, "CSR: column indices not sorted and unique");
    }
  }
  for (int64_t q = 0; q < h.nnz; ++q)
    if (!std::isfinite(h.val[q])) return fail(SPAI_ERR_NONFINITE, "CSR: non-finite value");
  return SPAI_OK;
}

int64_t find_entry(const HostCsr& h, int64_t i, int32_t j) {
  const int32_t* b = h.col.data() + h.rowptr[i];
  const int32_t* e = h.col.data() + h.rowptr[i + 1];
  const int32_t* p = std::lower_bound(b, e, j);
  return (p != e && *p == j) ? (int64_t)(p - h.col.data()) : -1;
}

int check_spd_symmetric(const HostCsr& h) {
  for (int64_t i = 0; i < h.n; ++i) {
    bool diag = false;
    for (int64_t q = h.rowptr[i]; q < h.rowptr[i + 1]; ++q) {
      const int32_t j = h.col[q];
      if (j == i) {
        diag = true;
        if (!(h.val[q] > 0.0)) return fail(SPAI_ERR_NOT_SPD, "A: non-positive diagonal entry");
        continue;
      }
      const int64_t t = find_entry(h, j, (int32_t)i);
      if (t < 0 || std::memcmp(&h.val[t], &h.val[q], sizeof(double)) != 0)
        return fail(SPAI_ERR_NOT_SYMMETRIC, "A: not exactly symmetric");
    }
    if (!diag) return fail(SPAI_ERR_NOT_SPD, "A: missing diagonal entry");
  }
  return SPAI_OK;
}

int check_symmetric_pattern(const HostCsr& h) {
  for (int64_t i = 0; i < h.n; ++i)
    for (int64_t q = h.rowptr[i]; q < h.rowptr[i + 1]; ++q)
      if (find_entry(h, h.col[q], (int32_t)i) < 0)
        return fail(SPAI_ERR_ARG, "pattern is not symmetric");
  return SPAI_OK;
}

// Processing order with locality: breadth-first balls of about `ball` rows grown in A's
// graph, each seeded at the smallest row not yet taken and limited to untaken rows,
// concatenated.  Rows processed at the same time then share most of the rows they
// gather, so an XCD's working set stays within its L2.
const int kBallRows = 2048;

void locality_order(const HostCsr& h, int ball, std::vector<int32_t>& order) {
  const int64_t n = h.n;
  order.clear();
  order.reserve((size_t)n);
  std::vector<char> taken((size_t)n, 0);
  std::vector<int32_t> queue;
  int64_t seed = 0;
  while ((int64_t)order.size() < n) {
    while (taken[(size_t)seed]) ++seed;
    queue.clear();
    queue.push_back((int32_t)seed);
    taken[(size_t)seed] = 1;
    size_t head = 0;
    while (head < queue.size() && (int)queue.size() < ball) {
      const int32_t u = queue[head++];
      for (int64_t q = h.rowptr[u]; q < h.rowptr[u + 1] && (int)queue.size() < ball; ++q) {
        const int32_t v = h.col[q];
        if (!taken[(size_t)v]) {
          taken[(size_t)v] = 1;
          queue.push_back(v);
        }
      }
    }
    order.insert(order.end(), queue.begin(), queue.end());
  }
}

int DevPool::alloc_bytes(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  if (limit > 0 && used + bytes > (size_t)limit)
    return fail(SPAI_ERR_NOMEM, "device pool limit exceeded");
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(SPAI_ERR_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  ptrs.push_back(*p);
  used += bytes;
  return SPAI_OK;
}

void DevPool::release() {
  for (void* p : ptrs) (void)hipFree(p);
  ptrs.clear();
  used = 0;
}

DevPool::~DevPool() { release(); }

}  // namespace spai

// ============================================================================
// engine: one handle's device state and iteration sequence
// ============================================================================

namespace {

// ---- column lists <-> compact CSC on the host ---------------------------------------

// out[colptr[j] ..] = the entries of column j (colptr: exclusive prefix of the lengths)
template <typename T>
__global__ void k_pack_cols(Cols<T> C, const int64_t* colptr, int64_t n, int32_t* idx, T* val) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t b = C.beg[j], o = colptr[j];
  const int len = C.len[j];
  for (int e = 0; e < len; ++e) {
    idx[o + e] = C.idx[b + e];
    val[o + e] = C.val[b + e];
  }
}

// download column lists as compact CSC (one packing kernel, three copies)
template <typename T>
int download_cols(const Cols<T>& C, int64_t n, hipStream_t s, std::vector<int64_t>& colptr,
                  std::vector<int32_t>& idx, std::vector<T>& val) {
  std::vector<int32_t> len((size_t)n);
  HIPCHK(hipMemcpyAsync(len.data(), C.len, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  colptr.assign((size_t)n + 1, 0);
  for (int64_t j = 0; j < n; ++j) colptr[j + 1] = colptr[j] + len[j];
  const int64_t nnz = colptr[n];
  idx.resize((size_t)nnz);
  val.resize((size_t)nnz);
  DevPool tmp;
  int rc;
  int64_t* dptr;
  int32_t* didx;
  T* dval;
  if ((rc = tmp.alloc(&dptr, n + 1)) || (rc = tmp.alloc(&didx, nnz)) || (rc = tmp.alloc(&dval, nnz)))
    return rc;
  HIPCHK(hipMemcpyAsync(dptr, colptr.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_pack_cols<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, dptr, n,
                     didx, dval);
  HIPCHK(hipGetLastError());
  if (nnz) {
    HIPCHK(hipMemcpyAsync(idx.data(), didx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(val.data(), dval, sizeof(T) * nnz, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  return SPAI_OK;
}

// check compact CSC lists before any of them is uploaded: column pointers from 0 and
// non-decreasing, at most the pool's capacity, rows in range and strictly ascending within
// each column (the per-column kernels' lock-step searches assume ascending rows)
template <typename T>
int check_cols(const Cols<T>& C, int64_t n, const int64_t* colptr, const int32_t* idx) {
  if (colptr[0] != 0) return fail(SPAI_ERR_ARG, "state: bad column pointers");
  const int64_t nnz = colptr[n];
  if (nnz < 0 || nnz > C.cap) return fail(SPAI_ERR_ARG, "state: a list exceeds this handle's pool");
  for (int64_t j = 0; j < n; ++j) {
    const int64_t l = colptr[j + 1] - colptr[j];
    if (l < 0 || l > INT32_MAX || colptr[j + 1] > nnz)
      return fail(SPAI_ERR_ARG, "state: bad column pointers");
    for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) {
      if (idx[q] < 0 || idx[q] >= n) return fail(SPAI_ERR_ARG, "state: row index out of range");
      if (q > colptr[j] && idx[q] <= idx[q - 1])
        return fail(SPAI_ERR_ARG, "state: rows not strictly ascending in a column");
    }
  }
  return SPAI_OK;
}

// upload compact CSC into column lists (columns laid out from offset 0); check_cols first
template <typename T>
int upload_cols(Cols<T>& C, int64_t n, hipStream_t s, const int64_t* colptr, const int32_t* idx,
                const T* val) {
  const int64_t nnz = colptr[n];
  std::vector<int32_t> len((size_t)n);
  for (int64_t j = 0; j < n; ++j) len[(size_t)j] = (int32_t)(colptr[j + 1] - colptr[j]);
  HIPCHK(hipMemcpyAsync(C.beg, colptr, sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(C.len, len.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  if (nnz) {
    HIPCHK(hipMemcpyAsync(C.idx, idx, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(C.val, val, sizeof(T) * nnz, hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  return SPAI_OK;
}

// serialized handle state: header, per-matrix scalars, then the lists as compact CSC
struct StateHeader {
  char magic[8];
  int32_t version, value_bytes;
  int64_t n;
  int32_t nseg, method, jacobi, implicit, symmetrize, nlists;
  int64_t iters_host, total_iters;
  int64_t nnz[5];
};
constexpr char kStateMagic[8] = {'S', 'P', 'A', 'I', 'S', 'T', 'A', 'T'};

struct EngineBase {
  virtual ~EngineBase() {}
  virtual int iterate(int k, int* done, double* hist) = 0;
  virtual int get(spai_csr_out_t* M) = 0;
  virtual int stats(int* iters, double* resid, int64_t* nnz_m, int64_t* nnz_p, double* s1,
                    double* s2, int* fb) = 0;
  virtual int batched_resid(double* out) = 0;
  virtual int reset() = 0;
  virtual int pcg(int nrhs, const double* B, double* X, double rtol, int max_iter, int* iters,
                  double* relres, int on_device) = 0;
  virtual int profile(double* ms, int64_t* calls, int64_t* counts) = 0;
  virtual int spectrum(int steps, const double* v0, int on_device, double* out,
                       int* steps_done) = 0;
  virtual int autotune(int warm_iters, int reps, int* chosen, double* best_ms) = 0;
  virtual int set_tiles(const int* tiles) = 0;
  virtual int get_state(void* buf, size_t* size) = 0;
  virtual int set_state(const void* buf, size_t size) = 0;
  virtual int history(int64_t* out, int cap, int* count) = 0;
};

template <typename T>
struct Engine : EngineBase {
  // configuration
  int method = 0;
  int64_t n = 0;
  int nseg = 1;
  spai_cap_t cap{};
  spai_opts_t opts{};
  double tol = 0.0;
  int max_iter = 0;
  hipStream_t s = nullptr;
  bool global = false, colcap = false;
  int64_t m_global = 0;
  bool batched_graph = false;
  // host mirror of A
  HostCsr hA;
  std::vector<int64_t> seg_beg_h;
  // device
  DevPool pool;
  PcgWork pcg_work;                  // spai_pcg's blocks, kept between solves of one size
  Csr A;
  Pair<T> M, P, PT;
  Cols<T> R;
  // implicit residual (opts.explicit_residual = 0): the next residual is formed in Rn
  // (and Zn, Pi-weighted) and copied over R; Pi-weighted, R holds Z and Rraw holds R
  Cols<T> Rn{}, Zn{}, Rraw{};
  bool implicit = false;
  int64_t *ub = nullptr, *off = nullptr, *total = nullptr, *scantmp = nullptr;
  double *colpart = nullptr, *colnorm = nullptr, *red = nullptr, *red_rr = nullptr;
  double *colrz = nullptr, *red_rz = nullptr;   // (R, Z)_F per column / matrix (weighted)
  double *blockpart = nullptr, *cvec = nullptr, *hist = nullptr;
  int32_t* kcol = nullptr;
  double *tM = nullptr, *tP = nullptr;
  BigList big[3];
  unsigned long long *selhist = nullptr, *selbuf = nullptr;
  DevState* st = nullptr;
  unsigned long long* cnt = nullptr;
  unsigned long long* rec = nullptr;   // per-iteration drop record, (max_iter + 1) x kRec
  SegState* segst = nullptr;
  int* seg_of = nullptr;
  int64_t* seg_beg = nullptr;
  Seg seg;
  Tile tRs{64, 512}, tRl{1024, 4096}, tDs{128, 512, 0, 1}, tDl{1024, 4096}, tUs{384, 512},
      tUl{2048, 4096};
  Tile tRh{0, 0}, tDh{0, 0}, tUh{0, 0};   // huge tiles (device-memory scratch), sized from n
  Tile tSs{128, 1024}, tSl{1024, 8192}, tSh{0, 0};   // heuristic-score tiles
  double *score = nullptr, *sigma = nullptr;          // per-candidate scores and pair sums
  int32_t* d_order = nullptr;             // locality order of the rows (breadth-first balls)
  int hist_cap = 0;
  int iters_host = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t own_stream = nullptr;
  // phase timing (opts.profile)
  bool prof = false;
  double ph_ms[SPAI_NPHASES] = {};
  int64_t ph_calls[SPAI_NPHASES] = {};
  int64_t total_iters = 0;
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  hipEvent_t ev_open = nullptr;
  int ph_open = -1;

  hipEvent_t ev_get() {
    hipEvent_t e = nullptr;
    if (!ev_free.empty()) {
      e = ev_free.back();
      ev_free.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return e;
  }
  void tb(int ph) {
    if (!prof) return;
    ev_open = ev_get();
    ph_open = ph;
    if (ev_open) (void)hipEventRecord(ev_open, s);
  }
  void te() {
    if (!prof || !ev_open) return;
    hipEvent_t b = ev_get();
    if (!b) return;
    (void)hipEventRecord(b, s);
    ev_pending.push_back({ph_open, {ev_open, b}});
    ev_open = nullptr;
  }
  void collect() {                     // after a synchronisation
    for (auto& p : ev_pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
        ph_ms[p.first] += ms;
        ph_calls[p.first] += 1;
      } else {
        (void)hipGetLastError();
      }
      ev_free.push_back(p.second.first);
      ev_free.push_back(p.second.second);
    }
    ev_pending.clear();
  }

  ~Engine() override {
    if (s) (void)hipStreamSynchronize(s);
    for (auto& p : ev_pending) {
      (void)hipEventDestroy(p.second.first);
      (void)hipEventDestroy(p.second.second);
    }
    for (auto e : ev_free) (void)hipEventDestroy(e);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (own_stream) {
      (void)hipStreamSynchronize(own_stream);
      (void)hipStreamDestroy(own_stream);
    }
  }

  template <typename U>
  int dalloc(U** p, int64_t count) {
    return pool.alloc_bytes((void**)p, sizeof(U) * (size_t)std::max<int64_t>(count, 1));
  }

  int alloc_cols(Cols<T>& c, int64_t capacity) {
    int rc;
    if ((rc = dalloc(&c.beg, n))) return rc;
    if ((rc = dalloc(&c.len, n))) return rc;
    if ((rc = dalloc(&c.idx, capacity))) return rc;
    if ((rc = dalloc(&c.val, capacity))) return rc;
    c.cap = capacity;
    return SPAI_OK;
  }

  int setup(const std::vector<int64_t>& segs) {
    int rc;
    seg_beg_h = segs;
    nseg = (int)segs.size() - 1;
    global = cap.mode == SPAI_CAP_GLOBAL;
    colcap = cap.mode == SPAI_CAP_COLUMN;
    s = (hipStream_t)opts.stream;
    if (batched_graph && !s) {          // graphs cannot be captured on the null stream
      HIPCHK(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
      s = own_stream;
    }
    pool.limit = opts.device_pool_limit;
    // ---- caps and worst-case sizes
    int64_t maxdeg = 0;
    for (int64_t i = 0; i < n; ++i) maxdeg = std::max(maxdeg, hA.rowptr[i + 1] - hA.rowptr[i]);
    const double n2 = (double)n * (double)n;
    double nnzM_max = n2;
    std::vector<int32_t> kc;
    if (global) {
      const double mv = cap.relative ? cap.value * (double)hA.nnz : cap.value;
      if (!(mv >= (double)n)) return fail(SPAI_ERR_ARG, "global cap below the diagonal count n");
      m_global = (int64_t)std::llround(mv);
      nnzM_max = std::min(n2, (double)m_global);
    } else if (colcap) {
      kc.resize(n);
      double sum = 0.0;
      for (int64_t j = 0; j < n; ++j) {
        const double deg = (double)(hA.rowptr[j + 1] - hA.rowptr[j]);
        const double kv = cap.relative ? cap.value * deg : cap.value;
        const int64_t k = (int64_t)std::llround(kv);
        if (k < 1) return fail(SPAI_ERR_ARG, "column cap below one (the diagonal)");
        kc[j] = (int32_t)std::min<int64_t>(k, n);
        sum += kc[j];
      }
      nnzM_max = std::min(n2, sum);
    } else if (cap.mode != SPAI_CAP_NONE) {
      return fail(SPAI_ERR_ARG, "unknown cap mode");
    }
    const double nnzP_max = method == SPAI_MR ? 0.0 : nnzM_max;
    // offsets come from per-column bounds that count duplicate products, so the pools
    // hold the sum of the bounds (not the number of distinct entries)
    // (the implicit update's bound also counts supp(R_i): up to n^2 more)
    const double capR_d = (double)n + nnzM_max * (double)maxdeg + (opts.explicit_residual ? 0.0 : n2);
    const double capU_d = (double)n + nnzM_max + capR_d + 2.0 * nnzP_max + nnzM_max * (double)maxdeg;
    if (capU_d > 4.0e9) return fail(SPAI_ERR_NOMEM, "worst-case pattern too large (set a cap)");
    const int64_t capR = (int64_t)capR_d, capU = (int64_t)capU_d;
    // ---- A
    int64_t* d_rowptr;
    int32_t* d_col;
    double* d_val;
    if ((rc = dalloc(&d_rowptr, n + 1)) || (rc = dalloc(&d_col, hA.nnz)) || (rc = dalloc(&d_val, hA.nnz)))
      return rc;
    HIPCHK(hipMemcpyAsync(d_rowptr, hA.rowptr.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_col, hA.col.data(), sizeof(int32_t) * hA.nnz, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_val, hA.val.data(), sizeof(double) * hA.nnz, hipMemcpyHostToDevice, s));
    A.n = n;
    A.nnz = hA.nnz;
    A.rowptr = d_rowptr;
    A.col = d_col;
    A.val = d_val;
    std::vector<float> v32;
    if (opts.precision == SPAI_PREC_MIXED) {
      float* d_v32;
      if ((rc = dalloc(&d_v32, hA.nnz))) return rc;
      v32.resize(hA.nnz);
      for (int64_t q = 0; q < hA.nnz; ++q) v32[q] = (float)hA.val[q];
      HIPCHK(hipMemcpyAsync(d_v32, v32.data(), sizeof(float) * hA.nnz, hipMemcpyHostToDevice, s));
      A.val32 = d_v32;
    }
    // ELL copy: row u in slots [u W, (u + 1) W), W = max(8, 2^ceil(log2 maxdeg))
    const bool ell_ok = maxdeg <= 64;
    if (opts.a_format == SPAI_AFMT_ELL && !ell_ok)
      return fail(SPAI_ERR_ARG, "a_format ELL: a row of A has more than 64 entries");
    if (opts.a_format != SPAI_AFMT_CSR && ell_ok) {
      int sh = 3;
      while ((int64_t(1) << sh) < maxdeg) ++sh;
      const int64_t W = int64_t(1) << sh, tot = n * W;
      std::vector<int32_t> ec((size_t)tot, -1);
      std::vector<double> evv((size_t)tot, 0.0);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t q = hA.rowptr[i]; q < hA.rowptr[i + 1]; ++q) {
          ec[(size_t)(i * W + q - hA.rowptr[i])] = hA.col[q];
          evv[(size_t)(i * W + q - hA.rowptr[i])] = hA.val[q];
        }
      int32_t* d_ec;
      double* d_ev;
      if ((rc = dalloc(&d_ec, tot)) || (rc = dalloc(&d_ev, tot))) return rc;
      HIPCHK(hipMemcpyAsync(d_ec, ec.data(), sizeof(int32_t) * tot, hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(d_ev, evv.data(), sizeof(double) * tot, hipMemcpyHostToDevice, s));
      if (opts.precision == SPAI_PREC_MIXED) {
        std::vector<float> ev32((size_t)tot);
        for (int64_t q = 0; q < tot; ++q) ev32[(size_t)q] = (float)evv[(size_t)q];
        float* d_ev32;
        if ((rc = dalloc(&d_ev32, tot))) return rc;
        HIPCHK(hipMemcpyAsync(d_ev32, ev32.data(), sizeof(float) * tot, hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        A.eval32 = d_ev32;
      }
      HIPCHK(hipStreamSynchronize(s));
      A.eshift = sh;
      A.ecol = d_ec;
      A.eval = d_ev;
      // A in ELL: the residual and dots run their lean resident tiers, whose ordered key
      // sets take any power-of-two H (the tiles the tuner picks on the 96^3 stencil)
      tRs = Tile{128, 1024};
      tDs = Tile{256, 1024, 0, 1};
      tUs = Tile{128, 256, 0, 1};                // the update's lean tier
    }
    // ---- locality order of the rows (for the PCG products)
    {
      std::vector<int32_t> ord;
      locality_order(hA, kBallRows, ord);
      if ((rc = dalloc(&d_order, n))) return rc;
      HIPCHK(hipMemcpyAsync(d_order, ord.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    // ---- state
    if ((rc = dalloc(&st, 1)) || (rc = dalloc(&segst, nseg)) || (rc = dalloc(&seg_beg, nseg + 1)) ||
        (rc = dalloc(&cnt, (int64_t)kNCnt * kCntSlots)))
      return rc;
    HIPCHK(hipMemsetAsync(st, 0, sizeof(DevState), s));
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * kNCnt * kCntSlots, s));
    HIPCHK(hipMemcpyAsync(&st->cnt, &cnt, sizeof(cnt), hipMemcpyHostToDevice, s));
    {   // per-iteration drop record (spai_history)
      const int rcap = max_iter + 1;
      if ((rc = dalloc(&rec, (int64_t)rcap * kRec))) return rc;
      HIPCHK(hipMemcpyAsync(&st->rec, &rec, sizeof(rec), hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(&st->rec_cap, &rcap, sizeof(int), hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemsetAsync(segst, 0, sizeof(SegState) * nseg, s));
    HIPCHK(hipMemcpyAsync(seg_beg, seg_beg_h.data(), sizeof(int64_t) * (nseg + 1), hipMemcpyHostToDevice, s));
    std::vector<int> segof_h;
    if (nseg > 1) {
      if ((rc = dalloc(&seg_of, n))) return rc;
      segof_h.resize(n);
      for (int g = 0; g < nseg; ++g)
        for (int64_t j = seg_beg_h[g]; j < seg_beg_h[g + 1]; ++j) segof_h[j] = g;
      HIPCHK(hipMemcpyAsync(seg_of, segof_h.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    }
    seg.nseg = nseg;
    seg.of = seg_of;
    seg.st = segst;
    // ---- iterate pools
    const int64_t capP = method == SPAI_MR ? 1 : capU;
    for (int b = 0; b < 2; ++b) {
      if ((rc = alloc_cols(M.b[b], capU))) return rc;
      if ((rc = alloc_cols(P.b[b], capP))) return rc;
      if ((rc = alloc_cols(PT.b[b], capP))) return rc;
    }
    if ((rc = alloc_cols(R, capR))) return rc;
    implicit = !opts.explicit_residual;
    if (implicit) {
      if ((rc = alloc_cols(Rn, capR))) return rc;
      if (opts.jacobi && ((rc = alloc_cols(Zn, capR)) || (rc = alloc_cols(Rraw, capR)))) return rc;
    }
    M.cur = &st->curM;
    P.cur = &st->curP;
    PT.cur = &st->curP;
    if ((rc = dalloc(&ub, n)) || (rc = dalloc(&off, n)) || (rc = dalloc(&total, 1)) ||
        (rc = dalloc(&scantmp, scan_tmp_elems(n))))
      return rc;
    if ((rc = dalloc(&colpart, n * kND)) || (rc = dalloc(&colnorm, n)) ||
        (rc = dalloc(&red, (int64_t)nseg * kND)) || (rc = dalloc(&red_rr, nseg)) ||
        (rc = dalloc(&blockpart, 1024 * kND)) || (rc = dalloc(&cvec, nseg)))
      return rc;
    if (opts.jacobi && ((rc = dalloc(&colrz, n)) || (rc = dalloc(&red_rz, nseg)))) return rc;
    hist_cap = std::max(max_iter, 1);
    if ((rc = dalloc(&hist, (int64_t)nseg * hist_cap))) return rc;
    if (colcap) {
      if ((rc = dalloc(&kcol, n)) || (rc = dalloc(&tM, n)) || (rc = dalloc(&tP, n))) return rc;
      HIPCHK(hipMemcpyAsync(kcol, kc.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    }
    for (int b = 0; b < 3; ++b)
      if ((rc = dalloc(&big[b].list, n)) || (rc = dalloc(&big[b].count, 1)) ||
          (rc = dalloc(&big[b].list2, n)) || (rc = dalloc(&big[b].count2, 1)))
        return rc;
    // huge tiles: a column's lists and key set can reach n entries (the residual's and the
    // dots' lists are held under 32768 so map positions fit in 16 bits)
    {
      auto p2 = [](int64_t x) { int64_t p = 1; while (p < x) p <<= 1; return p; };
      const bool ell = A.eshift >= 0;
      const int64_t Lr = std::max<int64_t>(2048, std::min<int64_t>(32768, p2(n)));
      const int64_t Ld = std::max<int64_t>(2048, std::min<int64_t>(32768, p2(2 * n)));
      const int64_t Lu = std::max<int64_t>(4096, std::min<int64_t>(131072, p2(4 * n)));
      const int64_t Hk = std::max<int64_t>(8192, std::min<int64_t>(131072, 2 * p2(n + 1)));
      tRh = Tile{(int)Lr, (int)Hk};
      tDh = Tile{(int)Ld, (int)Hk};
      tUh = Tile{(int)Lu, (int)Hk, (int)std::max<int64_t>(256, p2(maxdeg))};
      tSh = Tile{(int)Lr, (int)Hk};
      int64_t stride = (int64_t)std::max({resid_tile_bytes(tRh, ell), dots_tile_bytes(tDh, ell),
                                          update_tile_bytes(tUh)});
      if (opts.drop_score) stride = std::max<int64_t>(stride, (int64_t)score_tile_bytes(tSh, ell));
      stride = (stride + 255) / 256 * 256;
      const int grid2 = (int)std::min<int64_t>(
          kHugeGridMax, std::max<int64_t>(kHugeGridMin, kHugeBudget / stride / 8 * 8));
      char* scr;
      if ((rc = dalloc(&scr, stride * grid2))) return rc;
      for (int b = 0; b < 3; ++b) {
        big[b].scratch = scr;
        big[b].scratch_stride = stride;
        big[b].grid2 = grid2;
      }
    }
    if (global) {
      if ((rc = dalloc(&selhist, 8192)) || (rc = dalloc(&selbuf, capU))) return rc;
      if (opts.drop_score && ((rc = dalloc(&score, capU)) || (rc = dalloc(&sigma, capU)))) return rc;
    }
    prof = opts.profile != 0 && !batched_graph;
    return init_iterate();
  }

  // M_0 = c I, R_0, and CG's P_0
  int init_iterate() {
    launch_rec_clear(st, 0, s);
    launch_trace_parts(A, colpart, s);
    launch_reduce(colpart, 2, n, seg, nseg > 1 ? seg_beg : nullptr, red, blockpart, s);
    launch_init_state(seg, red, nseg > 1 ? seg_beg : nullptr, n, cvec, method, st, s);
    launch_init_m<T>(n, M.b[0], cvec, seg, s);
    if (method != SPAI_MR)
      for (int b = 0; b < 2; ++b) {
        launch_zero_cols<T>(n, P.b[b], s);
        launch_zero_cols<T>(n, PT.b[b], s);
      }
    resid_step(1);
    if (method == SPAI_CG) p_update_step();
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    collect();
    iters_host = 0;
    return check_err();
  }

  int reset() override { return init_iterate(); }

  int pcg(int nrhs, const double* B, double* X, double rtol, int max_iter, int* iters,
          double* relres, int on_device) override {
    if (!opts.symmetrize) return fail(SPAI_ERR_ARG, "spai_pcg needs a symmetrized iterate");
    if (nrhs < 1 || !B || !X || !(rtol >= 0.0) || max_iter < 0)
      return fail(SPAI_ERR_ARG, "spai_pcg: bad arguments");
    HIPCHK(hipStreamSynchronize(s));
    DevState h;
    HIPCHK(hipMemcpy(&h, st, sizeof(DevState), hipMemcpyDeviceToHost));
    const Cols<T>& C = M.b[h.curM];
    PcgMat pa, pm;
    pa.n = n;
    // A's ELL copy saves the row-pointer load of each row, but its padded rows are read
    // whole: with more than twice the stored entries in padding the CSR copy is faster
    // (measured: 1.15x padding at 96^3 favours ELL by 5%, 3.6x on the geometric graphs
    // favours CSR by 7%).  Both hold each row in ascending column order: same sums.
    if (A.eshift >= 0 && (n << A.eshift) <= 2 * A.nnz) {
      pa.eshift = A.eshift;
      pa.col = A.ecol;
      pa.val = A.eval;
    } else {
      pa.rowptr = A.rowptr;
      pa.col = A.col;
      pa.val = A.val;
    }
    pm.n = n;
    pm.beg = C.beg;
    pm.len = C.len;
    pm.col = C.idx;
    if (sizeof(T) == 4) pm.val32 = (const float*)C.val; else pm.val = (const double*)C.val;
    DevPool tmp;
    int rc;
    const int64_t tot = n * (int64_t)nrhs;
    const double* dB = B;
    double* dX = X;
    if (!on_device) {
      double *b2, *x2;
      if ((rc = tmp.alloc(&b2, tot)) || (rc = tmp.alloc(&x2, tot))) return rc;
      HIPCHK(hipMemcpyAsync(b2, B, sizeof(double) * tot, hipMemcpyHostToDevice, s));
      dB = b2;
      dX = x2;
    }
    tb(SPAI_PH_PCG);
    PcgTiming tm;
    rc = pcg_run(pa, pm, nrhs, dB, dX, rtol, max_iter, iters, relres, d_order, s,
                 prof ? &tm : nullptr, &pcg_work);
    te();
    if (prof) {
      ph_ms[SPAI_PH_PCG_AX] += tm.ms[0];
      ph_calls[SPAI_PH_PCG_AX] += tm.calls[0];
      ph_ms[SPAI_PH_PCG_MX] += tm.ms[1];
      ph_calls[SPAI_PH_PCG_MX] += tm.calls[1];
    }
    if (rc < 0) return rc;
    if (!on_device) {
      HIPCHK(hipMemcpyAsync(X, dX, sizeof(double) * tot, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    collect();
    return rc;
  }

  // the lists a state holds: M, and for CG / LOMR P and P^T, R, and the implicit
  // Pi-weighted form's R beside Z
  void state_lists(const DevState& h, Cols<T>* out[5], int& k) {
    k = 0;
    out[k++] = &M.b[h.curM];
    if (method != SPAI_MR) {
      out[k++] = &P.b[h.curP];
      out[k++] = &PT.b[h.curP];
    }
    out[k++] = &R;
    if (implicit && opts.jacobi) out[k++] = &Rraw;
  }

  int get_state(void* buf, size_t* size) override {
    if (!size) return fail(SPAI_ERR_ARG, "spai_get_state: null size");
    HIPCHK(hipStreamSynchronize(s));
    DevState h;
    HIPCHK(hipMemcpy(&h, st, sizeof(DevState), hipMemcpyDeviceToHost));
    Cols<T>* lists[5];
    int nl = 0;
    state_lists(h, lists, nl);
    StateHeader hd{};
    std::memcpy(hd.magic, kStateMagic, 8);
    hd.version = 1;
    hd.value_bytes = (int32_t)sizeof(T);
    hd.n = n;
    hd.nseg = nseg;
    hd.method = method;
    hd.jacobi = opts.jacobi;
    hd.implicit = implicit ? 1 : 0;
    hd.symmetrize = opts.symmetrize;
    hd.nlists = nl;
    hd.iters_host = iters_host;
    hd.total_iters = total_iters;
    std::vector<std::vector<int64_t>> cp(nl);
    std::vector<std::vector<int32_t>> ix(nl);
    std::vector<std::vector<T>> vl(nl);
    int rc;
    for (int l = 0; l < nl; ++l) {
      if ((rc = download_cols<T>(*lists[l], n, s, cp[l], ix[l], vl[l]))) return rc;
      hd.nnz[l] = cp[l][n];
    }
    size_t need = sizeof(StateHeader) + sizeof(SegState) * (size_t)nseg;
    for (int l = 0; l < nl; ++l)
      need += sizeof(int64_t) * (size_t)(n + 1) + (sizeof(int32_t) + sizeof(T)) * (size_t)hd.nnz[l];
    if (!buf) {
      *size = need;
      return SPAI_OK;
    }
    if (*size < need) return fail(SPAI_ERR_ARG, "spai_get_state: buffer too small");
    *size = need;
    char* o = (char*)buf;
    std::memcpy(o, &hd, sizeof(hd));
    o += sizeof(hd);
    HIPCHK(hipMemcpy(o, segst, sizeof(SegState) * nseg, hipMemcpyDeviceToHost));
    o += sizeof(SegState) * nseg;
    for (int l = 0; l < nl; ++l) {
      std::memcpy(o, cp[l].data(), sizeof(int64_t) * (n + 1));
      o += sizeof(int64_t) * (n + 1);
      std::memcpy(o, ix[l].data(), sizeof(int32_t) * hd.nnz[l]);
      o += sizeof(int32_t) * hd.nnz[l];
      std::memcpy(o, vl[l].data(), sizeof(T) * hd.nnz[l]);
      o += sizeof(T) * hd.nnz[l];
    }
    return SPAI_OK;
  }

  int set_state(const void* buf, size_t size) override {
    if (!buf || size < sizeof(StateHeader)) return fail(SPAI_ERR_ARG, "spai_set_state: bad buffer");
    StateHeader hd;
    std::memcpy(&hd, buf, sizeof(hd));
    if (std::memcmp(hd.magic, kStateMagic, 8) != 0 || hd.version != 1)
      return fail(SPAI_ERR_ARG, "spai_set_state: not a state of this library");
    if (hd.value_bytes != (int32_t)sizeof(T) || hd.n != n || hd.nseg != nseg ||
        hd.method != method || hd.jacobi != opts.jacobi || hd.implicit != (implicit ? 1 : 0) ||
        hd.symmetrize != opts.symmetrize)
      return fail(SPAI_ERR_ARG, "spai_set_state: state of a different problem or configuration");
    if (hd.iters_host < 0 || hd.iters_host > max_iter)
      return fail(SPAI_ERR_ARG, "spai_set_state: iterations beyond this handle's max_iter");
    HIPCHK(hipStreamSynchronize(s));
    DevState h;
    HIPCHK(hipMemcpy(&h, st, sizeof(DevState), hipMemcpyDeviceToHost));
    Cols<T>* lists[5];
    int nl = 0;
    state_lists(h, lists, nl);
    if (hd.nlists != nl) return fail(SPAI_ERR_ARG, "spai_set_state: list count differs");
    size_t need = sizeof(StateHeader) + sizeof(SegState) * (size_t)nseg;
    for (int l = 0; l < nl; ++l) {
      if (hd.nnz[l] < 0) return fail(SPAI_ERR_ARG, "spai_set_state: bad sizes");
      need += sizeof(int64_t) * (size_t)(n + 1) + (sizeof(int32_t) + sizeof(T)) * (size_t)hd.nnz[l];
    }
    if (size < need) return fail(SPAI_ERR_ARG, "spai_set_state: truncated buffer");
    const char* o = (const char*)buf + sizeof(hd);
    std::vector<SegState> g((size_t)nseg);
    std::memcpy(g.data(), o, sizeof(SegState) * nseg);
    o += sizeof(SegState) * nseg;
    bool any = false;
    for (auto& x : g) {
      if (x.iters < 0) return fail(SPAI_ERR_ARG, "spai_set_state: bad iteration count");
      any = any || !x.stop;
    }
    int rc;
    // every list is read and checked before the first one is uploaded, so a bad state
    // leaves the handle unchanged
    std::vector<std::vector<int64_t>> cps((size_t)nl);
    std::vector<std::vector<int32_t>> ixs((size_t)nl);
    std::vector<std::vector<T>> vls((size_t)nl);
    for (int l = 0; l < nl; ++l) {
      cps[l].resize((size_t)n + 1);
      std::memcpy(cps[l].data(), o, sizeof(int64_t) * (n + 1));
      o += sizeof(int64_t) * (n + 1);
      if (cps[l][n] != hd.nnz[l]) return fail(SPAI_ERR_ARG, "spai_set_state: bad column pointers");
      ixs[l].resize((size_t)hd.nnz[l]);
      std::memcpy(ixs[l].data(), o, sizeof(int32_t) * hd.nnz[l]);
      o += sizeof(int32_t) * hd.nnz[l];
      vls[l].resize((size_t)hd.nnz[l]);
      std::memcpy(vls[l].data(), o, sizeof(T) * hd.nnz[l]);
      o += sizeof(T) * hd.nnz[l];
      if ((rc = check_cols<T>(*lists[l], n, cps[l].data(), ixs[l].data()))) return rc;
    }
    for (int l = 0; l < nl; ++l)
      if ((rc = upload_cols<T>(*lists[l], n, s, cps[l].data(), ixs[l].data(), vls[l].data())))
        return rc;
    HIPCHK(hipMemcpy(segst, g.data(), sizeof(SegState) * nseg, hipMemcpyHostToDevice));
    h.any_active = any ? 1 : 0;
    h.iter_active = any ? 1 : 0;
    h.err = 0;
    HIPCHK(hipMemcpy(st, &h, sizeof(DevState), hipMemcpyHostToDevice));
    iters_host = (int)hd.iters_host;
    total_iters = hd.total_iters;
    launch_rec_clear(st, iters_host, s);   // records resume at the restored iteration
    HIPCHK(hipStreamSynchronize(s));
    return SPAI_OK;
  }

  // per-iteration drop record: 6 int64 per iteration i < *count (see spai_history)
  int history(int64_t* out, int cap, int* count) override {
    if (!count || cap < 0 || (cap > 0 && !out)) return fail(SPAI_ERR_ARG, "spai_history: bad arguments");
    HIPCHK(hipStreamSynchronize(s));
    const int nrec = std::min(iters_host, max_iter + 1);
    *count = nrec;
    const int k = std::min(cap, nrec);
    if (k > 0) {
      std::vector<unsigned long long> r((size_t)k * kRec);
      HIPCHK(hipMemcpy(r.data(), rec, sizeof(unsigned long long) * r.size(), hipMemcpyDeviceToHost));
      for (int i = 0; i < k; ++i) {
        const unsigned long long* x = &r[(size_t)i * kRec];
        int64_t* o = out + (size_t)i * 6;
        o[0] = (int64_t)x[0];              // nnz(M_{i+1}) (kept)
        o[1] = (int64_t)(x[1] - x[0]);     // M candidates dropped by the cap
        o[2] = (int64_t)x[2];              // of those, at the cut
        o[3] = (int64_t)x[3];              // nnz(P_i) (kept; 0 for MR)
        o[4] = (int64_t)(x[4] - x[3]);
        o[5] = (int64_t)x[5];
      }
    }
    return SPAI_OK;
  }

  static bool same_tile(const Tile& a, const Tile& b) {
    return a.L == b.L && a.H == b.H && a.waves == b.waves;
  }

  // Tiles chosen by the caller (for instance those a previous spai_autotune reported):
  // checked against what the kernels assume, then used from the next launch on.
  int set_tiles(const int* c) override {
    if (!c) return fail(SPAI_ERR_ARG, "spai_set_tiles: null tiles");
    auto pow2 = [](int x) { return x > 0 && (x & (x - 1)) == 0; };
    // H: the key set's insertion batches assume H >= 512 (limit + 256 < H); the
    // residual's and dots' position maps hold next_pow2(2 L) slots, so their L is a
    // power of two; every tile fits the 64 KB of LDS a workgroup may take.
    const bool ell = A.eshift >= 0;
    constexpr size_t kMaxLds = 64 * 1024;
    Tile r{c[0], c[1]}, d{c[2], c[3]}, u{c[4], c[5]};
    u.waves = c[6];
    d.waves = c[7];
    // d.waves 1 selects the lean dots tier (A in ELL), whose ordered key set takes any
    // power-of-two H >= 128
    const bool dlean = d.waves == 1;
    const bool ulean = u.waves == 1 && ell;              // the update's lean tier
    const bool ok = pow2(r.L) && r.L >= 32 && pow2(d.L) && d.L >= 32 && u.L >= 32 &&
                    pow2(r.H) && r.H >= (ell ? 128 : 512) && pow2(d.H) &&
                    d.H >= (dlean ? 128 : 512) &&
                    pow2(u.H) && u.H >= (ulean ? 128 : 512) &&
                    (u.waves == 0 || u.waves == 5 || ulean) &&
                    (d.waves == 0 || d.waves == 5 || (dlean && ell)) &&
                    resid_tile_bytes(r, ell) <= kMaxLds && dots_tile_bytes(d, ell) <= kMaxLds &&
                    update_tile_bytes(u) <= kMaxLds;
    if (!ok) return fail(SPAI_ERR_ARG, "spai_set_tiles: tile outside what the kernels accept");
    HIPCHK(hipStreamSynchronize(s));
    tRs = r;
    tDs = d;
    tUs = u;
    if (graph_exec) {                   // a captured iteration holds the old tiles
      (void)hipGraphExecDestroy(graph_exec);
      graph_exec = nullptr;
    }
    if (graph) {
      (void)hipGraphDestroy(graph);
      graph = nullptr;
    }
    return SPAI_OK;
  }

  // Tile autotuner: run warm_iters iterations, then time every candidate small tile of
  // the residual, dots and update kernels (all three tiers of one launch, best of reps)
  // on that one state, and restart from M_0.  A candidate replaces the handle's current
  // tile only when it is at least 3% faster: one state is a noisy stand-in for a whole
  // run, and near-ties measured on it have gone either way over the iterations that
  // follow.  A tile only moves the boundary between the tiers (which columns a kernel
  // defers to its larger tiles); every column's arithmetic and every sum's order are the
  // same in all tiers, so the results do not depend on the choice.
  int autotune(int warm_iters, int reps, int* chosen, double* best_ms) override {
    if (warm_iters < 0 || reps < 1) return fail(SPAI_ERR_ARG, "spai_autotune: bad arguments");
    int rc;
    if ((rc = init_iterate())) return rc;
    const int warm = std::min(warm_iters, max_iter);
    if (warm > 0) {
      int done = 0;
      rc = iterate(warm, &done, nullptr);
      if (rc < 0) return rc;
    }
    HIPCHK(hipStreamSynchronize(s));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return fail(SPAI_ERR_HIP, "spai_autotune: event creation failed");
    }
    auto timed = [&](auto&& launch) -> double {
      double best = 1e300;
      for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(e0, s);
        launch();
        (void)hipEventRecord(e1, s);
        float ms = 0.f;
        if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
          best = std::min(best, (double)ms);
        else
          (void)hipGetLastError();
      }
      return best;
    };
    const bool ell = A.eshift >= 0;
    constexpr size_t kMaxLds = 64 * 1024;
    // residual: R = I - A M on the current M (rewrites R with the same values)
    launch_bound_resid<T>(A, M, ub, n, st, s);
    launch_scan(ub, off, total, n, scantmp, s);
    Tile bestR = tRs;
    double tR = 1e300, curR = 1e300;
    for (int L : {64, 128, 256})
      for (int H : {256, 512, 1024}) {
        const Tile t{L, H};
        if (H < 512 && !ell) continue;
        if (resid_tile_bytes(t, ell) > kMaxLds) continue;
        const double ms = timed([&] {
          launch_resid<T>(A, M, R, off, total, colnorm, opts.jacobi, colrz, big[0], st, t, tRl,
                          tRh, s);
        });
        if (same_tile(t, tRs)) curR = ms;
        if (ms < tR) { tR = ms; bestR = t; }
      }
    // dots: A R, A P on the current R, P (per-column partials only)
    const int useR = method != SPAI_CG, useP = method != SPAI_MR;
    Tile bestD = tDs;
    double tD = 1e300, curD = 1e300;
    for (int L : {64, 128, 256, 512})
      for (int H : {256, 512, 1024})
        for (int waves : {0, 5, 1}) {        // 5: the register-capped tier, 1: the lean tier
          Tile t{L, H};
          t.waves = waves;
          if (waves == 1 && !ell) continue;
          if (waves != 1 && (H < 512 || L < 128)) continue;
          if (dots_tile_bytes(t, ell) > kMaxLds) continue;
          const double ms = timed([&] {
            launch_dots<T>(A, R, P, useR, useP, opts.jacobi, colpart, big[1], st, t, tDl, tDh, s);
          });
          if (same_tile(t, tDs)) curD = ms;
          if (ms < tD) { tD = ms; bestD = t; }
        }
    // update: the candidates of M (and P) written to the next buffers
    const UpdMode md = method == SPAI_MR ? mode(1, 1, 0, 0)
                       : method == SPAI_CG ? mode(1, 2, 0, 0) : mode(1, 1, 2, 1);
    launch_bound_update<T>(A, M, R, P, PT, md, ub, n, st, s);
    launch_scan(ub, off, total, n, scantmp, s);
    Tile bestU = tUs;
    double tU = 1e300, curU = 1e300;
    for (int L : {128, 256, 384, 512})
      for (int H : {128, 256, 512, 1024})
        for (int waves : {0, 5, 1}) {        // 5: the register-capped tier, 1: the lean tier
          Tile t{L, H};
          t.waves = waves;
          if (waves == 1 ? (A.eshift < 0 || L != 128) : (H < 512 || L < 256)) continue;
          if (update_tile_bytes(t) > kMaxLds) continue;
          const double ms = timed([&] {
            launch_update<T>(A, M, R, P, PT, md, off, total, kcol, tM, tP, big[2], seg, st, t,
                             tUl, tUh, s);
          });
          if (same_tile(t, tUs)) curU = ms;
          if (ms < tU) { tU = ms; bestU = t; }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipGetLastError());
    if ((rc = check_err())) return rc;
    constexpr double kGain = 0.97;   // a candidate must beat the current tile by 3%
    if (tR < kGain * curR) tRs = bestR; else if (curR < 1e300) tR = curR;
    if (tD < kGain * curD) tDs = bestD; else if (curD < 1e300) tD = curD;
    if (tU < kGain * curU) tUs = bestU; else if (curU < 1e300) tU = curU;
    if (chosen) {
      chosen[0] = tRs.L; chosen[1] = tRs.H;
      chosen[2] = tDs.L; chosen[3] = tDs.H;
      chosen[4] = tUs.L; chosen[5] = tUs.H;
      chosen[6] = tUs.waves;
      chosen[7] = tDs.waves;
    }
    if (best_ms) {
      best_ms[0] = tR < 1e300 ? tR : 0.0;
      best_ms[1] = tD < 1e300 ? tD : 0.0;
      best_ms[2] = tU < 1e300 ? tU : 0.0;
    }
    if (graph_exec) {                   // the captured iteration holds the old tiles
      (void)hipGraphExecDestroy(graph_exec);
      graph_exec = nullptr;
    }
    if (graph) {
      (void)hipGraphDestroy(graph);
      graph = nullptr;
    }
    return init_iterate();
  }

  int spectrum(int steps, const double* v0, int on_device, double* out,
               int* steps_done) override {
    if (!opts.symmetrize) return fail(SPAI_ERR_ARG, "spai_spectrum needs a symmetrized iterate");
    if (!v0 || !out) return fail(SPAI_ERR_ARG, "spai_spectrum: null argument");
    HIPCHK(hipStreamSynchronize(s));
    DevState h;
    HIPCHK(hipMemcpy(&h, st, sizeof(DevState), hipMemcpyDeviceToHost));
    const Cols<T>& C = M.b[h.curM];
    PcgMat pm;
    pm.n = n;
    pm.beg = C.beg;
    pm.len = C.len;
    pm.col = C.idx;
    if (sizeof(T) == 4) pm.val32 = (const float*)C.val; else pm.val = (const double*)C.val;
    DevPool tmp;
    int rc;
    const double* dv0 = v0;
    if (!on_device) {
      double* d;
      if ((rc = tmp.alloc(&d, n))) return rc;
      HIPCHK(hipMemcpyAsync(d, v0, sizeof(double) * n, hipMemcpyHostToDevice, s));
      dv0 = d;
    }
    const int64_t rest = opts.device_pool_limit > 0
                             ? std::max<int64_t>(1, opts.device_pool_limit - (int64_t)pool.used)
                             : 0;
    return lanczos_run(pm, steps, dv0, out, steps_done, rest, s);
  }

  int profile(double* ms, int64_t* calls, int64_t* counts) override {
    HIPCHK(hipStreamSynchronize(s));
    collect();
    for (int i = 0; i < SPAI_NPHASES; ++i) {
      if (ms) ms[i] = ph_ms[i];
      if (calls) calls[i] = ph_calls[i];
    }
    if (counts) {
      std::vector<unsigned long long> c((size_t)kNCnt * kCntSlots);
      HIPCHK(hipMemcpy(c.data(), cnt, sizeof(unsigned long long) * c.size(), hipMemcpyDeviceToHost));
      int64_t sums[kNCnt] = {};
      for (int k = 0; k < kNCnt; ++k)
        for (int b = 0; b < kCntSlots; ++b) sums[k] += (int64_t)c[(size_t)k * kCntSlots + b];
      for (int k = 0; k < 3; ++k) {
        counts[SPAI_CNT_CAND_M + k] = sums[k];
        counts[SPAI_CNT_KEPT_M + k] = sums[3 + k];
      }
      counts[SPAI_CNT_RESID] = sums[6];
      counts[SPAI_CNT_ITERS] = total_iters;
    }
    return SPAI_OK;
  }

  UpdMode mode(int doM, int x1, int x2, int doP) const {
    UpdMode md{};
    md.doM = doM;
    md.x1 = x1;
    md.x2 = x2;
    md.doP = doP;
    md.pR = 1;
    md.pP = 1;
    md.sym = opts.symmetrize ? 1 : 0;
    md.colcap = colcap ? 1 : 0;
    md.u = opts.drop_tol;
    md.weighted = opts.jacobi ? 1 : 0;
    return md;
  }

  void resid_step(int setup) {
    tb(SPAI_PH_BOUNDS);
    launch_bound_resid<T>(A, M, ub, n, st, s);
    launch_scan(ub, off, total, n, scantmp, s);
    te();
    tb(SPAI_PH_RESID);
    if (implicit && opts.jacobi)         // R_0 itself, for the implicit updates
      launch_resid<T>(A, M, Rraw, off, total, colnorm, 0, colrz, big[0], st, tRs, tRl, tRh, s);
    launch_resid<T>(A, M, R, off, total, colnorm, opts.jacobi, colrz, big[0], st, tRs, tRl, tRh,
                    s);
    te();
    tb(SPAI_PH_SCALAR);
    launch_reduce(colnorm, 1, n, seg, nseg > 1 ? seg_beg : nullptr, red_rr, blockpart, s);
    if (opts.jacobi)
      launch_reduce(colrz, 1, n, seg, nseg > 1 ? seg_beg : nullptr, red_rz, blockpart, s);
    launch_scal_post(method, seg, red_rr, opts.jacobi ? red_rz : nullptr, tol, hist, hist_cap,
                     setup, st, s);
    te();
  }

  // R_{i+1} = R_i - c A X without dropping; X = the direction list R (xsrc 0) or P.now()
  void implicit_step(int xsrc, int cidx) {
    Cols<T> Rin = opts.jacobi ? Rraw : R;
    tb(SPAI_PH_BOUNDS);
    launch_bound_impl<T>(A, Rin, R, P, xsrc, ub, n, st, s);
    launch_scan(ub, off, total, n, scantmp, s);
    te();
    tb(SPAI_PH_RESID);
    launch_resid_impl<T>(A, Rin, R, P, xsrc, cidx, seg, off, total, Rn, Zn, opts.jacobi, colnorm,
                         colrz, big[0], st, tDs, tDl, tDh, s);
    if (opts.jacobi) {
      launch_copy_cols<T>(Rn, Rraw, n, total, st, s);
      launch_copy_cols<T>(Zn, R, n, total, st, s);
    } else {
      launch_copy_cols<T>(Rn, R, n, total, st, s);
    }
    te();
    tb(SPAI_PH_SCALAR);
    launch_reduce(colnorm, 1, n, seg, nseg > 1 ? seg_beg : nullptr, red_rr, blockpart, s);
    if (opts.jacobi)
      launch_reduce(colrz, 1, n, seg, nseg > 1 ? seg_beg : nullptr, red_rz, blockpart, s);
    launch_scal_post(method, seg, red_rr, opts.jacobi ? red_rz : nullptr, tol, hist, hist_cap, 0,
                     st, s);
    te();
  }

  void dots_step(int useR, int useP) {
    tb(SPAI_PH_DOTS);
    launch_dots<T>(A, R, P, useR, useP, opts.jacobi, colpart, big[1], st, tDs, tDl, tDh, s);
    te();
    tb(SPAI_PH_SCALAR);
    launch_reduce(colpart, kND, n, seg, nseg > 1 ? seg_beg : nullptr, red, blockpart, s);
    launch_scal_step(method, seg, red, st, s);
    te();
  }

  void update_step(UpdMode md) {
    tb(SPAI_PH_BOUNDS);
    launch_bound_update<T>(A, M, R, P, PT, md, ub, n, st, s);
    launch_scan(ub, off, total, n, scantmp, s);
    te();
    tb(SPAI_PH_UPDATE);
    launch_update<T>(A, M, R, P, PT, md, off, total, kcol, tM, tP, big[2], seg, st, tUs, tUl, tUh,
                     s);
    te();
    const double* keyM = (global && md.doM && score) ? sigma : nullptr;
    // speculative floors (global cap on magnitudes, one matrix): the update has written
    // only candidates above a fraction of the last cut; where the cut does not clear it,
    // the update and the selection run once more without floors (masked otherwise)
    const bool floors = global && nseg == 1 && !score && opts.floor_frac > 0.0;
    if (global) {
      tb(SPAI_PH_SELECT);
      if (keyM) launch_score<T>(A, M, score, sigma, big[2], st, tSs, tSl, tSh, n, s);
      if (md.doM)
        launch_global_select<T>(M, 1, m_global, opts.tie_eta, 0, selhist, selbuf, n, st, s, keyM);
      if (md.doP) launch_global_select<T>(P, 0, m_global, opts.tie_eta, 1, selhist, selbuf, n, st, s);
      if (floors) {
        launch_redo_begin(st, s);
        launch_update<T>(A, M, R, P, PT, md, off, total, kcol, tM, tP, big[2], seg, st, tUs, tUl,
                         tUh, s, true);
        if (md.doM)
          launch_global_select<T>(M, 1, m_global, opts.tie_eta, 0, selhist, selbuf, n, st, s);
        if (md.doP)
          launch_global_select<T>(P, 0, m_global, opts.tie_eta, 1, selhist, selbuf, n, st, s);
        launch_redo_end(st, s);
      }
      te();
    }
    tb(SPAI_PH_COMPACT);
    if (md.doM) launch_compact<T>(M, 0, colcap, md.sym, global, tM, opts.tie_eta, n, st, s, keyM);
    if (md.doP) {
      launch_compact<T>(P, 1, colcap, 0, global, tP, opts.tie_eta, n, st, s);
      launch_compact<T>(PT, 2, colcap, 0, global, tP, opts.tie_eta, n, st, s);
    }
    // each compaction reads only its own pair, so both flips (and the floors) go last
    launch_drop_finish(st, md.doM, md.doP, floors ? 1 : 0, opts.floor_frac, s);
    te();
  }

  void p_update_step() { update_step(mode(0, 0, 0, 1)); }

  // one iteration of the handle's method, entirely on the device
  void enqueue_iteration() {
    if (method == SPAI_MR) {
      dots_step(1, 0);
      update_step(mode(1, 1, 0, 0));
      if (implicit) implicit_step(0, 0);     // R - alpha A R
      else resid_step(0);
    } else if (method == SPAI_CG) {
      dots_step(0, 1);
      update_step(mode(1, 2, 0, 0));
      if (implicit) implicit_step(1, 0);     // R - alpha A P
      else resid_step(0);
      p_update_step();
    } else {
      dots_step(1, 1);
      update_step(mode(1, 1, 2, 1));
      if (implicit) implicit_step(1, -1);    // R - A P_i, P_i = delta R + gamma P_{i-1}
      else resid_step(0);
    }
  }

  int check_err() {
    DevState h;
    HIPCHK(hipMemcpy(&h, st, sizeof(DevState), hipMemcpyDeviceToHost));
    if (h.err & 1) return fail(SPAI_ERR_CAPACITY, "a column exceeded the largest per-column tile");
    if (h.err & 2) return fail(SPAI_ERR_NOMEM, "an iterate exceeded its device pool");
    if (h.err & 4) return fail(SPAI_ERR_HIP, "internal: candidate pattern not symmetric");
    return SPAI_OK;
  }

  int read_segs(std::vector<SegState>& v) {
    v.resize(nseg);
    HIPCHK(hipMemcpy(v.data(), segst, sizeof(SegState) * nseg, hipMemcpyDeviceToHost));
    return SPAI_OK;
  }

  int iterate(int k, int* done, double* hout) override {
    if (k < 0) return fail(SPAI_ERR_ARG, "negative iteration count");
    if (iters_host + k > max_iter) return fail(SPAI_ERR_ARG, "iterations beyond max_iter");
    int rc;
    std::vector<SegState> before;
    if ((rc = read_segs(before))) return rc;
    if (batched_graph && k > 0) {
      if (!graph_exec) {
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        enqueue_iteration();
        HIPCHK(hipStreamEndCapture(s, &graph));
        HIPCHK(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
      }
      for (int t = 0; t < k; ++t) HIPCHK(hipGraphLaunch(graph_exec, s));
    } else {
      for (int t = 0; t < k; ++t) enqueue_iteration();
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    collect();
    if ((rc = check_err())) return rc;
    std::vector<SegState> after;
    if ((rc = read_segs(after))) return rc;
    const int d0 = after[0].iters - before[0].iters;
    iters_host += k;
    total_iters += d0;
    if (done) *done = d0;
    if (hout && d0 > 0)
      HIPCHK(hipMemcpy(hout, hist + before[0].iters, sizeof(double) * d0, hipMemcpyDeviceToHost));
    if (nseg == 1) {
      if (after[0].status == 3) return SPAI_BREAKDOWN;
      if (after[0].status == 1) return SPAI_CONVERGED;
      return SPAI_OK;
    }
    bool all_conv = true, any_break = false;
    for (auto& g : after) {
      all_conv = all_conv && g.status == 1;
      any_break = any_break || g.status == 3;
    }
    if (any_break) return SPAI_BREAKDOWN;
    if (all_conv) return SPAI_CONVERGED;
    return SPAI_OK;
  }

  int get(spai_csr_out_t* out) override {
    if (!out) return fail(SPAI_ERR_ARG, "null output");
    HIPCHK(hipStreamSynchronize(s));
    DevState h;
    HIPCHK(hipMemcpy(&h, st, sizeof(DevState), hipMemcpyDeviceToHost));
    const Cols<T>& C = M.b[h.curM];
    std::vector<int32_t> len(n);
    HIPCHK(hipMemcpy(len.data(), C.len, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    int64_t nnz = 0;
    for (int64_t j = 0; j < n; ++j) nnz += len[j];
    out->n = n;
    out->nnz = nnz;
    if (!out->rowptr) return SPAI_OK;
    if (out->capacity < nnz) return fail(SPAI_ERR_ARG, "output capacity below nnz(M)");
    // gather the columns (CSC, packed on the device), then transpose to CSR on the host
    std::vector<int64_t> cpk;
    std::vector<int32_t> ci;
    std::vector<T> cv;
    int rcp;
    if ((rcp = download_cols<T>(C, n, s, cpk, ci, cv))) return rcp;
    int64_t o = 0;
    std::vector<int64_t> rp(n + 1, 0);
    for (int64_t q = 0; q < nnz; ++q) rp[ci[q] + 1]++;
    for (int64_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
    std::vector<int64_t> cur(rp.begin(), rp.end() - 1);
    std::vector<int32_t> rc_col(nnz);
    std::vector<double> rc_val(nnz);
    o = 0;
    for (int64_t j = 0; j < n; ++j)
      for (int e = 0; e < len[j]; ++e, ++o) {
        const int64_t p = cur[ci[o]]++;
        rc_col[p] = (int32_t)j;
        rc_val[p] = (double)cv[o];
      }
    if (out->on_device) {
      HIPCHK(hipMemcpy(out->rowptr, rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
      if (nnz) {
        HIPCHK(hipMemcpy(out->colind, rc_col.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(out->val, rc_val.data(), sizeof(double) * nnz, hipMemcpyHostToDevice));
      }
    } else {
      std::memcpy(out->rowptr, rp.data(), sizeof(int64_t) * (n + 1));
      if (nnz) {
        std::memcpy(out->colind, rc_col.data(), sizeof(int32_t) * nnz);
        std::memcpy(out->val, rc_val.data(), sizeof(double) * nnz);
      }
    }
    return SPAI_OK;
  }

  int stats(int* iters, double* resid, int64_t* nnz_m, int64_t* nnz_p, double* s1, double* s2,
            int* fb) override {
    HIPCHK(hipStreamSynchronize(s));
    std::vector<SegState> g;
    int rc;
    if ((rc = read_segs(g))) return rc;
    DevState h;
    HIPCHK(hipMemcpy(&h, st, sizeof(DevState), hipMemcpyDeviceToHost));
    if (iters) *iters = g[0].iters;
    if (resid) *resid = std::sqrt(g[0].rr);
    if (s1) *s1 = g[0].step1;
    if (s2) *s2 = g[0].step2;
    if (fb) *fb = g[0].mr_fallbacks;
    if (nnz_m || nnz_p) {
      auto count = [&](const Cols<T>& C, int64_t* out) -> int {
        std::vector<int32_t> len(n);
        HIPCHK(hipMemcpy(len.data(), C.len, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
        int64_t t = 0;
        for (auto v : len) t += v;
        *out = t;
        return SPAI_OK;
      };
      if (nnz_m && (rc = count(M.b[h.curM], nnz_m))) return rc;
      if (nnz_p) {
        if (method == SPAI_MR) *nnz_p = 0;
        else if ((rc = count(P.b[h.curP], nnz_p))) return rc;
      }
    }
    return SPAI_OK;
  }

  int batched_resid(double* out) override {
    if (!out) return fail(SPAI_ERR_ARG, "null output");
    HIPCHK(hipStreamSynchronize(s));
    std::vector<SegState> g;
    int rc;
    if ((rc = read_segs(g))) return rc;
    for (int i = 0; i < nseg; ++i) out[i] = std::sqrt(g[i].rr);
    return SPAI_OK;
  }
};

}  // namespace

struct spai_handle {
  std::unique_ptr<EngineBase> eng;
};

static void fill_defaults(spai_opts_t* o) {
  o->precision = SPAI_PREC_F64;
  o->symmetrize = 1;
  o->drop_tol = std::ldexp(1.0, -53);
  o->tie_eta = 1e-9;
  o->stream = nullptr;
  o->device_pool_limit = 0;
  o->profile = 0;
  o->a_format = SPAI_AFMT_AUTO;
  o->jacobi = 0;
  o->explicit_residual = 1;
  o->drop_score = 0;
  o->floor_frac = 0.75;
}

template <typename T>
static int make_engine(HostCsr&& hA, const std::vector<int64_t>& segs, int method, spai_cap_t cap,
                       int max_iter, double tol, const spai_opts_t& o, bool graph,
                       spai_handle_t** out) {
  auto e = std::make_unique<Engine<T>>();
  e->method = method;
  e->n = hA.n;
  e->cap = cap;
  e->opts = o;
  e->tol = tol;
  e->max_iter = max_iter;
  e->hA = std::move(hA);
  e->batched_graph = graph;
  int rc = e->setup(segs);
  if (rc) return rc;
  auto* h = new (std::nothrow) spai_handle;
  if (!h) return fail(SPAI_ERR_NOMEM, "host allocation failed");
  h->eng = std::move(e);
  *out = h;
  return SPAI_OK;
}

static int check_common(int method, spai_cap_t cap, int max_iter, double tol,
                        const spai_opts_t* opts, spai_opts_t& o) {
  if (method != SPAI_MR && method != SPAI_CG && method != SPAI_LOMR)
    return fail(SPAI_ERR_ARG, "unknown method");
  if (max_iter < 0 || !(tol >= 0.0)) return fail(SPAI_ERR_ARG, "bad max_iter or tol");
  if (cap.mode != SPAI_CAP_NONE && !(cap.value > 0.0)) return fail(SPAI_ERR_ARG, "cap value <= 0");
  fill_defaults(&o);
  if (opts) o = *opts;
  if (o.precision != SPAI_PREC_F64 && o.precision != SPAI_PREC_MIXED)
    return fail(SPAI_ERR_ARG, "unknown precision");
  if (!(o.drop_tol >= 0.0) || !(o.tie_eta >= 0.0)) return fail(SPAI_ERR_ARG, "bad drop_tol / tie_eta");
  if (!(o.floor_frac >= 0.0) || !std::isfinite(o.floor_frac))
    return fail(SPAI_ERR_ARG, "floor_frac must be finite and >= 0");
  if (o.jacobi != 0 && o.jacobi != 1) return fail(SPAI_ERR_ARG, "jacobi must be 0 or 1");
  if (o.explicit_residual != 0 && o.explicit_residual != 1)
    return fail(SPAI_ERR_ARG, "explicit_residual must be 0 or 1");
  if (!o.explicit_residual &&
      (cap.mode != SPAI_CAP_NONE || o.drop_tol != 0.0 || o.symmetrize))
    return fail(SPAI_ERR_ARG,
                "the implicit residual needs no dropping: no cap, drop_tol 0, symmetrize 0");
  if (o.a_format != SPAI_AFMT_AUTO && o.a_format != SPAI_AFMT_CSR && o.a_format != SPAI_AFMT_ELL)
    return fail(SPAI_ERR_ARG, "unknown a_format");
  if (o.drop_score != 0 && o.drop_score != 1) return fail(SPAI_ERR_ARG, "drop_score must be 0 or 1");
  if (o.drop_score && (cap.mode != SPAI_CAP_GLOBAL || !o.symmetrize))
    return fail(SPAI_ERR_ARG, "the heuristic drop score needs a global cap and symmetrize = 1");
  return SPAI_OK;
}

extern "C" {

void spai_default_opts(spai_opts_t* opts) {
  if (opts) fill_defaults(opts);
}

int spai_create(const spai_csr_t* A, int method, spai_cap_t cap, int max_iter, double tol,
                const spai_opts_t* opts, spai_handle_t** out) {
  try {
    if (!out) return fail(SPAI_ERR_ARG, "null handle pointer");
    *out = nullptr;
    spai_opts_t o;
    int rc = check_common(method, cap, max_iter, tol, opts, o);
    if (rc) return rc;
    HostCsr hA;
    if ((rc = fetch_csr(A, hA))) return rc;
    if ((rc = check_spd_symmetric(hA))) return rc;
    std::vector<int64_t> segs{0, hA.n};
    if (o.precision == SPAI_PREC_MIXED)
      return make_engine<float>(std::move(hA), segs, method, cap, max_iter, tol, o, false, out);
    return make_engine<double>(std::move(hA), segs, method, cap, max_iter, tol, o, false, out);
  } catch (const std::bad_alloc&) {
    return fail(SPAI_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_create_batched(const spai_csr_t* As, int nb, int method, spai_cap_t cap, int max_iter,
                        double tol, const spai_opts_t* opts, spai_handle_t** out) {
  try {
    if (!out || !As || nb < 1) return fail(SPAI_ERR_ARG, "bad batch arguments");
    *out = nullptr;
    spai_opts_t o;
    int rc = check_common(method, cap, max_iter, tol, opts, o);
    if (rc) return rc;
    if (cap.mode == SPAI_CAP_GLOBAL) return fail(SPAI_ERR_ARG, "batched handles take column caps only");
    if (!o.explicit_residual) return fail(SPAI_ERR_ARG, "batched handles use the explicit residual");
    // block-diagonal assembly
    HostCsr big;
    big.n = 0;
    big.nnz = 0;
    std::vector<int64_t> segs{0};
    big.rowptr.push_back(0);
    for (int b = 0; b < nb; ++b) {
      HostCsr h;
      if ((rc = fetch_csr(&As[b], h))) return rc;
      if ((rc = check_spd_symmetric(h))) return rc;
      const int64_t base = big.n;
      for (int64_t i = 0; i < h.n; ++i) big.rowptr.push_back(big.nnz + h.rowptr[i + 1]);
      for (int64_t q = 0; q < h.nnz; ++q) {
        big.col.push_back((int32_t)(h.col[q] + base));
        big.val.push_back(h.val[q]);
      }
      big.n += h.n;
      big.nnz += h.nnz;
      segs.push_back(big.n);
      if (big.n > INT32_MAX - 1) return fail(SPAI_ERR_ARG, "batch exceeds the int32 index range");
    }
    if (o.precision == SPAI_PREC_MIXED)
      return make_engine<float>(std::move(big), segs, method, cap, max_iter, tol, o, true, out);
    return make_engine<double>(std::move(big), segs, method, cap, max_iter, tol, o, true, out);
  } catch (const std::bad_alloc&) {
    return fail(SPAI_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_iterate(spai_handle_t* h, int n_iter, int* iters_done, double* resid_hist) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->iterate(n_iter, iters_done, resid_hist);
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_get(spai_handle_t* h, spai_csr_out_t* M) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->get(M);
  } catch (const std::bad_alloc&) {
    return fail(SPAI_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_stats(spai_handle_t* h, int* iters, double* resid_fro, int64_t* nnz_m, int64_t* nnz_p,
               double* step1, double* step2, int* mr_fallbacks) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->stats(iters, resid_fro, nnz_m, nnz_p, step1, step2, mr_fallbacks);
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_batched_resid(spai_handle_t* h, double* resid) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->batched_resid(resid);
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_destroy(spai_handle_t* h) {
  delete h;
  return SPAI_OK;
}

int spai_reset(spai_handle_t* h) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->reset();
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_pcg(spai_handle_t* h, int nrhs, const double* B, double* X, double rtol, int max_iter,
             int* iters, double* relres, int on_device) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->pcg(nrhs, B, X, rtol, max_iter, iters, relres, on_device);
  } catch (const std::bad_alloc&) {
    return fail(SPAI_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_spectrum(spai_handle_t* h, int steps, const double* v0, int on_device, double* out,
                  int* steps_done) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->spectrum(steps, v0, on_device, out, steps_done);
  } catch (const std::bad_alloc&) {
    return fail(SPAI_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_get_state(spai_handle_t* h, void* buf, size_t* size) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->get_state(buf, size);
  } catch (const std::bad_alloc&) {
    return fail(SPAI_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_set_state(spai_handle_t* h, const void* buf, size_t size) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->set_state(buf, size);
  } catch (const std::bad_alloc&) {
    return fail(SPAI_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_history(spai_handle_t* h, int64_t* rec, int cap, int* count) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->history(rec, cap, count);
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_set_tiles(spai_handle_t* h, const int* tiles) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->set_tiles(tiles);
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_autotune(spai_handle_t* h, int warm_iters, int reps, int* chosen, double* best_ms) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->autotune(warm_iters, reps, chosen, best_ms);
  } catch (const std::bad_alloc&) {
    return fail(SPAI_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

int spai_profile(spai_handle_t* h, double* phase_ms, int64_t* phase_calls, int64_t* counts) {
  if (!h) return fail(SPAI_ERR_ARG, "null handle");
  try {
    return h->eng->profile(phase_ms, phase_calls, counts);
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}

const char* spai_last_error(void) { return g_last_error.c_str(); }

const char* spai_status_string(int status) {
  switch (status) {
    case SPAI_OK: return "SPAI_OK";
    case SPAI_CONVERGED: return "SPAI_CONVERGED";
    case SPAI_MAXITER: return "SPAI_MAXITER";
    case SPAI_BREAKDOWN: return "SPAI_BREAKDOWN";
    case PCG_INDEFINITE: return "PCG_INDEFINITE";
    case SPAI_ERR_ARG: return "SPAI_ERR_ARG";
    case SPAI_ERR_NOT_SYMMETRIC: return "SPAI_ERR_NOT_SYMMETRIC";
    case SPAI_ERR_NOT_SPD: return "SPAI_ERR_NOT_SPD";
    case SPAI_ERR_NONFINITE: return "SPAI_ERR_NONFINITE";
    case SPAI_ERR_NOMEM: return "SPAI_ERR_NOMEM";
    case SPAI_ERR_HIP: return "SPAI_ERR_HIP";
    case SPAI_ERR_CAPACITY: return "SPAI_ERR_CAPACITY";
    default: return "SPAI_UNKNOWN";
  }
}

}  // extern "C"
