// spai_spectrum.hip — extreme eigenvalues of a symmetric sparse matrix (the lambda_min /
// lambda_max columns the paper reports for its approximate inverses, Tables 4-6, and
// whether an iterate is positive definite, Section 7.1).
//
// Lanczos process with full reorthogonalisation (Lanczos 1950; Paige 1972; Golub and
// Van Loan, Matrix Computations, Section 10.1): v_0 = v0 / ||v0||, and per step
//   w = S v_j;  h = V_j^T w, w -= V_j h;  h' = V_j^T w, w -= V_j h'  (Gram-Schmidt twice)
//   alpha_j = h_j + h'_j,  beta_j = ||w||,  v_{j+1} = w / beta_j,
// stopping early once beta_j <= 1e-12 max_{i<=j} (|alpha_i| + beta_i) (an invariant
// subspace).  The Ritz values are the eigenvalues of the tridiagonal T_k =
// tridiag(beta, alpha, beta); its extreme ones are found by bisection on Sturm counts,
// and beta_k |y_k| (y the unit eigenvector of T_k, by inverse iteration) bounds the
// distance from each to an eigenvalue of S.  Ritz values are Rayleigh quotients, so
// lambda_min(S) <= theta_min and theta_max <= lambda_max(S).
//
// Device work: one thread per row for S v (ascending stored order), the basis products
// as fixed row chunks summed in a fixed order (deterministic), the basis kept as n x
// (steps + 1) doubles.  The host reads three scalars per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "spai.h"
#include "spai_host.hpp"

namespace spai {

namespace {

constexpr int kThreads = 256;
constexpr int kChunks = 512;        // row chunks of the partial basis products
constexpr int kMaxSteps = 2048;

__global__ void k_lz_spmv(PcgMat S, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  double acc = 0.0;
  const int64_t e = S.row_end(i);
  for (int64_t q = S.row_begin(i); q < e; ++q) {
    const int c = S.col[q];
    if (c >= 0) acc += S.v(q) * x[c];
  }
  y[i] = acc;
}

// part[t * kChunks + c] = sum over the rows of chunk c of V[i, t] w[i]
__global__ __launch_bounds__(kThreads) void k_lz_dots(const double* __restrict__ V, int64_t ldv,
                                                      int64_t n, const double* __restrict__ w,
                                                      double* __restrict__ part) {
  __shared__ double sh[kThreads];
  const int c = blockIdx.x, t = blockIdx.y;
  const int64_t per = (n + kChunks - 1) / kChunks;
  const int64_t lo = (int64_t)c * per, hi = std::min<int64_t>(n, lo + per);
  const double* v = V + (int64_t)t * ldv;
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) acc += v[i] * w[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int d = kThreads / 2; d >= 1; d >>= 1) {
    if ((int)threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)t * kChunks + c] = sh[0];
}

// h[t] = sum_c part[t * kChunks + c], c ascending
__global__ void k_lz_sum(const double* __restrict__ part, int k, double* __restrict__ h) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k) return;
  double acc = 0.0;
  for (int c = 0; c < kChunks; ++c) acc += part[(int64_t)t * kChunks + c];
  h[t] = acc;
}

// w[i] -= sum_{t<k} V[i, t] h[t]
__global__ void k_lz_sub(const double* __restrict__ V, int64_t ldv, int k, int64_t n,
                         const double* __restrict__ h, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int t = 0; t < k; ++t) acc += V[i + (int64_t)t * ldv] * h[t];
  w[i] -= acc;
}

__global__ void k_lz_div(const double* __restrict__ w, double b, int64_t n,
                         double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = w[i] / b;
}

// ---- host: the tridiagonal T_k

// number of eigenvalues of T below x (signs of the LDL^T pivots of T - x I)
int sturm_below(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double d = 1.0;
  const double tiny = 1e-300;
  for (size_t i = 0; i < a.size(); ++i) {
    d = (a[i] - x) - (i ? (b[i - 1] * b[i - 1]) / d : 0.0);
    if (d == 0.0) d = -tiny;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

// the r-th smallest eigenvalue of T (r = 1..k) by bisection inside the Gershgorin interval
double tri_eig(const std::vector<double>& a, const std::vector<double>& b, int r) {
  const size_t k = a.size();
  double lo = a[0], hi = a[0];
  for (size_t i = 0; i < k; ++i) {
    const double rad = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - rad);
    hi = std::max(hi, a[i] + rad);
  }
  for (int it = 0; it < 400; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_below(a, b, mid) >= r) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// last component of the unit eigenvector of T for the eigenvalue theta (inverse iteration
// with a tridiagonal LU with partial pivoting)
double tri_last_component(const std::vector<double>& a, const std::vector<double>& b,
                          double theta, double scale) {
  const size_t k = a.size();
  if (k == 1) return 1.0;
  const double shift = theta + 1e-14 * scale;
  std::vector<double> y(k, 1.0), dl(k), d(k), du(k), du2(k), rhs(k);
  std::vector<char> swapped(k, 0);
  for (int pass = 0; pass < 3; ++pass) {
    for (size_t i = 0; i < k; ++i) {
      d[i] = a[i] - shift;
      du[i] = i + 1 < k ? b[i] : 0.0;
      dl[i] = i + 1 < k ? b[i] : 0.0;   // subdiagonal entry below row i
      du2[i] = 0.0;
      swapped[i] = 0;
      rhs[i] = y[i];
    }
    // elimination down the rows
    for (size_t i = 0; i + 1 < k; ++i) {
      if (std::fabs(d[i]) >= std::fabs(dl[i])) {
        const double piv = d[i] != 0.0 ? d[i] : 1e-300;
        const double m = dl[i] / piv;
        d[i] = piv;
        d[i + 1] -= m * du[i];
        rhs[i + 1] -= m * rhs[i];
        dl[i] = m;
      } else {                          // swap rows i and i + 1
        const double m = d[i] / dl[i];
        d[i] = dl[i];
        const double t = d[i + 1];
        d[i + 1] = du[i] - m * t;
        du2[i] = i + 2 < k ? du[i + 1] : 0.0;
        if (i + 2 < k) du[i + 1] = -m * du2[i];
        du[i] = t;
        std::swap(rhs[i], rhs[i + 1]);
        rhs[i + 1] -= m * rhs[i];
        dl[i] = m;
        swapped[i] = 1;
      }
    }
    if (d[k - 1] == 0.0) d[k - 1] = 1e-300;
    // back substitution
    y[k - 1] = rhs[k - 1] / d[k - 1];
    if (k >= 2) y[k - 2] = (rhs[k - 2] - du[k - 2] * y[k - 1]) / d[k - 2];
    for (size_t ii = k - 2; ii-- > 0;) y[ii] = (rhs[ii] - du[ii] * y[ii + 1] - du2[ii] * y[ii + 2]) / d[ii];
    double nrm = 0.0;
    for (double v : y) nrm = std::max(nrm, std::fabs(v));
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return 1.0;
    for (double& v : y) v /= nrm;
  }
  double s2 = 0.0;
  for (double v : y) s2 += v * v;
  return y[k - 1] / std::sqrt(s2);
}

}  // namespace

int lanczos_run(const PcgMat& S, int steps, const double* dv0, double* out, int* steps_done,
                int64_t pool_limit, hipStream_t s) {
  const int64_t n = S.n;
  if (steps < 1 || steps > kMaxSteps) return fail(SPAI_ERR_ARG, "spectrum: steps outside 1..2048");
  if (!out) return fail(SPAI_ERR_ARG, "spectrum: null output");
  const int K = (int)std::min<int64_t>(steps, n);
  const int64_t ldv = n;
  DevPool pool;
  pool.limit = pool_limit;
  int rc;
  double *V, *w, *part, *h1, *h2, *nb;
  if ((rc = pool.alloc(&V, n * (int64_t)(K + 1))) || (rc = pool.alloc(&w, n)) ||
      (rc = pool.alloc(&part, (int64_t)kChunks * (K + 1))) || (rc = pool.alloc(&h1, K + 1)) ||
      (rc = pool.alloc(&h2, K + 1)) || (rc = pool.alloc(&nb, 1)))
    return rc;
  const dim3 rows((unsigned)((n + kThreads - 1) / kThreads)), bs(kThreads);
  auto dots = [&](const double* Vb, int k, const double* x, double* h) {
    hipLaunchKernelGGL(k_lz_dots, dim3(kChunks, k), bs, 0, s, Vb, ldv, n, x, part);
    hipLaunchKernelGGL(k_lz_sum, dim3((k + kThreads - 1) / kThreads), bs, 0, s, part, k, h);
  };
  // v_0 = v0 / ||v0||
  double nrm2 = 0.0;
  dots(dv0, 1, dv0, nb);
  HIPCHK(hipMemcpyAsync(&nrm2, nb, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (!(nrm2 > 0.0) || !std::isfinite(nrm2))
    return fail(SPAI_ERR_ARG, "spectrum: start vector zero or not finite");
  hipLaunchKernelGGL(k_lz_div, rows, bs, 0, s, dv0, std::sqrt(nrm2), n, V);
  std::vector<double> alpha, beta;
  double scale = 0.0;
  int done = 0;
  for (int j = 0; j < K; ++j) {
    const double* vj = V + (int64_t)j * ldv;
    hipLaunchKernelGGL(k_lz_spmv, rows, bs, 0, s, S, vj, w);
    dots(V, j + 1, w, h1);
    hipLaunchKernelGGL(k_lz_sub, rows, bs, 0, s, V, ldv, j + 1, n, h1, w);
    dots(V, j + 1, w, h2);
    hipLaunchKernelGGL(k_lz_sub, rows, bs, 0, s, V, ldv, j + 1, n, h2, w);
    dots(w, 1, w, nb);
    HIPCHK(hipGetLastError());
    double hj[3];
    HIPCHK(hipMemcpyAsync(&hj[0], h1 + j, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hj[1], h2 + j, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hj[2], nb, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double a = hj[0] + hj[1];
    const double b = std::sqrt(std::max(hj[2], 0.0));
    if (!std::isfinite(a) || !std::isfinite(b)) return fail(SPAI_ERR_NONFINITE, "spectrum: non-finite step");
    alpha.push_back(a);
    beta.push_back(b);
    scale = std::max(scale, std::fabs(a) + b);
    done = j + 1;
    if (b <= 1e-12 * scale) break;     // invariant subspace: T_k's eigenvalues are exact
    if (j + 1 < K)
      hipLaunchKernelGGL(k_lz_div, rows, bs, 0, s, w, b, n, V + (int64_t)(j + 1) * ldv);
  }
  HIPCHK(hipStreamSynchronize(s));
  const int k = done;
  std::vector<double> a(alpha.begin(), alpha.begin() + k), b(beta.begin(), beta.begin() + k);
  const double bl = b[k - 1];
  b.resize(k - 1 > 0 ? k - 1 : 0);
  const double tmin = tri_eig(a, b, 1), tmax = tri_eig(a, b, k);
  out[0] = tmin;
  out[1] = tmax;
  out[2] = bl * std::fabs(tri_last_component(a, b, tmin, scale));
  out[3] = bl * std::fabs(tri_last_component(a, b, tmax, scale));
  if (steps_done) *steps_done = k;
  return SPAI_OK;
}

}  // namespace spai

using namespace spai;

extern "C" int spai_csr_spectrum(const spai_csr_t* S, int steps, const double* v0, double* out,
                                 int* steps_done, const spai_opts_t* opts) {
  try {
    if (!S || !v0 || !out) return fail(SPAI_ERR_ARG, "spai_csr_spectrum: null argument");
    int rc;
    HostCsr h;
    if ((rc = fetch_csr(S, h))) return rc;
    for (int64_t i = 0; i < h.n; ++i)
      for (int64_t q = h.rowptr[i]; q < h.rowptr[i + 1]; ++q) {
        const int64_t t = find_entry(h, h.col[q], (int32_t)i);
        if (t < 0 || h.val[t] != h.val[q])
          return fail(SPAI_ERR_NOT_SYMMETRIC, "spai_csr_spectrum: matrix not symmetric");
      }
    spai_opts_t o;
    spai_default_opts(&o);
    if (opts) o = *opts;
    hipStream_t s = (hipStream_t)o.stream;
    DevPool pool;
    pool.limit = o.device_pool_limit;
    int64_t* rp;
    int32_t* ci;
    double* va;
    double* dv0;
    if ((rc = pool.alloc(&rp, h.n + 1)) || (rc = pool.alloc(&ci, h.nnz)) ||
        (rc = pool.alloc(&va, h.nnz)) || (rc = pool.alloc(&dv0, h.n)))
      return rc;
    HIPCHK(hipMemcpyAsync(rp, h.rowptr.data(), sizeof(int64_t) * (h.n + 1), hipMemcpyHostToDevice, s));
    if (h.nnz) {
      HIPCHK(hipMemcpyAsync(ci, h.col.data(), sizeof(int32_t) * h.nnz, hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(va, h.val.data(), sizeof(double) * h.nnz, hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipMemcpyAsync(dv0, v0, sizeof(double) * h.n,
                          S->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    PcgMat m;
    m.n = h.n;
    m.rowptr = rp;
    m.col = ci;
    m.val = va;
    const int64_t rest = o.device_pool_limit > 0
                             ? std::max<int64_t>(1, o.device_pool_limit - (int64_t)pool.used)
                             : 0;
    return lanczos_run(m, steps, dv0, out, steps_done, rest, s);
  } catch (const std::bad_alloc&) {
    return fail(SPAI_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SPAI_ERR_HIP, "unexpected exception");
  }
}
