// spai_pcg.hip — preconditioned CG with the SPAI as preconditioner (z = M r), many
// right-hand sides at once (the vector solves of Section 7, Experiments 04 and 06).
//
// Every right-hand side runs its own textbook recurrence in float64; the block of
// vectors is row-major (n x nrhs, the nrhs values of a row contiguous), so one
// wavefront reads the 64 values of a row of X as one coalesced 512-byte line and the
// SpMM gathers whole rows.  Frobenius-free per-RHS dots are reduced per workgroup in
// a fixed order and then across workgroups in a fixed order (deterministic).
#include <hip/hip_runtime.h>

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

constexpr int kThreads = 256;
constexpr int kGrid = 2048;

using Mat = PcgMat;

// Y[:, c0:c0+R) = A X[:, c0:c0+R) and per-block partials of sum_i W[i, r] Y[i, r].
// Threads are (row, rhs) pairs: R = pow2 >= the chunk width, 256 / R rows per block step.
__global__ __launch_bounds__(kThreads) void k_spmm_dot(Mat A, const double* X, double* Y,
                                                       const double* W, int nrhs, int c0, int cw,
                                                       int R, double* part) {
  __shared__ double sh[kThreads];
  const int t = threadIdx.x;
  const int r = t % R;
  const int rows_per = kThreads / R;
  const int roff = t / R;
  double acc = 0.0;
  const bool on = r < cw;
  for (int64_t base = (int64_t)blockIdx.x * rows_per; base < A.n; base += (int64_t)gridDim.x * rows_per) {
    const int64_t i = base + roff;
    if (i < A.n && on) {
      double y = 0.0;
      const int64_t q0 = A.row_begin(i), q1 = A.row_end(i);
      constexpr int U = 8;
      for (int64_t qb = q0; qb < q1; qb += U) {      // 8 gathers in flight, summed in order
        int cols[U];
        double vals[U], xs[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
          if (qb + k < q1) {
            cols[k] = A.col[qb + k];
            vals[k] = A.v(qb + k);
          }
#pragma unroll
        for (int k = 0; k < U; ++k)
          if (qb + k < q1) xs[k] = X[(int64_t)cols[k] * nrhs + c0 + r];
#pragma unroll
        for (int k = 0; k < U; ++k)
          if (qb + k < q1) y += vals[k] * xs[k];
      }
      Y[i * nrhs + c0 + r] = y;
      if (W) acc += W[i * nrhs + c0 + r] * y;
    }
  }
  if (!part) return;
  sh[t] = acc;
  __syncthreads();
  if (t < cw) {
    double s = 0.0;
    for (int k = t; k < kThreads; k += R) s += sh[k];
    part[(int64_t)blockIdx.x * nrhs + c0 + t] = s;
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
__global__ __launch_bounds__(kThreads) void k_reduce_parts(const double* part, int nblocks,
                                                           int nrhs, double* out) {
  __shared__ double sh[kThreads];
  const int r = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kThreads) s += part[(int64_t)b * nrhs + r];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = sh[0];
}

struct RhsState {
  double bnorm, rz, pq, rr, alpha, beta;
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
__global__ void k_alpha(RhsState* S, const double* pq, int nrhs, int* nactive) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  RhsState& g = S[r];
  g.alpha = 0.0;
  if (!g.active) return;
  g.pq = pq[r];
  if (!(g.rz > 0.0) || !(g.pq > 0.0)) {
    g.active = 0;
    g.status = 4;
    atomicSub(nactive, 1);
    return;
  }
  g.alpha = g.rz / g.pq;
  g.iters += 1;
}

// x += alpha p, r -= alpha q (inactive right-hand sides have alpha = 0)
// x += alpha p, r -= alpha q (inactive right-hand sides have alpha = 0), fused with the
// per-block partials of ||r||^2 for every right-hand side
__global__ __launch_bounds__(kThreads) void k_axpy(double* x, double* rv, const double* p,
                                                   const double* q, const RhsState* S, int64_t n,
                                                   int nrhs, int R, double* part) {
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
          x[o] = x[o] + a * p[o];
          rr = rr - a * q[o];
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

__global__ void k_conv(RhsState* S, const double* rr, double rtol, int nrhs, int* nactive) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  RhsState& g = S[r];
  if (!g.active) return;
  g.rr = rr[r];
  if (sqrt(g.rr) <= rtol * g.bnorm) {
    g.active = 0;
    g.status = 1;
    atomicSub(nactive, 1);
  }
}

__global__ void k_beta(RhsState* S, const double* rz_new, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  RhsState& g = S[r];
  g.beta = 0.0;
  if (!g.active) return;
  g.beta = rz_new[r] / g.rz;
  g.rz = rz_new[r];
}

// p = z + beta p for running right-hand sides
__global__ __launch_bounds__(kThreads) void k_pupd(double* p, const double* z, const RhsState* S,
                                                   int64_t n, int nrhs, int R) {
  const int t = threadIdx.x;
  const int r = t % R;
  const int rows_per = kThreads / R;
  const int roff = t / R;
  if (r >= nrhs || !S[r].active) return;
  const double b = S[r].beta;
  for (int64_t base = (int64_t)blockIdx.x * rows_per; base < n; base += (int64_t)gridDim.x * rows_per) {
    const int64_t i = base + roff;
    if (i < n) {
      const int64_t o = i * nrhs + r;
      p[o] = z[o] + b * p[o];
    }
  }
}

// the same updates for more than 64 right-hand sides (flat indexing)
__global__ __launch_bounds__(kThreads) void k_axpy_wide(double* x, double* rv, const double* p,
                                                        const double* q, const RhsState* S,
                                                        int64_t n, int nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < tot; o += (int64_t)gridDim.x * kThreads) {
    const double a = S[o % nrhs].alpha;
    if (a != 0.0) {
      x[o] = x[o] + a * p[o];
      rv[o] = rv[o] - a * q[o];
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_pupd_wide(double* p, const double* z,
                                                        const RhsState* S, int64_t n, int nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < tot; o += (int64_t)gridDim.x * kThreads) {
    const int r = (int)(o % nrhs);
    if (S[r].active) p[o] = z[o] + S[r].beta * p[o];
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
  int64_t n;
  int nrhs;
  hipStream_t s;
  double *x, *r, *z, *p, *q, *part, *tmp;
  const double* b;
  RhsState* S;
  int* nactive;

  static int pow2(int w) {
    int R = 1;
    while (R < w) R <<= 1;
    return R;
  }

  // Y = Mat X with optional per-RHS dot (W, Y)
  void spmm(const Mat& K, const double* X, double* Y, const double* W, double* out) {
    for (int c0 = 0; c0 < nrhs; c0 += 64) {
      const int cw = std::min(64, nrhs - c0);
      const int R = pow2(cw);
      hipLaunchKernelGGL(k_spmm_dot, dim3(kGrid), dim3(kThreads), 0, s, K, X, Y, W, nrhs, c0, cw, R,
                         out ? part : nullptr);
    }
    if (out)
      hipLaunchKernelGGL(k_reduce_parts, dim3(nrhs), dim3(kThreads), 0, s, part, kGrid, nrhs, out);
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

  void iteration(double rtol) {
    const dim3 gs((nrhs + 63) / 64), bs(64);
    spmm(A, p, q, p, tmp);                                       // q = A p, (p, q)
    hipLaunchKernelGGL(k_alpha, gs, bs, 0, s, S, tmp, nrhs, nactive);
    if (nrhs <= 64) {                                            // x, r update fused with ||r||^2
      hipLaunchKernelGGL(k_axpy, dim3(kGrid), dim3(kThreads), 0, s, x, r, p, q, S, n, nrhs,
                         pow2(nrhs), part);
      hipLaunchKernelGGL(k_reduce_parts, dim3(nrhs), dim3(kThreads), 0, s, part, kGrid, nrhs, tmp);
    } else {
      hipLaunchKernelGGL(k_axpy_wide, dim3(kGrid), dim3(kThreads), 0, s, x, r, p, q, S, n, nrhs);
      dot(r, r, nullptr, tmp);
    }
    hipLaunchKernelGGL(k_conv, gs, bs, 0, s, S, tmp, rtol, nrhs, nactive);
    spmm(M, r, z, r, tmp);                                       // z = M r, (r, z)
    hipLaunchKernelGGL(k_beta, gs, bs, 0, s, S, tmp, nrhs);
    if (nrhs <= 64)
      hipLaunchKernelGGL(k_pupd, dim3(kGrid), dim3(kThreads), 0, s, p, z, S, n, nrhs, pow2(nrhs));
    else
      hipLaunchKernelGGL(k_pupd_wide, dim3(kGrid), dim3(kThreads), 0, s, p, z, S, n, nrhs);
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
            int max_iter, int* iters, double* relres, hipStream_t s) {
  int rc;
  DevPool pool;
  Solver S{};
  S.A = A;
  S.M = M;
  S.n = A.n;
  S.nrhs = nrhs;
  S.s = s;
  const int64_t tot = S.n * nrhs;
  if ((rc = pool.alloc(&S.r, tot)) || (rc = pool.alloc(&S.z, tot)) || (rc = pool.alloc(&S.p, tot)) ||
      (rc = pool.alloc(&S.q, tot)) || (rc = pool.alloc(&S.part, (int64_t)kGrid * nrhs)) ||
      (rc = pool.alloc(&S.tmp, nrhs)) || (rc = pool.alloc(&S.S, nrhs)) || (rc = pool.alloc(&S.nactive, 1)))
    return rc;
  S.b = dB;
  S.x = dX;
  HIPCHK(hipMemsetAsync(S.nactive, 0, sizeof(int), s));
  HIPCHK(hipMemsetAsync(S.S, 0, sizeof(RhsState) * nrhs, s));
  const dim3 gs((nrhs + 63) / 64), bs(64);
  // x_0 = 0, r = b, z = M r, p = z
  hipLaunchKernelGGL(k_fill, dim3(kGrid), dim3(kThreads), 0, s, S.x, 0.0, tot);
  hipLaunchKernelGGL(k_copy, dim3(kGrid), dim3(kThreads), 0, s, S.r, dB, tot);
  S.dot(dB, dB, nullptr, S.tmp);
  hipLaunchKernelGGL(k_init_rhs, gs, bs, 0, s, S.S, S.tmp, nrhs, S.nactive);
  S.spmm(S.M, S.r, S.z, S.r, S.tmp);
  hipLaunchKernelGGL(k_set_rz, gs, bs, 0, s, S.S, S.tmp, nrhs);
  hipLaunchKernelGGL(k_copy, dim3(kGrid), dim3(kThreads), 0, s, S.p, S.z, tot);
  HIPCHK(hipGetLastError());
  // iterate in chunks, checking the running count between chunks
  int it = 0;
  const int chunk = 8;
  while (it < max_iter) {
    int nact = 0;
    HIPCHK(hipMemcpyAsync(&nact, S.nactive, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (nact == 0) break;
    const int k = std::min(chunk, max_iter - it);
    for (int t = 0; t < k; ++t) S.iteration(rtol);
    HIPCHK(hipGetLastError());
    it += k;
  }
  // true residual ||b - A x|| / ||b||
  S.spmm(S.A, S.x, S.q, nullptr, nullptr);
  S.dot(dB, dB, S.q, S.tmp);     // sum (b - Ax)^2
  std::vector<double> rr(nrhs);
  HIPCHK(hipMemcpyAsync(rr.data(), S.tmp, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
  std::vector<RhsState> hs(nrhs);
  HIPCHK(hipMemcpyAsync(hs.data(), S.S, sizeof(RhsState) * nrhs, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
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
    rc = pcg_run(dA, dM, nrhs, dB, dX, rtol, max_iter, iters, relres, s);
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
