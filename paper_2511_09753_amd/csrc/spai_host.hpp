// spai_host.hpp — host-side helpers of libspai: error reporting, CSR intake, device pool.
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <string>
#include <vector>

#include "spai.h"

namespace spai {

extern thread_local std::string g_last_error;
int fail(int code, const std::string& msg);

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      (void)hipGetLastError();                                                             \
      return ::spai::fail(SPAI_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));  \
    }                                                                                      \
  } while (0)

struct HostCsr {
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

// copy a borrowed CSR to the host and check its structure and finiteness
int fetch_csr(const spai_csr_t* A, HostCsr& h);
// exact symmetry (bitwise values) and a positive stored diagonal
int check_spd_symmetric(const HostCsr& h);
// symmetric pattern (values free)
int check_symmetric_pattern(const HostCsr& h);
// position of entry (i, j) or -1
int64_t find_entry(const HostCsr& h, int64_t i, int32_t j);
// permutation of the rows in breadth-first balls of about `ball` rows (locality order)
void locality_order(const HostCsr& h, int ball, std::vector<int32_t>& order);
extern const int kBallRows;   // ball size of the locality order (rows)

// owner of a handle's or a call's device allocations
struct DevPool {
  std::vector<void*> ptrs;
  size_t used = 0;
  int64_t limit = 0;
  int alloc_bytes(void** p, size_t bytes);
  template <typename U>
  int alloc(U** p, int64_t count) {
    return alloc_bytes((void**)p, sizeof(U) * (size_t)(count > 0 ? count : 1));
  }
  void release();                    // free everything allocated so far
  ~DevPool();
};

// matrix operand of the PCG kernels: ELL (eshift >= 0: row i in [i << eshift,
// (i + 1) << eshift), padding column -1), padded columns (beg, len) or CSR (rowptr),
// with float64 or float32 values
struct PcgMat {
  int64_t n = 0;
  int eshift = -1;
  const int64_t* rowptr = nullptr;
  const int64_t* beg = nullptr;
  const int32_t* len = nullptr;
  const int32_t* col = nullptr;
  const double* val = nullptr;
  const float* val32 = nullptr;
  // inside the PCG iterations: a product returns at once while *gate is 0 (no right-hand
  // side still running), and one that does its work adds 1 to *ran (null: not counted)
  const int* gate = nullptr;
  int* ran = nullptr;
  __device__ __forceinline__ int64_t row_begin(int64_t i) const {
    return eshift >= 0 ? (i << eshift) : beg ? beg[i] : rowptr[i];
  }
  __device__ __forceinline__ int64_t row_end(int64_t i) const {
    return eshift >= 0 ? ((i + 1) << eshift) : beg ? beg[i] + len[i] : rowptr[i + 1];
  }
  __device__ __forceinline__ double v(int64_t q) const { return val32 ? (double)val32[q] : val[q]; }
};

// preconditioned CG on device-resident operands (B, X on the device); `order` (device,
// n rows, or null for the natural order) is the order in which the products visit rows
// accumulated event-timed milliseconds and launches of the products inside the PCG
// iterations: [0] q = A p, [1] z = M r
struct PcgTiming {
  double ms[2] = {0.0, 0.0};
  int64_t calls[2] = {0, 0};
};

// the device blocks of a PCG solve, kept between solves of one size (a handle's): a solve
// of another size replaces them, and they are freed with the owner
struct PcgWork {
  DevPool pool;
  int64_t n = -1;
  int nrhs = 0;
  void* blk[9] = {};
};

int pcg_run(const PcgMat& A, const PcgMat& M, int nrhs, const double* dB, double* dX, double rtol,
            int max_iter, int* iters, double* relres, const int32_t* order, hipStream_t s,
            PcgTiming* timing, PcgWork* work = nullptr);

// extreme Ritz values of S (symmetric) after up to `steps` Lanczos steps with full
// reorthogonalisation from the device vector dv0: out = {theta_min, theta_max, res_min,
// res_max}; pool_limit bounds the call's device memory (0: none)
int lanczos_run(const PcgMat& S, int steps, const double* dv0, double* out, int* steps_done,
                int64_t pool_limit, hipStream_t s);

}  // namespace spai
