// spai_kern.hpp — device state and kernel launchers of libspai (host-visible declarations).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spai_dev.hpp"

namespace spai {

enum : int { kMR = 0, kCG = 1, kLOMR = 2 };

// Frobenius dots produced per column by the SpGEMM-dots kernel:
// 0 (R,AR)  1 (AR,AR)  2 (AR,AP)  3 (R,AP)  4 (AP,AP)  5 (P,AP)
constexpr int kND = 6;
constexpr int kCntSlots = 65536;   // workgroup slots per traffic counter
constexpr int kNCnt = 7;

// Per-matrix ("segment") scalar state; a single segment unless the handle is batched.
struct SegState {
  double dots[kND];   // reduced dots of the current iteration
  double rr;          // ||R_i||_F^2 of the current iterate
  double rz;          // (R_i, Z_i)_F with Z = Pi R (Pi-weighted CG), else ||R_i||_F^2
  double coef[4];     // a1, a2 (M + a1 X1 + a2 X2), c1, c2 (P = c1 R + c2 P)
  double step1, step2;// last step sizes (MR alpha | CG alpha, beta | LOMR delta, gamma)
  double inv_sqrt_n;  // 1 / sqrt(rows of this matrix)
  double last_resid;  // ||R||_F after the last completed iteration
  int iters;          // iterations completed
  int stop;           // 1 once converged or broken down
  int status;         // 0 running, 1 converged, 3 breakdown
  int first;          // LOMR: the next step is the first (MR) step
  int mr_fallbacks;   // LOMR degenerate steps taken as MR steps
  int pad;
};

// Global device state of a handle.
struct DevState {
  int any_active;     // 0 once every segment has stopped: kernels return at once
  int err;            // bit 0: a column exceeded the largest tile; bit 1: buffer overflow
  int curM, curP;     // which of the two buffers holds the current M / (P, P^T)
  int big_count[4];   // overflow-column list lengths (resid, dots, update)
  unsigned long long nnz_m, nnz_p;
  // cumulative entry counts for traffic accounting, one slot per workgroup and
  // counter (no contended atomics): counter c of workgroup b at cnt[c * kCntSlots + b];
  // counters 0-2 candidates in (M, P, P^T), 3-5 kept, 6 residual entries written
  unsigned long long* cnt;
  // global-cap radix selection
  double thrM, thrP;              // keep |x| > thr (thr already includes 1 + eta)
  double rawM, rawP;              // the (b+1)-th largest key itself (thrM/P + 2 doubles)
  unsigned long long sel_count;   // keys in the selection buffer
  unsigned long long sel_prefix;  // key bits fixed so far
  long long sel_rank;             // 1-based rank still to find inside the prefix
  long long sel_diag;             // diagonal candidates (excluded, always kept)
  int sel_done;                   // 1: threshold known
  int iter_active;                // 1: the current iteration runs (set by the step kernel)
  // per-iteration record of the drops (spai_history): rec[i * kRec + f], i = rec_i the
  // iteration in progress (-1: none), f = kept, seen, band of M (0-2) and of P (3-5)
  unsigned long long* rec;
  int rec_i, rec_cap;
  int rec_next, rec_pad;          // the next iteration's record
  // speculative floor of the global cap (magnitude keys, one matrix): the lean update
  // writes the off-diagonal candidates of M (all of P, P^T) only where |x| >= floor and
  // counts the others in below; the selection sets redo when its cut does not clear
  // floor / (1 - eta) (or there is no cut while entries were left out), and the update
  // and the selection then run again without floors.  0: no floor.
  double floorM, floorP;
  unsigned long long belowM, belowP;
  int redo, saved_active;
};
constexpr int kRec = 6;

struct Seg {                       // column -> matrix map for batched handles
  int nseg = 1;
  const int* of = nullptr;         // [n] matrix of each column (null when nseg == 1)
  SegState* st = nullptr;          // [nseg]
  __device__ __forceinline__ int segof(int64_t j) const { return nseg > 1 ? of[j] : 0; }
};

template <typename T>
struct Pair {                      // ping-pong pair of column buffers
  Cols<T> b[2];
  const int* cur = nullptr;        // device index of the current buffer
  __device__ __forceinline__ Cols<T> now() const { return b[*cur]; }
  __device__ __forceinline__ Cols<T> nxt() const { return b[*cur ^ 1]; }
};

// Columns too big for a tile are deferred to the next tier: small LDS tile -> large LDS
// tile -> huge tile, whose working set lives in device memory (`scratch`, one slice of
// `scratch_stride` bytes per workgroup); beyond that SPAI_ERR_CAPACITY.
struct BigList {
  int* list = nullptr;             // columns left to the large-tile pass
  int* count = nullptr;
  int* list2 = nullptr;            // columns left to the huge-tile pass
  int* count2 = nullptr;
  char* scratch = nullptr;
  int64_t scratch_stride = 0;
  int grid2 = 64;                  // workgroups of the huge-tile pass (scratch slices)
};

struct Tile {      // per-column tile
  int L, H;        // list entries, hash slots
  int DG = 0;      // update: neighbour columns (0: default)
  int waves = 0;   // dots, update: 5 = resident tier with registers capped at five waves per SIMD
};
// workgroups of the huge-tile pass: as many scratch slices as fit kHugeBudget bytes,
// between kHugeGridMin and kHugeGridMax (a multiple of 8, so every XCD gets as many)
constexpr int kHugeGridMin = 64, kHugeGridMax = 2048;
constexpr int64_t kHugeBudget = (int64_t)2 << 30;

struct UpdMode {
  int doM;       // form the (symmetrized, small-dropped) M candidates
  int x1, x2;    // lists added to M: 0 none, 1 R, 2 P, with coef[0], coef[1]
  int doP;       // form P and P^T candidates coef[2] R + coef[3] P
  int pR, pP;    // R / P take part in the P candidates
  int sym;       // symmetrize M
  int colcap;    // per-column caps: compute per-column thresholds
  double u;      // small-entry threshold on off-diagonal M (0 = off)
  int weighted;  // Pi = D_A^{-1}: the R list holds Z = Pi R, and R^T is scaled to Z^T
  int pad;
};

// ---------------- launchers (all enqueue on `s`) -----------------------------
int64_t scan_tmp_elems(int64_t n);
void launch_scan(const int64_t* in, int64_t* out, int64_t* total, int64_t n, int64_t* tmp,
                 hipStream_t s);

// per-segment sums of colpart[j * nd + d] in a fixed order -> red[seg * nd + d]
void launch_reduce(const double* colpart, int nd, int64_t n, const Seg& seg,
                   const int64_t* seg_beg, double* red, double* blockpart, hipStream_t s);

void launch_trace_parts(const Csr& A, double* colpart, hipStream_t s);
void launch_init_state(const Seg& seg, const double* red_tr, const int64_t* seg_beg, int64_t n,
                       double* cvec, int method, DevState* st, hipStream_t s);

template <typename T>
void launch_init_m(int64_t n, Cols<T> M, const double* cvec, const Seg& seg, hipStream_t s);

template <typename T>
void launch_zero_cols(int64_t n, Cols<T> X, hipStream_t s);

template <typename T>
void launch_bound_resid(const Csr& A, Pair<T> M, int64_t* ub, int64_t n, const DevState* st,
                        hipStream_t s);
template <typename T>
void launch_resid(const Csr& A, Pair<T> M, Cols<T> R, const int64_t* off, const int64_t* total,
                  double* colnorm, int weighted, double* colrz, BigList big, DevState* st,
                  Tile small, Tile large, Tile huge, hipStream_t s);

template <typename T>
void launch_dots(const Csr& A, Cols<T> R, Pair<T> P, int useR, int useP, int weighted,
                 double* colpart, BigList big, DevState* st, Tile small, Tile large, Tile huge,
                 hipStream_t s);

// implicit residual R_{i+1} = R_i - c A X (no dropping): X is Xr (xsrc 0) or P.now()
// (xsrc 1), c the segment's coef[cidx] (cidx -1: c = 1); Zout gets Pi R_{i+1} (weighted)
template <typename T>
void launch_bound_impl(const Csr& A, Cols<T> Rin, Cols<T> Xr, Pair<T> P, int xsrc, int64_t* ub,
                       int64_t n, const DevState* st, hipStream_t s);
template <typename T>
void launch_resid_impl(const Csr& A, Cols<T> Rin, Cols<T> Xr, Pair<T> P, int xsrc, int cidx,
                       const Seg& seg, const int64_t* off, const int64_t* total, Cols<T> Rout,
                       Cols<T> Zout, int weighted, double* colnorm, double* colrz, BigList big,
                       DevState* st, Tile small, Tile large, Tile huge, hipStream_t s);
template <typename T>
void launch_copy_cols(Cols<T> src, Cols<T> dst, int64_t n, const int64_t* total,
                      const DevState* st, hipStream_t s);

template <typename T>
void launch_bound_update(const Csr& A, Pair<T> M, Cols<T> R, Pair<T> P, Pair<T> PT, UpdMode md,
                         int64_t* ub, int64_t n, const DevState* st, hipStream_t s);
template <typename T>
void launch_update(const Csr& A, Pair<T> M, Cols<T> R, Pair<T> P, Pair<T> PT, UpdMode md,
                   const int64_t* off, const int64_t* total, const int32_t* kcol, double* tM,
                   double* tP, BigList big, const Seg& seg, DevState* st, Tile small,
                   Tile large, Tile huge, hipStream_t s, bool second = false);
// bytes of one workgroup's working set for a tile (the huge tier's scratch slice)
size_t resid_tile_bytes(Tile t, bool ell);
size_t dots_tile_bytes(Tile t, bool ell);
size_t update_tile_bytes(Tile t);

// global cap: exact (b+1)-th largest magnitude among the candidates in X.nxt() (score
// non-null: the (b+1)-th largest of the signed scores stored beside the candidates)
template <typename T>
void launch_global_select(Pair<T> X, int exclude_diag, int64_t m, double eta, int which,
                          unsigned long long* hist, unsigned long long* selbuf, int64_t n,
                          DevState* st, hipStream_t s, const double* score = nullptr);

// Appendix A heuristic scores of the M candidates in M.nxt(): sc per entry, sig the pair
// sums (the selection key); tiles as for the residual, sized by score_tile_bytes
template <typename T>
void launch_score(const Csr& A, Pair<T> M, double* sc, double* sig, BigList big, DevState* st,
                  Tile small, Tile large, Tile huge, int64_t n, hipStream_t s);
size_t score_tile_bytes(Tile t, bool ell);

// keep rule + in-place compaction of the candidates in X.nxt();
// kind 0: M (diagonal kept), 1: P (column threshold tcol[j]), 2: P^T (tcol[row]);
// score non-null (global cap): keep score > threshold instead of |x| > threshold
template <typename T>
void launch_compact(Pair<T> X, int kind, int colcap, int sym, int global, const double* tcol,
                    double eta, int64_t n, DevState* st, hipStream_t s,
                    const double* score = nullptr);

void launch_scal_step(int method, const Seg& seg, const double* red, DevState* st,
                      hipStream_t s);
void launch_scal_post(int method, const Seg& seg, const double* red, const double* red_rz,
                      double tol, double* hist, int hist_cap, int setup, DevState* st,
                      hipStream_t s);
extern int g_grid_cols;   // persistent grid of the per-column kernels (multiple of 8)
// zero the drop record; the next iteration's record is `next`
void launch_rec_clear(DevState* st, int next, hipStream_t s);
// the second, floor-free pass of the update and the selection runs only where the first
// pass's floors were too high: redo_begin masks the iteration unless st->redo (and clears
// the floors), redo_end restores it; drop_finish sets the next iteration's floors
void launch_redo_begin(DevState* st, hipStream_t s);
void launch_redo_end(DevState* st, hipStream_t s);
// the new M (doM) and P (doP) become current; with floors, the next iteration's floors
// are set from this iteration's cuts
void launch_drop_finish(DevState* st, int doM, int doP, int floors, double frac, hipStream_t s);

}  // namespace spai
