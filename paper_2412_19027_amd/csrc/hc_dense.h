// Dense Cholesky of the KKT Schur complement and triangular solves (gfx950).
#pragma once
#include "hc_common.h"

namespace hc {
// Optional HIP-event timing of the MFMA update launches of a factorisation.
struct Prof {
  std::vector<hipEvent_t> ev;   // pairs (start, stop)
  size_t used = 0;
  double flops = 0;             // algorithmic flops of the recorded launches
  int64_t launches = 0;
  hipEvent_t next();
  double collect_ms();          // synchronises, sums elapsed times, resets the pool
  ~Prof();
};
// A second stream (default priority) and a pool of events for the
// look-ahead factorisation: the trailing update of a panel runs on `side`
// while the next panel is factored on the caller's stream.
struct Aux {
  int64_t nb = 768;     // panel width (multiple of 64) of the delayed updates
  bool serial = false;  // every launch on the caller's stream, one at a time (timing)
  hipStream_t side = nullptr;
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  void init();          // creates the side stream (once)
  hipEvent_t next();    // event from the pool (timing disabled)
  ~Aux();
};
// In-place lower Cholesky of the n x n column-major S (leading dim ld).
// Linv receives the inverses of the 64 x 64 diagonal factor blocks
// (linv_elems(n) entries).  Pivots <= tol are replaced by fix and counted.
// The trailing updates overlap the next panel's factorisation on aux's side
// stream unless aux->serial; all work is complete with respect to `st` on
// return.
// `last` (host, n entries, or null for a dense matrix) is the envelope of
// the lower triangle: last[j] - 1 is the largest row i with a nonzero S[i, k]
// for some k <= j (non-decreasing in j).  Cholesky fill stays inside it, so
// the TRSM and trailing updates of a panel stop at the rows its columns
// reach; entries below the envelope are never touched and stay zero.
template <typename T>
void dense_cholesky(T* S, int64_t n, int64_t ld, T* Linv, double tol, double fix, unsigned long long* hits,
                    hipStream_t st, Prof* prof, Aux* aux, const int64_t* last = nullptr);
// flops of the envelope-limited factorisation (n^3 / 3 when last is null)
double envelope_cholesky_flops(int64_t n, const int64_t* last);
// Inverses X (and X') of the 256 x 256 diagonal blocks of the factor, from
// the 64 x 64 block inverses; inv256_elems(n) entries each.
template <typename T>
void dense_block_inverses(const T* L, int64_t n, int64_t ld, const T* Linv, T* X, T* XT, hipStream_t st);
int64_t inv256_elems(int64_t n);
// X = L^-T L^-1 B for nrhs <= 4 right-hand sides (column-major, leading dim
// n); B and Y are overwritten (Y receives the forward result).  With the
// factorisation's envelope `last` the updates skip the zero blocks.
template <typename T>
void dense_solve(const T* L, int64_t n, int64_t ld, const T* X256, const T* XT256, T* B, T* Y, T* X, int nrhs,
                 hipStream_t st, const int64_t* last = nullptr);
// C[i, j] += alpha * sum_k A[i, k] B[j, k] (column-major operands); with
// `lower`, tiles strictly above the diagonal of the global matrix (C[0,0] at
// global (gr, gc)) are skipped.
template <typename T>
void gemm_nt(T* C, int64_t ldc, const T* A, int64_t lda, const T* B, int64_t ldb, int64_t M, int64_t N, int64_t K,
             T alpha, bool lower, int64_t gr, int64_t gc, hipStream_t st);
int64_t linv_elems(int64_t n);
double cholesky_flops(int64_t n);
}  // namespace hc
