// Dense factorisation of the KKT Schur complement on gfx950.
//
// After the cone rows are eliminated (their pivots are the -(H_c + delta I)
// blocks), the quasi-definite LDL' of the regularised KKT matrix
// (eq. linsys_2x2, Sec. 3.7) continues on the positive definite Schur
// complement S = P + delta I + A' M A.  This file factors S = L L' (the
// positive pivots of the LDL', D = diag(L)^2 absorbed into L) and solves with
// L, in FP64 or -- for the mixed-precision mode of Sec. 3.7 -- FP32 with FP32
// accumulation.
//
// Layout: S is column-major with leading dimension ld, lower triangle used.
// Algorithm: blocked right-looking Cholesky with 64-wide diagonal blocks.
//   diag:   the 64x64 block is factored in registers by one workgroup, which
//           also writes the inverse of the factor block (Linv, 64x64 per block)
//   trsm:   L21 = A21 * Linv' in place, one workgroup per 64 rows
//   update: trailing C -= L21 L21' on MFMA (v_mfma_f64_16x16x4f64 or
//           v_mfma_f32_16x16x4f32), 256x128 tiles, lower tiles only.  The
//           update of the trailing matrix is delayed to every panel of
//           Aux::nb columns (the panel's own columns are updated eagerly),
//           so the trailing matrix is read and written once per panel.
// Triangular solves use the stored Linv blocks: one launch per 256 rows.
#include "hc_dense.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace hc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Both instructions take A[i][k] from lane i + 16 k and B[k][j] from lane
// j + 16 k.  Output element r of lane l is D[row(l, r)][l % 16]; the FP64
// form interleaves rows (l/16 + 4 r), the FP32 form blocks them (4 (l/16) + r).
template <> struct Mfma<double> {
  typedef v4d acc_t;
  __device__ static inline acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
  typedef v4f acc_t;
  __device__ static inline acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int BS = 64;    // diagonal block

// ---------------------------------------------------------------------------
// diagonal block: Cholesky + inverse of the factor, one wave
// ---------------------------------------------------------------------------
// value of v in a runtime-uniform lane
__device__ inline double lane_bcast_u(double v, int src) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, src);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ inline float lane_bcast_u(float v, int src) {
  return __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(v), src));
}
__device__ inline double lane_shfl(double v, int src) { return __shfl(v, src, 64); }
__device__ inline float lane_shfl(float v, int src) { return __shfl(v, src, 64); }

template <typename T>
__global__ __launch_bounds__(256) void k_chol_diag(T* __restrict__ A, int64_t ld, int64_t c, int64_t n,
                                                   T* __restrict__ Linv, double tol, double fix,
                                                   unsigned long long* __restrict__ hits) {
  // Cholesky of one 64 x 64 diagonal block and the inverse of its factor, by
  // 16-column blocks.  Thread (i, p) = (lane, wave) keeps r[q] = A[i][16p + q].
  // Column block pj is factored by wave pj alone: the pivot comes from lane
  // j by readlane and so do the multipliers of the later columns, so the 16
  // steps need no barrier.  The finished block goes to LDS and the waves to
  // its right apply it (a rank-16 update), one barrier per block.  L^-1 is
  // then built by 16 x 16 blocks: each wave inverts its diagonal block by
  // forward substitution (rows exchanged with shuffles), and the blocks
  // below the diagonal follow by distance from it,
  // Y_ij = -Y_ii sum_{k=j}^{i-1} L_ik Y_kj.
  __shared__ T Ls[BS][BS + 1];          // L, then read by the inverse
  __shared__ T Ys[BS][BS + 1];          // L^-1
  __shared__ T Ts[4][16][17];           // per-wave scratch of the inverse
  const int lane = threadIdx.x & 63;
  const int p = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int bs = (int)std::min<int64_t>(BS, n - c);
  T r[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = 16 * p + q;
    const T g = A[(c + std::min(lane, bs - 1)) + (c + std::min(k, bs - 1)) * ld];
    r[q] = (lane < bs && k < bs) ? (k <= lane ? g : T(0)) : (lane == k ? T(1) : T(0));
  }
  int nhits = 0;
  // ---- L: column block pj is factored by its owning wave alone (pivots by
  // readlane, no barrier), published, and applied by the waves to its right
#pragma unroll 1
  for (int pj = 0; pj < 4; ++pj) {
    if (p == pj) {
#pragma unroll
      for (int qj = 0; qj < 16; ++qj) {
        const int j = 16 * pj + qj;
        double d = (double)lane_bcast_u(r[qj], j);
        if (j < bs && !(d > tol)) {
          d = fix;
          ++nhits;
        }
        double e = __builtin_amdgcn_rsq(d);
        e = e * (1.5 - 0.5 * d * e * e);
        e = e * (1.5 - 0.5 * d * e * e);
        const T inv = (T)e, ljj = (T)(d * e);
        const T li = (lane > j) ? r[qj] * inv : T(0);
        r[qj] = (lane == j) ? ljj : li;   // zero above the diagonal
#pragma unroll
        for (int q = qj + 1; q < 16; ++q) r[q] -= li * lane_bcast_u(li, 16 * pj + q);
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) Ls[lane][16 * pj + q] = (16 * pj + q <= lane) ? r[q] : T(0);
    }
    __syncthreads();
    if (p > pj) {
      T a[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) a[t] = Ls[lane][16 * pj + t];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        T s = 0;
#pragma unroll
        for (int t = 0; t < 16; ++t) s += a[t] * Ls[16 * p + q][16 * pj + t];
        r[q] -= s;
      }
    }
  }
  if (lane == 0 && nhits) atomicAdd(hits, (unsigned long long)nhits);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = 16 * p + q;
    if (lane < bs && k < bs && k <= lane) A[(c + lane) + (c + k) * ld] = r[q];
  }
  // ---- L^-1 by 16 x 16 blocks.  Lane (s, g) = (lane % 16, lane / 16) holds
  // row s, columns 4g .. 4g + 3 of a block.
  const int s = lane & 15, g = lane >> 4;
  {
    // diagonal block p: forward substitution over its rows
    const int o = 16 * p;
    T y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) y[u] = (s == 4 * g + u) ? T(1) : T(0);
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const T dinv = T(1) / Ls[o + t][o + t];
      const T lst = Ls[o + s][o + t];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const T yt = lane_shfl(y[u], t + 16 * g) * dinv;   // row t, final
        y[u] = (s == t) ? yt : ((s > t) ? y[u] - lst * yt : y[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) Ys[o + s][o + 4 * g + u] = y[u];
  }
  __syncthreads();
  // off-diagonal blocks by distance from the diagonal:
  //   Y_ij = -Y_ii sum_{k=j}^{i-1} L_ik Y_kj
#pragma unroll 1
  for (int dist = 1; dist < 4; ++dist) {
    if (p + dist < 4) {
      const int i = p + dist, j = p;
      T t4[4] = {};
      for (int k = j; k < i; ++k)
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          const T l = Ls[16 * i + s][16 * k + m];
#pragma unroll
          for (int u = 0; u < 4; ++u) t4[u] += l * Ys[16 * k + m][16 * j + 4 * g + u];
        }
#pragma unroll
      for (int u = 0; u < 4; ++u) Ts[p][s][4 * g + u] = t4[u];
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // this wave's scratch writes landed
      T o4[4] = {};
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const T yim = Ys[16 * i + s][16 * i + m];
#pragma unroll
        for (int u = 0; u < 4; ++u) o4[u] -= yim * Ts[p][m][4 * g + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) Ys[16 * i + s][16 * j + 4 * g + u] = o4[u];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = 16 * p + q;
    Linv[lane + k * BS] = (k <= lane) ? Ys[lane][k] : T(0);
  }
}

// ---------------------------------------------------------------------------
// TRSM: rows [r0, r1) of the 64 columns starting at c: A21 <- A21 * Linv'
// ---------------------------------------------------------------------------
// On MFMA: each wave takes 16 rows and all 64 columns (four 16 x 16 output
// tiles, 16 k-steps of four).  A wave's 16 x 64 block of A21 is loaded into
// registers at once; Linv goes through an 8 KB LDS slice, the 16 rows of Linv
// that one output tile needs, one tile after another.  With few registers and
// 8 KB of LDS a workgroup fits beside a running trailing-update workgroup on
// the same compute unit instead of waiting for one to finish: this kernel sits
// on the factorisation's critical path while the trailing update runs.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_trsm(
    T* __restrict__ A, int64_t ld, int64_t c, int64_t r0, int64_t r1, const T* __restrict__ Linv) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T Ls[BS][16];   // Ls[k][jj] = Linv[16 t + jj][k] for the current tile t
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t rb = r0 + (int64_t)blockIdx.x * BS + wave * 16;   // first row of this wave
  // operand lanes: A[i = lane % 16][k = lane / 16], B[k = lane / 16][j = lane % 16]
  const int64_t ra = std::min<int64_t>(rb + (lane & 15), r1 - 1);   // rows past r1 repeat the last one
  const T* pa = A + ra + (c + (lane >> 4)) * ld;
  T a[BS / 4];
#pragma unroll
  for (int q = 0; q < BS / 4; ++q) a[q] = pa[(int64_t)(4 * q) * ld];
#pragma unroll 1
  for (int t = 0; t < 4; ++t) {
    __syncthreads();   // the previous slice has been read
#pragma unroll
    for (int q = 0; q < BS * 16 / 256; ++q) {
      const int e = tid + 256 * q;
      Ls[e >> 4][e & 15] = Linv[(16 * t + (e & 15)) + (e >> 4) * BS];
    }
    __syncthreads();
    acc_t acc = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < BS / 4; ++q) acc = Mfma<T>::op(a[q], Ls[4 * q + (lane >> 4)][lane & 15], acc);
    // X[i][j] = sum_k A[i][k] Linv[j][k]; this wave loaded its rows above,
    // other waves own other rows
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = rb + Mfma<T>::row(lane, r);
      if (row < r1) A[row + (c + 16 * t + (lane & 15)) * ld] = acc[r];
    }
  }
}

// ---------------------------------------------------------------------------
// In-panel update after a TRSM: C -= A B' with K <= 64 (one 64-column block
// of L), the shape of the TRSM so that it also fits beside a running
// trailing-update workgroup: a workgroup takes 64 rows x 64 columns of C,
// each wave 16 rows (its 16 x K block of A in registers) and four 16 x 16
// tiles, B through an 8 KB LDS slice per tile.  Tiles strictly above the
// global diagonal (C[0, 0] at global (gr, gc)) are skipped.  The products are
// the same MFMA chain as the large update kernels' (k in steps of four).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_gemm_panel(
    T* __restrict__ C, int64_t ldc, const T* __restrict__ A, int64_t lda, const T* __restrict__ B, int64_t ldb,
    int64_t M, int64_t N, int K, int64_t gr, int64_t gc) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T Bs[BS][16];   // Bs[k][jj] = B[j0 + jj][k] for the current tile
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i_blk = (int64_t)blockIdx.x * BS, j_blk = (int64_t)blockIdx.y * BS;
  if (gr + i_blk + BS - 1 < gc + j_blk) return;   // block strictly above the diagonal
  const int64_t rb = i_blk + wave * 16;             // first row of this wave
  const int64_t ra = std::min<int64_t>(rb + (lane & 15), M - 1);
  const T* pa = A + ra;
  T a[BS / 4];
#pragma unroll
  for (int q = 0; q < BS / 4; ++q) {
    const int k = 4 * q + (lane >> 4);
    const T v = pa[(int64_t)std::min(k, K - 1) * lda];
    a[q] = k < K ? v : T(0);
  }
#pragma unroll 1
  for (int t = 0; t < 4; ++t) {
    const int64_t j0 = j_blk + 16 * t;
    if (j0 >= N) break;
    __syncthreads();   // the previous slice has been read
#pragma unroll
    for (int q = 0; q < BS * 16 / 256; ++q) {
      const int e = tid + 256 * q, k = e >> 4, jj = e & 15;
      const T v = B[std::min<int64_t>(j0 + jj, N - 1) + (int64_t)std::min(k, K - 1) * ldb];
      Bs[k][jj] = k < K ? v : T(0);
    }
    __syncthreads();
    if (gr + rb + 15 < gc + j0) continue;   // this wave's rows lie above the tile's columns
    acc_t acc = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < BS / 4; ++q) acc = Mfma<T>::op(a[q], Bs[4 * q + (lane >> 4)][lane & 15], acc);
    const int64_t j = j0 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = rb + Mfma<T>::row(lane, r);
      if (i < M && j < N) C[i + j * ldc] -= acc[r];
    }
  }
}

// ---------------------------------------------------------------------------
// C[i, j] += alpha * sum_k A[i, k] * B[j, k]  (i < M, j < N, k < K), all
// column-major; 128 x 128 tiles of 4 waves, each wave 64 x 64 on 16 MFMA
// accumulators.  `lower` skips tiles strictly above the global diagonal, whose
// position is given by the global indices (gr, gc) of C[0, 0].
// ---------------------------------------------------------------------------
constexpr int TM = 128, TN = 128, TK = 16;
static_assert(TK * TM % 512 == 0, "staging layout");

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_nt(T* __restrict__ C, int64_t ldc, const T* __restrict__ A, int64_t lda,
                                                 const T* __restrict__ B, int64_t ldb, int64_t M, int64_t N, int64_t K,
                                                 T alpha, int lower, int64_t gr, int64_t gc, int tiles_n) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int PER = TK * TM / 256;   // staged elements per thread and operand
  __shared__ T As[TK][TM + 4];
  __shared__ T Bs[TK][TN + 4];
  const int tile_m = blockIdx.x / tiles_n, tile_n = blockIdx.x % tiles_n;
  const int64_t i_base = (int64_t)tile_m * TM, j_base = (int64_t)tile_n * TN;
  if (lower && gr + i_base + TM - 1 < gc + j_base) return;   // tile strictly above the diagonal
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  // thread tid stages rows i = tid % 128 (+0) for k = tid / 128 + 2 e, e < PER
  const int si = tid % TM, sk = tid / TM;
  const int64_t gi = i_base + si, gj = j_base + si;
  T ra[PER], rb[PER];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int64_t gk = k0 + sk + 2 * e;
      ra[e] = (gi < M && gk < K) ? A[gi + gk * lda] : T(0);
      rb[e] = (gj < N && gk < K) ? B[gj + gk * ldb] : T(0);
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      As[sk + 2 * e][si] = ra[e];
      Bs[sk + 2 * e][si] = rb[e];
    }
  };
  fetch(0);
  stage();
  __syncthreads();
  for (int64_t k0 = 0; k0 < K; k0 += TK) {
    const bool more = (k0 + TK < K);
    if (more) fetch(k0 + TK);   // global loads in flight during the MFMAs below
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      T a_op[4], b_op[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a_op[t] = As[kk + (lane >> 4)][wm + t * 16 + (lane & 15)];
        b_op[t] = Bs[kk + (lane >> 4)][wn + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<T>::op(a_op[a], b_op[b], acc[a][b]);
    }
    __syncthreads();
    if (more) {
      stage();
      __syncthreads();
    }
  }
  // lane holds D[row(lane, r)][lane % 16] of each 16 x 16 tile.  The C loads
  // of half a wave tile are issued together from clamped (always valid)
  // addresses so that their latencies overlap; only the stores are predicated.
#pragma unroll
  for (int h = 0; h < 4; h += 2) {
    T cv[2][4][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t j = std::min<int64_t>(j_base + wn + b * 16 + (lane & 15), N - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = std::min<int64_t>(i_base + wm + (h + a) * 16 + Mfma<T>::row(lane, r), M - 1);
          cv[a][b][r] = C[i + j * ldc];
        }
      }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t j = j_base + wn + b * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = i_base + wm + (h + a) * 16 + Mfma<T>::row(lane, r);
          if (i < M && j < N) C[i + j * ldc] = cv[a][b][r] + alpha * acc[h + a][b][r];
        }
      }
  }
}

// ---------------------------------------------------------------------------
// FP64 update kernel for K % 16 == 0: 256 x 128 tiles of 8 waves (4 x 2 wave
// tiles of 64 x 64, two waves per SIMD), operand panels streamed straight from
// global memory into a 3-stage LDS ring with global_load_lds_dwordx4 (no
// staging registers), so two chunks are always in flight while the MFMAs of
// the third run.  The operand reads from LDS are issued as inline asm with
// explicit waits: the compiler treats the LDS DMA as a store that may alias
// every LDS read and would otherwise wait for all outstanding DMA (including
// the prefetches) before each read.
// ---------------------------------------------------------------------------
constexpr int DM = 256, DN = 128, DK = 16, DST = 3;
#define HC_LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))

__device__ inline uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

__global__ __launch_bounds__(512) void k_gemm_nt_dma(double* __restrict__ C, int64_t ldc, const double* __restrict__ A,
                                                     int64_t lda, const double* __restrict__ B, int64_t ldb, int64_t M,
                                                     int64_t N, int64_t K, double alpha, int lower, int64_t gr,
                                                     int64_t gc, int tiles_n) {
  // one LDS block: the operand ring during the k loop, then the C staging
  // area of the epilogue
  __shared__ __align__(16) double smem[DST * DK * DM + DST * DK * DN];
  double(*As)[DK][DM] = reinterpret_cast<double(*)[DK][DM]>(smem);
  double(*Bs)[DK][DN] = reinterpret_cast<double(*)[DK][DN]>(smem + DST * DK * DM);
  const int tile_m = blockIdx.x / tiles_n, tile_n = blockIdx.x % tiles_n;
  const int64_t i_base = (int64_t)tile_m * DM, j_base = (int64_t)tile_n * DN;
  if (lower && gr + i_base + DM - 1 < gc + j_base) return;   // tile strictly above the diagonal
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 3) * 64, wn = (wave >> 2) * 64;
  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0, 0, 0, 0};
  // lane l loads rows (2l, 2l+1) of a 128-row half panel.  M and N are even
  // here (the caller leaves odd last rows / columns to the edge kernel), so
  // every pair below M is loaded whole; pairs past the end repeat the last
  // pair, and their products land in rows / columns that are never stored.
  const int64_t alast = (M - 2) & ~int64_t(1), blast = (N - 2) & ~int64_t(1);
  const double* pa0 = A + std::min<int64_t>(i_base + 2 * lane, alast);
  const double* pa1 = A + std::min<int64_t>(i_base + 128 + 2 * lane, alast);
  const double* pb = B + std::min<int64_t>(j_base + 2 * lane, blast);
  const int nk = (int)(K / DK);
  auto issue = [&](int kc, int stg) {   // wave w fills k-rows 2w and 2w + 1 of the chunk
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int k = wave * 2 + e;
      const int64_t gk = (int64_t)kc * DK + k;
      __builtin_amdgcn_global_load_lds((const void*)(pa0 + gk * lda), HC_LDS_PTR(&As[stg][k][0]), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(pa1 + gk * lda), HC_LDS_PTR(&As[stg][k][128]), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(pb + gk * ldb), HC_LDS_PTR(&Bs[stg][k][0]), 16, 0, 0);
    }
  };
  const uint32_t a_off = lds_addr(&As[0][lane >> 4][wm + (lane & 15)]);
  const uint32_t b_off = lds_addr(&Bs[0][lane >> 4][wn + (lane & 15)]);
  constexpr uint32_t SA = DK * DM * 8, SB_ = DK * DN * 8;
  issue(0, 0);
  if (nk > 1) issue(1, 1);
  for (int kc = 0; kc < nk; ++kc) {
    // each wave has 6 loads per chunk in flight: vmcnt(6) leaves only the
    // next chunk outstanding, i.e. chunk kc has landed
    if (kc + 1 < nk) __builtin_amdgcn_s_waitcnt(0xF76);
    else __builtin_amdgcn_s_waitcnt(0xF70);
    __builtin_amdgcn_s_barrier();
    if (kc + 2 < nk) issue(kc + 2, (kc + 2) % DST);   // that stage was last read before this barrier
    const int stg = kc % DST;
    const uint32_t sa = a_off + stg * SA, sb = b_off + stg * SB_;
#pragma unroll
    for (int kk = 0; kk < DK; kk += 4) {
      double a0, a1, a2, a3, b0, b1, b2, b3;
      const uint32_t ra = sa + kk * DM * 8, rb = sb + kk * DN * 8;
      asm volatile("ds_read_b64 %0, %1 offset:0" : "=v"(a0) : "v"(ra));
      asm volatile("ds_read_b64 %0, %1 offset:128" : "=v"(a1) : "v"(ra));
      asm volatile("ds_read_b64 %0, %1 offset:256" : "=v"(a2) : "v"(ra));
      asm volatile("ds_read_b64 %0, %1 offset:384" : "=v"(a3) : "v"(ra));
      asm volatile("ds_read_b64 %0, %1 offset:0" : "=v"(b0) : "v"(rb));
      asm volatile("ds_read_b64 %0, %1 offset:128" : "=v"(b1) : "v"(rb));
      asm volatile("ds_read_b64 %0, %1 offset:256" : "=v"(b2) : "v"(rb));
      asm volatile("ds_read_b64 %0, %1 offset:384" : "=v"(b3) : "v"(rb));
      asm volatile("s_waitcnt lgkmcnt(0)" : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(b0), "+v"(b1), "+v"(b2),
                   "+v"(b3));
      const double ao[4] = {a0, a1, a2, a3}, bo[4] = {b0, b1, b2, b3};
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<double>::op(ao[a], bo[b], acc[a][b]);
    }
  }
  // epilogue through LDS, one half of the tile's columns at a time: the four
  // waves owning those columns write their accumulators column-major (stride
  // CS doubles: two-way bank conflicts on the write, none on the read), then
  // all eight waves stream whole columns, lane l handling rows 4l .. 4l + 3
  // with 16-byte loads and stores of C (full cache lines per wave instead of
  // 32-byte pieces of 16 lines).  M and N are even here, so rows come in
  // pairs and each 16-byte piece is either wholly inside or wholly outside.
  constexpr int CS = DM + 2;
  static_assert(DN / 2 * CS <= DST * DK * (DM + DN), "C staging fits the operand ring");
  __syncthreads();   // every wave is done with the operand ring
  double* Cs = smem;
  const int64_t i0 = i_base + 4 * lane;
  const bool lo_ok = i0 < M, hi_ok = i0 + 2 < M;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (wn == 64 * h) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            Cs[(16 * b + (lane & 15)) * CS + wm + 16 * a + Mfma<double>::row(lane, r)] = acc[a][b][r];
    }
    __syncthreads();
    v2d cg[8][2];
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int64_t j = std::min<int64_t>(j_base + 64 * h + 8 * wave + cc, N - 1);
      cg[cc][0] = *reinterpret_cast<const v2d*>(C + std::min<int64_t>(i0, M - 2) + j * ldc);
      cg[cc][1] = *reinterpret_cast<const v2d*>(C + std::min<int64_t>(i0 + 2, M - 2) + j * ldc);
    }
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int col = 8 * wave + cc;
      const int64_t j = j_base + 64 * h + col;
      const v2d* cs = reinterpret_cast<const v2d*>(Cs + col * CS + 4 * lane);
      const v2d u0 = cs[0], u1 = cs[1];
      v2d* dst = reinterpret_cast<v2d*>(C + i0 + j * ldc);
      if (j < N && lo_ok) dst[0] = cg[cc][0] + alpha * u0;
      if (j < N && hi_ok) dst[1] = cg[cc][1] + alpha * u1;
    }
    __syncthreads();
  }
}

// FP32 counterpart (mixed mode): 32-deep chunks, so one k-row of the A panel
// (256 floats) is one dwordx4 DMA, and one dwordx4 DMA fills two adjacent
// k-rows of the B panel (128 floats each: lanes 0-31 the first, 32-63 the
// second); each wave fills 4 k-rows per chunk (6 loads in flight).
constexpr int FK = 32;
__global__ __launch_bounds__(512) void k_gemm_nt_dma32(float* __restrict__ C, int64_t ldc, const float* __restrict__ A,
                                                       int64_t lda, const float* __restrict__ B, int64_t ldb,
                                                       int64_t M, int64_t N, int64_t K, float alpha, int lower,
                                                       int64_t gr, int64_t gc, int tiles_n) {
  __shared__ __align__(16) float smem[DST * FK * DM + DST * FK * DN];
  float(*As)[FK][DM] = reinterpret_cast<float(*)[FK][DM]>(smem);
  float(*Bs)[FK][DN] = reinterpret_cast<float(*)[FK][DN]>(smem + DST * FK * DM);
  const int tile_m = blockIdx.x / tiles_n, tile_n = blockIdx.x % tiles_n;
  const int64_t i_base = (int64_t)tile_m * DM, j_base = (int64_t)tile_n * DN;
  if (lower && gr + i_base + DM - 1 < gc + j_base) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 3) * 64, wn = (wave >> 2) * 64;
  v4f acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0, 0, 0, 0};
  // lane l loads rows 4l..4l+3 of A, and rows 4 (l % 32) .. + 3 of B for
  // k-row (l / 32) of a pair.  M and N are multiples of four here (the caller
  // leaves the rest to the edge kernel); groups past the end repeat the last
  // group and only feed entries that are never stored.
  const int64_t alast = (M - 4) & ~int64_t(3), blast = (N - 4) & ~int64_t(3);
  const float* pa = A + std::min<int64_t>(i_base + 4 * lane, alast);
  const float* pb = B + std::min<int64_t>(j_base + 4 * (lane & 31), blast) + (int64_t)(lane >> 5) * ldb;
  const int nk = (int)(K / FK);
  auto issue = [&](int kc, int stg) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = wave * 4 + e;
      const int64_t gk = (int64_t)kc * FK + k;
      __builtin_amdgcn_global_load_lds((const void*)(pa + gk * lda), HC_LDS_PTR(&As[stg][k][0]), 16, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; e += 2) {
      const int k = wave * 4 + e;
      const int64_t gk = (int64_t)kc * FK + k;
      __builtin_amdgcn_global_load_lds((const void*)(pb + gk * ldb), HC_LDS_PTR(&Bs[stg][k][0]), 16, 0, 0);
    }
  };
  const uint32_t a_off = lds_addr(&As[0][lane >> 4][wm + (lane & 15)]);
  const uint32_t b_off = lds_addr(&Bs[0][lane >> 4][wn + (lane & 15)]);
  constexpr uint32_t SA = FK * DM * 4, SB_ = FK * DN * 4;
  issue(0, 0);
  if (nk > 1) issue(1, 1);
  for (int kc = 0; kc < nk; ++kc) {
    if (kc + 1 < nk) __builtin_amdgcn_s_waitcnt(0xF76);   // vmcnt(6): chunk kc landed
    else __builtin_amdgcn_s_waitcnt(0xF70);
    __builtin_amdgcn_s_barrier();
    if (kc + 2 < nk) issue(kc + 2, (kc + 2) % DST);
    const int stg = kc % DST;
    const uint32_t sa = a_off + stg * SA, sb = b_off + stg * SB_;
#pragma unroll
    for (int kk = 0; kk < FK; kk += 4) {
      float a0, a1, a2, a3, b0, b1, b2, b3;
      const uint32_t ra = sa + kk * DM * 4, rb = sb + kk * DN * 4;
      asm volatile("ds_read_b32 %0, %1 offset:0" : "=v"(a0) : "v"(ra));
      asm volatile("ds_read_b32 %0, %1 offset:64" : "=v"(a1) : "v"(ra));
      asm volatile("ds_read_b32 %0, %1 offset:128" : "=v"(a2) : "v"(ra));
      asm volatile("ds_read_b32 %0, %1 offset:192" : "=v"(a3) : "v"(ra));
      asm volatile("ds_read_b32 %0, %1 offset:0" : "=v"(b0) : "v"(rb));
      asm volatile("ds_read_b32 %0, %1 offset:64" : "=v"(b1) : "v"(rb));
      asm volatile("ds_read_b32 %0, %1 offset:128" : "=v"(b2) : "v"(rb));
      asm volatile("ds_read_b32 %0, %1 offset:192" : "=v"(b3) : "v"(rb));
      asm volatile("s_waitcnt lgkmcnt(0)" : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(b0), "+v"(b1), "+v"(b2),
                   "+v"(b3));
      const float ao[4] = {a0, a1, a2, a3}, bo[4] = {b0, b1, b2, b3};
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<float>::op(ao[a], bo[b], acc[a][b]);
    }
  }
  // epilogue through LDS as in the FP64 kernel; M is a multiple of four
  // here, so each lane's 16-byte piece of a column is wholly inside or
  // wholly outside
  constexpr int CS = DM + 4;
  static_assert(DN / 2 * CS <= DST * FK * (DM + DN), "C staging fits the operand ring");
  __syncthreads();
  float* Cs = smem;
  const int64_t i0 = i_base + 4 * lane;
  const bool ok = i0 < M;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (wn == 64 * h) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            Cs[(16 * b + (lane & 15)) * CS + wm + 16 * a + Mfma<float>::row(lane, r)] = acc[a][b][r];
    }
    __syncthreads();
    v4f cg[8];
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int64_t j = std::min<int64_t>(j_base + 64 * h + 8 * wave + cc, N - 1);
      cg[cc] = *reinterpret_cast<const v4f*>(C + std::min<int64_t>(i0, M - 4) + j * ldc);
    }
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int col = 8 * wave + cc;
      const int64_t j = j_base + 64 * h + col;
      const v4f u = *reinterpret_cast<const v4f*>(Cs + col * CS + 4 * lane);
      if (j < N && ok) *reinterpret_cast<v4f*>(C + i0 + j * ldc) = cg[cc] + alpha * u;
    }
    __syncthreads();
  }
}

static bool dma32_ok(const void* A, int64_t lda, const void* B, int64_t ldb, int64_t M, int64_t N, int64_t K) {
  return K % FK == 0 && M >= 4 && N >= 4 && lda % 4 == 0 && ldb % 4 == 0 && ((uintptr_t)A % 16) == 0 &&
         ((uintptr_t)B % 16) == 0;
}

static bool dma_ok(const void* A, int64_t lda, const void* B, int64_t ldb, int64_t M, int64_t N, int64_t K) {
  return K % DK == 0 && M >= 2 && N >= 2 && lda % 2 == 0 && ldb % 2 == 0 && ((uintptr_t)A % 16) == 0 &&
         ((uintptr_t)B % 16) == 0;
}

// Entries of C outside the leading M' x N' block (rows [M', M) and columns
// [N', N)) that the DMA kernels leave to this one: their loads come in whole
// 16-byte groups of rows, so the last M % g rows and N % g columns (g = 2 for
// FP64, 4 for FP32) are updated here, one thread per entry.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_nt_edge(T* __restrict__ C, int64_t ldc, const T* __restrict__ A,
                                                      int64_t lda, const T* __restrict__ B, int64_t ldb, int64_t M,
                                                      int64_t N, int64_t K, T alpha, int lower, int64_t gr,
                                                      int64_t gc, int64_t Mp, int64_t Np) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n_rows = (M - Mp) * N;          // rows [Mp, M), every column
  const int64_t n_cols = Mp * (N - Np);         // rows [0, Mp), columns [Np, N)
  if (e >= n_rows + n_cols) return;
  int64_t i, j;
  if (e < n_rows) {
    i = Mp + e / N;
    j = e % N;
  } else {
    i = (e - n_rows) % Mp;
    j = Np + (e - n_rows) / Mp;
  }
  if (lower && gr + i < gc + j) return;
  T acc = 0;
  for (int64_t k = 0; k < K; ++k) acc += A[i + k * lda] * B[j + k * ldb];
  C[i + j * ldc] += alpha * acc;
}

template <typename T>
static void gemm_edge(T* C, int64_t ldc, const T* A, int64_t lda, const T* B, int64_t ldb, int64_t M, int64_t N,
                      int64_t K, T alpha, bool lower, int64_t gr, int64_t gc, int64_t Mp, int64_t Np,
                      hipStream_t st) {
  const int64_t cnt = (M - Mp) * N + Mp * (N - Np);
  if (cnt <= 0) return;
  hipLaunchKernelGGL(k_gemm_nt_edge<T>, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st, C, ldc, A, lda, B, ldb,
                     M, N, K, alpha, lower ? 1 : 0, gr, gc, Mp, Np);
  HC_LAUNCH_CHECK();
}

template <typename T>
void gemm_nt(T* C, int64_t ldc, const T* A, int64_t lda, const T* B, int64_t ldb, int64_t M, int64_t N, int64_t K,
             T alpha, bool lower, int64_t gr, int64_t gc, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  if constexpr (std::is_same<T, double>::value) {
    const int64_t Mp = M & ~int64_t(1), Np = N & ~int64_t(1);   // whole row pairs
    if (dma_ok(A, lda, B, ldb, Mp, Np, K) && Mp >= 4 && ((uintptr_t)C % 16) == 0 && ldc % 2 == 0) {
      const int tm = (int)ceil_div(Mp, DM), tn = (int)ceil_div(Np, DN);
      hipLaunchKernelGGL(k_gemm_nt_dma, dim3(tm * tn), dim3(512), 0, st, C, ldc, A, lda, B, ldb, Mp, Np, K, alpha,
                         lower ? 1 : 0, gr, gc, tn);
      HC_LAUNCH_CHECK();
      gemm_edge<T>(C, ldc, A, lda, B, ldb, M, N, K, alpha, lower, gr, gc, Mp, Np, st);
      return;
    }
  } else {
    const int64_t Mp = M & ~int64_t(3), Np = N & ~int64_t(3);   // whole groups of four rows
    if (dma32_ok(A, lda, B, ldb, Mp, Np, K) && ((uintptr_t)C % 16) == 0 && ldc % 4 == 0) {
      const int tm = (int)ceil_div(Mp, DM), tn = (int)ceil_div(Np, DN);
      hipLaunchKernelGGL(k_gemm_nt_dma32, dim3(tm * tn), dim3(512), 0, st, C, ldc, A, lda, B, ldb, Mp, Np, K, alpha,
                         lower ? 1 : 0, gr, gc, tn);
      HC_LAUNCH_CHECK();
      gemm_edge<T>(C, ldc, A, lda, B, ldb, M, N, K, alpha, lower, gr, gc, Mp, Np, st);
      return;
    }
  }
  const int tm = (int)ceil_div(M, TM), tn = (int)ceil_div(N, TN);
  hipLaunchKernelGGL(k_gemm_nt<T>, dim3(tm * tn), dim3(256), 0, st, C, ldc, A, lda, B, ldb, M, N, K, alpha,
                     lower ? 1 : 0, gr, gc, tn);
  HC_LAUNCH_CHECK();
}

hipEvent_t Prof::next() {
  if (used == ev.size()) {
    hipEvent_t e;
    HC_HIP(hipEventCreate(&e));
    ev.push_back(e);
  }
  return ev[used++];
}

double Prof::collect_ms() {
  double ms = 0;
  for (size_t i = 0; i + 1 < used; i += 2) {
    HC_HIP(hipEventSynchronize(ev[i + 1]));
    float t = 0;
    HC_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
    ms += t;
  }
  used = 0;
  return ms;
}

Prof::~Prof() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

// lower-triangle entries (global row >= global col) of the C block
static double lower_entries(int64_t rc, int64_t cc, int64_t M, int64_t N) {
  double cnt = 0;
  for (int64_t j = cc; j < cc + N; ++j) cnt += (double)std::max<int64_t>(0, rc + M - std::max(rc, j));
  return cnt;
}

// C -= A B' with every operand inside the one column-major matrix S
template <typename T>
static void gemm_nt_sub(T* S, int64_t ld, int64_t rc, int64_t cc, int64_t ra, int64_t rb, int64_t ka, int64_t M,
                        int64_t N, int64_t K, bool lower, hipStream_t st, Prof* prof) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  if (prof) HC_HIP(hipEventRecord(prof->next(), st));
  gemm_nt<T>(S + rc + cc * ld, ld, S + ra + ka * ld, ld, S + rb + ka * ld, ld, M, N, K, T(-1), lower, rc, cc, st);
  if (prof) {
    HC_HIP(hipEventRecord(prof->next(), st));
    prof->flops += 2.0 * (double)K * lower_entries(rc, cc, M, N);
    prof->launches++;
  }
}

void Aux::init() {
  if (!side) HC_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
}

hipEvent_t Aux::next() {
  if (used == ev.size()) {
    hipEvent_t e;
    HC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ev.push_back(e);
  }
  return ev[used++];
}

Aux::~Aux() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  if (side) (void)hipStreamDestroy(side);
}

// rows [0, rows_below(j)) hold every nonzero of columns <= j: the envelope
// rounded up to whole 64-blocks (dense without an envelope)
static int64_t rows_below(const int64_t* last, int64_t n, int64_t j) {
  if (!last) return n;
  return std::min<int64_t>(n, ceil_div(std::max<int64_t>(last[j], j + 1), BS) * BS);
}

// factor the panel [K0, Kend): per 64-block the diagonal factor, the TRSM of
// the rows below (down to the envelope) and the eager update of the rest of
// the panel
template <typename T>
static void factor_panel(T* S, int64_t n, int64_t ld, T* Linv, double tol, double fix, unsigned long long* hits,
                         int64_t K0, int64_t Kend, const int64_t* last, hipStream_t st, Prof* prof) {
  for (int64_t c = K0; c < Kend; c += BS) {
    const int64_t cb = std::min<int64_t>(BS, n - c);
    hipLaunchKernelGGL(k_chol_diag<T>, dim3(1), dim3(256), 0, st, S, ld, c, n, Linv + (c / BS) * BS * BS, tol,
                       fix, hits);
    HC_LAUNCH_CHECK();
    const int64_t r0 = c + cb, R = rows_below(last, n, c + cb - 1);
    if (r0 < R) {
      hipLaunchKernelGGL(k_trsm<T>, dim3((unsigned)ceil_div(R - r0, BS)), dim3(256), 0, st, S, ld, c, r0, R,
                         (const T*)(Linv + (c / BS) * BS * BS));
      HC_LAUNCH_CHECK();
    }
    if (r0 < Kend && r0 < R) {
      // rows [r0, R) of the panel's remaining columns [r0, min(Kend, R)) (not in
      // the profile's MFMA-update figures, which cover the large update kernels)
      const int64_t M = R - r0, N = std::min(Kend, R) - r0;
      hipLaunchKernelGGL(k_gemm_panel<T>, dim3((unsigned)ceil_div(M, BS), (unsigned)ceil_div(N, BS)), dim3(256), 0,
                         st, S + r0 + r0 * ld, ld, (const T*)(S + r0 + c * ld), ld, (const T*)(S + r0 + c * ld), ld,
                         M, N, (int)cb, r0, r0);
      HC_LAUNCH_CHECK();
    }
  }
}

template <typename T>
void dense_cholesky(T* S, int64_t n, int64_t ld, T* Linv, double tol, double fix, unsigned long long* hits,
                    hipStream_t st, Prof* prof, Aux* aux, const int64_t* last) {
  if (n <= 0) return;
  // Look-ahead.  After panel k is factored: U1 updates panel k+1 on `st`, U2
  // updates every later column on `side`.  Panel k+1 is then factored on `st`
  // while U2 runs.  U1 writes the columns that the previous U2 wrote, so it
  // waits for that U2; U2 waits for panel k to be factored.  Both stop at the
  // rows the panel's columns reach (the envelope); a panel whose columns reach
  // no row past the next panel launches no U2.  In serial mode U2 runs on
  // `st` before U1: the same launches, one at a time.
  const bool serial = aux->serial;
  hipStream_t side = st;
  if (!serial) {
    aux->init();
    aux->used = 0;
    side = aux->side;
  }
  const int64_t W = std::max<int64_t>(BS, aux->nb / BS * BS);   // panel width
  if (!serial) {
    hipEvent_t start = aux->next();
    HC_HIP(hipEventRecord(start, st));
    HC_HIP(hipStreamWaitEvent(side, start, 0));
  }
  hipEvent_t u2_done = nullptr;
  for (int64_t K0 = 0; K0 < n; K0 += W) {
    const int64_t Kend = std::min<int64_t>(n, K0 + W);
    factor_panel<T>(S, n, ld, Linv, tol, fix, hits, K0, Kend, last, st, prof);
    if (Kend >= n) break;
    const int64_t K1 = std::min<int64_t>(n, Kend + W);
    const int64_t R = rows_below(last, n, Kend - 1);
    const bool u2 = K1 < R;
    if (u2) {
      if (!serial) {
        hipEvent_t factored = aux->next();
        HC_HIP(hipEventRecord(factored, st));
        HC_HIP(hipStreamWaitEvent(side, factored, 0));
      }
      // U2: rows and columns [K1, R)
      gemm_nt_sub<T>(S, ld, K1, K1, K1, K1, K0, R - K1, R - K1, Kend - K0, true, side, prof);
    }
    if (u2_done) HC_HIP(hipStreamWaitEvent(st, u2_done, 0));
    // U1 on the caller's stream: rows [Kend, R), columns [Kend, min(K1, R))
    if (Kend < R)
      gemm_nt_sub<T>(S, ld, Kend, Kend, Kend, Kend, K0, R - Kend, std::min(K1, R) - Kend, Kend - K0, true, st, prof);
    u2_done = nullptr;
    if (u2 && !serial) {
      u2_done = aux->next();
      HC_HIP(hipEventRecord(u2_done, side));
    }
  }
  if (u2_done) HC_HIP(hipStreamWaitEvent(st, u2_done, 0));
}

// ---------------------------------------------------------------------------
// Inverses of the 256 x 256 diagonal blocks of L (one workgroup per block),
// from the 64 x 64 block inverses:  X_ii = Linv_i,
// X_ij = -Linv_i sum_{k=j}^{i-1} L_ik X_kj  (i > j).  X and X' are stored
// column-major with leading dimension 256 (block b at b * 256 * 256).
// ---------------------------------------------------------------------------
constexpr int SB = 256;   // rows per triangular-solve step
constexpr int MAXRHS = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_inv256(const T* __restrict__ L, int64_t ld, const T* __restrict__ Linv,
                                                int64_t n, T* __restrict__ Xall, T* __restrict__ XTall) {
  __shared__ T Tt[BS][BS + 1];
  const int tid = threadIdx.x;
  const int64_t c = (int64_t)blockIdx.x * SB;
  const int cb = (int)std::min<int64_t>(SB, n - c);
  const int nsub = (cb + BS - 1) / BS;
  T* X = Xall + (int64_t)blockIdx.x * SB * SB;
  T* XT = XTall + (int64_t)blockIdx.x * SB * SB;
  for (int e = tid; e < SB * SB; e += 256) {
    const int i = e % SB, j = e / SB;
    T v = 0;
    if (i / BS == j / BS) {
      if (i / BS < nsub) v = Linv[((c + (i / BS) * BS) / BS) * BS * BS + (i % BS) + (j % BS) * BS];
      else v = (i == j) ? T(1) : T(0);
    }
    X[i + j * SB] = v;
  }
  __syncthreads();
  const int i0 = 4 * (tid % 16), j0 = 4 * (tid / 16);
  for (int jb = 0; jb < nsub; ++jb)
    for (int ib = jb + 1; ib < nsub; ++ib) {
      T acc[4][4] = {};
      for (int kb = jb; kb < ib; ++kb)
        for (int p = 0; p < BS; ++p) {
          T la[4], xb[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const int row = ib * BS + i0 + a;   // local row inside the 256 block
            la[a] = (row < cb && kb * BS + p < cb) ? L[(c + row) + (c + kb * BS + p) * ld] : T(0);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) xb[q] = X[(kb * BS + p) + (jb * BS + j0 + q) * SB];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[a][q] += la[a] * xb[q];
        }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) Tt[i0 + a][j0 + q] = acc[a][q];
      __syncthreads();
      const T* Li = X + (ib * BS) + (ib * BS) * SB;   // Linv_ib sits on X's diagonal
      T out[4][4] = {};
      for (int p = 0; p < BS; ++p) {
        T la[4], tb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) la[a] = Li[(i0 + a) + p * SB];
#pragma unroll
        for (int q = 0; q < 4; ++q) tb[q] = Tt[p][j0 + q];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int q = 0; q < 4; ++q) out[a][q] -= la[a] * tb[q];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) X[(ib * BS + i0 + a) + (jb * BS + j0 + q) * SB] = out[a][q];
      __syncthreads();
    }
  for (int e = tid; e < SB * SB; e += 256) {
    const int i = e % SB, j = e / SB;
    XT[i + j * SB] = X[j + i * SB];
  }
}

int64_t inv256_elems(int64_t n) { return ceil_div(n, SB) * SB * SB; }

template <typename T>
void dense_block_inverses(const T* L, int64_t n, int64_t ld, const T* Linv, T* X, T* XT, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_inv256<T>, dim3((unsigned)ceil_div(n, SB)), dim3(256), 0, st, L, ld, Linv, n, X, XT);
  HC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// triangular solves, nrhs <= 4 right-hand sides stored column-major with
// leading dimension n:  forward Y = L^-1 B (B overwritten), backward
// X = L^-T Y (Y overwritten).  Per 256-row block: one workgroup applies the
// block inverse (a 256 x 256 triangular matvec), then a bandwidth-bound kernel
// updates the rows below (forward) or the columns to the left (backward).
// ---------------------------------------------------------------------------
// Yout[c + i] = sum_k Xinv[i + k * 256] Bin[c + k] for the 256 x 256 block
// inverse Xinv (lower for the forward pass, upper for the backward one).
// 16 workgroups of 16 rows each; thread (row, g) sums k in [16 g, 16 g + 16)
// and the 16 partial sums meet in LDS.  The stored inverse is zero outside
// its triangle and bb is zero past cb, so loads and products need no masks.
constexpr int DIAG_ROWS = 16;
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_trsv_diag(const T* __restrict__ Xinv, int64_t c, int64_t n,
                                                   const T* __restrict__ Bin, T* __restrict__ Yout, int nrhs) {
  __shared__ T bb[SB][NR];
  __shared__ T part[16][DIAG_ROWS][NR];
  const int tid = threadIdx.x;
  const int cb = (int)std::min<int64_t>(SB, n - c);
  const int il = tid % DIAG_ROWS, g = tid / DIAG_ROWS;
  const int i = blockIdx.x * DIAG_ROWS + il;
  // the inverse's entries do not depend on the previous kernel: their loads
  // are issued before the right-hand side's, so the two latencies overlap
  T x[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) x[q] = Xinv[i + (int64_t)(g * 16 + q) * SB];
  for (int e = tid; e < SB * NR; e += 256) {
    const int ie = e % SB, r = e / SB;
    bb[ie][r] = (ie < cb && r < nrhs) ? Bin[(c + ie) + r * n] : T(0);
  }
  __syncthreads();
  T acc[NR] = {};
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = g * 16 + q;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] += x[q] * bb[k][r];
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) part[g][il][r] = acc[r];
  __syncthreads();
  if (tid < DIAG_ROWS * NR) {
    const int row = tid % DIAG_ROWS, r = tid / DIAG_ROWS;
    T v = 0;
#pragma unroll
    for (int gg = 0; gg < 16; ++gg) v += part[gg][row][r];
    const int ig = blockIdx.x * DIAG_ROWS + row;
    if (ig < cb && r < nrhs) Yout[(c + ig) + r * n] = v;
  }
}

// rows below the block: B[row] -= L[row, c:c+cb] y_c.  A workgroup takes 64
// rows; wave w sums columns [16 w, 16 w + 16) with one lane per row (each
// column read is 512 contiguous bytes, 16 loads in flight per lane), and the
// 16 partial sums meet in LDS.
template <typename T, int NR>
__global__ __launch_bounds__(1024) void k_trsv_fwd_update(const T* __restrict__ L, int64_t ld, int64_t c, int64_t n,
                                                          T* __restrict__ B, const T* __restrict__ Y, int nrhs) {
  __shared__ T yb[SB][NR];
  __shared__ T part[16][64][NR];
  const int tid = threadIdx.x;
  const int cb = (int)std::min<int64_t>(SB, n - c);
  const int lane = tid & 63, w = tid >> 6;
  const int64_t row = c + cb + (int64_t)blockIdx.x * 64 + lane;
  const int64_t rowc = std::min<int64_t>(row, n - 1);
  // L's entries do not depend on the previous kernel: loaded before y
  T l[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) l[q] = L[rowc + (c + std::min(w * 16 + q, cb - 1)) * ld];   // yb is zero past cb
  // the entry of B this thread updates at the end (final before this kernel)
  const int64_t rw = c + cb + (int64_t)blockIdx.x * 64 + (tid % 64);
  const int rr = tid / 64;
  const bool writer = tid < 64 * NR && rw < n && rr < nrhs;
  const T bold = writer ? B[rw + rr * n] : T(0);
  for (int e = tid; e < SB * NR; e += 1024) {
    const int i = e % SB, r = e / SB;
    yb[i][r] = (i < cb && r < nrhs) ? Y[(c + i) + r * n] : T(0);
  }
  __syncthreads();
  T acc[NR] = {};
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = w * 16 + q;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] += l[q] * yb[k][r];
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) part[w][lane][r] = acc[r];
  __syncthreads();
  if (tid < 64 * NR) {
    const int ln = tid % 64;
    T v = 0;
#pragma unroll
    for (int ww = 0; ww < 16; ++ww) v += part[ww][ln][rr];
    if (writer) B[rw + rr * n] = bold - v;
  }
}

// columns left of the block: Y[j] -= sum_i L[c + i, j] x[i]; each wave takes
// four columns (16 loads in flight per lane), lanes run over i
constexpr int BWD_COLS = 4;
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_trsv_bwd_update(const T* __restrict__ L, int64_t ld, int64_t c, int64_t n,
                                                         int64_t j_begin, T* __restrict__ Yv, const T* __restrict__ X,
                                                         int nrhs) {
  __shared__ T xb[SB][NR];
  const int tid = threadIdx.x;
  const int cb = (int)std::min<int64_t>(SB, n - c);
  const int lane = tid & 63;
  const int64_t j0 = j_begin + ((int64_t)blockIdx.x * 4 + (tid >> 6)) * BWD_COLS;
  // L's entries do not depend on the previous kernel: loaded before x
  T l[BWD_COLS][SB / 64];
#pragma unroll
  for (int cc = 0; cc < BWD_COLS; ++cc) {
    const int64_t j = std::min<int64_t>(j0 + cc, c - 1);
#pragma unroll
    for (int q = 0; q < SB / 64; ++q) l[cc][q] = L[(c + std::min(lane + 64 * q, cb - 1)) + j * ld];   // xb is zero past cb
  }
  // the entries of Y lane 0 updates at the end (final before this kernel)
  T yold[BWD_COLS][NR] = {};
  if (lane == 0)
#pragma unroll
    for (int cc = 0; cc < BWD_COLS; ++cc)
      if (j0 + cc < c)
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nrhs) yold[cc][r] = Yv[(j0 + cc) + r * n];
  for (int e = tid; e < SB * NR; e += 256) {
    const int i = e % SB, r = e / SB;
    xb[i][r] = (i < cb && r < nrhs) ? X[(c + i) + r * n] : T(0);
  }
  __syncthreads();
  T acc[BWD_COLS][NR] = {};
#pragma unroll
  for (int cc = 0; cc < BWD_COLS; ++cc) {
#pragma unroll
    for (int q = 0; q < SB / 64; ++q) {
      const int i = lane + 64 * q;
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[cc][r] += l[cc][q] * xb[i][r];
    }
  }
#pragma unroll
  for (int cc = 0; cc < BWD_COLS; ++cc)
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T v = acc[cc][r];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      acc[cc][r] = v;
    }
  if (lane == 0)
#pragma unroll
    for (int cc = 0; cc < BWD_COLS; ++cc)
      if (j0 + cc < c)
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nrhs) Yv[(j0 + cc) + r * n] = yold[cc][r] - acc[cc][r];
}

// With an envelope (`last`, see dense_cholesky) the forward updates stop at
// the rows a block's columns reach and the backward updates start at the
// first column its rows reach: entries outside are zero.
template <typename T, int NR>
static void dense_solve_nr(const T* L, int64_t n, int64_t ld, const T* X256, const T* XT256, T* B, T* Y, T* X,
                           int nrhs, const int64_t* last, hipStream_t st) {
  for (int64_t c = 0; c < n; c += SB) {
    const T* Xi = X256 + (c / SB) * SB * SB;
    hipLaunchKernelGGL((k_trsv_diag<T, NR>), dim3(SB / DIAG_ROWS), dim3(256), 0, st, Xi, c, n, (const T*)B, Y, nrhs);
    HC_LAUNCH_CHECK();
    const int64_t cend = std::min<int64_t>(n, c + SB);
    const int64_t below = rows_below(last, n, cend - 1) - cend;
    if (below > 0) {
      hipLaunchKernelGGL((k_trsv_fwd_update<T, NR>), dim3((unsigned)ceil_div(below, 64)), dim3(1024), 0, st, L, ld, c,
                         n, B, (const T*)Y, nrhs);
      HC_LAUNCH_CHECK();
    }
  }
  const int64_t lastb = ((n - 1) / SB) * SB;
  for (int64_t c = lastb; c >= 0; c -= SB) {
    const T* XTi = XT256 + (c / SB) * SB * SB;
    hipLaunchKernelGGL((k_trsv_diag<T, NR>), dim3(SB / DIAG_ROWS), dim3(256), 0, st, XTi, c, n, (const T*)Y, X, nrhs);
    HC_LAUNCH_CHECK();
    // first column with a nonzero in rows >= c (last is non-decreasing)
    int64_t jb = 0;
    if (last) jb = (std::upper_bound(last, last + c, c) - last) / (4 * BWD_COLS) * (4 * BWD_COLS);
    if (c > jb) {
      hipLaunchKernelGGL((k_trsv_bwd_update<T, NR>), dim3((unsigned)ceil_div(c - jb, 4 * BWD_COLS)), dim3(256), 0, st,
                         L, ld, c, n, jb, Y, (const T*)X, nrhs);
      HC_LAUNCH_CHECK();
    }
  }
}

// kernels specialised for one right-hand side (the iteration's case) and for
// up to MAXRHS
template <typename T>
void dense_solve(const T* L, int64_t n, int64_t ld, const T* X256, const T* XT256, T* B, T* Y, T* X, int nrhs,
                 hipStream_t st, const int64_t* last) {
  if (n <= 0) return;
  if (nrhs == 1) dense_solve_nr<T, 1>(L, n, ld, X256, XT256, B, Y, X, nrhs, last, st);
  else if (nrhs == 2) dense_solve_nr<T, 2>(L, n, ld, X256, XT256, B, Y, X, nrhs, last, st);
  else dense_solve_nr<T, MAXRHS>(L, n, ld, X256, XT256, B, Y, X, nrhs, last, st);
}

template void dense_cholesky<double>(double*, int64_t, int64_t, double*, double, double, unsigned long long*,
                                     hipStream_t, Prof*, Aux*, const int64_t*);
template void dense_cholesky<float>(float*, int64_t, int64_t, float*, double, double, unsigned long long*,
                                    hipStream_t, Prof*, Aux*, const int64_t*);
template void gemm_nt<double>(double*, int64_t, const double*, int64_t, const double*, int64_t, int64_t, int64_t,
                              int64_t, double, bool, int64_t, int64_t, hipStream_t);
template void gemm_nt<float>(float*, int64_t, const float*, int64_t, const float*, int64_t, int64_t, int64_t,
                             int64_t, float, bool, int64_t, int64_t, hipStream_t);
template void dense_solve<double>(const double*, int64_t, int64_t, const double*, const double*, double*, double*,
                                  double*, int, hipStream_t, const int64_t*);
template void dense_solve<float>(const float*, int64_t, int64_t, const float*, const float*, float*, float*, float*,
                                 int, hipStream_t, const int64_t*);
template void dense_block_inverses<double>(const double*, int64_t, int64_t, const double*, double*, double*,
                                           hipStream_t);
template void dense_block_inverses<float>(const float*, int64_t, int64_t, const float*, float*, float*, hipStream_t);

int64_t linv_elems(int64_t n) { return ceil_div(n, BS) * BS * BS; }

// factor flops of a dense n x n Cholesky
double cholesky_flops(int64_t n) { return (double)n * n * n / 3.0; }

double envelope_cholesky_flops(int64_t n, const int64_t* last) {
  if (!last) return cholesky_flops(n);
  double f = 0;
  for (int64_t j = 0; j < n; ++j) {
    const double h = (double)(std::max<int64_t>(last[j], j + 1) - j - 1);   // rows below the pivot
    f += h * h + h;
  }
  return f;
}

}  // namespace hc
