// Kernel-level test entry points of the C-ABI: each marshals one cone family
// between the caller's cone-by-cone layout and the solver's internal layout
// and then runs exactly the kernels the solver runs.
#include <cstring>
#include <vector>

#include "hc_cones.h"
#include "hc_dense.h"
#include "hc_symbolic.h"
#include "hc_vec.h"

using namespace hc;

namespace {

thread_local std::string g_test_error;

struct TestSeg {
  SegDev g{};
  int rows = 0;           // rows per cone (caller's view)
  int64_t count = 0;      // caller's cones
  bool cm = false;        // component-major internally
  std::vector<void*> owned;
  ~TestSeg() {
    for (void* p : owned) (void)hipFree(p);
  }
  double* alloc(int64_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<int64_t>(1, n) * sizeof(double)) != hipSuccess)
      throw Error{HC_ERR_OOM, "hipMalloc failed"};
    owned.push_back(p);
    return (double*)p;
  }
  // caller (AoS) -> internal
  double* in(const double* a, hipStream_t st) {
    double* d = alloc(count * rows);
    if (cm) aos_to_cm(count, rows, a, d, false, st);
    else HC_HIP(hipMemcpyAsync(d, a, count * rows * sizeof(double), hipMemcpyDeviceToDevice, st));
    return d;
  }
  void out(const double* d, double* a, hipStream_t st) {
    if (cm) aos_to_cm(count, rows, d, a, true, st);
    else HC_HIP(hipMemcpyAsync(a, d, count * rows * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
};

void make(TestSeg& T, int32_t type, int64_t count, int32_t dim, const double* alpha) {
  if (count <= 0) throw Error{HC_ERR_INVALID_ARG, "count must be positive"};
  T.count = count;
  T.g.kind = type;
  switch (type) {
    case HC_CONE_ZERO:
    case HC_CONE_NONNEG:
      T.rows = dim;
      T.g.dim = 1;
      T.g.count = count * dim;
      T.cm = false;
      break;
    case HC_CONE_SOC:
      if (dim < 2 || dim > (1 << 24)) throw Error{HC_ERR_UNSUPPORTED, "SOC dim outside [2, 2^24]"};
      T.rows = dim; T.g.dim = dim; T.g.count = count; T.cm = true;
      break;
    case HC_CONE_EXP:
    case HC_CONE_POW:
      if (dim != 3) throw Error{HC_ERR_CONE, "EXP/POW dim != 3"};
      if (type == HC_CONE_POW && !alpha) throw Error{HC_ERR_INVALID_ARG, "alpha is NULL"};
      T.rows = 3; T.g.dim = 3; T.g.count = count; T.cm = true;
      break;
    case HC_CONE_PSD:
      if (dim < 1 || dim > 32) throw Error{HC_ERR_CONE, "PSD side outside [1, 32]"};
      T.rows = dim * (dim + 1) / 2; T.g.dim = T.rows; T.g.k = dim; T.g.count = count; T.cm = false;
      break;
    default:
      throw Error{HC_ERR_CONE, "unknown cone type"};
  }
  T.g.base = 0;
  T.g.state = T.alloc(state_doubles(type, T.g.dim, T.g.k) * T.g.count);
  T.g.mblk = T.alloc(mblock_doubles(type, T.g.dim) * T.g.count);
  T.g.alpha = alpha;
}

template <typename F> int32_t guard(F&& f) {
  try {
    f();
  } catch (const Error& e) {
    g_test_error = e.msg;
    return e.code;
  }
  return HC_OK;
}

}  // namespace

// plain streaming copy, 16 bytes per lane per step (reference kernel for
// the HBM byte counters)
__global__ __launch_bounds__(256) void k_copy_reference(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                        int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

extern "C" {

int32_t hc_test_cone_scale(int32_t type, int64_t count, int32_t dim, const double* alpha, const double* s,
                           const double* z, double mu, int32_t force_dual, double* H_out, double* lam_out,
                           int32_t* branch_out, void* stream) {
  return guard([&] {
    hipStream_t st = (hipStream_t)stream;
    TestSeg T;
    make(T, type, count, dim, alpha);
    const int64_t tot = count * T.rows;
    double* si = T.in(s, st);
    double* zi = T.in(z, st);
    double* hd = T.alloc(tot);
    int* pd = (int*)T.alloc(1);
    HC_HIP(hipMemsetAsync(pd, 0, sizeof(double), st));
    cone_scale_all(std::vector<SegDev>{T.g}, si, zi, mu, force_dual ? 1 : 0, hd, pd, st);
    // H column by column: H e_j
    double* e = T.alloc(tot);
    double* y = T.alloc(tot);
    std::vector<double> he(tot), hy(tot), hH((size_t)count * T.rows * T.rows);
    for (int j = 0; j < T.rows; ++j) {
      for (int64_t c = 0; c < count; ++c)
        for (int i = 0; i < T.rows; ++i) he[c * T.rows + i] = (i == j) ? 1.0 : 0.0;
      double* ea = T.alloc(tot);
      HC_HIP(hipMemcpyAsync(ea, he.data(), tot * 8, hipMemcpyHostToDevice, st));
      double* ei = T.in(ea, st);
      cone_apply_all(std::vector<SegDev>{T.g}, 0, 0.0, ei, nullptr, y, st);
      double* ya = T.alloc(tot);
      T.out(y, ya, st);
      HC_HIP(hipMemcpyAsync(hy.data(), ya, tot * 8, hipMemcpyDeviceToHost, st));
      HC_HIP(hipStreamSynchronize(st));
      for (int64_t c = 0; c < count; ++c)
        for (int i = 0; i < T.rows; ++i) hH[(c * T.rows + i) * T.rows + j] = hy[c * T.rows + i];
    }
    (void)e;
    if (H_out) HC_HIP(hipMemcpyAsync(H_out, hH.data(), hH.size() * 8, hipMemcpyHostToDevice, st));
    if (lam_out) {
      double* li = T.alloc(tot);
      HC_HIP(hipMemsetAsync(li, 0, tot * 8, st));
      cone_test_extract(T.g, si, 0, li, st);
      T.out(li, lam_out, st);
    }
    if (branch_out) {
      double* bi = T.alloc(T.g.count);
      cone_test_extract(T.g, si, 2, bi, st);
      std::vector<double> hb(T.g.count);
      HC_HIP(hipMemcpyAsync(hb.data(), bi, T.g.count * 8, hipMemcpyDeviceToHost, st));
      HC_HIP(hipStreamSynchronize(st));
      std::vector<int32_t> ib(count);
      for (int64_t c = 0; c < count; ++c) ib[c] = (type == HC_CONE_EXP || type == HC_CONE_POW) ? (int32_t)hb[c] : 0;
      HC_HIP(hipMemcpyAsync(branch_out, ib.data(), count * 4, hipMemcpyHostToDevice, st));
    }
    HC_HIP(hipStreamSynchronize(st));
  });
}

int32_t hc_test_cone_mblock(int32_t type, int64_t count, int32_t dim, const double* alpha, const double* s,
                            const double* z, double mu, int32_t force_dual, double delta, double* M_out,
                            void* stream) {
  return guard([&] {
    if (!M_out || !(delta > 0.0)) throw Error{HC_ERR_INVALID_ARG, "M_out is NULL or delta <= 0"};
    hipStream_t st = (hipStream_t)stream;
    TestSeg T;
    make(T, type, count, dim, alpha);
    const int64_t tot = count * T.rows;
    double* si = T.in(s, st);
    double* zi = T.in(z, st);
    double* hd = T.alloc(tot);
    int* pd = (int*)T.alloc(1);
    HC_HIP(hipMemsetAsync(pd, 0, sizeof(double), st));
    cone_scale_all(std::vector<SegDev>{T.g}, si, zi, mu, force_dual ? 1 : 0, hd, pd, st);
    cone_mblock_all(std::vector<SegDev>{T.g}, delta, T.alloc(std::max<int64_t>(1, cone_mblock_work(T.g))), st);
    const int64_t per = mblock_doubles(type, T.g.dim);
    std::vector<double> hm(per * T.g.count), dense((size_t)count * T.rows * T.rows, 0.0);
    HC_HIP(hipMemcpyAsync(hm.data(), T.g.mblk, hm.size() * 8, hipMemcpyDeviceToHost, st));
    HC_HIP(hipStreamSynchronize(st));
    const int64_t N = T.g.count;
    std::vector<double> hs;
    if (soc_large(type, T.g.dim)) {   // the stored form: f_o I + (f_+ - f_o) v_+v_+' + (f_- - f_o) v_-v_-'
      hs.resize(state_doubles(type, T.g.dim, 0) * N);
      HC_HIP(hipMemcpyAsync(hs.data(), T.g.state, hs.size() * 8, hipMemcpyDeviceToHost, st));
      HC_HIP(hipStreamSynchronize(st));
    }
    for (int64_t c = 0; c < count; ++c) {
      double* D = dense.data() + (size_t)c * T.rows * T.rows;
      if (!hs.empty()) {
        const int d = T.rows;
        const double r = hs[(2 * (int64_t)d + 1) * N + c];
        std::vector<double> vp(d), vm(d);
        const double is2 = 0.70710678118654752440;
        vp[0] = vm[0] = is2;
        for (int j = 1; j < d; ++j) {
          const double u = r > 0.0 ? hs[(int64_t)j * N + c] / r : (j == 1 ? 1.0 : 0.0);
          vp[j] = is2 * u;
          vm[j] = -is2 * u;
        }
        const double fo = hm[c], cp = hm[N + c], cmn = hm[2 * N + c];
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b)
            D[a * d + b] = (a == b ? fo : 0.0) + cp * vp[a] * vp[b] + cmn * vm[a] * vm[b];
        continue;
      }
      if (type == HC_CONE_ZERO || type == HC_CONE_NONNEG) {
        for (int i = 0; i < T.rows; ++i) D[i * T.rows + i] = hm[c * T.rows + i];
        continue;
      }
      for (int a = 0; a < T.rows; ++a)
        for (int b = 0; b <= a; ++b) {
          const double v = hm[((int64_t)a * (a + 1) / 2 + b) * N + c];
          D[a * T.rows + b] = v;
          D[b * T.rows + a] = v;
        }
    }
    HC_HIP(hipMemcpyAsync(M_out, dense.data(), dense.size() * 8, hipMemcpyHostToDevice, st));
    HC_HIP(hipStreamSynchronize(st));
  });
}

int32_t hc_test_cone_ds(int32_t type, int64_t count, int32_t dim, const double* alpha, const double* s,
                        const double* z, const double* dsa, const double* dza, double mu, int32_t force_dual,
                        double sm, double* ds_out, void* stream) {
  return guard([&] {
    hipStream_t st = (hipStream_t)stream;
    TestSeg T;
    make(T, type, count, dim, alpha);
    const int64_t tot = count * T.rows;
    double* si = T.in(s, st);
    double* zi = T.in(z, st);
    double* ai = T.in(dsa, st);
    double* bi = T.in(dza, st);
    double* hd = T.alloc(tot);
    int* pd = (int*)T.alloc(1);
    HC_HIP(hipMemsetAsync(pd, 0, sizeof(double), st));
    cone_scale_all(std::vector<SegDev>{T.g}, si, zi, mu, force_dual ? 1 : 0, hd, pd, st);
    double* o = T.alloc(tot);
    cone_ds_all(std::vector<SegDev>{T.g}, si, zi, ai, bi, sm, o, st);
    T.out(o, ds_out, st);
    HC_HIP(hipStreamSynchronize(st));
  });
}

int32_t hc_test_cone_step(int32_t type, int64_t count, int32_t dim, const double* alpha, const double* s,
                          const double* z, const double* ds, const double* dz, double amax, double* alpha_out,
                          void* stream) {
  return guard([&] {
    hipStream_t st = (hipStream_t)stream;
    TestSeg T;
    make(T, type, count, dim, alpha);
    double* si = T.in(s, st);
    double* zi = T.in(z, st);
    double* a = T.in(ds, st);
    double* b = T.in(dz, st);
    double* o = T.alloc(T.g.count);
    cone_test_step(T.g, si, zi, a, b, amax, o, st);
    if (type == HC_CONE_ZERO || type == HC_CONE_NONNEG) {
      // per caller cone: minimum over its rows
      std::vector<double> h(T.g.count), r(count);
      HC_HIP(hipMemcpyAsync(h.data(), o, T.g.count * 8, hipMemcpyDeviceToHost, st));
      HC_HIP(hipStreamSynchronize(st));
      for (int64_t c = 0; c < count; ++c) {
        double v = amax;
        for (int i = 0; i < T.rows; ++i) v = std::min(v, h[c * T.rows + i]);
        r[c] = v;
      }
      HC_HIP(hipMemcpyAsync(alpha_out, r.data(), count * 8, hipMemcpyHostToDevice, st));
    } else {
      HC_HIP(hipMemcpyAsync(alpha_out, o, count * 8, hipMemcpyDeviceToDevice, st));
    }
    HC_HIP(hipStreamSynchronize(st));
  });
}

int32_t hc_test_cone_step_min(int32_t type, int64_t count, int32_t dim, const double* alpha, const double* s,
                              const double* z, const double* ds, const double* dz, double* alpha_min, void* stream) {
  return guard([&] {
    if (!alpha_min) throw Error{HC_ERR_INVALID_ARG, "alpha_min is NULL"};
    if (type != HC_CONE_NONNEG && type != HC_CONE_SOC && type != HC_CONE_PSD)
      throw Error{HC_ERR_INVALID_ARG, "the minimum step is for nonneg, SOC and PSD cones"};
    hipStream_t st = (hipStream_t)stream;
    TestSeg T;
    make(T, type, count, dim, alpha);
    double* si = T.in(s, st);
    double* zi = T.in(z, st);
    double* a = T.in(ds, st);
    double* b = T.in(dz, st);
    // as many partials as the solver's launch may write (one per workgroup)
    double* part = T.alloc(std::max<int64_t>(2 * T.g.count, cone_blocks(T.g)) + 64);
    const int nb = (int)cone_step_sym_all(std::vector<SegDev>{T.g}, si, zi, a, b, part, st);
    std::vector<double> h(std::max(nb, 1));
    if (nb) HC_HIP(hipMemcpyAsync(h.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    HC_HIP(hipStreamSynchronize(st));
    double v = INFINITY;
    for (int i = 0; i < nb; ++i) v = std::min(v, h[i]);
    *alpha_min = v;
  });
}

int32_t hc_test_dense_chol_solve(int32_t precision, int64_t n, int64_t ld, double* A, int32_t nrhs, double* B,
                                 int64_t* guard_hits, void* stream) {
  return hc_test_dense_chol_solve_env(precision, n, ld, A, nullptr, nrhs, B, guard_hits, stream);
}

int32_t hc_test_dense_chol_solve_env(int32_t precision, int64_t n, int64_t ld, double* A, const int64_t* last,
                                     int32_t nrhs, double* B, int64_t* guard_hits, void* stream) {
  return guard([&] {
    if (n <= 0 || ld < n || nrhs < 1 || nrhs > 4 || !A || !B) throw Error{HC_ERR_INVALID_ARG, "bad dense test args"};
    if (last)
      for (int64_t j = 0; j < n; ++j)
        if (last[j] <= j || last[j] > n || (j > 0 && last[j] < last[j - 1]))
          throw Error{HC_ERR_INVALID_ARG, "envelope must satisfy j < last[j] <= n and be non-decreasing"};
    hipStream_t st = (hipStream_t)stream;
    std::vector<void*> owned;
    Aux aux;
    auto al = [&](size_t bytes) {
      void* p = nullptr;
      if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) throw Error{HC_ERR_OOM, "hipMalloc failed"};
      owned.push_back(p);
      return p;
    };
    unsigned long long* hits = (unsigned long long*)al(8);
    HC_HIP(hipMemsetAsync(hits, 0, 8, st));
    try {
      if (precision == HC_PRECISION_MIXED) {
        float* A32 = (float*)al((size_t)ld * n * 4);
        float* L32 = (float*)al(linv_elems(n) * 4);
        float* b32 = (float*)al((size_t)n * nrhs * 4);
        float* y32 = (float*)al((size_t)n * nrhs * 4);
        float* x32 = (float*)al((size_t)n * nrhs * 4);
        lower_to_f32(n, ld, A, A32, st);
        dense_cholesky<float>(A32, n, ld, L32, 0.0, 1e-8, hits, st, nullptr, &aux, last);
        float* X32 = (float*)al(inv256_elems(n) * 4);
        float* XT32 = (float*)al(inv256_elems(n) * 4);
        dense_block_inverses<float>(A32, n, ld, L32, X32, XT32, st);
        double* one = (double*)al(8);
        const double h1 = 1.0;
        HC_HIP(hipMemcpyAsync(one, &h1, 8, hipMemcpyHostToDevice, st));
        to_f32((int64_t)n * nrhs, B, one, b32, st);
        dense_solve<float>(A32, n, ld, X32, XT32, b32, y32, x32, nrhs, st, last);
        from_f32((int64_t)n * nrhs, x32, one, B, st);
      } else {
        double* Li = (double*)al(linv_elems(n) * 8);
        double* y = (double*)al((size_t)n * nrhs * 8);
        double* x = (double*)al((size_t)n * nrhs * 8);
        dense_cholesky<double>(A, n, ld, Li, 0.0, 1e-8, hits, st, nullptr, &aux, last);
        double* X64 = (double*)al(inv256_elems(n) * 8);
        double* XT64 = (double*)al(inv256_elems(n) * 8);
        dense_block_inverses<double>(A, n, ld, Li, X64, XT64, st);
        dense_solve<double>(A, n, ld, X64, XT64, B, y, x, nrhs, st, last);
        HC_HIP(hipMemcpyAsync(B, x, (size_t)n * nrhs * 8, hipMemcpyDeviceToDevice, st));
      }
      unsigned long long h = 0;
      HC_HIP(hipMemcpyAsync(&h, hits, 8, hipMemcpyDeviceToHost, st));
      HC_HIP(hipStreamSynchronize(st));
      if (guard_hits) *guard_hits = (int64_t)h;
    } catch (...) {
      for (void* p : owned) (void)hipFree(p);
      throw;
    }
    for (void* p : owned) (void)hipFree(p);
  });
}

int32_t hc_test_copy(const void* src, void* dst, int64_t bytes, void* stream) {
  return guard([&] {
    if (!src || !dst || bytes < 0 || bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16)
      throw Error{HC_ERR_INVALID_ARG, "copy needs 16-byte aligned pointers and a multiple of 16 bytes"};
    if (bytes == 0) return;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n16 = bytes / 16;
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(n16, 256), 8192);
    hipLaunchKernelGGL(k_copy_reference, dim3(grid), dim3(256), 0, st, (const uint4*)src, (uint4*)dst, n16);
    HC_LAUNCH_CHECK();
    HC_HIP(hipStreamSynchronize(st));
  });
}

}  // extern "C"

// symbolic analysis of a caller's graph (host only)
int32_t hc_test_symbolic(int32_t n, const int64_t* ptr, const int32_t* adj, int32_t* order, int32_t* parent,
                         int64_t* count, int32_t* sn_first, int32_t* sn_parent, int32_t* sn_level, int32_t* nsuper,
                         int32_t* nlevels) {
  if (n < 0 || !ptr || (n > 0 && (!adj || !order || !parent || !count || !sn_first || !sn_parent || !sn_level)) ||
      !nsuper || !nlevels)
    return HC_ERR_INVALID_ARG;
  SymGraph g;
  g.n = n;
  g.ptr.assign(ptr, ptr + n + 1);
  if (g.ptr[0] != 0) return HC_ERR_CSR;
  for (int32_t i = 0; i < n; ++i)
    if (g.ptr[i + 1] < g.ptr[i]) return HC_ERR_CSR;
  g.adj.assign(adj, adj + g.ptr[n]);
  for (int32_t v : g.adj)
    if (v < 0 || v >= n) return HC_ERR_CSR;
  const SymbolicPlan P = symbolic_analysis(g);
  std::copy(P.order.begin(), P.order.end(), order);
  std::copy(P.parent.begin(), P.parent.end(), parent);
  std::copy(P.count.begin(), P.count.end(), count);
  const int32_t ns = (int32_t)P.sn.parent.size();
  std::copy(P.sn.first.begin(), P.sn.first.end(), sn_first);
  std::copy(P.sn.parent.begin(), P.sn.parent.end(), sn_parent);
  std::copy(P.sn.level.begin(), P.sn.level.end(), sn_level);
  *nsuper = ns;
  *nlevels = P.sn.nlevels;
  return HC_OK;
}
