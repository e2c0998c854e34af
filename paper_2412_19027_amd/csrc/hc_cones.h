// Cone-layer kernels (gfx950): one lane per small cone, component-major data.
#pragma once
#include <vector>

#include "hc_common.h"

namespace hc {

// Device view of one family segment (see Segment in hc_common.h).
struct SegDev {
  int32_t kind;
  int32_t dim;        // rows per cone
  int32_t k;          // PSD side
  int64_t base;       // first internal row
  int64_t count;      // cones
  double* state;      // state_doubles(kind, dim, k) * count, field-major
  double* mblk;       // mblock_doubles(kind, dim) * count, entry-major
  const double* alpha;  // POW exponents (count) or null
};

// Scaling at (s, z): fills the segment state and writes diag(H) into hdiag
// (m-vector, internal rows).  mu is the global mu; force_dual selects the
// dual scaling for exp/pow.  Exp/pow cones report in branch_any (device int)
// whether any cone took the primal-dual scaling.
void cone_scale(const SegDev& g, const double* s, const double* z, double mu, int force_dual, double* hdiag,
                int* branch_pd_count, hipStream_t st);
// the same over every segment: zero, nonneg and lane-per-cone SOC segments in
// one launch, the others by their own kernels
void cone_scale_all(const std::vector<SegDev>& segs, const double* s, const double* z, double mu, int force_dual,
                    double* hdiag, int* branch_pd_count, hipStream_t st);
// Explicit lower-triangle entries of (H + delta I)^-1 per cone into g.mblk.
// work: cone_mblock_work(g) doubles of device scratch (PSD: the G_i factors)
void cone_mblock(const SegDev& g, double delta, double* work, hipStream_t st);
// over every segment, all but the PSD ones in one launch
void cone_mblock_all(const std::vector<SegDev>& segs, double delta, double* work, hipStream_t st);
int64_t cone_mblock_work(const SegDev& g);
// y[rows] = H x[rows]  (mode 0) or (H + delta I)^-1 x[rows] (mode 1), spectral form.
void cone_apply(const SegDev& g, int mode, double delta, const double* x, double* y, hipStream_t st);
// y[rows] = -ds[rows] - H x[rows]  (direction recovery of Delta s)
void cone_recover_ds(const SegDev& g, const double* dsrhs, const double* dz, double* out, hipStream_t st);
// cone_apply (dsr null) or cone_recover_ds (dsr given, mode 0) over every
// segment: the lane-per-cone families (zero, nonneg, SOC up to SOC_DMAX,
// exp, pow) in one launch, PSD and larger SOC segments by their own kernels
void cone_apply_all(const std::vector<SegDev>& segs, int mode, double delta, const double* x, const double* dsr,
                    double* y, hipStream_t st);
// combined-step d_s (eq. ds-correction-step) from the scaling state
void cone_ds_combined(const SegDev& g, const double* s, const double* z, const double* dsa, const double* dza,
                      double sm, double* ds, hipStream_t st);
// the same over every segment, the lane-per-cone families in one launch
void cone_ds_all(const std::vector<SegDev>& segs, const double* s, const double* z, const double* dsa,
                 const double* dza, double sm, double* ds, hipStream_t st);
// symmetric families: per-block minimum of the exact boundary steps of s and z
// (written to partial[block]); returns number of blocks
int cone_step_sym(const SegDev& g, const double* s, const double* z, const double* ds, const double* dz,
                  double* partial, hipStream_t st);
// the same over every symmetric segment (nonneg rows and lane-per-cone SOCs in
// one launch); returns the number of partials written
int64_t cone_step_sym_all(const std::vector<SegDev>& segs, const double* s, const double* z, const double* ds,
                          const double* dz, double* partial, hipStream_t st);
// exp/pow: per block, bit j of the result (j < ntrial) is set when every cone
// of the block passes the trial alpha_j = a0 * ratio^j: s + a ds in int K and
// z + a dz in int K* and, when check_nbhd, 3 / <z~(s_a), s~(z_a)> >= beta mu(alpha_j)
// with mu(alpha) = (c0 + c1 alpha + c2 alpha^2) / (nu + 1).
int cone_trial_nonsym(const SegDev& g, const double* s, const double* z, const double* ds, const double* dz,
                      double a0, double ratio, int ntrial, int check_nbhd, double beta, double c0, double c1,
                      double c2, double nu1, unsigned long long* partial, hipStream_t st);
// initial point helpers
void cone_unit(const SegDev& g, double* v, hipStream_t st);   // v[rows] = unit point (e)
// per-block max over symmetric cones of -lambda_min(v_cone)
int cone_max_neg_eig(const SegDev& g, const double* v, double* partial, hipStream_t st);
void cone_add_e(const SegDev& g, double a, double* v, hipStream_t st);   // v += a e (symmetric cones)

// largest alpha > 0 with (x + alpha dx)'J(x + alpha dx) >= 0 given
// a = dx'J dx, b = x'J dx, c = x'J x: the smallest positive root of
// a t^2 + 2b t + c (INFINITY when there is none)
__device__ inline double soc_boundary_step(double a, double b, double c) {
  const double B = 2.0 * b;
  double best = INFINITY;
  if (a == 0.0) {
    if (B != 0.0) {
      const double t = -c / B;
      if (t > 0.0) best = t;
    }
    return best;
  }
  const double disc = B * B - 4.0 * a * c;
  if (disc < 0.0) return best;
  const double qq = -0.5 * (B + copysign(sqrt(disc), B));
  if (qq != 0.0) {
    const double r1 = qq / a, r2 = c / qq;
    if (r1 > 0.0) best = fmin(best, r1);
    if (r2 > 0.0) best = fmin(best, r2);
  }
  return best;
}

// second-order cones above SOC_DMAX: one workgroup per cone (hc_soc.hip), a
// grid of at most LS_GRID workgroups striding over the cones
constexpr int LS_GRID = 2048;
inline int lsoc_grid(int64_t count) { return (int)std::min<int64_t>(std::max<int64_t>(count, 1), LS_GRID); }
void lsoc_scale(const SegDev& g, const double* s, const double* z, double* hdiag, hipStream_t st);
// y = H x (mode 0) or (H + delta I)^-1 x (mode 1); with dsr: y = -dsr - H x
void lsoc_apply(const SegDev& g, int mode, double delta, const double* x, const double* dsr, double* y,
                hipStream_t st);
void lsoc_ds(const SegDev& g, const double* dsa, const double* dza, double sm, double* ds, hipStream_t st);
// per workgroup minimum step (or per cone, capped at amax); returns the grid
int lsoc_step(const SegDev& g, const double* s, const double* z, const double* ds, const double* dz, double amax,
              bool per_cone, double* out, hipStream_t st);
int lsoc_max_neg_eig(const SegDev& g, const double* v, double* partial, hipStream_t st);
// p_- = A_c' v_- at Ad[ent_dst[e]] and p_+ = A_c' v_+ at Ad[ent_dst[e] + plus_off]
// for each (cone, column) entry e of the segment
void lsoc_lowrank(const SegDev& g, int64_t nent, const int32_t* ent_cone, const int32_t* ent_col,
                  const int64_t* ent_dst, const Csr& At, int64_t plus_off, double* Ad, hipStream_t st);

constexpr int CONE_BLOCK = 256;
inline int cone_blocks(const SegDev& g) {
  if (g.kind == HC_CONE_PSD) return (int)std::max<int64_t>(1, ceil_div(g.count, CONE_BLOCK));
  if (soc_large(g.kind, g.dim)) return lsoc_grid(g.count);
  int64_t units = (g.kind == HC_CONE_ZERO || g.kind == HC_CONE_NONNEG) ? g.count : g.count;
  return (int)std::max<int64_t>(1, ceil_div(units, CONE_BLOCK));
}

// single-family test entry (AoS <-> internal layout) lives in hc_cones.hip
}  // namespace hc

namespace hc {
// test support: what = 0 -> lambda (nonneg: h = s/z; SOC: lambda; PSD: the k
// values of lambda then zeros; exp/pow: z~ = -grad f*(s)), what = 2 -> exp/pow
// branch (1 = dual scaling).  Output in the segment's layout.
void cone_test_extract(const SegDev& g, const double* s, int what, double* out, hipStream_t st);
// per-cone step (see hc_test_cone_step)
void cone_test_step(const SegDev& g, const double* s, const double* z, const double* ds, const double* dz,
                    double amax, double* out, hipStream_t st);
}  // namespace hc
