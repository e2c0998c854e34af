// Wave-per-problem engine: many small symmetric-cone problems (zero,
// nonnegative and second-order cones of at most SOC_DMAX rows) advance
// together, one 64-lane wavefront per problem and one kernel launch per
// interior-point iteration of every problem in flight (the served form's
// batched tick).  Each wave runs the whole loop body of Algorithm 1 for its
// problem: residuals and termination tests, Nesterov-Todd scalings, the
// Schur complement S = P + delta I + A'MA (eq. linsys_2x2 with the cone rows
// eliminated first) assembled into band storage, its band Cholesky with the
// active window in LDS, refined solves against the unregularised K, the
// direction, the step length and the update, in the arithmetic of the
// per-family kernels (the same Nesterov-Todd formulas, hc_soc_math.h).  The
// columns are renumbered at set-up by a reverse Cuthill-McKee ordering of the
// graph of S, so that S is banded with half-width w; a problem is eligible
// when w <= WAVE_WMAX.
#pragma once
#include <string>
#include <vector>

#include "hc_common.h"
#include "hipcone.h"

struct hc_solver;

namespace hc {

constexpr int WAVE_WB = 64;          // LDS window rows (circular)
constexpr int WAVE_PB = 8;           // rows fetched ahead per block of steps
constexpr int WAVE_WMAX = WAVE_WB - WAVE_PB;

// host image of one problem for the engine (columns in band order, rows:
// zero, then nonnegative, then the second-order cones one after another)
struct WavePlan {
  int32_t n = 0, m = 0, w = 0;           // w: band half-width of S
  int32_t nz = 0, nn = 0, nsoc = 0;      // zero rows, nonneg rows, second-order cones
  std::vector<int32_t> soc_off;          // nsoc + 1 row offsets (from nz + nn)
  std::vector<int32_t> soc_moff;         // offset of each cone's d x d M block
  int32_t mtot = 0;                      // M entries: one per zero/nonneg row + sum d^2
  std::vector<int32_t> Arp, Aci, Atrp, Atci, Prp, Pci;
  std::vector<double> Av, Atv, Pv, q, b, D, E;
  std::vector<double> Pband;             // P in band storage (n x (w + 1), column-major)
  std::vector<double> Zband;             // sum over zero rows of A_r'A_r (their M is 1/delta), same storage
  std::vector<int32_t> te, trp, tm;      // A'MA terms of the nonneg rows and cones: the band entries
  std::vector<double> tc;                // that have any (te), per such entry its terms (trp),
                                         // each a coefficient A_a A_b times M[tm]
  std::vector<int32_t> colperm;          // band column -> user column
  std::vector<int32_t> rowperm;          // engine row -> user row
  double cscale = 1, bnorm = 0, qnorm = 0, maxPdiag = 0;
  int64_t nu = 0;
  hc_settings st{};
  bool mixed = false;
  size_t blob_bytes() const;             // device bytes of one slot (data + work)
};

// eligibility and plan from a set-up handle; false with the reason otherwise
bool wave_plan(const hc_solver* S, WavePlan* out, std::string* why);
// the message hc_last_error(NULL) returns on this thread
void set_last_error(const std::string& msg);

// device view of one slot (pointers into its blob)
struct WaveDesc {
  int32_t n, m, w, W, nz, nn, nsoc, mtot;
  int32_t ir_max, max_iter, mixed, nte;   // nte: band entries with nonneg/cone terms
  double cscale, bnorm, qnorm, maxPdiag, nu1;
  double eps_feas, eps_inf, static_reg, dyn_reg, ir_abstol, ir_reltol, step_fraction, ir_mu_frac;
  const int32_t *Arp, *Aci, *Atrp, *Atci, *Prp, *Pci, *te, *trp, *tm, *soc_off, *soc_moff, *colperm, *rowperm;
  const double *Av, *Atv, *Pv, *q, *b, *D, *E, *Pband, *Zband, *tc;
  double* v;                      // WV_COUNT work vectors of max(n, m) doubles
  double *Sb, *dinv, *hst, *hdiag, *Mv, *sc;
  float *Sb32, *dinv32, *f32;     // mixed precision only
  double *xo, *so, *zo;           // the result in the user's coordinates
};

// per-slot scalars (WaveDesc::sc)
enum WaveScalar {
  SC_TAU = 0, SC_KAPPA, SC_PHASE, SC_K, SC_ITERS, SC_STATUS, SC_SDMAX, SC_HITS, SC_FALLBACKS, SC_IRS,
  SC_OBJP, SC_OBJD, SC_RESP, SC_RESD, SC_GAP, SC_MU, SC_XPX, SC_FACTS, SC_COUNT = 32
};
enum WavePhase { PH_NEW = 0, PH_RUN = 1, PH_DONE = 2 };

// lays the slot out in `blob` (device memory of plan.blob_bytes()), uploads
// the plan's data on `st` and fills `desc` (host copy of the descriptor)
void wave_upload(const WavePlan& plan, void* blob, WaveDesc* desc, hipStream_t st);
// interior-point iterations (the first starting from the initial point) of
// every active slot: descs[i] for i < nslots with active[i] != 0.  Each slot
// runs at least one iteration and then more while the next one is expected to
// end within *budget (device scalar, 10 ns clock ticks from the launch);
// status[i] receives the slot's phase after the tick (PH_DONE when its solve
// has ended)
void wave_tick(const WaveDesc* descs, const int32_t* active, int nslots, int32_t* status, const int64_t* budget,
               hipStream_t st);
// result of a finished slot (reads its scalars; host copies)
void wave_result(const WaveDesc& desc, const WavePlan& plan, hc_info* info, double* x, double* s, double* z,
                 hipStream_t st);

}  // namespace hc
