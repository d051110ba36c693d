// Host engine behind the C ABI of include/pou.h.
//
// Owns the device workspace of one system and drives the inner loop of
// Algorithm M (section 3.3, n_org = 1): per step the search direction
// z_i = H w_i - sigma_ii w_i (section 3.2) is never stored; the trial point
// W - tau Z is formed by one elementwise kernel, orthonormalised by Cholesky QR
// through the Gram matrix (section 3.2), its energy (eq. "energy") evaluated,
// and the non-monotone Armijo test of eq. "ene-de" decides on the host.  On
// acceptance one kernel writes the new iterate into the caller's block and
// forms the per-orbital dot products that the next Barzilai-Borwein step
// needs, so no copy of the previous iterate is kept.
#include "pou_internal.h"
#include "../../include/pou.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

using pou::i64;

namespace {

struct Report {
  // device layout of one evaluation report:
  // [sigma N | kin N | e4 | orth info 2*kMaxPass | Poisson rr, bb | E_nl]
  // e4 = (sum rho^(4/3), sum rho V_ext, sum rho V_H, sum rho eps_c) * h^3,
  // E_nl = sum_i f_i <u_i, V_nloc u_i> (zero without projectors)
  static constexpr int kMaxPass = 4;
  static int orth(int N) { return 2 * N + 4; }
  static int size(int N) { return 2 * N + 4 + 2 * kMaxPass + 3; }
  static int rr(int N) { return 2 * N + 4 + 2 * kMaxPass; }
  static int nl(int N) { return rr(N) + 2; }
};

// Every admitted grid (9 <= n <= 1024) gets at least one FFT line per
// workgroup within the LDS cap of the Hartree solve.
constexpr bool fft_fits_all_grids() {
  for (int n = 9; n <= 1024; ++n)
    if (pou::fft_lines_per_group(n) < 1 || pou::fft_lds_bytes(n, pou::fft_lines_per_group(n)) >
                                                pou::kFftLdsMax)
      return false;
  return true;
}
static_assert(fft_fits_all_grids(), "FFT line batch does not fit the LDS cap for some n");

double lambda1(int n, double h, int k) {
  // eigenvalue of -D2 (periodic 8th-order) on Fourier mode k: -(c0 + 2 sum c_m cos m theta)/h^2
  const double c[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
  const double th = 2.0 * M_PI * (double)k / (double)n;
  double s = c[0];
  for (int m = 1; m <= 4; ++m) s += 2.0 * c[m] * std::cos(m * th);
  return -s / (h * h);
}

}  // namespace

struct pou_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool have_system = false;

  // system
  int n = 0;
  double L = 0, h = 0, dv = 0;
  i64 ng = 0;
  int N = 0;
  int M = 0;
  pou_precision prec = POU_FP64;
  pou_params p{};
  std::vector<double> occ, atoms;  // atoms: [M][5]
  size_t es = 8;                   // element size of blocks

  // launch shapes
  pou::StencilArgs st{};
  int nblk_field = 0;   // blocks of field reductions
  int nblk_orb = 0;     // blocks per orbital for block reductions
  int nblk_commit = 0;  // blocks per orbital of the accept kernel
  int nsplit = 0;       // Gram K splits

  // device buffers
  double *d_occ = nullptr, *d_atoms = nullptr;
  double *d_rho = nullptr, *d_vh = nullptr, *d_vext = nullptr, *d_veff = nullptr;
  float *d_veff32 = nullptr;
  double *d_rhoion = nullptr, *d_lam1 = nullptr;
  double *d_cg_r = nullptr, *d_cg_p = nullptr, *d_cg_q = nullptr, *d_cg_z = nullptr;
  double2 *d_fft0 = nullptr, *d_fft1 = nullptr;
  double *d_sc = nullptr;      // CG scalars
  double *d_part = nullptr;    // generic partial sums
  size_t part_len = 0;
  double *d_gpart = nullptr;   // Gram partials
  double *d_G = nullptr, *d_Minv = nullptr, *d_Minv2 = nullptr, *d_Mcomb = nullptr;
  double *d_D64 = nullptr;
  float *d_D32 = nullptr;
  void *d_fsplit = nullptr;  // BF16 pieces of the factor (FP32 orbitals, N > 128)
  double *d_rhopart = nullptr;  // per-128-row-block density shares (N > 128)
  double *d_cholws = nullptr;  // blocked Cholesky tiles when N > 128
  double *d_red = nullptr;     // small reduction outputs
  double *d_S = nullptr, *d_P = nullptr, *d_xpart = nullptr;  // subspace rotation / residual
  double *d_scal = nullptr;    // (tau_BB, zz, ss, sy, yy) of the current step
  // nonlocal projectors (section 2.1 V_nloc), set by pou_set_projectors
  bool nl_on = false;
  int nl_bmax = 0;
  std::vector<pou::NlIon> nl_ions;
  std::vector<int> nl_col_off, nl_col_cnt;  // colours: ranges of d_nl_list
  pou::NlIon *d_nl = nullptr;
  int *d_nl_list = nullptr;
  double *d_nlpart = nullptr;  // overlap partials [M][splits][N][12]
  double *d_nlC = nullptr;     // <xi_l, u_i> of the last evaluation [4M][N]
  double *d_nlC2 = nullptr;    // the same for pou_hamiltonian_apply
  double *d_nlD = nullptr;     // derivative overlaps [M][12][N] (forces)
  std::vector<void *> nl_allocs;
  double *d_diag = nullptr;    // step size of a pou_trial_point call
  double *d_rep[2] = {nullptr, nullptr};  // evaluation reports (current, trial)
  void *d_HW = nullptr, *d_HWt = nullptr, *d_Wt = nullptr, *d_W1 = nullptr, *d_W2 = nullptr;
  std::vector<void *> allocs;

  // iteration state
  const void *last_U = nullptr;  // block the step cache belongs to
  bool cur_valid = false;        // d_HW / d_rep[0] hold H W, sigma of last_U
  bool hist = false;             // BB history available
  int l = 0;
  double E = 0, C = 0, Q = 1;
  double zz_next = 0, ss = 0, sy = 0, yy = 0;
  // last evaluation (pou_energy / step) for backward and diagnostics
  const void *eval_ptr = nullptr;
  void *eval_HU = nullptr;
  int last_cg_iters = 0;
  std::vector<double> rep_host;
  double *h_step = nullptr;  // pinned: trial report | step scalars (8) | accept flags (2)

  // event timing
  unsigned prof_mask = 0;  // kernel groups timed (bit k for group k)
  double prof_ms[POU_K_COUNT] = {};
  long long prof_n[POU_K_COUNT] = {};
  struct Pending { int tag; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  int cur_tag = -1;
  hipEvent_t cur_a = nullptr;
};

namespace {

pou_status fail(pou_ctx *c, pou_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, expr)                                                             \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, POU_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// launch with optional event timing of its kernel group
#define KL(tag, expr)                                                                 \
  do {                                                                                \
    prof_begin(c, tag);                                                               \
    hipError_t e_ = (expr);                                                           \
    prof_end(c);                                                                      \
    if (e_ != hipSuccess)                                                             \
      return fail(c, POU_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

void prof_begin(pou_ctx *c, int tag);
void prof_end(pou_ctx *c);
void prof_drain(pou_ctx *c);
void prof_discard_last(pou_ctx *c, int tag);

template <typename P>
pou_status dalloc(pou_ctx *c, P **ptr, size_t bytes) {
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes ? bytes : 8);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, POU_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  c->allocs.push_back(p);
  *ptr = (P *)p;
  return POU_OK;
}

void free_all(pou_ctx *c) {
  for (void *p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  if (c->h_step) (void)hipHostFree(c->h_step);
  c->h_step = nullptr;
  c->d_occ = c->d_atoms = c->d_rho = c->d_vh = c->d_vext = c->d_veff = nullptr;
  c->d_veff32 = nullptr;
  c->d_rhoion = c->d_lam1 = nullptr;
  c->d_cg_r = c->d_cg_p = c->d_cg_q = c->d_cg_z = nullptr;
  c->d_fft0 = c->d_fft1 = nullptr;
  c->d_sc = c->d_part = c->d_gpart = c->d_G = c->d_Minv = c->d_Minv2 = c->d_Mcomb = nullptr;
  c->d_red = nullptr;
  c->d_S = c->d_P = c->d_xpart = nullptr;
  c->d_scal = nullptr;
  c->d_diag = nullptr;
  for (void *p : c->nl_allocs) (void)hipFree(p);
  c->nl_allocs.clear();
  c->nl_on = false;
  c->nl_ions.clear();
  c->d_nl = nullptr;
  c->d_nl_list = nullptr;
  c->d_nlpart = c->d_nlC = c->d_nlC2 = c->d_nlD = nullptr;
  c->d_D64 = nullptr;
  c->d_D32 = nullptr;
  c->d_fsplit = nullptr;
  c->d_rhopart = nullptr;
  c->d_cholws = nullptr;
  c->d_rep[0] = c->d_rep[1] = nullptr;
  c->d_HW = c->d_HWt = c->d_Wt = c->d_W1 = c->d_W2 = nullptr;
  c->have_system = false;
}

#define CHK(expr)                       \
  do {                                  \
    pou_status s_ = (expr);             \
    if (s_ != POU_OK) return s_;        \
  } while (0)

// ---- event timing: a (start, stop) event pair around each timed launch
hipEvent_t pool_get(pou_ctx *c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void prof_begin(pou_ctx *c, int tag) {
  if (!((c->prof_mask >> tag) & 1u)) return;
  c->cur_tag = tag;
  c->cur_a = pool_get(c);
  if (c->cur_a) (void)hipEventRecord(c->cur_a, c->stream);
}

void prof_end(pou_ctx *c) {
  if (c->cur_tag < 0 || !c->cur_a) return;
  hipEvent_t b = pool_get(c);
  if (b) {
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back({c->cur_tag, c->cur_a, b});
  } else {
    c->pool.push_back(c->cur_a);
  }
  c->cur_tag = -1;
  c->cur_a = nullptr;
}

// Drop the newest timed launch of group `tag` (one that the device skipped:
// a gated accept of a declined trial), so per-launch averages cover real work.
void prof_discard_last(pou_ctx *c, int tag) {
  for (auto it = c->pending.rbegin(); it != c->pending.rend(); ++it) {
    if (it->tag == tag) {
      c->pool.push_back(it->a);
      c->pool.push_back(it->b);
      c->pending.erase(std::next(it).base());
      return;
    }
  }
}

// after a stream synchronisation every recorded event has completed
void prof_drain(pou_ctx *c) {
  for (auto &p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->prof_ms[p.tag] += ms;
      c->prof_n[p.tag] += 1;
    } else {
      (void)hipGetLastError();
    }
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
}

pou_status sync_read(pou_ctx *c, void *host, const void *dev, size_t bytes) {
  HIPCHK(c, hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_drain(c);
  return POU_OK;
}

// ------------------------------------------------------------------ Poisson

// Solve -Lap x = 4 pi (f - mean f) by conjugate gradients, warm-started from x,
// optionally preconditioned by the exact spectral inverse of -Lap.
pou_status poisson(pou_ctx *c, const double *f, double *x, double rtol, int maxit,
                   bool precond, int *iters) {
  hipStream_t s = c->stream;
  const i64 ng = c->ng;
  const int nb = c->nblk_field;
  const double ih2 = 1.0 / (c->h * c->h);
  double *sc = c->d_sc;  // [0] rz new, [1] rz old, [2] pq, [3] rr, [4] bb, [5] sum
  KL(POU_K_POISSON, pou::launch_dot2(f, nullptr, c->d_part, ng, nb, s));
  KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, sc + 5, 1, nb, 1, 1.0, s));
  KL(POU_K_POISSON, pou::launch_neg_lap(x, c->d_cg_q, nullptr, c->n, ih2, nb, s));
  KL(POU_K_POISSON, pou::launch_cg_rhs_residual(f, sc + 5, c->d_cg_q, c->d_cg_r, c->d_part, ng, nb, s));
  KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, sc + 3, 1, nb, 2, 1.0, s));
  double rb[2];
  CHK(sync_read(c, rb, sc + 3, sizeof(rb)));
  const double bb = rb[1];
  double rr = rb[0];
  if (!std::isfinite(bb) || !std::isfinite(rr))
    return fail(c, POU_ERR_NONFINITE, "Poisson right-hand side or residual is not finite");
  int it = 0;
  const int check = precond ? 1 : 8;
  bool conv = !(rr > rtol * rtol * bb);
  while (!conv && it < maxit) {
    const double *z = c->d_cg_r;
    if (precond) {
      KL(POU_K_POISSON, pou::launch_spectral_inverse(c->d_cg_r, c->d_cg_z, c->d_fft0, c->d_fft1,
                                             c->d_lam1, c->n, 1.0, s));
      z = c->d_cg_z;
    }
    KL(POU_K_POISSON, pou::launch_dot2(c->d_cg_r, z, c->d_part, ng, nb, s));
    KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, sc + 0, 1, nb, 1, 1.0, s));
    KL(POU_K_POISSON, pou::launch_cg_update_p(c->d_cg_p, z, sc + 0, sc + 1, it == 0, ng, s));
    KL(POU_K_POISSON, pou::launch_neg_lap(c->d_cg_p, c->d_cg_q, c->d_part, c->n, ih2, nb, s));
    KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, sc + 2, 1, nb, 1, 1.0, s));
    KL(POU_K_POISSON, pou::launch_cg_update_xr(x, c->d_cg_r, c->d_cg_p, c->d_cg_q, sc + 0, sc + 2,
                                       c->d_part, ng, nb, s));
    KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, sc + 3, 1, nb, 1, 1.0, s));
    HIPCHK(c, hipMemcpyAsync(sc + 1, sc + 0, sizeof(double), hipMemcpyDeviceToDevice, s));
    ++it;
    if (it % check == 0 || it == maxit) {
      CHK(sync_read(c, &rr, sc + 3, sizeof(double)));
      if (!std::isfinite(rr)) return fail(c, POU_ERR_NONFINITE, "Poisson CG residual is not finite");
      conv = !(rr > rtol * rtol * bb);
    }
  }
  // fix the gauge: zero mean
  KL(POU_K_POISSON, pou::launch_dot2(x, nullptr, c->d_part, ng, nb, s));
  KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, sc + 5, 1, nb, 1, 1.0, s));
  KL(POU_K_POISSON, pou::launch_remove_mean(x, sc + 5, ng, s));
  if (iters) *iters = it;
  if (!conv)
    return fail(c, POU_ERR_CG_NO_CONV,
                "Poisson CG did not reach rtol " + std::to_string(rtol) + " in " +
                    std::to_string(maxit) + " iterations");
  return POU_OK;
}

// Hartree solve without host synchronisation: x = 4 pi (-Lap)^+ (f - mean f)
// through the spectral inverse of the FD8 operator (the FFT zeroes the mean
// mode), then the residual of -Lap x = 4 pi (f - mean f) is measured; its
// r.r and b.b land in rrbb[0..1] for the caller's check.
pou_status poisson_async(pou_ctx *c, const double *f, double *x, double *rrbb) {
  hipStream_t s = c->stream;
  const int nb = c->nblk_field;
  const double ih2 = 1.0 / (c->h * c->h);
  double *sc = c->d_sc;  // [5] sum f
  const double fourpi = 12.566370614359172954;
  // sum f (for the residual's right-hand side) comes out of the forward FFT
  KL(POU_K_POISSON, pou::launch_spectral_inverse(f, x, c->d_fft0, c->d_fft1, c->d_lam1, c->n,
                                                 fourpi, s, sc + 5));
  KL(POU_K_POISSON, pou::launch_poisson_residual(x, f, sc + 5, c->d_part, c->n, ih2, nb, s));
  KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, rrbb, 1, nb, 2, 1.0, s));
  return POU_OK;
}

// ------------------------------------------------------------------ energy

bool nl_active(const pou_ctx *c) { return c->nl_on && (c->p.terms & POU_TERM_NLOC); }

// V_nloc of section 2.1 added to H W: the overlaps C = <xi_l, w_i> into C,
// sigma_ii (rep[0..N)) += sum_l C_li^2, rep[enl_off] = sum_i f_i sum_l C_li^2,
// then H w_i += sum_l C_li xi_l colour by colour.
template <typename T>
pou_status nonlocal_h(pou_ctx *c, const T *W, T *HW, double *C, double *rep, int enl_off) {
  hipStream_t s = c->stream;
  const int M = (int)c->nl_ions.size();
  KL(POU_K_HAMILTONIAN, pou::launch_nl_overlap<T>(W, c->d_nl, M, c->nl_bmax, c->N, c->n, c->L,
                                                  false, c->d_nlpart, s));
  KL(POU_K_OTHER, pou::launch_nl_finish(c->d_nlpart, M, c->nl_bmax, c->N, c->dv, c->d_occ, C,
                                        rep, enl_off, s));
  for (size_t k = 0; k < c->nl_col_off.size(); ++k)
    KL(POU_K_HAMILTONIAN, pou::launch_nl_apply<T>(HW, c->d_nl, c->d_nl_list + c->nl_col_off[k],
                                                  c->nl_col_cnt[k], c->nl_bmax, C, c->N, c->n,
                                                  c->L, s));
  return POU_OK;
}

// V_eff, H W and the energy partials of W for the current rho and V_H; the
// report (sigma, kin, energy sums) lands in rep on the device.
template <typename T>
pou_status potentials_and_h(pou_ctx *c, const T *W, T *HWout, double *rep) {
  hipStream_t s = c->stream;
  const int N = c->N;
  KL(POU_K_XC, pou::launch_xc_veff(c->d_rho, c->d_vh, c->d_vext, c->d_veff,
                                   sizeof(T) == 4 ? c->d_veff32 : nullptr, c->d_part, c->ng,
                                   c->p.terms, c->nblk_field, s));
  KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, rep + 2 * N, 1, c->nblk_field, 4, c->dv, s));
  const T *veff = sizeof(T) == 4 ? (const T *)c->d_veff32 : (const T *)c->d_veff;
  KL(POU_K_HAMILTONIAN, pou::launch_hamiltonian<T>(W, veff, HWout, c->d_part, N, c->st, s));
  KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, rep, N, c->st.ntile * c->st.nzc, 2, c->dv, s));
  if (nl_active(c)) CHK(nonlocal_h<T>(c, W, HWout, c->d_nlC, rep, Report::nl(N)));
  return POU_OK;
}

// Evaluate rho (unless already formed), V_H, V_eff, H W and the energy terms
// of W.  With the spectral preconditioner the Hartree solve runs without host
// synchronisation and its residual is checked when the report is read.
template <typename T>
pou_status evaluate(pou_ctx *c, const T *W, T *HWout, double *rep, bool rho_ready,
                    int *cg_iters) {
  hipStream_t s = c->stream;
  const int N = c->N;
  if (!rho_ready) KL(POU_K_DENSITY, pou::launch_density<T>(W, c->d_occ, c->d_rho, N, c->ng, s));
  int it = 0;
  double *rrbb = rep + Report::rr(N);
  if ((c->p.terms & POU_TERM_HARTREE) && c->p.cg_precond != 0) {
    CHK(poisson_async(c, c->d_rho, c->d_vh, rrbb));
    it = 1;
  } else {
    if (c->p.terms & POU_TERM_HARTREE)
      CHK(poisson(c, c->d_rho, c->d_vh, c->p.cg_rtol, c->p.cg_maxit, c->p.cg_precond != 0, &it));
    HIPCHK(c, hipMemsetAsync(rrbb, 0, 2 * sizeof(double), s));
  }
  c->last_cg_iters = it;
  if (cg_iters) *cg_iters = it;
  return potentials_and_h<T>(c, W, HWout, rep);
}

// evaluate(), then read the report (and the step scalars) to the host; if the
// one-iteration Hartree solve missed its tolerance, finish it with the checked
// solver and redo the potentials.
template <typename T>
pou_status eval_report(pou_ctx *c, const T *W, T *HWout, double *rep, bool rho_ready,
                       std::vector<double> &host, double *scal_host, int *cg_iters) {
  const int N = c->N;
  int it = 0;
  CHK(evaluate<T>(c, W, HWout, rep, rho_ready, &it));
  host.resize(Report::size(N));
  HIPCHK(c, hipMemcpyAsync(host.data(), rep, sizeof(double) * Report::size(N),
                           hipMemcpyDeviceToHost, c->stream));
  if (scal_host)
    HIPCHK(c, hipMemcpyAsync(scal_host, c->d_scal, 5 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_drain(c);
  const double rr = host[Report::rr(N)], bb = host[Report::rr(N) + 1];
  if (!std::isfinite(rr) || !std::isfinite(bb))
    return fail(c, POU_ERR_NONFINITE, "Poisson right-hand side or residual is not finite");
  if (rr > c->p.cg_rtol * c->p.cg_rtol * bb) {
    int more = 0;
    CHK(poisson(c, c->d_rho, c->d_vh, c->p.cg_rtol, c->p.cg_maxit, true, &more));
    it += more;
    c->last_cg_iters = it;
    CHK(potentials_and_h<T>(c, W, HWout, rep));
    CHK(sync_read(c, host.data(), rep, sizeof(double) * Report::size(N)));
  }
  if (cg_iters) *cg_iters = it;
  return POU_OK;
}

void terms_from_report(const pou_ctx *c, const double *rep, pou_energy_terms *t) {
  const int N = c->N;
  double ekin = 0.0;
  for (int i = 0; i < N; ++i) ekin += c->occ[i] * rep[N + i];
  if (!(c->p.terms & POU_TERM_KIN)) ekin = 0.0;
  const double cx = 0.73855876638202240;  // 3/4 (3/pi)^(1/3)
  const double ex = -cx * rep[2 * N + 0];
  const double eext = rep[2 * N + 1];
  const double eh = 0.5 * rep[2 * N + 2];
  t->E_kin = ekin;
  t->E_x = (c->p.terms & POU_TERM_XC) ? ex : 0.0;
  t->E_ext = (c->p.terms & POU_TERM_EXT) ? eext : 0.0;
  t->E_H = (c->p.terms & POU_TERM_HARTREE) ? eh : 0.0;
  t->E_c = (c->p.terms & POU_TERM_CORR) ? rep[2 * N + 3] : 0.0;
  t->E_nl = (c->p.terms & POU_TERM_NLOC) ? rep[Report::nl(N)] : 0.0;
  t->E = t->E_kin + t->E_x + t->E_ext + t->E_H + t->E_c + t->E_nl;
  t->cg_iters = c->last_cg_iters;
}

// ------------------------------------------------------------------ orth

template <typename T>
const T *dmat(const pou_ctx *c) {
  return sizeof(T) == 8 ? (const T *)c->d_D64 : (const T *)c->d_D32;
}

template <typename T>
pou_status gram(pou_ctx *c, const T *X, bool bf16) {
  hipStream_t s = c->stream;
  if (bf16 && sizeof(T) == 4)
    KL(POU_K_GRAM, pou::launch_gram_partial_bf16((const float *)X, c->N, c->ng, c->nsplit,
                                            c->d_gpart, s));
  else
    KL(POU_K_GRAM, pou::launch_gram_partial<T>(X, c->N, c->ng, c->nsplit, c->d_gpart, s));
  KL(POU_K_CHOLESKY, pou::launch_gram_reduce(c->d_gpart, c->N, c->nsplit, c->dv, c->d_G, s));
  return POU_OK;
}

// Cholesky-QR passes of X into out (X and out distinct, both not aliasing d_W1).
// info[2p], info[2p+1] = (not-SPD flag, max|G-I|) of pass p.  The last apply
// also forms rho when want_rho.
template <typename T>
pou_status orth_passes(pou_ctx *c, const T *X, T *out, int passes, double *info, bool want_rho,
                       bool *rho_done) {
  hipStream_t s = c->stream;
  const bool mixed = sizeof(T) == 4;
  const T *cur = X;
  *rho_done = false;
  for (int p = 0; p < passes; ++p) {
    // BF16 Gram only for the first of two passes: a single pass must be
    // FP32-accurate, since nothing after it corrects its factor
    CHK(gram<T>(c, cur, mixed && p == 0 && passes == 2));
    KL(POU_K_CHOLESKY, pou::launch_cholesky_inverse(c->d_G, c->d_Minv, c->d_D32, c->d_D64, c->N,
                                                       info + 2 * p, c->d_cholws, s));
    const bool last = (p == passes - 1);
    T *dst = last ? out : (T *)c->d_W1;
    if (cur == dst) return fail(c, POU_ERR_ARG, "internal: aliasing orth buffers");
    double *rho = (last && want_rho) ? c->d_rho : nullptr;
    KL(POU_K_APPLY, pou::launch_apply_lower<T>(c->d_Minv, dmat<T>(c), cur, dst, c->N, c->ng, c->d_occ,
                                               rho, s, info + 2 * p, c->d_fsplit,
                                               c->d_rhopart));
    if (rho) *rho_done = true;
    cur = dst;
  }
  return POU_OK;
}

// Trial point and its orthonormalisation for N <= 128: one pass forms
// Wt = W - tau Z and the first Gram; Cholesky; for two passes the first factor
// is applied once to measure the second Gram, and the product of both factors
// is applied to Wt in the final pass, which also forms rho.
template <typename T>
pou_status trial_orth_fused(pou_ctx *c, const T *W, double tscale, double *info) {
  hipStream_t s = c->stream;
  const bool mixed = sizeof(T) == 4;
  const int passes = c->p.orth_passes;
  KL(POU_K_TRIAL, pou::launch_trial_gram<T>(W, (const T *)c->d_HW, c->d_rep[0], c->d_scal, tscale,
                                           (T *)c->d_Wt, c->N, c->ng, c->nsplit,
                                           mixed && passes == 2, c->d_gpart, s));
  KL(POU_K_CHOLESKY, pou::launch_gram_reduce(c->d_gpart, c->N, c->nsplit, c->dv, c->d_G, s));
  // with two passes the first factor feeds the second pass's Gram (FP32 D
  // for the mixed fused apply, FP64 D otherwise) and the factor product (M)
  const int outs1 = passes == 2 ? pou::CHOL_OUT_MINV | (mixed ? pou::CHOL_OUT_D32 : pou::CHOL_OUT_D64)
                                : pou::CHOL_OUT_ALL;
  KL(POU_K_CHOLESKY, pou::launch_cholesky_inverse(c->d_G, c->d_Minv, c->d_D32, c->d_D64, c->N,
                                                  info, c->d_cholws, s, outs1));
  if (passes == 2) {
    if (mixed) {
      // W1 = Wt L1^-T stays on chip: only its Gram leaves the kernel
      KL(POU_K_APPLY_GRAM, pou::launch_apply_gram(c->d_D32, (const float *)c->d_Wt, c->N, c->ng,
                                             c->nsplit, c->d_gpart, s));
    } else {
      KL(POU_K_APPLY, pou::launch_apply_lower<T>(c->d_Minv, dmat<T>(c), (const T *)c->d_Wt,
                                                 (T *)c->d_W1, c->N, c->ng, nullptr, nullptr, s));
      KL(POU_K_GRAM, pou::launch_trial_gram<T>((const T *)c->d_W1, nullptr, nullptr, nullptr,
                                               0.0, nullptr, c->N, c->ng, c->nsplit, false,
                                               c->d_gpart, s));
    }
    KL(POU_K_CHOLESKY, pou::launch_gram_reduce(c->d_gpart, c->N, c->nsplit, c->dv, c->d_G, s));
    KL(POU_K_CHOLESKY, pou::launch_cholesky_inverse(c->d_G, c->d_Minv2, c->d_D32, c->d_D64, c->N,
                                                    info + 2, c->d_cholws, s,
                                                    pou::CHOL_OUT_MINV));
    KL(POU_K_CHOLESKY, pou::launch_combine_factors(c->d_Minv2, c->d_Minv, c->d_Mcomb, c->d_D64,
                                                   c->d_D32, c->N, mixed, s));
  }
  KL(POU_K_APPLY, pou::launch_apply_lower<T>(c->d_Minv, dmat<T>(c), (const T *)c->d_Wt,
                                             (T *)c->d_W2, c->N, c->ng, c->d_occ, c->d_rho, s));
  return POU_OK;
}

// ------------------------------------------------------------------ subspace rotation

template <typename T>
pou_status energy_impl(pou_ctx *c, const T *U, pou_energy_terms *out);

// Eigen-decomposition of a symmetric N x N matrix (row-major A, destroyed):
// A V = V diag(w), w ascending, V orthogonal with each column's largest-
// magnitude entry positive.  Householder reduction to tridiagonal form
// (A = Q T Q^T), then implicit symmetric QR steps with Wilkinson shifts on T
// (deflating off-diagonals below rounding level), the plane rotations
// accumulated into Q; all updates run along contiguous rows.
void symm_eigh(int N, std::vector<double> &A, std::vector<double> &V, std::vector<double> &w) {
  auto a = [&](int i, int j) -> double & { return A[(size_t)i * N + j]; };
  std::vector<double> Mt((size_t)N * N, 0.0);  // rows: columns of the accumulated orthogonal factor
  for (int i = 0; i < N; ++i) Mt[(size_t)i * N + i] = 1.0;
  std::vector<double> v(N), p(N), wv(N);
  // 1. A = Q T Q^T, Householder reflections on the trailing columns
  for (int k = 0; k + 2 < N; ++k) {
    const int m = N - k - 1;  // length of x = A[k+1 .., k]
    double sigma = 0.0;
    for (int i = 1; i < m; ++i) sigma += a(k + 1 + i, k) * a(k + 1 + i, k);
    const double x0 = a(k + 1, k);
    if (sigma == 0.0) continue;  // already tridiagonal in this column
    const double mu = std::sqrt(x0 * x0 + sigma);
    const double v0 = (x0 <= 0.0) ? x0 - mu : -sigma / (x0 + mu);
    const double beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
    v[0] = 1.0;
    for (int i = 1; i < m; ++i) v[i] = a(k + 1 + i, k) / v0;
    // p = beta * A22 v ; w = p - (beta p.v / 2) v
    for (int i = 0; i < m; ++i) {
      double acc = 0.0;
      const double *row = &A[(size_t)(k + 1 + i) * N + k + 1];
      for (int j = 0; j < m; ++j) acc += row[j] * v[j];
      p[i] = beta * acc;
    }
    double pv = 0.0;
    for (int i = 0; i < m; ++i) pv += p[i] * v[i];
    for (int i = 0; i < m; ++i) wv[i] = p[i] - 0.5 * beta * pv * v[i];
    for (int i = 0; i < m; ++i) {
      double *row = &A[(size_t)(k + 1 + i) * N + k + 1];
      for (int j = 0; j < m; ++j) row[j] -= v[i] * wv[j] + wv[i] * v[j];
    }
    a(k + 1, k) = mu;
    a(k, k + 1) = mu;
    for (int i = 1; i < m; ++i) a(k + 1 + i, k) = a(k, k + 1 + i) = 0.0;
    // Mt <- H_k Mt (rows k+1 ..)
    std::fill(p.begin(), p.end(), 0.0);  // p <- v^T Mt[k+1 .., :]
    for (int i = 0; i < m; ++i) {
      const double *row = &Mt[(size_t)(k + 1 + i) * N];
      for (int j = 0; j < N; ++j) p[j] += v[i] * row[j];
    }
    for (int i = 0; i < m; ++i) {
      double *row = &Mt[(size_t)(k + 1 + i) * N];
      const double f = beta * v[i];
      for (int j = 0; j < N; ++j) row[j] -= f * p[j];
    }
  }
  std::vector<double> d(N), e(N, 0.0);
  for (int i = 0; i < N; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < N; ++i) e[i] = a(i + 1, i);
  // 2. implicit symmetric QR steps with Wilkinson shifts on T = tridiag(d, e)
  const double eps = 2.220446049250313e-16;
  int hi = N - 1, guard = 0;
  while (hi > 0 && guard < 60 * N) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    ++guard;
    const double g = (d[hi - 1] - d[hi]) / (2.0 * e[hi - 1]);
    const double r0 = std::hypot(g, 1.0);
    const double mu = d[hi] - e[hi - 1] / (g + std::copysign(r0, g));
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      const double c = (r == 0.0) ? 1.0 : x / r, s = (r == 0.0) ? 0.0 : -z / r;
      if (k > lo) e[k - 1] = r;
      const double aa = d[k], bb = e[k], cc = d[k + 1];
      d[k] = c * c * aa - 2.0 * c * s * bb + s * s * cc;
      d[k + 1] = s * s * aa + 2.0 * c * s * bb + c * c * cc;
      e[k] = c * s * aa + (c * c - s * s) * bb - c * s * cc;
      if (k + 1 < hi) {
        z = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      x = e[k];
      double *rk = &Mt[(size_t)k * N], *rk1 = &Mt[(size_t)(k + 1) * N];
      for (int j = 0; j < N; ++j) {
        const double u = rk[j], t = rk1[j];
        rk[j] = c * u - s * t;
        rk1[j] = s * u + c * t;
      }
    }
  }
  // eigenvalues ascending; column j of V = row of Mt; largest entry positive
  std::vector<int> ord(N);
  for (int i = 0; i < N; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] < d[y]; });
  V.assign((size_t)N * N, 0.0);
  w.resize(N);
  for (int jn = 0; jn < N; ++jn) {
    const int jo = ord[jn];
    w[jn] = d[jo];
    const double *row = &Mt[(size_t)jo * N];
    int imax = 0;
    for (int i = 1; i < N; ++i)
      if (std::fabs(row[i]) > std::fabs(row[imax])) imax = i;
    const double sg = row[imax] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < N; ++i) V[(size_t)i * N + jn] = sg * row[i];
  }
}

// Subspace diagonalisation of the current iterate (section 3.3): Sigma =
// <(H W)^T W> (symmetrised), P^T Sigma P = Gamma, W <- W P and H W <- (H W) P,
// sigma_ii <- <(H W)_i, W_i>, and ||Z||^2 of the rotated iterate into the step
// scalars (the BB step already computed for the next iteration is kept: its
// traces are invariant under the rotation).
template <typename T>
pou_status rotate_subspace(pou_ctx *c, T *W) {
  hipStream_t s = c->stream;
  const int N = c->N;
  KL(POU_K_OTHER, pou::launch_cross_gram<T>((const T *)c->d_HW, (const T *)W, N, c->ng, c->dv,
                                            c->d_xpart, c->d_S, s));
  std::vector<double> A((size_t)N * N), V, w;
  CHK(sync_read(c, A.data(), c->d_S, sizeof(double) * A.size()));
  for (double x : A)
    if (!std::isfinite(x)) return fail(c, POU_ERR_NONFINITE, "subspace matrix is not finite");
  symm_eigh(N, A, V, w);
  // the rotation kernel multiplies by a row-major M with out_j = sum_i M[j][i] x_i,
  // so it takes P^T (P's columns are the eigenvectors)
  std::vector<double> &Pt = A;  // A is consumed by the eigensolver
  Pt.resize((size_t)N * N);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) Pt[(size_t)j * N + i] = V[(size_t)i * N + j];
  HIPCHK(c, hipMemcpyAsync(c->d_P, Pt.data(), sizeof(double) * Pt.size(), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));  // Pt is pageable host memory
  KL(POU_K_OTHER, pou::launch_rotate<T>(c->d_P, (const T *)W, (T *)c->d_W2, N, c->ng, s));
  HIPCHK(c, hipMemcpyAsync(W, c->d_W2, sizeof(T) * (size_t)N * c->ng, hipMemcpyDeviceToDevice, s));
  KL(POU_K_OTHER, pou::launch_rotate<T>(c->d_P, (const T *)c->d_HW, (T *)c->d_HWt, N, c->ng, s));
  std::swap(c->d_HW, c->d_HWt);
  // sigma of the rotated iterate into the report of the current iterate
  KL(POU_K_OTHER, pou::launch_rowdot<T>((const T *)c->d_HW, (const T *)W, false, c->d_part, N,
                                        c->ng, c->nblk_orb, s));
  KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, c->d_rep[0], N, c->nblk_orb, 1, c->dv, s));
  KL(POU_K_OTHER, pou::launch_zz<T>(W, (const T *)c->d_HW, c->d_rep[0], c->d_part, N, c->ng,
                                    c->nblk_orb, s));
  KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, c->d_red, N, c->nblk_orb, 1, c->dv, s));
  KL(POU_K_OTHER, pou::launch_bb_tau(c->d_red, N, 3, c->p.tau_init, c->d_scal, nullptr, s));
  c->eval_HU = c->d_HW;
  // the projector overlaps of the last evaluation belong to the unrotated
  // iterate: a backward pass re-evaluates the rotated one
  if (nl_active(c)) c->eval_ptr = nullptr;
  return POU_OK;
}

// Norm of the Stiefel gradient H U - U Sigma with Sigma = <(H U)^T U>.
template <typename T>
pou_status residual_impl(pou_ctx *c, const T *U, double *resid, double *Sigma) {
  hipStream_t s = c->stream;
  const int N = c->N;
  if (c->eval_ptr != U) CHK(energy_impl<T>(c, U, nullptr));
  const T *HU = (const T *)c->eval_HU;
  KL(POU_K_OTHER, pou::launch_cross_gram<T>(HU, U, N, c->ng, c->dv, c->d_xpart, c->d_S, s));
  KL(POU_K_OTHER, pou::launch_rotate<T>(c->d_S, U, (T *)c->d_Wt, N, c->ng, s));
  KL(POU_K_OTHER, pou::launch_rowdot<T>(HU, (const T *)c->d_Wt, true, c->d_part, N, c->ng,
                                        c->nblk_orb, s));
  KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, c->d_red, N, c->nblk_orb, 1, c->dv, s));
  std::vector<double> r(N);
  CHK(sync_read(c, r.data(), c->d_red, sizeof(double) * N));
  double acc = 0.0;
  for (double x : r) acc += x;
  if (!std::isfinite(acc)) return fail(c, POU_ERR_NONFINITE, "residual is not finite");
  if (resid) *resid = std::sqrt(acc);
  if (Sigma) CHK(sync_read(c, Sigma, c->d_S, sizeof(double) * (size_t)N * N));
  return POU_OK;
}

// ------------------------------------------------------------------ step
template <typename T>
pou_status restart(pou_ctx *c, const T *W) {
  hipStream_t s = c->stream;
  const int N = c->N;
  int it = 0;
  std::vector<double> &r = c->rep_host;
  CHK(eval_report<T>(c, W, (T *)c->d_HW, c->d_rep[0], false, r, nullptr, &it));
  pou_energy_terms t;
  terms_from_report(c, r.data(), &t);
  if (!std::isfinite(t.E)) return fail(c, POU_ERR_NONFINITE, "energy of U is not finite");
  c->E = t.E;
  c->C = t.E;
  c->Q = 1.0;
  c->l = 0;
  c->hist = false;
  c->last_U = W;
  c->cur_valid = true;
  c->eval_ptr = W;
  c->eval_HU = c->d_HW;
  // ||Z||^2 of the start and tau_init on the device (no history yet)
  KL(POU_K_OTHER, pou::launch_zz<T>(W, (const T *)c->d_HW, c->d_rep[0], c->d_part, N, c->ng,
                                    c->nblk_orb, s));
  KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, c->d_red, N, c->nblk_orb, 1, c->dv, s));
  KL(POU_K_OTHER, pou::launch_bb_tau(c->d_red, N, 0, c->p.tau_init, c->d_scal, nullptr, s));
  return POU_OK;
}

// Accept of the current trial (W <- W2, BB dot products, next tau_BB on the
// device), gated on flags[0]: enqueued before the host knows the decision.
template <typename T>
pou_status enqueue_accept(pou_ctx *c, T *W, const double *gate) {
  hipStream_t s = c->stream;
  const int N = c->N;
  KL(POU_K_COMMIT, pou::launch_commit<T>(W, (const T *)c->d_HW, c->d_rep[0], (const T *)c->d_W2,
                                         (const T *)c->d_HWt, c->d_rep[1], c->d_part, N, c->ng,
                                         c->nblk_commit, gate, s));
  KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, c->d_red, N, c->nblk_commit, 4, c->dv, s));
  const int lnext = c->l + 1;
  const int mode = (c->p.bb_mode == 1 || c->p.bb_mode == 2) ? c->p.bb_mode
                                                             : ((lnext % 2 == 1) ? 1 : 2);
  KL(POU_K_OTHER, pou::launch_bb_tau(c->d_red, N, mode, c->p.tau_init, c->d_scal, gate, s));
  return POU_OK;
}

// A step of Algorithm M with l mod n_org != 0 (section 3.3): the plain
// W <- W - tau_BB Z, no orthonormalisation, no energy test, no backtracking.
// H(rho(W)) of the new iterate is still formed (for the next direction) and
// the accept kernel updates U and the BB history as after any step; C, Q and
// the energy of the last orthonormal iterate are left alone.
template <typename T>
pou_status plain_step(pou_ctx *c, T *W, pou_step_info *info) {
  hipStream_t s = c->stream;
  const int N = c->N;
  const int RS = Report::size(N);
  double *rep_t = c->d_rep[1];
  double *hrep = c->h_step, *hscal = c->h_step + RS;
  KL(POU_K_TRIAL, pou::launch_trial<T>(W, (const T *)c->d_HW, c->d_rep[0], c->d_scal, 1.0,
                                       (T *)c->d_W2, N, c->ng, s));
  int it = 0;
  CHK(evaluate<T>(c, (const T *)c->d_W2, (T *)c->d_HWt, rep_t, false, &it));
  HIPCHK(c, hipMemcpyAsync(hrep, rep_t, sizeof(double) * RS, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(hscal, c->d_scal, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  prof_drain(c);
  const double tau_bb = hscal[0], zz = hscal[1];
  const double rr = hrep[Report::rr(N)], bb = hrep[Report::rr(N) + 1];
  if (!std::isfinite(rr) || !std::isfinite(bb))
    return fail(c, POU_ERR_NONFINITE, "Poisson right-hand side or residual is not finite");
  std::vector<double> &r = c->rep_host;
  r.assign(hrep, hrep + RS);
  if (rr > c->p.cg_rtol * c->p.cg_rtol * bb) {
    int more = 0;
    CHK(poisson(c, c->d_rho, c->d_vh, c->p.cg_rtol, c->p.cg_maxit, true, &more));
    it += more;
    c->last_cg_iters = it;
    CHK(potentials_and_h<T>(c, (const T *)c->d_W2, (T *)c->d_HWt, rep_t));
    CHK(sync_read(c, r.data(), rep_t, sizeof(double) * RS));
  }
  pou_energy_terms et{};
  terms_from_report(c, r.data(), &et);
  if (!std::isfinite(et.E)) return fail(c, POU_ERR_NONFINITE, "energy of the plain step is not finite");
  CHK(enqueue_accept<T>(c, W, nullptr));
  std::swap(c->d_HW, c->d_HWt);
  std::swap(c->d_rep[0], c->d_rep[1]);
  c->hist = true;
  c->eval_ptr = W;
  c->eval_HU = c->d_HW;
  if (info) {
    info->l = c->l;
    info->s = 0;
    info->accepted = 1;
    info->cg_iters = it;
    info->E = et.E;
    info->tau_bb = tau_bb;
    info->tau = tau_bb;
    info->zz = zz;
    info->df = std::numeric_limits<double>::quiet_NaN();
    info->C = c->C;
    info->Q = c->Q;
    info->gram_dev = 0.0;
    info->orthonormalized = 0;
    info->rotated = 0;
  }
  c->l = c->l + 1;
  return POU_OK;
}

// One iteration of Algorithm M.  tau_BB and ||Z||^2 of the current iterate
// live on the device (d_scal); the trial kernels read tau = tau_BB * delta^s
// from there.  After each trial the test of eq. "ene-de" runs on the device
// and the accept is enqueued behind it, gated on its outcome, so the one host
// synchronisation per trial (reading the report into pinned memory) does not
// stall the stream; the host then only follows the device's decision.  If the
// one-iteration Hartree solve missed its tolerance the device declines, and
// the host finishes the solve, redoes the potentials and decides itself.
template <typename T>
pou_status step_impl(pou_ctx *c, T *W, pou_step_info *info) {
  hipStream_t s = c->stream;
  const int N = c->N;
  if (W != c->last_U || !c->cur_valid) CHK(restart<T>(c, W));
  if (c->p.n_org > 1 && c->l % c->p.n_org != 0) return plain_step<T>(c, W, info);
  const int passes = c->p.orth_passes;
  const int RS = Report::size(N);
  double *hrep = c->h_step, *hscal = c->h_step + RS, *hflag = c->h_step + RS + 5;
  pou_energy_terms et{};
  double tau = 0.0, tau_bb = 0.0, zz = 0.0;
  int s_acc = 0, cg_total = 0;
  bool accepted = false;
  double gram_dev = 0.0;
  for (int sidx = 0; sidx <= c->p.s_max; ++sidx) {
    const double tscale = std::pow(c->p.delta, sidx);
    const bool last = (sidx == c->p.s_max);
    s_acc = sidx;
    bool rho_done = false;
    double *rep_t = c->d_rep[1];
    double *dflag = rep_t + RS + 5;  // written by the Armijo kernel, read by the gated accept
    if (N <= 128) {
      CHK(trial_orth_fused<T>(c, W, tscale, rep_t + Report::orth(N)));
      rho_done = true;
    } else {
      KL(POU_K_TRIAL, pou::launch_trial<T>(W, (const T *)c->d_HW, c->d_rep[0], c->d_scal, tscale,
                                           (T *)c->d_Wt, N, c->ng, s));
      CHK(orth_passes<T>(c, (const T *)c->d_Wt, (T *)c->d_W2, passes, rep_t + Report::orth(N), true,
                         &rho_done));
    }
    int it = 0;
    CHK(evaluate<T>(c, (const T *)c->d_W2, (T *)c->d_HWt, rep_t, rho_done, &it));
    cg_total += it;
    KL(POU_K_OTHER, pou::launch_armijo(rep_t, c->d_occ, N, c->p.terms, passes, Report::orth(N),
                                       Report::rr(N),
                                       c->p.cg_rtol * c->p.cg_rtol, c->d_scal, tscale, c->C,
                                       c->p.rho1, last ? 1 : 0, rep_t + RS, s));
    HIPCHK(c, hipMemcpyAsync(hrep, rep_t, sizeof(double) * (RS + 7), hipMemcpyDeviceToHost, s));
    CHK(enqueue_accept<T>(c, W, dflag));
    HIPCHK(c, hipStreamSynchronize(s));
    if (hflag[0] == 0.0) prof_discard_last(c, POU_K_COMMIT);
    prof_drain(c);
    tau_bb = hscal[0];
    zz = hscal[1];
    tau = tau_bb * tscale;
    const double rr = hrep[Report::rr(N)], bb = hrep[Report::rr(N) + 1];
    if (!std::isfinite(rr) || !std::isfinite(bb))
      return fail(c, POU_ERR_NONFINITE, "Poisson right-hand side or residual is not finite");
    if (hflag[0] != 0.0) {
      // accepted on the device: W, the BB history and tau_BB are updated
      accepted = hflag[1] != 0.0;
      terms_from_report(c, hrep, &et);
      gram_dev = hrep[Report::orth(N) + 1];
      break;
    }
    std::vector<double> &r = c->rep_host;
    r.assign(hrep, hrep + RS);
    const bool redo = rr > c->p.cg_rtol * c->p.cg_rtol * bb;
    if (redo) {
      // finish the Hartree solve with the checked solver and redo the potentials
      int more = 0;
      CHK(poisson(c, c->d_rho, c->d_vh, c->p.cg_rtol, c->p.cg_maxit, true, &more));
      cg_total += more;
      c->last_cg_iters = it + more;
      CHK(potentials_and_h<T>(c, (const T *)c->d_W2, (T *)c->d_HWt, rep_t));
      CHK(sync_read(c, r.data(), rep_t, sizeof(double) * RS));
    }
    for (int p = 0; p < passes; ++p)
      if (r[Report::orth(N) + 2 * p] != 0.0)
        return fail(c, POU_ERR_NOT_SPD, "trial Gram matrix is not positive definite (pass " +
                                             std::to_string(p) + ")");
    terms_from_report(c, r.data(), &et);
    if (!std::isfinite(et.E)) return fail(c, POU_ERR_NONFINITE, "trial energy is not finite");
    gram_dev = r[Report::orth(N) + 1];
    if (!redo && !last) continue;  // the device found eq. "ene-de" violated: backtrack
    // host decision after a finished Hartree solve (or the last trial)
    const bool pass = et.E <= c->C - c->p.rho1 * tau * zz;
    if (pass || last) {
      accepted = pass;
      KL(POU_K_OTHER, pou::launch_set_flags(dflag, 1.0, pass ? 1.0 : 0.0, s));
      CHK(enqueue_accept<T>(c, W, dflag));
      break;
    }
  }
  std::swap(c->d_HW, c->d_HWt);
  std::swap(c->d_rep[0], c->d_rep[1]);
  const double E_old = c->E;
  c->E = et.E;
  const double Qn = c->p.eta * c->Q + 1.0;
  c->C = (c->p.eta * c->Q * c->C + c->E) / Qn;
  c->Q = Qn;
  c->hist = true;
  c->eval_ptr = W;
  c->eval_HU = c->d_HW;
  // subspace diagonalisation of the new iterate after iteration l, l mod n_diag == 0
  bool rotated = false;
  if (c->p.n_diag > 0 && c->l % c->p.n_diag == 0) {
    CHK(rotate_subspace<T>(c, W));
    rotated = true;
  }
  if (info) {
    info->orthonormalized = 1;
    info->rotated = rotated ? 1 : 0;
    info->l = c->l;
    info->s = s_acc;
    info->accepted = accepted ? 1 : 0;
    info->cg_iters = cg_total;
    info->E = c->E;
    info->tau_bb = tau_bb;
    info->tau = tau;
    info->zz = zz;
    info->df = std::fabs(E_old - c->E) / (std::fabs(E_old) + 1.0);
    info->C = c->C;
    info->Q = c->Q;
    info->gram_dev = gram_dev;
  }
  c->l = c->l + 1;
  return POU_OK;
}

template <typename T>
pou_status orthonormalize_impl(pou_ctx *c, T *U, double *orth_err) {
  hipStream_t s = c->stream;
  const size_t bytes = (size_t)c->N * c->ng * sizeof(T);
  const double thr = sizeof(T) == 8 ? 1e-8 : 1e-4;
  // strong guarantee: work on copies, write U only at the end
  HIPCHK(c, hipMemcpyAsync(c->d_Wt, U, bytes, hipMemcpyDeviceToDevice, s));
  double info[2];
  T *src = (T *)c->d_Wt, *dst = (T *)c->d_W2;
  bool done = false;
  for (int p = 0; p < 3 && !done; ++p) {
    CHK(gram<T>(c, src, false));
    KL(POU_K_CHOLESKY, pou::launch_cholesky_inverse(c->d_G, c->d_Minv, c->d_D32, c->d_D64, c->N,
                                                       c->d_red, c->d_cholws, s));
    KL(POU_K_APPLY, pou::launch_apply_lower<T>(c->d_Minv, dmat<T>(c), src, dst, c->N, c->ng, nullptr,
                                               nullptr, s, c->d_red, c->d_fsplit));
    CHK(sync_read(c, info, c->d_red, sizeof(info)));
    if (!std::isfinite(info[1])) return fail(c, POU_ERR_NONFINITE, "U is not finite");
    if (info[0] != 0.0)
      return fail(c, POU_ERR_NOT_SPD, "Gram matrix of U is not positive definite");
    done = info[1] < thr && p > 0;
    if (info[1] < thr * 1e-4) done = true;
    std::swap(src, dst);
  }
  HIPCHK(c, hipMemcpyAsync(U, src, bytes, hipMemcpyDeviceToDevice, s));
  if (orth_err) {
    CHK(gram<T>(c, U, false));
    std::vector<double> G((size_t)c->N * c->N);
    CHK(sync_read(c, G.data(), c->d_G, sizeof(double) * G.size()));
    double m = 0.0;
    for (int i = 0; i < c->N; ++i)
      for (int j = 0; j < c->N; ++j)
        m = std::max(m, std::fabs(G[(size_t)i * c->N + j] - (i == j ? 1.0 : 0.0)));
    *orth_err = m;
  } else {
    HIPCHK(c, hipStreamSynchronize(s));
    prof_drain(c);
  }
  if (c->last_U == U) c->cur_valid = false;
  if (c->eval_ptr == U) c->eval_ptr = nullptr;
  c->hist = false;
  return POU_OK;
}

template <typename T>
pou_status energy_impl(pou_ctx *c, const T *U, pou_energy_terms *out) {
  T *hu = (T *)((c->last_U == U && c->cur_valid) ? c->d_HW : c->d_HWt);
  double *rep = (hu == (T *)c->d_HW) ? c->d_rep[0] : c->d_rep[1];
  int it = 0;
  std::vector<double> &r = c->rep_host;
  CHK(eval_report<T>(c, U, hu, rep, false, r, nullptr, &it));
  pou_energy_terms t;
  terms_from_report(c, r.data(), &t);
  t.cg_iters = it;
  if (!std::isfinite(t.E)) return fail(c, POU_ERR_NONFINITE, "energy of U is not finite");
  if (out) *out = t;
  c->eval_ptr = U;
  c->eval_HU = hu;
  return POU_OK;
}

template <typename T>
pou_status backward_impl(pou_ctx *c, const T *U, double gE, T *dU, double *dR, double *dsig) {
  hipStream_t s = c->stream;
  if (c->eval_ptr != U) CHK(energy_impl<T>(c, U, nullptr));
  if (dU)
    KL(POU_K_OTHER, pou::launch_backward_scale<T>((const T *)c->eval_HU, c->d_occ, gE * 2.0 * c->dv,
                                            dU, c->N, c->ng, s));
  if ((dR || dsig) && c->M > 0) {
    const int nb = std::min(256, c->nblk_field);
    KL(POU_K_OTHER, pou::launch_ion_forces(c->d_atoms, c->M, c->d_vh, c->d_part, c->n, c->L, nb, s));
    KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, c->d_red, c->M, nb, 4, -gE * c->dv, s));
    std::vector<double> f(4 * c->M);
    CHK(sync_read(c, f.data(), c->d_red, sizeof(double) * f.size()));
    std::vector<double> R(3 * c->M), S(c->M);
    for (int I = 0; I < c->M; ++I) {
      for (int a = 0; a < 3; ++a) R[3 * I + a] = f[a * c->M + I];
      S[I] = f[3 * c->M + I];
    }
    if (nl_active(c) && dR) {
      // dE_nl/dR_Ia = sum_i f_i sum_l 2 <xi_l, u_i> <d xi_l / dR_Ia, u_i>
      const int M = c->M, N = c->N;
      KL(POU_K_OTHER, pou::launch_nl_overlap<T>(U, c->d_nl, M, c->nl_bmax, N, c->n, c->L, true,
                                                c->d_nlpart, s));
      KL(POU_K_OTHER, pou::launch_nl_sum_deriv(c->d_nlpart, M, c->nl_bmax, N, c->dv, c->d_nlD, s));
      std::vector<double> Ch((size_t)4 * M * N), Dh((size_t)12 * M * N);
      CHK(sync_read(c, Ch.data(), c->d_nlC, sizeof(double) * Ch.size()));
      CHK(sync_read(c, Dh.data(), c->d_nlD, sizeof(double) * Dh.size()));
      for (int I = 0; I < M; ++I)
        for (int a = 0; a < 3; ++a) {
          double acc = 0.0;
          for (int l = 0; l < 4; ++l)
            for (int i = 0; i < N; ++i)
              acc += c->occ[i] * 2.0 * Ch[(size_t)(4 * I + l) * N + i] *
                     Dh[((size_t)I * 12 + 3 * l + a) * N + i];
          R[3 * I + a] += gE * acc;
        }
    }
    if (dR) HIPCHK(c, hipMemcpyAsync(dR, R.data(), sizeof(double) * R.size(),
                                     hipMemcpyHostToDevice, s));
    if (dsig) HIPCHK(c, hipMemcpyAsync(dsig, S.data(), sizeof(double) * S.size(),
                                       hipMemcpyHostToDevice, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  prof_drain(c);
  return POU_OK;
}

template <typename T>
pou_status hamiltonian_impl(pou_ctx *c, const T *U, T *HU, double *sigma) {
  hipStream_t s = c->stream;
  const T *veff = sizeof(T) == 4 ? (const T *)c->d_veff32 : (const T *)c->d_veff;
  KL(POU_K_HAMILTONIAN, pou::launch_hamiltonian<T>(U, veff, HU, c->d_part, c->N, c->st, s));
  KL(POU_K_OTHER, pou::launch_segment_sum(c->d_part, c->d_red, c->N, c->st.ntile * c->st.nzc, 2,
                                    c->dv, s));
  if (nl_active(c)) CHK(nonlocal_h<T>(c, U, HU, c->d_nlC2, c->d_red, 2 * c->N));
  if (sigma) CHK(sync_read(c, sigma, c->d_red, sizeof(double) * c->N));
  else HIPCHK(c, hipStreamSynchronize(s));
  prof_drain(c);
  return POU_OK;
}

template <typename T>
pou_status gram_impl(pou_ctx *c, const T *U, int mode, double *G) {
  CHK(gram<T>(c, U, mode == POU_GRAM_BF16));
  CHK(sync_read(c, G, c->d_G, sizeof(double) * c->N * c->N));
  return POU_OK;
}

// The trial point W - tau Z of U (Z from H(rho(U)), evaluated afresh) and its
// Gram, through the kernels a step's first orthonormalisation pass uses.
template <typename T>
pou_status trial_point_impl(pou_ctx *c, const T *U, double tau, T *Wt, double *G) {
  hipStream_t s = c->stream;
  CHK(energy_impl<T>(c, U, nullptr));
  const double *rep = (c->eval_HU == c->d_HW) ? c->d_rep[0] : c->d_rep[1];
  c->h_step[0] = tau;  // pinned: the copy reads it after the synchronisation above
  HIPCHK(c, hipMemcpyAsync(c->d_diag, c->h_step, sizeof(double), hipMemcpyHostToDevice, s));
  const bool bf16 = sizeof(T) == 4 && c->p.orth_passes == 2;
  if (c->N <= 128) {
    KL(POU_K_TRIAL, pou::launch_trial_gram<T>(U, (const T *)c->eval_HU, rep, c->d_diag, 1.0,
                                              (T *)c->d_Wt, c->N, c->ng, c->nsplit, bf16,
                                              c->d_gpart, s));
    KL(POU_K_CHOLESKY, pou::launch_gram_reduce(c->d_gpart, c->N, c->nsplit, c->dv, c->d_G, s));
  } else {
    KL(POU_K_TRIAL, pou::launch_trial<T>(U, (const T *)c->eval_HU, rep, c->d_diag, 1.0,
                                         (T *)c->d_Wt, c->N, c->ng, s));
    CHK(gram<T>(c, (const T *)c->d_Wt, bf16));
  }
  if (Wt)
    HIPCHK(c, hipMemcpyAsync(Wt, c->d_Wt, sizeof(T) * (size_t)c->N * c->ng,
                             hipMemcpyDeviceToDevice, s));
  if (G) CHK(sync_read(c, G, c->d_G, sizeof(double) * c->N * c->N));
  else {
    HIPCHK(c, hipStreamSynchronize(s));
    prof_drain(c);
  }
  return POU_OK;
}

// ---------------------------------------------------------------- non-allocating Gram
//
// Scratch of pou_gram_static: the Gram partials [kStaticSplits][128][128] of
// up to 128 orbitals, 32 MiB per device, held until the process ends.  In host
// code `scratch` names a host-side stand-in: kernels get the device address
// that hipGetSymbolAddress returns on each device.
constexpr int kStaticSplits = 256;
constexpr int kStaticMaxOrb = 128;
static __device__ __align__(256) double scratch[(size_t)kStaticSplits * 128 * 128];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved once per device).
hipError_t scratch_address(double **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

// ====================================================================== ABI

extern "C" {

void pou_default_params(pou_params *p) {
  if (!p) return;
  p->rho1 = 1e-4;
  p->delta = 0.1;
  p->eta = 0.85;
  p->bb_mode = 0;
  p->tau_init = 0.0;
  p->s_max = 10;
  p->orth_passes = 0;
  p->cg_rtol = 0.0;
  p->cg_maxit = 0;
  p->cg_precond = 1;
  p->terms = POU_TERM_ALL;
  p->n_org = 1;
  p->n_diag = 0;
}

pou_status pou_create(pou_ctx **out, int device, void *hip_stream) {
  if (!out) return POU_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return POU_ERR_ARG;
  }
  pou_ctx *c = new pou_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return POU_ERR_HIP;
  }
  *out = c;
  return POU_OK;
}

pou_status pou_destroy(pou_ctx *c) {
  if (!c) return POU_ERR_ARG;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_all(c);
  prof_drain(c);
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  delete c;
  return POU_OK;
}

const char *pou_last_error(const pou_ctx *c) { return c ? c->err.c_str() : "null context"; }

pou_status pou_set_system(pou_ctx *c, const pou_grid *grid, int natoms, const double *R,
                          const double *Z, const double *sigma, int norb, const double *occ,
                          pou_precision prec, const pou_params *params) {
  if (!c) return POU_ERR_ARG;
  if (!grid || !occ) return fail(c, POU_ERR_ARG, "null grid or occupation pointer");
  if (grid->n < 9 || grid->n > 1024) return fail(c, POU_ERR_ARG, "grid n must be in [9, 1024]");
  if (!(grid->L > 0.0) || !std::isfinite(grid->L)) return fail(c, POU_ERR_ARG, "box side L must be > 0");
  const i64 ng = (i64)grid->n * grid->n * grid->n;
  if (norb < 1 || norb > 512 || (i64)norb > ng)
    return fail(c, POU_ERR_ARG, "norb must be in [1, min(512, n^3)]");
  if (natoms < 0 || (natoms > 0 && (!R || !Z || !sigma)))
    return fail(c, POU_ERR_ARG, "bad atom arrays");
  if (prec != POU_FP64 && prec != POU_MIXED) return fail(c, POU_ERR_ARG, "bad precision");
  for (int I = 0; I < natoms; ++I) {
    if (!(sigma[I] > 0.0) || !std::isfinite(sigma[I]) || !std::isfinite(Z[I]) ||
        !std::isfinite(R[3 * I]) || !std::isfinite(R[3 * I + 1]) || !std::isfinite(R[3 * I + 2]))
      return fail(c, POU_ERR_ARG, "atom " + std::to_string(I) + ": bad position, charge or width");
  }
  for (int i = 0; i < norb; ++i)
    if (!(occ[i] >= 0.0) || !std::isfinite(occ[i]))
      return fail(c, POU_ERR_ARG, "occupations must be finite and >= 0");
  pou_params p;
  if (params) p = *params;
  else pou_default_params(&p);
  const double h = grid->L / grid->n;
  if (p.tau_init <= 0.0) {
    // 1 / lambda_max(K): K = -1/2 Lap has its largest eigenvalue at theta = pi on every axis
    p.tau_init = 1.0 / (1.5 * lambda1(2, h, 1));  // lambda1(2, h, 1) is the symbol at theta = pi
  }
  if (p.orth_passes <= 0) p.orth_passes = (prec == POU_FP64) ? 1 : 2;
  if (p.cg_rtol <= 0.0) p.cg_rtol = 1e-12;
  if (p.cg_maxit <= 0) p.cg_maxit = 2000;
  if (p.n_org <= 0) p.n_org = 1;
  if (!(p.delta > 0.0 && p.delta < 1.0) || !(p.rho1 >= 0.0) || !(p.eta >= 0.0 && p.eta <= 1.0) ||
      p.s_max < 0 || p.s_max > 60 || p.orth_passes > 2 || p.bb_mode < 0 || p.bb_mode > 2 ||
      !std::isfinite(p.tau_init) || p.n_diag < 0 || (p.terms & ~63u) != 0)
    return fail(c, POU_ERR_ARG, "bad algorithm parameters");
  if (p.n_diag > 0)
    for (int i = 1; i < norb; ++i)
      if (occ[i] != occ[0])
        return fail(c, POU_ERR_ARG, "subspace diagonalisation (n_diag > 0) needs equal occupations");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, POU_ERR_HIP, "hipSetDevice failed");
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_all(c);

  c->n = grid->n;
  c->L = grid->L;
  c->h = h;
  c->dv = h * h * h;
  c->ng = ng;
  c->N = norb;
  c->M = natoms;
  c->prec = prec;
  c->p = p;
  c->es = (prec == POU_FP64) ? 8 : 4;
  c->occ.assign(occ, occ + norb);
  c->atoms.assign(5 * (size_t)natoms, 0.0);
  for (int I = 0; I < natoms; ++I) {
    for (int a = 0; a < 3; ++a) c->atoms[5 * I + a] = R[3 * I + a];
    c->atoms[5 * I + 3] = Z[I];
    c->atoms[5 * I + 4] = sigma[I];
  }
  // launch shapes
  const int tiles = (c->n + pou::kTX - 1) / pou::kTX;
  c->st.n = c->n;
  c->st.inv_h2 = 1.0 / (h * h);
  c->st.ntile = tiles * tiles;
  int nzc = (int)std::ceil(2048.0 / ((double)c->st.ntile * norb));
  nzc = std::max(1, std::min(nzc, c->n / 8));
  c->st.zlen = (c->n + nzc - 1) / nzc;
  c->st.nzc = (c->n + c->st.zlen - 1) / c->st.zlen;
  c->nblk_field = (int)std::min<i64>(1024, (ng + 255) / 256);
  c->nblk_orb = (int)std::max<i64>(1, std::min<i64>(64, ng / 16384));
  // the accept kernel streams five blocks: more workgroups per orbital (128 at
  // 96^3) keep more of its accesses in flight
  c->nblk_commit = (int)std::max<i64>(1, std::min<i64>(128, ng / 4096));
  c->nsplit = (int)std::max<i64>(1, std::min<i64>(pou::gram_split(norb, c->es == 4), (ng + 31) / 32));

  const size_t fbytes = sizeof(double) * (size_t)ng;
  const size_t bbytes = c->es * (size_t)ng * norb;
  CHK(dalloc(c, &c->d_occ, sizeof(double) * norb));
  CHK(dalloc(c, &c->d_atoms, sizeof(double) * std::max<size_t>(1, c->atoms.size())));
  CHK(dalloc(c, &c->d_rho, fbytes));
  CHK(dalloc(c, &c->d_vh, fbytes));
  CHK(dalloc(c, &c->d_vext, fbytes));
  CHK(dalloc(c, &c->d_veff, fbytes));
  CHK(dalloc(c, &c->d_veff32, sizeof(float) * (size_t)ng));
  CHK(dalloc(c, &c->d_rhoion, fbytes));
  CHK(dalloc(c, &c->d_lam1, sizeof(double) * c->n));
  CHK(dalloc(c, &c->d_cg_r, fbytes));
  CHK(dalloc(c, &c->d_cg_p, fbytes));
  CHK(dalloc(c, &c->d_cg_q, fbytes));
  CHK(dalloc(c, &c->d_cg_z, fbytes));
  CHK(dalloc(c, &c->d_fft0, 2 * fbytes));
  CHK(dalloc(c, &c->d_fft1, 2 * fbytes));
  CHK(dalloc(c, &c->d_sc, sizeof(double) * 16));
  c->part_len = std::max<size_t>({(size_t)2 * norb * c->st.ntile * c->st.nzc,
                                  (size_t)4 * c->nblk_field, (size_t)4 * norb * c->nblk_orb,
                                  (size_t)4 * norb * c->nblk_commit,
                                  (size_t)4 * std::max(1, natoms) * 256, (size_t)16});
  CHK(dalloc(c, &c->d_part, sizeof(double) * c->part_len));
  CHK(dalloc(c, &c->d_gpart, sizeof(double) * pou::gram_partial_doubles(norb, c->nsplit)));
  CHK(dalloc(c, &c->d_D64, sizeof(double) * (size_t)norb * norb));
  CHK(dalloc(c, &c->d_D32, sizeof(float) * (size_t)norb * norb));
  if (c->es == 4 && norb > 128)
    CHK(dalloc(c, &c->d_fsplit, 2 * sizeof(uint16_t) * pou::split_factor_elems(norb)));
  if (norb > 128)
    CHK(dalloc(c, &c->d_rhopart, sizeof(double) * (size_t)((norb + 127) / 128) * c->ng));
  if (pou::chol_workspace_doubles(norb) > 0)
    CHK(dalloc(c, &c->d_cholws, sizeof(double) * pou::chol_workspace_doubles(norb)));
  CHK(dalloc(c, &c->d_G, sizeof(double) * (size_t)norb * norb));
  CHK(dalloc(c, &c->d_S, sizeof(double) * (size_t)norb * norb));
  CHK(dalloc(c, &c->d_P, sizeof(double) * (size_t)norb * norb));
  CHK(dalloc(c, &c->d_xpart, sizeof(double) * pou::cross_partial_doubles(norb)));
  CHK(dalloc(c, &c->d_Minv, sizeof(double) * (size_t)norb * norb));
  CHK(dalloc(c, &c->d_Minv2, sizeof(double) * (size_t)norb * norb));
  CHK(dalloc(c, &c->d_Mcomb, sizeof(double) * (size_t)norb * norb));
  CHK(dalloc(c, &c->d_red, sizeof(double) * (size_t)std::max(4 * norb, 4 * std::max(1, natoms)) + 64));
  CHK(dalloc(c, &c->d_scal, sizeof(double) * 8));
  CHK(dalloc(c, &c->d_diag, sizeof(double) * 8));
  // each report is followed by 8 doubles: step scalars and the accept flags
  CHK(dalloc(c, &c->d_rep[0], sizeof(double) * (Report::size(norb) + 8)));
  CHK(dalloc(c, &c->d_rep[1], sizeof(double) * (Report::size(norb) + 8)));
  if (hipHostMalloc((void **)&c->h_step, sizeof(double) * (Report::size(norb) + 10)) !=
      hipSuccess) {
    (void)hipGetLastError();
    c->h_step = nullptr;
    return fail(c, POU_ERR_OOM, "pinned host buffer for the step report");
  }
  CHK(dalloc(c, &c->d_HW, bbytes));
  CHK(dalloc(c, &c->d_HWt, bbytes));
  CHK(dalloc(c, &c->d_Wt, bbytes));
  CHK(dalloc(c, &c->d_W1, bbytes));
  CHK(dalloc(c, &c->d_W2, bbytes));

  hipStream_t s = c->stream;
  std::vector<double> lam(c->n);
  for (int k = 0; k < c->n; ++k) lam[k] = lambda1(c->n, h, k);
  HIPCHK(c, hipMemcpyAsync(c->d_lam1, lam.data(), sizeof(double) * c->n, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_occ, c->occ.data(), sizeof(double) * norb, hipMemcpyHostToDevice, s));
  if (natoms > 0)
    HIPCHK(c, hipMemcpyAsync(c->d_atoms, c->atoms.data(), sizeof(double) * c->atoms.size(),
                             hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemsetAsync(c->d_vh, 0, fbytes, s));
  HIPCHK(c, hipMemsetAsync(c->d_vext, 0, fbytes, s));
  HIPCHK(c, hipMemsetAsync(c->d_rep[0], 0, sizeof(double) * Report::size(norb), s));
  HIPCHK(c, hipMemsetAsync(c->d_rep[1], 0, sizeof(double) * Report::size(norb), s));
  // V_ext = -P[rho_ion]: the periodic, background-neutralised potential of the
  // Gaussian ion charges
  if (natoms > 0 && (p.terms & POU_TERM_EXT)) {
    KL(POU_K_OTHER, pou::launch_ion_density(c->d_atoms, natoms, c->d_rhoion, c->n, c->L, s));
    int it = 0;
    CHK(poisson(c, c->d_rhoion, c->d_vext, 1e-13, std::max(p.cg_maxit, 4000), p.cg_precond != 0,
                &it));
    KL(POU_K_POISSON, pou::launch_scale(c->d_vext, -1.0, ng, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  prof_drain(c);
  c->have_system = true;
  c->last_U = nullptr;
  c->cur_valid = false;
  c->hist = false;
  c->eval_ptr = nullptr;
  c->l = 0;
  return POU_OK;
}

#define NEED_SYSTEM(c)                                                        \
  do {                                                                        \
    if (!(c)) return POU_ERR_ARG;                                             \
    if (!(c)->have_system) return fail((c), POU_ERR_STATE, "call pou_set_system first"); \
    if (hipSetDevice((c)->device) != hipSuccess) return fail((c), POU_ERR_HIP, "hipSetDevice failed"); \
  } while (0)

pou_status pou_set_projectors(pou_ctx *c, const double *params) {
  NEED_SYSTEM(c);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (void *p : c->nl_allocs) (void)hipFree(p);
  c->nl_allocs.clear();
  c->nl_ions.clear();
  c->nl_col_off.clear();
  c->nl_col_cnt.clear();
  c->nl_on = false;
  c->d_nl = nullptr;
  c->d_nl_list = nullptr;
  c->d_nlpart = c->d_nlC = c->d_nlC2 = c->d_nlD = nullptr;
  c->p.terms &= ~(unsigned)POU_TERM_NLOC;
  c->cur_valid = false;  // cached H W no longer describes H
  c->eval_ptr = nullptr;
  if (!params || c->M == 0) return POU_OK;
  const int M = c->M, n = c->n;
  for (int I = 0; I < M; ++I) {
    const double rc = params[3 * I], bs = params[3 * I + 1], bp = params[3 * I + 2];
    if (!(rc > 0.0) || !std::isfinite(rc) || !std::isfinite(bs) || !std::isfinite(bp))
      return fail(c, POU_ERR_ARG, "projector " + std::to_string(I) + ": bad width or amplitude");
  }
  // cube: half width reaching the radius where exp(-r^2 / (2 rc^2)) < 1e-14
  const double tail = std::sqrt(2.0 * std::log(1e14));
  c->nl_ions.resize(M);
  c->nl_bmax = 1;
  for (int I = 0; I < M; ++I) {
    pou::NlIon a{};
    for (int k = 0; k < 3; ++k) a.R[k] = c->atoms[5 * I + k];
    a.rc = params[3 * I];
    a.bs = params[3 * I + 1];
    a.bp = params[3 * I + 2];
    const int hw = (int)std::ceil(tail * a.rc / c->h);
    a.b = 2 * hw + 1;
    for (int k = 0; k < 3; ++k) {
      if (a.b >= n) {
        a.o[k] = 0;
      } else {
        long long ctr = std::llround(a.R[k] / c->h);
        a.o[k] = (int)(((ctr - hw) % n + n) % n);
      }
    }
    if (a.b >= n) a.b = n;
    c->nl_bmax = std::max(c->nl_bmax, a.b);
    c->nl_ions[I] = a;
  }
  // greedy colouring: cubes of one colour share no grid point
  auto overlap1 = [n](int o1, int b1, int o2, int b2) {
    return ((o2 - o1) % n + n) % n < b1 || ((o1 - o2) % n + n) % n < b2;
  };
  std::vector<int> colour(M, -1);
  std::vector<std::vector<int>> cols;
  for (int I = 0; I < M; ++I) {
    const pou::NlIon &a = c->nl_ions[I];
    int k = 0;
    for (; k < (int)cols.size(); ++k) {
      bool clash = false;
      for (int J : cols[k]) {
        const pou::NlIon &b = c->nl_ions[J];
        if (overlap1(a.o[0], a.b, b.o[0], b.b) && overlap1(a.o[1], a.b, b.o[1], b.b) &&
            overlap1(a.o[2], a.b, b.o[2], b.b)) {
          clash = true;
          break;
        }
      }
      if (!clash) break;
    }
    if (k == (int)cols.size()) cols.emplace_back();
    cols[k].push_back(I);
  }
  std::vector<int> list;
  for (auto &cl : cols) {
    c->nl_col_off.push_back((int)list.size());
    c->nl_col_cnt.push_back((int)cl.size());
    list.insert(list.end(), cl.begin(), cl.end());
  }
  auto nalloc = [c](void **p, size_t bytes) -> pou_status {
    if (hipMalloc(p, bytes ? bytes : 8) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, POU_ERR_OOM, "hipMalloc of the projector buffers failed");
    }
    c->nl_allocs.push_back(*p);
    return POU_OK;
  };
  const int N = c->N;
  const size_t nsp = (size_t)pou::nl_splits(c->nl_bmax);
  CHK(nalloc((void **)&c->d_nl, sizeof(pou::NlIon) * M));
  CHK(nalloc((void **)&c->d_nl_list, sizeof(int) * M));
  CHK(nalloc((void **)&c->d_nlpart, sizeof(double) * (size_t)M * nsp * N * 12));
  CHK(nalloc((void **)&c->d_nlC, sizeof(double) * (size_t)4 * M * N));
  CHK(nalloc((void **)&c->d_nlC2, sizeof(double) * (size_t)4 * M * N));
  CHK(nalloc((void **)&c->d_nlD, sizeof(double) * (size_t)12 * M * N));
  HIPCHK(c, hipMemcpyAsync(c->d_nl, c->nl_ions.data(), sizeof(pou::NlIon) * M,
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_nl_list, list.data(), sizeof(int) * M, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->nl_on = true;
  c->p.terms |= POU_TERM_NLOC;
  return POU_OK;
}

pou_status pou_energy(pou_ctx *c, const void *U, pou_energy_terms *out) {
  NEED_SYSTEM(c);
  if (!U) return fail(c, POU_ERR_ARG, "null U");
  if (c->prec == POU_FP64) return energy_impl<double>(c, (const double *)U, out);
  return energy_impl<float>(c, (const float *)U, out);
}

pou_status pou_residual(pou_ctx *c, const void *U, double *resid, double *Sigma) {
  NEED_SYSTEM(c);
  if (!U) return fail(c, POU_ERR_ARG, "null U");
  if (c->prec == POU_FP64) return residual_impl<double>(c, (const double *)U, resid, Sigma);
  return residual_impl<float>(c, (const float *)U, resid, Sigma);
}

pou_status pou_orthonormalize(pou_ctx *c, void *U, double *orth_err) {
  NEED_SYSTEM(c);
  if (!U) return fail(c, POU_ERR_ARG, "null U");
  if (c->prec == POU_FP64) return orthonormalize_impl<double>(c, (double *)U, orth_err);
  return orthonormalize_impl<float>(c, (float *)U, orth_err);
}

pou_status pou_orbital_update_step(pou_ctx *c, void *U, pou_step_info *out) {
  NEED_SYSTEM(c);
  if (!U) return fail(c, POU_ERR_ARG, "null U");
  if (c->prec == POU_FP64) return step_impl<double>(c, (double *)U, out);
  return step_impl<float>(c, (float *)U, out);
}

pou_status pou_energy_backward(pou_ctx *c, const void *U, double gE, void *dU, double *dR,
                               double *dsigma) {
  NEED_SYSTEM(c);
  if (!U) return fail(c, POU_ERR_ARG, "null U");
  if (!std::isfinite(gE)) return fail(c, POU_ERR_ARG, "gE must be finite");
  if (c->prec == POU_FP64)
    return backward_impl<double>(c, (const double *)U, gE, (double *)dU, dR, dsigma);
  return backward_impl<float>(c, (const float *)U, gE, (float *)dU, dR, dsigma);
}

pou_status pou_hamiltonian_apply(pou_ctx *c, const void *U, void *HU, double *sigma) {
  NEED_SYSTEM(c);
  if (!U || !HU) return fail(c, POU_ERR_ARG, "null U or HU");
  if (c->eval_ptr == nullptr && !c->cur_valid)
    return fail(c, POU_ERR_STATE, "no potentials yet: call pou_energy first");
  if (c->prec == POU_FP64) return hamiltonian_impl<double>(c, (const double *)U, (double *)HU, sigma);
  return hamiltonian_impl<float>(c, (const float *)U, (float *)HU, sigma);
}

pou_status pou_get_fields(pou_ctx *c, double *rho, double *vh, double *veff, double *vext) {
  NEED_SYSTEM(c);
  const size_t b = sizeof(double) * (size_t)c->ng;
  if (rho) HIPCHK(c, hipMemcpyAsync(rho, c->d_rho, b, hipMemcpyDeviceToDevice, c->stream));
  if (vh) HIPCHK(c, hipMemcpyAsync(vh, c->d_vh, b, hipMemcpyDeviceToDevice, c->stream));
  if (veff) HIPCHK(c, hipMemcpyAsync(veff, c->d_veff, b, hipMemcpyDeviceToDevice, c->stream));
  if (vext) HIPCHK(c, hipMemcpyAsync(vext, c->d_vext, b, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return POU_OK;
}

pou_status pou_gram(pou_ctx *c, const void *U, int mode, double *G) {
  NEED_SYSTEM(c);
  if (!U || !G) return fail(c, POU_ERR_ARG, "null U or G");
  if (mode != POU_GRAM_ACCURATE && mode != POU_GRAM_BF16)
    return fail(c, POU_ERR_ARG, "bad Gram mode");
  if (mode == POU_GRAM_BF16 && c->prec == POU_FP64)
    return fail(c, POU_ERR_ARG, "the BF16 Gram needs FP32 orbitals (POU_MIXED)");
  if (c->prec == POU_FP64) return gram_impl<double>(c, (const double *)U, mode, G);
  return gram_impl<float>(c, (const float *)U, mode, G);
}

pou_status pou_trial_point(pou_ctx *c, const void *U, double tau, void *Wt, double *G) {
  NEED_SYSTEM(c);
  if (!U) return fail(c, POU_ERR_ARG, "null U");
  if (!std::isfinite(tau)) return fail(c, POU_ERR_ARG, "tau must be finite");
  if (c->prec == POU_FP64)
    return trial_point_impl<double>(c, (const double *)U, tau, (double *)Wt, G);
  return trial_point_impl<float>(c, (const float *)U, tau, (float *)Wt, G);
}

pou_status pou_gram_static(const void *U, int prec, int mode, int norb, long long ng, double dv,
                           double *G, void *hip_stream) {
  if (!U || !G) return POU_ERR_ARG;
  if (prec != POU_FP64 && prec != POU_MIXED) return POU_ERR_ARG;
  if (mode != POU_GRAM_ACCURATE && mode != POU_GRAM_BF16) return POU_ERR_ARG;
  if (mode == POU_GRAM_BF16 && prec != POU_MIXED) return POU_ERR_ARG;
  if (norb < 1 || norb > kStaticMaxOrb || ng < norb || !(dv > 0.0) || !std::isfinite(dv))
    return POU_ERR_ARG;
  double *part = nullptr;
  if (scratch_address(&part) != hipSuccess) {
    (void)hipGetLastError();
    return POU_ERR_HIP;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const int nsplit = (int)std::max<i64>(1, std::min<i64>(kStaticSplits, (ng + 31) / 32));
  hipError_t e;
  if (prec == POU_FP64)
    e = pou::launch_gram_partial<double>((const double *)U, norb, ng, nsplit, part, s);
  else if (mode == POU_GRAM_BF16)
    e = pou::launch_gram_partial_bf16((const float *)U, norb, ng, nsplit, part, s);
  else
    e = pou::launch_gram_partial<float>((const float *)U, norb, ng, nsplit, part, s);
  if (e == hipSuccess) e = pou::launch_gram_reduce(part, norb, nsplit, dv, G, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return POU_ERR_HIP;
  }
  return POU_OK;
}

pou_status pou_convert(pou_ctx *c, const void *src, int src_prec, void *dst, int dst_prec,
                       long long count) {
  if (!c) return POU_ERR_ARG;
  if (!src || !dst || count < 0) return fail(c, POU_ERR_ARG, "bad convert arguments");
  if ((src_prec != POU_FP64 && src_prec != POU_MIXED) || (dst_prec != POU_FP64 && dst_prec != POU_MIXED))
    return fail(c, POU_ERR_ARG, "bad precision code");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, POU_ERR_HIP, "hipSetDevice failed");
  hipStream_t s = c->stream;
  if (src_prec == POU_MIXED && dst_prec == POU_FP64)
    KL(POU_K_OTHER, (pou::launch_convert<float, double>((const float *)src, (double *)dst, count, s)));
  else if (src_prec == POU_FP64 && dst_prec == POU_MIXED)
    KL(POU_K_OTHER, (pou::launch_convert<double, float>((const double *)src, (float *)dst, count, s)));
  else if (src_prec == POU_FP64)
    KL(POU_K_OTHER, (pou::launch_convert<double, double>((const double *)src, (double *)dst, count, s)));
  else
    KL(POU_K_OTHER, (pou::launch_convert<float, float>((const float *)src, (float *)dst, count, s)));
  HIPCHK(c, hipStreamSynchronize(s));
  prof_drain(c);
  return POU_OK;
}

pou_status pou_profile_enable(pou_ctx *c, unsigned group_mask) {
  if (!c) return POU_ERR_ARG;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  prof_drain(c);
  c->prof_mask = group_mask & POU_PROFILE_ALL;
  for (int k = 0; k < POU_K_COUNT; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  return POU_OK;
}

pou_status pou_profile_read(pou_ctx *c, int group, double *total_ms, long long *launches) {
  if (!c) return POU_ERR_ARG;
  if (group < 0 || group >= POU_K_COUNT) return fail(c, POU_ERR_ARG, "bad kernel group");
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  prof_drain(c);
  if (total_ms) *total_ms = c->prof_ms[group];
  if (launches) *launches = c->prof_n[group];
  return POU_OK;
}

pou_status pou_reset_history(pou_ctx *c) {
  if (!c) return POU_ERR_ARG;
  c->hist = false;
  c->cur_valid = false;
  c->l = 0;
  return POU_OK;
}

}  // extern "C"
