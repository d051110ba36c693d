// Internal declarations shared by the HIP sources of the library.
// Kernels are launched through the host-side wrappers declared here; every
// wrapper enqueues on the given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <algorithm>
#include <cstdint>
#include <cstddef>

namespace pou {

using i64 = long long;

// Threads per workgroup used by the field / block kernels.
constexpr int kBlock = 256;
// Stencil tile: 32 (x) by 32 (y) points per workgroup, 8 thread rows each
// handling 4 y points; radius-4 halo.
constexpr int kTX = 32;
constexpr int kTY = 32;
constexpr int kRad = 4;

struct FD8 {
  // central 8th-order second-derivative weights for offsets 1..4 (offset 0
  // weight is minus twice their sum, so the operator annihilates constants)
  static constexpr double c1 = 8.0 / 5.0;
  static constexpr double c2 = -1.0 / 5.0;
  static constexpr double c3 = 8.0 / 315.0;
  static constexpr double c4 = -1.0 / 560.0;
};

// ---------------------------------------------------------------- reductions

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline float wave_sum(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Sum of K values per thread over a 256-thread workgroup, deterministic order.
// Result valid in thread 0 (out[k]).  scratch must hold 4*K doubles.
template <int K>
__device__ inline void block_sum(double (&v)[K], double *scratch) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) scratch[wave * K + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += scratch[w * K + k];
      v[k] = s;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- launchers
// Grid / block kernels (grid_kernels.hip)

struct StencilArgs {
  int n;          // points per axis
  double inv_h2;  // 1 / h^2
  int ntile;      // tiles per plane = ceil(n/32)^2
  int nzc;        // z chunks per orbital
  int zlen;       // planes per chunk
};

// HU = -1/2 Lap U + veff * U for N orbitals; per (orbital, tile, zchunk)
// partial sums of <u, H u> and <u, K u> (unscaled by h^3) into part[2*(o*nb + b) + {0,1}].
template <typename T>
hipError_t launch_hamiltonian(const T *U, const T *veff, T *HU, double *part, int N,
                              const StencilArgs &a, hipStream_t s);

// rho[g] = sum_i occ_i u_i[g]^2 (FP64 accumulation)
template <typename T>
hipError_t launch_density(const T *U, const double *occ, double *rho, int N, i64 ng,
                          hipStream_t s);

// xc + effective potential + energy partials.  part[4*b + {0,1,2,3}] =
// partial sums of (rho^(4/3), rho*vext, rho*vh, rho*eps_c).  veff32 nullable.
hipError_t launch_xc_veff(const double *rho, const double *vh, const double *vext,
                          double *veff, float *veff32, double *part, i64 ng,
                          unsigned terms, int nblk, hipStream_t s);

// out[k*nseg + seg] = scale * sum_j part[(seg*len + j)*K + k], j < len (deterministic)
hipError_t launch_segment_sum(const double *part, double *out, int nseg, int len, int K,
                              double scale, hipStream_t s);

// ---- Poisson (conjugate gradients) on one FP64 field
// q = -Lap p  and part[b] = partial of p.q
hipError_t launch_neg_lap(const double *p, double *q, double *part, int n, double inv_h2,
                          int nblk, hipStream_t s);
// b = 4 pi (rho - mean), mean read from dmean[0]; r = b - q (q = A x);
// part[2b] = r.r partial, part[2b+1] = b.b partial
hipError_t launch_cg_rhs_residual(const double *rho, const double *dmean, const double *q,
                                  double *r, double *part, i64 ng, int nblk, hipStream_t s);
// scalar dot / norm partials of two fields
hipError_t launch_dot2(const double *a, const double *b, double *part, i64 ng, int nblk,
                       hipStream_t s);
// p = z + beta p (beta = num[0]/den[0], or 0 when first != 0)
hipError_t launch_cg_update_p(double *p, const double *z, const double *num, const double *den,
                              int first, i64 ng, hipStream_t s);
// x += alpha p; r -= alpha q; alpha = num[0]/den[0]; part = r.r partial
hipError_t launch_cg_update_xr(double *x, double *r, const double *p, const double *q,
                               const double *num, const double *den, double *part, i64 ng,
                               int nblk, hipStream_t s);
// x *= a
hipError_t launch_scale(double *x, double a, i64 ng, hipStream_t s);
// dst = src - mean(src) with mean from dmean (used to fix the gauge)
hipError_t launch_remove_mean(double *x, const double *dmean, i64 ng, hipStream_t s);
// Spectral inverse of -Lap: out = scale * (-Lap)^+ r (zero mean) by 3-D FFT,
// exact for the FD8 operator; sum_r (nullable) receives sum_g r_g, the mean
// mode of the forward transform.
hipError_t launch_spectral_inverse(const double *r, double *out, double2 *w0, double2 *w1,
                                   const double *lam1, int n, double scale, hipStream_t s,
                                   double *sum_r = nullptr);
// Lines of the FFT per workgroup for an n-point axis: 8, or the largest
// divisor of n in 4..7 so that no workgroup holds a ragged batch (measured at
// 96^3: 8 lines 5% faster than 10 with a ragged last batch; 16 and 20 slower,
// fewer workgroups), reduced until the dynamic LDS of fft_lds_bytes fits in
// kFftLdsMax.  Returns 0 if not even one line fits (n > 1365).
constexpr size_t kFftLdsMax = 65536;
__host__ __device__ constexpr size_t fft_lds_bytes(int n, int lb) {
  return (size_t)(2 * lb + 1) * (size_t)n * 16;  // two line buffers + twiddle table (double2)
}
__host__ __device__ constexpr int fft_lines_per_group(int n) {
  int cap = 8;
  while (cap > 0 && fft_lds_bytes(n, cap) > kFftLdsMax) --cap;
  if (cap == 0) return 0;
  for (int d = cap; d >= 4; --d)
    if (n % d == 0) return d < n ? d : n;
  return cap < n ? cap : n;
}
hipError_t launch_poisson_residual(const double *x, const double *rho, const double *dsum,
                                   double *part, int n, double inv_h2, int nblk, hipStream_t s);

// ---- block elementwise / reductions
// Wt = (1 + tau sig_i) W - tau HW with tau = dtau[0] * tscale
template <typename T>
hipError_t launch_trial(const T *W, const T *HW, const double *sig, const double *dtau,
                        double tscale, T *Wt, int N, i64 ng, hipStream_t s);
// Barzilai-Borwein step on the device: out = (tau_BB, zz, ss, sy, yy); does
// nothing when gate is non-null and gate[0] == 0.  mode 0: tau_init and the zz
// of red[0..N); 1, 2: tau1 / tau2 from red[0..4N); 3: only out[1] = zz of red[0..N)
hipError_t launch_bb_tau(const double *red, int N, int mode, double tau_init, double *out,
                         const double *gate, hipStream_t s);
// device test of eq. "ene-de" for a trial report: ext[0..4] = scal, ext[5] = accept,
// ext[6] = inequality held
hipError_t launch_armijo(const double *rep, const double *occ, int N, unsigned terms, int npass,
                         int orth_off, int rr_off, double rtol2, const double *scal,
                         double tscale, double C, double rho1, int force, double *ext,
                         hipStream_t s);
hipError_t launch_set_flags(double *flags, double a, double b, hipStream_t s);
// accept: U <- Wn; partials per (orbital, block) of
//   s.s, s.y, y.y, zn.zn  with s = Wn - W, y = zn - z,
//   z = HW - sig W, zn = HWn - sign Wn
// (nothing when gate is non-null and gate[0] == 0)
template <typename T>
hipError_t launch_commit(T *U, const T *HW, const double *sig, const T *Wn, const T *HWn,
                         const double *sign, double *part, int N, i64 ng, int nblk,
                         const double *gate, hipStream_t s);
// per (orbital, block) partials of <a_i, b_i> or, with diff, |a_i - b_i|^2
template <typename T>
hipError_t launch_rowdot(const T *A, const T *B, bool diff, double *part, int N, i64 ng, int nblk,
                         hipStream_t s);
// z.z partials for z = HW - sig W
template <typename T>
hipError_t launch_zz(const T *W, const T *HW, const double *sig, double *part, int N,
                     i64 ng, int nblk, hipStream_t s);
// dU = gE * 2 occ_i dv * HU
template <typename T>
hipError_t launch_backward_scale(const T *HU, const double *occ, double scale, T *dU,
                                 int N, i64 ng, hipStream_t s);
template <typename S, typename D>
hipError_t launch_convert(const S *src, D *dst, i64 count, hipStream_t s);
// non-finite check: flag[0] |= 1 if any element is NaN/Inf
template <typename T>
hipError_t launch_nonfinite(const T *x, i64 count, int *flag, hipStream_t s);

// ---- ions
hipError_t launch_ion_density(const double *atoms, int M, double *rho_ion, int n, double L,
                              hipStream_t s);
// part[((I*nblk)+b)*4 + {0..3}] partial sums for dE/dR_{x,y,z}, dE/dsigma
hipError_t launch_ion_forces(const double *atoms, int M, const double *vh, double *part,
                             int n, double L, int nblk, hipStream_t s);

// ---- dense (dense_kernels.hip)
// Partial Gram of A [N][ng]: see gram.  part holds nsplit * nblkpairs * 64*64 doubles.
template <typename T>
hipError_t launch_gram_partial(const T *A, int N, i64 ng, int nsplit, double *part,
                               hipStream_t s);
// Pass-1 BF16 Gram of FP32 data (products of BF16-rounded values, FP32 accumulation
// flushed to FP64).
hipError_t launch_gram_partial_bf16(const float *A, int N, i64 ng, int nsplit, double *part,
                                    hipStream_t s);
// Trial point and Gram in one pass: Wt = (1 + tau sig_i) W - tau HW is written
// and its partial Gram accumulated (N <= 128; HW == nullptr: plain Gram of W).
// bf16: products of BF16-rounded FP32 values (first Cholesky-QR pass).
template <typename T>
hipError_t launch_trial_gram(const T *W, const T *HW, const double *sig, const double *dtau,
                             double tscale, T *Wt, int N, i64 ng, int nsplit, bool bf16,
                             double *part, hipStream_t s);
// First Cholesky-QR pass fused with the second Gram (FP32, N <= 128): the
// partial Gram of W1 = X + D~ X over nsplit workgroups into part (nothing else
// written), D~ the BF16 hi/lo split of D32, X in hi/lo pieces.  W1 enters the
// Gram as three BF16 pieces, so the Gram is that of the on-chip W1 to FP32
// accuracy; with two pieces (16 bits) the representation's residual leaves
// the diagonal off by ~1e-7 for localised orbitals, and with it the
// orthonormality of the block the combined factor produces.
hipError_t launch_apply_gram(const float *D32, const float *X, int N, i64 ng, int nsplit,
                             double *part, hipStream_t s);
// M = A B (lower-triangular), D64 = M - I, D32 = (float) D64; with split_b, B is
// taken as I + the BF16 hi/lo split of (float)(B - I) (the first factor as the
// fused mixed-precision apply uses it)
hipError_t launch_combine_factors(const double *A, const double *B, double *M, double *D64,
                                  float *D32, int N, bool split_b, hipStream_t s);
// G = dv * sum of partials (full symmetric N x N)
hipError_t launch_gram_reduce(const double *part, int N, int nsplit, double dv, double *G,
                              hipStream_t s);
// Cholesky G = L L^T and Minv = L^-1 (lower), plus D = Minv - I in FP64 and
// FP32; outs (CHOL_OUT_* bits) names the outputs written.  info[0] = 1.0 if G
// is not numerically SPD else 0.0; info[1] = max |G - I|.  Single workgroup;
// N <= 512, and above 128 the global workspace ws of chol_workspace_doubles(N)
// doubles is required.
enum { CHOL_OUT_MINV = 1, CHOL_OUT_D64 = 2, CHOL_OUT_D32 = 4, CHOL_OUT_ALL = 7 };
hipError_t launch_cholesky_inverse(double *G, double *Minv, float *D32, double *D64, int N,
                                   double *info, double *ws, hipStream_t s,
                                   int outs = CHOL_OUT_ALL);
// doubles of global workspace the blocked Cholesky needs for N > 128
size_t chol_workspace_doubles(int N);
// doubles needed by the Gram partial buffer
size_t gram_partial_doubles(int N, int nsplit);
// ---- subspace rotation and residual (rare: every n_diag steps or on request)
// splits of the cross product and the doubles of its partial buffer
int cross_gram_split(int N);
size_t cross_partial_doubles(int N);
// S = dv/2 (A B^T + B A^T) over the grid (A, B: [N][ng]) on FP64 MFMA; part:
// scratch of cross_partial_doubles(N)
template <typename T>
hipError_t launch_cross_gram(const T *A, const T *B, int N, i64 ng, double dv, double *part,
                             double *S, hipStream_t s);
// out = M X in the orbital index: out[j] = sum_i M[j][i] X[i] (M: FP64 N x N,
// row-major) on FP64 MFMA; out must not alias X
template <typename T>
hipError_t launch_rotate(const double *M, const T *X, T *out, int N, i64 ng, hipStream_t s);
// Number of K splits of the Gram kernels.  N <= 128: as many as are resident
// on the device at once, clamped to [256, 1024].  N > 128: a multiple of 8
// ranges sized to whole rounds of resident workgroups.
int gram_split(int N, bool fp32);
// out[j][g] = sum_i M[j][i] X[i][g] for M lower triangular N x N, formed as
// X + D X from D = M - I in the element type (FP32 with N > 128 multiplies on
// split-BF16 MFMA, FP64 on FP64 MFMA); M itself is read only for the
// split-BF16 kernel's far-from-identity form below.
// When rho is non-null also rho[g] = sum_j occ_j out[j][g]^2 (FP64); for
// N > 128 this needs rho_part, device memory for ceil(N / 128) * ng doubles
// (each 128-row block's share, summed in block order).
// ginfo (device, nullable): the Cholesky report of the Gram M came from; the
// split-BF16 kernel multiplies by M itself instead of adding D X to X when
// ginfo[1] = max |G - I| >= 0.25 (a factor far from the identity).  split_ws:
// device workspace of 2 * split_factor_elems(N) BF16 values, required for FP32
// orbitals with N > 128 (the factor's hi/lo pieces).
template <typename T>
hipError_t launch_apply_lower(const double *M, const T *D, const T *X, T *out, int N, i64 ng,
                              const double *occ, double *rho, hipStream_t s,
                              const double *ginfo = nullptr, void *split_ws = nullptr,
                              double *rho_part = nullptr);
// BF16 values in each piece of the padded factor split for N > 128
size_t split_factor_elems(int N);

// ---- nonlocal projectors (nonlocal_kernels.hip)
// One ion's projectors: position, width and amplitudes of xi_s = bs g,
// xi_a = bp (d_a / rc) g, and the cube of b^3 grid points (corner o, wrapped
// modulo n) on which they are evaluated.
struct NlIon {
  double R[3];
  double rc, bs, bp;
  int o[3];
  int b;
};
// cube splits per ion (parallel partial sums) for cubes of at most bmax^3 points
int nl_splits(int bmax);
// partial overlaps <xi_l, u_i> (deriv: <d xi_l / d R_a, u_i>, 12 per ion) into
// part[((I * nl_splits(bmax) + sp) * N + i) * K + k], K = 4 or 12, unscaled by h^3
template <typename T>
hipError_t launch_nl_overlap(const T *U, const NlIon *ions, int M, int bmax, int N, int n,
                             double L, bool deriv, double *part, hipStream_t s);
// C[4 M][N] = dv * sums of the partials; rep[i] += sum_l C[l][i]^2 (i < N);
// rep[enl_off] = sum_i occ_i sum_l C[l][i]^2
hipError_t launch_nl_finish(const double *part, int M, int bmax, int N, double dv,
                            const double *occ, double *C, double *rep, int enl_off,
                            hipStream_t s);
// out[(I * 12 + k) * N + i] = dv * sums of the derivative partials
hipError_t launch_nl_sum_deriv(const double *part, int M, int bmax, int N, double dv,
                               double *out, hipStream_t s);
// HU += V_nloc U over the cubes of the `count` ions in list (no two overlapping)
template <typename T>
hipError_t launch_nl_apply(T *HU, const NlIon *ions, const int *list, int count, int bmax,
                           const double *C, int N, int n, double L, hipStream_t s);

}  // namespace pou
