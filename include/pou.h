/*
 * pou.h -- C ABI of the MI355X library for the parallel orbital-updating
 * optimisation of Kohn-Sham DFT (Dai, Liu, Zhang, Zhou; arXiv 1510.07230).
 *
 * The library minimises the discrete Kohn-Sham energy over orthonormal
 * orbital blocks (section 2.1, eq. "emin" and eq. "energy") with the inner
 * loop of Algorithm M (section 3.3): per-orbital search directions
 * z_i = H w_i - sigma_ii w_i (section 3.2), one Barzilai-Borwein step size for
 * all orbitals, non-monotone backtracking (eq. "ene-de"), and
 * orthonormalisation through the Gram matrix <W^T W> (Cholesky-based QR,
 * section 3.2).  All arithmetic runs in HIP kernels on one gfx950 GPU.
 *
 * Discretisation: periodic cubic box of side L with n^3 points, h = L/n,
 * point g = (k*n + j)*n + i for (x,y,z) = h*(i,j,k) (x fastest); central
 * 8th-order finite-difference Laplacian; inner product <a,b> = h^3 sum a_g b_g.
 * Orbital blocks are [norb][n][n][n], orbital-major, contiguous.
 *
 * Energy: E = sum_i f_i <u_i, -1/2 Lap u_i> + <rho, V_ext> + 1/2 <rho, V_H>
 *           + E_x (+ E_c),  rho = sum_i f_i u_i^2;  V_H = P[rho], V_ext = -P[rho_ion],
 * P[f] = 4 pi (-Lap)^+ (f - mean f) (periodic Hartree potential with a
 * neutralising background), rho_ion = sum of normalised Gaussian charges
 * Z_I (pi s_I^2)^-3/2 exp(-|r-R_I|^2/s_I^2) (the periodic form of the local
 * pseudopotential -Z erf(r/s)/r), E_x the LDA exchange energy, E_c (opt in,
 * POU_TERM_CORR) the LDA correlation energy of the Perdew-Zunger fit that the
 * LDA of section 4 cites (spin-unpolarised).
 *
 * Conventions for every call:
 *   - Returns pou_status; POU_OK == 0.  On failure pou_last_error() gives a
 *     message.  A failed call that takes U in/out leaves U unchanged.
 *   - Orbital blocks (U, dU) are DEVICE pointers owned by the caller, of
 *     element type double (POU_FP64) or float (POU_MIXED), norb*n^3 elements.
 *   - Host pointers are marked "host".  The library never keeps a caller
 *     pointer after a call returns.
 *   - All device work is enqueued on the stream given to pou_create; calls
 *     that return host values synchronise that stream before returning.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef POU_H
#define POU_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pou_ctx pou_ctx;

typedef enum {
  POU_OK = 0,
  POU_ERR_ARG = -1,        /* invalid argument (null pointer, bad size)          */
  POU_ERR_STATE = -2,      /* call order (e.g. before pou_set_system)            */
  POU_ERR_HIP = -3,        /* a HIP runtime call failed                          */
  POU_ERR_OOM = -4,        /* device allocation failed                           */
  POU_ERR_NOT_SPD = -5,    /* Gram matrix not positive definite (rank deficient) */
  POU_ERR_CG_NO_CONV = -6, /* Poisson CG did not reach its tolerance             */
  POU_ERR_NONFINITE = -7   /* NaN or Inf in an input block or a result           */
} pou_status;

typedef enum {
  POU_FP64 = 0,  /* orbitals, H*U, stencil, Gram and apply in FP64 */
  POU_MIXED = 1  /* orbitals and stencil in FP32; Gram pass 1 in BF16 on MFMA with
                    FP32 accumulation; pass 2 and the applies FP32-accurate (BF16
                    hi/lo products on MFMA, or FP32 MFMA for the final apply of up
                    to 128 orbitals); Cholesky, energy and all reductions FP64
                    (section 3.2 Cholesky QR, applied twice) */
} pou_precision;

/* Energy-term mask for tests: the full model is POU_TERM_ALL. */
enum {
  POU_TERM_KIN = 1,
  POU_TERM_EXT = 2,
  POU_TERM_HARTREE = 4,
  POU_TERM_XC = 8,
  POU_TERM_ALL = 15,   /* the default model: exchange-only LDA */
  POU_TERM_CORR = 16,  /* add LDA correlation (not part of POU_TERM_ALL) */
  POU_TERM_NLOC = 32   /* nonlocal projectors; switched on by pou_set_projectors */
};

typedef struct {
  int n;     /* points per axis, 9 <= n <= 1024                 */
  double L;  /* box side in bohr, > 0                             */
} pou_grid;

typedef struct {
  double rho1;      /* Armijo constant of eq. "ene-de" (paper: 1e-4)             */
  double delta;     /* backtracking factor, tau = tau_BB * delta^s (paper: 0.1)  */
  double eta;       /* non-monotone averaging weight (paper: 0.85)               */
  int bb_mode;      /* 1: tau1 = tr<S^T S>/|tr<S^T Y>|, 2: tau2 = |tr<S^T Y>|/tr<Y^T Y>,
                       0: alternate (tau1 on odd l, tau2 on even l)              */
  double tau_init;  /* step size when no BB history exists; <= 0 -> 1/lambda_max(K) */
  int s_max;        /* largest backtracking exponent tried; if none passes, the
                       s_max trial is taken and step_info.accepted = 0          */
  int orth_passes;  /* Cholesky-QR passes per trial (1 or 2); 0 -> 1 for FP64, 2 for MIXED */
  double cg_rtol;   /* Poisson CG relative residual target; <= 0 -> 1e-12 (FP64) */
  int cg_maxit;     /* Poisson CG iteration cap; <= 0 -> 2000                    */
  int cg_precond;   /* 0: plain CG; 1: solve with the exact spectral inverse of
                       -Lap (FFT), check the residual against cg_rtol and, only
                       if it is missed, finish with CG preconditioned by that
                       inverse */
  unsigned terms;   /* energy-term mask, POU_TERM_*                              */
  int n_org;        /* orthonormalise, test eq. "ene-de" and backtrack only when
                       l mod n_org == 0; other iterations take the plain step
                       W <- W - tau_BB Z (section 3.3, Algorithm M); <= 0 -> 1   */
  int n_diag;       /* subspace diagonalisation of the new iterate after the
                       orthonormalising step of iteration l when l mod n_diag
                       == 0 (section 3.3; l counted before the increment):
                       W <- W P, P^T <(HW)^T W> P diagonal; 0 = off.  Needs
                       equal occupations                                        */
} pou_params;

typedef struct {
  double E, E_kin, E_ext, E_H, E_x;
  int cg_iters;     /* iterations of the Hartree solve for this evaluation */
  double E_c;       /* LDA correlation energy (0 unless POU_TERM_CORR) */
  double E_nl;      /* nonlocal energy sum_i f_i <u_i, V_nloc u_i> (0 without projectors) */
} pou_energy_terms;

typedef struct {
  int l;            /* iteration index of the step just taken (0-based)          */
  int s;            /* backtracking exponent accepted                            */
  int accepted;     /* 1 if eq. "ene-de" held at s, 0 if s_max was exhausted     */
  int cg_iters;     /* Poisson CG iterations summed over the trials              */
  double E;         /* energy of the new iterate W^(l+1)                         */
  double tau_bb;    /* BB (or initial) step before backtracking                  */
  double tau;       /* accepted step tau_BB * delta^s                            */
  double zz;        /* ||Z^(l)||_F^2 = sum_i <z_i, z_i>                          */
  double df;        /* |E^(l) - E^(l+1)| / (|E^(l)| + 1)                          */
  double C, Q;      /* non-monotone reference values after the update            */
  double gram_dev;  /* max |G - I| of the first Gram of the accepted trial       */
  int orthonormalized; /* 1: orthonormalising step with the energy test; 0: plain
                          step (n_org > 1), whose E is that of the non-orthonormal
                          iterate and whose df is NaN                            */
  int rotated;      /* 1 if the new iterate was rotated by subspace diagonalisation */
} pou_step_info;

/* Fill *p with the paper's constants (rho1 = 1e-4, delta = 0.1, eta = 0.85;
   section 3.2) and the defaults listed above. */
void pou_default_params(pou_params *p);

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t (may
   be NULL for the null stream).  The context owns all workspace. */
pou_status pou_create(pou_ctx **out, int device, void *hip_stream);
pou_status pou_destroy(pou_ctx *ctx);
const char *pou_last_error(const pou_ctx *ctx);

/* Define the system (section 2.1): grid, ions, occupations, precision and
   algorithm parameters.  R [natoms][3] (bohr), Z [natoms], sigma [natoms] > 0,
   occ [norb] are host arrays.  Allocates the workspace, builds rho_ion and
   V_ext = -P[rho_ion] on the device, and resets the iteration state
   (l = 0, no BB history).  Requires 1 <= norb <= min(512, n^3), natoms >= 0. */
pou_status pou_set_system(pou_ctx *ctx, const pou_grid *grid, int natoms,
                          const double *R, const double *Z, const double *sigma,
                          int norb, const double *occ, pou_precision prec,
                          const pou_params *params);

/* Nonlocal part of the pseudopotential (section 2.1): V_nloc u =
   sum_l <xi_l, u> xi_l with four projectors per ion I centred on R_I,
     xi_s = b_s g,  xi_a = b_p (d_a / rc) g  (a = x, y, z),
     g = exp(-|d|^2 / (2 rc^2)),  d = r - R_I (minimum image),
   params (host double [natoms][3]) = (rc > 0, b_s, b_p) per ion of the last
   pou_set_system, which this call must follow (pou_set_system clears the
   projectors).  Adds E_nl = sum_i f_i <u_i, V_nloc u_i> to E, V_nloc u to H u
   and its derivative to the forces; turns POU_TERM_NLOC on.  params NULL
   removes the projectors.  Each ion's projectors are evaluated on a cube of
   grid points reaching past the radius where g < 1e-14 (the whole grid if
   that does not fit), and nothing outside it.  The library keeps no pointer
   to params.  POU_ERR_ARG on a bad width or amplitude. */
pou_status pou_set_projectors(pou_ctx *ctx, const double *params);

/* Total energy E(U) of eq. "energy" for the device block U (not modified).
   Leaves rho, V_H, V_eff and H*U of this U cached in the context. */
pou_status pou_energy(pou_ctx *ctx, const void *U, pou_energy_terms *out);

/* Orth(U) of Algorithm B step 5, in place: U <- U R^-1 with R upper
   triangular, diag R > 0, <U^T U> = I (Cholesky QR through the Gram matrix
   with FP32-accurate or FP64 products, at most 3 passes: passes continue
   until the Gram measured by a pass is within 1e-8 (FP64) / 1e-4 (FP32
   orbitals) of I after at least two passes, or within 1e-12 / 1e-8 already
   after the first).
   orth_err (host, nullable) receives max |<U^T U> - I| after the call.
   POU_ERR_NOT_SPD if U is numerically rank deficient (U unchanged).
   Resets the BB history (U changed). */
pou_status pou_orthonormalize(pou_ctx *ctx, void *U, double *orth_err);

/* One iteration of Algorithm M with n_org = 1 (section 3.3): U holds an
   orthonormal W^(l) on entry and W^(l+1) = Orth(W^(l) - tau Z^(l)) on exit.
   The context keeps the BB history, C and Q between calls made with the same
   U pointer; a different pointer restarts at l = 0.  The caller must not
   modify U between consecutive calls. */
pou_status pou_orbital_update_step(pou_ctx *ctx, void *U, pou_step_info *out);

/* Gradient of gE * E(U) at fixed ions, and of E with respect to the ions.
   The orbital part is the derivative E_{u_i} of section 2.1 for this E,
   including the occupation factor (the discrete energy of eq. "energy" with
   rho = sum f_i u_i^2 gives dE/du_i = 2 f_i h^3 H(rho) u_i):
     dU     (device, nullable, precision of U): gE * 2 f_i h^3 (H u_i)
     dR     (device double [natoms][3], nullable): gE * dE/dR_I
     dsigma (device double [natoms], nullable):   gE * dE/dsigma_I
   dE/dq = -<V_H, d rho_ion/dq> with V_H = P[rho(U)]. */
pou_status pou_energy_backward(pou_ctx *ctx, const void *U, double gE, void *dU,
                               double *dR, double *dsigma);

/* ---- diagnostics and utilities (same stream, same error model) ---------- */

/* Norm of the Stiefel gradient of eq. "gra" (section 2.2) with the full
   Lagrange multiplier: Sigma = <(H U)^T U> (H = H(rho(U)), U evaluated as by
   pou_energy) and resid = sqrt(tr<R^T R>), R = H U - U Sigma, the residual
   reported in section 4.1.  Sigma (host double [norb][norb], nullable)
   receives the symmetrised Sigma.  U is not modified. */
pou_status pou_residual(pou_ctx *ctx, const void *U, double *resid, double *Sigma);

/* H U for the potentials of the last pou_energy / step evaluation; also
   sigma_ii = <u_i, H u_i> into sigma (host, nullable, [norb]). */
pou_status pou_hamiltonian_apply(pou_ctx *ctx, const void *U, void *HU, double *sigma);

/* Copy the FP64 fields of the last evaluation to device buffers of n^3
   doubles (each nullable): density, Hartree potential, V_eff, V_ext. */
pou_status pou_get_fields(pou_ctx *ctx, double *rho, double *vh, double *veff,
                          double *vext);

/* Gram matrix of section 3.2 (Cholesky QR), <U^T U> = h^3 U U^T, into G
   (host double [norb][norb], full symmetric), formed by the kernels of the
   orthonormalisation.  mode POU_GRAM_ACCURATE: FP64 MFMA for FP64 orbitals;
   FP32-accurate for FP32 orbitals (FP32 MFMA up to 128 orbitals, BF16 hi/lo
   products above).  mode POU_GRAM_BF16 (FP32 orbitals only, else
   POU_ERR_ARG): the first-pass Gram of the mixed form, products of
   BF16-rounded values summed in FP32 on MFMA and flushed to FP64.  U is not
   modified. */
enum { POU_GRAM_ACCURATE = 0, POU_GRAM_BF16 = 1 };
pou_status pou_gram(pou_ctx *ctx, const void *U, int mode, double *G);

/* Trial point of a step (section 3.2 and Algorithm M): for the device block
   U, H = H(rho(U)) is formed (as by pou_energy) and W~ = U - tau Z with
   z_i = H u_i - sigma_ii u_i, sigma_ii = <H u_i, u_i>, is written to Wt
   (device, nullable, precision and layout of U) and its Gram <W~^T W~> to G
   (host double [norb][norb], nullable), by the kernels a step's first
   Cholesky-QR pass uses (with POU_MIXED and two passes the Gram is the BF16
   first-pass Gram).  tau must be finite.  U is not modified; the iteration
   state is kept. */
pou_status pou_trial_point(pou_ctx *ctx, const void *U, double tau, void *Wt, double *G);

/* Gram matrix without a context and without any allocation, for callers
   that cannot allocate device memory (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): the same product as
   pou_gram, G = dv * U U^T (dv = h^3), by the same kernels, written to the
   DEVICE buffer G (double [norb][norb], full symmetric) on hip_stream
   (a hipStream_t, NULL for the null stream).  U: device block [norb][ng] of
   doubles (prec POU_FP64) or floats (POU_MIXED); mode as in pou_gram.
   Limits: 1 <= norb <= 128, ng >= norb, dv > 0 (else POU_ERR_ARG; no message,
   since there is no context).  The partial sums live in a static device array
   of 32 MiB (256 splits of 128 x 128 doubles) that each GPU holds from the
   first call on it until the process ends; calls that overlap on one GPU (on
   different streams) race on it.  The call only enqueues work: G is ready
   when the stream reaches it.  POU_ERR_HIP if a launch fails. */
pou_status pou_gram_static(const void *U, int prec, int mode, int norb, long long ng, double dv,
                           double *G, void *hip_stream);

/* Element-type conversion of a block of count elements between FP32 and
   FP64 device buffers (src_prec, dst_prec in {POU_FP64, POU_MIXED}). */
pou_status pou_convert(pou_ctx *ctx, const void *src, int src_prec, void *dst,
                       int dst_prec, long long count);

/* Reset the iteration state (l = 0, no BB history) without touching fields. */
pou_status pou_reset_history(pou_ctx *ctx);

/* ---- per-kernel timing with HIP events on the context's stream ---------- */

/* Kernel groups timed when profiling is on. */
enum {
  POU_K_HAMILTONIAN = 0, /* H*U stencil sweep over all orbitals        */
  POU_K_DENSITY = 1,     /* rho = sum f_i u_i^2 (when not fused)       */
  POU_K_XC = 2,          /* exchange potential, V_eff, energy partials */
  POU_K_POISSON = 3,     /* every kernel of the Hartree CG solve       */
  POU_K_GRAM = 4,        /* Gram partial contraction (MFMA)            */
  POU_K_CHOLESKY = 5,    /* Cholesky + triangular inverse, Gram reduce */
  POU_K_APPLY = 6,       /* W <- L^-1 W (MFMA), fused density          */
  POU_K_TRIAL = 7,       /* W - tau Z, fused with its first Gram        */
  POU_K_COMMIT = 8,      /* accept + Barzilai-Borwein dot products     */
  POU_K_OTHER = 9,       /* reductions and the remaining small kernels */
  POU_K_APPLY_GRAM = 10, /* first Cholesky-QR apply fused with the
                            second Gram (mixed precision, two passes)   */
  POU_K_COUNT = 11
};

#define POU_PROFILE_ALL ((1u << POU_K_COUNT) - 1u)

/* Time the kernel groups whose bit (1u << POU_K_*) is set in group_mask;
   0 turns timing off, POU_PROFILE_ALL times every group.  Synchronises the
   stream and clears the totals.  Each timed launch is bracketed by two
   hipEventRecord calls, which add a few microseconds of idle time between
   launches: leave groups that are not being measured untimed. */
pou_status pou_profile_enable(pou_ctx *ctx, unsigned group_mask);

/* Total milliseconds and number of launches of kernel group `group` since
   profiling was enabled (host outputs). */
pou_status pou_profile_read(pou_ctx *ctx, int group, double *total_ms,
                            long long *launches);

#ifdef __cplusplus
}
#endif

#endif /* POU_H */
