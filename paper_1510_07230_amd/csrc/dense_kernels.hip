// Dense kernels of the orthonormalisation (section 3.2: QR through a Cholesky
// factorisation of the Gram matrix <W^T W>): the Gram contraction over the
// grid on MFMA, its reduction to the symmetric N x N matrix, the FP64
// Cholesky factorisation with the triangular inverse, and the triangular
// apply W <- L^-1 W on MFMA.
#include "pou_internal.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

namespace pou {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));


__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row of output register r in lane group q (= lane / 16) of a 16x16 MFMA tile:
// the FP64 16x16x4 instruction spreads rows as q + 4r, the FP32 and BF16
// instructions as 4q + r (measured on gfx950; columns are lane % 16 for both).
template <typename T>
__device__ inline int out_row(int q, int r) {
  return sizeof(T) == 8 ? q + 4 * r : 4 * q + r;
}

// BF16 pieces of an FP32 value: hi = bf16(v), lo = bf16(v - hi); hi + lo
// equals v to about 2^-17 relative.  The same rounding (to nearest even) is
// used wherever a split value has to be reproduced.
__device__ inline void split_bf16(float v, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

template <typename T> struct AccOf;
template <> struct AccOf<double> { typedef d4 type; };
template <> struct AccOf<float> { typedef f4 type; };

__device__ inline void decode_pair(int pair, int nb, int &bi, int &bj) {
  int p = pair, i = 0;
  while (p >= nb - i) {
    p -= nb - i;
    ++i;
  }
  bi = i;
  bj = i + p;
}

// M = A B for lower-triangular A, B (N x N, zeros above the diagonal), with
// D64 = M - I and D32 its FP32 copy: the combined factor of two Cholesky-QR
// passes.  With split_b, B is replaced by the value the fused first apply
// used: I + Dh + Dl with Dh/Dl the BF16 pieces of (float)(B - I).  One wave
// per 16 x 16 output tile (I, J) on FP64 MFMA, summing the tile products
// A_IK B_KJ for J <= K <= I; tiles above the diagonal are zero.
__global__ __launch_bounds__(64) void k_combine_factors(const double *__restrict__ A,
                                                        const double *__restrict__ B,
                                                        double *__restrict__ M,
                                                        double *__restrict__ D64,
                                                        float *__restrict__ D32, int N,
                                                        int split_b) {
  const int NT = (N + 15) / 16;
  const int I = blockIdx.x / NT, J = blockIdx.x % NT;
  const int l = threadIdx.x, r16 = l & 15, q = l >> 4;
  d4 acc = d4{0, 0, 0, 0};
  if (J <= I) {
    const int ia = 16 * I + r16, jb = 16 * J + r16;
    const int iac = min(ia, N - 1), jbc = min(jb, N - 1);
    // K tiles in batches of eight whose loads are all issued before their
    // products (the tile is latency-bound: one wave, up to 32 K tiles).  The
    // loads read clamped, always-valid addresses and the values outside the
    // tile's range are replaced afterwards: a guarded load would sit in a
    // branch of its own and be waited on before the next one is issued.
    for (int K0 = J; K0 <= I; K0 += 8) {
      double a[8][4], b[8][4];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int K = K0 + kk;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int k = 16 * K + 4 * s4 + q;
          const int kc = min(k, N - 1);
          a[kk][s4] = A[(i64)iac * N + kc];
          b[kk][s4] = B[(i64)kc * N + jbc];
        }
      }
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int K = K0 + kk;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int k = 16 * K + 4 * s4 + q;
          const bool in = (K <= I) & (k < N);
          a[kk][s4] = (in & (ia < N)) ? a[kk][s4] : 0.0;
          double bv = (in & (jb < N)) ? b[kk][s4] : 0.0;
          if (split_b) {
            const double dlt = (in & (k == jb)) ? 1.0 : 0.0;
            __bf16 hi, lo;
            split_bf16((float)(bv - dlt), hi, lo);
            bv = dlt + ((double)(float)hi + (double)(float)lo);
          }
          b[kk][s4] = bv;
        }
      }
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) acc = mfma(a[kk][s4], b[kk][s4], acc);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 16 * I + out_row<double>(q, r), j = 16 * J + r16;
    if (i < N && j < N) {
      const double v = (j <= i) ? acc[r] : 0.0;
      const i64 e = (i64)i * N + j;
      M[e] = v;
      const double d = v - (i == j ? 1.0 : 0.0);
      D64[e] = d;
      D32[e] = (float)d;
    }
  }
}

// ---------------------------------------------------------------- blocked Cholesky

constexpr int kTP = 17;                 // padded pitch of a 16 x 16 FP64 tile in LDS
constexpr int kTile = 16 * kTP;         // doubles per tile slot

__device__ inline int tri_slot(int i, int j) { return i * (i + 1) / 2 + j; }

// D (+)= sign * X * Y^op for 16 x 16 FP64 tiles in LDS.  X is read as the
// MFMA A operand (X[l%16][4s + q]); Y is read as Y[4s + q][l%16] (ytrans = 0)
// or as Y^T, i.e. Y[l%16][4s + q] (ytrans = 1).  C is read from / written to
// the accumulator layout (row q + 4r, column l%16) of dst (and of dst2 when
// given); cin = 0 starts from 0.
__device__ inline void tile_mma(const double *X, const double *Y, int ytrans, double sign,
                                const double *C, double *dst, int l, double *dst2 = nullptr) {
  const int r16 = l & 15, q = l >> 4;
  d4 acc = d4{0, 0, 0, 0};
  if (C) {
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = C[(q + 4 * r) * kTP + r16];
  }
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    const double a = sign * X[r16 * kTP + 4 * s4 + q];
    const double b = ytrans ? Y[r16 * kTP + 4 * s4 + q] : Y[(4 * s4 + q) * kTP + r16];
    acc = mfma(a, b, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) dst[(q + 4 * r) * kTP + r16] = acc[r];
  if (dst2) {
#pragma unroll
    for (int r = 0; r < 4; ++r) dst2[(q + 4 * r) * kTP + r16] = acc[r];
  }
}

// Value of a (wave-uniform) lane of v, as two scalar reads.
__device__ inline double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// 1/sqrt(x) for a positive normal x: the hardware estimate refined by two
// Newton steps y <- y (3 - x y^2) / 2 (each roughly doubles the correct bits;
// the result is within a few units in the last place).  It replaces an
// IEEE square root and division on the serial chain of pivots, where their
// long expansions dominated the diagonal-block factorisation.
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

// One wave: [A_pp | I] -> [L_pp^T | L_pp^-1] for a 16 x 16 diagonal block
// (Gaussian elimination without pivoting).  Lane c < 32 holds column c of the
// 16 x 32 augmented block in registers (all 16 rows), so row k of step k is
// the lane's own register and the pivot and column k come from lane k by
// scalar lane reads; lanes 32..63 carry zero columns.  L_pp^-1 goes to Li
// (lower part; zeros above).  A pivot that is not above 1e-13 times the
// block's original diagonal entry (dg) flags numerical rank deficiency in
// *sbad.  All operands are in LDS and typed so (the function is not inlined:
// it keeps its own registers); a failed pivot is replaced without a branch.
typedef __attribute__((address_space(3))) double lds_double;
typedef __attribute__((address_space(3))) int lds_int;
__device__ inline lds_double *lds(double *p) { return (lds_double *)p; }
__device__ inline lds_int *lds(int *p) { return (lds_int *)p; }
__device__ __attribute__((noinline)) void chol_diag_block(const lds_double *App, lds_double *Li,
                                                          const lds_double *dg, int l,
                                                          lds_int *sbad) {
  const int c = l;
  double v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (c < 16) v[r] = (c <= r) ? App[r * kTP + c] : App[c * kTP + r];
    else v[r] = (c - 16 == r) ? 1.0 : 0.0;  // zero for c >= 32
  }
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    double piv = readlane_f64(v[k], k);
    const bool ok = (piv > 1e-13 * dg[k]) && isfinite(piv);
    bad |= !ok;
    piv = ok ? piv : 1.0;
    const double isp = rsqrt_nr(piv);
    const double rk = v[k];
    const double rki = rk * (isp * isp);
    v[k] = rk * isp;
#pragma unroll
    for (int r = k + 1; r < 16; ++r) v[r] -= readlane_f64(v[r], k) * rki;
  }
  if (c >= 16 && c < 32) {
#pragma unroll
    for (int r = 0; r < 16; ++r) Li[r * kTP + (c - 16)] = (c - 16 <= r) ? v[r] : 0.0;
  }
  if (bad && l == 0) *sbad = 1;
}

// Blocked Cholesky G = L L^T and L^-1 in one workgroup (16-wide panels,
// right-looking, one panel of lookahead).  Panel p: the panel L_ip = A_ip
// L_pp^-T and the block row B_pj <- L_pp^-1 B_pj of B = L^-1 on MFMA; then
// the trailing update A_ij -= L_ip L_jp^T and the eliminations B_ij -= L_ip
// B_pj.  Wave 0 takes the update of the next diagonal block A_{p+1,p+1}
// first and factors it (chol_diag_block) while the other waves do the rest
// of the trailing update, so the serial diagonal factorisations overlap the
// tile work.  A tile slot holds A_ij until its panel is processed and B_ij
// afterwards.  Padding rows beyond N carry an identity diagonal.
//
// LDS_TILES: tiles live in LDS (N <= 128, ~105 KB); otherwise in the global
// workspace ws (L2-resident; N <= 512: 528 tile slots), with the panel and the
// current block row of L^-1 in LDS (~148 KB) and the trailing tasks batched
// four per wave so that their workspace loads overlap.
template <bool LDS_TILES, int NTHR>
__global__ __launch_bounds__(NTHR) void k_chol_blocked(const double *__restrict__ G, int N,
                                                       double *__restrict__ Minv,
                                                       float *__restrict__ D32,
                                                       double *__restrict__ D64,
                                                       double *__restrict__ info,
                                                       double *__restrict__ ws, int outs) {
  __shared__ double slot_s[LDS_TILES ? 36 * kTile : 1];
  // panel tiles L_ip in LDS (8 for N <= 128, 32 for the workspace variant),
  // and for the workspace variant the current block row B_pj of L^-1 too:
  // the trailing tasks then read only their own tile from the workspace
  __shared__ double P_s[(LDS_TILES ? 8 : 32) * kTile];
  __shared__ double Brow_s[LDS_TILES ? 1 : 32 * kTile];
  __shared__ double Li2[2][kTile];
  // the workspace variant's copy of the diagonal block being factored
  __shared__ double Ad_s[LDS_TILES ? 1 : kTile];
  __shared__ double sdg[512];
  __shared__ double sred[NTHR / 64];
  __shared__ int sbad;
  double *slot = LDS_TILES ? slot_s : ws;
  double *P = P_s;
  constexpr int NW = NTHR / 64;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int NT = (N + 15) / 16;
  const int NP = 16 * NT;
  double m = 0.0;
  // the lower triangle of G into the tile slots: wave w takes rows w, w + NW,
  // ..., lanes take columns, ROWB rows per batch of independent loads
  constexpr int CPR = LDS_TILES ? 2 : 8;       // 64-column chunks per row (NP <= 64 CPR)
  constexpr int ROWB = LDS_TILES ? 16 : 2;      // N <= 128: all of a wave's rows in one batch
  for (int r0 = w; r0 < NP; r0 += NW * ROWB) {
    double v[ROWB][CPR];
#pragma unroll
    for (int u = 0; u < ROWB; ++u) {
      const int r = r0 + NW * u;
#pragma unroll
      for (int j = 0; j < CPR; ++j) {
        // clamped, always-valid address; the value is zeroed below the test
        // (a guarded load would be issued in a branch of its own)
        const int c = l + 64 * j;
        const double g = G[(i64)min(r, N - 1) * N + min(c, N - 1)];
        v[u][j] = ((r < N) & (c <= r)) ? g : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < ROWB; ++u) {
      const int r = r0 + NW * u;
#pragma unroll
      for (int j = 0; j < CPR; ++j) {
        const int c = l + 64 * j;
        if (r < NP && c <= r) {
          double x = v[u][j];
          if (r < N) {
            const double d = x - (r == c ? 1.0 : 0.0);
            m = isfinite(d) ? fmax(m, fabs(d)) : INFINITY;
          } else {
            x = (r == c) ? 1.0 : 0.0;
          }
          slot[tri_slot(r >> 4, c >> 4) * kTile + (r & 15) * kTP + (c & 15)] = x;
          if (r == c) sdg[r] = x;
        }
      }
    }
  }
  m = wave_max(m);
  if (l == 0) sred[w] = m;
  if (t == 0) sbad = 0;
  __syncthreads();
  if (t == 0) {
    double mx = 0.0;
    for (int k = 0; k < NW; ++k) mx = fmax(mx, sred[k]);
    info[1] = mx;
  }
  if (w == 0) {
    double *A0 = slot + tri_slot(0, 0) * kTile;
    if (!LDS_TILES) {
      for (int e = l; e < 16 * kTP; e += 64) Ad_s[e] = A0[e];
      A0 = Ad_s;
    }
    chol_diag_block(lds(A0), lds(Li2[0]), lds(sdg), l, lds(&sbad));
  }
  __syncthreads();
  for (int p = 0; p < NT; ++p) {
    const double *Li = Li2[p & 1];
    // (b) panel L_ip = A_ip Li^T (i > p) into P[i]; B_pj <- Li B_pj (j < p); B_pp = Li
    {
      const int nb = NT - 1 - p;  // panel tiles
      const int nd = p;           // B row tiles
      for (int task = w; task < nb + nd + 1; task += NW) {
        if (task < nb) {
          const int i = p + 1 + task;
          tile_mma(slot + tri_slot(i, p) * kTile, Li, 1, 1.0, nullptr, P + i * kTile, l);
        } else if (task < nb + nd) {
          const int j = task - nb;
          double *Bpj = slot + tri_slot(p, j) * kTile;
          // in place: the MFMA chain reads the whole tile before the write; the
          // workspace variant also keeps the result in LDS (from registers)
          tile_mma(Li, Bpj, 0, 1.0, nullptr, Bpj, l,
                   LDS_TILES ? nullptr : Brow_s + (LDS_TILES ? 0 : j * kTile));
        } else {
          double *Bpp = slot + tri_slot(p, p) * kTile;
          for (int e = l; e < 256; e += 64) Bpp[(e >> 4) * kTP + (e & 15)] = Li[(e >> 4) * kTP + (e & 15)];
          if (!LDS_TILES) {
            double *Bl = Brow_s + (LDS_TILES ? 0 : p * kTile);
            for (int e = l; e < 256; e += 64) Bl[(e >> 4) * kTP + (e & 15)] = Li[(e >> 4) * kTP + (e & 15)];
          }
        }
      }
    }
    __syncthreads();
    // (c) A_ij -= L_ip L_jp^T (p < j <= i); (e) B_ij -= L_ip B_pj (i > p, j <= p).
    // With a next panel, wave 0 updates and factors A_{p+1,p+1} (task 0 of (c))
    // and the other waves share the remaining tasks.
    {
      const int m1 = NT - 1 - p;
      const int nc = m1 * (m1 + 1) / 2;
      const int ne = m1 * (p + 1);
      const bool look = (m1 > 0);
      if (look && w == 0) {
        // the workspace variant factors an LDS copy (the tile in the
        // workspace is not read again: its slot takes B_{p+1,p+1} next)
        double *A1 = slot + tri_slot(p + 1, p + 1) * kTile;
        tile_mma(P + (p + 1) * kTile, P + (p + 1) * kTile, 1, -1.0, A1, LDS_TILES ? A1 : Ad_s, l);
        __threadfence_block();
        chol_diag_block(lds(LDS_TILES ? A1 : Ad_s), lds(Li2[(p + 1) & 1]), lds(sdg + 16 * (p + 1)),
                        l, lds(&sbad));
      }
      const int first = look ? 1 : 0;                // task 0 is wave 0's when looking ahead
      const int ww = look ? w - 1 : w, nww = look ? NW - 1 : NW;
      if (!LDS_TILES && ww >= 0) {
        // workspace variant: four tasks per wave per round, their workspace
        // tiles loaded before any product (the operands come from LDS)
        constexpr int TB = 4;
        const int r16 = l & 15, q = l >> 4;
        for (int t0 = first + ww; t0 < nc + ne; t0 += TB * nww) {
          double *cp[TB];
          const double *xp[TB], *yp[TB];
          bool yt[TB], cin[TB], ok[TB];
          d4 acc[TB];
#pragma unroll
          for (int u = 0; u < TB; ++u) {
            const int task = t0 + u * nww;
            ok[u] = task < nc + ne;
            cp[u] = slot;
            xp[u] = yp[u] = P;
            yt[u] = true;
            cin[u] = false;
            if (!ok[u]) continue;
            if (task < nc) {
              int a = task, ii = 0;
              while (a > ii) { a -= ii + 1; ++ii; }
              const int i = p + 1 + ii, j = p + 1 + a;
              cp[u] = slot + tri_slot(i, j) * kTile;
              xp[u] = P + i * kTile;
              yp[u] = P + j * kTile;
              cin[u] = true;
            } else {
              const int a = task - nc;
              const int i = p + 1 + a / (p + 1), j = a % (p + 1);
              cp[u] = slot + tri_slot(i, j) * kTile;
              xp[u] = P + i * kTile;
              yp[u] = Brow_s + (LDS_TILES ? 0 : j * kTile);
              yt[u] = false;
              cin[u] = j < p;
            }
          }
#pragma unroll
          for (int u = 0; u < TB; ++u) {
            acc[u] = d4{0, 0, 0, 0};
            if (ok[u] && cin[u]) {
#pragma unroll
              for (int r = 0; r < 4; ++r) acc[u][r] = cp[u][(q + 4 * r) * kTP + r16];
            }
          }
#pragma unroll
          for (int u = 0; u < TB; ++u) {
            if (!ok[u]) continue;
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
              const double a = -xp[u][r16 * kTP + 4 * s4 + q];
              const double b = yt[u] ? yp[u][r16 * kTP + 4 * s4 + q] : yp[u][(4 * s4 + q) * kTP + r16];
              acc[u] = mfma(a, b, acc[u]);
            }
          }
#pragma unroll
          for (int u = 0; u < TB; ++u) {
            if (!ok[u]) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) cp[u][(q + 4 * r) * kTP + r16] = acc[u][r];
          }
        }
      } else if (ww >= 0) {
        for (int task = first + ww; task < nc + ne; task += nww) {
          if (task < nc) {
            // decode (i, j) with p < j <= i
            int a = task, ii = 0;
            while (a > ii) { a -= ii + 1; ++ii; }
            const int i = p + 1 + ii, j = p + 1 + a;
            double *Aij = slot + tri_slot(i, j) * kTile;
            tile_mma(P + i * kTile, P + j * kTile, 1, -1.0, Aij, Aij, l);
          } else {
            const int a = task - nc;
            const int i = p + 1 + a / (p + 1), j = a % (p + 1);
            double *Bij = slot + tri_slot(i, j) * kTile;
            tile_mma(P + i * kTile, slot + tri_slot(p, j) * kTile, 0, -1.0, j < p ? Bij : nullptr,
                     Bij, l);
          }
        }
      }
    }
    __syncthreads();
  }
  // outputs named in outs (CHOL_OUT_*): the single workgroup's stores are a
  // large part of the kernel, so callers ask only for what they read.  For
  // even N <= 128 each lane takes a column pair of four rows at a time, all
  // LDS reads ahead of the stores.
  if (LDS_TILES && (N & 1) == 0) {
    typedef double dbl2 __attribute__((ext_vector_type(2)));
    typedef float flt2 __attribute__((ext_vector_type(2)));
    const int c = 2 * l;
    for (int r0 = w; r0 < N; r0 += 4 * NW) {
      dbl2 vv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = r0 + NW * u;
        const double *tp = slot + tri_slot(r >> 4, c >> 4) * kTile + (r & 15) * kTP + (c & 15);
        const bool in = r < N && c < N;
        vv[u][0] = (in && c <= r) ? tp[0] : 0.0;
        vv[u][1] = (in && c + 1 <= r) ? tp[1] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = r0 + NW * u;
        if (r >= N || c >= N) continue;
        const i64 e = (i64)r * N + c;
        const dbl2 d = dbl2{vv[u][0] - (r == c ? 1.0 : 0.0), vv[u][1] - (r == c + 1 ? 1.0 : 0.0)};
        if (outs & CHOL_OUT_MINV) *(dbl2 *)(Minv + e) = vv[u];
        if (outs & CHOL_OUT_D64) *(dbl2 *)(D64 + e) = d;
        if (outs & CHOL_OUT_D32) *(flt2 *)(D32 + e) = flt2{(float)d[0], (float)d[1]};
      }
    }
    if (t == 0) info[0] = sbad ? 1.0 : 0.0;
    return;
  }
  for (int r = w; r < N; r += NW) {
    for (int c = l; c < N; c += 64) {
      const double v =
          (c <= r) ? slot[tri_slot(r >> 4, c >> 4) * kTile + (r & 15) * kTP + (c & 15)] : 0.0;
      const i64 e = (i64)r * N + c;
      const double d = v - (r == c ? 1.0 : 0.0);
      if (outs & CHOL_OUT_MINV) Minv[e] = v;
      if (outs & CHOL_OUT_D64) D64[e] = d;
      if (outs & CHOL_OUT_D32) D32[e] = (float)d;
    }
  }
  if (t == 0) info[0] = sbad ? 1.0 : 0.0;
}

// Tiles of the N <= 128 Gram owned by wave W: row tiles W and 7 - W with the
// column tiles on or right of the diagonal (8 - W and W + 1 tiles, 9 in all).
template <int W, int U>
struct GramTile {
  static constexpr int nfirst = 8 - W;
  static constexpr int rt = U < nfirst ? W : 7 - W;
  static constexpr int ct = U < nfirst ? W + U : (7 - W) + (U - nfirst);
};

// One staged chunk of KC points for wave W: 9 accumulating MFMA tiles.
template <typename T, int NT, int W, int KC, int PITCH, typename Acc>
__device__ inline void gram_chunk(const T (*s)[PITCH], Acc (&acc)[9], int r16, int q) {
#pragma unroll
  for (int ks = 0; ks < KC / 4; ++ks) {
    T f[8];
#pragma unroll
    for (int ct = 0; ct < 8; ++ct)
      f[ct] = (ct < NT && ct >= W) ? s[16 * ct + r16][4 * ks + q] : (T)0;
#define POU_GT(U)                                                              \
  if (GramTile<W, U>::rt < NT && GramTile<W, U>::ct < NT)                      \
    acc[U] = mfma(f[GramTile<W, U>::rt], f[GramTile<W, U>::ct], acc[U]);
    POU_GT(0) POU_GT(1) POU_GT(2) POU_GT(3) POU_GT(4) POU_GT(5) POU_GT(6) POU_GT(7) POU_GT(8)
#undef POU_GT
  }
}

template <int NT, int W, int KC, int PB>
__device__ inline void gram_chunk_bf16(const __bf16 (*s)[PB], double (&accd)[9][4], int r16,
                                       int q) {
#pragma unroll
  for (int kk = 0; kk < KC / 32; ++kk) {
    bf8 f[8];
#pragma unroll
    for (int ct = 0; ct < 8; ++ct)
      f[ct] = (ct < NT && ct >= W) ? *(const bf8 *)&s[16 * ct + r16][32 * kk + 8 * q]
                                   : bf8{0, 0, 0, 0, 0, 0, 0, 0};
#define POU_GTB(U)                                                                        \
  if (GramTile<W, U>::rt < NT && GramTile<W, U>::ct < NT) {                               \
    f4 c = f4{0, 0, 0, 0};                                                                \
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[GramTile<W, U>::rt], f[GramTile<W, U>::ct], \
                                                c, 0, 0, 0);                              \
    accd[U][0] += (double)c[0];                                                           \
    accd[U][1] += (double)c[1];                                                           \
    accd[U][2] += (double)c[2];                                                           \
    accd[U][3] += (double)c[3];                                                           \
  }
    POU_GTB(0) POU_GTB(1) POU_GTB(2) POU_GTB(3) POU_GTB(4) POU_GTB(5) POU_GTB(6) POU_GTB(7)
    POU_GTB(8)
#undef POU_GTB
  }
}

template <int W, int U>
__device__ inline void gram_tile_rc(int &rt, int &ct) {
  rt = GramTile<W, U>::rt;
  ct = GramTile<W, U>::ct;
}

__device__ inline void gram_tile_runtime(int w, int u, int &rt, int &ct) {
  const int nfirst = 8 - w;
  rt = u < nfirst ? w : 7 - w;
  ct = u < nfirst ? w + u : (7 - w) + (u - nfirst);
}

// Partial Gram over a range of grid points, whole N x N (N <= 128) upper
// triangle per workgroup so every row is read once.  Chunks of KC points are
// staged in LDS; the next chunk is loaded into registers while the current one
// is multiplied.  The per-wave tile choice is resolved at compile time.
// TRIAL: A is the trial point W - tau Z formed on the fly from W = A and
// HW (z_i = H w_i - sigma_ii w_i, section 3.2) and written to Wt.
template <typename T, int NT, int KC, bool TRIAL>
__global__ __launch_bounds__(kBlock) void k_gram_small(const T *__restrict__ A, int N, i64 ng,
                                                          i64 kper, double *__restrict__ part,
                                                          const T *__restrict__ HW,
                                                          const double *__restrict__ sig,
                                                          const double *__restrict__ dtau,
                                                          double tscale, T *__restrict__ Wt) {
  constexpr int ROWS = 16 * NT;
  constexpr int PITCH = KC + 1;
  constexpr int TPR = KC;                      // threads per staged row
  constexpr int RSTEP = kBlock / TPR;          // rows per load round
  constexpr int PER = (ROWS + RSTEP - 1) / RSTEP;
  __shared__ T s[ROWS][PITCH];
  typedef typename AccOf<T>::type Acc;
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63, r16 = l & 15, q = l >> 4;
  const i64 k_beg = (i64)blockIdx.x * kper;
  const i64 k_end = min(ng, k_beg + kper);
  Acc acc[9];
  double accd[9][4];
#pragma unroll
  for (int u = 0; u < 9; ++u) {
    acc[u] = Acc{0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r) accd[u][r] = 0.0;
  }
  const int col = t % TPR, row0 = t / TPR;
  T nxt[PER];
  T nxh[TRIAL ? PER : 1];
  T ca[TRIAL ? PER : 1];
  const double tau = TRIAL ? dtau[0] * tscale : 0.0;
  if (TRIAL) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int row = row0 + RSTEP * e;
      // clamped load, then the test: a guarded load would wait in a branch of its own
      const double sv = sig[min(row, N - 1)];
      ca[e] = (row < N) ? (T)(1.0 + tau * sv) : (T)0;
    }
  }
  auto load = [&](i64 k0) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int row = row0 + RSTEP * e;
      const i64 g = k0 + col;
      const bool ok = row < N && g < k_end;
      nxt[e] = ok ? A[(i64)row * ng + g] : (T)0;
      if (TRIAL) nxh[e] = ok ? HW[(i64)row * ng + g] : (T)0;
    }
  };
  if (k_beg < k_end) load(k_beg);
  const T tt = (T)tau;
  for (i64 k0 = k_beg; k0 < k_end; k0 += KC) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int row = row0 + RSTEP * e;
      T v = nxt[e];
      if (TRIAL) {
        v = ca[e] * v - tt * nxh[e];
        const i64 g = k0 + col;
        if (row < N && g < k_end) Wt[(i64)row * ng + g] = v;
      }
      if (row < ROWS) s[row][col] = v;
    }
    __syncthreads();
    if (k0 + KC < k_end) load(k0 + KC);
    switch (w) {
      case 0: gram_chunk<T, NT, 0, KC, PITCH>(s, acc, r16, q); break;
      case 1: gram_chunk<T, NT, 1, KC, PITCH>(s, acc, r16, q); break;
      case 2: gram_chunk<T, NT, 2, KC, PITCH>(s, acc, r16, q); break;
      default: gram_chunk<T, NT, 3, KC, PITCH>(s, acc, r16, q); break;
    }
    __syncthreads();
    if (sizeof(T) == 4) {
#pragma unroll
      for (int u = 0; u < 9; ++u) {
#pragma unroll
        for (int r = 0; r < 4; ++r) accd[u][r] += (double)acc[u][r];
        acc[u] = Acc{0, 0, 0, 0};
      }
    }
  }
  double *outp = part + (i64)blockIdx.x * 128 * 128;
#pragma unroll
  for (int u = 0; u < 9; ++u) {
    int rt, ct;
    gram_tile_runtime(w, u, rt, ct);
    if (rt < NT && ct < NT) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * rt + out_row<T>(q, r);
        const int cl = 16 * ct + r16;
        outp[row * 128 + cl] = (sizeof(T) == 4) ? accd[u][r] : (double)acc[u][r];
      }
    }
  }
}

// The same contraction with the FP32 values rounded to BF16 (MFMA 16x16x32,
// FP32 accumulation per 32 points, flushed into FP64).  Each chunk is staged
// in LDS already rounded, so an MFMA fragment is one 16-byte read; with TRIAL
// the kernel also forms and stores the FP32 trial point W - tau Z it rounds.
template <int NT, int KC, bool TRIAL>
__global__ __launch_bounds__(kBlock) void k_gram_small_bf16(const float *__restrict__ A, int N,
                                                               i64 ng, i64 kper,
                                                               double *__restrict__ part,
                                                               const float *__restrict__ HW,
                                                               const double *__restrict__ sig,
                                                               const double *__restrict__ dtau,
                                                               double tscale,
                                                               float *__restrict__ Wt) {
  constexpr int ROWS = 16 * NT;
  constexpr int PB = KC + 8;  // BF16 rows of 16-byte multiples: fragments are single reads
  constexpr int TPR = KC;
  constexpr int RSTEP = kBlock / TPR;
  constexpr int PER = (ROWS + RSTEP - 1) / RSTEP;
  __shared__ __attribute__((aligned(16))) __bf16 s[ROWS][PB];
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63, r16 = l & 15, q = l >> 4;
  const i64 k_beg = (i64)blockIdx.x * kper;
  const i64 k_end = min(ng, k_beg + kper);
  double accd[9][4];
#pragma unroll
  for (int u = 0; u < 9; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) accd[u][r] = 0.0;
  const int col = t % TPR, row0 = t / TPR;
  float nxt[PER];
  float nxh[TRIAL ? PER : 1];
  float ca[TRIAL ? PER : 1];
  const double tau = TRIAL ? dtau[0] * tscale : 0.0;
  if (TRIAL) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int row = row0 + RSTEP * e;
      const double sv = sig[min(row, N - 1)];  // clamped load, then the test
      ca[e] = (row < N) ? (float)(1.0 + tau * sv) : 0.0f;
    }
  }
  // chunks with every row and point inside the range load and store with no
  // per-element tests (the tests would put each access in a branch of its own)
  const bool all_rows = N == ROWS;
  // Whole chunks address row row0 + RSTEP e as a per-lane pointer plus a
  // uniform row step.  The lane offset passes through an empty asm each
  // time, so the compiler cannot hoist one 64-bit pointer per row out of the
  // chunk loop (which would hold 2 PER registers per array for the launch).
  const i64 lane_off = (i64)row0 * ng + col;
  const i64 rstep = (i64)RSTEP * ng;
  auto lane_base = [&](i64 k0) __attribute__((always_inline)) -> i64 {
    i64 o = lane_off;
    asm volatile("" : "+v"(o));
    return o + k0;
  };
  auto load = [&](i64 k0) __attribute__((always_inline)) {
    const i64 g = k0 + col;
    if (all_rows && k0 + KC <= k_end) {
      const i64 o = lane_base(k0);
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        nxt[e] = A[o + e * rstep];
        if (TRIAL) nxh[e] = HW[o + e * rstep];
      }
    } else {
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int row = row0 + RSTEP * e;
        const bool ok = row < N && g < k_end;
        nxt[e] = ok ? A[(i64)row * ng + g] : 0.0f;
        if (TRIAL) nxh[e] = ok ? HW[(i64)row * ng + g] : 0.0f;
      }
    }
  };
  if (k_beg < k_end) load(k_beg);
  const float tt = (float)tau;
  for (i64 k0 = k_beg; k0 < k_end; k0 += KC) {
    const bool full = all_rows && k0 + KC <= k_end;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int row = row0 + RSTEP * e;
      float v = nxt[e];
      if (TRIAL) v = ca[e] * v - tt * nxh[e];
      if (row < ROWS) s[row][col] = (__bf16)v;
      nxt[e] = v;
    }
    if (TRIAL) {
      const i64 g = k0 + col;
      if (full) {
        const i64 o = lane_base(k0);
#pragma unroll
        for (int e = 0; e < PER; ++e) Wt[o + e * rstep] = nxt[e];
      } else {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          const int row = row0 + RSTEP * e;
          if (row < N && g < k_end) Wt[(i64)row * ng + g] = nxt[e];
        }
      }
    }
    __syncthreads();
    if (k0 + KC < k_end) load(k0 + KC);
    switch (w) {
      case 0: gram_chunk_bf16<NT, 0, KC, PB>(s, accd, r16, q); break;
      case 1: gram_chunk_bf16<NT, 1, KC, PB>(s, accd, r16, q); break;
      case 2: gram_chunk_bf16<NT, 2, KC, PB>(s, accd, r16, q); break;
      default: gram_chunk_bf16<NT, 3, KC, PB>(s, accd, r16, q); break;
    }
    __syncthreads();
  }
  double *outp = part + (i64)blockIdx.x * 128 * 128;
#pragma unroll
  for (int u = 0; u < 9; ++u) {
    int rt, ct;
    gram_tile_runtime(w, u, rt, ct);
    if (rt < NT && ct < NT) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        outp[(16 * rt + 4 * q + r) * 128 + 16 * ct + r16] = accd[u][r];
    }
  }
}

// Row tiles of the N <= 128 apply owned by wave W: W and 7 - W (balances the
// triangle: 4(W+1) + 4(8-W) = 36 k-steps of 4 per wave).
template <typename T, int NT, int W>
__device__ inline void apply_load_a(const T *__restrict__ D, int N, T (&a0)[4 * NT],
                                    T (&a1)[4 * NT], int r16, int q) {
  constexpr int jt0 = W, jt1 = 7 - W;
  // clamped, always-valid addresses; entries outside the factor's triangle
  // or size are zeroed after the load (no branch per load)
#pragma unroll
  for (int ks = 0; ks < 4 * NT; ++ks) {
    const int i = 4 * ks + q;
    const int j0 = 16 * jt0 + r16, j1 = 16 * jt1 + r16;
    const int ic = min(i, N - 1);
    const T v0 = D[(i64)min(j0, N - 1) * N + ic];
    const T v1 = D[(i64)min(j1, N - 1) * N + ic];
    a0[ks] = ((jt0 < NT) & (ks < 4 * (jt0 + 1)) & (j0 < N) & (i < N)) ? v0 : (T)0;
    a1[ks] = ((jt1 < NT) & (ks < 4 * (jt1 + 1)) & (j1 < N) & (i < N)) ? v1 : (T)0;
  }
}

// FP32 value as three BF16 pieces, v = hi + mid + lo exactly (each split
// takes the next 8 significant bits; barring underflow of lo, the three carry
// all 24 bits of the FP32 significand).
__device__ inline void split3_bf16(float v, __bf16 &hi, __bf16 &mid, __bf16 &lo) {
  hi = (__bf16)v;
  const float r1 = v - (float)hi;
  mid = (__bf16)r1;
  lo = (__bf16)(r1 - (float)mid);
}

constexpr int kS3P = 136;  // LDS pitch (BF16) of a point's 128 orbitals: 16-byte aligned rows
constexpr int kS3X = 36;   // LDS pitch (FP32) of an orbital's 32 points

// FP32 apply for N <= 128 on BF16 MFMA: out = X + D X with D = L^-1 - I
// (FP32, lower triangular), both operands split into three BF16 pieces.  Of
// the nine piece products the six down to 2^-16 of the leading one are
// summed (smallest first) in the FP32 accumulator; the three dropped are at
// most 2^-24 relative, so the product keeps the accuracy of an FP32
// contraction at 3/8 of the FP32 matrix-core cycles (six 16x16x32 BF16
// products against eight 16x16x4 FP32 ones per 32 orbitals).  Four waves,
// wave W owning row tiles W and 7 - W (which balances the triangle); the
// workgroup walks 32-point blocks staged in LDS (FP32 for the identity term
// and the three pieces transposed to [point][orbital] for the MFMA B operand)
// while the next block is loaded.  Optional fused density rho[g] = sum_j
// occ_j out[j][g]^2 (FP64): each wave leaves its partial of a block in LDS and
// the partials are summed after the next block's first barrier.  The FP32
// block has a row pitch of 36 floats: the epilogue's reads (four rows apart
// across lane groups) then fall in distinct banks, and so do the loader's
// writes, whose wave halves take rows eight apart.
template <int NT, int W>
__device__ __attribute__((always_inline)) inline void apply_s3_body(
    const float *__restrict__ D, const float *__restrict__ X, float *__restrict__ out, int N,
    i64 ng, const double *__restrict__ occ, double *__restrict__ rho, float (*xs)[kS3X],
    __bf16 (*xp)[32][kS3P], double (*srho)[4][32]) {
  constexpr int GC = 32, NC = 2;
  constexpr int NOG = 2 * ((NT + 1) / 2);  // 16-orbital loader groups: whole 32-orbital chunks
  constexpr int jt0 = W, jt1 = 7 - W;
  constexpr int kc0 = jt0 < NT ? (16 * jt0 + 15) / 32 + 1 : 0;  // chunks reaching row tile jt0
  constexpr int kc1 = jt1 < NT ? (16 * jt1 + 15) / 32 + 1 : 0;
  constexpr int kcm = kc0 > kc1 ? kc0 : kc1;
  const int t = threadIdx.x;
  const int l = t & 63, r16 = l & 15, q = l >> 4;
  // D fragments (A operand): row 16 jt + r16, orbitals 32 kc + 8 q .. + 7
  bf8 d0[kc0 > 0 ? kc0 : 1][3], d1[kc1 > 0 ? kc1 : 1][3];
  auto load_d = [&](bf8 (*d)[3], int jt, int nkc) __attribute__((always_inline)) {
    const int j = 16 * jt + r16;
    for (int kc = 0; kc < nkc; ++kc) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int i = 32 * kc + 8 * q + e;
        // clamped load, zeroed outside the factor (no branch per load)
        const float dv = D[(i64)min(j, N - 1) * N + min(i, N - 1)];
        const float v = ((j < N) & (i < N)) ? dv : 0.0f;
        __bf16 a, b, c;
        split3_bf16(v, a, b, c);
        d[kc][0][e] = a;
        d[kc][1][e] = b;
        d[kc][2][e] = c;
      }
    }
  };
  if (kc0 > 0) load_d(d0, jt0, kc0);
  if (kc1 > 0) load_d(d1, jt1, kc1);
  // occupations of the lane's output rows (clamped loads under one uniform
  // test; zero for rows outside the problem)
  double occv[2][4] = {};
  if (rho != nullptr) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int jt = u == 0 ? jt0 : jt1;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = 16 * jt + 4 * q + r;
        const double o = occ[min(j, N - 1)];
        occv[u][r] = ((jt < NT) & (j < N)) ? o : 0.0;
      }
    }
  }
  // loader: point col; orbitals 32 wv + 8 hf + e and 32 wv + 16 + 8 hf + e
  // (e < 8) for wave wv and wave half hf; rows past N load as zero
  const bool all_rows = N == 16 * NOG;
  const i64 nblk = (ng + GC - 1) / GC;
  const int col = t & 31, hf = (t >> 5) & 1, wv = t >> 6;
  const bool loader = 2 * wv < NOG;
  auto lrow = [&](int e) { return 32 * wv + 8 * hf + (e < 8 ? e : e + 8); };
  float na[16];
  auto load = [&](float (&dst)[16], i64 blk) __attribute__((always_inline)) {
    if (!loader) return;
    const i64 g = blk * GC + col;
    if (all_rows && blk * GC + GC <= ng) {
#pragma unroll
      for (int e = 0; e < 16; ++e) dst[e] = X[(i64)lrow(e) * ng + g];
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = lrow(e);
        dst[e] = (row < N && g < ng) ? X[(i64)row * ng + g] : 0.0f;
      }
    }
  };
  auto flush_rho = [&](i64 pblk, int pbuf) __attribute__((always_inline)) {
    if (t < GC) {
      const i64 g = pblk * GC + t;
      if (g < ng)
        rho[g] = srho[pbuf][0][t] + srho[pbuf][1][t] + srho[pbuf][2][t] + srho[pbuf][3][t];
    }
  };
  i64 pending = -1;
  int buf = 0;
  i64 blk = blockIdx.x;
  const i64 G = gridDim.x;
  if (blk < nblk) load(na, blk);
  for (; blk < nblk; blk += G) {
    __syncthreads();
    if (rho != nullptr && pending >= 0) flush_rho(pending, buf ^ 1);
    if (loader) {
#pragma unroll
      for (int e = 0; e < 16; ++e) xs[lrow(e)][col] = na[e];
#pragma unroll
      for (int hlf = 0; hlf < 2; ++hlf) {
        bf8 vh, vm, vl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 a, b, c;
          split3_bf16(na[8 * hlf + e], a, b, c);
          vh[e] = a;
          vm[e] = b;
          vl[e] = c;
        }
        const int o = lrow(8 * hlf);
        *(bf8 *)&xp[0][col][o] = vh;
        *(bf8 *)&xp[1][col][o] = vm;
        *(bf8 *)&xp[2][col][o] = vl;
      }
    }
    __syncthreads();
    if (blk + G < nblk) load(na, blk + G);
    f4 acc0[NC], acc1[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      acc0[cc] = f4{0, 0, 0, 0};
      acc1[cc] = f4{0, 0, 0, 0};
    }
#pragma unroll
    for (int kc = 0; kc < kcm; ++kc) {
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const bf8 bh = *(const bf8 *)&xp[0][16 * cc + r16][32 * kc + 8 * q];
        const bf8 bm = *(const bf8 *)&xp[1][16 * cc + r16][32 * kc + 8 * q];
        const bf8 bl = *(const bf8 *)&xp[2][16 * cc + r16][32 * kc + 8 * q];
        auto prod = [&](const bf8 (&a)[3], f4 c) __attribute__((always_inline)) {
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], bm, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], bh, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bl, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], bh, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bm, c, 0, 0, 0);
          return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bh, c, 0, 0, 0);
        };
        if (kc < kc0) acc0[cc] = prod(d0[kc], acc0[cc]);
        if (kc < kc1) acc1[cc] = prod(d1[kc], acc1[cc]);
      }
    }
    const i64 g0 = blk * GC;
    double rp[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) rp[cc] = 0.0;
    auto epilogue = [&](auto tested) __attribute__((always_inline)) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int jt = u == 0 ? jt0 : jt1;
        if (jt >= NT) continue;
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
          const i64 g = g0 + 16 * cc + r16;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j = 16 * jt + 4 * q + r;
            const float v = xs[j][16 * cc + r16] + (u == 0 ? acc0[cc][r] : acc1[cc][r]);
            if (!decltype(tested)::value || (j < N && g < ng)) {
              out[(i64)j * ng + g] = v;
              rp[cc] += occv[u][r] * ((double)v * (double)v);
            }
          }
        }
      }
    };
    if (all_rows && g0 + GC <= ng)
      epilogue(std::false_type());
    else
      epilogue(std::true_type());
    if (rho != nullptr) {
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        double v = rp[cc];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (q == 0) srho[buf][W][16 * cc + r16] = v;
      }
      pending = blk;
      buf ^= 1;
    }
  }
  if (rho != nullptr && pending >= 0) {
    __syncthreads();
    flush_rho(pending, buf ^ 1);
  }
}

template <int NT>
__global__ __launch_bounds__(kBlock) void k_apply_s3(const float *__restrict__ D,
                                                     const float *__restrict__ X,
                                                     float *__restrict__ out, int N, i64 ng,
                                                     const double *__restrict__ occ,
                                                     double *__restrict__ rho) {
  __shared__ float xs[16 * 2 * ((NT + 1) / 2)][kS3X];
  __shared__ __attribute__((aligned(16))) __bf16 xp[3][32][kS3P];
  __shared__ double srho[2][4][32];
  switch (threadIdx.x >> 6) {
    case 0: apply_s3_body<NT, 0>(D, X, out, N, ng, occ, rho, xs, xp, srho); break;
    case 1: apply_s3_body<NT, 1>(D, X, out, N, ng, occ, rho, xs, xp, srho); break;
    case 2: apply_s3_body<NT, 2>(D, X, out, N, ng, occ, rho, xs, xp, srho); break;
    default: apply_s3_body<NT, 3>(D, X, out, N, ng, occ, rho, xs, xp, srho); break;
  }
}

// ---------------------------------------------------------------- 8-wave apply

constexpr int kAB = 512;  // threads of the 8-wave apply kernels

// One 16-point column group cc of the apply for wave pair W (row tiles W and
// 7 - W): acc0/acc1 += D_tile X[:, 16 cc .. 16 cc + 15].  TRANS swaps the
// MFMA operands, which leaves (D X)^T in the accumulators (lane l then holds
// grid points 4 (l / 16) + r of orbital l % 16).
template <typename T, int NT, int W, int PITCH, bool TRANS, typename Acc>
__device__ inline void apply_cc(const T (*xs)[PITCH], const T (&a0)[4 * NT],
                                const T (&a1)[4 * NT], Acc &acc0, Acc &acc1, int cc, int r16,
                                int q) {
  constexpr int jt0 = W, jt1 = 7 - W;
  constexpr int ke0 = jt0 < NT ? 4 * (jt0 + 1) : 0;
  constexpr int ke1 = jt1 < NT ? 4 * (jt1 + 1) : 0;
  constexpr int ke = ke0 > ke1 ? ke0 : ke1;
#pragma unroll
  for (int ks = 0; ks < ke; ++ks) {
    const T b = xs[4 * ks + q][16 * cc + r16];
    if (ks < ke0) acc0 = TRANS ? mfma(b, a0[ks], acc0) : mfma(a0[ks], b, acc0);
    if (ks < ke1) acc1 = TRANS ? mfma(b, a1[ks], acc1) : mfma(a1[ks], b, acc1);
  }
}

// FP64 apply for N <= 128: out[j][g] = X[j][g] + sum_{i<=j} D[j][i] X[i][g],
// D = L^-1 - I, on FP64 MFMA, optional fused density.  Wave w = (pair
// p = w % 4, half h = w / 4) owns row tiles p and 7 - p (36 k-steps of 4 for
// every pair) and the 16-point column group h of each 32-point block, so a
// wave keeps half the accumulators of the 4-wave form and twice as many
// waves share the CU.  Blocks of 32 grid points are staged through LDS; the
// next two blocks are in flight in registers while a block is computed.
template <typename T, int NT>
__global__ __launch_bounds__(kAB) void k_apply8(const T *__restrict__ D, const T *__restrict__ X,
                                                T *__restrict__ out, int N, i64 ng,
                                                const double *__restrict__ occ,
                                                double *__restrict__ rho) {
  constexpr int GC = 32;
  constexpr int ROWS = 16 * NT;
  constexpr int PITCH = GC + 1;
  constexpr int RSTEP = kAB / GC;
  constexpr int PER = (ROWS + RSTEP - 1) / RSTEP;
  __shared__ T xs[ROWS][PITCH];
  __shared__ double srho[2][4][GC];
  typedef typename AccOf<T>::type Acc;
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63, r16 = l & 15, q = l >> 4;
  const int pw = w & 3, h = w >> 2;
  T a0[4 * NT], a1[4 * NT];
  switch (pw) {
    case 0: apply_load_a<T, NT, 0>(D, N, a0, a1, r16, q); break;
    case 1: apply_load_a<T, NT, 1>(D, N, a0, a1, r16, q); break;
    case 2: apply_load_a<T, NT, 2>(D, N, a0, a1, r16, q); break;
    default: apply_load_a<T, NT, 3>(D, N, a0, a1, r16, q); break;
  }
  const int jt0 = pw, jt1 = 7 - pw;
  // occupations of the lane's output rows (clamped loads under one uniform
  // test; zero for rows outside the problem)
  double occv[2][4] = {};
  if (rho != nullptr) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int jt = u == 0 ? jt0 : jt1;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = 16 * jt + out_row<T>(q, r);
        const double o = occ[min(j, N - 1)];
        occv[u][r] = ((jt < NT) & (j < N)) ? o : 0.0;
      }
    }
  }
  const i64 nblk = (ng + GC - 1) / GC;
  const int col = t % GC, row0 = t / GC;
  const i64 G = gridDim.x;
  T na[PER] = {}, nb[PER] = {};
  // blocks with every row and point inside the problem load with no
  // per-element tests (the tests would put each load in a branch of its own)
  const bool all_rows = N == ROWS && ROWS % RSTEP == 0;
  auto load = [&](T (&dst)[PER], i64 blk) {
    const i64 g = blk * GC + col;
    if (all_rows && blk * GC + GC <= ng) {
#pragma unroll
      for (int e = 0; e < PER; ++e) dst[e] = X[(i64)(row0 + RSTEP * e) * ng + g];
      return;
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int row = row0 + RSTEP * e;
      dst[e] = (row < N && g < ng) ? X[(i64)row * ng + g] : (T)0;
    }
  };
  auto flush_rho = [&](i64 pblk, int pbuf) {
    if (t < GC) {
      const i64 g = pblk * GC + t;
      if (g < ng)
        rho[g] = srho[pbuf][0][t] + srho[pbuf][1][t] + srho[pbuf][2][t] + srho[pbuf][3][t];
    }
  };
  i64 pending = -1;
  int buf = 0;
  i64 blk = blockIdx.x;
  if (blk < nblk) load(na, blk);
  if (blk + G < nblk) load(nb, blk + G);
  for (; blk < nblk; blk += G) {
    __syncthreads();
    if (rho != nullptr && pending >= 0) flush_rho(pending, buf ^ 1);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int row = row0 + RSTEP * e;
      if (row < ROWS) xs[row][col] = na[e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PER; ++e) na[e] = nb[e];
    if (blk + 2 * G < nblk) load(nb, blk + 2 * G);
    Acc acc0 = Acc{0, 0, 0, 0}, acc1 = Acc{0, 0, 0, 0};
    switch (pw) {
      case 0: apply_cc<T, NT, 0, PITCH, false>(xs, a0, a1, acc0, acc1, h, r16, q); break;
      case 1: apply_cc<T, NT, 1, PITCH, false>(xs, a0, a1, acc0, acc1, h, r16, q); break;
      case 2: apply_cc<T, NT, 2, PITCH, false>(xs, a0, a1, acc0, acc1, h, r16, q); break;
      default: apply_cc<T, NT, 3, PITCH, false>(xs, a0, a1, acc0, acc1, h, r16, q); break;
    }
    const i64 g = blk * GC + 16 * h + r16;
    double rp = 0.0;
    auto epilogue = [&](auto tested) __attribute__((always_inline)) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int jt = u == 0 ? jt0 : jt1;
        if (jt >= NT) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = 16 * jt + out_row<T>(q, r);
          if (!decltype(tested)::value || (j < N && g < ng)) {
            const T v = xs[j][16 * h + r16] + (u == 0 ? acc0[r] : acc1[r]);
            out[(i64)j * ng + g] = v;
            rp += occv[u][r] * ((double)v * (double)v);
          }
        }
      }
    };
    // a full block stores without per-element tests
    if (all_rows && blk * GC + GC <= ng)
      epilogue(std::false_type());
    else
      epilogue(std::true_type());
    if (rho != nullptr) {
      rp += __shfl_xor(rp, 16, 64);
      rp += __shfl_xor(rp, 32, 64);
      if (q == 0) srho[buf][pw][16 * h + r16] = rp;
      pending = blk;
      buf ^= 1;
    }
  }
  if (rho != nullptr && pending >= 0) {
    __syncthreads();
    flush_rho(pending, buf ^ 1);
  }
}

// Gram tiles u in [U0, U1) of pair W (GramTile ownership: row tile W with
// column tiles W..7, then row tile 7 - W with 7 - W..7) over one 32-point
// chunk of W1 held in LDS as three BF16 pieces, W1 = hi + mid + lo exactly
// (split3_bf16).  Each tile sums the six piece products down to 2^-16 of the
// leading one (mid mid^T, lo hi^T, hi lo^T, mid hi^T, hi mid^T, hi hi^T,
// smallest first) in FP32 on BF16 MFMA, flushed into FP64 per chunk; the
// dropped products are 2^-24 relative and uncorrelated from point to point.
// Two pieces (16 significant bits) are not enough here: the residual's
// correlation with W1 over the few thousand points where an orbital lives
// leaves each diagonal entry off by ~5e-8 (1e-7 for the worst of 128
// orbitals), which the factor then turns into the same departure of the new
// block from orthonormality.  The fragments of two tiles are read ahead of
// their products, so two accumulation chains are in flight together.
template <int NT, int W, int U0, int U1, int PB>
__device__ inline void gram_tiles_split(const __bf16 (*hs)[PB], const __bf16 (*ms)[PB],
                                        const __bf16 (*ls)[PB], double (&gd)[U1 - U0][4],
                                        int r16, int q) {
  constexpr int NU = U1 - U0;
  constexpr int nfirst = 8 - W;
#pragma unroll
  for (int u0 = 0; u0 < NU; u0 += 2) {
    bf8 rh[2], rm[2], rl[2], ch[2], cm[2], cl[2];
    bool ok[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int u = u0 + v;
      const int rt = U0 + u < nfirst ? W : 7 - W;
      const int ct = U0 + u < nfirst ? W + U0 + u : (7 - W) + (U0 + u - nfirst);
      ok[v] = u < NU && rt < NT && ct < NT;
      const int ri = ok[v] ? rt : 0, ci = ok[v] ? ct : 0;  // unused tiles read tile 0
      rh[v] = *(const bf8 *)&hs[16 * ri + r16][8 * q];
      rm[v] = *(const bf8 *)&ms[16 * ri + r16][8 * q];
      rl[v] = *(const bf8 *)&ls[16 * ri + r16][8 * q];
      ch[v] = *(const bf8 *)&hs[16 * ci + r16][8 * q];
      cm[v] = *(const bf8 *)&ms[16 * ci + r16][8 * q];
      cl[v] = *(const bf8 *)&ls[16 * ci + r16][8 * q];
    }
    f4 c[2] = {f4{0, 0, 0, 0}, f4{0, 0, 0, 0}};
#define POU_GP(A, B)                                                                   \
  _Pragma("unroll") for (int v = 0; v < 2; ++v) if (ok[v]) c[v] =                     \
      __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[v], B[v], c[v], 0, 0, 0);
    POU_GP(rm, cm) POU_GP(rl, ch) POU_GP(rh, cl) POU_GP(rm, ch) POU_GP(rh, cm) POU_GP(rh, ch)
#undef POU_GP
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      if (u0 + v >= NU) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) gd[u0 + v][r] += (double)c[v][r];
    }
  }
}

// LDS stages of k_apply_gram8 for NT row tiles: X of one 32-point block as
// FP32 [orbital][point] (identity term) and BF16 hi/lo [point][orbital]
// (products); W1 of one block as three BF16 pieces [orbital][point].  FP32
// pitch 36: the loader's writes (wave halves eight rows apart) and the
// 16-byte identity reads fall in distinct banks.
template <int NT>
struct Ag8X {
  static constexpr int NCH = (16 * NT + 31) / 32;  // K chunks of 32 orbitals
  static constexpr int PX = 32 * NCH + 8;         // 16-byte aligned rows
  float xs[16 * NT][36];
  __bf16 xh[32][PX];
  __bf16 xl[32][PX];
};
template <int NT>
struct Ag8P {
  __bf16 hs[16 * NT][40];
  __bf16 ms[16 * NT][40];
  __bf16 ls[16 * NT][40];
};

// The body of k_apply_gram8 for wave (pair PW, half H), with the wave's row
// tiles and Gram tiles known at compile time, so that one block's apply and
// the previous block's Gram lie in one basic block the scheduler can
// interleave.  Two stages of each kind: block i is multiplied out of one X
// stage while block i + 1 is staged in the other, and the Gram of block i - 1
// reads one W1 stage while block i's pieces go to the other, so one barrier
// per block separates every write from the reads of the same stage.
template <int NT, int PW, int H>
__device__ __attribute__((always_inline)) inline void apply_gram8_body(
    const float *__restrict__ D, const float *__restrict__ X, int N, i64 ng,
    double *__restrict__ part, Ag8X<NT> &xa, Ag8X<NT> &xb, Ag8P<NT> &pa, Ag8P<NT> &pb) {
  typedef Ag8X<NT> XStage;
  typedef Ag8P<NT> PStage;
  constexpr int GC = 32;
  constexpr int ROWS = 16 * NT;
  constexpr int PB = 40;
  constexpr int NCH = XStage::NCH;
  const int t = threadIdx.x;
  const int l = t & 63, r16 = l & 15, q = l >> 4;
  constexpr int pw = PW, h = H;
  constexpr int jt0 = pw, jt1 = 7 - pw;
  // orbitals ROWS .. 32 NCH - 1 of the last K chunk are never loaded: keep their
  // pieces zero (an uninitialised NaN pattern times a zero D entry is NaN)
  if (32 * NCH > ROWS) {
    constexpr int PAD = 32 * NCH - ROWS;
    for (int e = t; e < GC * PAD; e += kAB) {
      xa.xh[e / PAD][ROWS + e % PAD] = (__bf16)0.0f;
      xa.xl[e / PAD][ROWS + e % PAD] = (__bf16)0.0f;
      xb.xh[e / PAD][ROWS + e % PAD] = (__bf16)0.0f;
      xb.xl[e / PAD][ROWS + e % PAD] = (__bf16)0.0f;
    }
  }
  // B operands: D^T fragments, lane = (output orbital 16 jt + r16, orbitals 32 kc + 8q .. +7)
  bf8 dh[2][NCH], dl[2][NCH];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int jt = u == 0 ? jt0 : jt1;
    const int j = 16 * jt + r16;
#pragma unroll
    for (int kc = 0; kc < NCH; ++kc) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int i = 32 * kc + 8 * q + e;
        // clamped load, zeroed outside the factor (no branch per load)
        const float dv = D[(i64)min(j, N - 1) * N + min(i, N - 1)];
        const float d = ((jt < NT) & (j < N) & (i < N)) ? dv : 0.0f;
        __bf16 a, b;
        split_bf16(d, a, b);
        dh[u][kc][e] = a;
        dl[u][kc][e] = b;
      }
    }
  }
  double gd[5][4];
#pragma unroll
  for (int u = 0; u < 5; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) gd[u][r] = 0.0;
  const i64 nblk = (ng + GC - 1) / GC;
  const int col = t % GC, rg = t / GC;  // rg < 16: orbitals 8 rg .. 8 rg + 7
  const bool loader = 8 * rg < ROWS;
  const i64 G = gridDim.x;
  float na[8] = {}, nb[8] = {};  // zero where no block is loaded into them
  // blocks with every row and point inside the problem load with no
  // per-element tests (the tests would put each load in a branch of its own)
  const bool all_rows = N == ROWS;
  auto load = [&](float (&dst)[8], i64 blk) __attribute__((always_inline)) {
    const i64 g = blk * GC + col;
    if (!loader) return;  // rows 8 rg .. 8 rg + 7 lie beyond the problem
    if (all_rows && blk * GC + GC <= ng) {
#pragma unroll
      for (int e = 0; e < 8; ++e) dst[e] = X[(i64)(8 * rg + e) * ng + g];
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int row = 8 * rg + e;
        dst[e] = (row < N && g < ng) ? X[(i64)row * ng + g] : 0.0f;
      }
    }
  };
  // X of one block into a stage: FP32 [orbital][point] for the identity term,
  // BF16 hi/lo [point][orbital] for the products
  auto stash = [&](XStage &xd) __attribute__((always_inline)) {
    if (!loader) return;
    bf8 vh, vl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      xd.xs[8 * rg + e][col] = na[e];
      __bf16 a, b;
      split_bf16(na[e], a, b);
      vh[e] = a;
      vl[e] = b;
    }
    *(bf8 *)&xd.xh[col][8 * rg] = vh;
    *(bf8 *)&xd.xl[col][8 * rg] = vl;
  };
  // W1 = X + (D X) for this wave's row tiles and points 16 h .. 16 h + 15, as
  // three BF16 pieces (rows beyond N are zero: X and D are)
  auto apply = [&](const XStage &xc, PStage &pd) __attribute__((always_inline)) {
    f4 acc[2] = {f4{0, 0, 0, 0}, f4{0, 0, 0, 0}};
#pragma unroll
    for (int kc = 0; kc < NCH; ++kc) {
      const bf8 ah = *(const bf8 *)&xc.xh[16 * h + r16][32 * kc + 8 * q];
      const bf8 al = *(const bf8 *)&xc.xl[16 * h + r16][32 * kc + 8 * q];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int jt = u == 0 ? jt0 : jt1;
        // chunk kc holds orbitals >= 32 kc; tile jt needs orbitals <= 16 jt + 15
        if (jt >= NT || 32 * kc > 16 * jt + 15) continue;
        f4 c = acc[u];
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, dl[u][kc], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, dl[u][kc], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, dh[u][kc], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, dh[u][kc], c, 0, 0, 0);
        acc[u] = c;
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int jt = u == 0 ? jt0 : jt1;
      if (jt >= NT) continue;
      const int j = 16 * jt + r16;
      const int p0 = 16 * h + 4 * q;
      __bf16 h4[4], m4[4], l4[4];
      const float4 x4 = *(const float4 *)&xc.xs[j][p0];
      const float xv[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
      for (int r = 0; r < 4; ++r) split3_bf16(xv[r] + acc[u][r], h4[r], m4[r], l4[r]);
      typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
      *(bf4 *)&pd.hs[j][p0] = bf4{h4[0], h4[1], h4[2], h4[3]};
      *(bf4 *)&pd.ms[j][p0] = bf4{m4[0], m4[1], m4[2], m4[3]};
      *(bf4 *)&pd.ls[j][p0] = bf4{l4[0], l4[1], l4[2], l4[3]};
    }
  };
  auto gram = [&](const PStage &pc) __attribute__((always_inline)) {
    if constexpr (H == 0)
      gram_tiles_split<NT, PW, 0, 5, PB>(pc.hs, pc.ms, pc.ls, gd, r16, q);
    else
      gram_tiles_split<NT, PW, 5, 9, PB>(pc.hs, pc.ms, pc.ls, *(double(*)[4][4]) & gd, r16, q);
  };
  // Invariant at the top of a step on block b: stage xc holds block b, na
  // holds block b + G and nb has block b + 2G in flight; the other W1 stage
  // holds block b - G when that exists.
  auto step = [&](const XStage &xc, XStage &xn, PStage &pd, const PStage &pp, i64 b,
                  bool prev) __attribute__((always_inline)) {
    if (b + G < nblk) {
      stash(xn);
#pragma unroll
      for (int e = 0; e < 8; ++e) na[e] = nb[e];
      if (b + 3 * G < nblk) load(nb, b + 3 * G);
    }
    apply(xc, pd);
    if (prev) gram(pp);
    __syncthreads();
  };
  i64 b = blockIdx.x;
  if (b < nblk) {
    load(na, b);
    if (b + G < nblk) load(nb, b + G);
    stash(xa);
#pragma unroll
    for (int e = 0; e < 8; ++e) na[e] = nb[e];
    if (b + 2 * G < nblk) load(nb, b + 2 * G);
    __syncthreads();
    for (bool prev = false;; prev = true) {
      step(xa, xb, pa, pb, b, prev);
      b += G;
      if (b >= nblk) {
        gram(pa);
        break;
      }
      step(xb, xa, pb, pa, b, true);
      b += G;
      if (b >= nblk) {
        gram(pb);
        break;
      }
    }
  }
  double *outp = part + (i64)blockIdx.x * 128 * 128;
  const int u0 = h == 0 ? 0 : 5, nu = h == 0 ? 5 : 4;
#pragma unroll
  for (int uu = 0; uu < 5; ++uu) {
    if (uu >= nu) continue;
    int rt, ct;
    gram_tile_runtime(pw, u0 + uu, rt, ct);
    if (rt < NT && ct < NT) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        outp[(16 * rt + 4 * q + r) * 128 + 16 * ct + r16] = gd[uu][r];
    }
  }
}

template <int NT>
__global__ __launch_bounds__(kAB) void k_apply_gram8(const float *__restrict__ D,
                                                     const float *__restrict__ X, int N, i64 ng,
                                                     double *__restrict__ part) {
  __shared__ __attribute__((aligned(16))) Ag8X<NT> xa, xb;
  __shared__ __attribute__((aligned(16))) Ag8P<NT> pa, pb;
  // the wave index as a scalar: a divergent branch would put EXEC masks
  // around the MFMA instructions of each path
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  switch (w) {
    case 0: apply_gram8_body<NT, 0, 0>(D, X, N, ng, part, xa, xb, pa, pb); break;
    case 1: apply_gram8_body<NT, 1, 0>(D, X, N, ng, part, xa, xb, pa, pb); break;
    case 2: apply_gram8_body<NT, 2, 0>(D, X, N, ng, part, xa, xb, pa, pb); break;
    case 3: apply_gram8_body<NT, 3, 0>(D, X, N, ng, part, xa, xb, pa, pb); break;
    case 4: apply_gram8_body<NT, 0, 1>(D, X, N, ng, part, xa, xb, pa, pb); break;
    case 5: apply_gram8_body<NT, 1, 1>(D, X, N, ng, part, xa, xb, pa, pb); break;
    case 6: apply_gram8_body<NT, 2, 1>(D, X, N, ng, part, xa, xb, pa, pb); break;
    default: apply_gram8_body<NT, 3, 1>(D, X, N, ng, part, xa, xb, pa, pb); break;
  }
}

// ---------------------------------------------------------------- Gram reduction

// G = dv * sum over splits of the 128 x 128 partial upper triangles; both
// halves.  Lane = element (coalesced over the 128 x 128 partial), the
// sixteen waves of a workgroup take every sixteenth split and combine
// through LDS in wave order.
constexpr int kRedW = 16;  // waves of the small Gram reduction
__global__ __launch_bounds__(64 * kRedW) void k_gram_reduce_small(const double *__restrict__ part,
                                                                  int N, int nsplit, double dv,
                                                                  double *__restrict__ G) {
  __shared__ double sacc[kRedW][64];
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int e = blockIdx.x * 64 + lane;  // element of the 128 x 128 partial
  // the partials hold the upper triangle only: skip ranges entirely below it
  if (((blockIdx.x * 64) & 127) + 63 < (int)((blockIdx.x * 64) >> 7)) return;
  // 16 independent loads in flight per lane (the sum is latency-bound: few
  // workgroups, each reading one 64-element column of every partial); with
  // sixteen waves, 256 splits take one round of loads
  constexpr int U = 16;
  double acc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) acc[u] = 0.0;
  int sp = w;
  for (; sp + kRedW * (U - 1) < nsplit; sp += kRedW * U) {
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] += part[(i64)(sp + kRedW * u) * 128 * 128 + e];
  }
  for (; sp < nsplit; sp += kRedW) acc[0] += part[(i64)sp * 128 * 128 + e];
#pragma unroll
  for (int h = U / 2; h >= 1; h /= 2)
#pragma unroll
    for (int u = 0; u < h; ++u) acc[u] += acc[u + h];
  sacc[w][lane] = acc[0];
  __syncthreads();
  if (w == 0) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kRedW; ++k) v += sacc[k][lane];
    v *= dv;
    const int r = e >> 7, c = e & 127;
    if (r <= c && c < N) {
      G[(i64)r * N + c] = v;
      G[(i64)c * N + r] = v;
    }
  }
}

// ---------------------------------------------------------------- N > 128, FP32

constexpr int kBB = 128;  // row block of the N > 128 Gram and apply kernels
constexpr int kBP = 40;   // LDS pitch (BF16) of a 32-wide chunk: 80-byte, 16-byte aligned rows
constexpr int kAT = 256;  // threads of the N > 128 apply
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

// Work item of workgroup b when items come in groups of `per` that read the
// same grid points: dispatch sends workgroup b to XCD b mod 8, so the members
// of a group take consecutive slots on one XCD and meet in its L2.
__device__ inline void xcd_group(int b, int per, int &group, int &member) {
  const int x = b & 7, j = b >> 3;
  group = x + 8 * (j / per);
  member = j % per;
}

// Gram of FP32 orbitals for N > 128 on BF16 MFMA: 128 x 128 output blocks
// (bi <= bj) over nsplit contiguous ranges of kper grid points (the grid is
// padded to a multiple of 8 ranges; the block pairs of one range share an XCD).
// Eight waves in a 4 x 2 grid: wave (rw, cw) holds rows 32 rw .. 32 rw + 31 and
// columns 64 cw .. 64 cw + 63 of the block (2 x 4 tiles of 16 x 16).  Per
// 64-point chunk the rows of both blocks are loaded as float4 (the next chunk
// in flight while the current one is multiplied), rounded to BF16 and stored in
// LDS as [row][point], double-buffered; each tile takes two 16x16x32 MFMAs per
// chunk, or with SPLIT the four products of the hi/lo pieces (FP32-accurate),
// whose FP32 sums are flushed into FP64 every chunk.  Without SPLIT (the first
// Cholesky-QR pass, whose factor is refined by the second) the FP32 sums run
// over the whole range: that keeps the kernel at two workgroups per CU.  On a
// diagonal block the wave whose tiles all lie below the diagonal skips the
// products (the reduction reads the upper triangle only).
template <bool SPLIT, bool VEC>
__global__ __launch_bounds__(kAB) __attribute__((amdgpu_waves_per_eu(SPLIT ? 2 : 4)))
void k_gram_big(const float *__restrict__ A, int N, i64 ng,
                                                  i64 kper, int nsplit, int npairs,
                                                  double *__restrict__ part) {
  constexpr int KC = 64;       // points per chunk
  constexpr int PG = KC + 8;   // LDS pitch (BF16): 144-byte rows, conflict-free 16-byte reads
  constexpr int NV = 2 * kBB * KC / 4 / kAB;  // float4 loads per thread per chunk (8)
  __shared__ __attribute__((aligned(16))) __bf16 sh[2][2][kBB][PG];
  __shared__ __attribute__((aligned(16))) __bf16 sl[2][SPLIT ? 2 : 1][SPLIT ? kBB : 1][PG];
  int split, pair;
  xcd_group(blockIdx.x, npairs, split, pair);
  if (split >= nsplit) return;  // padding to a multiple of 8 ranges (before any barrier)
  const int nb = (N + kBB - 1) / kBB;
  int bi, bj;
  decode_pair(pair, nb, bi, bj);
  const bool diag = bi == bj;
  const i64 k_beg = (i64)split * kper;
  const i64 k_end = min(ng, k_beg + kper);
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63, r16 = l & 15, q = l >> 4;
  const int rw = w >> 1, cw = w & 1;
  const bool idle = diag && cw == 0 && rw >= 2;
  // loader slot e: float4 f = t + 512 e, row f / 16 (block bi for e < NV / 2, bj
  // after), points 4 (f % 16) .. + 3.  Loads read clamped (always valid)
  // addresses and zero what lies outside, with non-short-circuit tests: no
  // branch, so they all stay in flight (a diagonal block loads its rows twice;
  // the second copy comes from the caches).
  // VEC (ng % 4 == 0 and 128 rows of a block span < 4 GiB): 32-bit offsets
  // inside the row block, fixed per lane (rows past N clamped to the last one:
  // their Gram entries are never read), on a uniform base per block and chunk;
  // the chunk start is clamped so that the last chunk ends at ng, and the points
  // it repeats are zeroed (a uniform test, false but for that chunk).
  float4 v[NV];
  unsigned voff[VEC ? NV : 1];
  const int c4l = (t & 15) * 4;  // the point offset of every slot of this lane
  if (VEC) {
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int row = (t + kAB * e) >> 4;
      const int rb = row < kBB ? bi : bj, r = row & (kBB - 1);
      voff[VEC ? e : 0] = (unsigned)((i64)min(r, N - 1 - rb * kBB) * ng + c4l);
    }
  }
  const float *abase = A + (i64)bi * kBB * ng, *bbase = A + (i64)bj * kBB * ng;
  auto load = [&](i64 k0) {
    if (VEC) {
      const i64 k0c = min(k0, ng - KC);
      const float *pa = abase + k0c, *pb = bbase + k0c;
#pragma unroll
      for (int e = 0; e < NV; ++e)
        v[e] = *(const float4 *)((e < NV / 2 ? pa : pb) + voff[VEC ? e : 0]);
      const int shift = (int)(k0 - k0c);
      if (shift > 0) {
        const bool ok = c4l >= shift;
#pragma unroll
        for (int e = 0; e < NV; ++e) {
          v[e].x = ok ? v[e].x : 0.f;
          v[e].y = ok ? v[e].y : 0.f;
          v[e].z = ok ? v[e].z : 0.f;
          v[e].w = ok ? v[e].w : 0.f;
        }
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int f = t + kAB * e;
      const int row = f >> 4, c4 = (f & 15) * 4;
      const int grow = row < kBB ? bi * kBB + row : bj * kBB + row - kBB;
      const bool rok = grow < N;
      const float *p = A + (i64)min(grow, N - 1) * ng;
      const i64 g = k0 + c4;
      float4 x;
      {
        x.x = p[min(g, ng - 1)];
        x.y = p[min(g + 1, ng - 1)];
        x.z = p[min(g + 2, ng - 1)];
        x.w = p[min(g + 3, ng - 1)];
        x.x = (rok & (g < k_end)) ? x.x : 0.f;
        x.y = (rok & (g + 1 < k_end)) ? x.y : 0.f;
        x.z = (rok & (g + 2 < k_end)) ? x.z : 0.f;
        x.w = (rok & (g + 3 < k_end)) ? x.w : 0.f;
      }
      v[e] = x;
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int f = t + kAB * e;
      const int row = f >> 4, c4 = (f & 15) * 4;
      const int blk = row >= kBB ? 1 : 0, r = row & (kBB - 1);
      const float x[4] = {v[e].x, v[e].y, v[e].z, v[e].w};
      bf4 hv, lv;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        __bf16 hh, ll;
        split_bf16(x[k], hh, ll);
        hv[k] = hh;
        lv[k] = ll;
      }
      *(bf4 *)&sh[b][blk][r][c4] = hv;
      if (SPLIT) *(bf4 *)&sl[b][SPLIT ? blk : 0][SPLIT ? r : 0][c4] = lv;
    }
  };
  f4 acc[2][4];
  double gd[SPLIT ? 2 : 1][SPLIT ? 4 : 1][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = f4{0, 0, 0, 0};
  if (SPLIT) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) gd[SPLIT ? a : 0][SPLIT ? c : 0][r] = 0.0;
  }
  auto compute = [&](int b) {
    if (idle) return;
#pragma unroll
    for (int ks = 0; ks < KC / 32; ++ks) {
      const int k8 = 32 * ks + 8 * q;
      bf8 ah[2], bh[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) ah[a] = *(const bf8 *)&sh[b][0][32 * rw + 16 * a + r16][k8];
#pragma unroll
      for (int c = 0; c < 4; ++c) bh[c] = *(const bf8 *)&sh[b][1][64 * cw + 16 * c + r16][k8];
      if (SPLIT) {
        bf8 al[2], bl[4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
          al[a] = *(const bf8 *)&sl[b][0][SPLIT ? 32 * rw + 16 * a + r16 : 0][k8];
#pragma unroll
        for (int c = 0; c < 4; ++c)
          bl[c] = *(const bf8 *)&sl[b][SPLIT ? 1 : 0][SPLIT ? 64 * cw + 16 * c + r16 : 0][k8];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            f4 x = acc[a][c];
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bl[c], x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[c], x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[c], x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[c], x, 0, 0, 0);
            acc[a][c] = x;
          }
      } else {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[c], acc[a][c], 0, 0, 0);
      }
    }
    if (SPLIT) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
          for (int r = 0; r < 4; ++r) gd[SPLIT ? a : 0][SPLIT ? c : 0][r] += (double)acc[a][c][r];
          acc[a][c] = f4{0, 0, 0, 0};
        }
    }
  };
  // the last chunk is peeled off the loop so that the loads and stores of the
  // next chunk are unconditional there: guarded by a shared test they would be
  // merged into one block ahead of the products, waiting on the loads at once
  const i64 nchunk = k_end > k_beg ? (k_end - k_beg + KC - 1) / KC : 0;
  if (nchunk > 0) {
    load(k_beg);
    stash(0);
  }
  __syncthreads();
  int b = 0;
  for (i64 ch = 0; ch + 1 < nchunk; ++ch, b ^= 1) {
    load(k_beg + KC * (ch + 1));
    compute(b);
    __builtin_amdgcn_sched_barrier(0);
    stash(b ^ 1);
    __syncthreads();
  }
  if (nchunk > 0) compute(b);
  if (idle) return;
  double *out = part + ((i64)split * npairs + pair) * kBB * kBB;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(32 * rw + 16 * a + 4 * q + r) * kBB + 64 * cw + 16 * c + r16] =
            SPLIT ? gd[SPLIT ? a : 0][SPLIT ? c : 0][r] : (double)acc[a][c][r];
}

// G = dv * sum over splits of the 128 x 128 block partials of k_gram_big; one
// thread per element of the upper block triangle, both halves of G written.
__global__ __launch_bounds__(kBlock) void k_gram_reduce_big(const double *__restrict__ part,
                                                            int N, int nsplit, int npairs,
                                                            double dv, double *__restrict__ G) {
  const i64 e = (i64)blockIdx.x * kBlock + threadIdx.x;
  const i64 stride = (i64)npairs * kBB * kBB;
  if (e >= stride) return;
  const int pair = (int)(e / (kBB * kBB)), rc = (int)(e % (kBB * kBB));
  const int ri = rc / kBB, cj = rc % kBB;
  int bi, bj;
  decode_pair(pair, (N + kBB - 1) / kBB, bi, bj);
  if (bi == bj && ri > cj) return;
  const int i = bi * kBB + ri, j = bj * kBB + cj;
  if (i >= N || j >= N) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int sp = 0;
  for (; sp + 3 < nsplit; sp += 4) {
    a0 += part[(i64)sp * stride + e];
    a1 += part[(i64)(sp + 1) * stride + e];
    a2 += part[(i64)(sp + 2) * stride + e];
    a3 += part[(i64)(sp + 3) * stride + e];
  }
  for (; sp < nsplit; ++sp) a0 += part[(i64)sp * stride + e];
  const double val = ((a0 + a1) + (a2 + a3)) * dv;
  G[(i64)i * N + j] = val;
  G[(i64)j * N + i] = val;
}

// FP64 Gram for N > 128: the block pairs, ranges and XCD grouping of
// k_gram_big, on FP64 MFMA 16x16x4 (lane l supplies row l%16 at point
// k = l/16; FP64 accumulation, so no flushes).  Eight waves in a 4 x 2 grid:
// wave (rw, cw) holds rows 32 rw .. 32 rw + 31 and columns 64 cw .. 64 cw + 63
// of the block.  16-point chunks of both row blocks are staged in LDS
// ([row][point], pitch 17 doubles: sixteen rows of one point column fall in
// distinct bank pairs), double-buffered with the next chunk in flight in
// registers.  VEC (ng even and 128 rows of a block span < 4 GiB): double2
// loads at fixed per-lane 32-bit offsets on a uniform block base, the last
// chunk clamped to the grid end and its repeated points zeroed.
template <bool VEC>
__global__ __launch_bounds__(kAB) __attribute__((amdgpu_waves_per_eu(4)))
void k_gram_big64(const double *__restrict__ A, int N, i64 ng,
                                                    i64 kper, int nsplit, int npairs,
                                                    double *__restrict__ part) {
  constexpr int KC = 16;
  constexpr int PD = KC + 1;
  constexpr int NV = 2 * kBB * KC / 2 / kAB;  // double2 loads per thread per chunk (4)
  __shared__ double sd[2][2][kBB][PD];
  int split, pair;
  xcd_group(blockIdx.x, npairs, split, pair);
  if (split >= nsplit) return;
  const int nb = (N + kBB - 1) / kBB;
  int bi, bj;
  decode_pair(pair, nb, bi, bj);
  const bool diag = bi == bj;
  const i64 k_beg = (i64)split * kper;
  const i64 k_end = min(ng, k_beg + kper);
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63, r16 = l & 15, q = l >> 4;
  const int rw = w >> 1, cw = w & 1;
  const bool idle = diag && cw == 0 && rw >= 2;
  // slot e: double2 f = t + 512 e, row f / 8 (block bi for e < NV / 2, bj after), points 2 (f % 8)
  const int c2 = (t & 7) * 2;
  double2 v[NV];
  unsigned voff[VEC ? NV : 1];
  if (VEC) {
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int row = (t + kAB * e) >> 3;
      const int rb = row < kBB ? bi : bj, r = row & (kBB - 1);
      voff[VEC ? e : 0] = (unsigned)((i64)min(r, N - 1 - rb * kBB) * ng + c2);
    }
  }
  const double *abase = A + (i64)bi * kBB * ng, *bbase = A + (i64)bj * kBB * ng;
  auto load = [&](i64 k0) {
    if (VEC) {
      const i64 k0c = min(k0, ng - KC);
      const double *pa = abase + k0c, *pb = bbase + k0c;
#pragma unroll
      for (int e = 0; e < NV; ++e)
        v[e] = *(const double2 *)((e < NV / 2 ? pa : pb) + voff[VEC ? e : 0]);
      const int shift = (int)(k0 - k0c);
      if (shift > 0) {
        const bool ok = c2 >= shift;
#pragma unroll
        for (int e = 0; e < NV; ++e) {
          v[e].x = ok ? v[e].x : 0.0;
          v[e].y = ok ? v[e].y : 0.0;
        }
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int row = (t + kAB * e) >> 3;
      const int grow = row < kBB ? bi * kBB + row : bj * kBB + row - kBB;
      const double *p = A + (i64)min(grow, N - 1) * ng;
      const i64 g = k0 + c2;
      double2 x;
      x.x = p[min(g, ng - 1)];
      x.y = p[min(g + 1, ng - 1)];
      x.x = (g < k_end) ? x.x : 0.0;
      x.y = (g + 1 < k_end) ? x.y : 0.0;
      v[e] = x;
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int row = (t + kAB * e) >> 3;
      const int blk = row >= kBB ? 1 : 0, r = row & (kBB - 1);
      sd[b][blk][r][c2] = v[e].x;
      sd[b][blk][r][c2 + 1] = v[e].y;
    }
  };
  d4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = d4{0, 0, 0, 0};
  auto compute = [&](int b) {
    if (idle) return;
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      double av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = sd[b][0][32 * rw + 16 * a + r16][4 * ks + q];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = sd[b][1][64 * cw + 16 * c + r16][4 * ks + q];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = mfma(av[a], bv[c], acc[a][c]);
    }
  };
  const i64 nchunk = k_end > k_beg ? (k_end - k_beg + KC - 1) / KC : 0;
  if (nchunk > 0) {
    load(k_beg);
    stash(0);
  }
  __syncthreads();
  int b = 0;
  for (i64 ch = 0; ch + 1 < nchunk; ++ch, b ^= 1) {
    load(k_beg + KC * (ch + 1));
    compute(b);
    __builtin_amdgcn_sched_barrier(0);
    stash(b ^ 1);
    __syncthreads();
  }
  if (nchunk > 0) compute(b);
  if (idle) return;
  double *out = part + ((i64)split * npairs + pair) * kBB * kBB;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(32 * rw + 16 * a + q + 4 * r) * kBB + 64 * cw + 16 * c + r16] = acc[a][c][r];
}

// Cross product C = A B^T of two orbital blocks (N x ng each, FP64 or FP32
// values) on FP64 MFMA, for the subspace matrix <(HW)^T W> and the residual
// of section 3.3: the structure of k_gram_big64 (128 x 128 output blocks over
// nsplit ranges of kper points, the ranges of one block pair on one XCD,
// 16-point chunks of both row blocks staged in LDS as doubles, double
// buffered) with the column block taken from B and every ordered block pair
// (bi, bj) = (pair / nb, pair % nb) computed in full.  FP32 values are
// converted exactly on load, so the products and sums are FP64.
template <typename T, bool VEC>
__global__ __launch_bounds__(kAB) __attribute__((amdgpu_waves_per_eu(4)))
void k_cross_big64(const T *__restrict__ A, const T *__restrict__ B, int N, i64 ng, i64 kper,
                   int nsplit, int npairs, double *__restrict__ part) {
  constexpr int KC = 16;
  constexpr int PD = KC + 1;
  constexpr int NV = 2 * kBB * KC / 2 / kAB;  // point pairs per thread per chunk (4)
  __shared__ double sd[2][2][kBB][PD];
  int split, pair;
  xcd_group(blockIdx.x, npairs, split, pair);
  if (split >= nsplit) return;
  const int nb = (N + kBB - 1) / kBB;
  const int bi = pair / nb, bj = pair % nb;
  const i64 k_beg = (i64)split * kper;
  const i64 k_end = min(ng, k_beg + kper);
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63, r16 = l & 15, q = l >> 4;
  const int rw = w >> 1, cw = w & 1;
  // slot e: pair f = t + 512 e, row f / 8 (block bi of A for e < NV / 2, block
  // bj of B after), points 2 (f % 8) and 2 (f % 8) + 1
  const int c2 = (t & 7) * 2;
  double2 v[NV];
  unsigned voff[VEC ? NV : 1];
  if (VEC) {
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int row = (t + kAB * e) >> 3;
      const int rb = row < kBB ? bi : bj, r = row & (kBB - 1);
      voff[VEC ? e : 0] = (unsigned)((i64)min(r, N - 1 - rb * kBB) * ng + c2);
    }
  }
  const T *abase = A + (i64)bi * kBB * ng, *bbase = B + (i64)bj * kBB * ng;
  typedef T pair_t __attribute__((ext_vector_type(2)));
  auto load = [&](i64 k0) {
    if (VEC) {
      const i64 k0c = min(k0, ng - KC);
      const T *pa = abase + k0c, *pb = bbase + k0c;
#pragma unroll
      for (int e = 0; e < NV; ++e) {
        const pair_t x = *(const pair_t *)((e < NV / 2 ? pa : pb) + voff[VEC ? e : 0]);
        v[e] = make_double2((double)x[0], (double)x[1]);
      }
      const int shift = (int)(k0 - k0c);
      if (shift > 0) {
        const bool ok = c2 >= shift;
#pragma unroll
        for (int e = 0; e < NV; ++e) {
          v[e].x = ok ? v[e].x : 0.0;
          v[e].y = ok ? v[e].y : 0.0;
        }
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int row = (t + kAB * e) >> 3;
      const bool first = row < kBB;
      const int grow = first ? bi * kBB + row : bj * kBB + row - kBB;
      const T *p = (first ? A : B) + (i64)min(grow, N - 1) * ng;
      const i64 g = k0 + c2;
      double2 x;
      x.x = (double)p[min(g, ng - 1)];
      x.y = (double)p[min(g + 1, ng - 1)];
      x.x = (g < k_end) ? x.x : 0.0;
      x.y = (g + 1 < k_end) ? x.y : 0.0;
      v[e] = x;
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int row = (t + kAB * e) >> 3;
      const int blk = row >= kBB ? 1 : 0, r = row & (kBB - 1);
      sd[b][blk][r][c2] = v[e].x;
      sd[b][blk][r][c2 + 1] = v[e].y;
    }
  };
  d4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = d4{0, 0, 0, 0};
  auto compute = [&](int b) {
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      double av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = sd[b][0][32 * rw + 16 * a + r16][4 * ks + q];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = sd[b][1][64 * cw + 16 * c + r16][4 * ks + q];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = mfma(av[a], bv[c], acc[a][c]);
    }
  };
  const i64 nchunk = k_end > k_beg ? (k_end - k_beg + KC - 1) / KC : 0;
  if (nchunk > 0) {
    load(k_beg);
    stash(0);
  }
  __syncthreads();
  int b = 0;
  for (i64 ch = 0; ch + 1 < nchunk; ++ch, b ^= 1) {
    load(k_beg + KC * (ch + 1));
    compute(b);
    __builtin_amdgcn_sched_barrier(0);
    stash(b ^ 1);
    __syncthreads();
  }
  if (nchunk > 0) compute(b);
  double *out = part + ((i64)split * npairs + pair) * kBB * kBB;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(32 * rw + 16 * a + q + 4 * r) * kBB + 64 * cw + 16 * c + r16] = acc[a][c][r];
}

// S[i][j] = dv / 2 (C[i][j] + C[j][i]) from the split partials of k_cross_big64
// (block pair (i / 128, j / 128) holds C rows i, columns j), fixed order.
__global__ __launch_bounds__(kBlock) void k_cross_reduce_big(const double *__restrict__ part,
                                                             int N, int nsplit, int npairs,
                                                             double dv, double *__restrict__ S) {
  const int nb = (N + kBB - 1) / kBB;
  const i64 stride = (i64)npairs * kBB * kBB;
  for (i64 e = (i64)blockIdx.x * kBlock + threadIdx.x; e < (i64)N * N;
       e += (i64)gridDim.x * kBlock) {
    const int i = (int)(e / N), j = (int)(e % N);
    if (j < i) continue;
    const i64 eij = (i64)((i / kBB) * nb + j / kBB) * kBB * kBB + (i % kBB) * kBB + j % kBB;
    const i64 eji = (i64)((j / kBB) * nb + i / kBB) * kBB * kBB + (j % kBB) * kBB + i % kBB;
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
    int sp = 0;
    for (; sp + 1 < nsplit; sp += 2) {
      a0 += part[(i64)sp * stride + eij];
      a1 += part[(i64)(sp + 1) * stride + eij];
      b0 += part[(i64)sp * stride + eji];
      b1 += part[(i64)(sp + 1) * stride + eji];
    }
    for (; sp < nsplit; ++sp) {
      a0 += part[(i64)sp * stride + eij];
      b0 += part[(i64)sp * stride + eji];
    }
    const double v = 0.5 * dv * ((a0 + a1) + (b0 + b1));
    S[(i64)i * N + j] = v;
    S[(i64)j * N + i] = v;
  }
}

// out = M X for a full N x N matrix M (FP64, row-major) and orbital blocks of
// FP64 or FP32 values, on FP64 MFMA: the (row block J, 128-point tile)
// workgroups and 4 x 2 wave grid of k_apply_big64 with the K loop over every
// 16-orbital chunk and no identity term.  FP32 values are converted exactly
// on load; the result is rounded to the element type once.  out must not
// alias X.
template <typename T>
__global__ __launch_bounds__(kAB) void k_mult_full64(const double *__restrict__ M,
                                                     const T *__restrict__ X, T *__restrict__ out,
                                                     int N, i64 ng) {
  constexpr int KC = 16;
  __shared__ double ds[2][kBB][KC + 1];
  __shared__ double xs[2][KC][kBB];
  const int nJ = (N + kBB - 1) / kBB;
  int ptile, J;
  xcd_group(blockIdx.x, nJ, ptile, J);
  const i64 g0 = (i64)ptile * kBB;
  if (g0 >= ng) return;
  const int nkc = (N + KC - 1) / KC;
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63, r16 = l & 15, q = l >> 4;
  const int rw = w >> 1, cw = w & 1;
  // loaders: M row dr, columns dc .. dc + 3 of the chunk; X orbital xo, points xq .. xq + 3
  const int dr = t >> 2, dc = 4 * (t & 3);
  const int jrow = J * kBB + dr;
  const double *mrow = M + (i64)min(jrow, N - 1) * N;
  const int xo = t >> 5, xq = 4 * (t & 31);
  double dv[4], xv[4];
  auto load = [&](int kc) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = KC * kc + dc + e;
      const double d = mrow[min(i, N - 1)];
      dv[e] = ((jrow < N) & (i < N)) ? d : 0.0;
    }
    const T *xr = X + (i64)min(KC * kc + xo, N - 1) * ng;
#pragma unroll
    for (int e = 0; e < 4; ++e) xv[e] = (double)xr[min(g0 + xq + e, ng - 1)];
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ds[b][dr][dc + e] = dv[e];
      xs[b][xo][xq + e] = xv[e];
    }
  };
  d4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = d4{0, 0, 0, 0};
  auto compute = [&](int b) {
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      double av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = ds[b][32 * rw + 16 * a + r16][4 * ks + q];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = xs[b][4 * ks + q][64 * cw + 16 * c + r16];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = mfma(av[a], bv[c], acc[a][c]);
    }
  };
  load(0);
  stash(0);
  __syncthreads();
  int kc = 0;
  for (; kc + 1 < nkc; ++kc) {
    load(kc + 1);
    compute(kc & 1);
    __builtin_amdgcn_sched_barrier(0);
    stash((kc & 1) ^ 1);
    __syncthreads();
  }
  compute(kc & 1);
  // lane (r16, q) of tile (a, c) holds rows q + 4 r of the tile at point r16
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = J * kBB + 32 * rw + 16 * a + q + 4 * r;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const i64 g = g0 + 64 * cw + 16 * c + r16;
        if (j < N && g < ng) out[(i64)j * ng + g] = (T)acc[a][c][r];
      }
    }
}

// out = X + D X for lower-triangular D = L^-1 - I (FP64 N x N) and FP64
// orbitals, N > 128, on FP64 MFMA: the (row block J, 128-point tile)
// workgroups of k_apply_big, eight waves in a 4 x 2 grid, wave (rw, cw)
// forming rows 32 rw .. 32 rw + 31 of the block at points 64 cw .. 64 cw + 63
// (2 x 4 tiles).  An FP64 MFMA needs one value per lane (lane l: row l%16 of
// D at k = l/16; X at k = l/16, point l%16), so X is staged in LDS in its own
// [orbital][point] layout and D as [row][k] (pitch 17 doubles), 16-orbital
// chunks, double-buffered.  Loads read clamped addresses: rows of X past N
// meet zero D columns, points past ng are never stored.  out must not alias X.
// With rhop, the block's share of the density as in k_apply_big.
__global__ __launch_bounds__(kAB) __attribute__((amdgpu_waves_per_eu(4)))
void k_apply_big64(const double *__restrict__ D, const double *__restrict__ X,
                   double *__restrict__ out, int N, i64 ng, const double *__restrict__ occ,
                   double *__restrict__ rhop) {
  constexpr int KC = 16;
  __shared__ double ds[2][kBB][KC + 1];
  __shared__ double xs[2][KC][kBB];
  const int nJ = (N + kBB - 1) / kBB;
  int ptile, jj;
  xcd_group(blockIdx.x, nJ, ptile, jj);
  const int J = nJ - 1 - jj;
  const i64 g0 = (i64)ptile * kBB;
  if (g0 >= ng) return;
  const int nkc = min(8 * (J + 1), (N + KC - 1) / KC);
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63, r16 = l & 15, q = l >> 4;
  const int rw = w >> 1, cw = w & 1;
  const int wkc = min(nkc, 8 * J + 2 * rw + 2);  // 16-orbital chunks reaching this wave's rows
  // loaders: D row dr, columns dc .. dc + 3 of the chunk; X orbital xo, points xq .. xq + 3
  const int dr = t >> 2, dc = 4 * (t & 3);
  const int jrow = J * kBB + dr;
  const double *drow = D + (i64)min(jrow, N - 1) * N;
  const int xo = t >> 5, xq = 4 * (t & 31);
  double dv[4], xv[4];
  auto load = [&](int kc) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = KC * kc + dc + e;
      const double d = drow[min(i, N - 1)];
      dv[e] = ((jrow < N) & (i < N)) ? d : 0.0;
    }
    const double *xr = X + (i64)min(KC * kc + xo, N - 1) * ng;
#pragma unroll
    for (int e = 0; e < 4; ++e) xv[e] = xr[min(g0 + xq + e, ng - 1)];
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ds[b][dr][dc + e] = dv[e];
      xs[b][xo][xq + e] = xv[e];
    }
  };
  d4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = d4{0, 0, 0, 0};
  auto compute = [&](int b, int kc) {
    if (kc >= wkc) return;
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      double av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = ds[b][32 * rw + 16 * a + r16][4 * ks + q];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = xs[b][4 * ks + q][64 * cw + 16 * c + r16];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = mfma(av[a], bv[c], acc[a][c]);
    }
  };
  load(0);
  stash(0);
  __syncthreads();
  int kc = 0;
  for (; kc + 1 < nkc; ++kc) {
    load(kc + 1);
    compute(kc & 1, kc);
    __builtin_amdgcn_sched_barrier(0);
    stash((kc & 1) ^ 1);
    __syncthreads();
  }
  compute(kc & 1, kc);
  // lane (r16, q) of tile (a, c) holds rows q + 4 r of the tile at point r16
  double rp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = J * kBB + 32 * rw + 16 * a + q + 4 * r;
      const double *xr = X + (i64)min(j, N - 1) * ng;
      double xi[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) xi[c] = xr[min(g0 + 64 * cw + 16 * c + r16, ng - 1)];
      const double fj = (rhop != nullptr && j < N) ? occ[j] : 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const i64 g = g0 + 64 * cw + 16 * c + r16;
        const double o = xi[c] + acc[a][c][r];
        rp[c] += fj * (o * o);
        if (j < N && g < ng) out[(i64)j * ng + g] = o;
      }
    }
  }
  if (rhop == nullptr) return;
  // sum over the row groups q of a tile (lanes r16 + 16 q), then over the four
  // row bands rw through LDS; point 64 cw + 16 c + r16
  __shared__ double srho[4][kBB];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double v = rp[c];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (q == 0) srho[rw][64 * cw + 16 * c + r16] = v;
  }
  __syncthreads();
  if (t < kBB && g0 + t < ng)
    rhop[(i64)J * ng + g0 + t] = (srho[0][t] + srho[1][t]) + (srho[2][t] + srho[3][t]);
}

// BF16 hi/lo pieces of the factor for k_apply_big, padded to whole 128-row
// blocks and 32-column chunks (zeros outside N x N, so the apply loads them
// without bounds tests): the correction D, or M = I + D (formed in FP32) when
// ginfo[1] = max |G - I| of the Gram the factor came from is 0.25 or more.
// Pieces are [NR][NC] with NR = N rounded up to 128, NC = N rounded up to 32.
__global__ __launch_bounds__(kBlock) void k_split_factor(const float *__restrict__ D,
                                                         const double *__restrict__ ginfo,
                                                         int N, __bf16 *__restrict__ Dh,
                                                         __bf16 *__restrict__ Dl) {
  const int NR = (N + kBB - 1) / kBB * kBB, NC = (N + 31) / 32 * 32;
  const float diag1 = (ginfo == nullptr || !(ginfo[1] >= 0.25)) ? 0.0f : 1.0f;
  const i64 total = (i64)NR * NC;
  for (i64 e = (i64)blockIdx.x * kBlock + threadIdx.x; e < total; e += (i64)gridDim.x * kBlock) {
    const int r = (int)(e / NC), c = (int)(e % NC);
    float d = 0.0f;
    if (r < N && c < N) d = D[(i64)r * N + c] + (r == c ? diag1 : 0.0f);
    __bf16 h, l;
    split_bf16(d, h, l);
    Dh[e] = h;
    Dl[e] = l;
  }
}

// out = X + D X for lower-triangular D (FP32 N x N, zero above the diagonal)
// and N > 128, on BF16 MFMA with both operands split into hi/lo pieces (four
// products, FP32 accumulation); the identity is added in FP32, so the rounding
// is relative to the correction D X.  That form loses accuracy when the factor
// shrinks the rows strongly (D near -I: the sum cancels), as in the first pass
// over an unnormalised block; when ginfo[1] (max |G - I| of the Gram the factor
// came from) is 0.25 or more, the kernel multiplies by M = I + D itself (the
// pieces from k_split_factor hold M then) and adds nothing.  With rhop, the
// workgroup also writes its rows' share of the density, sum_j occ_j out_j^2
// (FP64) over the block's 128 orbitals, to rhop[J][g].
//
// Workgroup = (row block J of 128 output orbitals, tile of 128 grid points);
// the row blocks of one point tile share an XCD, heaviest first.  Four waves
// in a 2 x 2 grid: wave (rw, cw) forms (D X)^T for orbitals 64 rw .. 64 rw + 63
// of the block and points 64 cw .. 64 cw + 63 (4 x 4 tiles), so each fragment
// read from LDS feeds four products.  The K loop runs over 32-orbital chunks
// up to the wave's diagonal; per chunk X is staged in LDS transposed
// ([point][orbital], split into hi/lo pieces on the way) and the block's rows
// of the factor pieces as [orbital][k], in two LDS stages, while two register
// sets keep the loads of the next two chunks in flight.  out must not alias X.
template <bool VEC>
__global__ __launch_bounds__(kAT) __attribute__((amdgpu_waves_per_eu(2)))
void k_apply_big(const __bf16 *__restrict__ Dh, const __bf16 *__restrict__ Dl,
                 const double *__restrict__ ginfo, const float *__restrict__ X,
                 float *__restrict__ out, int N, i64 ng, const double *__restrict__ occ,
                 double *__restrict__ rhop) {
  __shared__ __attribute__((aligned(16))) __bf16 xh[2][kBB][kBP];
  __shared__ __attribute__((aligned(16))) __bf16 xl[2][kBB][kBP];
  __shared__ __attribute__((aligned(16))) __bf16 dh[2][kBB][kBP];
  __shared__ __attribute__((aligned(16))) __bf16 dl[2][kBB][kBP];
  const int nJ = (N + kBB - 1) / kBB;
  int ptile, jj;
  xcd_group(blockIdx.x, nJ, ptile, jj);
  const int J = nJ - 1 - jj;
  const i64 g0 = (i64)ptile * kBB;
  if (g0 >= ng) return;  // padding workgroup: the whole group leaves before any barrier
  const int nkc = min(4 * (J + 1), (N + 31) / 32);
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63, r16 = l & 15, q = l >> 4;
  const int rw = w >> 1, cw = w & 1;
  const int wkc = min(nkc, 4 * J + 2 * rw + 2);  // chunks that reach this wave's orbitals
  const bool ident = ginfo == nullptr || !(ginfo[1] >= 0.25);
  // loaders: X point xp, orbitals xo .. xo + 15 of the chunk; factor row dr,
  // columns dc .. dc + 15
  // The orbital of an X load is uniform over a wave (xo is), so its row base
  // sits in scalar registers and each lane adds only its 32-bit point offset.
  // Rows past N and points past ng are clamped to the last ones instead of
  // tested: such rows meet zero factor columns (the pieces are padded), and a
  // point's column of D X depends on that point's values only, so clamped
  // points affect nothing that is stored.
  const int xp = t & (kBB - 1);
  const int xo = 16 * __builtin_amdgcn_readfirstlane(t >> 7);
  const int dr = t >> 1, dc = 16 * (t & 1);
  const unsigned gxc = (unsigned)min(g0 + xp, ng - 1);
  const int NC = (N + 31) / 32 * 32;
  const unsigned doff = (unsigned)(dr * NC + dc);
  const __bf16 *dhb = Dh + (i64)J * kBB * NC, *dlb = Dl + (i64)J * kBB * NC;
  struct Stage {
    float x[16];
    bf8 h0, h1, l0, l1;
  };
  auto load = [&](Stage &st, int kc) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int i = min(32 * kc + xo + e, N - 1);
      st.x[e] = (X + (i64)i * ng)[gxc];
    }
    const __bf16 *ph = dhb + 32 * kc, *pl = dlb + 32 * kc;
    st.h0 = *(const bf8 *)(ph + doff);
    st.h1 = *(const bf8 *)(ph + doff + 8);
    st.l0 = *(const bf8 *)(pl + doff);
    st.l1 = *(const bf8 *)(pl + doff + 8);
  };
  auto stash = [&](const Stage &st, int b) {
#pragma unroll
    for (int hlf = 0; hlf < 2; ++hlf) {
      bf8 hv, lv;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        __bf16 a, c;
        split_bf16(st.x[8 * hlf + e], a, c);
        hv[e] = a;
        lv[e] = c;
      }
      *(bf8 *)&xh[b][xp][xo + 8 * hlf] = hv;
      *(bf8 *)&xl[b][xp][xo + 8 * hlf] = lv;
    }
    *(bf8 *)&dh[b][dr][dc] = st.h0;
    *(bf8 *)&dh[b][dr][dc + 8] = st.h1;
    *(bf8 *)&dl[b][dr][dc] = st.l0;
    *(bf8 *)&dl[b][dr][dc + 8] = st.l1;
  };
  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = f4{0, 0, 0, 0};
  auto compute = [&](int b) __attribute__((always_inline)) {
    bf8 bh[4], bl[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      bh[a] = *(const bf8 *)&dh[b][64 * rw + 16 * a + r16][8 * q];
      bl[a] = *(const bf8 *)&dl[b][64 * rw + 16 * a + r16][8 * q];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const bf8 ah = *(const bf8 *)&xh[b][64 * cw + 16 * c + r16][8 * q];
      const bf8 al = *(const bf8 *)&xl[b][64 * cw + 16 * c + r16][8 * q];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        f4 x = acc[a][c];
        x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bl[a], x, 0, 0, 0);
        x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[a], x, 0, 0, 0);
        x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[a], x, 0, 0, 0);
        x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[a], x, 0, 0, 0);
        acc[a][c] = x;
      }
    }
  };
  // The staging of the next chunk (the split of X into BF16 pieces and the
  // LDS stores) is spread over the products of this one: an MFMA holds the
  // matrix pipe for 16 cycles, in which the wave can issue a few independent
  // vector instructions.
  auto interleave = [&]() __attribute__((always_inline)) {
    __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);  // factor fragment reads
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);  // X fragment reads
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one product
        __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // two vector instructions
        if (i % 8 == 7) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // an LDS store
      }
    }
  };
  // Two chunks per trip, every load and store unconditional (chunk indices
  // beyond the last are clamped to it: their stages are never multiplied), so
  // the compiler cannot merge them ahead of the products.  Invariant at the
  // top: LDS stage 0 holds chunk kc and register set sa has chunk kc + 1 in
  // flight.
  Stage sa, sb;
  load(sa, 0);
  stash(sa, 0);
  __syncthreads();
  load(sa, min(1, nkc - 1));
  for (int kc = 0; kc < nkc; kc += 2) {
    load(sb, min(kc + 2, nkc - 1));
    // the chunk test is uniform: products and staging stay in one block
    if (kc < wkc) {
      compute(0);
      stash(sa, 1);
      interleave();
    } else {
      stash(sa, 1);
    }
    __syncthreads();
    load(sa, min(kc + 3, nkc - 1));
    if (kc + 1 < wkc) {
      compute(1);
      stash(sb, 0);
      interleave();
    } else {
      stash(sb, 0);
    }
    __syncthreads();
  }
  // lane (r16, q) of tile (a, c) holds orbital 16 a + r16 at points 4 q .. 4 q + 3;
  // per row tile, the identity loads are issued (clamped) before any store
  double rp[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) rp[c][r] = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int j = J * kBB + 64 * rw + 16 * a + r16;
    const double fj = (rhop != nullptr && j < N) ? occ[j] : 0.0;
    float4 xi[4];
    const float *xr = X + (i64)min(j, N - 1) * ng;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const i64 g = g0 + 64 * cw + 16 * c + 4 * q;
      if (VEC) {
        xi[c] = *(const float4 *)(xr + min(g, ng - 4));
      } else {
        xi[c] = make_float4(xr[min(g, ng - 1)], xr[min(g + 1, ng - 1)], xr[min(g + 2, ng - 1)],
                            xr[min(g + 3, ng - 1)]);
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const i64 g = g0 + 64 * cw + 16 * c + 4 * q;
      const float wgt = ident ? 1.0f : 0.0f;
      const float4 x = xi[c];
      const float4 o = make_float4(wgt * x.x + acc[a][c][0], wgt * x.y + acc[a][c][1],
                                   wgt * x.z + acc[a][c][2], wgt * x.w + acc[a][c][3]);
      rp[c][0] += fj * ((double)o.x * (double)o.x);
      rp[c][1] += fj * ((double)o.y * (double)o.y);
      rp[c][2] += fj * ((double)o.z * (double)o.z);
      rp[c][3] += fj * ((double)o.w * (double)o.w);
      float *orow = out + (i64)j * ng + g;
      if (j < N) {
        if (VEC) {
          if (g < ng) *(float4 *)orow = o;
        } else {
          if (g < ng) orow[0] = o.x;
          if (g + 1 < ng) orow[1] = o.y;
          if (g + 2 < ng) orow[2] = o.z;
          if (g + 3 < ng) orow[3] = o.w;
        }
      }
    }
  }
  if (rhop == nullptr) return;
  // sum over the 16 orbitals of a tile (lanes of equal q), then over the two
  // row halves rw through LDS (stage buffers are free: every wave is past the
  // loop's last barrier); point 64 cw + 16 c + 4 q + r
  double(*srho)[kBB] = reinterpret_cast<double(*)[kBB]>(&xh[0][0][0]);
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = rp[c][r];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      if (r16 == 0) srho[rw][64 * cw + 16 * c + 4 * q + r] = v;
    }
  __syncthreads();
  if (t < kBB && g0 + t < ng) rhop[(i64)J * ng + g0 + t] = srho[0][t] + srho[1][t];
}

// Workgroups of `kernel` (`block` threads, static LDS only) that are resident
// on the current device at once: the grid of a kernel that walks its work in
// a grid-stride loop.  Cached per kernel and device.
// rho[g] = sum over the nJ row blocks of rhop[J][g], in block order
__global__ __launch_bounds__(kBlock) void k_rho_sum(const double *__restrict__ rhop, int nJ,
                                                    i64 ng, double *__restrict__ rho) {
  for (i64 g = (i64)blockIdx.x * kBlock + threadIdx.x; g < ng; g += (i64)gridDim.x * kBlock) {
    double v = 0.0;
    for (int J = 0; J < nJ; ++J) v += rhop[(i64)J * ng + g];
    rho[g] = v;
  }
}

int resident_workgroups(const void *kernel, int block = kBlock) {
  static std::mutex mu;
  static std::map<std::pair<const void *, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 512;
  }
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find({kernel, dev});
  if (it != cache.end()) return it->second;
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 512;
  }
  const int g = std::max(1, per) * std::max(1, cus);
  cache[{kernel, dev}] = g;
  return g;
}

}  // namespace

#define POU_NT_SWITCH(NTV, MACRO) \
  switch (NTV) {                  \
    case 1: MACRO(1); break;      \
    case 2: MACRO(2); break;      \
    case 3: MACRO(3); break;      \
    case 4: MACRO(4); break;      \
    case 5: MACRO(5); break;      \
    case 6: MACRO(6); break;      \
    case 7: MACRO(7); break;      \
    default: MACRO(8); break;     \
  }

int gram_split(int N, bool fp32) {
  if (N > 128) {
    // k_gram_big / k_gram_big64: a multiple of 8 ranges (one XCD per range),
    // the workgroup count as close to whole rounds of the resident ones as
    // 2 .. 6 rounds allow
    const int nb = (N + kBB - 1) / kBB;
    const int npairs = nb * (nb + 1) / 2;
    const int res =
        fp32 ? std::min(resident_workgroups((const void *)k_gram_big<true, true>, kAB),
                        resident_workgroups((const void *)k_gram_big<false, true>, kAB))
             : resident_workgroups((const void *)k_gram_big64<true>, kAB);
    int best = 8;
    double best_eff = 0.0;
    for (int rounds = 2; rounds <= 6; ++rounds) {
      const int ns = std::max(8, (rounds * res / npairs) / 8 * 8);
      const int wg = ns * npairs;
      const double eff = (double)wg / (double)(((wg + res - 1) / res) * res);
      if (eff > best_eff + 1e-9) {
        best_eff = eff;
        best = ns;
      }
    }
    return best;
  }
  const int NT = (N + 15) / 16;
  int g = 1 << 30;
  auto take = [&](const void *k) { g = std::min(g, resident_workgroups(k)); };
#define POU_GSPLIT(K)                                                         \
  if (fp32) {                                                                 \
    take((const void *)k_gram_small_bf16<K, 32, true>);                       \
    take((const void *)k_gram_small_bf16<K, 64, false>);                      \
    take((const void *)k_gram_small<float, K, 32, true>);                     \
    take((const void *)k_gram_small<float, K, 64, false>);                    \
    g = std::min(g, resident_workgroups((const void *)k_apply_gram8<K>, kAB)); \
  } else {                                                                    \
    take((const void *)k_gram_small<double, K, 32, true>);                    \
    take((const void *)k_gram_small<double, K, 32, false>);                   \
  }
  POU_NT_SWITCH(NT, POU_GSPLIT)
#undef POU_GSPLIT
  return std::max(256, std::min(g, 1024));
}

size_t split_factor_elems(int N) {
  return (size_t)((N + kBB - 1) / kBB * kBB) * (size_t)((N + 31) / 32 * 32);
}

size_t chol_workspace_doubles(int N) { return N <= 128 ? 0 : (size_t)528 * kTile; }

size_t gram_partial_doubles(int N, int nsplit) {
  if (N <= 128) return (size_t)nsplit * 128 * 128;
  const int nbb = (N + kBB - 1) / kBB;
  return (size_t)nsplit * (size_t)(nbb * (nbb + 1) / 2) * kBB * kBB;
}

template <typename T>
hipError_t launch_gram_partial(const T *A, int N, i64 ng, int nsplit, double *part,
                               hipStream_t s) {
  return launch_trial_gram<T>(A, nullptr, nullptr, nullptr, 0.0, nullptr, N, ng, nsplit, false,
                              part, s);
}

hipError_t launch_gram_partial_bf16(const float *A, int N, i64 ng, int nsplit, double *part,
                                    hipStream_t s) {
  return launch_trial_gram<float>(A, nullptr, nullptr, nullptr, 0.0, nullptr, N, ng, nsplit, true,
                                  part, s);
}

template <typename T>
hipError_t launch_trial_gram(const T *W, const T *HW, const double *sig, const double *dtau,
                             double tscale, T *Wt, int N, i64 ng, int nsplit, bool bf16,
                             double *part, hipStream_t s) {
  i64 kper = (ng + nsplit - 1) / nsplit;
  kper = ((kper + 63) / 64) * 64;
  const bool trial = HW != nullptr;
  if (N <= 128) {
    const int NT = (N + 15) / 16;
    if (bf16 && sizeof(T) == 4) {
      const float *Wf = (const float *)W;
      const float *Hf = (const float *)HW;
      float *Wtf = (float *)Wt;
#define POU_GB(K)                                                                          \
  if (trial)                                                                               \
    hipLaunchKernelGGL((k_gram_small_bf16<K, 32, true>), dim3(nsplit), dim3(kBlock), 0, s, Wf, \
                       N, ng, kper, part, Hf, sig, dtau, tscale, Wtf);                             \
  else                                                                                     \
    hipLaunchKernelGGL((k_gram_small_bf16<K, 64, false>), dim3(nsplit), dim3(kBlock), 0, s, Wf, \
                       N, ng, kper, part, Hf, sig, dtau, tscale, Wtf)
      POU_NT_SWITCH(NT, POU_GB)
#undef POU_GB
      return hipGetLastError();
    }
#define POU_GS(K)                                                                             \
  if (trial)                                                                                  \
    hipLaunchKernelGGL((k_gram_small<T, K, 32, true>), dim3(nsplit), dim3(kBlock), 0, s, W, N, \
                       ng, kper, part, HW, sig, dtau, tscale, Wt);                                     \
  else                                                                                        \
    hipLaunchKernelGGL((k_gram_small<T, K, (sizeof(T) == 4 ? 64 : 32), false>), dim3(nsplit),  \
                       dim3(kBlock), 0, s, W, N, ng, kper, part, HW, sig, dtau, tscale, Wt)
    POU_NT_SWITCH(NT, POU_GS)
#undef POU_GS
    return hipGetLastError();
  }
  if (trial) return hipErrorInvalidValue;  // the engine forms the trial separately for N > 128
  if (sizeof(T) == 8) {
    const int nbb = (N + kBB - 1) / kBB;
    const int npairs = nbb * (nbb + 1) / 2;
    kper = ((kper + 15) / 16) * 16;
    const int grid = ((nsplit + 7) / 8) * 8 * npairs;
    const bool vec = (ng & 1) == 0 && ng >= 16 && (i64)kBB * ng * 8 < (1LL << 32);
    if (vec)
      hipLaunchKernelGGL(k_gram_big64<true>, dim3(grid), dim3(kAB), 0, s, (const double *)W, N,
                         ng, kper, nsplit, npairs, part);
    else
      hipLaunchKernelGGL(k_gram_big64<false>, dim3(grid), dim3(kAB), 0, s, (const double *)W, N,
                         ng, kper, nsplit, npairs, part);
    return hipGetLastError();
  }
  if (sizeof(T) == 4) {
    const int nbb = (N + kBB - 1) / kBB;
    const int npairs = nbb * (nbb + 1) / 2;
    kper = ((kper + 63) / 64) * 64;
    const int grid = ((nsplit + 7) / 8) * 8 * npairs;
    const bool vec = (ng & 3) == 0 && ng >= 64 && (i64)kBB * ng * 4 < (1LL << 32);
#define POU_GBIG(SP, V)                                                                   \
  hipLaunchKernelGGL((k_gram_big<SP, V>), dim3(grid), dim3(kAB), 0, s, (const float *)W, N, ng, \
                     kper, nsplit, npairs, part)
    if (bf16) {
      if (vec) POU_GBIG(false, true);
      else POU_GBIG(false, false);
    } else {
      if (vec) POU_GBIG(true, true);
      else POU_GBIG(true, false);
    }
#undef POU_GBIG
    return hipGetLastError();
  }
return hipErrorInvalidValue;
}

hipError_t launch_gram_reduce(const double *part, int N, int nsplit, double dv, double *G,
                              hipStream_t s) {
  if (N <= 128) {
    hipLaunchKernelGGL(k_gram_reduce_small, dim3(128 * 128 / 64), dim3(64 * kRedW), 0, s, part,
                       N, nsplit, dv, G);
    return hipGetLastError();
  }
  const int nbb = (N + kBB - 1) / kBB;
  const int npairs = nbb * (nbb + 1) / 2;
  const int blocks = npairs * kBB * kBB / kBlock;
  hipLaunchKernelGGL(k_gram_reduce_big, dim3(blocks), dim3(kBlock), 0, s, part, N, nsplit, npairs,
                     dv, G);
  return hipGetLastError();
}

hipError_t launch_cholesky_inverse(double *G, double *Minv, float *D32, double *D64, int N,
                                   double *info, double *ws, hipStream_t s, int outs) {
  if (N <= 128) {
    hipLaunchKernelGGL((k_chol_blocked<true, 512>), dim3(1), dim3(512), 0, s, G, N, Minv, D32,
                       D64, info, ws, outs);
    return hipGetLastError();
  }
  // above 128 orbitals: the workspace variant (the library admits at most 512)
  if (N > 512 || ws == nullptr) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_chol_blocked<false, 1024>), dim3(1), dim3(1024), 0, s, G, N, Minv, D32,
                     D64, info, ws, outs);
  return hipGetLastError();
}

hipError_t launch_apply_gram(const float *D32, const float *X, int N, i64 ng, int nsplit,
                             double *part, hipStream_t s) {
  if (N > 128) return hipErrorInvalidValue;
  const int NT = (N + 15) / 16;
#define POU_AG(K)                                                                        \
  hipLaunchKernelGGL((k_apply_gram8<K>), dim3(nsplit), dim3(kAB), 0, s, D32, X, N, ng, part)
  POU_NT_SWITCH(NT, POU_AG)
#undef POU_AG
  return hipGetLastError();
}

hipError_t launch_combine_factors(const double *A, const double *B, double *M, double *D64,
                                  float *D32, int N, bool split_b, hipStream_t s) {
  if (N > 512) return hipErrorInvalidValue;
  const int NT = (N + 15) / 16;
  hipLaunchKernelGGL(k_combine_factors, dim3(NT * NT), dim3(64), 0, s, A, B, M, D64, D32, N,
                     split_b ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_lower(const double *M, const T *D, const T *X, T *out, int N, i64 ng,
                              const double *occ, double *rho, hipStream_t s,
                              const double *ginfo, void *split_ws, double *rho_part) {
  if (N <= 128) {
    const int NT = (N + 15) / 16;
    constexpr int GC = sizeof(T) == 4 ? 32 : 16;
    i64 nblk = (ng + GC - 1) / GC;
    // FP32: the 4-wave kernel (measured faster); FP64: the 8-wave kernel
#define POU_APPLY_SMALL(K)                                                                    \
  if (sizeof(T) == 4) {                                                                       \
    const int grid =                                                                          \
        (int)std::min<i64>(nblk, resident_workgroups((const void *)k_apply_s3<K>));           \
    hipLaunchKernelGGL((k_apply_s3<K>), dim3(grid), dim3(kBlock), 0, s, (const float *)D,     \
                       (const float *)X, (float *)out, N, ng, occ, rho);                      \
  } else {                                                                                    \
    const i64 nb8 = (ng + 31) / 32;                                                           \
    const int grid =                                                                          \
        (int)std::min<i64>(nb8, resident_workgroups((const void *)k_apply8<T, K>, kAB));      \
    hipLaunchKernelGGL((k_apply8<T, K>), dim3(grid), dim3(kAB), 0, s, D, X, out, N, ng, occ,  \
                       rho);                                                                  \
  }
    POU_NT_SWITCH(NT, POU_APPLY_SMALL)
#undef POU_APPLY_SMALL
    return hipGetLastError();
  }
  // above 128 orbitals the density goes through the row blocks' partials
  if (rho != nullptr && rho_part == nullptr) return hipErrorInvalidValue;
  double *rhop = rho != nullptr ? rho_part : nullptr;
  const int nJr = (N + kBB - 1) / kBB;
  auto rho_sum = [&]() {
    if (rho == nullptr) return;
    const int blocks = (int)std::min<i64>(2048, (ng + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_rho_sum, dim3(blocks), dim3(kBlock), 0, s, (const double *)rho_part,
                       nJr, ng, rho);
  };
  if (sizeof(T) == 4) {
    const int nJ = (N + kBB - 1) / kBB;
    const i64 npt = (ng + kBB - 1) / kBB;
    const i64 grid = ((npt + 7) / 8) * 8 * nJ;
    if (grid > 0x7fffffff || split_ws == nullptr) return hipErrorInvalidValue;
    __bf16 *Dh = (__bf16 *)split_ws;
    __bf16 *Dl = Dh + split_factor_elems(N);
    const int sb = (int)std::min<i64>(1024, (split_factor_elems(N) + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_split_factor, dim3(sb), dim3(kBlock), 0, s, (const float *)D, ginfo, N,
                       Dh, Dl);
    if ((ng & 3) == 0)
      hipLaunchKernelGGL(k_apply_big<true>, dim3((unsigned)grid), dim3(kAT), 0, s, Dh, Dl, ginfo,
                         (const float *)X, (float *)out, N, ng, occ, rhop);
    else
      hipLaunchKernelGGL(k_apply_big<false>, dim3((unsigned)grid), dim3(kAT), 0, s, Dh, Dl, ginfo,
                         (const float *)X, (float *)out, N, ng, occ, rhop);
    rho_sum();
    return hipGetLastError();
  }
  {
    const int nJ = (N + kBB - 1) / kBB;
    const i64 npt = (ng + kBB - 1) / kBB;
    const i64 grid = ((npt + 7) / 8) * 8 * nJ;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_apply_big64, dim3((unsigned)grid), dim3(kAB), 0, s, (const double *)D,
                       (const double *)X, (double *)out, N, ng, occ, rhop);
    rho_sum();
    return hipGetLastError();
  }
}

template hipError_t launch_trial_gram<double>(const double *, const double *, const double *,
                                              const double *, double, double *, int, i64, int,
                                              bool, double *, hipStream_t);
template hipError_t launch_trial_gram<float>(const float *, const float *, const double *,
                                             const double *, double, float *, int, i64, int, bool,
                                             double *, hipStream_t);
template hipError_t launch_gram_partial<double>(const double *, int, i64, int, double *,
                                                hipStream_t);
template hipError_t launch_gram_partial<float>(const float *, int, i64, int, double *,
                                               hipStream_t);
template hipError_t launch_apply_lower<double>(const double *, const double *, const double *,
                                               double *, int, i64, const double *, double *,
                                               hipStream_t, const double *, void *, double *);
template hipError_t launch_apply_lower<float>(const double *, const float *, const float *,
                                              float *, int, i64, const double *, double *,
                                              hipStream_t, const double *, void *, double *);


int cross_gram_split(int N) {
  // k_cross_big64: about two rounds of resident workgroups, a multiple of 8
  // ranges, at most 128 MiB of partials
  const int nb = (N + kBB - 1) / kBB;
  const i64 npairs = (i64)nb * nb;
  const int res = resident_workgroups((const void *)k_cross_big64<double, true>, kAB);
  i64 sp = (2 * (i64)res + npairs - 1) / npairs;
  const i64 cap = ((i64)128 << 20) / (npairs * kBB * kBB * 8);
  sp = std::min<i64>(sp, std::min<i64>(cap, 1024));
  sp = std::max<i64>(8, sp / 8 * 8);
  return (int)sp;
}

size_t cross_partial_doubles(int N) {
  const int nb = (N + kBB - 1) / kBB;
  return (size_t)cross_gram_split(N) * nb * nb * kBB * kBB;
}

template <typename T>
hipError_t launch_cross_gram(const T *A, const T *B, int N, i64 ng, double dv, double *part,
                             double *S, hipStream_t s) {
  const int nsplit = cross_gram_split(N);
  const int nb = (N + kBB - 1) / kBB;
  const int npairs = nb * nb;
  i64 kper = (ng + nsplit - 1) / nsplit;
  kper = ((kper + 15) / 16) * 16;
  const int grid = ((nsplit + 7) / 8) * 8 * npairs;
  const bool vec = (ng & 1) == 0 && ng >= 16 && (i64)kBB * ng * (i64)sizeof(T) < (1LL << 32);
  if (vec)
    hipLaunchKernelGGL((k_cross_big64<T, true>), dim3(grid), dim3(kAB), 0, s, A, B, N, ng, kper,
                       nsplit, npairs, part);
  else
    hipLaunchKernelGGL((k_cross_big64<T, false>), dim3(grid), dim3(kAB), 0, s, A, B, N, ng, kper,
                       nsplit, npairs, part);
  int blocks = (int)std::min<i64>(1024, ((i64)N * N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_cross_reduce_big, dim3(blocks), dim3(kBlock), 0, s, part, N, nsplit, npairs,
                     dv, S);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rotate(const double *P, const T *X, T *out, int N, i64 ng, hipStream_t s) {
  const int nJ = (N + kBB - 1) / kBB;
  const i64 npt = (ng + kBB - 1) / kBB;
  const i64 grid = ((npt + 7) / 8) * 8 * nJ;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mult_full64<T>, dim3((unsigned)grid), dim3(kAB), 0, s, P, X, out, N, ng);
  return hipGetLastError();
}

template hipError_t launch_cross_gram<double>(const double *, const double *, int, i64, double,
                                              double *, double *, hipStream_t);
template hipError_t launch_cross_gram<float>(const float *, const float *, int, i64, double,
                                             double *, double *, hipStream_t);
template hipError_t launch_rotate<double>(const double *, const double *, double *, int, i64,
                                          hipStream_t);
template hipError_t launch_rotate<float>(const double *, const float *, float *, int, i64,
                                         hipStream_t);

}  // namespace pou
