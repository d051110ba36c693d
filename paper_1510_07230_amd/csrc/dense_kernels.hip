// Dense kernels of the orthonormalisation (section 3.2: QR through a Cholesky
// factorisation of the Gram matrix <W^T W>): the Gram contraction over the
// grid on MFMA, its reduction to the symmetric N x N matrix, the FP64
// Cholesky factorisation with the triangular inverse, and the triangular
// apply W <- L^-1 W on MFMA.
#include "pou_internal.h"

namespace pou {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kGB = 64;   // Gram output block (rows and columns)
constexpr int kKC = 32;   // grid points staged per chunk
constexpr int kPitch = kKC + 1;

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

// Partial Gram over a contiguous range of grid points for one 64x64 output
// block (bi <= bj).  MFMA 16x16x4: lane l supplies A[l%16][k = l/16] and
// B[k = l/16][l%16]; output register r of lane l is row out_row(l/16, r),
// column l%16.  FP32 accumulators are flushed into FP64 after every chunk.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gram(const T *__restrict__ A, int N, i64 ng,
                                                 i64 kper, double *__restrict__ part) {
  __shared__ T sA[kGB][kPitch];
  __shared__ T sB[kGB][kPitch];
  typedef typename AccOf<T>::type Acc;
  const int split = blockIdx.x;
  const int pair = blockIdx.y;
  const int npairs = gridDim.y;
  const int nb = (N + kGB - 1) / kGB;
  int bi, bj;
  decode_pair(pair, nb, bi, bj);
  const i64 k_beg = (i64)split * kper;
  const i64 k_end = min(ng, k_beg + kper);
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63, r16 = l & 15, q = l >> 4;
  Acc acc[4];
  double accd[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    acc[c] = Acc{0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r) accd[c][r] = 0.0;
  }
  const bool diag = (bi == bj);
  for (i64 k0 = k_beg; k0 < k_end; k0 += kKC) {
    const int col = t & 31;
    const i64 g = k0 + col;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int row = (t >> 5) + 8 * e;
      const int ra = bi * kGB + row;
      sA[row][col] = (ra < N && g < k_end) ? A[(i64)ra * ng + g] : (T)0;
      if (!diag) {
        const int rb = bj * kGB + row;
        sB[row][col] = (rb < N && g < k_end) ? A[(i64)rb * ng + g] : (T)0;
      }
    }
    __syncthreads();
    const T(*sb)[kPitch] = diag ? sA : sB;
#pragma unroll
    for (int ks = 0; ks < kKC / 4; ++ks) {
      const T a = sA[16 * w + r16][4 * ks + q];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T b = sb[16 * c + r16][4 * ks + q];
        acc[c] = mfma(a, b, acc[c]);
      }
    }
    __syncthreads();
    if (sizeof(T) == 4) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int r = 0; r < 4; ++r) accd[c][r] += (double)acc[c][r];
        acc[c] = Acc{0, 0, 0, 0};
      }
    }
  }
  double *out = part + ((i64)split * npairs + pair) * kGB * kGB;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * w + out_row<T>(q, r);
      const int colo = 16 * c + r16;
      out[row * kGB + colo] = (sizeof(T) == 4) ? accd[c][r] : (double)acc[c][r];
    }
  }
}

// Same contraction with the FP32 values rounded to BF16 and MFMA 16x16x32
// (lane l supplies A[l%16][8(l/16) .. 8(l/16)+7]); FP32 accumulation per
// 32-point chunk, flushed into FP64.
constexpr int kPitchB = kKC + 4;
__global__ __launch_bounds__(kBlock) void k_gram_bf16(const float *__restrict__ A, int N,
                                                      i64 ng, i64 kper,
                                                      double *__restrict__ part) {
  __shared__ float sA[kGB][kPitchB];
  __shared__ float sB[kGB][kPitchB];
  const int split = blockIdx.x;
  const int pair = blockIdx.y;
  const int npairs = gridDim.y;
  const int nb = (N + kGB - 1) / kGB;
  int bi, bj;
  decode_pair(pair, nb, bi, bj);
  const i64 k_beg = (i64)split * kper;
  const i64 k_end = min(ng, k_beg + kper);
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63, r16 = l & 15, q = l >> 4;
  double accd[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) accd[c][r] = 0.0;
  const bool diag = (bi == bj);
  for (i64 k0 = k_beg; k0 < k_end; k0 += kKC) {
    const int col = t & 31;
    const i64 g = k0 + col;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int row = (t >> 5) + 8 * e;
      const int ra = bi * kGB + row;
      sA[row][col] = (ra < N && g < k_end) ? A[(i64)ra * ng + g] : 0.0f;
      if (!diag) {
        const int rb = bj * kGB + row;
        sB[row][col] = (rb < N && g < k_end) ? A[(i64)rb * ng + g] : 0.0f;
      }
    }
    __syncthreads();
    const float(*sb)[kPitchB] = diag ? sA : sB;
    bf8 a;
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = (__bf16)sA[16 * w + r16][8 * q + e];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      bf8 b;
#pragma unroll
      for (int e = 0; e < 8; ++e) b[e] = (__bf16)sb[16 * c + r16][8 * q + e];
      f4 acc = f4{0, 0, 0, 0};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) accd[c][r] += (double)acc[r];
    }
    __syncthreads();
  }
  double *out = part + ((i64)split * npairs + pair) * kGB * kGB;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      out[(16 * w + 4 * q + r) * kGB + 16 * c + r16] = accd[c][r];
}

// G[i][j] = dv * sum over splits of the block partials; both triangles.
__global__ __launch_bounds__(kBlock) void k_gram_reduce(const double *__restrict__ part, int N,
                                                        int nsplit, int npairs, double dv,
                                                        double *__restrict__ G) {
  const int nb = (N + kGB - 1) / kGB;
  const i64 total = (i64)N * N;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (i64)gridDim.x * blockDim.x) {
    int i = (int)(e / N), j = (int)(e % N);
    if (i > j) continue;  // fill both from the upper triangle
    const int bi = i / kGB, bj = j / kGB;
    // pair index for (bi, bj), bi <= bj
    const int pair = bi * nb - (bi * (bi - 1)) / 2 + (bj - bi);
    const int ri = i - bi * kGB, cj = j - bj * kGB;
    double s = 0.0;
    for (int sp = 0; sp < nsplit; ++sp)
      s += part[(((i64)sp * npairs + pair) * kGB + ri) * kGB + cj];
    s *= dv;
    G[(i64)i * N + j] = s;
    G[(i64)j * N + i] = s;
  }
}

// Cholesky G = L L^T (lower, in place in G) and Minv = L^-1.  One workgroup.
// info[0] = 1 when a pivot is not finite or not above 1e-13 times its original
// diagonal entry (G not numerically SPD);
// info[1] = max |G - I| measured before factorising.
__global__ __launch_bounds__(1024) void k_cholesky_inverse(double *__restrict__ G,
                                                           double *__restrict__ Minv, int N,
                                                           double *__restrict__ info) {
  __shared__ double sred[16];
  __shared__ double sdiag[512];
  __shared__ double spiv;
  __shared__ int sbad;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int i = t; i < N; i += nt) sdiag[i] = G[(i64)i * N + i];
  double m = 0.0;
  for (int e = t; e < N * N; e += nt) {
    const int i = e / N, j = e % N;
    const double v = G[e] - (i == j ? 1.0 : 0.0);
    m = fmax(m, fabs(v));
    if (!isfinite(v)) m = INFINITY;
  }
  m = wave_max(m);
  if ((t & 63) == 0) sred[t >> 6] = m;
  if (t == 0) sbad = 0;
  __syncthreads();
  if (t == 0) {
    double mm = 0.0;
    for (int w = 0; w < (nt >> 6); ++w) mm = fmax(mm, sred[w]);
    info[1] = mm;
  }
  for (int k = 0; k < N; ++k) {
    if (t == 0) {
      double d = G[(i64)k * N + k];
      // a pivot at rounding level of the original diagonal means the
      // columns are numerically dependent
      if (!(d > 1e-13 * sdiag[k]) || !isfinite(d)) {
        sbad = 1;
        d = 1.0;
      }
      spiv = sqrt(d);
      G[(i64)k * N + k] = spiv;
    }
    __syncthreads();
    const double piv = spiv;
    for (int i = k + 1 + t; i < N; i += nt) G[(i64)i * N + k] /= piv;
    __syncthreads();
    const int mm = N - k - 1;
    for (int e = t; e < mm * mm; e += nt) {
      const int i = k + 1 + e / mm, j = k + 1 + e % mm;
      if (j <= i) G[(i64)i * N + j] -= G[(i64)i * N + k] * G[(i64)j * N + k];
    }
    __syncthreads();
  }
  // triangular inverse, one column per thread
  for (int c = t; c < N; c += nt) {
    for (int i = 0; i < c; ++i) Minv[(i64)i * N + c] = 0.0;
    Minv[(i64)c * N + c] = 1.0 / G[(i64)c * N + c];
    for (int i = c + 1; i < N; ++i) {
      double s = 0.0;
      for (int k = c; k < i; ++k) s += G[(i64)i * N + k] * Minv[(i64)k * N + c];
      Minv[(i64)i * N + c] = -s / G[(i64)i * N + i];
    }
  }
  __syncthreads();
  if (t == 0) info[0] = sbad ? 1.0 : 0.0;
}

// C = A B for lower-triangular A, B (upper parts zero).
__global__ __launch_bounds__(kBlock) void k_lower_matmul(const double *__restrict__ A,
                                                         const double *__restrict__ B,
                                                         double *__restrict__ C, int N) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N * N; e += gridDim.x * blockDim.x) {
    const int i = e / N, j = e % N;
    double s = 0.0;
    for (int k = j; k <= i; ++k) s += A[(i64)i * N + k] * B[(i64)k * N + j];
    C[e] = (j <= i) ? s : 0.0;
  }
}

// out[j][g] = X[j][g] + sum_i (M - I)[j][i] X[i][g] for lower-triangular M.
// Written as identity plus correction so that the rounding of the result is
// relative to the (small) correction.  Workgroup: 64 grid points x a group of
// up to 8 row tiles of 16 orbitals; wave w takes row tiles w and w+4 of the
// group.  X fragments are read straight from global memory in the MFMA
// layout (16 consecutive grid points per k row).  Optional fused density
// rho[g] = sum_j occ_j out[j][g]^2 when the group covers all orbitals.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_apply_lower(const double *__restrict__ M,
                                                        const T *__restrict__ X,
                                                        T *__restrict__ out, int N, i64 ng,
                                                        const double *__restrict__ occ,
                                                        double *__restrict__ rho) {
  __shared__ double srho[4][64];
  typedef typename AccOf<T>::type Acc;
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63, r16 = l & 15, q = l >> 4;
  const i64 g0 = (i64)blockIdx.x * 64;
  const int NT = (N + 15) / 16;
  const int jt[2] = {(int)blockIdx.y * 8 + w, (int)blockIdx.y * 8 + w + 4};
  const bool jv[2] = {jt[0] < NT, jt[1] < NT};
  Acc acc[2][4];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[u][c] = Acc{0, 0, 0, 0};
  const int ks_end0 = jv[0] ? min(4 * (jt[0] + 1), (N + 3) / 4) : 0;
  const int ks_end1 = jv[1] ? min(4 * (jt[1] + 1), (N + 3) / 4) : 0;
  const int ks_end = max(ks_end0, ks_end1);
  for (int ks = 0; ks < ks_end; ++ks) {
    const int i = 4 * ks + q;
    T b[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const i64 g = g0 + 16 * c + r16;
      b[c] = (i < N && g < ng) ? X[(i64)i * ng + g] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (ks < (u == 0 ? ks_end0 : ks_end1)) {
        const int j = 16 * jt[u] + r16;
        const T a = (j < N && i < N) ? (T)(M[(i64)j * N + i] - (i == j ? 1.0 : 0.0)) : (T)0;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[u][c] = mfma(a, b[c], acc[u][c]);
      }
    }
  }
  double rp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    if (!jv[u]) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const i64 g = g0 + 16 * c + r16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = 16 * jt[u] + out_row<T>(q, r);
        if (j < N && g < ng) {
          const T v = X[(i64)j * ng + g] + acc[u][c][r];
          out[(i64)j * ng + g] = v;
          rp[c] += occ ? occ[j] * (double)v * (double)v : 0.0;
        }
      }
    }
  }
  if (rho != nullptr) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double v = rp[c];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (q == 0) srho[w][16 * c + r16] = v;
    }
    __syncthreads();
    if (t < 64) {
      const i64 g = g0 + t;
      if (g < ng) rho[g] = srho[0][t] + srho[1][t] + srho[2][t] + srho[3][t];
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_gram_partial(const T *A, int N, i64 ng, int nsplit, double *part,
                               hipStream_t s) {
  const int nb = (N + kGB - 1) / kGB;
  const int npairs = nb * (nb + 1) / 2;
  i64 kper = (ng + nsplit - 1) / nsplit;
  kper = ((kper + kKC - 1) / kKC) * kKC;
  hipLaunchKernelGGL(k_gram<T>, dim3(nsplit, npairs), dim3(kBlock), 0, s, A, N, ng, kper, part);
  return hipGetLastError();
}

hipError_t launch_gram_partial_bf16(const float *A, int N, i64 ng, int nsplit, double *part,
                                    hipStream_t s) {
  const int nb = (N + kGB - 1) / kGB;
  const int npairs = nb * (nb + 1) / 2;
  i64 kper = (ng + nsplit - 1) / nsplit;
  kper = ((kper + kKC - 1) / kKC) * kKC;
  hipLaunchKernelGGL(k_gram_bf16, dim3(nsplit, npairs), dim3(kBlock), 0, s, A, N, ng, kper,
                     part);
  return hipGetLastError();
}

hipError_t launch_gram_reduce(const double *part, int N, int nsplit, double dv, double *G,
                              hipStream_t s) {
  const int nb = (N + kGB - 1) / kGB;
  const int npairs = nb * (nb + 1) / 2;
  const i64 total = (i64)N * N;
  int blocks = (int)((total + kBlock - 1) / kBlock);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_gram_reduce, dim3(blocks), dim3(kBlock), 0, s, part, N, nsplit, npairs,
                     dv, G);
  return hipGetLastError();
}

hipError_t launch_cholesky_inverse(double *G, double *Minv, int N, double *info,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_cholesky_inverse, dim3(1), dim3(1024), 0, s, G, Minv, N, info);
  return hipGetLastError();
}

hipError_t launch_lower_matmul(const double *A, const double *B, double *C, int N,
                               hipStream_t s) {
  int blocks = (N * N + kBlock - 1) / kBlock;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_lower_matmul, dim3(blocks), dim3(kBlock), 0, s, A, B, C, N);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_lower(const double *M, const T *X, T *out, int N, i64 ng,
                              const double *occ, double *rho, hipStream_t s) {
  const int NT = (N + 15) / 16;
  const int groups = (NT + 7) / 8;
  if (rho != nullptr && groups != 1) return hipErrorInvalidValue;
  dim3 grid((unsigned)((ng + 63) / 64), groups);
  hipLaunchKernelGGL(k_apply_lower<T>, grid, dim3(kBlock), 0, s, M, X, out, N, ng, occ, rho);
  return hipGetLastError();
}

template hipError_t launch_gram_partial<double>(const double *, int, i64, int, double *,
                                                hipStream_t);
template hipError_t launch_gram_partial<float>(const float *, int, i64, int, double *,
                                               hipStream_t);
template hipError_t launch_apply_lower<double>(const double *, const double *, double *, int,
                                               i64, const double *, double *, hipStream_t);
template hipError_t launch_apply_lower<float>(const double *, const float *, float *, int, i64,
                                              const double *, double *, hipStream_t);

}  // namespace pou
