// Grid kernels: the Hamiltonian stencil sweep over all orbitals, the density,
// exchange and effective potential, the Poisson CG building blocks with the
// FFT-based spectral inverse, the ionic charge and forces, and the per-orbital
// elementwise steps of Algorithm M (trial point, accept/BB dot products).
#include "pou_internal.h"

#include <cmath>
#include <cstdint>

namespace pou {

namespace {

constexpr int kNB = 4;  // y points per thread in the stencil tile (kTY / 8 rows)

__host__ __device__ inline int wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Periodic index for -n <= i < 2n (a stencil offset from a point of the grid):
// one compare and add instead of an integer division.
__host__ __device__ inline int wrap_near(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Plane access through a buffer descriptor: a uniform plane base in scalar
// registers, a 32-bit unsigned byte offset per lane, and the plane size as
// the record count (an access beyond the plane reads zero and writes nothing).
typedef unsigned pou_v2u __attribute__((ext_vector_type(2)));

__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                           0x00020000);
}

template <typename T>
__device__ inline T plane_load(__amdgpu_buffer_rsrc_t r, unsigned boff);
template <>
__device__ inline float plane_load<float>(__amdgpu_buffer_rsrc_t r, unsigned boff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, boff, 0, 0));
}
template <>
__device__ inline double plane_load<double>(__amdgpu_buffer_rsrc_t r, unsigned boff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
}

// Stores of H U are used once by a later kernel: cache policy 2 marks them
// non-temporal (the NT bit of gfx940-class buffer stores)
constexpr int kStoreNT = 2;
__device__ inline void plane_store(__amdgpu_buffer_rsrc_t r, unsigned boff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, boff, 0, kStoreNT);
}
__device__ inline void plane_store(__amdgpu_buffer_rsrc_t r, unsigned boff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(pou_v2u, v), r, boff, 0, kStoreNT);
}

// ----------------------------------------------------------------- stencil

// H u = -1/2 Lap_h u + V_eff u on the periodic grid (section 2.1 H(rho), with
// the 8th-order finite-difference Laplacian).  Each workgroup owns a 32x32 x-y
// tile of one orbital and marches over a chunk of z planes: the current plane
// with its radius-4 x/y halo is staged in LDS and the z neighbours live in a
// per-thread register queue (2.5-D blocking).  A thread computes 4 consecutive
// y rows of one x column, so the y neighbours of its points overlap.  The
// second differences are formed as sums of (u_{+m} - u_0) + (u_{-m} - u_0),
// exact in real arithmetic because the weights sum to zero, which keeps FP32
// cancellation small.
//
// Workgroup order: the 1-D grid is walked XCD by XCD (workgroup id mod 8
// selects the XCD) so that all tiles of one (orbital, z chunk) run on the
// same XCD one after another and their halos hit that XCD's L2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_hamiltonian(const T *__restrict__ U,
                                                        const T *__restrict__ veff,
                                                        T *__restrict__ HU,
                                                        double *__restrict__ part,
                                                        StencilArgs a, int N) {
  // the plane with its halo, double-buffered: plane z uses buffer z mod 2, so
  // one barrier per plane separates the stores from the reads
  __shared__ T s2[2][kTY + 2 * kRad][kTX + 2 * kRad + 1];
  __shared__ double red[4 * 2];
  const int n = a.n;
  const i64 ng = (i64)n * n * n;
  const int tiles_x = (n + kTX - 1) / kTX;
  // XCD-aware decode: L = 8 j + x -> group g = x + 8 (j / ntile), tile = j % ntile
  const int L = blockIdx.x;
  const int xcd = L & 7, j = L >> 3;
  const int grp = xcd + 8 * (j / a.ntile);
  const int tile = j % a.ntile;
  if (grp >= N * a.nzc) return;  // padding workgroups (before any barrier)
  const int orb = grp / a.nzc;
  const int zc = grp % a.nzc;
  const int x0 = (tile % tiles_x) * kTX;
  const int y0 = (tile / tiles_x) * kTY;
  const int tx = threadIdx.x & 31;
  const int trow = threadIdx.x >> 5;  // 0..7, owns rows 4*trow .. 4*trow+3
  const T *u = U + (i64)orb * ng;
  T *hu = HU + (i64)orb * ng;

  const int gx = x0 + tx;
  const bool vx = gx < n;
  const int gxw = wrap(gx, n);
  // in-plane byte offsets (32-bit: n <= 1024) of this thread's rows and halo
  // cells; every plane access is a buffer access at one of these offsets
  const int nn = n * n;
  const unsigned pbytes = (unsigned)(n * n) * (unsigned)sizeof(T);
  unsigned offr[kNB], offw[kNB];
  T vmask[kNB];
#pragma unroll
  for (int r = 0; r < kNB; ++r) {
    const int gy = y0 + 4 * trow + r;
    const bool valid = vx && gy < n;
    offr[r] = (unsigned)(wrap(gy, n) * n + gxw) * (unsigned)sizeof(T);
    offw[r] = valid ? offr[r] : 0x80000000u;  // beyond the plane: not written
    vmask[r] = valid ? (T)1 : (T)0;
  }
  // halo assignments (independent of z)
  const int hx_row = threadIdx.x >> 3;  // 0..31
  const int hx_c = threadIdx.x & 7;     // 0..7
  const int hx_lc = hx_c < 4 ? hx_c - 4 : kTX + hx_c - 4;
  const unsigned off_hx =
      (unsigned)(wrap(y0 + hx_row, n) * n + wrap(x0 + hx_lc, n)) * (unsigned)sizeof(T);
  const int hy_col = threadIdx.x & 31;
  const int hy_r = threadIdx.x >> 5;  // 0..7
  const int hy_lr = hy_r < 4 ? hy_r - 4 : kTY + hy_r - 4;
  const unsigned off_hy =
      (unsigned)(wrap(y0 + hy_lr, n) * n + wrap(x0 + hy_col, n)) * (unsigned)sizeof(T);
  auto at = [&](const T *base, unsigned boff) -> T {
    return plane_load<T>(plane_rsrc(base, pbytes), boff);
  };

  const int z0 = zc * a.zlen;
  const int z1 = min(n, z0 + a.zlen);

  // z neighbours: a circular register queue of kQ planes, plane p in slot
  // (p - z0 + kRad) mod kQ.  The queue holds the nine planes of the stencil
  // plus the kPD planes whose loads are in flight, so a load goes straight
  // into the slot it is read from; the z loop is unrolled by kQ so every slot
  // index is a compile-time constant.
  constexpr int kPD = 3;
  constexpr int kQ = 2 * kRad + 1 + kPD;
  T q[kNB][kQ];
#pragma unroll
  for (int m = 0; m < 2 * kRad; ++m) {
    const T *pz = u + (i64)wrap(z0 - kRad + m, n) * nn;
#pragma unroll
    for (int r = 0; r < kNB; ++r) q[r][m] = at(pz, offr[r]);
  }
  const T c1 = (T)FD8::c1, c2 = (T)FD8::c2, c3 = (T)FD8::c3, c4 = (T)FD8::c4;
  const T cm[5] = {(T)0, c1, c2, c3, c4};
  const T mh = (T)(-0.5 * a.inv_h2);
  double acc_sig = 0.0, acc_kin = 0.0;

  // Loads for plane zz are issued kPD planes ahead of their use: the halo of
  // plane zz and V_eff on plane zz into a ring of kR = kPD + 1 register sets
  // (plane zz in set (zz - z0) mod kR, so a load never lands in the set being
  // read), the queue head zz + kRad into its queue slot.
  constexpr int kR = kPD + 1;
  static_assert(kQ % kR == 0, "prefetch ring must divide the z unroll");
  static_assert(kQ % 2 == 0, "the plane buffers alternate within the z unroll");
  T nhx[kR], nhy[kR], nvf[kR][kNB];
  auto issue = [&](int slot, int qs, int zz) {
    const T *pz = u + (i64)zz * nn;
    const T *pq = u + (i64)wrap_near(zz + kRad, n) * nn;
    const T *pv = veff + (i64)zz * nn;
    const T hx = at(pz, off_hx);
    const T hy = at(pz, off_hy);
    T qq[kNB], vv[kNB];
#pragma unroll
    for (int r = 0; r < kNB; ++r) qq[r] = at(pq, offr[r]);
#pragma unroll
    for (int r = 0; r < kNB; ++r) vv[r] = at(pv, offr[r]);
#pragma unroll
    for (int k = 0; k < kR; ++k) {
      if (k == slot) {
        nhx[k] = hx;
        nhy[k] = hy;
#pragma unroll
        for (int r = 0; r < kNB; ++r) nvf[k][r] = vv[r];
      }
    }
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      if (k == qs) {
#pragma unroll
        for (int r = 0; r < kNB; ++r) q[r][k] = qq[r];
      }
    }
  };
#pragma unroll
  for (int k = 0; k < kPD; ++k)
    if (z0 + k < z1) issue(k, (k + 2 * kRad) % kQ, z0 + k);

  for (int zb = z0; zb < z1; zb += kQ) {
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      const int z = zb + k;
      if (z < z1) {
        const __amdgpu_buffer_rsrc_t hz = plane_rsrc(hu + (i64)z * nn, pbytes);
        const int ps = k % kR;
        const int qc = (k + kRad) % kQ;  // slot of plane z
        // buffer k mod 2 was last read for plane z - 2, and every wave passed
        // plane z - 1's barrier after those reads
        T(*s)[kTX + 2 * kRad + 1] = s2[k & 1];
#pragma unroll
        for (int r = 0; r < kNB; ++r) s[4 * trow + r + kRad][tx + kRad] = q[r][qc];
        s[hx_row + kRad][hx_lc + kRad] = nhx[ps];
        s[hy_lr + kRad][hy_col + kRad] = nhy[ps];
        const T *vf = nvf[ps];
        // plane z + kPD: its queue head z + kPD + kRad goes to the slot of
        // plane z - kRad - 1, which no later plane reads
        if (z + kPD < z1) issue((k + kPD) % kR, (k + kRad + kPD + kRad) % kQ, z + kPD);
        __syncthreads();
        // y column of this thread: rows 4 trow - 4 .. 4 trow + 7 (local + kRad offset)
        T col[kNB + 2 * kRad];
#pragma unroll
        for (int kk = 0; kk < kNB + 2 * kRad; ++kk) col[kk] = s[4 * trow + kk][tx + kRad];
        // sigma and kinetic partials of this plane's four points in T, then
        // FP64; every point is computed (its loads are in bounds by the
        // periodic wrap) and a point outside the grid is stored at an offset
        // beyond the plane, which the buffer range check drops, so no branch
        // splits the work of the four points
        T psig = (T)0, pkin = (T)0;
#pragma unroll
        for (int r = 0; r < kNB; ++r) {
          const int ly = 4 * trow + r + kRad;
          const int lx = tx + kRad;
          const T c0 = col[r + kRad];
          T lap = (T)0;
#pragma unroll
          for (int m = 1; m <= kRad; ++m) {
            const T dxm = (s[ly][lx + m] - c0) + (s[ly][lx - m] - c0);
            const T dym = (col[r + kRad + m] - c0) + (col[r + kRad - m] - c0);
            const T dzm = (q[r][(qc + m) % kQ] - c0) + (q[r][(qc - m + kQ) % kQ] - c0);
            lap += cm[m] * ((dxm + dym) + dzm);
          }
          const T ku = mh * lap;
          const T h = ku + vf[r] * c0;
          plane_store(hz, offw[r], h);
          const T cv = c0 * vmask[r];
          psig += cv * h;
          pkin += cv * ku;
        }
        acc_sig += (double)psig;
        acc_kin += (double)pkin;
      }
    }
  }
  double v[2] = {acc_sig, acc_kin};
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    const int nb = a.ntile * a.nzc;
    const i64 idx = (i64)orb * nb + (i64)tile * a.nzc + zc;
    part[2 * idx + 0] = v[0];
    part[2 * idx + 1] = v[1];
  }
}

// ----------------------------------------------------------------- density

template <typename T>
__global__ __launch_bounds__(kBlock) void k_density(const T *__restrict__ U,
                                                    const double *__restrict__ occ,
                                                    double *__restrict__ rho, int N, i64 ng) {
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x) {
    double acc = 0.0;
    int i = 0;
    for (; i + 4 <= N; i += 4) {
      const double u0 = (double)U[(i64)i * ng + g];
      const double u1 = (double)U[(i64)(i + 1) * ng + g];
      const double u2 = (double)U[(i64)(i + 2) * ng + g];
      const double u3 = (double)U[(i64)(i + 3) * ng + g];
      acc += occ[i] * u0 * u0 + occ[i + 1] * u1 * u1 + occ[i + 2] * u2 * u2 +
             occ[i + 3] * u3 * u3;
    }
    for (; i < N; ++i) {
      const double u0 = (double)U[(i64)i * ng + g];
      acc += occ[i] * u0 * u0;
    }
    rho[g] = acc;
  }
}

// ------------------------------------------------------- exchange and V_eff

// LDA exchange (section 2.1 v_xc, exchange part only):
//   e_x density = -C_x rho^(4/3), v_x = -(3/pi)^(1/3) rho^(1/3).
// LDA correlation per electron of the uniform gas, Perdew-Zunger fit
// (spin-unpolarised), and its potential d(rho eps_c)/d rho, for rho > 0 with
// r13 = rho^(1/3): r_s = (3 / (4 pi))^(1/3) / r13;
//   r_s >= 1: eps = G / (1 + B1 sqrt(r_s) + B2 r_s),
//             v = eps (1 + 7/6 B1 sqrt(r_s) + 4/3 B2 r_s) / (1 + B1 sqrt(r_s) + B2 r_s)
//   r_s <  1: eps = A ln r_s + B + C r_s ln r_s + D r_s,
//             v = A ln r_s + (B - A/3) + 2/3 C r_s ln r_s + (2 D - C)/3 r_s
__device__ inline void pz_correlation(double rho, double r13, double &eps, double &v) {
  const double rs = 0.62035049089940001667 / r13;  // (3/(4 pi))^(1/3) rho^(-1/3)
  if (rs >= 1.0) {
    const double G = -0.1423, B1 = 1.0529, B2 = 0.3334;
    const double sq = sqrt(rs);
    const double den = 1.0 + B1 * sq + B2 * rs;
    eps = G / den;
    v = eps * (1.0 + (7.0 / 6.0) * B1 * sq + (4.0 / 3.0) * B2 * rs) / den;
  } else {
    const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
    const double lr = log(rs);
    eps = A * lr + B + C * rs * lr + D * rs;
    v = A * lr + (B - A / 3.0) + (2.0 / 3.0) * C * rs * lr + ((2.0 * D - C) / 3.0) * rs;
  }
  (void)rho;
}

__global__ __launch_bounds__(kBlock) void k_xc_veff(const double *__restrict__ rho,
                                                    const double *__restrict__ vh,
                                                    const double *__restrict__ vext,
                                                    double *__restrict__ veff,
                                                    float *__restrict__ veff32,
                                                    double *__restrict__ part, i64 ng,
                                                    unsigned terms) {
  __shared__ double red[4 * 4];
  const double kv = 0.98474502184269640;  // (3/pi)^(1/3)
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x) {
    const double r = rho[g];
    const double r13 = cbrt(fmax(r, 0.0));
    double v = 0.0;
    if (terms & 8u) {
      v -= kv * r13;
      a0 += r * r13;
    }
    if ((terms & 16u) && r > 0.0) {
      double eps, vc;
      pz_correlation(r, r13, eps, vc);
      v += vc;
      a3 += r * eps;
    }
    if (terms & 4u) {
      v += vh[g];
      a2 += r * vh[g];
    }
    if (terms & 2u) {
      v += vext[g];
      a1 += r * vext[g];
    }
    veff[g] = v;
    if (veff32) veff32[g] = (float)v;
  }
  double vals[4] = {a0, a1, a2, a3};
  block_sum<4>(vals, red);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x + 0] = vals[0];
    part[4 * blockIdx.x + 1] = vals[1];
    part[4 * blockIdx.x + 2] = vals[2];
    part[4 * blockIdx.x + 3] = vals[3];
  }
}

// out[k*nseg + seg] = sum_j part[(seg*len + j)*K + k]
__global__ __launch_bounds__(kBlock) void k_segment_sum(const double *__restrict__ part,
                                                        double *__restrict__ out, int nseg,
                                                        int len, int K, double scale) {
  __shared__ double red[4];
  const int seg = blockIdx.x;
  for (int k = 0; k < K; ++k) {
    double acc = 0.0;
    for (int j = threadIdx.x; j < len; j += blockDim.x)
      acc += part[((i64)seg * len + j) * K + k];
    double v[1] = {acc};
    block_sum<1>(v, red);
    if (threadIdx.x == 0) out[(i64)k * nseg + seg] = scale * v[0];
  }
}

// ----------------------------------------------------------------- Poisson

// -Lap p at point g = (z*n + y)*n + x of a periodic FP64 field; c0 = p[g].
// Indices are 32-bit (n <= 1024 keeps n^3 below 2^31).
__device__ inline double neg_lap_at(const double *__restrict__ p, unsigned g, int n,
                                    double inv_n, double inv_h2, double &c0) {
  const unsigned un = (unsigned)n;
  // g = (z n + y) n + x by floating-point quotients (exact after the +-1
  // correction for g < 2^31), not integer divisions
  unsigned yz = (unsigned)((double)g * inv_n);
  int x = (int)(g - yz * un);
  if (x < 0) { --yz; x += n; } else if (x >= n) { ++yz; x -= n; }
  unsigned zq = (unsigned)((double)yz * inv_n);
  int y = (int)(yz - zq * un);
  if (y < 0) { --zq; y += n; } else if (y >= n) { ++zq; y -= n; }
  const int z = (int)zq;
  const unsigned row = g - (unsigned)x;            // (z*n + y)*n
  const unsigned plane = (unsigned)z * un * un;    // z*n*n
  const unsigned nn = un * un;
  const double c[5] = {0.0, FD8::c1, FD8::c2, FD8::c3, FD8::c4};
  c0 = p[g];
  double lap = 0.0;
#pragma unroll
  for (int m = 1; m <= kRad; ++m) {
    const double dx = (p[row + wrap_near(x + m, n)] - c0) + (p[row + wrap_near(x - m, n)] - c0);
    const double dy = (p[plane + (unsigned)wrap_near(y + m, n) * un + x] - c0) +
                      (p[plane + (unsigned)wrap_near(y - m, n) * un + x] - c0);
    const double dz = (p[(unsigned)wrap_near(z + m, n) * nn + (g - plane)] - c0) +
                      (p[(unsigned)wrap_near(z - m, n) * nn + (g - plane)] - c0);
    lap += c[m] * ((dx + dy) + dz);
  }
  return -lap * inv_h2;
}

__global__ __launch_bounds__(kBlock) void k_neg_lap(const double *__restrict__ p,
                                                    double *__restrict__ q,
                                                    double *__restrict__ part, int n,
                                                    double inv_h2) {
  __shared__ double red[4];
  const unsigned ng = (unsigned)n * n * n;
  const double inv_n = 1.0 / (double)n;
  double acc = 0.0;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += gridDim.x * blockDim.x) {
    double c0;
    const double v = neg_lap_at(p, g, n, inv_n, inv_h2, c0);
    q[g] = v;
    acc += c0 * v;
  }
  if (part) {
    double v[1] = {acc};
    block_sum<1>(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
  }
}

// Residual of the Hartree equation -Lap x = 4 pi (rho - mean rho) without
// storing it: partials of (r.r, b.b) per block into part[2*block + k].
__global__ __launch_bounds__(kBlock) void k_poisson_residual(const double *__restrict__ x,
                                                             const double *__restrict__ rho,
                                                             const double *__restrict__ dsum,
                                                             double *__restrict__ part, int n,
                                                             double inv_h2) {
  __shared__ double red[4 * 2];
  const unsigned ng = (unsigned)n * n * n;
  const double inv_n = 1.0 / (double)n;
  const double mean = dsum[0] / (double)ng;
  const double fourpi = 12.566370614359172954;
  double a0 = 0.0, a1 = 0.0;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += gridDim.x * blockDim.x) {
    double c0;
    const double b = fourpi * (rho[g] - mean);
    const double rr = b - neg_lap_at(x, g, n, inv_n, inv_h2, c0);
    a0 += rr * rr;
    a1 += b * b;
  }
  double v[2] = {a0, a1};
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = v[0];
    part[2 * blockIdx.x + 1] = v[1];
  }
}

__global__ __launch_bounds__(kBlock) void k_cg_rhs_residual(const double *__restrict__ rho,
                                                            const double *__restrict__ dsum,
                                                            const double *__restrict__ q,
                                                            double *__restrict__ r,
                                                            double *__restrict__ part, i64 ng) {
  __shared__ double red[4 * 2];
  const double mean = dsum[0] / (double)ng;
  const double fourpi = 12.566370614359172954;
  double a0 = 0.0, a1 = 0.0;
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x) {
    const double b = fourpi * (rho[g] - mean);
    const double rr = b - q[g];
    r[g] = rr;
    a0 += rr * rr;
    a1 += b * b;
  }
  double v[2] = {a0, a1};
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = v[0];
    part[2 * blockIdx.x + 1] = v[1];
  }
}

__global__ __launch_bounds__(kBlock) void k_dot2(const double *__restrict__ a,
                                                 const double *__restrict__ b,
                                                 double *__restrict__ part, i64 ng) {
  __shared__ double red[4];
  double acc = 0.0;
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x)
    acc += a[g] * (b ? b[g] : 1.0);
  double v[1] = {acc};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void k_cg_update_p(double *__restrict__ p,
                                                        const double *__restrict__ z,
                                                        const double *__restrict__ num,
                                                        const double *__restrict__ den,
                                                        int first, i64 ng) {
  double beta = first ? 0.0 : num[0] / den[0];
  if (!isfinite(beta)) beta = 0.0;  // exact zero residual
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x)
    p[g] = z[g] + beta * (first ? 0.0 : p[g]);
}

__global__ __launch_bounds__(kBlock) void k_cg_update_xr(double *__restrict__ x,
                                                         double *__restrict__ r,
                                                         const double *__restrict__ p,
                                                         const double *__restrict__ q,
                                                         const double *__restrict__ num,
                                                         const double *__restrict__ den,
                                                         double *__restrict__ part, i64 ng) {
  __shared__ double red[4];
  double alpha = num[0] / den[0];
  if (!isfinite(alpha)) alpha = 0.0;  // exact zero residual
  double acc = 0.0;
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x) {
    x[g] += alpha * p[g];
    const double rr = r[g] - alpha * q[g];
    r[g] = rr;
    acc += rr * rr;
  }
  double v[1] = {acc};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void k_scale(double *__restrict__ x, double a, i64 ng) {
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x)
    x[g] *= a;
}

__global__ __launch_bounds__(kBlock) void k_remove_mean(double *__restrict__ x,
                                                        const double *__restrict__ dsum,
                                                        i64 ng) {
  const double mean = dsum[0] / (double)ng;
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x)
    x[g] -= mean;
}

// ----------------------------------------------------------------- FFT
// Batched 1-D complex FFTs of length n held in LDS, mixed radix (4, 2, 3, 5,
// any leftover factor by direct DFT), self-sorting (Stockham) stages.  A
// workgroup transforms `lb` lines; lines along x are contiguous, lines along
// y and z are strided and the batch takes consecutive x so global accesses of
// one element index stay contiguous.

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// multiply by sign*i
__device__ inline double2 cmuli(double2 a, double sign) { return make_double2(-sign * a.y, sign * a.x); }

struct Radices {
  int nr;
  int r[16];
};

// Radix plan of a length-n transform (4s first, then 2, 3, 5, other primes);
// constexpr, so the transforms specialised on n take it at compile time.
constexpr Radices factorize(int n) {
  Radices f{};
  f.nr = 0;
  int m = n;
  while (m % 4 == 0) { f.r[f.nr++] = 4; m /= 4; }
  while (m % 2 == 0) { f.r[f.nr++] = 2; m /= 2; }
  while (m % 3 == 0) { f.r[f.nr++] = 3; m /= 3; }
  while (m % 5 == 0) { f.r[f.nr++] = 5; m /= 5; }
  for (int p = 7; p * p <= m; p += 2)
    while (m % p == 0) { f.r[f.nr++] = p; m /= p; }
  if (m > 1) f.r[f.nr++] = m;
  return f;
}

// One Stockham stage over all lines: a -> b.  Twiddles come from the table
// tw[m] = exp(-2 pi i m / n) of the workgroup (conjugated for sign > 0): the
// stage's factor exp(sign 2 pi i k / (Ns R)) is tw[k n / (Ns R)].
__device__ inline void fft_stage(const double2 *a, double2 *b, int n, int lb, int R, int Ns,
                                 double sign, const double2 *tw) {
  const int nbf = n / R;  // butterflies per line
  const int step = n / (Ns * R);
  auto twid = [&](int idx) {
    const double2 w = tw[idx];
    return sign > 0.0 ? make_double2(w.x, -w.y) : w;
  };
  for (int t = threadIdx.x; t < lb * nbf; t += blockDim.x) {
    const int line = t / nbf;
    const int j = t - line * nbf;
    const double2 *src = a + line * n;
    double2 *dst = b + line * n;
    const int k = j % Ns;
    const int base = (j / Ns) * Ns * R + k;
    const int m = k * step;  // < n / R
    if (R == 4) {
      double2 x0 = src[j], x1 = src[j + nbf], x2 = src[j + 2 * nbf], x3 = src[j + 3 * nbf];
      if (k) {
        x1 = cmul(x1, twid(m));
        x2 = cmul(x2, twid(2 * m));
        x3 = cmul(x3, twid(3 * m));
      }
      const double2 s02 = cadd(x0, x2), d02 = csub(x0, x2);
      const double2 s13 = cadd(x1, x3), d13 = cmuli(csub(x1, x3), sign);
      dst[base] = cadd(s02, s13);
      dst[base + Ns] = cadd(d02, d13);
      dst[base + 2 * Ns] = csub(s02, s13);
      dst[base + 3 * Ns] = csub(d02, d13);
    } else if (R == 2) {
      double2 x0 = src[j], x1 = src[j + nbf];
      if (k) x1 = cmul(x1, twid(m));
      dst[base] = cadd(x0, x1);
      dst[base + Ns] = csub(x0, x1);
    } else if (R == 3) {
      double2 x0 = src[j], x1 = src[j + nbf], x2 = src[j + 2 * nbf];
      if (k) {
        x1 = cmul(x1, twid(m));
        x2 = cmul(x2, twid(2 * m));
      }
      const double2 t1 = cadd(x1, x2);
      const double2 t2 = cmuli(csub(x1, x2), sign * 0.86602540378443864676);
      const double2 mm = make_double2(x0.x - 0.5 * t1.x, x0.y - 0.5 * t1.y);
      dst[base] = cadd(x0, t1);
      dst[base + Ns] = cadd(mm, t2);
      dst[base + 2 * Ns] = csub(mm, t2);
    } else {
      // generic radix: twiddle, then a direct DFT of length R; the total
      // phase tt k / (Ns R) + (s tt mod R) / R turns is the table entry
      // tt m + (s tt mod R) n / R (mod n)
      for (int s = 0; s < R; ++s) {
        double2 acc = make_double2(0.0, 0.0);
        for (int tt = 0; tt < R; ++tt) {
          const double2 x = src[j + tt * nbf];
          acc = cadd(acc, cmul(x, twid((tt * m + ((s * tt) % R) * (n / R)) % n)));
        }
        dst[base + s * Ns] = acc;
      }
    }
  }
}

constexpr int radix_span(const Radices &f, int st) {
  int p = 1;
  for (int i = 0; i < st; ++i) p *= f.r[i];
  return p;
}

// fft_stage with the line length, the batch, the radix and the span Ns known
// at compile time: the same butterflies and twiddle indices, with the index
// arithmetic folded into constants instead of run-time divisions.
template <int N, int LB, int R, int NS>
__device__ inline void fft_stage_c(const double2 *a, double2 *b, double sign, const double2 *tw) {
  constexpr int NBF = N / R;
  constexpr int STEP = N / (NS * R);
  auto twid = [&](int idx) {
    const double2 w = tw[idx];
    return sign > 0.0 ? make_double2(w.x, -w.y) : w;
  };
#pragma unroll
  for (int t0 = 0; t0 < LB * NBF; t0 += kBlock) {
    const int t = t0 + (int)threadIdx.x;
    if (LB * NBF % kBlock != 0 && t >= LB * NBF) break;
    const int line = t / NBF;
    const int j = t - line * NBF;
    const double2 *src = a + line * N;
    double2 *dst = b + line * N;
    const int k = j % NS;
    const int base = (j / NS) * NS * R + k;
    const int m = k * STEP;
    if constexpr (R == 4) {
      double2 x0 = src[j], x1 = src[j + NBF], x2 = src[j + 2 * NBF], x3 = src[j + 3 * NBF];
      if (k) {
        x1 = cmul(x1, twid(m));
        x2 = cmul(x2, twid(2 * m));
        x3 = cmul(x3, twid(3 * m));
      }
      const double2 s02 = cadd(x0, x2), d02 = csub(x0, x2);
      const double2 s13 = cadd(x1, x3), d13 = cmuli(csub(x1, x3), sign);
      dst[base] = cadd(s02, s13);
      dst[base + NS] = cadd(d02, d13);
      dst[base + 2 * NS] = csub(s02, s13);
      dst[base + 3 * NS] = csub(d02, d13);
    } else if constexpr (R == 2) {
      double2 x0 = src[j], x1 = src[j + NBF];
      if (k) x1 = cmul(x1, twid(m));
      dst[base] = cadd(x0, x1);
      dst[base + NS] = csub(x0, x1);
    } else if constexpr (R == 3) {
      double2 x0 = src[j], x1 = src[j + NBF], x2 = src[j + 2 * NBF];
      if (k) {
        x1 = cmul(x1, twid(m));
        x2 = cmul(x2, twid(2 * m));
      }
      const double2 t1 = cadd(x1, x2);
      const double2 t2 = cmuli(csub(x1, x2), sign * 0.86602540378443864676);
      const double2 mm = make_double2(x0.x - 0.5 * t1.x, x0.y - 0.5 * t1.y);
      dst[base] = cadd(x0, t1);
      dst[base + NS] = cadd(mm, t2);
      dst[base + 2 * NS] = csub(mm, t2);
    } else {
      for (int s = 0; s < R; ++s) {
        double2 acc = make_double2(0.0, 0.0);
        for (int tt = 0; tt < R; ++tt) {
          const double2 x = src[j + tt * NBF];
          acc = cadd(acc, cmul(x, twid((tt * m + ((s * tt) % R) * (N / R)) % N)));
        }
        dst[base + s * NS] = acc;
      }
    }
  }
}

template <int N, int LB, int ST>
__device__ inline double2 *fft_lines_c(double2 *a, double2 *b, double sign, const double2 *tw) {
  constexpr Radices F = factorize(N);
  if constexpr (ST == F.nr) {
    return a;
  } else {
    fft_stage_c<N, LB, F.r[ST], radix_span(F, ST)>(a, b, sign, tw);
    __syncthreads();
    return fft_lines_c<N, LB, ST + 1>(b, a, sign, tw);
  }
}

// Transform lb lines in LDS buffers a/b; returns the buffer holding the result.
__device__ inline double2 *fft_lines(double2 *a, double2 *b, int n, int lb, Radices f,
                                     double sign, const double2 *tw) {
  int Ns = 1;
  for (int st = 0; st < f.nr; ++st) {
    fft_stage(a, b, n, lb, f.r[st], Ns, sign, tw);
    __syncthreads();
    double2 *t = a;
    a = b;
    b = t;
    Ns *= f.r[st];
  }
  return a;
}

// mode 0: complex -> complex forward; 1: real input, forward; 2: inverse, real
// output scaled by `scale`; 3: forward, multiply by scale / (Laplacian symbol),
// inverse (z lines only); 4: complex -> complex inverse.  axis: 0 = x, 1 = y, 2 = z.
// NC > 0: a transform specialised on n = NC (the n and lb arguments are then
// NC and its batch); NC = 0: any n.
template <int NC>
__global__ __launch_bounds__(kBlock) void k_fft(const void *__restrict__ in,
                                                void *__restrict__ out, int n_arg, int axis,
                                                int lb_arg, int mode, Radices f,
                                                const double *__restrict__ lam1,
                                                double scale, double *__restrict__ dc) {
  constexpr int LBC = NC > 0 ? fft_lines_per_group(NC) : 0;
  const int n = NC > 0 ? NC : n_arg;
  const int lb = NC > 0 ? LBC : lb_arg;
  extern __shared__ double2 lds[];
  double2 *a = lds;
  double2 *b = lds + lb * n;
  double2 *tw = lds + 2 * lb * n;  // tw[m] = exp(-2 pi i m / n)
  auto twiddles = [&]() {
    for (int m = threadIdx.x; m < n; m += kBlock) {
      double sv, cv;
      sincospi(-2.0 * (double)m / (double)n, &sv, &cv);
      tw[m] = make_double2(cv, sv);
    }
  };
  if (NC == 0) twiddles();
  const i64 n2 = (i64)n * n;
  // batch decoding: for x lines the batch is lb consecutive y rows of one z;
  // for y and z lines the batch is lb consecutive x of one (z) or (y).
  const int groups_per_row = (n + lb - 1) / lb;
  const int grp = blockIdx.x % groups_per_row;
  const int outer = blockIdx.x / groups_per_row;  // z for x/y lines, y for z lines
  const int first = grp * lb;
  const int nl = min(lb, n - first);
  i64 stride, base0, lstride;
  if (axis == 0) {  // element stride 1, line stride n, lines = y rows
    stride = 1;
    lstride = n;
    base0 = (i64)outer * n2 + (i64)first * n;
  } else if (axis == 1) {  // element stride n, lines = consecutive x
    stride = n;
    lstride = 1;
    base0 = (i64)outer * n2 + first;
  } else {  // element stride n^2, lines = consecutive x of row `outer` (y)
    stride = n2;
    lstride = 1;
    base0 = (i64)outer * n + first;
  }
  const double sign = (mode == 2 || mode == 4) ? 1.0 : -1.0;
  // load: element index e over lines, consecutive threads take consecutive lines
  auto load_elem = [&](int t) -> double2 {
    int line, e;
    if (axis == 0) { line = t / n; e = t % n; } else { e = t / lb; line = t % lb; }
    double2 v = make_double2(0.0, 0.0);
    if (line < nl) {
      const i64 gi = base0 + (i64)line * lstride + (i64)e * stride;
      if (mode == 1) v = make_double2(((const double *)in)[gi], 0.0);
      else v = ((const double2 *)in)[gi];
    }
    return v;
  };
  auto lds_index = [&](int t) {
    return axis == 0 ? t : (t % lb) * n + t / lb;
  };
  double2 *res;
  if constexpr (NC > 0) {
    // every load of the batch in flight before the twiddle table is computed
    constexpr int PER = (LBC * NC + kBlock - 1) / kBlock;
    double2 v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int t = (int)threadIdx.x + i * kBlock;
      v[i] = (t < LBC * NC) ? load_elem(t) : make_double2(0.0, 0.0);
    }
    twiddles();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int t = (int)threadIdx.x + i * kBlock;
      if (t < LBC * NC) a[lds_index(t)] = v[i];
    }
    __syncthreads();
    res = fft_lines_c<NC, LBC, 0>(a, b, sign, tw);
  } else {
    for (int t = threadIdx.x; t < lb * n; t += kBlock) a[lds_index(t)] = load_elem(t);
    __syncthreads();
    res = fft_lines(a, b, n, lb, f, sign, tw);
  }
  if (mode == 3) {
    // z lines: element e is kz; the line is (kx = first + line, ky = outer)
    for (int t = threadIdx.x; t < lb * n; t += kBlock) {
      const int line = t / n, e = t % n;
      double2 v = res[t];
      if (line < nl) {
        const bool mean_mode = first + line == 0 && outer == 0 && e == 0;
        // the (0,0,0) coefficient of the unnormalised forward transform is
        // the sum of the input over the grid
        if (mean_mode && dc != nullptr) dc[0] = v.x;
        const double lam = lam1[first + line] + lam1[outer] + lam1[e];
        const double w = mean_mode ? 0.0 : scale / lam;
        v = make_double2(v.x * w, v.y * w);
      }
      res[t] = v;
    }
    __syncthreads();
    double2 *other = (res == a) ? b : a;
    if constexpr (NC > 0) res = fft_lines_c<NC, LBC, 0>(res, other, 1.0, tw);
    else res = fft_lines(res, other, n, lb, f, 1.0, tw);
  }
  for (int t = threadIdx.x; t < lb * n; t += kBlock) {
    int line, e;
    if (axis == 0) { line = t / n; e = t % n; } else { e = t / lb; line = t % lb; }
    if (line < nl) {
      const i64 gi = base0 + (i64)line * lstride + (i64)e * stride;
      const double2 v = res[line * n + e];
      if (mode == 2) ((double *)out)[gi] = v.x * scale;
      else ((double2 *)out)[gi] = v;
    }
  }
}

// ----------------------------------------------------------------- ions

// atoms: [M][5] = (Rx, Ry, Rz, Z, sigma)
__global__ __launch_bounds__(kBlock) void k_ion_density(const double *__restrict__ atoms,
                                                        int M, double *__restrict__ rho,
                                                        int n, double L) {
  const i64 ng = (i64)n * n * n;
  const double h = L / n;
  const double pi = 3.14159265358979323846;
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x) {
    const double x = h * (double)(g % n);
    const double y = h * (double)((g / n) % n);
    const double z = h * (double)(g / ((i64)n * n));
    double acc = 0.0;
    for (int I = 0; I < M; ++I) {
      double dx = x - atoms[5 * I + 0];
      double dy = y - atoms[5 * I + 1];
      double dz = z - atoms[5 * I + 2];
      dx -= L * rint(dx / L);
      dy -= L * rint(dy / L);
      dz -= L * rint(dz / L);
      const double s = atoms[5 * I + 4];
      const double d2 = dx * dx + dy * dy + dz * dz;
      acc += atoms[5 * I + 3] * exp(-d2 / (s * s)) / (s * s * s * pi * sqrt(pi));
    }
    rho[g] = acc;
  }
}

// Partials of <V_H, d rho_I/dR_a> and <V_H, d rho_I/d sigma> (unscaled).
__global__ __launch_bounds__(kBlock) void k_ion_forces(const double *__restrict__ atoms,
                                                       const double *__restrict__ vh,
                                                       double *__restrict__ part, int n,
                                                       double L) {
  __shared__ double red[4 * 4];
  const int I = blockIdx.y;
  const i64 ng = (i64)n * n * n;
  const double h = L / n;
  const double pi = 3.14159265358979323846;
  const double Rx = atoms[5 * I + 0], Ry = atoms[5 * I + 1], Rz = atoms[5 * I + 2];
  const double Zi = atoms[5 * I + 3], s = atoms[5 * I + 4];
  const double norm = Zi / (s * s * s * pi * sqrt(pi));
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x) {
    double dx = h * (double)(g % n) - Rx;
    double dy = h * (double)((g / n) % n) - Ry;
    double dz = h * (double)(g / ((i64)n * n)) - Rz;
    dx -= L * rint(dx / L);
    dy -= L * rint(dy / L);
    dz -= L * rint(dz / L);
    const double d2 = dx * dx + dy * dy + dz * dz;
    const double gv = norm * exp(-d2 / (s * s)) * vh[g];
    const double t = 2.0 / (s * s);
    a[0] += gv * t * dx;
    a[1] += gv * t * dy;
    a[2] += gv * t * dz;
    a[3] += gv * (2.0 * d2 / (s * s * s) - 3.0 / s);
  }
  block_sum<4>(a, red);
  if (threadIdx.x == 0) {
    const i64 idx = ((i64)I * gridDim.x + blockIdx.x) * 4;
    part[idx + 0] = a[0];
    part[idx + 1] = a[1];
    part[idx + 2] = a[2];
    part[idx + 3] = a[3];
  }
}

// ----------------------------------------------------------------- block steps

// Trial point of Algorithm M (section 3.2): W - tau z_i with
// z_i = H w_i - sigma_ii w_i.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_trial(const T *__restrict__ W,
                                                  const T *__restrict__ HW,
                                                  const double *__restrict__ sig,
                                                  const double *__restrict__ dtau, double tscale,
                                                  T *__restrict__ Wt, i64 ng) {
  const int orb = blockIdx.y;
  const double tau = dtau[0] * tscale;
  const double a = 1.0 + tau * sig[orb];
  const T ta = (T)a, tt = (T)tau;
  const i64 off = (i64)orb * ng;
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x)
    Wt[off + g] = ta * W[off + g] - tt * HW[off + g];
}

// Accept the trial: U <- Wn, and per-orbital partial dot products for the
// next Barzilai-Borwein step (S = Wn - W, Y = Zn - Z) and ||Zn||^2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_commit(T *__restrict__ U, const T *__restrict__ HW,
                                                   const double *__restrict__ sig,
                                                   const T *__restrict__ Wn,
                                                   const T *__restrict__ HWn,
                                                   const double *__restrict__ sign,
                                                   double *__restrict__ part, i64 ng,
                                                   const double *__restrict__ gate) {
  if (gate != nullptr && gate[0] == 0.0) return;
  __shared__ double red[4 * 4];
  const int orb = blockIdx.y;
  const double so = sig[orb], sn = sign[orb];
  const i64 off = (i64)orb * ng;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  auto point = [&](T uo, T un, T ho, T hn) __attribute__((always_inline)) {
    const double wo = (double)uo, wn = (double)un;
    const double zo = (double)ho - so * wo;
    const double zn = (double)hn - sn * wn;
    const double s = wn - wo;
    const double y = zn - zo;
    a[0] += s * s;
    a[1] += s * y;
    a[2] += y * y;
    a[3] += zn * zn;
  };
  // 16-byte accesses when every orbital row starts 16-byte aligned (a
  // quarter of the load and store instructions of the element loop), two per
  // stream in flight per thread, all marked non-temporal: each value is used
  // once, and keeping the five streams out of the caches measured 16% faster
  // (450 -> 380 us at 96^3 x 128 FP32) than plain accesses
  constexpr int V = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(V)));
  const bool aligned = ng % V == 0 && (((uintptr_t)U | (uintptr_t)HW | (uintptr_t)Wn |
                                        (uintptr_t)HWn) & 15) == 0;
  if (aligned) {
    const i64 nv = ng / V, ov = off / V;
    const i64 stride = (i64)gridDim.x * blockDim.x;
    for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < nv; g += 2 * stride) {
      const i64 g2 = g + stride;
      const bool two = g2 < nv;
      const i64 gb = two ? g2 : g;  // a valid index either way; unused when !two
      const vec uo = __builtin_nontemporal_load(&((const vec *)U)[ov + g]);
      const vec un = __builtin_nontemporal_load(&((const vec *)Wn)[ov + g]);
      const vec ho = __builtin_nontemporal_load(&((const vec *)HW)[ov + g]);
      const vec hn = __builtin_nontemporal_load(&((const vec *)HWn)[ov + g]);
      const vec uo2 = __builtin_nontemporal_load(&((const vec *)U)[ov + gb]);
      const vec un2 = __builtin_nontemporal_load(&((const vec *)Wn)[ov + gb]);
      const vec ho2 = __builtin_nontemporal_load(&((const vec *)HW)[ov + gb]);
      const vec hn2 = __builtin_nontemporal_load(&((const vec *)HWn)[ov + gb]);
#pragma unroll
      for (int e = 0; e < V; ++e) point(uo[e], un[e], ho[e], hn[e]);
      __builtin_nontemporal_store(un, &((vec *)U)[ov + g]);
      if (two) {
#pragma unroll
        for (int e = 0; e < V; ++e) point(uo2[e], un2[e], ho2[e], hn2[e]);
        __builtin_nontemporal_store(un2, &((vec *)U)[ov + g2]);
      }
    }
  } else {
    for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
         g += (i64)gridDim.x * blockDim.x) {
      point(U[off + g], Wn[off + g], HW[off + g], HWn[off + g]);
      U[off + g] = Wn[off + g];
    }
  }
  block_sum<4>(a, red);
  if (threadIdx.x == 0) {
    const i64 idx = ((i64)orb * gridDim.x + blockIdx.x) * 4;
    part[idx + 0] = a[0];
    part[idx + 1] = a[1];
    part[idx + 2] = a[2];
    part[idx + 3] = a[3];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_zz(const T *__restrict__ W, const T *__restrict__ HW,
                                               const double *__restrict__ sig,
                                               double *__restrict__ part, i64 ng) {
  __shared__ double red[4];
  const int orb = blockIdx.y;
  const double so = sig[orb];
  const i64 off = (i64)orb * ng;
  double acc = 0.0;
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x) {
    const double z = (double)HW[off + g] - so * (double)W[off + g];
    acc += z * z;
  }
  double v[1] = {acc};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) part[(i64)orb * gridDim.x + blockIdx.x] = v[0];
}

// Per (orbital, block) partials of <a_i, b_i> (diff == 0) or of
// |a_i - b_i|^2 (diff != 0), FP64 accumulation.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rowdot(const T *__restrict__ A, const T *__restrict__ B,
                                                   int diff, double *__restrict__ part, i64 ng) {
  __shared__ double red[4];
  const int orb = blockIdx.y;
  const i64 off = (i64)orb * ng;
  double acc = 0.0;
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x) {
    const double a = (double)A[off + g], b = (double)B[off + g];
    acc += diff ? (a - b) * (a - b) : a * b;
  }
  double v[1] = {acc};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) part[(i64)orb * gridDim.x + blockIdx.x] = v[0];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_backward_scale(const T *__restrict__ HU,
                                                           const double *__restrict__ occ,
                                                           double scale, T *__restrict__ dU,
                                                           i64 ng) {
  const int orb = blockIdx.y;
  const T f = (T)(scale * occ[orb]);
  const i64 off = (i64)orb * ng;
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (i64)gridDim.x * blockDim.x)
    dU[off + g] = f * HU[off + g];
}

template <typename S, typename D>
__global__ __launch_bounds__(kBlock) void k_convert(const S *__restrict__ src,
                                                    D *__restrict__ dst, i64 count) {
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < count;
       g += (i64)gridDim.x * blockDim.x)
    dst[g] = (D)src[g];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_nonfinite(const T *__restrict__ x, i64 count,
                                                      int *__restrict__ flag) {
  bool bad = false;
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < count;
       g += (i64)gridDim.x * blockDim.x)
    bad |= !isfinite((double)x[g]);
  if (bad) flag[0] = 1;
}

// Barzilai-Borwein step from the per-orbital dot products (section 3.2):
// tau1 = tr<S^T S> / |tr<S^T Y>|, tau2 = |tr<S^T Y>| / tr<Y^T Y>; mode 0 means
// no history (tau_init).  red holds [k * N + i] per-orbital sums (k = 0 ss,
// 1 sy, 2 yy, 3 zz) or, in mode 0, zz per orbital in [i].  One wave, fixed
// summation order.  out = (tau_BB, zz, ss, sy, yy).
__global__ __launch_bounds__(64) void k_bb_tau(const double *__restrict__ red, int N, int mode,
                                                double tau_init, double *__restrict__ out,
                                                const double *__restrict__ gate) {
  if (gate != nullptr && gate[0] == 0.0) return;
  const int l = threadIdx.x;
  double ss = 0.0, sy = 0.0, yy = 0.0, zz = 0.0;
  // lane l sums orbitals l, l + 64, ...; the wave then combines in a fixed order
  for (int i = l; i < N; i += 64) {
    if (mode == 0 || mode == 3) {
      zz += red[i];
    } else {
      ss += red[i];
      sy += red[N + i];
      yy += red[2 * N + i];
      zz += red[3 * N + i];
    }
  }
  ss = wave_sum(ss);
  sy = wave_sum(sy);
  yy = wave_sum(yy);
  zz = wave_sum(zz);
  if (l != 0) return;
  if (mode == 3) {  // ||Z||^2 only (after a subspace rotation); tau_BB is kept
    out[1] = zz;
    return;
  }
  double tau = tau_init;
  if (mode != 0) {
    const double asy = fabs(sy);
    const double t = (mode == 1) ? ss / asy : asy / yy;
    if (isfinite(t) && t > 0.0) tau = t;
  }
  out[0] = tau;
  out[1] = zz;
  out[2] = ss;
  out[3] = sy;
  out[4] = yy;
}

constexpr int kArmijoMaxN = 512;  // the library admits at most 512 orbitals

// Test of eq. "ene-de" for a trial on the device, so that the accept can be
// enqueued before the host has read the trial's energy.  rep is the trial's
// evaluation report (sigma N | kin N | e4 | orth info 2*npass at orth_off |
// rr, bb at rr_off), scal = (tau_BB, ||Z||^2, ...).  The energy is assembled as the
// host does (occupation-weighted kinetic sum in orbital order, then the
// exchange, external and Hartree terms).  ext[0..4] receives a copy of scal
// (so that one copy brings report, scalars and decision to the host);
// ext[5] = 1 when the trial is to be accepted: the Hartree residual met its
// target, every Cholesky pass was positive definite, E is finite, and
// E <= C - rho1 tau ||Z||^2 (or force, the last backtrack); ext[6] = 1 when
// the inequality itself held.
__global__ void k_armijo(const double *__restrict__ rep, const double *__restrict__ occ, int N,
                         unsigned terms, int npass, int orth_off, int rr_off, double rtol2,
                         const double *__restrict__ scal, double tscale, double C, double rho1,
                         int force, double *__restrict__ ext) {
  // no fused multiply-adds: the energy is rounded step by step as the host
  // rounds it when it reports the trial's terms
#pragma clang fp contract(off)
  // the wave forms the N products f_i t_i (N <= kArmijoMaxN) in LDS; lane 0
  // sums them in orbital order and takes the decision
  __shared__ double sp[kArmijoMaxN];
  if (blockIdx.x != 0) return;
  for (int i = threadIdx.x; i < N; i += blockDim.x) sp[i] = occ[i] * rep[N + i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 0; k < 5; ++k) ext[k] = scal[k];
  double *flags = ext + 5;
  const double rr = rep[rr_off], bb = rep[rr_off + 1];
  bool ok = isfinite(rr) && isfinite(bb) && rr <= rtol2 * bb;
  for (int p = 0; p < npass; ++p) ok = ok && rep[orth_off + 2 * p] == 0.0;
  double ekin = 0.0;
  for (int i = 0; i < N; ++i) ekin += sp[i];
  const double cx = 0.73855876638202240;  // 3/4 (3/pi)^(1/3)
  double E = (terms & 1u) ? ekin : 0.0;
  E += (terms & 8u) ? -cx * rep[2 * N + 0] : 0.0;
  E += (terms & 2u) ? rep[2 * N + 1] : 0.0;
  E += (terms & 4u) ? 0.5 * rep[2 * N + 2] : 0.0;
  E += (terms & 16u) ? rep[2 * N + 3] : 0.0;
  E += (terms & 32u) ? rep[rr_off + 2] : 0.0;  // nonlocal term (zero without projectors)
  ok = ok && isfinite(E);
  const double tau = scal[0] * tscale;
  const bool pass = E <= C - rho1 * tau * scal[1];
  flags[0] = (ok && (pass || force != 0)) ? 1.0 : 0.0;
  flags[1] = pass ? 1.0 : 0.0;
}

__global__ void k_set_flags(double *__restrict__ flags, double a, double b) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    flags[0] = a;
    flags[1] = b;
  }
}

inline int grid_for(i64 work, int cap = 4096) {
  i64 b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

}  // namespace

// ----------------------------------------------------------------- launchers

template <typename T>
hipError_t launch_hamiltonian(const T *U, const T *veff, T *HU, double *part, int N,
                              const StencilArgs &a, hipStream_t s) {
  const int groups = N * a.nzc;
  const int per_xcd = (groups + 7) / 8;
  dim3 grid(8 * per_xcd * a.ntile);
  hipLaunchKernelGGL(k_hamiltonian<T>, grid, dim3(kBlock), 0, s, U, veff, HU, part, a, N);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_density(const T *U, const double *occ, double *rho, int N, i64 ng,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_density<T>, dim3(grid_for(ng, 8192)), dim3(kBlock), 0, s, U, occ, rho,
                     N, ng);
  return hipGetLastError();
}

hipError_t launch_xc_veff(const double *rho, const double *vh, const double *vext,
                          double *veff, float *veff32, double *part, i64 ng, unsigned terms,
                          int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_xc_veff, dim3(nblk), dim3(kBlock), 0, s, rho, vh, vext, veff, veff32,
                     part, ng, terms);
  return hipGetLastError();
}

hipError_t launch_segment_sum(const double *part, double *out, int nseg, int len, int K,
                              double scale, hipStream_t s) {
  hipLaunchKernelGGL(k_segment_sum, dim3(nseg), dim3(kBlock), 0, s, part, out, nseg, len, K,
                     scale);
  return hipGetLastError();
}

hipError_t launch_neg_lap(const double *p, double *q, double *part, int n, double inv_h2,
                          int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_neg_lap, dim3(nblk), dim3(kBlock), 0, s, p, q, part, n, inv_h2);
  return hipGetLastError();
}

hipError_t launch_poisson_residual(const double *x, const double *rho, const double *dsum,
                                  double *part, int n, double inv_h2, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_poisson_residual, dim3(nblk), dim3(kBlock), 0, s, x, rho, dsum, part, n,
                     inv_h2);
  return hipGetLastError();
}

hipError_t launch_cg_rhs_residual(const double *rho, const double *dsum, const double *q,
                                  double *r, double *part, i64 ng, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_rhs_residual, dim3(nblk), dim3(kBlock), 0, s, rho, dsum, q, r, part,
                     ng);
  return hipGetLastError();
}

hipError_t launch_dot2(const double *a, const double *b, double *part, i64 ng, int nblk,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_dot2, dim3(nblk), dim3(kBlock), 0, s, a, b, part, ng);
  return hipGetLastError();
}

hipError_t launch_cg_update_p(double *p, const double *z, const double *num, const double *den,
                              int first, i64 ng, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update_p, dim3(grid_for(ng)), dim3(kBlock), 0, s, p, z, num, den,
                     first, ng);
  return hipGetLastError();
}

hipError_t launch_cg_update_xr(double *x, double *r, const double *p, const double *q,
                               const double *num, const double *den, double *part, i64 ng,
                               int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update_xr, dim3(nblk), dim3(kBlock), 0, s, x, r, p, q, num, den, part,
                     ng);
  return hipGetLastError();
}

hipError_t launch_scale(double *x, double a, i64 ng, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(ng)), dim3(kBlock), 0, s, x, a, ng);
  return hipGetLastError();
}

hipError_t launch_remove_mean(double *x, const double *dsum, i64 ng, hipStream_t s) {
  hipLaunchKernelGGL(k_remove_mean, dim3(grid_for(ng)), dim3(kBlock), 0, s, x, dsum, ng);
  return hipGetLastError();
}

hipError_t launch_spectral_inverse(const double *r, double *out, double2 *w0, double2 *w1,
                                   const double *lam1, int n, double scale, hipStream_t s,
                                   double *sum_r) {
  const Radices f = factorize(n);
  const int lb = fft_lines_per_group(n);
  if (lb < 1) return hipErrorInvalidValue;
  const size_t lds = fft_lds_bytes(n, lb);
  const int groups = (n + lb - 1) / lb;
  const dim3 grid(groups * n), block(kBlock);
  const double invn3 = scale / ((double)n * n * n);
  // x forward (real in) -> y forward -> z forward, divide, z inverse -> y inverse -> x inverse;
  // the grid sizes of the workloads have transforms specialised on n
  auto run = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, block, lds, s, (const void *)r, (void *)w0, n, 0, lb, 1, f,
                       lam1, 1.0, (double *)nullptr);
    hipLaunchKernelGGL(kern, grid, block, lds, s, (const void *)w0, (void *)w1, n, 1, lb, 0, f,
                       lam1, 1.0, (double *)nullptr);
    hipLaunchKernelGGL(kern, grid, block, lds, s, (const void *)w1, (void *)w0, n, 2, lb, 3, f,
                       lam1, invn3, sum_r);
    hipLaunchKernelGGL(kern, grid, block, lds, s, (const void *)w0, (void *)w1, n, 1, lb, 4, f,
                       lam1, 1.0, (double *)nullptr);
    hipLaunchKernelGGL(kern, grid, block, lds, s, (const void *)w1, (void *)out, n, 0, lb, 2, f,
                       lam1, 1.0, (double *)nullptr);
  };
  switch (n) {
    case 16: run(k_fft<16>); break;
    case 32: run(k_fft<32>); break;
    case 48: run(k_fft<48>); break;
    case 64: run(k_fft<64>); break;
    case 96: run(k_fft<96>); break;
    case 128: run(k_fft<128>); break;
    default: run(k_fft<0>); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_trial(const T *W, const T *HW, const double *sig, const double *dtau,
                        double tscale, T *Wt, int N, i64 ng, hipStream_t s) {
  dim3 grid(grid_for(ng, 1024), N);
  hipLaunchKernelGGL(k_trial<T>, grid, dim3(kBlock), 0, s, W, HW, sig, dtau, tscale, Wt, ng);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_commit(T *U, const T *HW, const double *sig, const T *Wn, const T *HWn,
                         const double *sign, double *part, int N, i64 ng, int nblk,
                         const double *gate, hipStream_t s) {
  dim3 grid(nblk, N);
  hipLaunchKernelGGL(k_commit<T>, grid, dim3(kBlock), 0, s, U, HW, sig, Wn, HWn, sign, part,
                     ng, gate);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zz(const T *W, const T *HW, const double *sig, double *part, int N, i64 ng,
                     int nblk, hipStream_t s) {
  dim3 grid(nblk, N);
  hipLaunchKernelGGL(k_zz<T>, grid, dim3(kBlock), 0, s, W, HW, sig, part, ng);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rowdot(const T *A, const T *B, bool diff, double *part, int N, i64 ng, int nblk,
                         hipStream_t s) {
  dim3 grid(nblk, N);
  hipLaunchKernelGGL(k_rowdot<T>, grid, dim3(kBlock), 0, s, A, B, diff ? 1 : 0, part, ng);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_backward_scale(const T *HU, const double *occ, double scale, T *dU, int N,
                                 i64 ng, hipStream_t s) {
  dim3 grid(grid_for(ng, 1024), N);
  hipLaunchKernelGGL(k_backward_scale<T>, grid, dim3(kBlock), 0, s, HU, occ, scale, dU, ng);
  return hipGetLastError();
}

template <typename S, typename D>
hipError_t launch_convert(const S *src, D *dst, i64 count, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<S, D>), dim3(grid_for(count, 16384)), dim3(kBlock), 0, s, src,
                     dst, count);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_nonfinite(const T *x, i64 count, int *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite<T>, dim3(grid_for(count, 16384)), dim3(kBlock), 0, s, x, count,
                     flag);
  return hipGetLastError();
}

hipError_t launch_bb_tau(const double *red, int N, int mode, double tau_init, double *out,
                         const double *gate, hipStream_t s) {
  hipLaunchKernelGGL(k_bb_tau, dim3(1), dim3(64), 0, s, red, N, mode, tau_init, out, gate);
  return hipGetLastError();
}

hipError_t launch_armijo(const double *rep, const double *occ, int N, unsigned terms, int npass,
                         int orth_off, int rr_off, double rtol2, const double *scal,
                         double tscale, double C, double rho1, int force, double *ext,
                         hipStream_t s) {
  if (N < 1 || N > kArmijoMaxN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_armijo, dim3(1), dim3(64), 0, s, rep, occ, N, terms, npass, orth_off,
                     rr_off, rtol2, scal, tscale, C, rho1, force, ext);
  return hipGetLastError();
}

hipError_t launch_set_flags(double *flags, double a, double b, hipStream_t s) {
  hipLaunchKernelGGL(k_set_flags, dim3(1), dim3(64), 0, s, flags, a, b);
  return hipGetLastError();
}

hipError_t launch_ion_density(const double *atoms, int M, double *rho_ion, int n, double L,
                              hipStream_t s) {
  const i64 ng = (i64)n * n * n;
  hipLaunchKernelGGL(k_ion_density, dim3(grid_for(ng, 16384)), dim3(kBlock), 0, s, atoms, M,
                     rho_ion, n, L);
  return hipGetLastError();
}

hipError_t launch_ion_forces(const double *atoms, int M, const double *vh, double *part, int n,
                             double L, int nblk, hipStream_t s) {
  dim3 grid(nblk, M);
  hipLaunchKernelGGL(k_ion_forces, grid, dim3(kBlock), 0, s, atoms, vh, part, n, L);
  return hipGetLastError();
}

#define POU_INST_T(T)                                                                       \
  template hipError_t launch_hamiltonian<T>(const T *, const T *, T *, double *, int,       \
                                            const StencilArgs &, hipStream_t);              \
  template hipError_t launch_density<T>(const T *, const double *, double *, int, i64,      \
                                        hipStream_t);                                       \
  template hipError_t launch_trial<T>(const T *, const T *, const double *, const double *, \
                                      double, T *, int, i64, hipStream_t);                  \
  template hipError_t launch_commit<T>(T *, const T *, const double *, const T *, const T *, \
                                       const double *, double *, int, i64, int,             \
                                       const double *, hipStream_t);                        \
  template hipError_t launch_zz<T>(const T *, const T *, const double *, double *, int, i64, \
                                   int, hipStream_t);                                       \
  template hipError_t launch_rowdot<T>(const T *, const T *, bool, double *, int, i64, int,   \
                                       hipStream_t);                                        \
  template hipError_t launch_backward_scale<T>(const T *, const double *, double, T *, int, \
                                               i64, hipStream_t);                           \
  template hipError_t launch_nonfinite<T>(const T *, i64, int *, hipStream_t);

POU_INST_T(double)
POU_INST_T(float)
template hipError_t launch_convert<float, double>(const float *, double *, i64, hipStream_t);
template hipError_t launch_convert<double, float>(const double *, float *, i64, hipStream_t);
template hipError_t launch_convert<double, double>(const double *, double *, i64, hipStream_t);
template hipError_t launch_convert<float, float>(const float *, float *, i64, hipStream_t);

}  // namespace pou
