// Nonlocal part of the pseudopotential (section 2.1): V_nloc u = sum_l
// <xi_l, u> xi_l with four atom-centred Gaussian projectors per ion,
//   xi_s = b_s g,  xi_a = b_p (d_a / rc) g,  g = exp(-|d|^2 / (2 rc^2)),
// d = r - R_I by minimum image.  Each ion's projectors are evaluated on the
// fly inside a cube of b^3 grid points around it (b odd, the cube reaches
// past the radius where g falls below 1e-14, or the whole grid when that
// radius does not fit), so nothing is tabulated.
//
// The work is a gather over the ions' cubes, bound by the loads of the
// orbital values there; it stays on the vector units (two flops per load
// leave nothing for the matrix cores to do):
//   * k_nl_overlap: C[l][i] = <xi_l, u_i> (or, for the forces, the overlaps
//     with d xi_l / d R_I) as fixed-order partial sums per (ion, orbital
//     chunk, cube split);
//   * k_nl_apply: H u_i += sum_l xi_l C[l][i] over the cubes of one colour
//     (ions whose cubes do not overlap), so no two workgroups write the same
//     point and the colours are added in a fixed order;
//   * k_nl_finish: sigma_ii += sum_l C[l][i]^2 and E_nl = sum_i f_i sum_l C[l][i]^2.
#include "pou_internal.h"

namespace pou {
namespace {

// Minimum-image offset of grid coordinate x from position r on a period L.
__device__ inline double mic(double x, double r, double L) {
  double d = x - r;
  return d - L * rint(d / L);
}

// Grid point and offsets (dx, dy, dz) of cube point e of ion a.
__device__ inline i64 cube_point(const NlIon &a, int e, int n, double h, double L, double &dx,
                                 double &dy, double &dz) {
  const int b = a.b;
  const int i = e % b, j = (e / b) % b, k = e / (b * b);
  int x = a.o[0] + i, y = a.o[1] + j, z = a.o[2] + k;
  x -= (x >= n) ? n : 0;
  y -= (y >= n) ? n : 0;
  z -= (z >= n) ? n : 0;
  dx = mic(h * x, a.R[0], L);
  dy = mic(h * y, a.R[1], L);
  dz = mic(h * z, a.R[2], L);
  return ((i64)z * n + y) * n + x;
}

// The four projector values (s, x, y, z) at offset d.
__device__ inline void proj_values(const NlIon &a, double dx, double dy, double dz,
                                   double (&xi)[4]) {
  const double irc = 1.0 / a.rc;
  const double g = exp(-0.5 * (dx * dx + dy * dy + dz * dz) * irc * irc);
  const double gp = a.bp * irc * g;
  xi[0] = a.bs * g;
  xi[1] = gp * dx;
  xi[2] = gp * dy;
  xi[3] = gp * dz;
}

// d xi_l / d R_a (l = s, x, y, z; a = x, y, z) at offset d, index 3 l + a:
// the ion enters through d = r - R, so d/dR = -d/dd.
__device__ inline void proj_derivatives(const NlIon &a, double dx, double dy, double dz,
                                        double (&dxi)[12]) {
  const double irc = 1.0 / a.rc, irc2 = irc * irc;
  const double g = exp(-0.5 * (dx * dx + dy * dy + dz * dz) * irc2);
  const double d[3] = {dx, dy, dz};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double dg = -d[ax] * irc2 * g;  // d g / d d_ax
    dxi[ax] = -a.bs * dg;
#pragma unroll
    for (int l = 0; l < 3; ++l)
      dxi[3 * (l + 1) + ax] = -(a.bp * irc * (d[l] * dg + (l == ax ? g : 0.0)));
  }
}

// grid (ions, orbital chunks of OC, cube splits); part[((I * nsp + sp) * N + i) * K + l]
template <typename T, int OC, bool DER>
__global__ __launch_bounds__(kBlock) void k_nl_overlap(const T *__restrict__ U,
                                                       const NlIon *__restrict__ ions, int N,
                                                       int n, double L,
                                                       double *__restrict__ part) {
  constexpr int K = DER ? 12 : 4;
  __shared__ double red[4 * K * OC];
  const NlIon a = ions[blockIdx.x];
  const int i0 = blockIdx.y * OC;
  const int nsp = gridDim.z, sp = blockIdx.z;
  const i64 ng = (i64)n * n * n;
  const double h = L / n;
  const int vol = a.b * a.b * a.b;
  const int per = (vol + nsp - 1) / nsp;
  const int e0 = sp * per, e1 = min(vol, e0 + per);
  double acc[OC * K];
#pragma unroll
  for (int k = 0; k < OC * K; ++k) acc[k] = 0.0;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += kBlock) {
    double dx, dy, dz;
    const i64 g = cube_point(a, e, n, h, L, dx, dy, dz);
    double f[K];
    if constexpr (DER) proj_derivatives(a, dx, dy, dz, f);
    else proj_values(a, dx, dy, dz, f);
#pragma unroll
    for (int o = 0; o < OC; ++o) {
      const double u = (i0 + o < N) ? (double)U[(i64)(i0 + o) * ng + g] : 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) acc[o * K + k] += f[k] * u;
    }
  }
  block_sum<OC * K>(acc, red);
  if (threadIdx.x == 0) {
    for (int o = 0; o < OC; ++o) {
      if (i0 + o >= N) break;
      double *dst = part + (((i64)blockIdx.x * nsp + sp) * N + (i0 + o)) * K;
#pragma unroll
      for (int k = 0; k < K; ++k) dst[k] = acc[o * K + k];
    }
  }
}

// H u_i += sum_l xi_l C[l][i] over the cubes of the ions listed in `list`
// (one colour: no two cubes share a point).  grid (listed ions, orbital
// chunks of OC, cube splits).  C: [4 M][N].
template <typename T, int OC>
__global__ __launch_bounds__(kBlock) void k_nl_apply(T *__restrict__ HU,
                                                     const NlIon *__restrict__ ions,
                                                     const int *__restrict__ list,
                                                     const double *__restrict__ C, int N, int n,
                                                     double L) {
  const int I = list[blockIdx.x];
  const NlIon a = ions[I];
  const int i0 = blockIdx.y * OC;
  const int nsp = gridDim.z, sp = blockIdx.z;
  const i64 ng = (i64)n * n * n;
  const double h = L / n;
  const int vol = a.b * a.b * a.b;
  const int per = (vol + nsp - 1) / nsp;
  const int e0 = sp * per, e1 = min(vol, e0 + per);
  double c[OC][4];
#pragma unroll
  for (int o = 0; o < OC; ++o)
#pragma unroll
    for (int l = 0; l < 4; ++l)
      c[o][l] = (i0 + o < N) ? C[(i64)(4 * I + l) * N + (i0 + o)] : 0.0;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += kBlock) {
    double dx, dy, dz;
    const i64 g = cube_point(a, e, n, h, L, dx, dy, dz);
    double xi[4];
    proj_values(a, dx, dy, dz, xi);
#pragma unroll
    for (int o = 0; o < OC; ++o) {
      if (i0 + o >= N) break;
      const double v = xi[0] * c[o][0] + xi[1] * c[o][1] + xi[2] * c[o][2] + xi[3] * c[o][3];
      T *p = HU + (i64)(i0 + o) * ng + g;
      *p = (T)((double)*p + v);
    }
  }
}

// C[l][i] = dv * sum over splits; sigma_ii (rep[i]) += sum_l C[l][i]^2;
// rep[enl_off] = sum_i f_i sum_l C[l][i]^2.  One workgroup, fixed order.
__global__ __launch_bounds__(kBlock) void k_nl_finish(const double *__restrict__ part, int M,
                                                      int nsp, int N, double dv,
                                                      const double *__restrict__ occ,
                                                      double *__restrict__ C,
                                                      double *__restrict__ rep, int enl_off) {
  __shared__ double red[4];
  double e = 0.0;
  for (int i = threadIdx.x; i < N; i += kBlock) {
    double s2 = 0.0;
    for (int I = 0; I < M; ++I) {
      for (int l = 0; l < 4; ++l) {
        double v = 0.0;
        for (int sp = 0; sp < nsp; ++sp) v += part[(((i64)I * nsp + sp) * N + i) * 4 + l];
        v *= dv;
        C[(i64)(4 * I + l) * N + i] = v;
        s2 += v * v;
      }
    }
    rep[i] += s2;
    e += occ[i] * s2;
  }
  double v[1] = {e};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) rep[enl_off] = v[0];
}

// out[(I * 12 + k) * N + i] = dv * sum over splits of the derivative overlaps
__global__ __launch_bounds__(kBlock) void k_nl_sum_deriv(const double *__restrict__ part, int M,
                                                         int nsp, int N, double dv,
                                                         double *__restrict__ out) {
  const i64 total = (i64)M * 12 * N;
  for (i64 t = (i64)blockIdx.x * kBlock + threadIdx.x; t < total; t += (i64)gridDim.x * kBlock) {
    const int k = (int)(t % 12);
    const i64 r = t / 12;
    const int i = (int)(r % N);
    const int I = (int)(r / N);
    double v = 0.0;
    for (int sp = 0; sp < nsp; ++sp) v += part[(((i64)I * nsp + sp) * N + i) * 12 + k];
    out[((i64)I * 12 + k) * N + i] = v * dv;
  }
}

}  // namespace

int nl_splits(int b) {
  const int vol = b * b * b;
  // about 4096 cube points per workgroup, at most 64 splits
  return std::max(1, std::min(64, (vol + 4095) / 4096));
}

template <typename T>
hipError_t launch_nl_overlap(const T *U, const NlIon *ions, int M, int bmax, int N, int n,
                             double L, bool deriv, double *part, hipStream_t s) {
  const int nsp = nl_splits(bmax);
  if (deriv) {
    dim3 grid(M, (N + 1) / 2, nsp);
    hipLaunchKernelGGL((k_nl_overlap<T, 2, true>), grid, dim3(kBlock), 0, s, U, ions, N, n, L,
                       part);
  } else {
    dim3 grid(M, (N + 7) / 8, nsp);
    hipLaunchKernelGGL((k_nl_overlap<T, 8, false>), grid, dim3(kBlock), 0, s, U, ions, N, n, L,
                       part);
  }
  return hipGetLastError();
}

hipError_t launch_nl_finish(const double *part, int M, int bmax, int N, double dv,
                            const double *occ, double *C, double *rep, int enl_off,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_nl_finish, dim3(1), dim3(kBlock), 0, s, part, M, nl_splits(bmax), N, dv,
                     occ, C, rep, enl_off);
  return hipGetLastError();
}

hipError_t launch_nl_sum_deriv(const double *part, int M, int bmax, int N, double dv,
                               double *out, hipStream_t s) {
  const i64 total = (i64)M * 12 * N;
  const int blocks = (int)std::min<i64>(1024, (total + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_nl_sum_deriv, dim3(std::max(1, blocks)), dim3(kBlock), 0, s, part, M,
                     nl_splits(bmax), N, dv, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_nl_apply(T *HU, const NlIon *ions, const int *list, int count, int bmax,
                           const double *C, int N, int n, double L, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  dim3 grid(count, (N + 3) / 4, nl_splits(bmax));
  hipLaunchKernelGGL((k_nl_apply<T, 4>), grid, dim3(kBlock), 0, s, HU, ions, list, C, N, n, L);
  return hipGetLastError();
}

template hipError_t launch_nl_overlap<double>(const double *, const NlIon *, int, int, int, int,
                                              double, bool, double *, hipStream_t);
template hipError_t launch_nl_overlap<float>(const float *, const NlIon *, int, int, int, int,
                                             double, bool, double *, hipStream_t);
template hipError_t launch_nl_apply<double>(double *, const NlIon *, const int *, int, int,
                                            const double *, int, int, double, hipStream_t);
template hipError_t launch_nl_apply<float>(float *, const NlIon *, const int *, int, int,
                                           const double *, int, int, double, hipStream_t);

}  // namespace pou
