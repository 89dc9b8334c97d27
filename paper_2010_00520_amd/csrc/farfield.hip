// The steps either side of the translation (Section II-A): far-field
// patterns of the basis functions (Eq. (3), FP64 setup), aggregation into box
// radiation patterns (Eq. (4)) and projection of the translated spectra back
// onto the basis functions with the direction quadrature (Eq. (6)).
//
// Basis functions are point dipoles (position r_n, unit orientation u_n), kept
// sorted by box: box v owns the sorted range [start[v], start[v+1]).  The
// pattern table holds, per (direction p, sorted basis n), the float4
//   (theta_p . u_n, phi_p . u_n, Re e, Im e),  e = exp(+jk k_p . (r_n - r_v)),
// so P+_c = g_c e and the receive pattern P-_c = g_c / e (= g_c conj(e) for a
// real k, the conjugate Eq. (6) names).  Both kernels are bound by streaming
// the table: consecutive threads read consecutive basis functions of one
// direction.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace tfmm {

__global__ void k_dipole_patterns(float4* __restrict__ pat, const double* __restrict__ khat,
                                  const double* __restrict__ geo, int N, double kre, double kim) {
  // geo[n] = (r_n - r_v (3), u_n (3)) in sorted order
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (n >= N) return;
  const double kx = khat[3 * p], ky = khat[3 * p + 1], kz = khat[3 * p + 2];
  const double th = acos(fmin(1.0, fmax(-1.0, kz))), ph = atan2(ky, kx);
  double st, ct, sp, cp;
  sincos(th, &st, &ct);
  sincos(ph, &sp, &cp);
  const double* g = geo + 6 * (size_t)n;
  const double gt = ct * cp * g[3] + ct * sp * g[4] - st * g[5];  // theta_p . u_n
  const double gp = -sp * g[3] + cp * g[4];                        // phi_p . u_n
  const double x = kx * g[0] + ky * g[1] + kz * g[2];              // k_p . (r_n - r_v)
  // exp(j k x) with k = kre + j kim: e^{-kim x} (cos kre x + j sin kre x)
  double s, c;
  sincos(kre * x, &s, &c);
  const double a = exp(-kim * x);
  pat[(size_t)p * N + n] = make_float4((float)gt, (float)gp, (float)(a * c), (float)(a * s));
}

hipError_t launch_dipole_patterns(float4* pat, const double* khat, const double* geo, int N, int ndir, double kre,
                                  double kim, hipStream_t st) {
  dim3 grid((N + 255) / 256, ndir);
  hipLaunchKernelGGL(k_dipole_patterns, grid, dim3(256), 0, st, pat, khat, geo, N, kre, kim);
  return hipGetLastError();
}

// Eq. (4): A[2r + c][p][v] = sum_{n in B_v} g_c e I_r[orig(n)], one thread per
// (box, direction); empty boxes get zero.
__global__ void k_aggregate(const float4* __restrict__ pat, const int* __restrict__ start,
                            const int* __restrict__ orig, const float2* __restrict__ I, float2* __restrict__ A, int N,
                            int nbox, int ndir, int nrhs) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (v >= nbox) return;
  const int b = start[v], e = start[v + 1];
  const float4* row = pat + (size_t)p * N;
  for (int r = 0; r < nrhs; ++r) {
    float tr = 0.f, ti = 0.f, fr = 0.f, fi = 0.f;
    const float2* Ir = I + (size_t)r * N;
    for (int n = b; n < e; ++n) {
      const float4 q = row[n];
      const float2 cur = Ir[orig[n]];
      // e * I
      const float er = q.z * cur.x - q.w * cur.y, ei = q.z * cur.y + q.w * cur.x;
      tr += q.x * er;
      ti += q.x * ei;
      fr += q.y * er;
      fi += q.y * ei;
    }
    A[((size_t)(2 * r) * ndir + p) * nbox + v] = make_float2(tr, ti);
    A[((size_t)(2 * r + 1) * ndir + p) * nbox + v] = make_float2(fr, fi);
  }
}

hipError_t launch_aggregate(const float4* pat, const int* start, const int* orig, const float2* I, float2* A, int N,
                            int nbox, int ndir, int nrhs, hipStream_t st) {
  dim3 grid((nbox + 255) / 256, ndir);
  hipLaunchKernelGGL(k_aggregate, grid, dim3(256), 0, st, pat, start, orig, I, A, N, nbox, ndir, nrhs);
  return hipGetLastError();
}

// Eq. (6): y_r[orig(n)] = sum_p w_p sum_c (g_c / e) B[2r + c][p][box(n)], one
// thread per sorted basis function, RHS in groups of RG sharing each table read.
template <int RG>
__global__ void k_disaggregate(const float4* __restrict__ pat, const int* __restrict__ boxof,
                               const int* __restrict__ orig, const float* __restrict__ w, const float2* __restrict__ B,
                               float2* __restrict__ y, int N, int nbox, int ndir, int r0, int nr) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int v = boxof[n];
  float ar[RG], ai[RG];
#pragma unroll
  for (int i = 0; i < RG; ++i) ar[i] = ai[i] = 0.f;
  for (int p = 0; p < ndir; ++p) {
    const float4 q = pat[(size_t)p * N + n];
    // w_p / e = w_p conj(e) / |e|^2
    const float s = w[p] / (q.z * q.z + q.w * q.w);
    const float er = q.z * s, ei = -q.w * s;
#pragma unroll
    for (int i = 0; i < RG; ++i) {
      if (i < nr) {
        const int r = r0 + i;
        const float2 bt = B[((size_t)(2 * r) * ndir + p) * nbox + v];
        const float2 bf = B[((size_t)(2 * r + 1) * ndir + p) * nbox + v];
        const float sr = q.x * bt.x + q.y * bf.x, si = q.x * bt.y + q.y * bf.y;
        ar[i] += er * sr - ei * si;
        ai[i] += er * si + ei * sr;
      }
    }
  }
  const int m = orig[n];
#pragma unroll
  for (int i = 0; i < RG; ++i)
    if (i < nr) y[(size_t)(r0 + i) * N + m] = make_float2(ar[i], ai[i]);
}

hipError_t launch_disaggregate(const float4* pat, const int* boxof, const int* orig, const float* w, const float2* B,
                               float2* y, int N, int nbox, int ndir, int nrhs, hipStream_t st) {
  constexpr int RG = 4;
  for (int r0 = 0; r0 < nrhs; r0 += RG) {
    hipLaunchKernelGGL(k_disaggregate<RG>, dim3((N + 255) / 256), dim3(256), 0, st, pat, boxof, orig, w, B, y, N,
                       nbox, ndir, r0, std::min(RG, nrhs - r0));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tfmm

namespace tfmm {

// Near-field matrix product y_r = Zn x_r (CSR, complex64), one wavefront per
// row: lanes stride over the row's entries, then a butterfly sum.
__global__ void k_near_spmv(const int* __restrict__ rp, const int* __restrict__ ci, const float2* __restrict__ val,
                            const float2* __restrict__ x, float2* __restrict__ y, int n, int nrhs) {
  const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (row >= n) return;
  const int b = rp[row], e = rp[row + 1];
  for (int r = 0; r < nrhs; ++r) {
    const float2* xr = x + (size_t)r * n;
    float sr = 0.f, si = 0.f;
    for (int j = b + l; j < e; j += 64) {
      const float2 a = val[j], v = xr[ci[j]];
      sr += a.x * v.x - a.y * v.y;
      si += a.x * v.y + a.y * v.x;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      sr += __shfl_xor(sr, m);
      si += __shfl_xor(si, m);
    }
    if (l == 0) y[(size_t)r * n + row] = make_float2(sr, si);
  }
}

hipError_t launch_near_spmv(const int* rp, const int* ci, const float2* val, const float2* x, float2* y, int n,
                            int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_near_spmv, dim3((n + 3) / 4), dim3(256), 0, st, rp, ci, val, x, y, n, nrhs);
  return hipGetLastError();
}

__global__ void k_narrow128(const double2* __restrict__ a, float2* __restrict__ b, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}
__global__ void k_widen(const float2* __restrict__ a, double2* __restrict__ b, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_double2(a[i].x, a[i].y);
}
__global__ void k_sum_widen(const float2* __restrict__ a, const float2* __restrict__ c, double2* __restrict__ b,
                            int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_double2((double)a[i].x + (double)c[i].x, (double)a[i].y + (double)c[i].y);
}

hipError_t launch_narrow128(const double2* a, float2* b, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_narrow128, dim3((n + 255) / 256), dim3(256), 0, st, a, b, n);
  return hipGetLastError();
}
hipError_t launch_widen(const float2* a, double2* b, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_widen, dim3((n + 255) / 256), dim3(256), 0, st, a, b, n);
  return hipGetLastError();
}
hipError_t launch_sum_widen(const float2* a, const float2* c, double2* b, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_widen, dim3((n + 255) / 256), dim3(256), 0, st, a, c, b, n);
  return hipGetLastError();
}

}  // namespace tfmm
