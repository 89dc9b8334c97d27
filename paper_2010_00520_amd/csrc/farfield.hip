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

// Eq. (4): A[2r + c][p][v] = sum_{n in B_v} g_c e I_r[orig(n)].  One wavefront
// per (box v, group of kAggPG directions): its lanes stride over the box's
// sorted range, so each table row is read as one contiguous run, the group's
// rows are in flight together, and a butterfly sum per (direction, component)
// leaves the box total in every lane.  Consecutive waves of a block take the
// direction groups of one box (its currents stay in cache).  An empty box's
// wave writes its zeros.
constexpr int kAggPG = 8;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

__global__ __launch_bounds__(256) void k_aggregate(const float4* __restrict__ pat, const int* __restrict__ start,
                                                   const int* __restrict__ orig, const float2* __restrict__ I,
                                                   float2* __restrict__ A, int N, int nbox, int ndir, int nrhs,
                                                   int npg) {
  const int l = threadIdx.x & 63;
  const long long item = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= (long long)nbox * npg) return;
  const int v = (int)(item / npg), p0 = (int)(item - (long long)v * npg) * kAggPG;
  const int b = start[v], e = start[v + 1];
  if (b == e) {
    for (int t = l; t < kAggPG * 2 * nrhs; t += 64) {
      const int k = t % kAggPG, rc = t / kAggPG;
      if (p0 + k < ndir) A[((size_t)rc * ndir + p0 + k) * nbox + v] = make_float2(0.f, 0.f);
    }
    return;
  }
  for (int r = 0; r < nrhs; ++r) {
    const float2* Ir = I + (size_t)r * N;
    float tr[kAggPG], ti[kAggPG], fr[kAggPG], fi[kAggPG];
#pragma unroll
    for (int k = 0; k < kAggPG; ++k) tr[k] = ti[k] = fr[k] = fi[k] = 0.f;
    for (int n = b + l; n < e; n += 64) {
      const float2 cur = Ir[orig[n]];
      float4 q[kAggPG];
#pragma unroll
      for (int k = 0; k < kAggPG; ++k)
        q[k] = p0 + k < ndir ? pat[(size_t)(p0 + k) * N + n] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int k = 0; k < kAggPG; ++k) {
        // e * I, then the theta and phi components
        const float er = q[k].z * cur.x - q[k].w * cur.y, ei = q[k].z * cur.y + q[k].w * cur.x;
        tr[k] += q[k].x * er;
        ti[k] += q[k].x * ei;
        fr[k] += q[k].y * er;
        fi[k] += q[k].y * ei;
      }
    }
#pragma unroll
    for (int k = 0; k < kAggPG; ++k) {
      const float a0 = wave_sum(tr[k]), a1 = wave_sum(ti[k]), a2 = wave_sum(fr[k]), a3 = wave_sum(fi[k]);
      if (l == 0 && p0 + k < ndir) {
        A[((size_t)(2 * r) * ndir + p0 + k) * nbox + v] = make_float2(a0, a1);
        A[((size_t)(2 * r + 1) * ndir + p0 + k) * nbox + v] = make_float2(a2, a3);
      }
    }
  }
}

hipError_t launch_aggregate(const float4* pat, const int* start, const int* orig, const float2* I, float2* A, int N,
                            int nbox, int ndir, int nrhs, hipStream_t st) {
  const int npg = (ndir + kAggPG - 1) / kAggPG;
  const long long waves = (long long)nbox * npg;
  hipLaunchKernelGGL(k_aggregate, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, pat, start, orig, I, A, N,
                     nbox, ndir, nrhs, npg);
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
  // directions in groups of DG: the group's table loads are in flight together
  constexpr int DG = 4;
  for (int p0 = 0; p0 < ndir; p0 += DG) {
    float4 q[DG];
#pragma unroll
    for (int k = 0; k < DG; ++k)
      q[k] = p0 + k < ndir ? pat[(size_t)(p0 + k) * N + n] : make_float4(0.f, 0.f, 1.f, 0.f);
#pragma unroll
    for (int k = 0; k < DG; ++k) {
      const int p = p0 + k;
      if (p >= ndir) break;
      // w_p / e = w_p conj(e) / |e|^2
      const float s = w[p] / (q[k].z * q[k].z + q[k].w * q[k].w);
      const float er = q[k].z * s, ei = -q[k].w * s;
#pragma unroll
      for (int i = 0; i < RG; ++i) {
        if (i < nr) {
          const int r = r0 + i;
          const float2 bt = B[((size_t)(2 * r) * ndir + p) * nbox + v];
          const float2 bf = B[((size_t)(2 * r + 1) * ndir + p) * nbox + v];
          const float sr = q[k].x * bt.x + q[k].y * bf.x, si = q[k].x * bt.y + q[k].y * bf.y;
          ar[i] += er * sr - ei * si;
          ai[i] += er * si + ei * sr;
        }
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
