// xy-FFT stages shared by the three-pass pipeline and the fused kernel.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace tfmm {

// ---------------------------------------------------------------------------
// xy stages on a slab of zg z-planes held in LDS as [fx][y][z] with padded z
// stride zp (odd), i.e. element (q = fx*N2 + y, z) at q*zp + z.  Lines along x
// and y are processed one per thread with the generated codelets; the odd
// stride keeps both the line accesses and pencil-wise accesses conflict free.
//
// x lines longer than 64 points (N1 = 16*NB, NB = 8 or 16) are split over
// threads: with j = NB*j1 + j2 and k = k1 + 16*k2,
//   X[k1 + 16 k2] = sum_j2 w_NB^{j2 k2} w_N1^{j2 k1} sum_j1 x[NB j1 + j2] w_16^{j1 k1},
// i.e. pruned 16-point DFTs per j2, a twiddle from the FP64-built table
// twx[m] = exp(-2 pi i m / N1), then full NB-point DFTs per k1.  The
// intermediate of (k1, j2) is kept at x position k1 + 16*j2, so each step
// reads and writes the same positions.  The inverse runs the steps backwards.
// ---------------------------------------------------------------------------
template <int NB>
__device__ __forceinline__ void dft_full_fwd_nb(const float2* x, float2* y) {
  if constexpr (NB == 8) dft_full_fwd_8(x, y);
  else dft_full_fwd_16(x, y);
}
template <int NB>
__device__ __forceinline__ void dft_full_inv_nb(const float2* x, float2* y) {
  if constexpr (NB == 8) dft_full_inv_8(x, y);
  else dft_full_inv_16(x, y);
}

// Element (x, y, z) of a box block: caller layout [x][y][z] (z fastest), or,
// with zm set, z-major [z][x][y] (the three-pass pipeline's staged copy, so a
// block's z-slab is contiguous).
template <int K1, int K2>
__device__ __forceinline__ long long box_at(int x, int y, int z, int K3, bool zm) {
  return zm ? ((long long)z * K1 + x) * K2 + y : ((long long)x * K2 + y) * K3 + z;
}

template <int N1, int N2, int NT>
__device__ __forceinline__ void xy_forward(float2* lds, const float2* __restrict__ Ab, int K3, int zg, int zp,
                                           int z0, const float2* __restrict__ twx, bool zm = false) {
  constexpr int K1 = N1 / 2, K2 = N2 / 2;
  if constexpr (N1 <= 64) {
    for (int task = threadIdx.x; task < K2 * zg; task += NT) {
      const int z = task % zg, y = task / zg;
      float2 x[K1], X[N1];
#pragma unroll
      for (int i = 0; i < K1; ++i) x[i] = Ab[box_at<K1, K2>(i, y, z0 + z, K3, zm)];
      Dft<N1>::fwd(x, X);
#pragma unroll
      for (int f = 0; f < N1; ++f) lds[(f * N2 + y) * zp + z] = X[f];
    }
  } else {
    constexpr int NA = 16, NB = N1 / 16;
    for (int task = threadIdx.x; task < NB * K2 * zg; task += NT) {
      const int z = task % zg, r = task / zg, y = r % K2, j2 = r / K2;
      float2 a[NA / 2], Y[NA];
#pragma unroll
      for (int j1 = 0; j1 < NA / 2; ++j1) a[j1] = Ab[box_at<K1, K2>(NB * j1 + j2, y, z0 + z, K3, zm)];
      Dft<NA>::fwd(a, Y);
#pragma unroll
      for (int k1 = 0; k1 < NA; ++k1) lds[((k1 + NA * j2) * N2 + y) * zp + z] = cmul(Y[k1], twx[j2 * k1]);
    }
    __syncthreads();
    for (int task = threadIdx.x; task < NA * K2 * zg; task += NT) {
      const int z = task % zg, r = task / zg, y = r % K2, k1 = r / K2;
      float2 b[NB], X[NB];
#pragma unroll
      for (int j2 = 0; j2 < NB; ++j2) b[j2] = lds[((k1 + NA * j2) * N2 + y) * zp + z];
      dft_full_fwd_nb<NB>(b, X);
#pragma unroll
      for (int k2 = 0; k2 < NB; ++k2) lds[((k1 + NA * k2) * N2 + y) * zp + z] = X[k2];
    }
  }
  __syncthreads();
  for (int task = threadIdx.x; task < N1 * zg; task += NT) {
    const int z = task % zg, fx = task / zg;
    float2 y[K2], Y[N2];
#pragma unroll
    for (int i = 0; i < K2; ++i) y[i] = lds[(fx * N2 + i) * zp + z];
    Dft<N2>::fwd(y, Y);
#pragma unroll
    for (int f = 0; f < N2; ++f) lds[(fx * N2 + f) * zp + z] = Y[f];
  }
}

template <int N1, int N2, int NT>
__device__ __forceinline__ void xy_inverse(float2* lds, float2* __restrict__ Bb, int K3, int zg, int zp, int z0,
                                           float scale, const float2* __restrict__ twx, bool zm = false) {
  constexpr int K1 = N1 / 2, K2 = N2 / 2;
  for (int task = threadIdx.x; task < N1 * zg; task += NT) {
    const int z = task % zg, fx = task / zg;
    float2 y[N2], Y[K2];
#pragma unroll
    for (int i = 0; i < N2; ++i) y[i] = lds[(fx * N2 + i) * zp + z];
    Dft<N2>::inv(y, Y);
#pragma unroll
    for (int f = 0; f < K2; ++f) lds[(fx * N2 + f) * zp + z] = Y[f];
  }
  __syncthreads();
  if constexpr (N1 <= 64) {
    for (int task = threadIdx.x; task < K2 * zg; task += NT) {
      const int z = task % zg, y = task / zg;
      float2 x[N1], X[K1];
#pragma unroll
      for (int i = 0; i < N1; ++i) x[i] = lds[(i * N2 + y) * zp + z];
      Dft<N1>::inv(x, X);
#pragma unroll
      for (int i = 0; i < K1; ++i) Bb[box_at<K1, K2>(i, y, z0 + z, K3, zm)] = cscale(X[i], scale);
    }
  } else {
    constexpr int NA = 16, NB = N1 / 16;
    for (int task = threadIdx.x; task < NA * K2 * zg; task += NT) {
      const int z = task % zg, r = task / zg, y = r % K2, k1 = r / K2;
      float2 b[NB], Z[NB];
#pragma unroll
      for (int k2 = 0; k2 < NB; ++k2) b[k2] = lds[((k1 + NA * k2) * N2 + y) * zp + z];
      dft_full_inv_nb<NB>(b, Z);
#pragma unroll
      for (int j2 = 0; j2 < NB; ++j2) lds[((k1 + NA * j2) * N2 + y) * zp + z] = cmulconj(Z[j2], twx[j2 * k1]);
    }
    __syncthreads();
    for (int task = threadIdx.x; task < NB * K2 * zg; task += NT) {
      const int z = task % zg, r = task / zg, y = r % K2, j2 = r / K2;
      float2 c[NA], xo[NA / 2];
#pragma unroll
      for (int k1 = 0; k1 < NA; ++k1) c[k1] = lds[((k1 + NA * j2) * N2 + y) * zp + z];
      Dft<NA>::inv(c, xo);
#pragma unroll
      for (int j1 = 0; j1 < NA / 2; ++j1)
        Bb[box_at<K1, K2>(NB * j1 + j2, y, z0 + z, K3, zm)] = cscale(xo[j1], scale);
    }
  }
}

}  // namespace tfmm
