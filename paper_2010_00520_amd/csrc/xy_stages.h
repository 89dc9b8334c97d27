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
// ---------------------------------------------------------------------------
template <int N1, int N2, int NT>
__device__ __forceinline__ void xy_forward(float2* lds, const float2* __restrict__ Ab, int K3, int zg, int zp,
                                           int z0) {
  constexpr int K1 = N1 / 2, K2 = N2 / 2;
  for (int task = threadIdx.x; task < K2 * zg; task += NT) {
    const int z = task % zg, y = task / zg;
    float2 x[K1], X[N1];
#pragma unroll
    for (int i = 0; i < K1; ++i) x[i] = Ab[((long long)i * K2 + y) * K3 + z0 + z];
    Dft<N1>::fwd(x, X);
#pragma unroll
    for (int f = 0; f < N1; ++f) lds[(f * N2 + y) * zp + z] = X[f];
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
                                           float scale) {
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
  for (int task = threadIdx.x; task < K2 * zg; task += NT) {
    const int z = task % zg, y = task / zg;
    float2 x[N1], X[K1];
#pragma unroll
    for (int i = 0; i < N1; ++i) x[i] = lds[(i * N2 + y) * zp + z];
    Dft<N1>::inv(x, X);
#pragma unroll
    for (int i = 0; i < K1; ++i) Bb[((long long)i * K2 + y) * K3 + z0 + z] = cscale(X[i], scale);
  }
}

}  // namespace tfmm
