// x passes of the three-pass translation pipeline (Eq. (5)).
//
//   k_fwd_x   zero-padded x-FFT of A:   G[s][d][fx][y][z] = sum_x A[x][y][z] w^{x fx},
//             y < Ky, z < Kz (the x lines of every (y, z) of a box block)
//   k_inv_x   inverse x-FFT, crop to x < Kx and scale by 1/N: B[x][y][z]
//
// Lines along x of a box block are strided by Ky*Kz, so consecutive threads
// take consecutive (y, z) lines: every load and store of a wavefront is one
// contiguous run.  For n1 <= 64 a thread transforms its line in registers
// with the generated codelets; longer lines (128, 256) are split 16 x NB over
// threads through LDS, X[k1 + 16 k2] = sum_j2 w_NB^{j2 k2} w_N1^{j2 k1}
// sum_j1 x[NB j1 + j2] w_16^{j1 k1}, with the FP64-built table twx[m] =
// exp(-2 pi i m / n1).  The y- and z-stages run in the z-stage kernel on the
// G planes of its pencil tile.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "launch.h"

namespace tfmm {

namespace {

template <int NB>
__device__ __forceinline__ void full_fwd_nb(const float2* x, float2* y) {
  if constexpr (NB == 8) dft_full_fwd_8(x, y);
  else dft_full_fwd_16(x, y);
}
template <int NB>
__device__ __forceinline__ void full_inv_nb(const float2* x, float2* y) {
  if constexpr (NB == 8) dft_full_inv_8(x, y);
  else dft_full_inv_16(x, y);
}

constexpr int kLinesSplit = 16;  // lines per block of the split (n1 > 64) kernels

}  // namespace

// n1 <= 64: one line per thread.  grid (ceil(K2 K3 / 256), ndl, nrhs).
template <int N1>
__global__ __launch_bounds__(256) void k_fwd_x(RhsPtrs P, float2* __restrict__ G, int lines, int ndl, int p0,
                                               const int* __restrict__ perm) {
  constexpr int K1 = N1 / 2;
  const int l = blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.z, pl = blockIdx.y;
  if (l >= lines) return;
  const int p = perm ? perm[p0 + pl] : p0 + pl;
  const float2* __restrict__ a = P.a[s] + (long long)p * K1 * lines + l;
  float2* __restrict__ g = G + ((long long)s * ndl + pl) * (long long)N1 * lines + l;
  float2 x[K1], X[N1];
#pragma unroll
  for (int i = 0; i < K1; ++i) x[i] = a[(long long)i * lines];
  Dft<N1>::fwd(x, X);
#pragma unroll
  for (int f = 0; f < N1; ++f) g[(long long)f * lines] = X[f];
}

template <int N1>
__global__ __launch_bounds__(256) void k_inv_x(RhsPtrs P, const float2* __restrict__ G, int lines, int ndl, int p0,
                                               const int* __restrict__ perm, float scale) {
  constexpr int K1 = N1 / 2;
  const int l = blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.z, pl = blockIdx.y;
  if (l >= lines) return;
  const int p = perm ? perm[p0 + pl] : p0 + pl;
  const float2* __restrict__ g = G + ((long long)s * ndl + pl) * (long long)N1 * lines + l;
  float2* __restrict__ b = P.b[s] + (long long)p * K1 * lines + l;
  float2 x[N1], X[K1];
#pragma unroll
  for (int f = 0; f < N1; ++f) x[f] = g[(long long)f * lines];
  Dft<N1>::inv(x, X);
#pragma unroll
  for (int i = 0; i < K1; ++i) b[(long long)i * lines] = cscale(X[i], scale);
}

// n1 = 16 NB (128, 256): 16 lines per block of 256 threads, LDS [x][line].
template <int N1>
__global__ __launch_bounds__(256) void k_fwd_x_split(RhsPtrs P, float2* __restrict__ G, int lines, int ndl, int p0,
                                                     const int* __restrict__ perm, const float2* __restrict__ twx) {
  constexpr int NA = 16, NB = N1 / 16, K1 = N1 / 2, LB = kLinesSplit;
  __shared__ float2 lds[N1 * LB];
  const int s = blockIdx.z, pl = blockIdx.y, l0 = blockIdx.x * LB;
  const int p = perm ? perm[p0 + pl] : p0 + pl;
  const float2* __restrict__ a = P.a[s] + (long long)p * K1 * lines;
  float2* __restrict__ g = G + ((long long)s * ndl + pl) * (long long)N1 * lines;
  // step 1: per (j2, line) the pruned 16-point DFT over j1 (inputs x = NB j1 + j2 < K1), twiddled
  for (int task = threadIdx.x; task < NB * LB; task += 256) {
    const int li = task % LB, j2 = task / LB, l = l0 + li;
    if (l >= lines) continue;
    float2 x[NA / 2], Y[NA];
#pragma unroll
    for (int j1 = 0; j1 < NA / 2; ++j1) x[j1] = a[(long long)(NB * j1 + j2) * lines + l];
    Dft<NA>::fwd(x, Y);
#pragma unroll
    for (int k1 = 0; k1 < NA; ++k1) lds[(k1 + NA * j2) * LB + li] = cmul(Y[k1], twx[j2 * k1]);
  }
  __syncthreads();
  // step 2: per (k1, line) the full NB-point DFT over j2
  for (int task = threadIdx.x; task < NA * LB; task += 256) {
    const int li = task % LB, k1 = task / LB, l = l0 + li;
    if (l >= lines) continue;
    float2 b[NB], X[NB];
#pragma unroll
    for (int j2 = 0; j2 < NB; ++j2) b[j2] = lds[(k1 + NA * j2) * LB + li];
    full_fwd_nb<NB>(b, X);
#pragma unroll
    for (int k2 = 0; k2 < NB; ++k2) g[(long long)(k1 + NA * k2) * lines + l] = X[k2];
  }
}

template <int N1>
__global__ __launch_bounds__(256) void k_inv_x_split(RhsPtrs P, const float2* __restrict__ G, int lines, int ndl,
                                                     int p0, const int* __restrict__ perm, float scale,
                                                     const float2* __restrict__ twx) {
  constexpr int NA = 16, NB = N1 / 16, K1 = N1 / 2, LB = kLinesSplit;
  __shared__ float2 lds[N1 * LB];
  const int s = blockIdx.z, pl = blockIdx.y, l0 = blockIdx.x * LB;
  const int p = perm ? perm[p0 + pl] : p0 + pl;
  const float2* __restrict__ g = G + ((long long)s * ndl + pl) * (long long)N1 * lines;
  float2* __restrict__ b = P.b[s] + (long long)p * K1 * lines;
  // step 1: per (k1, line) the inverse NB-point DFT over k2, untwiddled
  for (int task = threadIdx.x; task < NA * LB; task += 256) {
    const int li = task % LB, k1 = task / LB, l = l0 + li;
    if (l >= lines) continue;
    float2 c[NB], Z[NB];
#pragma unroll
    for (int k2 = 0; k2 < NB; ++k2) c[k2] = g[(long long)(k1 + NA * k2) * lines + l];
    full_inv_nb<NB>(c, Z);
#pragma unroll
    for (int j2 = 0; j2 < NB; ++j2) lds[(k1 + NA * j2) * LB + li] = cmulconj(Z[j2], twx[j2 * k1]);
  }
  __syncthreads();
  // step 2: per (j2, line) the inverse 16-point DFT over k1, outputs j1 < 8 (x = NB j1 + j2 < K1)
  for (int task = threadIdx.x; task < NB * LB; task += 256) {
    const int li = task % LB, j2 = task / LB, l = l0 + li;
    if (l >= lines) continue;
    float2 c[NA], xo[NA / 2];
#pragma unroll
    for (int k1 = 0; k1 < NA; ++k1) c[k1] = lds[(k1 + NA * j2) * LB + li];
    Dft<NA>::inv(c, xo);
#pragma unroll
    for (int j1 = 0; j1 < NA / 2; ++j1) b[(long long)(NB * j1 + j2) * lines + l] = cscale(xo[j1], scale);
  }
}

hipError_t launch_fwd_x(const RhsPtrs& P, float2* G, int n1, int lines, int nrhs, int p0, int ndl, const int* perm,
                        const float2* twx, hipStream_t st, bool* supported) {
  *supported = true;
  const dim3 g1((lines + 255) / 256, ndl, nrhs), gs((lines + kLinesSplit - 1) / kLinesSplit, ndl, nrhs);
  switch (n1) {
#define FX(N)                                                                                \
  case N:                                                                                    \
    hipLaunchKernelGGL(k_fwd_x<N>, g1, dim3(256), 0, st, P, G, lines, ndl, p0, perm);        \
    return hipGetLastError();
    FX(8) FX(16) FX(24) FX(32) FX(48) FX(64)
#undef FX
    case 128:
      hipLaunchKernelGGL(k_fwd_x_split<128>, gs, dim3(256), 0, st, P, G, lines, ndl, p0, perm, twx);
      return hipGetLastError();
    case 256:
      hipLaunchKernelGGL(k_fwd_x_split<256>, gs, dim3(256), 0, st, P, G, lines, ndl, p0, perm, twx);
      return hipGetLastError();
  }
  *supported = false;
  return hipSuccess;
}

hipError_t launch_inv_x(const RhsPtrs& P, const float2* G, int n1, int lines, int nrhs, int p0, int ndl,
                        const int* perm, float scale, const float2* twx, hipStream_t st, bool* supported) {
  *supported = true;
  const dim3 g1((lines + 255) / 256, ndl, nrhs), gs((lines + kLinesSplit - 1) / kLinesSplit, ndl, nrhs);
  switch (n1) {
#define IX(N)                                                                                     \
  case N:                                                                                         \
    hipLaunchKernelGGL(k_inv_x<N>, g1, dim3(256), 0, st, P, G, lines, ndl, p0, perm, scale);      \
    return hipGetLastError();
    IX(8) IX(16) IX(24) IX(32) IX(48) IX(64)
#undef IX
    case 128:
      hipLaunchKernelGGL(k_inv_x_split<128>, gs, dim3(256), 0, st, P, G, lines, ndl, p0, perm, scale, twx);
      return hipGetLastError();
    case 256:
      hipLaunchKernelGGL(k_inv_x_split<256>, gs, dim3(256), 0, st, P, G, lines, ndl, p0, perm, scale, twx);
      return hipGetLastError();
  }
  *supported = false;
  return hipSuccess;
}

}  // namespace tfmm
