// Setup kernels of the device-side FP64 compression: layout permutations of
// the FFT'ed operator tensor (complex128).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"

namespace tfmm {

// out[c][r] = in[r][c] for a rows x cols matrix (32 x 32 tiles through LDS).
__global__ void k_transpose64(const double2* __restrict__ in, double2* __restrict__ out, long long rows,
                              long long cols) {
  __shared__ double2 tile[32][33];
  const long long c0 = (long long)blockIdx.x * 32, r0 = (long long)blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int j = ty; j < 32; j += 8) {
    const long long r = r0 + j, c = c0 + tx;
    if (r < rows && c < cols) tile[j][tx] = in[r * cols + c];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const long long c = c0 + j, r = r0 + tx;
    if (c < cols && r < rows) out[c * rows + r] = tile[tx][j];
  }
}

hipError_t launch_transpose64(const double2* in, double2* out, long long rows, long long cols, hipStream_t st) {
  const long long gx = (cols + 31) / 32, gy = (rows + 31) / 32;
  if (gy > 65535 || gx > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_transpose64, dim3((unsigned)gx, (unsigned)gy), dim3(32, 8), 0, st, in, out, rows, cols);
  return hipGetLastError();
}

// [P][D][Q] <-> [D][P][Q]: to_first: out[(a P + p) Q + c] = in[(p D + a) Q + c];
// else the inverse.  One thread per output element.
__global__ void k_perm_mode(const double2* __restrict__ in, double2* __restrict__ out, long long P, long long D,
                            long long Q, int to_first) {
  const long long total = P * D * Q;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long c = i % Q;
    const long long t = i / Q;
    long long src;
    if (to_first) {  // i indexes [a][p][c]
      const long long p = t % P, a = t / P;
      src = (p * D + a) * Q + c;
    } else {  // i indexes [p][a][c], source [a][p][c]
      const long long a = t % D, p = t / D;
      src = (a * P + p) * Q + c;
    }
    out[i] = in[src];
  }
}

hipError_t launch_perm_mode(const double2* in, double2* out, long long P, long long D, long long Q, bool to_first,
                            hipStream_t st) {
  const long long total = P * D * Q;
  const long long blocks = std::min<long long>((total + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(k_perm_mode, dim3((unsigned)std::max<long long>(blocks, 1)), dim3(256), 0, st, in, out, P, D,
                     Q, to_first ? 1 : 0);
  return hipGetLastError();
}

}  // namespace tfmm
