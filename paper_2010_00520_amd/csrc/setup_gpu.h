// Device-side FP64 setup of the FFT'ed operator: 3-D FFT and the compression
// of the 4-D formats (setup_gpu.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "host_math.h"

namespace tfmm {

// In-place forward 3-D DFT (unnormalised, exp(-2 pi i m k / n)) of `batch`
// contiguous n1 x n2 x n3 complex128 blocks on the device.  Empty string on
// success.
std::string fft3d_forward_device(double2* T, const int n[3], int batch, hipStream_t st);

// Compress the FFT'ed operator T~[p][x][y][z] (device, complex128, n_dir blocks;
// left unchanged) in a 4-D format (fmt 3 Tucker-4D, 4 TT-4D, 5 H-Tucker-4D) on
// the device; the factors come back to `out` in the tfmm_op_import layout.
// Same truncation rule as compress_operator.  Empty string on success.
std::string compress_4d_device(double2* T, int ndir, const int n[3], int fmt, double gamma, Factors& out,
                               int nthreads, hipStream_t st);

}  // namespace tfmm
