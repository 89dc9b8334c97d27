// Device-side building blocks shared by the translation kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dft_codelets.h"

typedef float v4f __attribute__((ext_vector_type(4)));

#define TFMM_WAVE 64
#define TFMM_BLOCK 256
#define TFMM_NWAVES (TFMM_BLOCK / TFMM_WAVE)

// complex helpers not in the codelet header
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cmulconj(float2 a, float2 b) {  // a * conj(b)
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// An operand of a complex GEMM held in LDS: element (i, j) of batch `bat`
// lives at off + i*s0 + j*s1 + bat*sb (float2 units).
struct LOp {
  int off, s0, s1, sb;
};

// Block-cooperative batched complex GEMM on the matrix cores, operands and
// result in LDS:  C_b[m][n] = sum_k A_b[m][k] B_b[k][n]  for b < nb.
// The complex product is embedded in real arithmetic: a 16 x 16 real output
// tile covers 8 complex rows (re/im interleaved) x 16 complex columns, the
// real K index is (k, re/im) so one 16x16x4 MFMA step consumes 2 complex k.
// Every wave walks its share of the tiles; all lanes take part in each MFMA.
template <int NW>
__device__ __forceinline__ void block_cgemm(float2* lds, int M, int N, int K, int nb, LOp A, LOp B, LOp C) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int tmN = (M + 7) >> 3, tnN = (N + 15) >> 4;
  const int per = tmN * tnN, ntiles = nb * per;
  const int ks = (K + 1) >> 1;
  const int kofs = (l >> 4) >> 1, ki = (l >> 4) & 1, ari = l & 1;
  for (int tile = w; tile < ntiles; tile += NW) {
    const int bat = tile / per, rem = tile - bat * per;
    const int tm = rem / tnN, tn = rem - tm * tnN;
    const int am = tm * 8 + ((l & 15) >> 1);
    const int bn = tn * 16 + (l & 15);
    const bool aok = am < M, bok = bn < N;
    const float2* ap = lds + A.off + am * A.s0 + bat * A.sb;
    const float2* bp = lds + B.off + bn * B.s1 + bat * B.sb;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < ks; ++s) {
      const int k = 2 * s + kofs;
      float a = 0.f, b = 0.f;
      if (aok && k < K) {
        const float2 v = ap[k * A.s1];
        a = ari == 0 ? (ki == 0 ? v.x : -v.y) : (ki == 0 ? v.y : v.x);
      }
      if (bok && k < K) {
        const float2 v = bp[k * B.s0];
        b = ki == 0 ? v.x : v.y;
      }
      acc = mfma4(a, b, acc);
    }
    const int cn = tn * 16 + (l & 15), cm0 = tm * 8 + 2 * (l >> 4);
    if (cn < N) {
      float2* cp = lds + C.off + cn * C.s1 + bat * C.sb;
      if (cm0 < M) cp[cm0 * C.s0] = make_float2(acc[0], acc[1]);
      if (cm0 + 1 < M) cp[(cm0 + 1) * C.s0] = make_float2(acc[2], acc[3]);
    }
  }
}
