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
// Every wave walks its share of the work in units of one 8-row x 32-column
// block (two output tiles sharing the A fragment); the K loop is unrolled by
// four with all operand loads issued before the MFMAs that consume them.
__device__ __forceinline__ float embed_a(float2 v, int ri, int ki) {
  // real embedding of a complex A entry: [[re, -im], [im, re]]
  return ri == 0 ? (ki == 0 ? v.x : -v.y) : (ki == 0 ? v.y : v.x);
}

template <int NW>
__device__ __forceinline__ void block_cgemm(float2* lds, int M, int N, int K, int nb, LOp A, LOp B, LOp C) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int tmN = (M + 7) >> 3, tpN = (N + 31) >> 5;
  const int per = tmN * tpN, ntiles = nb * per;
  const int ks = (K + 1) >> 1;
  const int kofs = (l >> 4) >> 1, ki = (l >> 4) & 1, ari = l & 1;
  for (int tile = w; tile < ntiles; tile += NW) {
    const int bat = tile / per, rem = tile - bat * per;
    const int tm = rem / tpN, tp = rem - tm * tpN;
    const int am = tm * 8 + ((l & 15) >> 1);
    const int bn0 = tp * 32 + (l & 15), bn1 = bn0 + 16;
    const bool aok = am < M, b0ok = bn0 < N, b1ok = bn1 < N;
    const float2* ap = lds + A.off + (aok ? am : 0) * A.s0 + bat * A.sb;
    const float2* bp0 = lds + B.off + (b0ok ? bn0 : 0) * B.s1 + bat * B.sb;
    const float2* bp1 = lds + B.off + (b1ok ? bn1 : 0) * B.s1 + bat * B.sb;
    v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    int s = 0;
    for (; s + 4 <= ks; s += 4) {
      float ar[4], ai[4], b0r[4], b0i[4], b1r[4], b1i[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = 2 * (s + u) + kofs;
        const bool kok = k < K;
        const float2 va = (aok && kok) ? ap[k * A.s1] : make_float2(0.f, 0.f);
        const float2 vb0 = (b0ok && kok) ? bp0[k * B.s0] : make_float2(0.f, 0.f);
        const float2 vb1 = (b1ok && kok) ? bp1[k * B.s0] : make_float2(0.f, 0.f);
        ar[u] = va.x; ai[u] = va.y;
        b0r[u] = vb0.x; b0i[u] = vb0.y;
        b1r[u] = vb1.x; b1i[u] = vb1.y;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float a = embed_a(make_float2(ar[u], ai[u]), ari, ki);
        acc0 = mfma4(a, ki == 0 ? b0r[u] : b0i[u], acc0);
        acc1 = mfma4(a, ki == 0 ? b1r[u] : b1i[u], acc1);
      }
    }
    for (; s < ks; ++s) {
      const int k = 2 * s + kofs;
      const bool kok = k < K;
      const float2 va = (aok && kok) ? ap[k * A.s1] : make_float2(0.f, 0.f);
      const float2 vb0 = (b0ok && kok) ? bp0[k * B.s0] : make_float2(0.f, 0.f);
      const float2 vb1 = (b1ok && kok) ? bp1[k * B.s0] : make_float2(0.f, 0.f);
      const float a = embed_a(va, ari, ki);
      acc0 = mfma4(a, ki == 0 ? vb0.x : vb0.y, acc0);
      acc1 = mfma4(a, ki == 0 ? vb1.x : vb1.y, acc1);
    }
    const int cm0 = tm * 8 + 2 * (l >> 4);
    float2* cb = lds + C.off + bat * C.sb;
    if (b0ok) {
      if (cm0 < M) cb[cm0 * C.s0 + bn0 * C.s1] = make_float2(acc0[0], acc0[1]);
      if (cm0 + 1 < M) cb[(cm0 + 1) * C.s0 + bn0 * C.s1] = make_float2(acc0[2], acc0[3]);
    }
    if (b1ok) {
      if (cm0 < M) cb[cm0 * C.s0 + bn1 * C.s1] = make_float2(acc1[0], acc1[1]);
      if (cm0 + 1 < M) cb[(cm0 + 1) * C.s0 + bn1 * C.s1] = make_float2(acc1[2], acc1[3]);
    }
  }
}

// ---------------------------------------------------------------------------
// Split-BF16 (bf16x3) arithmetic.  A complex FP32 value v is stored as two
// dwords: hi = (bf16(v.x), bf16(v.y)) and lo = (bf16(v.x - hi.x),
// bf16(v.y - hi.y)), round to nearest even, so an operand occupies the same
// 8 bytes as complex64.  Products use hi*hi + hi*lo + lo*hi with FP32
// accumulation; the dropped lo*lo term and the split itself leave a relative
// error of a few 2^-18 per product.
// ---------------------------------------------------------------------------
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

typedef float v2f_t __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf_t __attribute__((ext_vector_type(2)));

// Two floats to packed bf16 (round to nearest even): one v_cvt_pk_bf16_f32.
__device__ __forceinline__ unsigned cvt_pk_bf16(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((v2f_t{a, b}), v2bf_t));
}

__device__ __forceinline__ uint2 split_bf3(float2 v) {
  const unsigned h = cvt_pk_bf16(v.x, v.y);
  const float rl = v.x - __uint_as_float(h << 16), il = v.y - __uint_as_float(h & 0xFFFF0000u);
  return make_uint2(h, cvt_pk_bf16(rl, il));
}

// Store of a staged operand value: complex64 as is, or split into bf16 hi/lo.
template <bool BF>
__device__ __forceinline__ void stage(float2* lds, int i, float2 v) {
  if constexpr (BF)
    reinterpret_cast<uint2*>(lds)[i] = split_bf3(v);
  else
    lds[i] = v;
}

__device__ __forceinline__ v4f mfma_bf16(v4u a, v4u b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0,
                                                 0, 0);
}

// Real embedding of a packed (re, im) bf16 dword for the A operand:
// row ri = 0 takes (re, -im), row ri = 1 takes (im, re).
// Branch-free (a select here is compiled into divergent branches that wait
// for each LDS load separately): rotate by 16 ri, then flip the sign bit
// when ri == 0.
__device__ __forceinline__ unsigned embed_a_bf(unsigned d, int ri) {
  return __builtin_amdgcn_alignbit(d, d, (unsigned)ri << 4) ^ ((unsigned)(ri ^ 1) << 31);
}

// acc += A' B' for one 16x16x32 bf16 K-step in split arithmetic.
__device__ __forceinline__ v4f mfma_bf3(v4u ahi, v4u alo, v4u bhi, v4u blo, v4f acc) {
  acc = mfma_bf16(ahi, bhi, acc);
  acc = mfma_bf16(ahi, blo, acc);
  acc = mfma_bf16(alo, bhi, acc);
  return acc;
}

// Block-cooperative batched complex GEMM, split-BF16 operands and result in
// LDS (uint2 per complex, see split_bf3).  Same tiling as block_cgemm: a wave
// computes an 8-row x 32-column block; one 16x16x32 bf16 step consumes 16
// complex k (lane group kg = l/16 supplies k0 + 4kg .. k0 + 4kg + 3).
template <int NW>
__device__ __forceinline__ void block_cgemm_bf3(uint2* lds, int M, int N, int K, int nb, LOp A, LOp B, LOp C) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int tmN = (M + 7) >> 3, tpN = (N + 31) >> 5;
  const int per = tmN * tpN, ntiles = nb * per;
  const int ks = (K + 15) >> 4;
  const int kg = l >> 4, ri = l & 1;
  for (int tile = w; tile < ntiles; tile += NW) {
    const int bat = tile / per, rem = tile - bat * per;
    const int tm = rem / tpN, tp = rem - tm * tpN;
    const int am = tm * 8 + ((l & 15) >> 1);
    const int bn0 = tp * 32 + (l & 15), bn1 = bn0 + 16;
    const bool aok = am < M, b0ok = bn0 < N, b1ok = bn1 < N;
    const uint2* ap = lds + A.off + (aok ? am : 0) * A.s0 + bat * A.sb;
    const uint2* bp0 = lds + B.off + (b0ok ? bn0 : 0) * B.s1 + bat * B.sb;
    const uint2* bp1 = lds + B.off + (b1ok ? bn1 : 0) * B.s1 + bat * B.sb;
    v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < ks; ++s) {
      v4u ahi, alo, b0hi, b0lo, b1hi, b1lo;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int k = 16 * s + 4 * kg + d;
        const bool kok = k < K;
        const uint2 va = (aok && kok) ? ap[k * A.s1] : make_uint2(0u, 0u);
        const uint2 vb0 = (b0ok && kok) ? bp0[k * B.s0] : make_uint2(0u, 0u);
        const uint2 vb1 = (b1ok && kok) ? bp1[k * B.s0] : make_uint2(0u, 0u);
        ahi[d] = embed_a_bf(va.x, ri);
        alo[d] = embed_a_bf(va.y, ri);
        b0hi[d] = vb0.x;
        b0lo[d] = vb0.y;
        b1hi[d] = vb1.x;
        b1lo[d] = vb1.y;
      }
      acc0 = mfma_bf3(ahi, alo, b0hi, b0lo, acc0);
      acc1 = mfma_bf3(ahi, alo, b1hi, b1lo, acc1);
    }
    const int cm0 = tm * 8 + 2 * (l >> 4);
    uint2* cb = lds + C.off + bat * C.sb;
    if (b0ok) {
      if (cm0 < M) cb[cm0 * C.s0 + bn0 * C.s1] = split_bf3(make_float2(acc0[0], acc0[1]));
      if (cm0 + 1 < M) cb[(cm0 + 1) * C.s0 + bn0 * C.s1] = split_bf3(make_float2(acc0[2], acc0[3]));
    }
    if (b1ok) {
      if (cm0 < M) cb[cm0 * C.s0 + bn1 * C.s1] = split_bf3(make_float2(acc1[0], acc1[1]));
      if (cm0 + 1 < M) cb[(cm0 + 1) * C.s0 + bn1 * C.s1] = split_bf3(make_float2(acc1[2], acc1[3]));
    }
  }
}
