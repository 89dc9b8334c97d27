// Device stages of the translation (Eq. (5) with on-the-fly restoration) and
// the kernels built from them.  Included by one translation unit per operator
// family so the template instantiations compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "device_common.h"
#include "launch.h"
#include "tucker_restore.h"
#include "xy_stages.h"

namespace tfmm {

// ---------------------------------------------------------------------------
// Restoration of an operator tile into MFMA accumulators.
//
// Accumulator layout (16x16x4 f32 MFMA, D[i][j] in lane j + 16*(i/4), reg i%4):
// real row R = 16 t + 4 g + r of row tile t is (fz, re/im) = (8t + 2g + r/2,
// r%2); column j of column block c is pencil q0 + (w*CB + c)*16 + j.  The tile
// is T~_p[fz][q] = sum_k V[fz][k] W[q][k] (V = U3, or the TT-4D direction slice;
// W = the pencil-side partial contraction), accumulated chunk by chunk of k.
// ---------------------------------------------------------------------------
template <int T, int CB>
__device__ __forceinline__ void restore_final_chunk(v4f (&acc)[T][CB], const float2* sV, const float2* sW, int KC,
                                                    int kc) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, j = l & 15;
  const int kofs = (l >> 4) >> 1, ki = (l >> 4) & 1, ri = l & 1;
  const int ks = (kc + 1) >> 1;
  for (int s = 0; s < ks; ++s) {
    const int k = 2 * s + kofs;
    const bool kok = k < kc;
    float av[T], bv[CB];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int fz = 8 * t + (j >> 1);
      const float2 v = kok ? sV[fz * KC + k] : make_float2(0.f, 0.f);
      av[t] = ri == 0 ? (ki == 0 ? v.x : -v.y) : (ki == 0 ? v.y : v.x);
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int ql = (w * CB + c) * 16 + j;
      const float2 v = kok ? sW[ql * KC + k] : make_float2(0.f, 0.f);
      bv[c] = ki == 0 ? v.x : v.y;
    }
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int c = 0; c < CB; ++c) acc[t][c] = mfma4(av[t], bv[c], acc[t][c]);
  }
}

// Split-BF16 variant of restore_final_chunk: one 16x16x32 bf16 step covers 16
// complex k (lane group kg supplies k = 16s + 4kg .. +3), three MFMAs per step.
template <int T, int CB>
__device__ __forceinline__ void restore_final_chunk_bf3(v4f (&acc)[T][CB], const uint2* sV, const uint2* sW, int KC,
                                                        int kc) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, j = l & 15;
  const int kg = l >> 4, ri = l & 1;
  const int ks = (kc + 15) >> 4;
  for (int s = 0; s < ks; ++s) {
    v4u ahi[T], alo[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int fz = 8 * t + (j >> 1);
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int k = 16 * s + 4 * kg + d;
        const uint2 v = k < kc ? sV[fz * KC + k] : make_uint2(0u, 0u);
        ahi[t][d] = embed_a_bf(v.x, ri);
        alo[t][d] = embed_a_bf(v.y, ri);
      }
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int ql = (w * CB + c) * 16 + j;
      v4u bhi, blo;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int k = 16 * s + 4 * kg + d;
        const uint2 v = k < kc ? sW[ql * KC + k] : make_uint2(0u, 0u);
        bhi[d] = v.x;
        blo[d] = v.y;
      }
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t][c] = mfma_bf3(ahi[t], alo[t], bhi, blo, acc[t][c]);
    }
  }
}

template <bool BF, int NW>
__device__ __forceinline__ void stage_gemm(float2* lds, int M, int N, int K, int nb, LOp A, LOp B, LOp C) {
  if constexpr (BF)
    block_cgemm_bf3<NW>(reinterpret_cast<uint2*>(lds), M, N, K, nb, A, B, C);
  else
    block_cgemm<NW>(lds, M, N, K, nb, A, B, C);
}

template <bool BF, int T, int CB>
__device__ __forceinline__ void stage_final(v4f (&acc)[T][CB], float2* sV, float2* sW, int KC, int kc) {
  if constexpr (BF)
    restore_final_chunk_bf3<T, CB>(acc, reinterpret_cast<const uint2*>(sV), reinterpret_cast<const uint2*>(sW), KC,
                                   kc);
  else
    restore_final_chunk<T, CB>(acc, sV, sW, KC, kc);
}

// A chunk of a factor copied to LDS: element e (row e >> kcs, column e & (KC-1))
// is base[row*rstride + c0 + col] for col < kc and row < rows, else zero.
struct ChunkSrc {
  const float2* base;
  int rstride, rows, kcs, KC;
  __device__ __forceinline__ float2 at(int e, int c0, int kc) const {
    const int col = e & (KC - 1), row = e >> kcs;
    return (col < kc && row < rows) ? base[(long long)row * rstride + c0 + col] : make_float2(0.f, 0.f);
  }
};

// Register prefetch of the next chunk: its first PF*NT elements are loaded
// into registers while the current chunk is consumed (block barriers only
// drain LDS traffic, so the loads stay in flight); the rest is loaded at
// store time.
template <int NT>
struct ChunkPrefetch {
  static constexpr int PF = 8;
  float rx[PF], ry[PF];
  __device__ __forceinline__ void load(const ChunkSrc& src, int count, int c0, int kc) {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = threadIdx.x + i * NT;
      const float2 v = e < count ? src.at(e, c0, kc) : make_float2(0.f, 0.f);
      rx[i] = v.x;
      ry[i] = v.y;
    }
  }
  template <bool BF>
  __device__ __forceinline__ void store(float2* dst, const ChunkSrc& src, int count, int c0, int kc) {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = threadIdx.x + i * NT;
      if (e < count) stage<BF>(dst, e, make_float2(rx[i], ry[i]));
    }
    for (int e = threadIdx.x + PF * NT; e < count; e += NT) stage<BF>(dst, e, src.at(e, c0, kc));
  }
};

// N2C: n2 when known at compile time (fused kernels), else 0.
template <int FMT, int T, int CB, int NW, bool BF, int N2C = 0>
__device__ __forceinline__ void restore_tile(v4f (&acc)[T][CB], const ZArgs& a, int p, int q0, float2* lds) {
  constexpr int NT = 64 * NW, QT = 16 * CB * NW, N3 = 8 * T;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, j = l & 15, g = l >> 4;
  const int tid = threadIdx.x;
  const int nq = a.nq, n2 = a.n2;
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[t][c] = v4f{0.f, 0.f, 0.f, 0.f};
  if constexpr (FMT == ZF_FULL) {
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int q = q0 + (w * CB + c) * 16 + j;
        if (q < nq) {
          const float4 v = a.Tfull[((long long)p * (N3 / 2) + 4 * t + g) * nq + q];
          acc[t][c] = v4f{v.x, v.y, v.z, v.w};
        }
      }
  } else {
    const int* d = a.desc + 8 * p;
    const int KC = a.KC, kcs = 31 - __builtin_clz(KC);  // KC is a power of two
    if constexpr (FMT == ZF_TUCKER_W1) {
      restore_tucker_w1<T, CB, NW, BF>(acc, a, d, p, q0, lds);
      (void)KC;
      (void)kcs;
    } else if constexpr (FMT == ZF_TUCKER) {
      if (a.tk2) {
        restore_tucker<T, CB, NW, BF, N2C>(acc, a, d, q0, lds);
        return;
      }
      const int r1 = d[4], r2 = d[5], r3 = d[6];
      const float2* C = a.cbase + d[0];
      const float2* U1 = a.fbase + d[1];
      const float2* U2 = a.fbase + d[2];
      const float2* U3 = a.fbase + d[3];
      const int nfx = QT / n2, fx0 = q0 / n2;
      const int oU1 = 0, oU2 = oU1 + nfx * r1, oC = oU2 + n2 * r2, oW1 = oC + r1 * r2 * KC,
                oW = oW1 + nfx * r2 * KC, oV = oW + QT * KC;
      for (int e = tid; e < nfx * r1; e += NT) stage<BF>(lds, oU1 + e, U1[fx0 * r1 + e]);
      for (int e = tid; e < n2 * r2; e += NT) stage<BF>(lds, oU2 + e, U2[e]);
      // core chunk element e = (a*r2 + b)*KC + cl  <-  C[a][b][c0 + cl]
      const int csz = r1 * r2 * KC;
      const ChunkSrc src{C, r3, r1 * r2, kcs, KC};
      ChunkPrefetch<NT> pf;
      pf.load(src, csz, 0, min(KC, r3));
      for (int c0 = 0; c0 < r3; c0 += KC) {
        const int kc = min(KC, r3 - c0);
        pf.template store<BF>(lds + oC, src, csz, c0, kc);
        for (int e = tid; e < N3 * KC; e += NT) {
          const int cl = e & (KC - 1), fz = e >> kcs;
          stage<BF>(lds, oV + e, cl < kc ? U3[fz * r3 + c0 + cl] : make_float2(0.f, 0.f));
        }
        __syncthreads();
        if (c0 + KC < r3) pf.load(src, csz, c0 + KC, min(KC, r3 - c0 - KC));
        // W1[fx][(b,cl)] = sum_a U1[fx][a] C[a][(b,cl)]             (Fig. 3(a) step 1)
        stage_gemm<BF, NW>(lds, nfx, r2 * KC, r1, 1, LOp{oU1, r1, 1, 0}, LOp{oC, r2 * KC, 1, 0},
                           LOp{oW1, r2 * KC, 1, 0});
        __syncthreads();
        // W[(fx,fy)][cl] = sum_b W1[fx][b][cl] U2[fy][b]              (step 2), batch over cl
        stage_gemm<BF, NW>(lds, nfx, n2, r2, kc, LOp{oW1, r2 * KC, KC, 1}, LOp{oU2, 1, r2, 0},
                           LOp{oW, n2 * KC, KC, 1});
        __syncthreads();
        // T~[fz][q] += sum_c U3[fz][c] W[q][c]                         (step 3)
        stage_final<BF, T, CB>(acc, lds + oV, lds + oW, KC, kc);
        __syncthreads();
      }
    } else if constexpr (FMT == ZF_TT3D) {
      if (a.tk2) {  // W_p formed ahead of the z-stage (launch_cgemm_tt3d)
        restore_tt_chained<T, CB, NW, BF>(acc, a, d[5], a.fbase + d[3], a.wbase + d[7], q0, lds);
        return;
      }
      const int r1 = d[4], r2 = d[5];
      const float2* C = a.cbase + d[0];
      const float2* U1 = a.fbase + d[1];
      const float2* U3 = a.fbase + d[3];
      const int nfx = QT / n2, fx0 = q0 / n2;
      const int oU1 = 0, oC = oU1 + nfx * r1, oW = oC + r1 * n2 * KC, oV = oW + QT * KC;
      for (int e = tid; e < nfx * r1; e += NT) stage<BF>(lds, oU1 + e, U1[fx0 * r1 + e]);
      // core chunk element e = (a*n2 + y)*KC + bl  <-  C[a][y][b0 + bl]
      const int csz = r1 * n2 * KC;
      const ChunkSrc src{C, r2, r1 * n2, kcs, KC};
      ChunkPrefetch<NT> pf;
      pf.load(src, csz, 0, min(KC, r2));
      for (int b0 = 0; b0 < r2; b0 += KC) {
        const int kc = min(KC, r2 - b0);
        pf.template store<BF>(lds + oC, src, csz, b0, kc);
        for (int e = tid; e < N3 * KC; e += NT) {
          const int bl = e & (KC - 1), fz = e >> kcs;
          stage<BF>(lds, oV + e, bl < kc ? U3[fz * r2 + b0 + bl] : make_float2(0.f, 0.f));
        }
        __syncthreads();
        if (b0 + KC < r2) pf.load(src, csz, b0 + KC, min(KC, r2 - b0 - KC));
        // W[(fx,fy)][bl] = sum_a U1[fx][a] C[a][(fy,bl)]              (Fig. 4(a) step 1)
        stage_gemm<BF, NW>(lds, nfx, n2 * KC, r1, 1, LOp{oU1, r1, 1, 0}, LOp{oC, n2 * KC, 1, 0},
                           LOp{oW, n2 * KC, 1, 0});
        __syncthreads();
        stage_final<BF, T, CB>(acc, lds + oV, lds + oW, KC, kc);  // step 2
        __syncthreads();
      }
    } else {  // ZF_TT4D: W = T1 (direction-independent), V = S_p (Fig. 4(b))
      if (a.tk2) {
        restore_tt_chained<T, CB, NW, BF>(acc, a, d[5], a.vbase + d[3], a.wbase, q0, lds);
        return;
      }
      const int r2 = d[5];
      const float2* V = a.vbase + d[3];
      const int oW = 0, oV = QT * KC;
      // W chunk element e = ql*KC + bl  <-  T1[q0 + ql][b0 + bl]
      const int wsz = QT * KC;
      const ChunkSrc src{a.wbase + (long long)q0 * r2, r2, nq - q0, kcs, KC};
      ChunkPrefetch<NT> pf;
      pf.load(src, wsz, 0, min(KC, r2));
      for (int b0 = 0; b0 < r2; b0 += KC) {
        const int kc = min(KC, r2 - b0);
        pf.template store<BF>(lds + oW, src, wsz, b0, kc);
        for (int e = tid; e < N3 * KC; e += NT) {
          const int bl = e & (KC - 1), fz = e >> kcs;
          stage<BF>(lds, oV + e, bl < kc ? V[fz * r2 + b0 + bl] : make_float2(0.f, 0.f));
        }
        __syncthreads();
        if (b0 + KC < r2) pf.load(src, wsz, b0 + KC, min(KC, r2 - b0 - KC));
        stage_final<BF, T, CB>(acc, lds + oV, lds + oW, KC, kc);
        __syncthreads();
      }
    }
  }
}

// ---------------------------------------------------------------------------
// z-FFT, product and inverse z-FFT of one RHS in the accumulator layout.
// Lane (g, j) owns fz = 8t + b, b in {2g, 2g+1}, t < T (n3 = 8T):
//   forward  X[8t+b] = DFT_T over v of  w^{vb} sum_{u<4} x[Tu+v] w8^{ub}
//   inverse  out[Tu'+v'] = sum_b w8^{-bu'} w^{-bv'} IDFT_T over t of Y[8t+b]
// (w = exp(-2 pi i/n3), w8 = exp(-2 pi i/8)).  The inverse partial sums of the
// four lane groups are reduce-scattered with two cross-lane exchanges, after
// which lane group g holds out[z'] for z' in [T g, T g + T).
// Element (z, q) of the half spectrum is at H[z*zs + q*qs].
// ---------------------------------------------------------------------------
template <int T>
__device__ __forceinline__ void dft_small_fwd(const float2* x, float2* y) {
  if constexpr (T == 1) dft_full_fwd_1(x, y);
  else if constexpr (T == 2) dft_full_fwd_2(x, y);
  else if constexpr (T == 3) dft_full_fwd_3(x, y);
  else if constexpr (T == 4) dft_full_fwd_4(x, y);
  else if constexpr (T == 6) dft_full_fwd_6(x, y);
  else dft_full_fwd_8(x, y);
}
template <int T>
__device__ __forceinline__ void dft_small_inv(const float2* x, float2* y) {
  if constexpr (T == 1) dft_full_inv_1(x, y);
  else if constexpr (T == 2) dft_full_inv_2(x, y);
  else if constexpr (T == 3) dft_full_inv_3(x, y);
  else if constexpr (T == 4) dft_full_inv_4(x, y);
  else if constexpr (T == 6) dft_full_inv_6(x, y);
  else dft_full_inv_8(x, y);
}

__device__ __forceinline__ float2 shfl_xor2(float2 v, int mask) {
  return make_float2(__shfl_xor(v.x, mask), __shfl_xor(v.y, mask));
}

template <int T>
struct ZTwiddles {
  float2 tw[2][T], w8[4][2];
  __device__ __forceinline__ void load(const float2* roots) {
    constexpr int N3 = 8 * T;
    const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int b = 2 * g + e;
#pragma unroll
      for (int v = 0; v < T; ++v) tw[e][v] = roots[(v * b) % N3];
#pragma unroll
      for (int u = 0; u < 4; ++u) w8[u][e] = roots[(u * b * T) % N3];
    }
  }
};

template <int T, int CB>
__device__ __forceinline__ void zfft_rhs(const v4f (&acc)[T][CB], float2* H, long long zs, int qs, int qbase, int nq,
                                         const ZTwiddles<T>& Z) {
  constexpr int KZ = 4 * T;
  const int l = threadIdx.x & 63, j = l & 15, g = l >> 4;
  const bool hi = g >= 2, odd = (g & 1) != 0;
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int q = qbase + c * 16 + j;
    const bool qok = q < nq;
    float2 x[KZ];
#pragma unroll
    for (int z = 0; z < KZ; ++z) x[z] = qok ? H[z * zs + (long long)q * qs] : make_float2(0.f, 0.f);
    float2 zt[2][T];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      float2 yv[T], X[T], Y[T], Zi[T];
#pragma unroll
      for (int v = 0; v < T; ++v) {
        float2 sacc = x[v];
#pragma unroll
        for (int u = 1; u < 4; ++u) sacc = cadd(sacc, cmul(x[T * u + v], Z.w8[u][e]));
        yv[v] = cmul(sacc, Z.tw[e][v]);
      }
      dft_small_fwd<T>(yv, X);
#pragma unroll
      for (int t = 0; t < T; ++t) Y[t] = cmul(X[t], make_float2(acc[t][c][2 * e], acc[t][c][2 * e + 1]));
      dft_small_inv<T>(Y, Zi);
#pragma unroll
      for (int v = 0; v < T; ++v) zt[e][v] = cmulconj(Zi[v], Z.tw[e][v]);
    }
    float2 kept[2][T];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int v = 0; v < T; ++v) {
        const float2 plo = cadd(cmulconj(zt[0][v], Z.w8[k][0]), cmulconj(zt[1][v], Z.w8[k][1]));
        const float2 phi = cadd(cmulconj(zt[0][v], Z.w8[2 + k][0]), cmulconj(zt[1][v], Z.w8[2 + k][1]));
        kept[k][v] = cadd(hi ? phi : plo, shfl_xor2(hi ? plo : phi, 32));
      }
#pragma unroll
    for (int v = 0; v < T; ++v) {
      const float2 out = cadd(odd ? kept[1][v] : kept[0][v], shfl_xor2(odd ? kept[0][v] : kept[1][v], 16));
      if (qok) H[(T * g + v) * zs + (long long)q * qs] = out;
    }
  }
}

// ---------------------------------------------------------------------------
// z-stage of the fused 32^3 kernel with whole pencils per lane.  After the
// restoration, each wave moves its 128 accumulator columns through LDS so that
// lane l holds all 32 frequencies of pencils l and 64 + l of the wave.  Per RHS
// a lane then transforms its pencils alone, splitting the pruned 32-point
// transform (16 nonzero inputs) into even and odd outputs:
//   X[2m]   = DFT16(x)[m],        X[2m+1] = DFT16(x[z] w^z)[m],
//   y[z']   = IDFT16(P_even)[z'] + w^-z' IDFT16(P_odd)[z'],   z' < 16,
// with w = exp(-2 pi i / 32); the 1/N scale is applied by the xy stage.
// ---------------------------------------------------------------------------
__device__ constexpr float kW32[16][2] = {
    {0x1.0000000000000p+0f, 0.0f},
    {0x1.f6297c0000000p-1f, -0x1.8f8b840000000p-3f},
    {0x1.d906bc0000000p-1f, -0x1.87de2a0000000p-2f},
    {0x1.a9b6620000000p-1f, -0x1.1c73b40000000p-1f},
    {0x1.6a09e60000000p-1f, -0x1.6a09e60000000p-1f},
    {0x1.1c73b40000000p-1f, -0x1.a9b6620000000p-1f},
    {0x1.87de2a0000000p-2f, -0x1.d906bc0000000p-1f},
    {0x1.8f8b840000000p-3f, -0x1.f6297c0000000p-1f},
    {0.0f, -0x1.0000000000000p+0f},
    {-0x1.8f8b840000000p-3f, -0x1.f6297c0000000p-1f},
    {-0x1.87de2a0000000p-2f, -0x1.d906bc0000000p-1f},
    {-0x1.1c73b40000000p-1f, -0x1.a9b6620000000p-1f},
    {-0x1.6a09e60000000p-1f, -0x1.6a09e60000000p-1f},
    {-0x1.a9b6620000000p-1f, -0x1.1c73b40000000p-1f},
    {-0x1.d906bc0000000p-1f, -0x1.87de2a0000000p-2f},
    {-0x1.f6297c0000000p-1f, -0x1.8f8b840000000p-3f}};

template <int CB>
__device__ __forceinline__ void acc_to_pencils32(const v4f (&acc)[4][CB], float2 (&tz)[CB / 4][32], float2* lds) {
  static_assert(CB % 4 == 0, "whole pencils per lane need 64 columns per round");
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, j = l & 15;
  float2* reg = lds + w * (64 * 33);
#pragma unroll
  for (int r = 0; r < CB / 4; ++r) {
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int e = 0; e < 2; ++e)
          reg[(cc * 16 + j) * 33 + 8 * t + 2 * g + e] =
              make_float2(acc[t][4 * r + cc][2 * e], acc[t][4 * r + cc][2 * e + 1]);
    __syncthreads();
#pragma unroll
    for (int f = 0; f < 32; ++f) tz[r][f] = reg[l * 33 + f];
    __syncthreads();
  }
}

// H: the wave's half-spectrum slab, element (z, pencil q) at q*ZP + z.
template <int NP, int ZP>
__device__ __forceinline__ void zfft_pencils32(const float2 (&tz)[NP][32], float2* H, int qbase) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    float2* h = H + (qbase + 64 * u + l) * ZP;
    float2 x[16], xo[16], E[16];
#pragma unroll
    for (int z = 0; z < 16; ++z) {
      x[z] = h[z];
      xo[z] = cmul(x[z], make_float2(kW32[z][0], kW32[z][1]));
    }
    dft_full_fwd_16(x, E);
#pragma unroll
    for (int m = 0; m < 16; ++m) E[m] = cmul(E[m], tz[u][2 * m]);
    dft_full_inv_16(E, x);  // x <- even part of the output
    dft_full_fwd_16(xo, E);
#pragma unroll
    for (int m = 0; m < 16; ++m) E[m] = cmul(E[m], tz[u][2 * m + 1]);
    dft_full_inv_16(E, xo);
#pragma unroll
    for (int z = 0; z < 16; ++z) h[z] = cadd(x[z], cmulconj(xo[z], make_float2(kW32[z][0], kW32[z][1])));
  }
}

// ---------------------------------------------------------------------------
// y- and z-stages of the three-pass pipeline on the tile's x-FFT'ed planes.
// A tile of QT = 64 CB pencils (q = fx n2 + fy) covers nf = QT / n2 whole fx
// planes.  The restored tile (wave w: 16 CB pencils, lane (g, j) of column
// block c holding fz = 8t + 2g + {0,1} of pencil 16c + j) is written once to an
// LDS region, one row of N3 frequencies per pencil (odd row stride); lane l of
// wave w then owns tile pencil w 16 CB + l.  Per RHS the block
//   1. runs the zero-padded y-FFTs of every (fx, z) line of its planes
//      G[fx][y][z] (y < n2/2, z < K3 = N3/2), read straight from device memory
//      (consecutive threads take consecutive z), into the tile's half spectrum
//      in LDS, one row of K3 per pencil,
//   3. per pencil (one lane each) splits the pruned N3-point z transform into
//      even and odd outputs, X[2m] = DFT_K3(x)[m], X[2m+1] = DFT_K3(x[z] w^z)[m],
//      multiplies by T~ and inverts: y[z'] = IDFT_K3(P_even)[z'] + w^-z'
//      IDFT_K3(P_odd)[z'], z' < K3 (w = exp(-2 pi i / N3)),
//   4. runs the inverse y-FFTs of every (fx, z) line, keeping y < n2/2, and
//      writes the planes back in place.
// The RHS go through in groups of rg (a.rg, as many half spectra as LDS holds)
// so that each phase has rg times the independent lines and pencils.
// ---------------------------------------------------------------------------
template <int N2>
__device__ __forceinline__ void yline_fwd(const float2* src, int ss, float2* dst, int ds) {
  float2 x[N2 / 2], X[N2];
#pragma unroll
  for (int i = 0; i < N2 / 2; ++i) x[i] = src[i * ss];
  Dft<N2>::fwd(x, X);
#pragma unroll
  for (int f = 0; f < N2; ++f) dst[f * ds] = X[f];
}

template <int N2>
__device__ __forceinline__ void yline_inv(const float2* src, int ss, float2* dst, int ds) {
  float2 x[N2], X[N2 / 2];
#pragma unroll
  for (int f = 0; f < N2; ++f) x[f] = src[f * ss];
  Dft<N2>::inv(x, X);
#pragma unroll
  for (int i = 0; i < N2 / 2; ++i) dst[i * ds] = X[i];
}

// y lines of length n2 = 64 CB / nf (a divisor of the tile width)
template <int CB>
__device__ __forceinline__ void yline(bool fwd, int n2, const float2* src, int ss, float2* dst, int ds) {
#define TFMM_YL(N)                                                    \
  case N:                                                             \
    if constexpr ((64 * CB) % N == 0) {                               \
      if (fwd) yline_fwd<N>(src, ss, dst, ds);                        \
      else yline_inv<N>(src, ss, dst, ds);                            \
    }                                                                 \
    break;
  switch (n2) { TFMM_YL(8) TFMM_YL(16) TFMM_YL(24) TFMM_YL(32) TFMM_YL(48) TFMM_YL(64) }
#undef TFMM_YL
}

// The restored tile reaches the per-lane pencil layout through LDS (lane l of
// wave w takes pencil 16 CB w + l, all n3 frequencies).  With n3 <= 32 it is
// then held in registers (zplanes_tile_in_regs), so the tile's LDS is free for
// the half spectra (and, where the kernel is built for two waves per SIMD, two
// blocks share a compute unit); longer pencils keep it in LDS next to the half
// spectra.
template <int T, int CB>
__device__ __forceinline__ void zstage_planes(const v4f (&acc)[T][CB], const ZArgs& a, int pl, int q0,
                                              float2* lds) {
  constexpr int N3 = 8 * T, K = 4 * T, PS = N3 + 1, NPW = 16 * CB, QT = 4 * NPW, KP = K | 1;
  constexpr bool REG = zplanes_tile_in_regs(T);
  static_assert(NPW <= 64, "one pencil per lane");  // LDS: zplanes_lds_bytes
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, j = l & 15;
  const int n2 = a.n2, K2 = n2 / 2, nf = QT / n2, fx0 = q0 / n2, rg = a.rg;
  float2* reg = lds + w * (NPW * PS);
  float2* Hl = REG ? lds : lds + QT * PS;  // [rg][QT][KP]: half spectra of rg RHS
  __syncthreads();  // the restoration is done with its LDS
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int e = 0; e < 2; ++e)
        reg[(c * 16 + j) * PS + 8 * t + 2 * g + e] = make_float2(acc[t][c][2 * e], acc[t][c][2 * e + 1]);
  float2 tr[REG ? N3 : 1];
  if constexpr (REG) {
    __syncthreads();
    if (l < NPW) {
#pragma unroll
      for (int m = 0; m < N3; ++m) tr[m] = reg[l * PS + m];
    }
  }
  const int nline = nf * K;       // (fx, z) lines per RHS
  const long long plane = (long long)K2 * K;
  const float2* tz = reg + l * PS;
  auto T_at = [&](int m) { return REG ? tr[m] : tz[m]; };
  const float2* wz = a.roots;     // wz[z] = w^z
  for (int s0 = 0; s0 < a.nrhs; s0 += rg) {
    const int nr = min(rg, a.nrhs - s0);
    __syncthreads();  // the previous group is done with the half spectra (and the tile is in place)
    // forward y lines, read straight from the planes (consecutive threads: consecutive z)
    for (int task = threadIdx.x; task < nr * nline; task += TFMM_BLOCK) {
      const int r = task / nline, t2 = task - r * nline, f = t2 / K, z = t2 - f * K;
      const float2* gp = a.H + (((long long)(s0 + r) * a.ndl + pl) * a.n1 + fx0) * plane;
      yline<CB>(true, n2, gp + f * K2 * K + z, K, Hl + (r * QT + f * n2) * KP + z, KP);
    }
    __syncthreads();
    if (l < NPW) {
      for (int r = 0; r < nr; ++r) {
        float2* h = Hl + (r * QT + w * NPW + l) * KP;
        float2 x[K], E[K], ye[K];
#pragma unroll
        for (int z = 0; z < K; ++z) x[z] = h[z];
        DftFull<K>::fwd(x, E);
#pragma unroll
        for (int z = 0; z < K; ++z) x[z] = cmul(x[z], wz[z]);
#pragma unroll
        for (int m = 0; m < K; ++m) E[m] = cmul(E[m], T_at(2 * m));
        DftFull<K>::inv(E, ye);
        DftFull<K>::fwd(x, E);
#pragma unroll
        for (int m = 0; m < K; ++m) E[m] = cmul(E[m], T_at(2 * m + 1));
        DftFull<K>::inv(E, x);
#pragma unroll
        for (int z = 0; z < K; ++z) h[z] = cadd(ye[z], cmulconj(x[z], wz[z]));
      }
    }
    __syncthreads();
    // inverse y lines with the crop, written straight back to the planes
    for (int task = threadIdx.x; task < nr * nline; task += TFMM_BLOCK) {
      const int r = task / nline, t2 = task - r * nline, f = t2 / K, z = t2 - f * K;
      float2* gp = a.H + (((long long)(s0 + r) * a.ndl + pl) * a.n1 + fx0) * plane;
      yline<CB>(false, n2, Hl + (r * QT + f * n2) * KP + z, KP, gp + f * K2 * K + z, K);
    }
  }
  __syncthreads();  // the region is reused by the next item's restoration
}

// ---------------------------------------------------------------------------
// Work items of the z-stage and fused kernels.  Block b starts with item b;
// when the launch has more items than resident blocks (a.counter set), each
// block then takes further items from counter[0] (offset by the grid size),
// broadcast by thread 0 through the LDS slot past the working set.  A block
// leaves once the items are exhausted; the last block to leave (counted in
// counter[1]) resets both counters, so a launch, captured or not, needs no
// clearing step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int next_item(const ZArgs& a, float2* lds) {
  if (!a.counter) return 0x7fffffff;
  int* slot = reinterpret_cast<int*>(reinterpret_cast<char*>(lds) + a.lds_bytes);
  if (threadIdx.x == 0) *slot = (int)gridDim.x + atomicAdd(a.counter, 1);
  __syncthreads();
  return *slot;
}

__device__ __forceinline__ void leave_queue(const ZArgs& a) {
  if (a.counter && threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(a.counter + 1, 1) == (int)gridDim.x - 1) {
      atomicExch(a.counter, 0);
      atomicExch(a.counter + 1, 0);
    }
  }
}

// ---------------------------------------------------------------------------
// Pass 2 of the three-pass pipeline: a persistent grid walks the (direction,
// pencil tile) items of the launch, costliest directions first; the restored
// tile is shared by every RHS of the launch.
// ---------------------------------------------------------------------------
template <int FMT, int T, int CB, bool BF>
__device__ __forceinline__ void zstage_item(const ZArgs& a, int it, float2* lds) {
  constexpr int NW = 4, QT = 16 * CB * NW;
  const int ntile = a.nq / QT;
  // TT-4D restores every direction's tile from the same rows of T1: items run
  // tile-major there, so the blocks resident together share those rows in L2
  int pl, q0;
  if constexpr (FMT == ZF_TT4D) {
    const int tile = it / a.ndl;
    pl = it - tile * a.ndl;
    q0 = tile * QT;
  } else {
    pl = it / ntile;
    q0 = (it - pl * ntile) * QT;
  }
  const int p = a.perm ? a.perm[a.p0 + pl] : a.p0 + pl;
  v4f acc[T][CB];
  restore_tile<FMT, T, CB, NW, BF>(acc, a, p, q0, lds);
  zstage_planes<T, CB>(acc, a, pl, q0, lds);
}

// The first item of every block is its own index; only a launch with more
// items than resident blocks enters the queue loop (a separate copy of the
// item body, so the common single-item path carries no loop state).
template <int FMT, int T, int CB, bool BF>
__global__ __launch_bounds__(256, zplanes_waves_per_simd(FMT, T)) void k_zstage(ZArgs a) {
  extern __shared__ float2 lds[];
  constexpr int QT = 16 * CB * 4;
  const int nitems = a.nq / QT * a.ndl;
  zstage_item<FMT, T, CB, BF>(a, blockIdx.x, lds);
  if (a.counter) {
    for (int it = next_item(a, lds); it < nitems; it = next_item(a, lds)) zstage_item<FMT, T, CB, BF>(a, it, lds);
    leave_queue(a);
  }
}

// ---------------------------------------------------------------------------
// Fused translation for grids whose half spectrum fits in LDS: per direction
// a block restores the whole T~_p into accumulators once, then for every RHS
// runs the xy-FFTs, the z-stage and the inverse xy-FFTs on chip.  A and B are
// the only device-memory traffic besides the stored operator.
// ---------------------------------------------------------------------------
template <int FMT, int N, int NW, int CB, bool BF>
__device__ __forceinline__ void fused_item(const ZArgs& a, const RhsPtrs& P, float scale, int it, float2* lds) {
  constexpr int T = N / 8, K = N / 2, NQ = N * N, NT = 64 * NW;
  constexpr int ZP = (K & 1) ? K : K + 1;
  static_assert(NQ == 16 * CB * NW, "tile must cover every pencil");
  const int w = threadIdx.x >> 6;
  const int p = a.perm ? a.perm[it] : it;
  v4f acc[T][CB];
  restore_tile<FMT, T, CB, NW, BF, N>(acc, a, p, 0, lds);
  const long long blk = (long long)K * K * K;
  if constexpr (N == 32 && CB % 4 == 0) {
    float2 tz[CB / 4][32];
    __syncthreads();
    acc_to_pencils32<CB>(acc, tz, lds);
    for (int s = 0; s < a.nrhs; ++s) {
      xy_forward<N, N, NT>(lds, P.a[s] + (long long)p * blk, K, K, ZP, 0, nullptr);
      __syncthreads();
      zfft_pencils32<CB / 4, ZP>(tz, lds, w * CB * 16);
      __syncthreads();
      xy_inverse<N, N, NT>(lds, P.b[s] + (long long)p * blk, K, K, ZP, 0, scale, nullptr);
      __syncthreads();
    }
  } else {
    ZTwiddles<T> Z;
    Z.load(a.roots);
    __syncthreads();
    for (int s = 0; s < a.nrhs; ++s) {
      xy_forward<N, N, NT>(lds, P.a[s] + (long long)p * blk, K, K, ZP, 0, nullptr);
      __syncthreads();
      zfft_rhs<T, CB>(acc, lds, 1, ZP, w * CB * 16, NQ, Z);
      __syncthreads();
      xy_inverse<N, N, NT>(lds, P.b[s] + (long long)p * blk, K, K, ZP, 0, scale, nullptr);
      __syncthreads();
    }
  }
}

// One block per direction, blocks numbered in cost order: the hardware
// dispatcher hands directions to compute units as they free up, i.e. it is
// the work queue.  (A queue loop inside this kernel keeps its restoration
// state live across items and spills the 256 registers a wave has here.)
template <int FMT, int N, int NW, int CB, bool BF>
__global__ __launch_bounds__(64 * NW) void k_fused(ZArgs a, RhsPtrs P, float scale) {
  extern __shared__ float2 lds[];
  fused_item<FMT, N, NW, CB, BF>(a, P, scale, blockIdx.x, lds);
}

// Resident blocks per compute unit of a kernel at a dynamic LDS size (the
// runtime query is cached: it costs host time on every launch otherwise).
inline int resident_blocks(const void* fn, int threads, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, int, size_t>, int> cache;
  const auto key = std::make_tuple(fn, threads, lds);
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, lds) != hipSuccess || n < 1) n = 1;
  cache[key] = n;
  return n;
}

// fused shape per grid: (waves, column blocks)
template <int N> struct FusedShape;
template <> struct FusedShape<8> { static constexpr int NW = 4, CB = 1; };
template <> struct FusedShape<16> { static constexpr int NW = 8, CB = 2; };
template <> struct FusedShape<24> { static constexpr int NW = 6, CB = 6; };
template <> struct FusedShape<32> { static constexpr int NW = 8, CB = 8; };

template <int FMT, int T, int CB, bool BF>
hipError_t run_zstage_p(const ZArgs& a, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_zstage<FMT, T, CB, BF>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr = true;
  }
  const size_t lds = (size_t)a.lds_bytes + TFMM_LDS_SLOT;
  const int nitems = a.nq / (64 * CB) * a.ndl;
  const int cap = a.ncu * resident_blocks((const void*)k_zstage<FMT, T, CB, BF>, 256, lds);
  ZArgs b = a;
  if (nitems <= cap) b.counter = nullptr;  // one item per block, no queue
  hipLaunchKernelGGL((k_zstage<FMT, T, CB, BF>), dim3(std::min(nitems, cap)), dim3(256), lds, st, b);
  return hipGetLastError();
}

// FULL has no restoration arithmetic, so it has no split-BF16 variant.
template <int FMT, int T, int CB>
hipError_t run_zstage(const ZArgs& a, hipStream_t st) {
  if constexpr (FMT != ZF_FULL)
    if (a.bf) return run_zstage_p<FMT, T, CB, true>(a, st);
  return run_zstage_p<FMT, T, CB, false>(a, st);
}

template <int FMT, int N, bool BF>
hipError_t run_fused_p(const ZArgs& a, const RhsPtrs& P, float scale, hipStream_t st) {
  constexpr int NW = FusedShape<N>::NW, CB = FusedShape<N>::CB;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_fused<FMT, N, NW, CB, BF>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL((k_fused<FMT, N, NW, CB, BF>), dim3(a.ndl), dim3(64 * NW), (size_t)a.lds_bytes, st, a, P,
                     scale);
  return hipGetLastError();
}

template <int FMT, int N>
hipError_t run_fused(const ZArgs& a, const RhsPtrs& P, float scale, hipStream_t st) {
  if constexpr (FMT != ZF_FULL)
    if (a.bf) return run_fused_p<FMT, N, true>(a, P, scale, st);
  return run_fused_p<FMT, N, false>(a, P, scale, st);
}

template <int FMT>
hipError_t launch_zstage_fmt(const ZArgs& a, hipStream_t st, bool* supported) {
  *supported = true;
  switch ((a.n3 / 8) * 10 + a.cb) {
#define ZC(TT, C) \
  case TT * 10 + C: return run_zstage<FMT, TT, C>(a, st);
    ZC(1, 1) ZC(1, 2) ZC(1, 3) ZC(1, 4)
    ZC(2, 1) ZC(2, 2) ZC(2, 3) ZC(2, 4)
    ZC(3, 1) ZC(3, 2) ZC(3, 3) ZC(3, 4)
    ZC(4, 1) ZC(4, 2) ZC(4, 3) ZC(4, 4)
    ZC(6, 1) ZC(6, 2) ZC(6, 3)
    ZC(8, 1) ZC(8, 2)
#undef ZC
  }
  *supported = false;
  return hipSuccess;
}

template <int FMT>
hipError_t launch_fused_fmt(const ZArgs& a, const RhsPtrs& P, float scale, hipStream_t st, bool* supported) {
  *supported = true;
  if (a.n1 == a.n2 && a.n2 == a.n3) {
    switch (a.n1) {
      case 8: return run_fused<FMT, 8>(a, P, scale, st);
      case 16: return run_fused<FMT, 16>(a, P, scale, st);
      case 24: return run_fused<FMT, 24>(a, P, scale, st);
      case 32: return run_fused<FMT, 32>(a, P, scale, st);
    }
  }
  *supported = false;
  return hipSuccess;
}

}  // namespace tfmm
