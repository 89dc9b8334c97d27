// Translation kernels for gfx950: Eq. (5) with operators restored on the fly.
//
//   pass 1  k_fwd_xy   zero-padded x- and y-FFTs of A per (rhs, direction, z-slab), in LDS
//   pass 2  k_zstage   per (direction, pencil tile): restore the operator tile on the
//                      matrix cores (Figs. 3-4), then z-FFT, multiply, inverse z-FFT of
//                      every RHS directly in the accumulator lane layout
//   pass 3  k_inv_xy   inverse y- and x-FFTs, crop to the box grid, scale 1/N
//   a1      k_cgemm    batched complex GEMMs producing per-direction cores of the
//                      4-D formats (Fig. 3(b)(c), Fig. 4(b) step 1)
//   setup   k_sample   FP64 operator samples, Eq. (7)
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "launch.h"

namespace tfmm {

// ---------------------------------------------------------------------------
// Setup: Eq. (7) in FP64.  h_l^(2) by upward recurrence from the closed forms
// of h_0 and h_1 (the recurrence is stable for the dominant y_l part), P_l by
// Bonnet's recurrence.  Near offsets and the unused slot m_i = K_i are zero.
// ---------------------------------------------------------------------------
__global__ void k_sample(double2* __restrict__ T, const double* __restrict__ khat, int K1, int K2, int K3,
                         double box, double k, int L, int near_rule, double near_param, double sre, double sim) {
  const int n1 = 2 * K1, n2 = 2 * K2, n3 = 2 * K3;
  const long long N = (long long)n1 * n2 * n3;
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (m >= N) return;
  const int m3 = (int)(m % n3), m2 = (int)((m / n3) % n2), m1 = (int)(m / ((long long)n2 * n3));
  double2 out = make_double2(0.0, 0.0);
  const bool slot = (m1 == K1) || (m2 == K2) || (m3 == K3);
  if (!slot) {
    const int d1 = m1 < K1 ? m1 : m1 - n1;
    const int d2 = m2 < K2 ? m2 : m2 - n2;
    const int d3 = m3 < K3 ? m3 : m3 - n3;
    bool near;
    if (near_rule == 0) {
      int cm = max(abs(d1), max(abs(d2), abs(d3)));
      near = cm <= near_param;
    } else {
      near = 4.0 * (double)(d1 * d1 + d2 * d2 + d3 * d3) < 3.0 * near_param * near_param;
    }
    near = near || (d1 == 0 && d2 == 0 && d3 == 0);
    if (!near) {
      const double Rx = box * d1, Ry = box * d2, Rz = box * d3;
      const double r = sqrt(Rx * Rx + Ry * Ry + Rz * Rz);
      const double x = k * r;
      const double c = (khat[3 * p] * Rx + khat[3 * p + 1] * Ry + khat[3 * p + 2] * Rz) / r;
      double sx, cx;
      sincos(x, &sx, &cx);
      // e^{-ix} = cx - i sx
      // h0 = i e^{-ix}/x = (sx + i cx)/x ; h1 = e^{-ix}(i/x^2 - 1/x)
      double h0r = sx / x, h0i = cx / x;
      const double ar = -1.0 / x, ai = 1.0 / (x * x);  // (i/x^2 - 1/x)
      double h1r = cx * ar + sx * ai, h1i = cx * ai - sx * ar;
      double P0 = 1.0, P1 = c;
      // l = 0 term: h0 * P0
      double sr = h0r * P0, si = h0i * P0;
      if (L >= 1) {  // (-i)^1 * 3 * h1 * P1
        sr += 3.0 * P1 * h1i;
        si += -3.0 * P1 * h1r;
      }
      double hmr = h0r, hmi = h0i, hr = h1r, hi = h1i;
      for (int l = 1; l < L; ++l) {
        // advance to l+1
        const double f = (2.0 * l + 1.0) / x;
        const double nr = f * hr - hmr, ni = f * hi - hmi;
        hmr = hr; hmi = hi; hr = nr; hi = ni;
        const double P2 = ((2.0 * l + 1.0) * c * P1 - l * P0) / (l + 1.0);
        P0 = P1; P1 = P2;
        const int lp = l + 1;
        const double wgt = (2.0 * lp + 1.0) * P1;
        // (-i)^lp
        switch (lp & 3) {
          case 0: sr += wgt * hr; si += wgt * hi; break;
          case 1: sr += wgt * hi; si -= wgt * hr; break;
          case 2: sr -= wgt * hr; si -= wgt * hi; break;
          default: sr -= wgt * hi; si += wgt * hr; break;
        }
      }
      out = make_double2(sre * sr - sim * si, sre * si + sim * sr);
    }
  }
  T[(long long)p * N + m] = out;
}

hipError_t launch_sample(double2* T, const double* khat, int ndir, const int K[3], double box, double k, int L,
                         int near_rule, double near_param, double sre, double sim, hipStream_t st) {
  const long long N = 8LL * K[0] * K[1] * K[2];
  dim3 grid((unsigned)((N + 255) / 256), (unsigned)ndir);
  hipLaunchKernelGGL(k_sample, grid, dim3(256), 0, st, T, khat, K[0], K[1], K[2], box, k, L, near_rule,
                     near_param, sre, sim);
  return hipGetLastError();
}

__global__ void k_pack_full(const float2* __restrict__ src, float4* __restrict__ dst, int nq, int n3) {
  // src [p][x][y][z] (q = x*n2 + y), dst [p][z/2][q]
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int zp = blockIdx.y, p = blockIdx.z;
  if (q >= nq) return;
  const float2* s = src + ((long long)p * nq + q) * n3 + 2 * zp;
  dst[((long long)p * (n3 / 2) + zp) * nq + q] = make_float4(s[0].x, s[0].y, s[1].x, s[1].y);
}

hipError_t launch_pack_full(const float2* src, float4* dst, int ndir, int nq, int n3, hipStream_t st) {
  dim3 grid((nq + 255) / 256, n3 / 2, ndir);
  hipLaunchKernelGGL(k_pack_full, grid, dim3(256), 0, st, src, dst, nq, n3);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pass 1 / pass 3: xy-FFTs of a slab of zg z-planes in LDS.
// LDS layout [fx][y][z] with z stride 1 and padded slab width zp (odd), so
// line accesses and the copy to/from the z-major half spectrum are
// bank-conflict free.
// ---------------------------------------------------------------------------
template <int N1, int N2>
__global__ __launch_bounds__(TFMM_BLOCK) void k_fwd_xy(RhsPtrs P, float2* __restrict__ H, int K3, int zg, int zp,
                                                       int ndl, int p0) {
  extern __shared__ float2 lds[];
  constexpr int K1 = N1 / 2, K2 = N2 / 2, NQ = N1 * N2;
  const int s = blockIdx.z, pl = blockIdx.y, z0 = blockIdx.x * zg;
  const float2* __restrict__ Ab = P.a[s] + (long long)(p0 + pl) * ((long long)K1 * K2 * K3);
  for (int task = threadIdx.x; task < K2 * zg; task += TFMM_BLOCK) {
    const int z = task % zg, y = task / zg;
    float2 x[K1], X[N1];
#pragma unroll
    for (int i = 0; i < K1; ++i) x[i] = Ab[((long long)i * K2 + y) * K3 + z0 + z];
    Dft<N1>::fwd(x, X);
#pragma unroll
    for (int f = 0; f < N1; ++f) lds[(f * N2 + y) * zp + z] = X[f];
  }
  __syncthreads();
  for (int task = threadIdx.x; task < N1 * zg; task += TFMM_BLOCK) {
    const int z = task % zg, fx = task / zg;
    float2 y[K2], Y[N2];
#pragma unroll
    for (int i = 0; i < K2; ++i) y[i] = lds[(fx * N2 + i) * zp + z];
    Dft<N2>::fwd(y, Y);
#pragma unroll
    for (int f = 0; f < N2; ++f) lds[(fx * N2 + f) * zp + z] = Y[f];
  }
  __syncthreads();
  float2* Hb = H + ((long long)s * ndl + pl) * ((long long)K3 * NQ) + (long long)z0 * NQ;
  for (int e = threadIdx.x; e < zg * NQ; e += TFMM_BLOCK) {
    const int z = e / NQ, q = e - z * NQ;
    Hb[e] = lds[q * zp + z];
  }
}

template <int N1, int N2>
__global__ __launch_bounds__(TFMM_BLOCK) void k_inv_xy(RhsPtrs P, const float2* __restrict__ H, int K3, int zg,
                                                       int zp, int ndl, int p0, float scale) {
  extern __shared__ float2 lds[];
  constexpr int K1 = N1 / 2, K2 = N2 / 2, NQ = N1 * N2;
  const int s = blockIdx.z, pl = blockIdx.y, z0 = blockIdx.x * zg;
  const float2* Hb = H + ((long long)s * ndl + pl) * ((long long)K3 * NQ) + (long long)z0 * NQ;
  for (int e = threadIdx.x; e < zg * NQ; e += TFMM_BLOCK) {
    const int z = e / NQ, q = e - z * NQ;
    lds[q * zp + z] = Hb[e];
  }
  __syncthreads();
  for (int task = threadIdx.x; task < N1 * zg; task += TFMM_BLOCK) {
    const int z = task % zg, fx = task / zg;
    float2 y[N2], Y[K2];
#pragma unroll
    for (int i = 0; i < N2; ++i) y[i] = lds[(fx * N2 + i) * zp + z];
    Dft<N2>::inv(y, Y);
#pragma unroll
    for (int f = 0; f < K2; ++f) lds[(fx * N2 + f) * zp + z] = Y[f];
  }
  __syncthreads();
  float2* __restrict__ Bb = P.b[s] + (long long)(p0 + pl) * ((long long)K1 * K2 * K3);
  for (int task = threadIdx.x; task < K2 * zg; task += TFMM_BLOCK) {
    const int z = task % zg, y = task / zg;
    float2 x[N1], X[K1];
#pragma unroll
    for (int i = 0; i < N1; ++i) x[i] = lds[(i * N2 + y) * zp + z];
    Dft<N1>::inv(x, X);
#pragma unroll
    for (int i = 0; i < K1; ++i) Bb[((long long)i * K2 + y) * K3 + z0 + z] = cscale(X[i], scale);
  }
}

static void xy_slab(int n1, int n2, int K3, int* zg, int* zp) {
  // largest divisor of K3 whose padded slab fits 64 KB of LDS
  int best = 1;
  for (int d = 1; d <= K3; ++d) {
    if (K3 % d) continue;
    int p = (d & 1) ? d : d + 1;
    if ((size_t)n1 * n2 * p * sizeof(float2) <= 65536) best = d;
  }
  *zg = best;
  *zp = (best & 1) ? best : best + 1;
}

#define TFMM_XY_SIZES(X) X(8) X(16) X(24) X(32) X(48) X(64)

template <int N1>
static bool dispatch_fwd_n2(int n2, const RhsPtrs& P, float2* H, int K3, int nrhs, int p0, int ndl,
                            hipStream_t st) {
  int zg, zp;
  switch (n2) {
#define CASE2(N2)                                                                                      \
  case N2: {                                                                                           \
    xy_slab(N1, N2, K3, &zg, &zp);                                                                     \
    size_t lds = (size_t)N1 * N2 * zp * sizeof(float2);                                                \
    hipLaunchKernelGGL((k_fwd_xy<N1, N2>), dim3(K3 / zg, ndl, nrhs), dim3(TFMM_BLOCK), lds, st, P, H, K3, \
                       zg, zp, ndl, p0);                                                               \
    return true;                                                                                       \
  }
    TFMM_XY_SIZES(CASE2)
#undef CASE2
  }
  return false;
}

template <int N1>
static bool dispatch_inv_n2(int n2, const RhsPtrs& P, const float2* H, int K3, int nrhs, int p0, int ndl,
                            float scale, hipStream_t st) {
  int zg, zp;
  switch (n2) {
#define CASE2(N2)                                                                                      \
  case N2: {                                                                                           \
    xy_slab(N1, N2, K3, &zg, &zp);                                                                     \
    size_t lds = (size_t)N1 * N2 * zp * sizeof(float2);                                                \
    hipLaunchKernelGGL((k_inv_xy<N1, N2>), dim3(K3 / zg, ndl, nrhs), dim3(TFMM_BLOCK), lds, st, P, H, K3, \
                       zg, zp, ndl, p0, scale);                                                        \
    return true;                                                                                       \
  }
    TFMM_XY_SIZES(CASE2)
#undef CASE2
  }
  return false;
}

hipError_t launch_fwd_xy(const RhsPtrs& P, float2* H, int n1, int n2, int K3, int nrhs, int p0, int ndl,
                         hipStream_t st, bool* supported) {
  bool ok = false;
  switch (n1) {
#define CASE1(N1) \
  case N1: ok = dispatch_fwd_n2<N1>(n2, P, H, K3, nrhs, p0, ndl, st); break;
    TFMM_XY_SIZES(CASE1)
#undef CASE1
  }
  *supported = ok;
  return ok ? hipGetLastError() : hipSuccess;
}

hipError_t launch_inv_xy(const RhsPtrs& P, const float2* H, int n1, int n2, int K3, int nrhs, int p0, int ndl,
                         float scale, hipStream_t st, bool* supported) {
  bool ok = false;
  switch (n1) {
#define CASE1(N1) \
  case N1: ok = dispatch_inv_n2<N1>(n2, P, H, K3, nrhs, p0, ndl, scale, st); break;
    TFMM_XY_SIZES(CASE1)
#undef CASE1
  }
  *supported = ok;
  return ok ? hipGetLastError() : hipSuccess;
}

// ---------------------------------------------------------------------------
// Pass 2: the z-stage.
//
// Accumulator layout (16x16x4 f32 MFMA, D[i][j] in lane j + 16*(i/4), reg i%4):
// real row R = 16 t + 4 g + r of row tile t maps to (fz, re/im) = (8t + 2g + r/2,
// r%2); column j of column block cb is pencil q0 + (w*CB + cb)*16 + j.  So lane
// (g, j) owns, for its pencil, the frequencies fz = 8t + b with b in {2g, 2g+1},
// t < T (n3 = 8T).  The pruned z-DFTs are split to match that ownership:
//   forward  X[8t+b] = DFT_T over v of  w^{vb} sum_{u<4} x[Tu+v] w8^{ub}
//   inverse  out[Tu'+v'] = sum_b w8^{-bu'} w^{-bv'} IDFT_T over t of Y[8t+b]
// (w = exp(-2 pi i/n3), w8 = exp(-2 pi i/8)); the inverse partial sums of the
// four lane groups are reduce-scattered with two cross-lane exchanges, after
// which lane group g holds out[z'] for z' in [T g, T g + T).
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

template <int T, int CB>
__device__ __forceinline__ void zstage_final_chunk(v4f (&acc)[T][CB], const float2* sV, const float2* sW, int KC,
                                                   int kc) {
  // acc[t][cb] += V'(16 real rows of tile t, chunk) x W'(chunk, 16 pencils of cb)
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
      float2 v = kok ? sV[fz * KC + k] : make_float2(0.f, 0.f);
      av[t] = ri == 0 ? (ki == 0 ? v.x : -v.y) : (ki == 0 ? v.y : v.x);
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int ql = (w * CB + c) * 16 + j;
      float2 v = kok ? sW[ql * KC + k] : make_float2(0.f, 0.f);
      bv[c] = ki == 0 ? v.x : v.y;
    }
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int c = 0; c < CB; ++c) acc[t][c] = mfma4(av[t], bv[c], acc[t][c]);
  }
}

template <int T, int CB>
__global__ __launch_bounds__(TFMM_BLOCK) void k_zstage(ZArgs a) {
  extern __shared__ float2 lds[];
  constexpr int QT = 64 * CB;
  constexpr int N3 = 8 * T, KZ = 4 * T;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, j = l & 15, g = l >> 4;
  const int tid = threadIdx.x;
  const int q0 = blockIdx.x * QT;
  const int pl = blockIdx.y, p = a.p0 + pl;
  const int nq = a.nq, n2 = a.n2;

  v4f acc[T][CB];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[t][c] = v4f{0.f, 0.f, 0.f, 0.f};

  if (a.fmt == ZF_FULL) {
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
    const int KC = a.KC;
    if (a.fmt == ZF_TUCKER) {
      const int r1 = d[4], r2 = d[5], r3 = d[6];
      const float2* C = a.cbase + d[0];
      const float2* U1 = a.fbase + d[1];
      const float2* U2 = a.fbase + d[2];
      const float2* U3 = a.fbase + d[3];
      const int nfx = QT / n2, fx0 = q0 / n2;
      // LDS carve-up (float2 offsets)
      const int oU1 = 0, oU2 = oU1 + nfx * r1, oC = oU2 + n2 * r2, oW1 = oC + r1 * r2 * KC,
                oW = oW1 + nfx * r2 * KC, oV = oW + QT * KC;
      for (int e = tid; e < nfx * r1; e += TFMM_BLOCK) lds[oU1 + e] = U1[fx0 * r1 + e];
      for (int e = tid; e < n2 * r2; e += TFMM_BLOCK) lds[oU2 + e] = U2[e];
      for (int c0 = 0; c0 < r3; c0 += KC) {
        const int kc = min(KC, r3 - c0);
        for (int e = tid; e < r1 * r2 * KC; e += TFMM_BLOCK) {
          const int cl = e % KC, ab = e / KC;
          lds[oC + e] = cl < kc ? C[(long long)ab * r3 + c0 + cl] : make_float2(0.f, 0.f);
        }
        for (int e = tid; e < N3 * KC; e += TFMM_BLOCK) {
          const int cl = e % KC, fz = e / KC;
          lds[oV + e] = cl < kc ? U3[fz * r3 + c0 + cl] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        // W1[fx][(b,cl)] = sum_a U1[fx][a] C[a][(b,cl)]                  (Fig. 3(a) step 1)
        block_cgemm(lds, nfx, r2 * KC, r1, 1, LOp{oU1, r1, 1, 0}, LOp{oC, r2 * KC, 1, 0},
                    LOp{oW1, r2 * KC, 1, 0});
        __syncthreads();
        // W[(fx,fy)][cl] = sum_b W1[fx][b][cl] U2[fy][b]                   (step 2), batch over cl
        block_cgemm(lds, nfx, n2, r2, kc, LOp{oW1, r2 * KC, KC, 1}, LOp{oU2, 1, r2, 0},
                    LOp{oW, n2 * KC, KC, 1});
        __syncthreads();
        // T~[fz][q] += sum_c U3[fz][c] W[q][c]                              (step 3)
        zstage_final_chunk<T, CB>(acc, lds + oV, lds + oW, KC, kc);
        __syncthreads();
      }
    } else if (a.fmt == ZF_TT3D) {
      const int r1 = d[4], r2 = d[5];
      const float2* C = a.cbase + d[0];
      const float2* U1 = a.fbase + d[1];
      const float2* U3 = a.fbase + d[3];
      const int nfx = QT / n2, fx0 = q0 / n2;
      const int oU1 = 0, oC = oU1 + nfx * r1, oW = oC + r1 * n2 * KC, oV = oW + QT * KC;
      for (int e = tid; e < nfx * r1; e += TFMM_BLOCK) lds[oU1 + e] = U1[fx0 * r1 + e];
      for (int b0 = 0; b0 < r2; b0 += KC) {
        const int kc = min(KC, r2 - b0);
        for (int e = tid; e < r1 * n2 * KC; e += TFMM_BLOCK) {
          const int bl = e % KC, ay = e / KC;
          lds[oC + e] = bl < kc ? C[(long long)ay * r2 + b0 + bl] : make_float2(0.f, 0.f);
        }
        for (int e = tid; e < N3 * KC; e += TFMM_BLOCK) {
          const int bl = e % KC, fz = e / KC;
          lds[oV + e] = bl < kc ? U3[fz * r2 + b0 + bl] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        // W[(fx,fy)][bl] = sum_a U1[fx][a] C[a][(fy,bl)]                   (Fig. 4(a) step 1)
        block_cgemm(lds, nfx, n2 * KC, r1, 1, LOp{oU1, r1, 1, 0}, LOp{oC, n2 * KC, 1, 0},
                    LOp{oW, n2 * KC, 1, 0});
        __syncthreads();
        zstage_final_chunk<T, CB>(acc, lds + oV, lds + oW, KC, kc);  // step 2
        __syncthreads();
      }
    } else {  // ZF_TT4D: W = T1 (direction-independent), V = S_p
      const int r2 = d[5];
      const float2* V = a.vbase + d[3];
      const int oW = 0, oV = QT * KC;
      for (int b0 = 0; b0 < r2; b0 += KC) {
        const int kc = min(KC, r2 - b0);
        for (int e = tid; e < QT * KC; e += TFMM_BLOCK) {
          const int bl = e % KC, ql = e / KC;
          const int q = q0 + ql;
          lds[oW + e] = (bl < kc && q < nq) ? a.wbase[(long long)q * r2 + b0 + bl] : make_float2(0.f, 0.f);
        }
        for (int e = tid; e < N3 * KC; e += TFMM_BLOCK) {
          const int bl = e % KC, fz = e / KC;
          lds[oV + e] = bl < kc ? V[fz * r2 + b0 + bl] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        zstage_final_chunk<T, CB>(acc, lds + oV, lds + oW, KC, kc);  // Fig. 4(b) step 2
        __syncthreads();
      }
    }
  }

  // ---- per-lane twiddles: tw[e][v] = w^{v b_e}, w8[u][e] = w8^{u b_e}, b_e = 2g + e
  float2 tw[2][T], w8[4][2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int b = 2 * g + e;
#pragma unroll
    for (int v = 0; v < T; ++v) tw[e][v] = a.roots[(v * b) % N3];
#pragma unroll
    for (int u = 0; u < 4; ++u) w8[u][e] = a.roots[(u * b * T) % N3];
  }

  const bool hi = g >= 2, odd = (g & 1) != 0;
  for (int s = 0; s < a.nrhs; ++s) {
    float2* Hs = a.H + ((long long)s * a.ndl + pl) * ((long long)a.K3 * nq);
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int q = q0 + (w * CB + c) * 16 + j;
      const bool qok = q < nq;
      float2 x[KZ];
#pragma unroll
      for (int z = 0; z < KZ; ++z) x[z] = qok ? Hs[(long long)z * nq + q] : make_float2(0.f, 0.f);
      float2 zt[2][T];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        float2 yv[T], X[T], Y[T], Z[T];
#pragma unroll
        for (int v = 0; v < T; ++v) {
          float2 sacc = x[v];
#pragma unroll
          for (int u = 1; u < 4; ++u) {
            const float2 m = cmul(x[T * u + v], w8[u][e]);
            sacc = cadd(sacc, m);
          }
          yv[v] = cmul(sacc, tw[e][v]);
        }
        dft_small_fwd<T>(yv, X);
#pragma unroll
        for (int t = 0; t < T; ++t) Y[t] = cmul(X[t], make_float2(acc[t][c][2 * e], acc[t][c][2 * e + 1]));
        dft_small_inv<T>(Y, Z);
#pragma unroll
        for (int v = 0; v < T; ++v) zt[e][v] = cmulconj(Z[v], tw[e][v]);
      }
      // partial[u][v] = sum_e zt[e][v] * conj(w8[u][e]); reduce-scatter over the 4 lane groups
      float2 kept[2][T];
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int v = 0; v < T; ++v) {
          const int ulo = k, uhi = 2 + k;
          const float2 plo = cadd(cmulconj(zt[0][v], w8[ulo][0]), cmulconj(zt[1][v], w8[ulo][1]));
          const float2 phi = cadd(cmulconj(zt[0][v], w8[uhi][0]), cmulconj(zt[1][v], w8[uhi][1]));
          const float2 keep = hi ? phi : plo;
          const float2 send = hi ? plo : phi;
          kept[k][v] = cadd(keep, shfl_xor2(send, 32));
        }
#pragma unroll
      for (int v = 0; v < T; ++v) {
        const float2 keep = odd ? kept[1][v] : kept[0][v];
        const float2 send = odd ? kept[0][v] : kept[1][v];
        const float2 out = cadd(keep, shfl_xor2(send, 16));
        if (qok) Hs[(long long)(T * g + v) * nq + q] = out;
      }
    }
  }
}

size_t zstage_lds_bytes(int fmt, int n1, int n2, int n3, int cb, int KC, int r1, int r2) {
  const int QT = 64 * cb, nfx = QT / n2;
  size_t e = 0;
  if (fmt == ZF_TUCKER)
    e = (size_t)nfx * r1 + (size_t)n2 * r2 + (size_t)r1 * r2 * KC + (size_t)nfx * r2 * KC + (size_t)QT * KC +
        (size_t)n3 * KC;
  else if (fmt == ZF_TT3D)
    e = (size_t)nfx * r1 + (size_t)r1 * n2 * KC + (size_t)QT * KC + (size_t)n3 * KC;
  else if (fmt == ZF_TT4D)
    e = (size_t)QT * KC + (size_t)n3 * KC;
  (void)n1;
  return e * sizeof(float2);
}

template <int T, int CB>
static hipError_t run_zstage(const ZArgs& a, hipStream_t st) {
  const size_t lds = (size_t)a.lds_bytes;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_zstage<T, CB>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  dim3 grid(a.nq / (64 * CB), a.ndl);
  hipLaunchKernelGGL((k_zstage<T, CB>), grid, dim3(TFMM_BLOCK), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_zstage(const ZArgs& a, hipStream_t st, bool* supported) {
  *supported = true;
  const int T = a.n3 / 8;
  switch (T * 10 + a.cb) {
#define ZC(TT, C) \
  case TT * 10 + C: return run_zstage<TT, C>(a, st);
    ZC(1, 1) ZC(1, 2) ZC(1, 3) ZC(1, 4)
    ZC(2, 1) ZC(2, 2) ZC(2, 3) ZC(2, 4)
    ZC(3, 1) ZC(3, 2) ZC(3, 3) ZC(3, 4)
    ZC(4, 1) ZC(4, 2) ZC(4, 3) ZC(4, 4)
    ZC(6, 1) ZC(6, 2) ZC(6, 3) ZC(6, 4)
    ZC(8, 1) ZC(8, 2) ZC(8, 3)
#undef ZC
  }
  *supported = false;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// a1: batched complex GEMM on global memory (one 8 x 16 complex tile per wave).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TFMM_BLOCK) void k_cgemm(int M, int N, int K, int nb, GOp A, GOp B, float2* C,
                                                      long long cs0, long long cs1, long long csb) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int tmN = (M + 7) >> 3, tnN = (N + 15) >> 4;
  const long long per = (long long)tmN * tnN;
  const long long tile = (long long)blockIdx.x * TFMM_NWAVES + w;
  if (tile >= per * nb) return;  // wave-uniform
  const int bat = (int)(tile / per);
  const int rem = (int)(tile - (long long)bat * per);
  const int tm = rem / tnN, tn = rem - tm * tnN;
  const int kofs = (l >> 4) >> 1, ki = (l >> 4) & 1, ari = l & 1;
  const int am = tm * 8 + ((l & 15) >> 1), bn = tn * 16 + (l & 15);
  const bool aok = am < M, bok = bn < N;
  const float2* ap = A.p + (long long)am * A.s0 + (long long)bat * A.sb;
  const float2* bp = B.p + (long long)bn * B.s1 + (long long)bat * B.sb;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  const int ks = (K + 1) >> 1;
  for (int s = 0; s < ks; ++s) {
    const int k = 2 * s + kofs;
    float av = 0.f, bv = 0.f;
    if (aok && k < K) {
      const float2 v = ap[(long long)k * A.s1];
      av = ari == 0 ? (ki == 0 ? v.x : -v.y) : (ki == 0 ? v.y : v.x);
    }
    if (bok && k < K) {
      const float2 v = bp[(long long)k * B.s0];
      bv = ki == 0 ? v.x : v.y;
    }
    acc = mfma4(av, bv, acc);
  }
  const int cn = tn * 16 + (l & 15), cm0 = tm * 8 + 2 * (l >> 4);
  if (cn < N) {
    float2* cp = C + (long long)cn * cs1 + (long long)bat * csb;
    if (cm0 < M) cp[(long long)cm0 * cs0] = make_float2(acc[0], acc[1]);
    if (cm0 + 1 < M) cp[(long long)(cm0 + 1) * cs0] = make_float2(acc[2], acc[3]);
  }
}

hipError_t launch_cgemm(int M, int N, int K, int nb, GOp A, GOp B, float2* C, long long cs0, long long cs1,
                        long long csb, hipStream_t st) {
  const long long tiles = (long long)((M + 7) / 8) * ((N + 15) / 16) * nb;
  const long long blocks = (tiles + TFMM_NWAVES - 1) / TFMM_NWAVES;
  hipLaunchKernelGGL(k_cgemm, dim3((unsigned)blocks), dim3(TFMM_BLOCK), 0, st, M, N, K, nb, A, B, C, cs0, cs1, csb);
  return hipGetLastError();
}

}  // namespace tfmm
