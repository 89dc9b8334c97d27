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
#include "tucker_restore.h"
#include "xy_stages.h"

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
// Pass 1 / pass 3 of the three-pass pipeline: xy-FFTs of a slab of zg
// z-planes per (rhs, direction); the half spectrum goes through device memory
// as H[rhs][dir][z][q] (pencil index q = fx*n2 + fy fastest).
// ---------------------------------------------------------------------------
template <int N1, int N2>
__global__ __launch_bounds__(TFMM_BLOCK) void k_fwd_xy(RhsPtrs P, float2* __restrict__ H, int K3, int zg, int zp,
                                                       int ndl, int p0, const int* __restrict__ perm,
                                                       const float2* __restrict__ twx) {
  extern __shared__ float2 lds[];
  constexpr int K1 = N1 / 2, K2 = N2 / 2, NQ = N1 * N2;
  const int s = blockIdx.z, pl = blockIdx.y, z0 = blockIdx.x * zg;
  const int p = perm ? perm[p0 + pl] : p0 + pl;
  const float2* __restrict__ Ab = P.a[s] + (long long)p * ((long long)K1 * K2 * K3);
  xy_forward<N1, N2, TFMM_BLOCK>(lds, Ab, K3, zg, zp, z0, twx);
  __syncthreads();
  float2* Hb = H + ((long long)s * ndl + pl) * ((long long)K3 * NQ) + (long long)z0 * NQ;
  for (int e = threadIdx.x; e < zg * NQ; e += TFMM_BLOCK) {
    const int z = e / NQ, q = e - z * NQ;
    Hb[e] = lds[q * zp + z];
  }
}

template <int N1, int N2>
__global__ __launch_bounds__(TFMM_BLOCK) void k_inv_xy(RhsPtrs P, const float2* __restrict__ H, int K3, int zg,
                                                       int zp, int ndl, int p0, const int* __restrict__ perm,
                                                       float scale, const float2* __restrict__ twx) {
  extern __shared__ float2 lds[];
  constexpr int K1 = N1 / 2, K2 = N2 / 2, NQ = N1 * N2;
  const int s = blockIdx.z, pl = blockIdx.y, z0 = blockIdx.x * zg;
  const float2* Hb = H + ((long long)s * ndl + pl) * ((long long)K3 * NQ) + (long long)z0 * NQ;
  for (int e = threadIdx.x; e < zg * NQ; e += TFMM_BLOCK) {
    const int z = e / NQ, q = e - z * NQ;
    lds[q * zp + z] = Hb[e];
  }
  __syncthreads();
  const int p = perm ? perm[p0 + pl] : p0 + pl;
  float2* __restrict__ Bb = P.b[s] + (long long)p * ((long long)K1 * K2 * K3);
  xy_inverse<N1, N2, TFMM_BLOCK>(lds, Bb, K3, zg, zp, z0, scale, twx);
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
#define TFMM_X_SIZES(X) X(8) X(16) X(24) X(32) X(48) X(64) X(128) X(256)

template <int N1>
static bool dispatch_fwd_n2(int n2, const RhsPtrs& P, float2* H, int K3, int nrhs, int p0, int ndl,
                            const int* perm, const float2* twx, hipStream_t st) {
  int zg, zp;
  switch (n2) {
#define CASE2(N2)                                                                                      \
  case N2: {                                                                                           \
    xy_slab(N1, N2, K3, &zg, &zp);                                                                     \
    size_t lds = (size_t)N1 * N2 * zp * sizeof(float2);                                                \
    hipLaunchKernelGGL((k_fwd_xy<N1, N2>), dim3(K3 / zg, ndl, nrhs), dim3(TFMM_BLOCK), lds, st, P, H, K3, \
                       zg, zp, ndl, p0, perm, twx);                                                    \
    return true;                                                                                       \
  }
    TFMM_XY_SIZES(CASE2)
#undef CASE2
  }
  return false;
}

template <int N1>
static bool dispatch_inv_n2(int n2, const RhsPtrs& P, const float2* H, int K3, int nrhs, int p0, int ndl,
                            const int* perm, float scale, const float2* twx, hipStream_t st) {
  int zg, zp;
  switch (n2) {
#define CASE2(N2)                                                                                      \
  case N2: {                                                                                           \
    xy_slab(N1, N2, K3, &zg, &zp);                                                                     \
    size_t lds = (size_t)N1 * N2 * zp * sizeof(float2);                                                \
    hipLaunchKernelGGL((k_inv_xy<N1, N2>), dim3(K3 / zg, ndl, nrhs), dim3(TFMM_BLOCK), lds, st, P, H, K3, \
                       zg, zp, ndl, p0, perm, scale, twx);                                             \
    return true;                                                                                       \
  }
    TFMM_XY_SIZES(CASE2)
#undef CASE2
  }
  return false;
}

hipError_t launch_fwd_xy(const RhsPtrs& P, float2* H, int n1, int n2, int K3, int nrhs, int p0, int ndl,
                         const int* perm, const float2* twx, hipStream_t st, bool* supported) {
  bool ok = false;
  switch (n1) {
#define CASE1(N1) \
  case N1: ok = dispatch_fwd_n2<N1>(n2, P, H, K3, nrhs, p0, ndl, perm, twx, st); break;
    TFMM_X_SIZES(CASE1)
#undef CASE1
  }
  *supported = ok;
  return ok ? hipGetLastError() : hipSuccess;
}

hipError_t launch_inv_xy(const RhsPtrs& P, const float2* H, int n1, int n2, int K3, int nrhs, int p0, int ndl,
                         const int* perm, float scale, const float2* twx, hipStream_t st, bool* supported) {
  bool ok = false;
  switch (n1) {
#define CASE1(N1) \
  case N1: ok = dispatch_inv_n2<N1>(n2, P, H, K3, nrhs, p0, ndl, perm, scale, twx, st); break;
    TFMM_X_SIZES(CASE1)
#undef CASE1
  }
  *supported = ok;
  return ok ? hipGetLastError() : hipSuccess;
}

__global__ void k_zero(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

hipError_t launch_zero(int* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// z-stage / fused dispatch to the per-family instantiations
// ---------------------------------------------------------------------------
hipError_t launch_zstage(const ZArgs& a, hipStream_t st, bool* supported) {
  switch (a.fmt) {
    case ZF_FULL: return launch_zstage_fmt<ZF_FULL>(a, st, supported);
    case ZF_TUCKER: return launch_zstage_fmt<ZF_TUCKER>(a, st, supported);
    case ZF_TT3D: return launch_zstage_fmt<ZF_TT3D>(a, st, supported);
    case ZF_TT4D: return launch_zstage_fmt<ZF_TT4D>(a, st, supported);
  }
  *supported = false;
  return hipSuccess;
}

hipError_t launch_fused(const ZArgs& a, const RhsPtrs& P, float scale, hipStream_t st, bool* supported) {
  switch (a.fmt) {
    case ZF_FULL: return launch_fused_fmt<ZF_FULL>(a, P, scale, st, supported);
    case ZF_TUCKER: return launch_fused_fmt<ZF_TUCKER>(a, P, scale, st, supported);
    case ZF_TT3D: return launch_fused_fmt<ZF_TT3D>(a, P, scale, st, supported);
    case ZF_TT4D: return launch_fused_fmt<ZF_TT4D>(a, P, scale, st, supported);
  }
  *supported = false;
  return hipSuccess;
}

size_t zstage_lds_bytes(int fmt, int n1, int n2, int n3, int qt, int KC, int r1, int r2) {
  const int nfx = qt / n2;
  size_t e = 0;
  if (fmt == ZF_TUCKER)
    e = (size_t)nfx * r1 + (size_t)n2 * r2 + (size_t)r1 * r2 * KC + (size_t)nfx * r2 * KC + (size_t)qt * KC +
        (size_t)n3 * KC;
  else if (fmt == ZF_TT3D)
    e = (size_t)nfx * r1 + (size_t)r1 * n2 * KC + (size_t)qt * KC + (size_t)n3 * KC;
  else if (fmt == ZF_TT4D)
    e = (size_t)qt * KC + (size_t)n3 * KC;
  (void)n1;
  return e * sizeof(float2);
}

size_t tucker2_lds_bytes(int n2, int n3, int qt, int r1, int r2, bool bf) {
  TuckerLds L;
  if (bf)
    L.plan<true>(qt / n2, n2, n3, r1, r2);
  else
    L.plan<false>(qt / n2, n2, n3, r1, r2);
  return (size_t)L.total * sizeof(float2);
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
