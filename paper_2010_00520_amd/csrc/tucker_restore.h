// Tucker-3D restoration of an operator tile straight into the z-stage
// accumulators (Fig. 3(a): x-mode, then y-mode, then z-mode products), with
// the y-mode product kept in registers:
//
//   W1[fx][c][b]   = sum_a U1[fx][a] C[a][b][c]          block-wide, via LDS
//   W[q][c]        = sum_b W1[fx(q)][c][b] U2[fy(q)][b]   per wave, in registers
//   T~[fz][q]     += sum_c U3[fz][c] W[q][c]              per wave, accumulators
//
// processed in chunks of 8 core columns c.  The second product's MFMA output
// tile (rows (c, re/im), columns = the wave's 16 pencils) already has the
// register layout of the third product's B operand, so W never touches LDS
// and each chunk needs only two block barriers.
//
// All operands sit in LDS "k-contiguous" (each row of a complex matrix holds
// consecutive values of the contraction index), zero-padded to whole K-steps,
// so fragment loads are unconditional.  Two arithmetics share the code:
//   FP32 : 16x16x4 f32 MFMA; a K-step is 2 complex k, lane group kg supplies
//          complex k0 + kg/2, component kg%2.
//   BF16X3: 16x16x32 bf16 MFMA on split operands (hi*hi + hi*lo + lo*hi); a
//          K-step is 16 complex k, lane group kg supplies complex k0+4kg..+3.
//          The third product has only 8 complex k (16 real) per chunk, so its
//          K-step instead concatenates hi and lo parts along k:
//          [A_hi, A_lo] . [W_hi; W_hi] + [A_hi, A_lo] . [W_lo; 0], two MFMAs.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "launch.h"

namespace tfmm {

template <bool BF>
struct Cx;

template <>
struct Cx<false> {
  static constexpr int KS = 2;  // complex k per K-step
  typedef float A;
  typedef float B;
  // p: the k-contiguous row at the step's first k.  A is real-embedded (row
  // ri): re for ri == ki, im otherwise, negated for (ri, ki) = (0, 1); one
  // 32-bit load and a sign flip.
  static __device__ __forceinline__ A load_a(const float2* p, int kg, int ri) {
    const float* f = reinterpret_cast<const float*>(p);
    const unsigned neg = (ri == 0 && (kg & 1)) ? 0x80000000u : 0u;
    return __uint_as_float(__float_as_uint(f[2 * (kg >> 1) + (ri ^ (kg & 1))]) ^ neg);
  }
  // stacked operand: component kg % 2 of complex kg / 2, i.e. float kg
  static __device__ __forceinline__ B load_b(const float2* p, int kg) {
    return reinterpret_cast<const float*>(p)[kg];
  }
  static __device__ __forceinline__ B zero_b() { return 0.f; }
  static __device__ __forceinline__ v4f mma(A a, B b, v4f c) { return mfma4(a, b, c); }
};

struct BfFrag {
  v4u hi, lo;
};

template <>
struct Cx<true> {
  static constexpr int KS = 16;
  typedef BfFrag A;
  typedef BfFrag B;
  // p + 4 kg starts a quartet (see stq): hi parts of its 4 k, then lo parts
  static __device__ __forceinline__ A load_a(const float2* p, int kg, int ri) {
    const uint4* q = reinterpret_cast<const uint4*>(p + 4 * kg);
    const uint4 x = q[0], y = q[1];
    A r;
    r.hi = v4u{embed_a_bf(x.x, ri), embed_a_bf(x.y, ri), embed_a_bf(x.z, ri), embed_a_bf(x.w, ri)};
    r.lo = v4u{embed_a_bf(y.x, ri), embed_a_bf(y.y, ri), embed_a_bf(y.z, ri), embed_a_bf(y.w, ri)};
    return r;
  }
  static __device__ __forceinline__ B load_b(const float2* p, int kg) {
    const v4u* q = reinterpret_cast<const v4u*>(p + 4 * kg);
    B r;
    r.hi = q[0];
    r.lo = q[1];
    return r;
  }
  static __device__ __forceinline__ B zero_b() {
    B r;
    r.hi = v4u{0u, 0u, 0u, 0u};
    r.lo = v4u{0u, 0u, 0u, 0u};
    return r;
  }
  static __device__ __forceinline__ v4f mma(A a, B b, v4f c) { return mfma_bf3(a.hi, a.lo, b.hi, b.lo, c); }
};

// Row stride (complex elements) of a k-contiguous operand with r valid k:
// padded to whole K-steps plus a skew (one element for FP32, two for the
// 16-byte split-BF16 loads) so the rows a fragment touches fall in
// different LDS banks.
template <bool BF>
__host__ __device__ __forceinline__ int tk_kpad(int r) {
  return BF ? (r + 15) & ~15 : (r + 1) & ~1;
}
template <bool BF>
__host__ __device__ __forceinline__ int tk_stride(int r) {
  return BF ? tk_kpad<BF>(r) + 2 : tk_kpad<BF>(r) + 1;
}
__host__ __device__ __forceinline__ int tk_align4(int e) { return (e + 3) & ~3; }

// Store of operand value v at position k of an LDS row (row start 16-byte
// aligned).  FP32: complex64 at row[k].  BF16X3: the row is cut into
// quartets of 4 k (32 bytes); a quartet holds the four split hi dwords, then
// the four lo dwords, so one K-step fragment is two 16-byte loads that land
// in the MFMA operand registers as they are.
template <bool BF>
__device__ __forceinline__ void stq(float2* row, int k, float2 v) {
  if constexpr (BF) {
    const uint2 h = split_bf3(v);
    unsigned* u = reinterpret_cast<unsigned*>(row) + 8 * (k >> 2) + (k & 3);
    u[0] = h.x;
    u[4] = h.y;
  } else {
    row[k] = v;
  }
}

// LDS layout (complex elements) of the Tucker restoration of a tile with nfx
// x-rows: U1 (FP32: embedded, two rows per x-row), U2, U3 columns of the
// chunk, C chunk (rows padded to an even number of b), W1 chunk.
struct TuckerLds {
  int s1, s2, fs, oU1, oU2, oV, oC, oW1, total;
  int oW1b, total_w1;  // restoration from a formed W1 (plan_w1): U2, V and two W1 buffers
  template <bool BF>
  __host__ __device__ __forceinline__ void plan(int nfx, int n2, int n3, int r1, int r2) {
    s1 = tk_stride<BF>(r1);
    s2 = tk_stride<BF>(r2);
    fs = 8 * s2 + 2;  // W1 x-row stride, skewed against the 16 x-rows of a GEMM tile
    oU1 = 0;
    oU2 = tk_align4(oU1 + (BF ? 1 : 2) * nfx * s1);
    oV = tk_align4(oU2 + n2 * s2);
    oC = tk_align4(oV + 8 * n3);
    oW1 = tk_align4(oC + 8 * (r2 + (r2 & 1)) * s1);
    total = tk_align4(oW1 + nfx * fs);
    oW1b = total;
    total_w1 = tk_align4(oW1b + nfx * fs);
  }
  // restoration from a formed W1: no U1 and no core chunk
  template <bool BF>
  __host__ __device__ __forceinline__ void plan_w1(int nfx, int n2, int n3, int r2) {
    s1 = 0;
    s2 = tk_stride<BF>(r2);
    fs = 8 * s2 + 2;
    oU1 = oC = 0;
    oU2 = 0;
    oV = tk_align4(oU2 + n2 * s2);
    oW1 = tk_align4(oV + 8 * n3);
    oW1b = tk_align4(oW1 + nfx * fs);
    total = total_w1 = tk_align4(oW1b + nfx * fs);
  }
};

// D0 += A . B0 and (if two) D1 += A . B1 over ks K-steps, A shared.  Steps
// are taken in blocks of U with every fragment load of a block issued before
// its MFMAs, so LDS latency overlaps the matrix-core work.
template <bool BF, int U, bool TWO>
__device__ __forceinline__ void tk_kloop(const float2* pa, const float2* pb0, const float2* pb1, int ks, v4f& D0,
                                         v4f& D1) {
  typedef Cx<BF> X;
  const int l = threadIdx.x & 63, kg = l >> 4, ri = l & 1;
  int s = 0;
  for (; s + U <= ks; s += U) {
    typename X::A av[U];
    typename X::B b0[U], b1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      av[u] = X::load_a(pa + (s + u) * X::KS, kg, ri);
      b0[u] = X::load_b(pb0 + (s + u) * X::KS, kg);
      if constexpr (TWO) b1[u] = X::load_b(pb1 + (s + u) * X::KS, kg);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      D0 = X::mma(av[u], b0[u], D0);
      if constexpr (TWO) D1 = X::mma(av[u], b1[u], D1);
    }
  }
  for (; s < ks; ++s) {
    const typename X::A av = X::load_a(pa + s * X::KS, kg, ri);
    D0 = X::mma(av, X::load_b(pb0 + s * X::KS, kg), D0);
    if constexpr (TWO) D1 = X::mma(av, X::load_b(pb1 + s * X::KS, kg), D1);
  }
}

// Same, both operands stacked (A rows hold plain (re, im) pairs): for the
// product whose embedded operand was prepared in LDS.
template <bool BF, int U, bool TWO>
__device__ __forceinline__ void tk_kloop_st(const float2* pa, const float2* pb0, const float2* pb1, int ks, v4f& D0,
                                            v4f& D1) {
  typedef Cx<BF> X;
  const int kg = (threadIdx.x & 63) >> 4;
  int s = 0;
  for (; s + U <= ks; s += U) {
    typename X::B av[U], b0[U], b1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      av[u] = X::load_b(pa + (s + u) * X::KS, kg);
      b0[u] = X::load_b(pb0 + (s + u) * X::KS, kg);
      if constexpr (TWO) b1[u] = X::load_b(pb1 + (s + u) * X::KS, kg);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      D0 = X::mma(av[u], b0[u], D0);
      if constexpr (TWO) D1 = X::mma(av[u], b1[u], D1);
    }
  }
  for (; s < ks; ++s) {
    const typename X::B av = X::load_b(pa + s * X::KS, kg);
    D0 = X::mma(av, X::load_b(pb0 + s * X::KS, kg), D0);
    if constexpr (TWO) D1 = X::mma(av, X::load_b(pb1 + s * X::KS, kg), D1);
  }
}

// Second product for one column block of 16 pencils (lane j owns pencil q_j
// with x-row fx_j of the tile and y-row fy_j).  A block whose pencils span
// two x-rows is done in two passes, each with the other row's lanes masked.
template <bool BF>
__device__ __forceinline__ v4f tk_wgemm(const float2* sW1, const float2* sU2, int s2, int fs, int ks2, int fxa, int fxb,
                                        int fxj, int fyj) {
  typedef Cx<BF> X;
  const int l = threadIdx.x & 63, kg = l >> 4, i = l & 15;
  v4f D = {0.f, 0.f, 0.f, 0.f};
  const float2* pb = sU2 + fyj * s2;
  for (int seg = fxa; seg <= fxb; ++seg) {
    const float2* pa = sW1 + seg * fs + (i >> 1) * s2;
    const bool mine = fxj == seg;
    for (int s = 0; s < ks2; ++s) {
      const typename X::A av = X::load_a(pa + s * X::KS, kg, i & 1);
      const typename X::B bv = mine ? X::load_b(pb + s * X::KS, kg) : X::zero_b();
      D = X::mma(av, bv, D);
    }
  }
  return D;
}

// Two column blocks with the same single x-row share the A fragments.
template <bool BF>
__device__ __forceinline__ void tk_wgemm2(const float2* sW1, const float2* sU2, int s2, int fs, int ks2, int fx, int fy0,
                                          int fy1, v4f& D0, v4f& D1) {
  const int i = threadIdx.x & 15;
  D0 = v4f{0.f, 0.f, 0.f, 0.f};
  D1 = v4f{0.f, 0.f, 0.f, 0.f};
  tk_kloop<BF, BF ? 1 : 4, true>(sW1 + fx * fs + (i >> 1) * s2, sU2 + fy0 * s2, sU2 + fy1 * s2, ks2, D0, D1);
}

// Core chunk source: element e = (a*r2 + b)*8 + cl  <-  C[a][b][c0 + cl],
// staged at LDS row 8b + cl, column a.  a = ab / r2 is taken as a multiply-
// high by m = ceil(2^32 / r2), exact for ab < 2^16 and r2 <= 64.
struct TkCoreSrc {
  const float2* C;
  int r2, r3;
  unsigned m;
  __device__ __forceinline__ float2 at(int e, int c0, int kc) const {
    const int cl = e & 7, ab = e >> 3;
    return cl < kc ? C[c0 + ab * r3 + cl] : make_float2(0.f, 0.f);
  }
  // LDS row (8b + cl) and column a of element e
  __device__ __forceinline__ int lds_row(int e, int& a) const {
    const int cl = e & 7, ab = e >> 3;
    a = (int)__umulhi((unsigned)ab, m);
    return 8 * (ab - a * r2) + cl;
  }
};

// N2C: the grid's n2 when the caller knows it at compile time (fused
// kernels), else 0.  With n2 a multiple of 32 every pair of 16-pencil blocks
// lies in one x-row, and the per-pair row test and its fallback drop out of
// the code (keeping the kernel's chunk loop within the instruction cache).
template <int T, int CB, int NW, bool BF, int N2C = 0>
__device__ __forceinline__ void restore_tucker(v4f (&acc)[T][CB], const ZArgs& a, const int* d, int q0,
                                               float2* lds) {
  typedef Cx<BF> X;
  // PF: core elements per thread of a staging part.  Parts are loaded behind
  // the column-block pairs of the second/third products; the 4-wave block has
  // few pairs, so its parts are larger (fewer of them wait at the chunk end).
  constexpr int NT = 64 * NW, QT = 16 * CB * NW, N3 = 8 * T, PF = NW >= 8 ? 4 : 8;
  constexpr bool kPairs = N2C > 0 && N2C % 32 == 0 && CB % 2 == 0;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, kg = l >> 4, i = l & 15, j = l & 15;
  const int n2 = N2C > 0 ? N2C : a.n2;
  const int r1 = d[4], r2 = d[5], r3 = d[6];
  const float2* C = a.cbase + d[0];
  const float2* U1 = a.fbase + d[1];
  const float2* U2 = a.fbase + d[2];
  const float2* U3 = a.fbase + d[3];
  const int nfx = QT / n2, fx0 = q0 / n2;
  TuckerLds L;
  L.plan<BF>(nfx, n2, N3, r1, r2);
  const int s1 = L.s1, s2 = L.s2, fs = L.fs, kp1 = tk_kpad<BF>(r1), kp2 = tk_kpad<BF>(r2);
  const int ks1 = kp1 / X::KS, ks2 = kp2 / X::KS;
  float2* sU1 = lds + L.oU1;
  float2* sU2 = lds + L.oU2;
  float2* sV = lds + L.oV;
  float2* sC = lds + L.oC;
  float2* sW1 = lds + L.oW1;

  // factors, and the zero padding of the C and W1 chunk rows (never rewritten)
  // FP32: U1 enters the first product as its embedded operand (row (fx, 0)
  // holds (re, -im), row (fx, 1) holds (im, re) of U1[fx][a]); bf16x3 keeps
  // it stacked and embeds the C^T fragments instead (measured faster there)
  for (int e = tid; e < nfx * kp1; e += NT) {
    const int fx = e / kp1, k = e - fx * kp1;
    const float2 u = k < r1 ? U1[(long long)(fx0 + fx) * r1 + k] : make_float2(0.f, 0.f);
    if constexpr (BF) {
      stq<BF>(sU1 + fx * s1, k, u);
    } else {
      stq<BF>(sU1 + 2 * fx * s1, k, make_float2(u.x, -u.y));
      stq<BF>(sU1 + (2 * fx + 1) * s1, k, make_float2(u.y, u.x));
    }
  }
  if (r2 & 1)  // the padding b = r2 of the C chunk rows
    for (int e = tid; e < 8 * kp1; e += NT) stq<BF>(sC + (8 * r2 + e / kp1) * s1, e % kp1, make_float2(0.f, 0.f));
  // U2 rows in batches of 4 per thread: the loads of a batch are in flight
  // together rather than one round trip per element
  for (int e0 = tid; e0 < n2 * kp2; e0 += 4 * NT) {
    float2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * NT, fy = e / kp2, k = e - fy * kp2;
      v[u] = (e < n2 * kp2 && k < r2) ? U2[fy * r2 + k] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * NT, fy = e / kp2, k = e - fy * kp2;
      if (e < n2 * kp2) stq<BF>(sU2 + fy * s2, k, v[u]);
    }
  }
  if (kp1 > r1)
    for (int e = tid; e < 8 * r2 * (kp1 - r1); e += NT) {
      const int row = e / (kp1 - r1);
      stq<BF>(sC + row * s1, r1 + (e - row * (kp1 - r1)), make_float2(0.f, 0.f));
    }
  if (kp2 > r2)
    for (int e = tid; e < 8 * nfx * (kp2 - r2); e += NT) {
      const int row = e / (kp2 - r2);
      stq<BF>(sW1 + (row >> 3) * fs + (row & 7) * s2, r2 + (e - row * (kp2 - r2)), make_float2(0.f, 0.f));
    }

  // Core chunks are staged through registers in parts of PF elements per
  // thread, one part in flight at a time: part 0 (with the U3 columns) is
  // loaded during the first product and stored after it; the later parts are
  // loaded and stored between column-block pairs of the second/third
  // products, so their latency hides behind matrix-core work.
  const TkCoreSrc src{C, r2, r3, (unsigned)(((1ull << 32) + (unsigned)r2 - 1) / (unsigned)r2)};
  const int csz = 8 * r2 * r1;
  constexpr int PART = PF * NT, VP = (8 * N3 + NT - 1) / NT;
  const int nparts = (csz + PART - 1) / PART;
  float px[PF], py[PF], vx[VP], vy[VP];
  // The element indices of a part do not change between chunks; `to` is made
  // opaque so the index arithmetic is redone per chunk rather than hoisted out
  // of the chunk loop into registers (which would spill).
  auto load_part = [&](int P, int c0) {
    const int kc = min(8, r3 - c0);
    int to = tid;
    asm volatile("" : "+v"(to));
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = P * PART + to + u * NT;
      const float2 v = e < csz ? src.at(e, c0, kc) : make_float2(0.f, 0.f);
      px[u] = v.x;
      py[u] = v.y;
    }
  };
  auto store_part = [&](int P) {
    int to = tid;
    asm volatile("" : "+v"(to));
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = P * PART + to + u * NT;
      if (e < csz) {
        int ka;
        const int row = src.lds_row(e, ka);
        stq<BF>(sC + row * s1, ka, make_float2(px[u], py[u]));
      }
    }
  };
  auto load_v = [&](int c0) {
    int to = tid;
    asm volatile("" : "+v"(to));
#pragma unroll
    for (int u = 0; u < VP; ++u) {
      const int e = to + u * NT, fz = e >> 3, cl = e & 7;
      const float2 v = (e < 8 * N3 && c0 + cl < r3) ? U3[fz * r3 + c0 + cl] : make_float2(0.f, 0.f);
      vx[u] = v.x;
      vy[u] = v.y;
    }
  };
  auto store_v = [&]() {
#pragma unroll
    for (int u = 0; u < VP; ++u) {
      const int e = tid + u * NT;
      if (e < 8 * N3) stq<BF>(sV + (e & ~7), e & 7, make_float2(vx[u], vy[u]));
    }
  };
  load_v(0);
  store_v();
  for (int P = 0; P < nparts; ++P) {
    load_part(P, 0);
    store_part(P);
  }
  __syncthreads();

  // third-product A fragments of the chunk: FP32 4 steps x 1 float; BF16X3
  // [hi(c0), hi(c1), lo(c0), lo(c1)] of the embedded U3 entries, c0 = 2kg
  float a3f[T][BF ? 1 : 4];
  v4u a3b[T];
  const int nch = (r3 + 7) >> 3;
  for (int h = 0; h < nch; ++h) {
    const int c0 = 8 * h;
    const bool more = h + 1 < nch;
    // lane indices made opaque per chunk (see load_part): fragment addresses
    // are recomputed rather than kept live across the chunk loop
    int lo = tid & 63;
    asm volatile("" : "+v"(lo));
    const int kg = lo >> 4, i = lo & 15, j = lo & 15;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int fz = 8 * t + (i >> 1), ri = i & 1;
      if constexpr (BF) {
        // c = 2kg, 2kg+1 of row fz: quartet kg/2, positions 2(kg%2), +1
        const uint2* pv = reinterpret_cast<const uint2*>(reinterpret_cast<const unsigned*>(sV + fz * 8) +
                                                         8 * (kg >> 1) + 2 * (kg & 1));
        const uint2 vh = pv[0], vl = pv[2];
        a3b[t] = v4u{embed_a_bf(vh.x, ri), embed_a_bf(vh.y, ri), embed_a_bf(vl.x, ri), embed_a_bf(vl.y, ri)};
      } else {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) a3f[t][s4] = embed_a(sV[fz * 8 + 2 * kg + (s4 >> 1)], ri, s4 & 1);
      }
    }
    if (more) {  // U3 columns first: nothing of theirs may wait behind the core loads
      load_v(c0 + 8);
      load_part(0, c0 + 8);
    }
    if constexpr (BF) {
      // first product, block-wide: W1^T[(b,cl)][fx] = sum_a C^T[(b,cl)][a] U1^T[a][fx];
      // a task is one b (8 rows of C^T) against up to two 16-column fx tiles
      {
        const int fxc0 = min(j, nfx - 1), fxc1 = min(16 + j, nfx - 1);
        const float2* pb0 = sU1 + fxc0 * s1;
        const float2* pb1 = sU1 + fxc1 * s1;
        auto put1 = [&](const v4f& D, int b) {
          if (j < nfx) {
            stq<BF>(sW1 + j * fs + 2 * kg * s2, b, make_float2(D[0], D[1]));
            stq<BF>(sW1 + j * fs + (2 * kg + 1) * s2, b, make_float2(D[2], D[3]));
          }
        };
        if (nfx > 16 || ks1 > 4) {
          for (int b = w; b < r2; b += NW) {
            const float2* pa = sC + (8 * b + (i >> 1)) * s1;
            v4f D0 = {0.f, 0.f, 0.f, 0.f}, D1 = {0.f, 0.f, 0.f, 0.f};
            if (nfx > 16)
              tk_kloop<BF, BF ? 1 : 4, true>(pa, pb0, pb1, ks1, D0, D1);
            else
              tk_kloop<BF, BF ? 1 : 4, false>(pa, pb0, pb1, ks1, D0, D1);
            put1(D0, b);
            if (16 + j < nfx) {
              stq<BF>(sW1 + (16 + j) * fs + 2 * kg * s2, b, make_float2(D1[0], D1[1]));
              stq<BF>(sW1 + (16 + j) * fs + (2 * kg + 1) * s2, b, make_float2(D1[2], D1[3]));
            }
          }
        } else {
          // one fx tile: its U1 fragments (at most 4 K-steps, r1 <= 64) are
          // the same for every b and stay in registers; two b per pass give
          // two independent accumulation chains
          typename X::B bu[4];
#pragma unroll
          for (int s = 0; s < 4; ++s)
            if (s < ks1) bu[s] = X::load_b(pb0 + s * X::KS, kg);
          const int ri = i & 1;
          int b = w;
          for (; b + NW < r2; b += 2 * NW) {
            const float2* pa0 = sC + (8 * b + (i >> 1)) * s1;
            const float2* pa1 = pa0 + 8 * NW * s1;
            typename X::A a0[4], a1[4];
#pragma unroll
            for (int s = 0; s < 4; ++s)
              if (s < ks1) {
                a0[s] = X::load_a(pa0 + s * X::KS, kg, ri);
                a1[s] = X::load_a(pa1 + s * X::KS, kg, ri);
              }
            v4f D0 = {0.f, 0.f, 0.f, 0.f}, D1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 4; ++s)
              if (s < ks1) {
                D0 = X::mma(a0[s], bu[s], D0);
                D1 = X::mma(a1[s], bu[s], D1);
              }
            put1(D0, b);
            put1(D1, b + NW);
          }
          if (b < r2) {
            const float2* pa0 = sC + (8 * b + (i >> 1)) * s1;
            v4f D0 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 4; ++s)
              if (s < ks1) D0 = X::mma(X::load_a(pa0 + s * X::KS, kg, ri), bu[s], D0);
            put1(D0, b);
          }
        }
      }
    } else {
      // first product, block-wide, with the small operand embedded:
      //   [Re, Im] W1^T[(b,cl)][fx] = sum_(a,ki) [Re, Im] C^T[(b,cl)][(a,ki)] . E(U1^T)[(a,ki)][(fx,comp)]
      // so the C^T fragments are loaded as they are.  A task is 16 rows of C^T
      // (two b) against up to two 16-column tiles of (fx, comp).  Lane (g, j)
      // ends with component j % 2 of four W1 entries; it swaps with lane j ^ 1 and
      // writes two complex values.
      {
        const int nrt = (r2 + 1) >> 1, nct = (nfx + 7) >> 3, ncp = (nct + 1) >> 1;
        const int comp = j & 1;
        for (int task = w; task < nrt * ncp; task += NW) {
          const int rt = task / ncp, ct0 = 2 * (task - rt * ncp), ct1 = min(ct0 + 1, nct - 1);
          const float2* pa = sC + (16 * rt + i) * s1;
          const int fxa = 8 * ct0 + (j >> 1), fxb = 8 * ct1 + (j >> 1);
          const float2* pb0 = sU1 + (2 * min(fxa, nfx - 1) + comp) * s1;
          const float2* pb1 = sU1 + (2 * min(fxb, nfx - 1) + comp) * s1;
          v4f D0 = {0.f, 0.f, 0.f, 0.f}, D1 = {0.f, 0.f, 0.f, 0.f};
          const bool two = (nct % 2 == 0) || ct0 + 1 < nct;  // even nct: ct0 <= nct - 2
          if (two)
            tk_kloop_st<BF, 4, true>(pa, pb0, pb1, ks1, D0, D1);
          else
            tk_kloop_st<BF, 4, false>(pa, pb0, pb1, ks1, D0, D1);
          auto put = [&](const v4f& D, int fx) {
            float o[4];
  #pragma unroll
            for (int r = 0; r < 4; ++r) o[r] = __shfl_xor(D[r], 1);
  #pragma unroll
            for (int rr = 0; rr < 2; ++rr) {
              const float own = comp ? D[2 + rr] : D[rr], oth = comp ? o[2 + rr] : o[rr];
              const int row = 4 * kg + 2 * comp + rr, b = 2 * rt + (row >> 3);
              if (fx < nfx && b < r2)
                stq<BF>(sW1 + fx * fs + (row & 7) * s2, b, comp ? make_float2(oth, own) : make_float2(own, oth));
            }
          };
          put(D0, fxa);
          if (two) put(D1, fxb);
        }
      }
    }
    __syncthreads();
    int part = 0;  // part of the next chunk currently in registers
    if (more) {
      store_part(0);
      store_v();
      if (++part < nparts) load_part(part, c0 + 8);
    }
    // second and third products, per wave
    auto finish = [&](int c, v4f D) {
      if constexpr (BF) {
        // [A_hi, A_lo] . [W_hi; W_hi] + [A_hi, A_lo] . [W_lo; 0]
        const uint2 e0 = split_bf3(make_float2(D[0], D[1])), e1 = split_bf3(make_float2(D[2], D[3]));
        const v4u bh = v4u{e0.x, e1.x, e0.x, e1.x}, bl = v4u{e0.y, e1.y, 0u, 0u};
#pragma unroll
        for (int t = 0; t < T; ++t) {
          acc[t][c] = mfma_bf16(a3b[t], bh, acc[t][c]);
          acc[t][c] = mfma_bf16(a3b[t], bl, acc[t][c]);
        }
      } else {
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) acc[t][c] = mfma4(a3f[t][s4], D[s4], acc[t][c]);
      }
    };
#pragma unroll
    for (int c = 0; c < CB; c += 2) {
      if constexpr (kPairs) {
        // blocks c, c+1 are 32 consecutive pencils starting on a multiple of 32
        const int qb = q0 + (w * CB + c) * 16, fx = qb / n2 - fx0, fy = qb - (qb / n2) * n2 + j;
        v4f D0, D1;
        tk_wgemm2<BF>(sW1, sU2, s2, L.fs, ks2, fx, fy, fy + 16, D0, D1);
        finish(c, D0);
        finish(c + 1, D1);
        if (more && part < nparts) {
          store_part(part);
          if (++part < nparts) load_part(part, c0 + 8);
        }
        continue;
      }
      // pencils of blocks c and c+1: x-row of lane 0 (fa), of lane 15 (fb); a
      // block spans at most two x-rows since n2 >= 8
      int fa[2], fb[2], fxj[2], fyj[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int qb = q0 + (w * CB + min(c + u, CB - 1)) * 16;
        const int xa = qb / n2, off = qb - xa * n2 + j, wrap = off >= n2 ? 1 : 0;
        fa[u] = xa - fx0;
        fb[u] = (qb + 15) / n2 - fx0;
        fxj[u] = fa[u] + wrap;
        fyj[u] = off - wrap * n2;
      }
      if (c + 1 < CB && fa[0] == fb[0] && fa[1] == fb[1] && fa[0] == fa[1]) {
        v4f D0, D1;
        tk_wgemm2<BF>(sW1, sU2, s2, L.fs, ks2, fa[0], fyj[0], fyj[1], D0, D1);
        finish(c, D0);
        finish(c + 1, D1);
      } else {
        finish(c, tk_wgemm<BF>(sW1, sU2, s2, L.fs, ks2, fa[0], fb[0], fxj[0], fyj[0]));
        if (c + 1 < CB) finish(c + 1, tk_wgemm<BF>(sW1, sU2, s2, L.fs, ks2, fa[1], fb[1], fxj[1], fyj[1]));
      }
      if (more && part < nparts) {
        store_part(part);
        if (++part < nparts) load_part(part, c0 + 8);
      }
    }
    while (more && part < nparts) {
      store_part(part);
      if (++part < nparts) load_part(part, c0 + 8);
    }
    __syncthreads();
  }
}

// Restoration from a formed x-mode product W1[fx][b][c] (ZF_TUCKER_W1, the
// 4-D formats on the three-pass path): only the second and third products run
// here.  W1 chunks of 8 columns c alternate between two LDS buffers, the next
// chunk staged while the current one feeds the second product.  The split of
// (fx, b) by r2 is a multiply-high by ceil(2^32 / r2), exact for fx * r2 + b <
// 2^16 and r2 <= 512.
template <int T, int CB, int NW, bool BF>
__device__ __forceinline__ void restore_tucker_w1(v4f (&acc)[T][CB], const ZArgs& a, const int* d, int p, int q0,
                                                  float2* lds) {
  typedef Cx<BF> X;
  constexpr int NT = 64 * NW, QT = 16 * CB * NW, N3 = 8 * T, PF = 8;
  const int tid = threadIdx.x, w = tid >> 6;
  const int n2 = a.n2;
  const int r2 = d[5], r3 = d[6];
  const float2* W1g = a.cbase + (long long)(p - a.p0) * a.w1dir;  // [fx][b][c]
  const float2* U2 = a.fbase + d[2];
  const float2* U3 = a.fbase + d[3];
  const int nfx = QT / n2, fx0 = q0 / n2;
  TuckerLds L;
  L.plan_w1<BF>(nfx, n2, N3, r2);
  const int s2 = L.s2, fs = L.fs, kp2 = tk_kpad<BF>(r2);
  const int ks2 = kp2 / X::KS;
  float2* sU2 = lds + L.oU2;
  float2* sV = lds + L.oV;
  float2* sWa = lds + L.oW1;
  float2* sWb = lds + L.oW1b;

  for (int e0 = tid; e0 < n2 * kp2; e0 += 4 * NT) {
    float2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * NT, fy = e / kp2, k = e - fy * kp2;
      v[u] = (e < n2 * kp2 && k < r2) ? U2[fy * r2 + k] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * NT, fy = e / kp2, k = e - fy * kp2;
      if (e < n2 * kp2) stq<BF>(sU2 + fy * s2, k, v[u]);
    }
  }
  if (kp2 > r2)  // zero padding k = r2 .. kp2 - 1 of the W1 rows of both buffers (never rewritten)
    for (int e = tid; e < 2 * 8 * nfx * (kp2 - r2); e += NT) {
      const int row = e / (kp2 - r2), k = r2 + (e - row * (kp2 - r2));
      float2* sw = row < 8 * nfx ? sWa : sWb;
      const int rr = row < 8 * nfx ? row : row - 8 * nfx;
      stq<BF>(sw + (rr >> 3) * fs + (rr & 7) * s2, k, make_float2(0.f, 0.f));
    }

  // W1 chunk element e = (fx * r2 + b) * 8 + cl  <-  W1[fx0 + fx][b][c0 + cl]
  // (eight consecutive c of one (fx, b) are one contiguous run)
  const int wsz = nfx * 8 * r2;
  const unsigned m1 = (unsigned)(((1ull << 32) + (unsigned)r2 - 1) / (unsigned)r2);
  constexpr int PART = PF * NT, VP = (8 * N3 + NT - 1) / NT;
  const int nparts = (wsz + PART - 1) / PART;
  float px[PF], py[PF], vx[VP], vy[VP];
  auto split_e = [&](int e, int& fx, int& cl, int& b) {
    const int fb = e >> 3;
    cl = e & 7;
    fx = (int)__umulhi((unsigned)fb, m1);
    b = fb - fx * r2;
  };
  auto load_w = [&](int P, int c0) {
    const int kc = min(8, r3 - c0);
    int to = tid;
    asm volatile("" : "+v"(to));
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = P * PART + to + u * NT;
      int fx, cl, b;
      split_e(e, fx, cl, b);
      const float2 v = (e < wsz && cl < kc) ? W1g[((long long)fx0 * r2 + (e >> 3)) * r3 + c0 + cl]
                                            : make_float2(0.f, 0.f);
      px[u] = v.x;
      py[u] = v.y;
    }
  };
  auto store_w = [&](int P, float2* sw) {
    int to = tid;
    asm volatile("" : "+v"(to));
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = P * PART + to + u * NT;
      if (e < wsz) {
        int fx, cl, b;
        split_e(e, fx, cl, b);
        stq<BF>(sw + fx * fs + cl * s2, b, make_float2(px[u], py[u]));
      }
    }
  };
  auto load_v = [&](int c0) {
    int to = tid;
    asm volatile("" : "+v"(to));
#pragma unroll
    for (int u = 0; u < VP; ++u) {
      const int e = to + u * NT, fz = e >> 3, cl = e & 7;
      const float2 v = (e < 8 * N3 && c0 + cl < r3) ? U3[fz * r3 + c0 + cl] : make_float2(0.f, 0.f);
      vx[u] = v.x;
      vy[u] = v.y;
    }
  };
  auto store_v = [&]() {
#pragma unroll
    for (int u = 0; u < VP; ++u) {
      const int e = tid + u * NT;
      if (e < 8 * N3) stq<BF>(sV + (e & ~7), e & 7, make_float2(vx[u], vy[u]));
    }
  };
  load_v(0);
  store_v();
  for (int P = 0; P < nparts; ++P) {
    load_w(P, 0);
    store_w(P, sWa);
  }
  __syncthreads();

  float a3f[T][BF ? 1 : 4];
  v4u a3b[T];
  const int nch = (r3 + 7) >> 3;
  for (int h = 0; h < nch; ++h) {
    const int c0 = 8 * h;
    const bool more = h + 1 < nch;
    const float2* cur = (h & 1) ? sWb : sWa;
    float2* nxt = (h & 1) ? sWa : sWb;
    int lo = tid & 63;
    asm volatile("" : "+v"(lo));
    const int kg = lo >> 4, i = lo & 15, j = lo & 15;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int fz = 8 * t + (i >> 1), ri = i & 1;
      if constexpr (BF) {
        const uint2* pv = reinterpret_cast<const uint2*>(reinterpret_cast<const unsigned*>(sV + fz * 8) +
                                                         8 * (kg >> 1) + 2 * (kg & 1));
        const uint2 vh = pv[0], vl = pv[2];
        a3b[t] = v4u{embed_a_bf(vh.x, ri), embed_a_bf(vh.y, ri), embed_a_bf(vl.x, ri), embed_a_bf(vl.y, ri)};
      } else {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) a3f[t][s4] = embed_a(sV[fz * 8 + 2 * kg + (s4 >> 1)], ri, s4 & 1);
      }
    }
    if (more) {
      load_v(c0 + 8);
      load_w(0, c0 + 8);
    }
    __syncthreads();  // every wave holds its U3 fragments: sV may be rewritten
    int part = 0;     // part of the next chunk currently in registers
    if (more) {
      store_w(0, nxt);
      store_v();
      if (++part < nparts) load_w(part, c0 + 8);
    }
    auto finish = [&](int c, v4f D) {
      if constexpr (BF) {
        const uint2 e0 = split_bf3(make_float2(D[0], D[1])), e1 = split_bf3(make_float2(D[2], D[3]));
        const v4u bh = v4u{e0.x, e1.x, e0.x, e1.x}, bl = v4u{e0.y, e1.y, 0u, 0u};
#pragma unroll
        for (int t = 0; t < T; ++t) {
          acc[t][c] = mfma_bf16(a3b[t], bh, acc[t][c]);
          acc[t][c] = mfma_bf16(a3b[t], bl, acc[t][c]);
        }
      } else {
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) acc[t][c] = mfma4(a3f[t][s4], D[s4], acc[t][c]);
      }
    };
#pragma unroll
    for (int c = 0; c < CB; c += 2) {
      int fa[2], fb[2], fxj[2], fyj[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int qb = q0 + (w * CB + min(c + u, CB - 1)) * 16;
        const int xa = qb / n2, off = qb - xa * n2 + j, wrap = off >= n2 ? 1 : 0;
        fa[u] = xa - fx0;
        fb[u] = (qb + 15) / n2 - fx0;
        fxj[u] = fa[u] + wrap;
        fyj[u] = off - wrap * n2;
      }
      if (c + 1 < CB && fa[0] == fb[0] && fa[1] == fb[1] && fa[0] == fa[1]) {
        v4f D0, D1;
        tk_wgemm2<BF>(cur, sU2, s2, fs, ks2, fa[0], fyj[0], fyj[1], D0, D1);
        finish(c, D0);
        finish(c + 1, D1);
      } else {
        finish(c, tk_wgemm<BF>(cur, sU2, s2, fs, ks2, fa[0], fb[0], fxj[0], fyj[0]));
        if (c + 1 < CB) finish(c + 1, tk_wgemm<BF>(cur, sU2, s2, fs, ks2, fa[1], fb[1], fxj[1], fyj[1]));
      }
      if (more && part < nparts) {
        store_w(part, nxt);
        if (++part < nparts) load_w(part, c0 + 8);
      }
    }
    while (more && part < nparts) {
      store_w(part, nxt);
      if (++part < nparts) load_w(part, c0 + 8);
    }
    __syncthreads();  // the next chunk is staged; this one is no longer read
  }
}

// TT restoration T~_p[fz][q] = sum_k V[fz][k] W[q][k] with W read straight
// into MFMA B operands: TT-4D (Fig. 4(b)) with V = V_p (a1) and W = T1, the
// direction-independent x-y product; TT-3D (Fig. 4(a)) with V = U3_p and W =
// W_p, the per-direction x-y product formed ahead of the z-stage.  V (n3 x r2)
// is staged once in LDS in chunks of 8 columns k (the layout of the Tucker
// third product's A operand); per chunk, lane (kg, j) of column block c loads
// W[q_j][8h + 2kg .. + 1] from device memory, which is exactly the B fragment
// the Tucker third product takes from its second product.  No LDS staging of
// W and no block barrier inside the chunk loop.
template <bool BF>
__host__ __device__ __forceinline__ int tt4d_chained_lds_elems(int n3, int r2) {
  return ((r2 + 7) >> 3) * 8 * n3;
}

template <int T, int CB, int NW, bool BF>
__device__ __forceinline__ void restore_tt_chained(v4f (&acc)[T][CB], const ZArgs& a, int r2, const float2* V,
                                                   const float2* T1, int q0, float2* lds) {
  constexpr int NT = 64 * NW, N3 = 8 * T;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, kg = l >> 4, i = l & 15, j = l & 15;
  const int nch = (r2 + 7) >> 3;
  // V: [n3][r2]; T1 (W): [nq][r2]
  // sV chunk h, row fz: the 8 columns k = 8h .. 8h + 7 (zero past r2); loads
  // in batches of 4 per thread
  const int vsz = nch * 8 * N3;
  for (int e0 = tid; e0 < vsz; e0 += 4 * NT) {
    float2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * NT, h = e / (8 * N3), rem = e - h * 8 * N3, fz = rem >> 3, k = 8 * h + (rem & 7);
      v[u] = (e < vsz && k < r2) ? V[fz * r2 + k] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * NT, h = e / (8 * N3), rem = e - h * 8 * N3;
      if (e < vsz) stq<BF>(lds + h * 8 * N3 + (rem >> 3) * 8, rem & 7, v[u]);
    }
  }
  __syncthreads();
  const float2* rows[CB];
  bool ok[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int q = q0 + (w * CB + c) * 16 + j;
    ok[c] = q < a.nq;
    rows[c] = T1 + (long long)(ok[c] ? q : 0) * r2;
  }
  auto load_b = [&](int h, float2 (&b)[CB][2]) {
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int k = 8 * h + 2 * kg + u;
        b[c][u] = (ok[c] && k < r2) ? rows[c][k] : make_float2(0.f, 0.f);
      }
  };
  float2 bcur[CB][2], bnxt[CB][2];
  load_b(0, bcur);
  for (int h = 0; h < nch; ++h) {
    if (h + 1 < nch) load_b(h + 1, bnxt);
    const float2* sV = lds + h * 8 * N3;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int fz = 8 * t + (i >> 1), ri = i & 1;
      if constexpr (BF) {
        const uint2* pv = reinterpret_cast<const uint2*>(reinterpret_cast<const unsigned*>(sV + fz * 8) +
                                                         8 * (kg >> 1) + 2 * (kg & 1));
        const uint2 vh = pv[0], vl = pv[2];
        const v4u a3 = v4u{embed_a_bf(vh.x, ri), embed_a_bf(vh.y, ri), embed_a_bf(vl.x, ri), embed_a_bf(vl.y, ri)};
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          // [A_hi, A_lo] . [B_hi; B_hi] + [A_hi, A_lo] . [B_lo; 0]
          const uint2 e0 = split_bf3(bcur[c][0]), e1 = split_bf3(bcur[c][1]);
          acc[t][c] = mfma_bf16(a3, v4u{e0.x, e1.x, e0.x, e1.x}, acc[t][c]);
          acc[t][c] = mfma_bf16(a3, v4u{e0.y, e1.y, 0u, 0u}, acc[t][c]);
        }
      } else {
        float a3[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) a3[s4] = embed_a(sV[fz * 8 + 2 * kg + (s4 >> 1)], ri, s4 & 1);
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          acc[t][c] = mfma4(a3[0], bcur[c][0].x, acc[t][c]);
          acc[t][c] = mfma4(a3[1], bcur[c][0].y, acc[t][c]);
          acc[t][c] = mfma4(a3[2], bcur[c][1].x, acc[t][c]);
          acc[t][c] = mfma4(a3[3], bcur[c][1].y, acc[t][c]);
        }
      }
    }
    if (h + 1 < nch) {
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        bcur[c][0] = bnxt[c][0];
        bcur[c][1] = bnxt[c][1];
      }
    }
  }
}

}  // namespace tfmm
