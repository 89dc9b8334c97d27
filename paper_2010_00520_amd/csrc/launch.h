// Host-side launch interface of the translation kernels (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace tfmm {

// Operator family seen by the z-stage kernel.
// ZF_TUCKER_W1: Tucker-family restoration whose first product, the x-mode
// product W1[fx][b][c] = sum_a U1[fx][a] C[a][b][c], was formed beforehand for
// a chunk of directions (the 4-D formats, whose per-direction cores are
// themselves formed per call); the z-stage starts from the second product.
enum ZFmt { ZF_FULL = 0, ZF_TUCKER = 1, ZF_TT3D = 2, ZF_TT4D = 3, ZF_TUCKER_W1 = 4 };

// Per-direction restoration descriptor (8 ints, float2 offsets):
//   Tucker : offC, offU1, offU2, offU3, r1, r2, r3, 0     (C may live in scratch)
//   TT-3D  : offC, offU1, 0, offU3, r1, r2, 0, 0
//   TT-4D  : 0, 0, 0, offV, 0, r2, 0, 0                    (V_p in scratch)
struct ZArgs {
  int fmt;
  int n1, n2, n3, K3, nq;
  int p0, nrhs, ndl;          // first direction, RHS count, directions in this launch
  float2* H;                  // x-FFT'ed planes G [nrhs][ndl][n1][n2/2][K3]
  const float4* Tfull;        // FULL: [n_dir][n3/2][nq] (consecutive fz pairs)
  const float2* cbase;        // cores (op data or scratch); ZF_TUCKER_W1: W1 of directions p0.. (scratch)
  long long w1dir;            // ZF_TUCKER_W1: W1 elements per direction (n1 r2 r3)
  const float2* fbase;        // factors (op data)
  const float2* wbase;        // TT-4D: T1 [nq][r2]; register-chained TT-3D: W_p [nq][r2_p] at desc[7] (scratch)
  const float2* vbase;        // TT-4D: V [n_dir][n3][r2] (scratch)
  const int* desc;            // [n_dir][8]
  const float2* roots;        // exp(-2 pi i m / n3), m < n3 (FP64-built, rounded)
  int KC;                     // complex contraction chunk
  int cb;                     // column blocks per wave (pencil tile = 64*cb)
  int lds_bytes;              // dynamic LDS of the launch (0 for FULL)
  int bf;                     // 1: split-BF16 (bf16x3) restoration, 0: FP32
  int tk2;                    // Tucker, TT-4D: 1 = register-chained restoration (tucker_restore.h)
  int rg;                     // three-pass z-stage: RHS per group (half spectra held in LDS)
  // persistent launch: work items are taken from counter[0], counter[1]
  // counts finished blocks (both zero between launches; the last block
  // resets them); direction order perm[] (costliest first, NULL = identity)
  const int* perm;
  int* counter;
  int ncu;                    // compute units of the device
};

// Dynamic LDS bytes a persistent launch adds past its working set (the
// work-item broadcast slot).
#define TFMM_LDS_SLOT 16

// LDS bytes a restoration of a qt-pencil tile needs for a format / ranks /
// chunk (host-side planning; qt = n1*n2 for the fused kernel).
size_t zstage_lds_bytes(int fmt, int n1, int n2, int n3, int qt, int KC, int r1, int r2);
// LDS of the three-pass z-stage's y- and z-stages (zstage_planes): the
// restored tile (64 cb pencils, rows of n3 + 1 complex) and the tile's half
// spectra of rg RHS at a time (rows of K3 | 1).
// With n3 <= 32 the tile moves into registers after a pass through LDS and its
// region is then reused for the half spectra (the larger of the two counts);
// a 48-point pencil with its transforms needs more than 256 vector registers,
// so longer pencils keep the tile in LDS.  Kernels whose whole item fits 256
// registers per lane without spilling (FULL and the restoration from a formed
// W1 up to n3 = 32, TT-4D up to n3 = 24, TT-3D at n3 = 8) are built for two
// waves per SIMD; the others for one.
__host__ __device__ constexpr bool zplanes_tile_in_regs(int T) { return T <= 4; }
__host__ __device__ constexpr int zplanes_waves_per_simd(int fmt, int T) {
  return !zplanes_tile_in_regs(T)                           ? 1
         : (fmt == ZF_FULL || fmt == ZF_TUCKER_W1)          ? 2
         : (fmt == ZF_TT4D && T <= 3) || (fmt == ZF_TT3D && T <= 1) ? 2
                                                              : 1;
}
inline size_t zplanes_lds_bytes(int n3, int cb, int rg) {
  const size_t qt = (size_t)64 * cb, kp = (size_t)((n3 / 2) | 1);
  const size_t tile = qt * (n3 + 1), half = (size_t)rg * qt * kp;
  return (zplanes_tile_in_regs(n3 / 8) ? std::max(tile, half) : tile + half) * 8;
}
// LDS bytes of the register-chained Tucker restoration of a qt-pencil tile.
size_t tucker2_lds_bytes(int n2, int n3, int qt, int r1, int r2, bool bf, bool w1 = false);
// LDS bytes of the TT-4D restoration with T1 read straight into MFMA operands
// (V_p of one direction, n3 x r2 in chunks of 8 columns).
size_t tt4d_chained_lds_bytes(int n3, int r2, bool bf);

// Per-RHS base pointers of one launch: rhs s reads A_s[n_dir][Kx][Ky][Kz] and
// writes B_s of the same shape (complex64).  Passed by value.
#define TFMM_MAX_RHS_PER_LAUNCH 32
struct RhsPtrs {
  const float2* a[TFMM_MAX_RHS_PER_LAUNCH];
  float2* b[TFMM_MAX_RHS_PER_LAUNCH];
};

// x passes of the three-pass pipeline (xpass.hip): G[s][d][fx][y][z] (y, z
// over the box grid; `lines` = Ky Kz) from A, and back to B with the crop and
// scale.  n1 in {8, ..., 64, 128, 256}; twx = exp(-2 pi i m / n1), m < n1, is
// read only when n1 > 64.  Direction p0 + d of the launch is perm[p0 + d]
// (perm NULL: p0 + d).
hipError_t launch_fwd_x(const RhsPtrs& P, float2* G, int n1, int lines, int nrhs, int p0, int ndl, const int* perm,
                        const float2* twx, hipStream_t st, bool* supported);
hipError_t launch_inv_x(const RhsPtrs& P, const float2* G, int n1, int lines, int nrhs, int p0, int ndl,
                        const int* perm, float scale, const float2* twx, hipStream_t st, bool* supported);
// Zero n ints (a kernel, so that it may be captured in a graph).
hipError_t launch_zero(int* p, int n, hipStream_t st);
hipError_t launch_zstage(const ZArgs& a, hipStream_t st, bool* supported);

// Fused single-kernel translation (one block per direction) for cubic grids
// n in {8, 16, 24, 32}; a.lds_bytes must cover both the restoration and the
// half spectrum n*n*(n/2 | 1) complex64.
hipError_t launch_fused(const ZArgs& a, const RhsPtrs& P, float scale, hipStream_t st, bool* supported);

// Per-family instantiations (zstage_<family>.hip).
template <int FMT>
hipError_t launch_zstage_fmt(const ZArgs& a, hipStream_t st, bool* supported);
template <int FMT>
hipError_t launch_fused_fmt(const ZArgs& a, const RhsPtrs& P, float scale, hipStream_t st, bool* supported);

// Batched complex GEMM on global memory: C_b[m][n] = sum_k A_b[m][k] B_b[k][n],
// element (i, j, b) of X at X.p + i*s0 + j*s1 + b*sb (float2 units).
struct GOp {
  const float2* p;
  long long s0, s1, sb;
};
// bf: split-BF16 products (bf16x3, FP32 accumulation), for operators restored
// in that arithmetic; otherwise FP32 MFMA.
hipError_t launch_cgemm(int M, int N, int K, int nb, GOp A, GOp B, float2* C, long long cs0, long long cs1,
                        long long csb, hipStream_t st, bool bf = false);
// While on (per thread), a GEMM shape without a measured tile configuration
// times them all on its stream and keeps the fastest (tfmm_autotune).
void set_gemm_tuning(bool on);
// TT-3D: W_p[q][b] = sum_a U1_p[fx][a] C_p[a][fy][b] for every direction p
// (q = fx n2 + fy; per-direction ranks from desc[8p + 4], desc[8p + 5]; W_p at
// wout + desc[8p + 7]); nmax = n2 * max r2.
hipError_t launch_cgemm_tt3d(int n1, int n2, int nmax, int nd, const int* desc, const float2* fbase, float2* wout,
                             bool bf, hipStream_t st);

// FP64 operator sampling, Eq. (7): T[p][m1][m2][m3] (double2) for every direction,
// wavenumber k = kre + i kim.
hipError_t launch_sample(double2* T, const double* khat, int ndir, const int K[3], double box, double kre,
                         double kim, int L, int near_rule, double near_param, double scale_re, double scale_im,
                         hipStream_t st);

// Setup permutations of complex128 tensors (setup_kernels.hip):
// out[c][r] = in[r][c] for a rows x cols matrix (rows <= 2^21);
hipError_t launch_transpose64(const double2* in, double2* out, long long rows, long long cols, hipStream_t st);
// [P][D][Q] -> [D][P][Q] (to_first) or back.
hipError_t launch_perm_mode(const double2* in, double2* out, long long P, long long D, long long Q, bool to_first,
                            hipStream_t st);

// Far-field matvec around the translation (farfield.hip): point-dipole
// patterns pat[p][n] = (theta.u, phi.u, Re e, Im e) from geo[n] = (r_n - r_v, u_n)
// in FP64 (Eq. (3)); aggregation A[2r+c][p][v] (Eq. (4)); projection
// y[r][orig(n)] (Eq. (6)); the near-field CSR product; precision conversions.
hipError_t launch_dipole_patterns(float4* pat, const double* khat, const double* geo, int N, int ndir, double kre,
                                  double kim, hipStream_t st);
hipError_t launch_aggregate(const float4* pat, const int* start, const int* orig, const float2* I, float2* A, int N,
                            int nbox, int ndir, int nrhs, hipStream_t st);
hipError_t launch_disaggregate(const float4* pat, const int* boxof, const int* orig, const float* w, const float2* B,
                               float2* y, int N, int nbox, int ndir, int nrhs, hipStream_t st);
hipError_t launch_near_spmv(const int* rp, const int* ci, const float2* val, const float2* x, float2* y, int n,
                            int nrhs, hipStream_t st);
hipError_t launch_narrow128(const double2* a, float2* b, int n, hipStream_t st);
hipError_t launch_widen(const float2* a, double2* b, int n, hipStream_t st);
hipError_t launch_sum_widen(const float2* a, const float2* c, double2* b, int n, hipStream_t st);

// Pack complex64 FULL operator [p][n1 n2 n3] into the [p][n3/2][nq] float4 layout.
hipError_t launch_pack_full(const float2* src, float4* dst, int ndir, int nq, int n3, hipStream_t st);

}  // namespace tfmm
