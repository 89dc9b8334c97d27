// Device-side FP64 setup of the FFT'ed operator (Section II-B): the 3-D FFT of
// the sampled operator (hipFFT), and the compression of the 4-D formats
// (Algorithms 1-3 on X4[x][y][z][p]) with Gram matrices and projections on the
// FP64 matrix cores (rocBLAS zherk / zgemm) and Hermitian eigensolves on the
// device (rocSOLVER zheevd).  Only the rank choices and the small product
// forming the H-Tucker root run on the host.
//
// Truncation is the same as the host compressors': the smallest rank whose
// discarded eigenvalues of the Gram matrix (squared singular values) sum to at
// most the tail budget, with 4 eps lambda_max charged per discarded value for
// the eigenvalue error of the Gram approach.
#include "setup_gpu.h"

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "launch.h"

namespace tfmm {

namespace {

struct DevBuf {
  double2* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  bool alloc(size_t count) {
    release();
    if (count == 0) return true;
    if (hipMalloc(&p, count * sizeof(double2)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return false;
    }
    n = count;
    return true;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void swap(DevBuf& o) {
    std::swap(p, o.p);
    std::swap(n, o.n);
  }
};

struct Linalg {
  rocblas_handle h = nullptr;
  hipStream_t st = nullptr;
  std::string err;
  Linalg(hipStream_t s) : st(s) {
    if (rocblas_create_handle(&h) != rocblas_status_success) {
      err = "rocblas_create_handle failed";
      h = nullptr;
      return;
    }
    (void)rocblas_set_stream(h, st);
    (void)rocblas_set_pointer_mode(h, rocblas_pointer_mode_host);
  }
  ~Linalg() {
    if (h) (void)rocblas_destroy_handle(h);
  }
  bool check(rocblas_status s, const char* what) {
    if (s != rocblas_status_success && err.empty()) err = std::string(what) + " failed (rocblas status " +
                                                          std::to_string((int)s) + ")";
    return err.empty();
  }
  bool hip(hipError_t e, const char* what) {
    if (e != hipSuccess && err.empty()) err = std::string(what) + ": " + hipGetErrorString(e);
    return err.empty();
  }
};

inline rocblas_double_complex* rb(double2* p) { return reinterpret_cast<rocblas_double_complex*>(p); }
inline const rocblas_double_complex* rb(const double2* p) {
  return reinterpret_cast<const rocblas_double_complex*>(p);
}

double norm2_dev(Linalg& L, const double2* x, long long n) {
  double r = 0.0;
  if (!L.check(rocblas_dznrm2_64(L.h, n, rb(x), 1, &r), "rocblas_dznrm2")) return 0.0;
  return r * r;
}

// Eigen-decomposition of the Hermitian D x D device matrix H (column-major,
// upper triangle significant; overwritten).  vals: descending; vecs: host,
// column-major, column j = eigenvector of vals[j].
bool eig_desc(Linalg& L, double2* H, int D, std::vector<double>& vals, std::vector<cd>& vecs) {
  double *dW = nullptr, *dE = nullptr;
  int* dinfo = nullptr;
  bool ok = L.hip(hipMalloc(&dW, D * sizeof(double)), "hipMalloc") &&
            L.hip(hipMalloc(&dE, D * sizeof(double)), "hipMalloc") &&
            L.hip(hipMalloc(&dinfo, sizeof(int)), "hipMalloc");
  ok = ok && L.check(rocsolver_zheevd(L.h, rocblas_evect_original, rocblas_fill_upper, D, rb(H), D, dW, dE, dinfo),
                     "rocsolver_zheevd");
  std::vector<double> w(D);
  std::vector<cd> v((size_t)D * D);
  int info = 0;
  ok = ok && L.hip(hipMemcpyAsync(w.data(), dW, D * sizeof(double), hipMemcpyDeviceToHost, L.st), "copy") &&
       L.hip(hipMemcpyAsync(v.data(), H, (size_t)D * D * sizeof(double2), hipMemcpyDeviceToHost, L.st), "copy") &&
       L.hip(hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, L.st), "copy") &&
       L.hip(hipStreamSynchronize(L.st), "sync");
  if (dW) (void)hipFree(dW);
  if (dE) (void)hipFree(dE);
  if (dinfo) (void)hipFree(dinfo);
  if (!ok) return false;
  if (info != 0) {
    L.err = "rocsolver_zheevd did not converge (info " + std::to_string(info) + ")";
    return false;
  }
  vals.resize(D);
  vecs.resize((size_t)D * D);
  for (int j = 0; j < D; ++j) {  // ascending -> descending
    const int s = D - 1 - j;
    vals[j] = w[s];
    std::copy(v.begin() + (size_t)s * D, v.begin() + (size_t)(s + 1) * D, vecs.begin() + (size_t)j * D);
  }
  return true;
}

int rank_of(const std::vector<double>& vals, double budget2) {
  const double lmax = vals.empty() ? 0.0 : std::max(0.0, vals[0]);
  return truncation_rank(vals, budget2, 4.0 * 2.2e-16 * lmax);
}

// Y (r x M, row-major) = U^H X for X row-major D x M and U row-major D x r (device).
bool project_first(Linalg& L, const double2* X, int D, long long M, const double2* U, int r, double2* Y) {
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  return L.check(rocblas_zgemm_64(L.h, rocblas_operation_none, rocblas_operation_conjugate_transpose, M, r, D, &one,
                                  rb(X), M, rb(U), r, &zero, rb(Y), M),
                 "rocblas_zgemm");
}

// Truncated left singular basis of a row-major m x n device matrix M (Algorithm
// 1/3 step): U (host, m x r row-major) and the carry U^H M (device, r x n).
// m <= n: eigenvectors of M M^H.  m > n: eigenvectors V of M^H M, U = M V S^-1
// and carry = S V^H (the truncated product U carry = M V V^H either way).
bool svd_left(Linalg& L, const double2* M, int m, long long n, double budget2, std::vector<cd>& U, int& r,
              DevBuf& carry) {
  const double one = 1.0, zero = 0.0;
  std::vector<double> vals;
  std::vector<cd> vecs;
  if ((long long)m <= n) {
    DevBuf H;
    if (!H.alloc((size_t)m * m)) return L.hip(hipErrorOutOfMemory, "Gram buffer");
    // column-major H = A^H A with A the column-major n x m view of M: H = conj(M M^H)
    if (!L.check(rocblas_zherk_64(L.h, rocblas_fill_upper, rocblas_operation_conjugate_transpose, m, n, &one, rb(M),
                                  n, &zero, rb(H.p), m),
                 "rocblas_zherk"))
      return false;
    if (!eig_desc(L, H.p, m, vals, vecs)) return false;
    r = rank_of(vals, budget2);
    // eigenvectors of conj(M M^H) are the conjugates of M's left singular vectors
    U.assign((size_t)m * r, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < r; ++j) U[(size_t)i * r + j] = std::conj(vecs[(size_t)j * m + i]);
    DevBuf Ud;
    if (!Ud.alloc(U.size()) || !carry.alloc((size_t)r * n)) return L.hip(hipErrorOutOfMemory, "basis buffers");
    if (!L.hip(hipMemcpyAsync(Ud.p, U.data(), U.size() * sizeof(double2), hipMemcpyHostToDevice, L.st), "copy"))
      return false;
    if (!project_first(L, M, m, n, Ud.p, r, carry.p)) return false;
    return L.hip(hipStreamSynchronize(L.st), "sync");
  }
  const int nn = (int)n;
  DevBuf H;
  if (!H.alloc((size_t)nn * nn)) return L.hip(hipErrorOutOfMemory, "Gram buffer");
  // column-major H = A A^H with A the column-major n x m view of M: H = conj(M^H M)
  if (!L.check(rocblas_zherk_64(L.h, rocblas_fill_upper, rocblas_operation_none, nn, m, &one, rb(M), nn, &zero,
                                rb(H.p), nn),
               "rocblas_zherk"))
    return false;
  if (!eig_desc(L, H.p, nn, vals, vecs)) return false;
  r = rank_of(vals, budget2);
  // V[:, j] = conj(w_j); W = V S^-1 (n x r row-major); carry[j][c] = s_j conj(V[c][j]) = s_j w_j[c]
  std::vector<cd> W((size_t)nn * r), C((size_t)r * nn);
  for (int j = 0; j < r; ++j) {
    const double s = std::sqrt(std::max(0.0, vals[j]));
    const double inv = s > 0 ? 1.0 / s : 0.0;
    for (int a = 0; a < nn; ++a) {
      const cd w = vecs[(size_t)j * nn + a];
      W[(size_t)a * r + j] = std::conj(w) * inv;
      C[(size_t)j * nn + a] = s * w;
    }
  }
  DevBuf Wd, Ud;
  if (!Wd.alloc(W.size()) || !Ud.alloc((size_t)m * r) || !carry.alloc(C.size()))
    return L.hip(hipErrorOutOfMemory, "basis buffers");
  if (!L.hip(hipMemcpyAsync(Wd.p, W.data(), W.size() * sizeof(double2), hipMemcpyHostToDevice, L.st), "copy") ||
      !L.hip(hipMemcpyAsync(carry.p, C.data(), C.size() * sizeof(double2), hipMemcpyHostToDevice, L.st), "copy"))
    return false;
  // U (m x r row-major) = M W: column-major r x m result = W (r x n) times A (n x m)
  const rocblas_double_complex c1 = {1.0, 0.0}, c0 = {0.0, 0.0};
  if (!L.check(rocblas_zgemm_64(L.h, rocblas_operation_none, rocblas_operation_none, r, m, nn, &c1, rb(Wd.p), r,
                                rb(M), nn, &c0, rb(Ud.p), r),
               "rocblas_zgemm"))
    return false;
  U.resize((size_t)m * r);
  return L.hip(hipMemcpyAsync(U.data(), Ud.p, U.size() * sizeof(double2), hipMemcpyDeviceToHost, L.st), "copy") &&
         L.hip(hipStreamSynchronize(L.st), "sync");
}

// Mode-m Gram basis of a device tensor with shape d (C order), truncated.
bool mode_basis(Linalg& L, const double2* X, const std::vector<long long>& d, int m, double budget2,
                std::vector<cd>& U, int& r) {
  long long P = 1, Q = 1;
  for (int i = 0; i < m; ++i) P *= d[i];
  for (size_t i = m + 1; i < d.size(); ++i) Q *= d[i];
  const int D = (int)d[m];
  DevBuf T;
  const double2* Xf = X;
  if (P > 1) {  // mode first: [P][D][Q] -> [D][P][Q]
    if (!T.alloc((size_t)P * D * Q)) return L.hip(hipErrorOutOfMemory, "permute buffer");
    if (!L.hip(launch_perm_mode(X, T.p, P, D, Q, true, L.st), "permute")) return false;
    Xf = T.p;
  }
  const long long K = P * Q;
  DevBuf H;
  if (!H.alloc((size_t)D * D)) return L.hip(hipErrorOutOfMemory, "Gram buffer");
  const double one = 1.0, zero = 0.0;
  if (!L.check(rocblas_zherk_64(L.h, rocblas_fill_upper, rocblas_operation_conjugate_transpose, D, K, &one, rb(Xf), K,
                                &zero, rb(H.p), D),
               "rocblas_zherk"))
    return false;
  std::vector<double> vals;
  std::vector<cd> vecs;
  if (!eig_desc(L, H.p, D, vals, vecs)) return false;
  r = rank_of(vals, budget2);
  U.assign((size_t)D * r, 0.0);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < r; ++j) U[(size_t)i * r + j] = std::conj(vecs[(size_t)j * D + i]);
  return true;
}

// Y = X x_m U^H (mode m of shape d shrinks from d[m] to r); d is updated.
bool mode_project(Linalg& L, DevBuf& X, std::vector<long long>& d, int m, const std::vector<cd>& U, int r) {
  long long P = 1, Q = 1;
  for (int i = 0; i < m; ++i) P *= d[i];
  for (size_t i = m + 1; i < d.size(); ++i) Q *= d[i];
  const int D = (int)d[m];
  DevBuf Ud, T, Y;
  if (!Ud.alloc(U.size()) || !Y.alloc((size_t)P * r * Q)) return L.hip(hipErrorOutOfMemory, "projection buffers");
  if (!L.hip(hipMemcpyAsync(Ud.p, U.data(), U.size() * sizeof(double2), hipMemcpyHostToDevice, L.st), "copy"))
    return false;
  if (P == 1) {
    if (!project_first(L, X.p, D, Q, Ud.p, r, Y.p)) return false;
  } else {
    if (!T.alloc((size_t)P * D * Q)) return L.hip(hipErrorOutOfMemory, "permute buffer");
    if (!L.hip(launch_perm_mode(X.p, T.p, P, D, Q, true, L.st), "permute")) return false;
    X.release();
    DevBuf Z;
    if (!Z.alloc((size_t)r * P * Q)) return L.hip(hipErrorOutOfMemory, "projection buffer");
    if (!project_first(L, T.p, D, P * Q, Ud.p, r, Z.p)) return false;
    if (!L.hip(launch_perm_mode(Z.p, Y.p, P, r, Q, false, L.st), "permute")) return false;
    if (!L.hip(hipStreamSynchronize(L.st), "sync")) return false;
  }
  if (!L.hip(hipStreamSynchronize(L.st), "sync")) return false;
  X.swap(Y);
  d[m] = r;
  return true;
}

void append(std::vector<cd>& dst, const std::vector<cd>& src) { dst.insert(dst.end(), src.begin(), src.end()); }

bool download(Linalg& L, const DevBuf& B, std::vector<cd>& h) {
  h.resize(B.n);
  return L.hip(hipMemcpyAsync(h.data(), B.p, B.n * sizeof(double2), hipMemcpyDeviceToHost, L.st), "copy") &&
         L.hip(hipStreamSynchronize(L.st), "sync");
}

}  // namespace

std::string fft3d_forward_device(double2* T, const int n[3], int batch, hipStream_t st) {
  hipfftHandle plan;
  int dims[3] = {n[0], n[1], n[2]};
  if (hipfftPlanMany(&plan, 3, dims, nullptr, 1, 0, nullptr, 1, 0, HIPFFT_Z2Z, batch) != HIPFFT_SUCCESS)
    return "hipfftPlanMany failed";
  std::string err;
  if (hipfftSetStream(plan, st) != HIPFFT_SUCCESS) err = "hipfftSetStream failed";
  if (err.empty() && hipfftExecZ2Z(plan, reinterpret_cast<hipfftDoubleComplex*>(T),
                                   reinterpret_cast<hipfftDoubleComplex*>(T), HIPFFT_FORWARD) != HIPFFT_SUCCESS)
    err = "hipfftExecZ2Z failed";
  if (err.empty() && hipStreamSynchronize(st) != hipSuccess) err = "FFT synchronisation failed";
  (void)hipfftDestroy(plan);
  return err;
}

std::string compress_4d_device(double2* dT, int ndir, const int n[3], int fmt, double gamma, Factors& out,
                               int nthreads, hipStream_t st) {
  const long long N = (long long)n[0] * n[1] * n[2];
  out = Factors();
  out.fmt = fmt;
  for (int i = 0; i < 3; ++i) out.n[i] = n[i];
  out.ndir = ndir;
  if (fmt < 3 || fmt > 5) return "not a 4-D format";
  Linalg L(st);
  if (!L.err.empty()) return L.err;
  // X4[x][y][z][p] (mode order x, y, z, direction)
  DevBuf X;
  if (!X.alloc((size_t)N * ndir)) return "no device memory for the 4-D operator tensor";
  if (!L.hip(launch_transpose64(dT, X.p, ndir, N, st), "transpose")) return L.err;
  const double nx2 = norm2_dev(L, X.p, N * ndir);
  if (!L.err.empty()) return L.err;
  if (!(nx2 > 0)) return "operator is zero";
  std::vector<long long> d = {n[0], n[1], n[2], ndir};
  if (fmt == 3 || fmt == 5) {
    const double budget2 = gamma * gamma / (fmt == 3 ? 4.0 : 6.0) * nx2;
    std::vector<std::vector<cd>> U(4);
    int r[4];
    for (int m = 0; m < 4; ++m)
      if (!mode_basis(L, X.p, d, m, budget2, U[m], r[m])) return L.err;
    // core = X x_m U_m^H, the mode that shrinks most first
    std::vector<int> order = {0, 1, 2, 3};
    std::sort(order.begin(), order.end(),
              [&](int a, int b) { return (double)d[a] / r[a] > (double)d[b] / r[b]; });
    for (int m : order)
      if (!mode_project(L, X, d, m, U[m], r[m])) return L.err;
    std::vector<cd> C;
    if (!download(L, X, C)) return L.err;
    double c2 = 0.0;
    for (const cd& v : C) c2 += std::norm(v);
    if (fmt == 3) {
      out.ranks = {r[0], r[1], r[2], r[3]};
      out.rel_err = std::sqrt(std::max(0.0, nx2 - c2) / nx2);
      append(out.data, C);
      for (int m = 0; m < 4; ++m) append(out.data, U[m]);
      return "";
    }
    // H-Tucker interior nodes (Algorithm 2, steps 5-10) on the device: the core
    // as W12 = (r1 r2) x (r3 r4); C12 = leading left singular vectors of W12,
    // C34 those of W12^T (same singular values, so r34 = r12); root
    // B = C12^H W12 conj(C34)
    (void)nthreads;
    const int m12 = r[0] * r[1], m34 = r[2] * r[3];
    std::vector<cd> U12, U34;
    int r12 = 0, r34 = 0;
    DevBuf T12, Wt, T34;
    if (!svd_left(L, X.p, m12, m34, budget2, U12, r12, T12)) return L.err;  // T12 = C12^H W12 (r12 x m34)
    if (!Wt.alloc((size_t)m12 * m34)) return "no device memory for the transposed core";
    if (!L.hip(launch_transpose64(X.p, Wt.p, m12, m34, st), "transpose")) return L.err;
    if (!svd_left(L, Wt.p, m34, m12, budget2, U34, r34, T34)) return L.err;
    std::vector<cd> T;
    if (!download(L, T12, T)) return L.err;
    std::vector<cd> Bm((size_t)r12 * r34, 0.0);
    for (int i = 0; i < r12; ++i)
      for (int k = 0; k < m34; ++k) {
        const cd t = T[(size_t)i * m34 + k];
        const cd* u = &U34[(size_t)k * r34];
        cd* b = &Bm[(size_t)i * r34];
        for (int j = 0; j < r34; ++j) b[j] += t * std::conj(u[j]);
      }
    double b2 = 0.0;
    for (const cd& v : Bm) b2 += std::norm(v);
    out.ranks = {r[0], r[1], r[2], r[3], r12, r34};
    out.rel_err = std::sqrt(std::max(0.0, nx2 - b2) / nx2);
    for (int m = 0; m < 4; ++m) append(out.data, U[m]);
    append(out.data, U12);  // C12[a1][a2][b]
    append(out.data, U34);  // C34[a3][a4][b']
    append(out.data, Bm);
    return "";
  }
  // TT-4D (Algorithm 3): x | y | z | direction
  const double budget2 = gamma * gamma / 3.0 * nx2;
  std::vector<cd> U1, U2, U3;
  int r1 = 0, r2 = 0, r3 = 0;
  DevBuf C1, C2, carry;
  if (!svd_left(L, X.p, n[0], (long long)n[1] * n[2] * ndir, budget2, U1, r1, C1)) return L.err;
  X.release();
  if (!svd_left(L, C1.p, r1 * n[1], (long long)n[2] * ndir, budget2, U2, r2, C2)) return L.err;
  C1.release();
  if (!svd_left(L, C2.p, r2 * n[2], ndir, budget2, U3, r3, carry)) return L.err;
  C2.release();
  std::vector<cd> cr;
  if (!download(L, carry, cr)) return L.err;
  double c2 = 0.0;
  for (const cd& v : cr) c2 += std::norm(v);
  out.ranks = {r1, r2, r3};
  out.rel_err = std::sqrt(std::max(0.0, nx2 - c2) / nx2);
  append(out.data, U1);  // U1 n1 x r1
  append(out.data, U2);  // C1 r1 x n2 x r2
  append(out.data, U3);  // C2 r2 x n3 x r3
  std::vector<cd> Ul((size_t)ndir * r3);
  for (int c = 0; c < r3; ++c)
    for (int p = 0; p < ndir; ++p) Ul[(size_t)p * r3 + c] = cr[(size_t)c * ndir + p];
  append(out.data, Ul);  // U3 n_dir x r3
  return "";
}

}  // namespace tfmm
