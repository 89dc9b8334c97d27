// Iterative solution of the method-of-moments system Z I = V (Eq. (2)) with
// TFQMR (Section II-A): Z = near-field matrix (sparse, caller-supplied) + the
// far-field product of the library (aggregation, compressed-operator
// translation, projection).  The Krylov vectors are complex128 on the device
// (rocBLAS level-1 in FP64); each product with Z runs the complex64 kernels.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>

#include "launch.h"
#include "internal.h"
#include "tfmm.h"

namespace {

using zc = rocblas_double_complex;

struct Dev128 {
  double2* p = nullptr;
  ~Dev128() {
    if (p) (void)hipFree(p);
  }
};

struct Solver {
  tfmm_ctx c;
  tfmm_op op;
  tfmm_basis basis;
  tfmm_near near;
  int n;
  hipStream_t st = nullptr;
  rocblas_handle h = nullptr;
  float2 *x32 = nullptr, *yn32 = nullptr, *yf32 = nullptr;
  std::string err;
  tfmm_status status = TFMM_OK;

  bool rb(rocblas_status s, const char* what) {
    if (s != rocblas_status_success && status == TFMM_OK) {
      status = TFMM_ERR_INTERNAL;
      err = std::string(what) + " failed";
    }
    return status == TFMM_OK;
  }
  bool hip(hipError_t e, const char* what) {
    if (e != hipSuccess && status == TFMM_OK) {
      status = TFMM_ERR_HIP;
      err = std::string(what) + ": " + hipGetErrorString(e);
    }
    return status == TFMM_OK;
  }
  bool abi(tfmm_status s) {
    if (s != TFMM_OK && status == TFMM_OK) {
      status = s;
      err = tfmm_last_error();
    }
    return status == TFMM_OK;
  }
  // y = Z x: near-field CSR product plus the far-field product, complex64 inside
  bool apply(const double2* x, double2* y) {
    return hip(tfmm::launch_narrow128(x, x32, n, st), "convert") && abi(tfmm_near_matvec(c, near, x32, yn32, 1, st)) &&
           abi(tfmm_farfield_matvec(c, op, basis, x32, yf32, 1, st)) &&
           hip(tfmm::launch_sum_widen(yn32, yf32, y, n, st), "convert");
  }
  std::complex<double> dotc(const double2* a, const double2* b) {  // b^H a
    zc r{0, 0};
    rb(rocblas_zdotc(h, n, (const zc*)b, 1, (const zc*)a, 1, &r), "rocblas_zdotc");
    return {r.real(), r.imag()};
  }
  double nrm(const double2* a) {
    double r = 0;
    rb(rocblas_dznrm2(h, n, (const zc*)a, 1, &r), "rocblas_dznrm2");
    return r;
  }
  void axpy(std::complex<double> a, const double2* x, double2* y) {  // y += a x
    const zc za(a.real(), a.imag());
    rb(rocblas_zaxpy(h, n, &za, (const zc*)x, 1, (zc*)y, 1), "rocblas_zaxpy");
  }
  void scal(std::complex<double> a, double2* x) {
    const zc za(a.real(), a.imag());
    rb(rocblas_zscal(h, n, &za, (zc*)x, 1), "rocblas_zscal");
  }
  void copy(const double2* x, double2* y) { rb(rocblas_zcopy(h, n, (const zc*)x, 1, (zc*)y, 1), "rocblas_zcopy"); }
};

}  // namespace

// TFQMR in the steps of Freund's algorithm: per iteration one coefficient
// alpha = rho / (r*, v) for two half steps; each half step quasi-minimises the
// residual through (theta, c, tau, eta) and moves the iterate along the
// smoothed direction d; the bound tau sqrt(m + 1) on the residual norm of half
// step m triggers a check of the true residual.
extern "C" tfmm_status tfmm_solve_tfqmr(tfmm_ctx ctx, tfmm_op op, tfmm_basis basis, tfmm_near near, const void* V,
                                        void* I, double tol, int32_t maxit, int32_t* iters, double* relres) {
  if (!ctx || !op || !basis || !near || !V || !I) {
    tfmm::set_last_error("ctx, op, basis, near, V or I is NULL");
    return TFMM_ERR_INVALID_ARG;
  }
  if (!(tol > 0 && tol < 1) || maxit < 1) {
    tfmm::set_last_error("need 0 < tol < 1 and maxit >= 1");
    return TFMM_ERR_INVALID_ARG;
  }
  const int n = tfmm::near_rows(near);
  if (n < 1) {
    tfmm::set_last_error("empty near-field matrix");
    return TFMM_ERR_INVALID_ARG;
  }
  Solver S{ctx, op, basis, near, n};
  Dev128 b, x, r, w, u, un, v, Au, Aun, d, t;
  Dev128* all[] = {&b, &x, &r, &w, &u, &un, &v, &Au, &Aun, &d, &t};
  for (Dev128* p : all)
    if (!S.hip(hipMalloc(&p->p, (size_t)n * sizeof(double2)), "hipMalloc")) return S.status;
  if (!S.hip(hipStreamCreateWithFlags(&S.st, hipStreamNonBlocking), "stream")) return S.status;
  if (rocblas_create_handle(&S.h) != rocblas_status_success) {
    (void)hipStreamDestroy(S.st);
    return TFMM_ERR_INTERNAL;
  }
  (void)rocblas_set_stream(S.h, S.st);
  (void)rocblas_set_pointer_mode(S.h, rocblas_pointer_mode_host);
  int it = 0;
  double res = 1.0;
  bool done = false;
  if (S.hip(hipMalloc(&S.x32, (size_t)n * sizeof(float2)), "hipMalloc") &&
      S.hip(hipMalloc(&S.yn32, (size_t)n * sizeof(float2)), "hipMalloc") &&
      S.hip(hipMalloc(&S.yf32, (size_t)n * sizeof(float2)), "hipMalloc") &&
      S.hip(tfmm::launch_widen(static_cast<const float2*>(V), b.p, n, S.st), "convert") &&
      S.hip(hipMemsetAsync(x.p, 0, (size_t)n * sizeof(double2), S.st), "memset")) {
    const double nb = S.nrm(b.p);
    // x0 = 0: r0 = b
    S.copy(b.p, r.p);
    S.copy(r.p, w.p);
    S.copy(r.p, u.p);
    S.apply(u.p, v.p);
    S.copy(v.p, Au.p);
    S.hip(hipMemsetAsync(d.p, 0, (size_t)n * sizeof(double2), S.st), "memset");
    double tau = S.nrm(r.p), theta = 0.0;
    std::complex<double> eta = 0.0;
    std::complex<double> rho = S.dotc(r.p, r.p);  // shadow residual r* = r0
    res = nb > 0 ? tau / nb : 0.0;
    done = !(nb > 0) || res <= tol;
    for (it = 1; !done && it <= maxit && S.status == TFMM_OK; ++it) {
      const std::complex<double> sigma = S.dotc(v.p, r.p);
      if (std::abs(sigma) == 0.0) break;  // breakdown
      const std::complex<double> alpha = rho / sigma;
      S.copy(u.p, un.p);
      S.axpy(-alpha, v.p, un.p);  // u_{2n} = u_{2n-1} - alpha v
      for (int half = 0; half < 2 && !done && S.status == TFMM_OK; ++half) {
        const int m = 2 * (it - 1) + half;
        double2* um = half == 0 ? u.p : un.p;
        double2* Aum = Au.p;
        if (half == 1) {
          S.apply(un.p, Aun.p);
          Aum = Aun.p;
        }
        S.axpy(-alpha, Aum, w.p);
        // d = u_m + (theta^2 eta / alpha) d
        S.scal(theta * theta * eta / alpha, d.p);
        S.axpy(1.0, um, d.p);
        theta = S.nrm(w.p) / tau;
        const double cc = 1.0 / std::sqrt(1.0 + theta * theta);
        tau = tau * theta * cc;
        eta = cc * cc * alpha;
        S.axpy(eta, d.p, x.p);
        res = tau * std::sqrt((double)m + 2.0) / nb;  // Freund's bound until a true residual is taken
        if (res <= tol) {
          // true residual of the complex128 iterate through the operator
          S.apply(x.p, t.p);
          S.copy(b.p, r.p);
          S.axpy(-1.0, t.p, r.p);
          res = S.nrm(r.p) / nb;
          done = res <= tol;
        }
      }
      if (done) break;
      // rho with the fixed shadow residual r* = r0 = b (r is reused for the true residual)
      const std::complex<double> rho2 = S.dotc(w.p, b.p);
      const std::complex<double> beta = rho2 / rho;
      rho = rho2;
      S.copy(w.p, u.p);
      S.axpy(beta, un.p, u.p);  // u_{2n+1} = w + beta u_{2n}
      S.apply(u.p, Au.p);
      // v = A u_{2n+1} + beta (A u_{2n} + beta v)
      S.scal(beta, v.p);
      S.axpy(1.0, Aun.p, v.p);
      S.scal(beta, v.p);
      S.axpy(1.0, Au.p, v.p);
    }
    if (done && S.status == TFMM_OK) S.hip(tfmm::launch_narrow128(x.p, static_cast<float2*>(I), n, S.st), "convert");
    S.hip(hipStreamSynchronize(S.st), "sync");
  }
  if (S.x32) (void)hipFree(S.x32);
  if (S.yn32) (void)hipFree(S.yn32);
  if (S.yf32) (void)hipFree(S.yf32);
  (void)rocblas_destroy_handle(S.h);
  (void)hipStreamDestroy(S.st);
  if (iters) *iters = std::min(it, maxit);
  if (relres) *relres = res;
  if (S.status != TFMM_OK) {
    tfmm::set_last_error("TFQMR: " + S.err);
    return S.status;
  }
  if (!done) {
    tfmm::set_last_error("TFQMR: relative residual " + std::to_string(res) + " after " + std::to_string(std::min(it, maxit)) +
                         " iterations");
    return TFMM_ERR_NOT_CONVERGED;
  }
  return TFMM_OK;
}
