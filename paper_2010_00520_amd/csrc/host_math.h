// Host-side FP64 setup mathematics: plane-wave directions, multipole order,
// 3-D FFT, Hermitian eigensolver and the five operator compressors.
// Plain C++17 (no HIP), so the setup logic can be tested on a CPU-only host.
#pragma once
#include <complex>
#include <functional>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace tfmm {

using cd = std::complex<double>;

// Gauss-Legendre nodes (ascending) and weights on [-1, 1], by Newton iteration
// on P_n with the three-term recurrence.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Direction grid of Section II-A: n_theta GL nodes in cos(theta) times n_phi
// uniform phi; p = i_theta * n_phi + j_phi.  khat is n_dir x 3 (row-major).
void direction_grid(int n_theta, int n_phi, std::vector<double>& khat, std::vector<double>& w);

// L = ceil(x + 1.8 digits^(2/3) x^(1/3)), x = k a sqrt(3).
int multipole_order_ceil(double k, double box, double digits);

// In-place forward 3-D DFT (unnormalised, exp(-2 pi i m k / n)) of `batch`
// contiguous n1 x n2 x n3 blocks.  n_i must factor into 2s and 3s.
void fft3d_forward(cd* data, int n1, int n2, int n3, int batch);

// Eigen-decomposition of a Hermitian n x n matrix (row-major, overwritten) by
// cyclic complex Jacobi rotations.  Eigenvalues descending; eigenvectors are
// the columns of `vecs` (n x n row-major).
void hermitian_eig(int n, std::vector<cd>& a, std::vector<double>& vals, std::vector<cd>& vecs);

// Smallest r >= 1 with sum_{j >= r} s2[j] + r_margin <= budget2 (s2 = squared
// singular values, descending).  `margin` is added per discarded value to cover
// the eigenvalue error of the Gram approach.
int truncation_rank(const std::vector<double>& s2, double budget2, double margin);

// Compressed operator in the host exchange layout documented for
// tfmm_op_import (complex128).
struct Factors {
  int fmt = 0;                 // tfmm_format value
  int n[3] = {0, 0, 0};
  int ndir = 0;
  std::vector<int32_t> ranks;  // format-specific (per direction for 3-D formats)
  std::vector<cd> data;
  double rel_err = 0.0;        // ||X - Xhat||_F / ||X||_F over the whole operator
  double max_dir_err = -1.0;   // per-direction maximum (3-D formats), -1 if not computed
};

// Compress the FFT'ed operator That[p][x][y][z] (n_dir blocks of n1 n2 n3).
// fmt: 0 FULL .. 5 HTUCKER4D (tfmm_format).  Truncation: tail singular values
// root-sum-square <= gamma/sqrt(m) ||X||_F with m = d (Tucker), d-1 (TT), 6 (H-Tucker).
// Returns an empty string on success, else an error message.
std::string compress_operator(const std::vector<cd>& That, int ndir, const int n[3], int fmt,
                              double gamma, Factors& out, int nthreads);

// Interior nodes of the balanced H-Tucker tree {1,2}{3,4} (Algorithm 2, steps
// 5-10) from the leaf core C (r1 x r2 x r3 x r4, C order) and the leaf bases
// U_m (n_m x r_m, row-major): truncation with the tail budget budget2 (squared),
// relative error from nx2 = ||X||_F^2.  Writes ranks, rel_err and the import
// layout U1..U4, C12, C34, root into `out`.
void htucker_interior(const std::vector<cd>& C, const int r[4], const std::vector<std::vector<cd>>& leaves,
                      double budget2, double nx2, Factors& out, int nthreads);

// Number of complex entries the import layout holds for a format and ranks;
// -1 if the ranks are inconsistent.
long long factor_elems(int fmt, const int n[3], int ndir, const std::vector<int32_t>& ranks);

// Run f(i) for i in [0, count) on up to nthreads threads (dynamic scheduling).
void parallel_for(int count, int nthreads, const std::function<void(int)>& f);

}  // namespace tfmm
