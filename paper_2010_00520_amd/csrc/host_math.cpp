// Host-side FP64 setup mathematics (see host_math.h).
#include "host_math.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>

namespace tfmm {

static const double kPi = 3.14159265358979323846264338327950288;

void parallel_for(int count, int nthreads, const std::function<void(int)>& f) {
  if (count <= 0) return;
  int nt = std::max(1, std::min(nthreads, count));
  if (nt == 1) {
    for (int i = 0; i < count; ++i) f(i);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&]() {
      for (int i = next.fetch_add(1); i < count; i = next.fetch_add(1)) f(i);
    });
  for (auto& th : pool) th.join();
}

// ---------------------------------------------------------------------------
// Directions and multipole order (Section II-A, text after Eq. (4))
// ---------------------------------------------------------------------------

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    // Chebyshev-like initial guess for the i-th largest root, then Newton on P_n.
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int l = 2; l <= n; ++l) {
        double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 0) ? 1.0 : p1, pm = (n == 0) ? 0.0 : p0;
      if (n == 1) { pn = z; pm = 1.0; }
      dp = n * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged root
    double p0 = 1.0, p1 = z;
    for (int l = 2; l <= n; ++l) {
      double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
      p0 = p1;
      p1 = p2;
    }
    double pn = (n == 1) ? z : p1, pm = (n == 1) ? 1.0 : p0;
    dp = n * (z * pn - pm) / (z * z - 1.0);
    x[n - 1 - i] = z;  // roots come out descending; store ascending
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void direction_grid(int n_theta, int n_phi, std::vector<double>& khat, std::vector<double>& w) {
  std::vector<double> x, wt;
  gauss_legendre(n_theta, x, wt);
  khat.assign(3 * (size_t)n_theta * n_phi, 0.0);
  w.assign((size_t)n_theta * n_phi, 0.0);
  for (int i = 0; i < n_theta; ++i) {
    double ct = x[i], st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
    for (int j = 0; j < n_phi; ++j) {
      double ph = 2.0 * kPi * j / n_phi;
      size_t p = (size_t)i * n_phi + j;
      khat[3 * p + 0] = st * std::cos(ph);
      khat[3 * p + 1] = st * std::sin(ph);
      khat[3 * p + 2] = ct;
      w[p] = wt[i] * 2.0 * kPi / n_phi;
    }
  }
}

int multipole_order_ceil(double k, double box, double digits) {
  double x = k * box * std::sqrt(3.0);
  return (int)std::ceil(x + 1.8 * std::pow(digits, 2.0 / 3.0) * std::cbrt(x));
}

// ---------------------------------------------------------------------------
// FP64 FFT (mixed radix 2/3, recursive decimation in time)
// ---------------------------------------------------------------------------

namespace {

void dft_rec(const cd* in, int stride, cd* out, int n, const std::vector<cd>& tw, int twstep, cd* scratch) {
  if (n == 1) {
    out[0] = in[0];
    return;
  }
  int r = (n % 2 == 0) ? 2 : (n % 3 == 0 ? 3 : n);
  if (r == n) {  // direct DFT (prime length)
    for (int k = 0; k < n; ++k) {
      cd s = 0.0;
      for (int j = 0; j < n; ++j) s += in[(size_t)j * stride] * tw[(size_t)((j * k) % n) * twstep];
      out[k] = s;
    }
    return;
  }
  int m = n / r;
  // sub-DFTs of the r decimated sequences into scratch, then combine into out
  for (int i = 0; i < r; ++i) dft_rec(in + (size_t)i * stride, stride * r, scratch + (size_t)i * m, m, tw, twstep * r, out);
  for (int k = 0; k < m; ++k) {
    cd t[3];
    for (int i = 0; i < r; ++i) t[i] = scratch[(size_t)i * m + k] * tw[(size_t)(i * k) * twstep];
    if (r == 2) {
      out[k] = t[0] + t[1];
      out[k + m] = t[0] - t[1];
    } else {
      const cd w3 = tw[(size_t)(n / 3) * twstep];  // exp(-2 pi i / 3)
      const cd w3b = std::conj(w3);
      out[k] = t[0] + t[1] + t[2];
      out[k + m] = t[0] + w3 * t[1] + w3b * t[2];
      out[k + 2 * m] = t[0] + w3b * t[1] + w3 * t[2];
    }
  }
}

void fft_lines(cd* data, int n, size_t stride, size_t count, size_t line_step_outer, size_t inner,
               int nthreads) {
  // lines: for o in [0, count/inner), i in [0, inner): base = o*line_step_outer + i
  std::vector<cd> tw(n);
  for (int k = 0; k < n; ++k) tw[k] = std::polar(1.0, -2.0 * kPi * k / n);
  size_t outer = count / inner;
  parallel_for((int)std::min<size_t>(outer, 1u << 30), nthreads, [&](int o) {
    std::vector<cd> line(n), res(n), scr(n);
    for (size_t i = 0; i < inner; ++i) {
      cd* base = data + (size_t)o * line_step_outer + i;
      for (int j = 0; j < n; ++j) line[j] = base[(size_t)j * stride];
      // scratch must hold n values for every recursion level; levels reuse `res`/`scr`
      dft_rec(line.data(), 1, res.data(), n, tw, 1, scr.data());
      for (int j = 0; j < n; ++j) base[(size_t)j * stride] = res[j];
    }
  });
}

}  // namespace

void fft3d_forward(cd* data, int n1, int n2, int n3, int batch) {
  int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  size_t N = (size_t)n1 * n2 * n3;
  // axis 3 (contiguous): lines start at every (b, x, y)
  fft_lines(data, n3, 1, (size_t)batch * n1 * n2, n3, 1, nt);
  // axis 2: per (b, x) block of n2*n3, lines at z offsets
  fft_lines(data, n2, n3, (size_t)batch * n1 * n3, (size_t)n2 * n3, n3, nt);
  // axis 1: per b block of N, lines at (y, z) offsets
  fft_lines(data, n1, (size_t)n2 * n3, (size_t)batch * n2 * n3, N, (size_t)n2 * n3, nt);
}

// ---------------------------------------------------------------------------
// Hermitian eigensolver: cyclic Jacobi with complex rotations
// ---------------------------------------------------------------------------

void hermitian_eig(int n, std::vector<cd>& a, std::vector<double>& vals, std::vector<cd>& vecs) {
  vecs.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) vecs[(size_t)i * n + i] = 1.0;
  auto A = [&](int i, int j) -> cd& { return a[(size_t)i * n + j]; };
  double fro = 0.0;
  for (auto& v : a) fro += std::norm(v);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += std::norm(A(i, j));
    if (off <= 1e-32 * fro || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        cd apq = A(p, q);
        double mag = std::abs(apq);
        if (mag == 0.0) continue;
        double app = A(p, p).real(), aqq = A(q, q).real();
        if (mag < 1e-300) continue;
        // Phase e^{i phi} = apq/|apq|; rotate the real symmetric 2x2 [[app, mag],[mag, aqq]].
        cd ph = apq / mag;
        double theta = (aqq - app) / (2.0 * mag);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        // Unitary J acts on columns p, q: col_p' = c col_p - s conj(ph) col_q,
        //                                 col_q' = s ph col_p + c col_q.
        cd sp = s * ph, sq = s * std::conj(ph);
        for (int k = 0; k < n; ++k) {  // A <- A J
          cd akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - sq * akq;
          A(k, q) = sp * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^H A
          cd apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - std::conj(sq) * aqk;
          A(q, k) = std::conj(sp) * apk + c * aqk;
        }
        A(p, q) = 0.0;
        A(q, p) = 0.0;
        A(p, p) = A(p, p).real();
        A(q, q) = A(q, q).real();
        for (int k = 0; k < n; ++k) {  // V <- V J
          cd vkp = vecs[(size_t)k * n + p], vkq = vecs[(size_t)k * n + q];
          vecs[(size_t)k * n + p] = c * vkp - sq * vkq;
          vecs[(size_t)k * n + q] = sp * vkp + c * vkq;
        }
      }
    }
  }
  // sort descending
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return A(x, x).real() > A(y, y).real(); });
  vals.resize(n);
  std::vector<cd> sorted((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    vals[j] = A(idx[j], idx[j]).real();
    for (int k = 0; k < n; ++k) sorted[(size_t)k * n + j] = vecs[(size_t)k * n + idx[j]];
  }
  vecs.swap(sorted);
}

int truncation_rank(const std::vector<double>& s2, double budget2, double margin) {
  int m = (int)s2.size();
  // tail[r] = sum_{j >= r} s2[j]
  std::vector<double> tail(m + 1, 0.0);
  for (int j = m - 1; j >= 0; --j) tail[j] = tail[j + 1] + std::max(0.0, s2[j]);
  for (int r = 1; r <= m; ++r)
    if (tail[r] + margin * (m - r) <= budget2) return r;
  return m;
}

// ---------------------------------------------------------------------------
// Dense helpers on tensors viewed as (pre, d, post), C order
// ---------------------------------------------------------------------------

namespace {

struct Shape {
  std::vector<long long> d;
  long long size() const {
    long long s = 1;
    for (auto v : d) s *= v;
    return s;
  }
  long long pre(int m) const {
    long long s = 1;
    for (int i = 0; i < m; ++i) s *= d[i];
    return s;
  }
  long long post(int m) const {
    long long s = 1;
    for (size_t i = m + 1; i < d.size(); ++i) s *= d[i];
    return s;
  }
};

double norm2(const std::vector<cd>& x) {
  double s = 0.0;
  for (auto& v : x) s += std::norm(v);
  return s;
}

// G[a][b] = sum_{pre,post} X[pre,a,post] conj(X[pre,b,post])  (Gram of the mode-m unfolding)
std::vector<cd> mode_gram(const cd* X, const Shape& sh, int m, int nthreads) {
  long long P = sh.pre(m), D = sh.d[m], Q = sh.post(m);
  std::vector<cd> G((size_t)D * D, 0.0);
  // tasks: blocks of (pre, post-chunk); each thread accumulates its own Gram
  const long long chunk = 256;
  long long nchunks = (Q + chunk - 1) / chunk;
  long long ntasks = P * nchunks;
  int nt = (int)std::max<long long>(1, std::min<long long>(nthreads, ntasks));
  std::vector<std::vector<cd>> part(nt, std::vector<cd>((size_t)D * D, 0.0));
  std::atomic<long long> next(0);
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&, t]() {
      std::vector<cd>& g = part[t];
      for (long long task = next.fetch_add(1); task < ntasks; task = next.fetch_add(1)) {
        long long p = task / nchunks, c0 = (task % nchunks) * chunk, c1 = std::min(Q, c0 + chunk);
        const cd* base = X + (size_t)p * D * Q;
        for (long long a = 0; a < D; ++a) {
          const cd* ra = base + (size_t)a * Q;
          for (long long b = a; b < D; ++b) {
            const cd* rb = base + (size_t)b * Q;
            double sr = 0.0, si = 0.0;
            for (long long c = c0; c < c1; ++c) {
              double xr = ra[c].real(), xi = ra[c].imag(), yr = rb[c].real(), yi = rb[c].imag();
              sr += xr * yr + xi * yi;
              si += xi * yr - xr * yi;
            }
            g[(size_t)a * D + b] += cd(sr, si);
          }
        }
      }
    });
  for (auto& th : pool) th.join();
  for (int t = 0; t < nt; ++t)
    for (size_t i = 0; i < G.size(); ++i) G[i] += part[t][i];
  for (long long a = 0; a < D; ++a)
    for (long long b = 0; b < a; ++b) G[(size_t)a * D + b] = std::conj(G[(size_t)b * D + a]);
  return G;
}

// Y = X x_m U^H: Y[pre,j,post] = sum_a conj(U[a][j]) X[pre,a,post]; U is D x r row-major.
std::vector<cd> project_mode(const cd* X, const Shape& sh, int m, const std::vector<cd>& U, int r,
                             int nthreads) {
  long long P = sh.pre(m), D = sh.d[m], Q = sh.post(m);
  std::vector<cd> Y((size_t)P * r * Q, 0.0);
  parallel_for((int)(P * r), nthreads, [&](int task) {
    long long p = task / r, j = task % r;
    cd* y = Y.data() + ((size_t)p * r + j) * Q;
    const cd* xb = X + (size_t)p * D * Q;
    for (long long a = 0; a < D; ++a) {
      cd u = std::conj(U[(size_t)a * r + j]);
      const cd* x = xb + (size_t)a * Q;
      double ur = u.real(), ui = u.imag();
      for (long long c = 0; c < Q; ++c) {
        double xr = x[c].real(), xi = x[c].imag();
        y[c] += cd(ur * xr - ui * xi, ur * xi + ui * xr);
      }
    }
  });
  return Y;
}

// Leading left singular vectors of the mode-m unfolding, truncated so the
// discarded energy stays within budget2.  Returns U (D x r row-major) and r.
struct Basis {
  std::vector<cd> U;
  int r = 0;
};

Basis basis_from_gram(std::vector<cd> G, int D, double budget2) {
  std::vector<double> vals;
  std::vector<cd> vecs;
  hermitian_eig(D, G, vals, vecs);
  double lmax = vals.empty() ? 0.0 : std::max(0.0, vals[0]);
  // Eigenvalues of the FP64 Gram carry an absolute error of a few eps * lambda_max;
  // count that against the budget for every discarded value.
  double margin = 4.0 * 2.2e-16 * lmax;
  Basis b;
  b.r = truncation_rank(vals, budget2, margin);
  b.U.resize((size_t)D * b.r);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < b.r; ++j) b.U[(size_t)i * b.r + j] = vecs[(size_t)i * D + j];
  return b;
}

// Modified Gram-Schmidt on the columns of U (m x r row-major), twice.
void orthonormalize(std::vector<cd>& U, int m, int r) {
  for (int pass = 0; pass < 2; ++pass)
    for (int j = 0; j < r; ++j) {
      for (int k = 0; k < j; ++k) {
        cd dot = 0.0;
        for (int i = 0; i < m; ++i) dot += std::conj(U[(size_t)i * r + k]) * U[(size_t)i * r + j];
        for (int i = 0; i < m; ++i) U[(size_t)i * r + j] -= dot * U[(size_t)i * r + k];
      }
      double nr = 0.0;
      for (int i = 0; i < m; ++i) nr += std::norm(U[(size_t)i * r + j]);
      nr = std::sqrt(nr);
      if (nr > 0)
        for (int i = 0; i < m; ++i) U[(size_t)i * r + j] /= nr;
    }
}

// Truncated left singular basis of a row-major matrix M (m x n).  Uses the
// smaller Gram: M M^H when m <= n, else M^H M followed by U = orth(M V).
Basis left_basis(const std::vector<cd>& M, int m, long long n, double budget2, int nthreads) {
  if ((long long)m <= n) {
    Shape sh{{m, n}};
    return basis_from_gram(mode_gram(M.data(), sh, 0, nthreads), m, budget2);
  }
  Shape sh{{m, n}};
  Basis v = basis_from_gram(mode_gram(M.data(), sh, 1, nthreads), (int)n, budget2);
  // mode_gram over mode 1 gives sum_i conj(M[i][a]) M[i][b] conjugated: G[a][b] = sum_i M[i][a] conj(M[i][b]).
  // Its eigenvectors are conj(V); right singular vectors V = conj(eigvecs).
  Basis u;
  u.r = v.r;
  u.U.assign((size_t)m * u.r, 0.0);
  parallel_for(m, nthreads, [&](int i) {
    for (int j = 0; j < u.r; ++j) {
      cd s = 0.0;
      for (long long a = 0; a < n; ++a) s += M[(size_t)i * n + a] * std::conj(v.U[(size_t)a * v.r + j]);
      u.U[(size_t)i * u.r + j] = s;
    }
  });
  orthonormalize(u.U, m, u.r);
  return u;
}

// C = U^H M for U (m x r), M (m x n): r x n
std::vector<cd> adjoint_times(const std::vector<cd>& U, int m, int r, const std::vector<cd>& M, long long n,
                              int nthreads) {
  Shape sh{{m, n}};
  return project_mode(M.data(), sh, 0, U, r, nthreads);
}

void append(std::vector<cd>& dst, const std::vector<cd>& src) { dst.insert(dst.end(), src.begin(), src.end()); }

// Core = X x_i U_i^H over all modes, contracted in the order that shrinks the tensor fastest.
std::vector<cd> project_all(const std::vector<cd>& X, Shape sh, const std::vector<Basis>& B, int nthreads) {
  int d = (int)sh.d.size();
  std::vector<int> order(d);
  for (int i = 0; i < d; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return (double)sh.d[a] / B[a].r > (double)sh.d[b] / B[b].r;
  });
  std::vector<cd> cur = X;
  for (int m : order) {
    cur = project_mode(cur.data(), sh, m, B[m].U, B[m].r, nthreads);
    sh.d[m] = B[m].r;
  }
  return cur;
}

}  // namespace

// ---------------------------------------------------------------------------
// Compressors (Algorithms 1-3 with the tail-energy truncation rule)
// ---------------------------------------------------------------------------

long long factor_elems(int fmt, const int n[3], int ndir, const std::vector<int32_t>& r) {
  long long n1 = n[0], n2 = n[1], n3 = n[2];
  switch (fmt) {
    case 0:
      return (long long)ndir * n1 * n2 * n3;
    case 1: {
      if ((long long)r.size() != 3LL * ndir) return -1;
      long long s = 0;
      for (int p = 0; p < ndir; ++p) {
        long long a = r[3 * p], b = r[3 * p + 1], c = r[3 * p + 2];
        if (a < 1 || b < 1 || c < 1) return -1;
        s += a * b * c + n1 * a + n2 * b + n3 * c;
      }
      return s;
    }
    case 2: {
      if ((long long)r.size() != 2LL * ndir) return -1;
      long long s = 0;
      for (int p = 0; p < ndir; ++p) {
        long long a = r[2 * p], b = r[2 * p + 1];
        if (a < 1 || b < 1) return -1;
        s += n1 * a + a * n2 * b + n3 * b;
      }
      return s;
    }
    case 3: {
      if (r.size() != 4) return -1;
      for (auto v : r)
        if (v < 1) return -1;
      return (long long)r[0] * r[1] * r[2] * r[3] + n1 * r[0] + n2 * r[1] + n3 * r[2] + (long long)ndir * r[3];
    }
    case 4: {
      if (r.size() != 3) return -1;
      for (auto v : r)
        if (v < 1) return -1;
      return n1 * r[0] + (long long)r[0] * n2 * r[1] + (long long)r[1] * n3 * r[2] + (long long)ndir * r[2];
    }
    case 5: {
      if (r.size() != 6) return -1;
      for (auto v : r)
        if (v < 1) return -1;
      return n1 * r[0] + n2 * r[1] + n3 * r[2] + (long long)ndir * r[3] + (long long)r[0] * r[1] * r[4] +
             (long long)r[2] * r[3] * r[5] + (long long)r[4] * r[5];
    }
  }
  return -1;
}

// Interior nodes of the balanced H-Tucker tree {1,2}{3,4} (Algorithm 2, steps
// 5-10) from the leaf core C (r1 x r2 x r3 x r4) and the leaf bases; fills the
// import layout U1..U4, C12, C34, root.
void htucker_interior(const std::vector<cd>& C, const int r[4], const std::vector<std::vector<cd>>& leaves,
                      double budget2, double nx2, Factors& out, int nthreads) {
  const int r1 = r[0], r2 = r[1], r3 = r[2], r4 = r[3];
  int m12 = r1 * r2, m34 = r3 * r4;
  // W12 = core as (r1 r2) x (r3 r4); C12 from W12, C34 from W12^T (Algorithm 2 steps 5-8)
  Basis c12 = left_basis(C, m12, m34, budget2, nthreads);
  std::vector<cd> Wt((size_t)m34 * m12);
  for (int i = 0; i < m12; ++i)
    for (int j = 0; j < m34; ++j) Wt[(size_t)j * m12 + i] = C[(size_t)i * m34 + j];
  Basis c34 = left_basis(Wt, m34, m12, budget2, nthreads);
  // root B = C12^H W12 conj(C34)  (steps 9-10): first T = C12^H W12 (r12 x m34)
  std::vector<cd> T = adjoint_times(c12.U, m12, c12.r, C, m34, nthreads);
  std::vector<cd> Bm((size_t)c12.r * c34.r, 0.0);
  for (int i = 0; i < c12.r; ++i)
    for (int j = 0; j < c34.r; ++j) {
      cd s = 0.0;
      for (int k = 0; k < m34; ++k) s += T[(size_t)i * m34 + k] * std::conj(c34.U[(size_t)k * c34.r + j]);
      Bm[(size_t)i * c34.r + j] = s;
    }
  out.ranks = {r1, r2, r3, r4, c12.r, c34.r};
  out.rel_err = std::sqrt(std::max(0.0, nx2 - norm2(Bm)) / nx2);
  for (int m = 0; m < 4; ++m) append(out.data, leaves[m]);
  append(out.data, c12.U);  // C12[a1][a2][b]
  append(out.data, c34.U);  // C34[a3][a4][b']
  append(out.data, Bm);
}

std::string compress_operator(const std::vector<cd>& That, int ndir, const int n[3], int fmt, double gamma,
                              Factors& out, int nthreads) {
  const long long N = (long long)n[0] * n[1] * n[2];
  out = Factors();
  out.fmt = fmt;
  for (int i = 0; i < 3; ++i) out.n[i] = n[i];
  out.ndir = ndir;
  if ((long long)That.size() != N * ndir) return "operator size mismatch";
  if (fmt == 0) {
    out.data = That;
    out.rel_err = 0.0;
    out.max_dir_err = 0.0;
    return "";
  }
  if (fmt == 1 || fmt == 2) {
    // per-direction 3-D formats: directions in parallel, each single-threaded
    std::vector<std::vector<cd>> blocks(ndir);
    std::vector<std::vector<int32_t>> rk(ndir);
    std::vector<double> e2(ndir), x2(ndir);
    parallel_for(ndir, nthreads, [&](int p) {
      std::vector<cd> X(That.begin() + (size_t)p * N, That.begin() + (size_t)(p + 1) * N);
      double nx2 = norm2(X);
      x2[p] = nx2;
      Shape sh{{n[0], n[1], n[2]}};
      if (fmt == 1) {
        double budget2 = gamma * gamma / 3.0 * nx2;
        std::vector<Basis> B(3);
        for (int m = 0; m < 3; ++m) B[m] = basis_from_gram(mode_gram(X.data(), sh, m, 1), n[m], budget2);
        std::vector<cd> C = project_all(X, sh, B, 1);
        e2[p] = std::max(0.0, nx2 - norm2(C));
        rk[p] = {B[0].r, B[1].r, B[2].r};
        std::vector<cd>& blk = blocks[p];
        append(blk, C);
        for (int m = 0; m < 3; ++m) append(blk, B[m].U);
      } else {
        double budget2 = gamma * gamma / 2.0 * nx2;
        // step 1: n1 x (n2 n3)
        Basis b1 = left_basis(X, n[0], (long long)n[1] * n[2], budget2, 1);
        std::vector<cd> C1 = adjoint_times(b1.U, n[0], b1.r, X, (long long)n[1] * n[2], 1);  // r1 x (n2 n3)
        // step 2: (r1 n2) x n3
        int m2 = b1.r * n[1];
        Basis b2 = left_basis(C1, m2, n[2], budget2, 1);
        std::vector<cd> carry = adjoint_times(b2.U, m2, b2.r, C1, n[2], 1);  // r2 x n3
        e2[p] = std::max(0.0, nx2 - norm2(carry));
        rk[p] = {b1.r, b2.r};
        std::vector<cd>& blk = blocks[p];
        append(blk, b1.U);  // U1 n1 x r1
        append(blk, b2.U);  // C r1 x n2 x r2 (rows (a, y), column b)
        std::vector<cd> U3((size_t)n[2] * b2.r);  // U3[z][b] = carry[b][z]
        for (int b = 0; b < b2.r; ++b)
          for (int z = 0; z < n[2]; ++z) U3[(size_t)z * b2.r + b] = carry[(size_t)b * n[2] + z];
        append(blk, U3);
      }
    });
    double te2 = 0.0, tx2 = 0.0, mx = 0.0;
    for (int p = 0; p < ndir; ++p) {
      te2 += e2[p];
      tx2 += x2[p];
      mx = std::max(mx, x2[p] > 0 ? std::sqrt(e2[p] / x2[p]) : 0.0);
      out.ranks.insert(out.ranks.end(), rk[p].begin(), rk[p].end());
      append(out.data, blocks[p]);
    }
    out.rel_err = tx2 > 0 ? std::sqrt(te2 / tx2) : 0.0;
    out.max_dir_err = mx;
    return "";
  }
  // 4-D formats on X4[x][y][z][p]
  std::vector<cd> X4((size_t)N * ndir);
  parallel_for(ndir, nthreads, [&](int p) {
    for (long long i = 0; i < N; ++i) X4[(size_t)i * ndir + p] = That[(size_t)p * N + i];
  });
  double nx2 = norm2(X4);
  Shape sh{{n[0], n[1], n[2], ndir}};
  if (fmt == 3 || fmt == 5) {
    double budget2 = gamma * gamma / (fmt == 3 ? 4.0 : 6.0) * nx2;
    std::vector<Basis> B(4);
    for (int m = 0; m < 4; ++m) B[m] = basis_from_gram(mode_gram(X4.data(), sh, m, nthreads), (int)sh.d[m], budget2);
    std::vector<cd> C = project_all(X4, sh, B, nthreads);  // r1 x r2 x r3 x r4
    if (fmt == 3) {
      out.ranks = {B[0].r, B[1].r, B[2].r, B[3].r};
      out.rel_err = std::sqrt(std::max(0.0, nx2 - norm2(C)) / nx2);
      append(out.data, C);
      for (int m = 0; m < 4; ++m) append(out.data, B[m].U);
      return "";
    }
    std::vector<std::vector<cd>> leaves(4);
    for (int m = 0; m < 4; ++m) leaves[m] = B[m].U;
    const int r[4] = {B[0].r, B[1].r, B[2].r, B[3].r};
    htucker_interior(C, r, leaves, budget2, nx2, out, nthreads);
    return "";
  }
  if (fmt == 4) {
    double budget2 = gamma * gamma / 3.0 * nx2;
    long long rest1 = (long long)n[1] * n[2] * ndir;
    Basis b1 = left_basis(X4, n[0], rest1, budget2, nthreads);
    std::vector<cd> C1 = adjoint_times(b1.U, n[0], b1.r, X4, rest1, nthreads);  // r1 x (n2 n3 ndir)
    int m2 = b1.r * n[1];
    long long rest2 = (long long)n[2] * ndir;
    Basis b2 = left_basis(C1, m2, rest2, budget2, nthreads);
    std::vector<cd> C2 = adjoint_times(b2.U, m2, b2.r, C1, rest2, nthreads);  // r2 x (n3 ndir)
    int m3 = b2.r * n[2];
    Basis b3 = left_basis(C2, m3, ndir, budget2, nthreads);
    std::vector<cd> carry = adjoint_times(b3.U, m3, b3.r, C2, ndir, nthreads);  // r3 x ndir
    out.ranks = {b1.r, b2.r, b3.r};
    out.rel_err = std::sqrt(std::max(0.0, nx2 - norm2(carry)) / nx2);
    append(out.data, b1.U);  // U1 n1 x r1
    append(out.data, b2.U);  // C1 r1 x n2 x r2
    append(out.data, b3.U);  // C2 r2 x n3 x r3
    std::vector<cd> U3((size_t)ndir * b3.r);
    for (int c = 0; c < b3.r; ++c)
      for (int p = 0; p < ndir; ++p) U3[(size_t)p * b3.r + c] = carry[(size_t)c * ndir + p];
    append(out.data, U3);
    return "";
  }
  return "unknown format";
}

}  // namespace tfmm
