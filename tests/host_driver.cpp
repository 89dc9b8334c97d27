// Test driver for the library's host setup code (host_math.cpp), built with g++
// by tests/test_host_math.py.  Reads a request from stdin-named files and writes
// the compressed factors in the tfmm_op_import layout.
//
//   host_driver compress <in.bin> <out.bin>
//     in:  int32 fmt, ndir, n1, n2, n3; double gamma; complex128 That[ndir][n1][n2][n3]
//     out: int32 nranks, ranks[nranks]; double rel_err, max_dir_err, seconds;
//          int64 ndata; complex128 data[ndata]
//   host_driver eig <in.bin> <out.bin>      (Hermitian eigensolver)
//     in:  int32 n; complex128 A[n][n];  out: double vals[n]; complex128 vecs[n][n]
//   host_driver fft <in.bin> <out.bin>      (3-D forward FFT)
//     in:  int32 batch, n1, n2, n3; complex128 x[...];  out: complex128 X[...]
//   host_driver gl <n> <out.bin>            (Gauss-Legendre nodes and weights)
#include <chrono>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "host_math.h"

using tfmm::cd;

static std::vector<char> slurp(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) std::exit(2);
  std::vector<char> b;
  char buf[1 << 16];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) b.insert(b.end(), buf, buf + n);
  std::fclose(f);
  return b;
}

int main(int argc, char** argv) {
  if (argc < 4) return 1;
  std::string cmd = argv[1];
  FILE* out = std::fopen(argv[3], "wb");
  if (!out) return 2;
  if (cmd == "gl") {
    std::vector<double> x, w;
    tfmm::gauss_legendre(std::atoi(argv[2]), x, w);
    std::fwrite(x.data(), 8, x.size(), out);
    std::fwrite(w.data(), 8, w.size(), out);
    std::fclose(out);
    return 0;
  }
  std::vector<char> in = slurp(argv[2]);
  const char* p = in.data();
  if (cmd == "compress") {
    int32_t hdr[5];
    std::memcpy(hdr, p, sizeof hdr);
    p += sizeof hdr;
    double gamma;
    std::memcpy(&gamma, p, 8);
    p += 8;
    const int fmt = hdr[0], ndir = hdr[1];
    const int n[3] = {hdr[2], hdr[3], hdr[4]};
    const size_t cnt = (size_t)ndir * n[0] * n[1] * n[2];
    std::vector<cd> T(cnt);
    std::memcpy((void*)T.data(), p, cnt * sizeof(cd));
    tfmm::Factors F;
    auto t0 = std::chrono::steady_clock::now();
    std::string err = tfmm::compress_operator(T, ndir, n, fmt, gamma, F, 8);
    double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (!err.empty()) {
      std::fprintf(stderr, "%s\n", err.c_str());
      return 3;
    }
    int32_t nr = (int32_t)F.ranks.size();
    std::fwrite(&nr, 4, 1, out);
    std::fwrite(F.ranks.data(), 4, F.ranks.size(), out);
    std::fwrite(&F.rel_err, 8, 1, out);
    std::fwrite(&F.max_dir_err, 8, 1, out);
    std::fwrite(&sec, 8, 1, out);
    int64_t nd = (int64_t)F.data.size();
    std::fwrite(&nd, 8, 1, out);
    std::fwrite((const void*)F.data.data(), sizeof(cd), F.data.size(), out);
  } else if (cmd == "eig") {
    int32_t nn;
    std::memcpy(&nn, p, 4);
    p += 4;
    std::vector<cd> A((size_t)nn * nn);
    std::memcpy((void*)A.data(), p, A.size() * sizeof(cd));
    std::vector<double> vals;
    std::vector<cd> vecs;
    tfmm::hermitian_eig(nn, A, vals, vecs);
    std::fwrite(vals.data(), 8, vals.size(), out);
    std::fwrite((const void*)vecs.data(), sizeof(cd), vecs.size(), out);
  } else if (cmd == "fft") {
    int32_t hdr[4];
    std::memcpy(hdr, p, sizeof hdr);
    p += sizeof hdr;
    const size_t cnt = (size_t)hdr[0] * hdr[1] * hdr[2] * hdr[3];
    std::vector<cd> X(cnt);
    std::memcpy((void*)X.data(), p, cnt * sizeof(cd));
    tfmm::fft3d_forward(X.data(), hdr[1], hdr[2], hdr[3], hdr[0]);
    std::fwrite((const void*)X.data(), sizeof(cd), X.size(), out);
  } else {
    return 1;
  }
  std::fclose(out);
  return 0;
}
