"""Generate straight-line DFT codelets for the translation kernels (build step).

Writes dft_codelets.h: for each line length n used by the padded FFT grids,

  dft_fwd_<n>(x, y)   forward DFT (exp(-2 pi i jk/n)) of a length-n line whose
                      last n/2 entries are zero (zero padding); x holds n/2
                      values, y receives all n outputs;
  dft_inv_<n>(x, y)   unnormalised inverse DFT (exp(+2 pi i jk/n)) of n values,
                      of which only the first n/2 outputs are produced (the crop
                      back to the box grid);
  dft_full_fwd_<t> / dft_full_inv_<t>   plain length-t DFTs (t <= 8, 12, 16, 24, 32).

Each codelet is a recursive decimation-in-time mixed-radix (4, 2, 3) DFT
unrolled into SSA statements on float2 registers.  Known-zero inputs are
propagated symbolically and never touched; outputs nobody asks for are
removed by the compiler.  Twiddles are evaluated in double precision and
rounded once to float literals (hex), so no table is read at run time.
"""
from __future__ import annotations

import math
import os
import sys

import numpy as np

LINE_SIZES = (2, 4, 6, 8, 12, 16, 24, 32, 48, 64)
SMALL_SIZES = (1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 24, 32)


def f32hex(v: float) -> str:
    v32 = float(np.float32(v))
    if v32 == 0.0:
        return "0.0f"
    return v32.hex() + "f"


class Emitter:
    def __init__(self):
        self.lines = []
        self.count = 0

    def tmp(self, expr: str) -> str:
        name = f"v{self.count}"
        self.count += 1
        self.lines.append(f"  const float2 {name} = {expr};")
        return name

    # symbolic complex ops; None means an exact zero
    def add(self, a, b):
        if a is None:
            return b
        if b is None:
            return a
        return self.tmp(f"cadd({a}, {b})")

    def sub(self, a, b):
        if b is None:
            return a
        if a is None:
            return self.tmp(f"cneg({b})")
        return self.tmp(f"csub({a}, {b})")

    def mul_i(self, a, s):
        """a * (s*i), s = +1 or -1."""
        if a is None:
            return None
        return self.tmp(f"cmul_i({a})" if s > 0 else f"cmul_mi({a})")

    def twiddle(self, a, num: int, den: int, sign: int):
        """a * exp(sign * 2 pi i num / den)."""
        if a is None:
            return None
        num %= den
        if num == 0:
            return a
        g = math.gcd(num, den)
        num, den = num // g, den // g
        if den == 2:
            return self.tmp(f"cneg({a})")
        if den == 4:
            s = sign if num == 1 else -sign
            return self.mul_i(a, s)
        ang = sign * 2.0 * math.pi * num / den
        c, s = math.cos(ang), math.sin(ang)
        if den == 8:
            h = f32hex(math.sqrt(0.5))
            # (c + i s) with |c| = |s| = 1/sqrt(2)
            sc = "+" if c > 0 else "-"
            ss = "+" if s > 0 else "-"
            return self.tmp(f"cmul_diag({a}, {sc}{h}, {ss}{h})")
        return self.tmp(f"cmulc({a}, {f32hex(c)}, {f32hex(s)})")

    def butterfly(self, t, sign):
        r = len(t)
        if r == 1:
            return list(t)
        if r == 2:
            return [self.add(t[0], t[1]), self.sub(t[0], t[1])]
        if r == 4:
            a, b, c, d = t
            s0 = self.add(a, c)
            s1 = self.sub(a, c)
            s2 = self.add(b, d)
            s3 = self.mul_i(self.sub(b, d), sign)
            return [self.add(s0, s2), self.add(s1, s3), self.sub(s0, s2), self.sub(s1, s3)]
        if r == 3:
            a, b, c = t
            s = self.add(b, c)
            d = self.sub(b, c)
            if s is None and d is None:
                return [a, a, a]
            h = self.tmp(f"cscale({s}, -0.5f)") if s is not None else None
            base = self.add(a, h)
            rot = self.tmp(f"cscale({self.mul_i(d, sign)}, {f32hex(math.sqrt(3.0) / 2.0)})") if d is not None else None
            return [self.add(a, s), self.add(base, rot), self.sub(base, rot)]
        # generic (unused for the sizes above): direct sum
        out = []
        for q in range(r):
            acc = None
            for i in range(r):
                acc = self.add(acc, self.twiddle(t[i], i * q, r, sign))
            out.append(acc)
        return out

    def dft(self, x, sign):
        n = len(x)
        if all(v is None for v in x):
            return [None] * n
        if n == 1:
            return list(x)
        if n % 4 == 0 and n != 8:
            r = 4
        elif n % 2 == 0:
            r = 2
        elif n % 3 == 0:
            r = 3
        else:
            r = n
        if r == n:
            return self.butterfly(x, sign)
        m = n // r
        subs = [self.dft(x[i::r], sign) for i in range(r)]
        out = [None] * n
        for k in range(m):
            t = [self.twiddle(subs[i][k], i * k, n, sign) for i in range(r)]
            y = self.butterfly(t, sign)
            for q in range(r):
                out[k + q * m] = y[q]
        return out


def codelet(name, n, n_in, n_out, sign, comment):
    e = Emitter()
    x = [f"x[{j}]" if j < n_in else None for j in range(n)]
    y = e.dft(x, sign)
    body = list(e.lines)
    for k in range(n_out):
        body.append(f"  y[{k}] = {y[k]};" if y[k] is not None else f"  y[{k}] = make_float2(0.0f, 0.0f);")
    return (f"// {comment}\n"
            f"__device__ __forceinline__ void {name}(const float2* __restrict__ x, float2* __restrict__ y) {{\n"
            + "\n".join(body) + "\n}\n")


HEADER = """// Generated by gen_dft.py -- do not edit.
// Straight-line DFT codelets on float2 registers (see gen_dft.py for the scheme).
#pragma once
#include <hip/hip_runtime.h>

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cneg(float2 a) { return make_float2(-a.x, -a.y); }
__device__ __forceinline__ float2 cmul_i(float2 a) { return make_float2(-a.y, a.x); }
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmulc(float2 a, float c, float s) {
  return make_float2(fmaf(a.x, c, -a.y * s), fmaf(a.x, s, a.y * c));
}
// a * (c + i s) with |c| = |s|
__device__ __forceinline__ float2 cmul_diag(float2 a, float c, float s) {
  return make_float2(fmaf(a.x, c, -a.y * s), fmaf(a.x, s, a.y * c));
}

template <int N> struct Dft;
"""


def main(out_path):
    parts = [HEADER]
    for n in LINE_SIZES:
        h = n // 2
        parts.append(codelet(f"dft_fwd_{n}", n, h, n, -1,
                             f"length {n}, inputs {h}..{n - 1} zero, all {n} outputs"))
        parts.append(codelet(f"dft_inv_{n}", n, n, h, +1,
                             f"length {n} inverse (unnormalised), outputs 0..{h - 1} only"))
        parts.append(f"template <> struct Dft<{n}> {{\n"
                     f"  static constexpr int N = {n};\n"
                     f"  __device__ __forceinline__ static void fwd(const float2* x, float2* y) {{ dft_fwd_{n}(x, y); }}\n"
                     f"  __device__ __forceinline__ static void inv(const float2* x, float2* y) {{ dft_inv_{n}(x, y); }}\n"
                     f"}};\n")
    parts.append("template <int N> struct DftFull;\n")
    for t in SMALL_SIZES:
        parts.append(codelet(f"dft_full_fwd_{t}", t, t, t, -1, f"full forward DFT of length {t}"))
        parts.append(codelet(f"dft_full_inv_{t}", t, t, t, +1, f"full inverse DFT of length {t} (unnormalised)"))
        parts.append(f"template <> struct DftFull<{t}> {{\n"
                     f"  __device__ __forceinline__ static void fwd(const float2* x, float2* y) {{ dft_full_fwd_{t}(x, y); }}\n"
                     f"  __device__ __forceinline__ static void inv(const float2* x, float2* y) {{ dft_full_inv_{t}(x, y); }}\n"
                     f"}};\n")
    src = "\n".join(parts)
    with open(out_path, "w") as f:
        f.write(src)


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(here, "dft_codelets.h"))
