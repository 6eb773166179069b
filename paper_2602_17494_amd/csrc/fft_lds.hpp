// Mixed-radix (2, 3, 4, 5, 8, 9) Stockham FFT staged in LDS.
//
// A workgroup of NT threads transforms `batch` independent complex sequences
// of length n.  Two LDS buffers are used in turn: each pass reads every
// butterfly's inputs from one buffer and writes the outputs to their
// self-sorting positions (Stockham autosort) in the other, with one barrier
// per pass.  The first pass may read its inputs from anywhere (global memory,
// a fused pre-processing step) and the last pass may write anywhere, which
// saves the LDS round trips of loading and storing the data.  Twiddles come from a table tw[m] = exp(-2 pi i m/n)
// in global memory (L1/L2 resident).  Forward transforms use the exp(-...)
// convention and are unnormalised; the inverse uses exp(+...).
#pragma once

#include <type_traits>

#include "tvs_internal.hpp"

namespace tvs {

constexpr int kFftThreads = 256;       // workgroup size for short transforms
constexpr int kFftThreadsLong = 1024;  // workgroup size for long transforms

// Elements per thread per pass the engine is sized for (butterflies per
// thread = elems / radix, rounded up).
template <typename T, int NT> struct FftCap { static constexpr int elems = 8; };
template <> struct FftCap<float, 1024> { static constexpr int elems = 10; };

template <typename T>
__device__ __forceinline__ void dft2(cplx<T>& a, cplx<T>& b) {
  const cplx<T> s = cadd(a, b), d = csub(a, b);
  a = s;
  b = d;
}

template <typename T>
__device__ __forceinline__ void dft3(cplx<T>& a, cplx<T>& b, cplx<T>& c, bool inv) {
  using C = cplx<T>;
  const T s = inv ? T(-0.86602540378443864676) : T(0.86602540378443864676);
  const C sum = cadd(b, c), dif = csub(b, c);
  const C mid = C{a.x - T(0.5) * sum.x, a.y - T(0.5) * sum.y};
  const C rot = C{s * dif.y, -s * dif.x};  // -i s (b - c)
  a = cadd(a, sum);
  b = cadd(mid, rot);
  c = csub(mid, rot);
}

template <typename T>
__device__ __forceinline__ void dft4(cplx<T>& a, cplx<T>& b, cplx<T>& c, cplx<T>& d, bool inv) {
  using C = cplx<T>;
  const C s0 = cadd(a, c), d0 = csub(a, c);
  const C s1 = cadd(b, d), d1 = csub(b, d);
  const C mi = inv ? C{-d1.y, d1.x} : C{d1.y, -d1.x};  // (+i or -i) d1
  a = cadd(s0, s1);
  c = csub(s0, s1);
  b = cadd(d0, mi);
  d = csub(d0, mi);
}

// Last stage of the radix-8 butterfly: the 4-point DFTs e of the even and o
// of the odd inputs, o twiddled by w8^k, combined by 2-point DFTs.
template <typename T>
__device__ __forceinline__ void radix8_combine(cplx<T>* v, cplx<T> e0, cplx<T> e1, cplx<T> e2, cplx<T> e3,
                                               cplx<T> o0, cplx<T> o1, cplx<T> o2, cplx<T> o3, bool inv) {
  using C = cplx<T>;
  const T h = T(0.70710678118654752440);
  // forward w8 = (1 - i)/sqrt2, w8^2 = -i, w8^3 = (-1 - i)/sqrt2; the inverse conjugates
  const C t1 = inv ? C{h * (o1.x - o1.y), h * (o1.x + o1.y)} : C{h * (o1.x + o1.y), h * (o1.y - o1.x)};
  const C t2 = inv ? C{-o2.y, o2.x} : C{o2.y, -o2.x};
  const C t3 = inv ? C{-h * (o3.x + o3.y), h * (o3.x - o3.y)} : C{h * (o3.y - o3.x), -h * (o3.x + o3.y)};
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1);
  v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2);
  v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3);
  v[7] = csub(e3, t3);
}

// The radix-8 butterfly when inputs 4..7 are zero (the first pass of a
// transform of a sequence that is zero on its upper half): each 4-point DFT
// has two non-zero inputs a, b and gives a + b, a -/+ i b, a - b, a +/- i b.
// Equal to butterfly<8> on such inputs up to the sign of zero results.
template <typename T>
__device__ __forceinline__ void butterfly8_half(cplx<T>* v, bool inv) {
  using C = cplx<T>;
  const C m2 = inv ? C{-v[2].y, v[2].x} : C{v[2].y, -v[2].x};  // (+i or -i) v2, as in dft4
  const C m3 = inv ? C{-v[3].y, v[3].x} : C{v[3].y, -v[3].x};
  radix8_combine(v, cadd(v[0], v[2]), cadd(v[0], m2), csub(v[0], v[2]), csub(v[0], m2), cadd(v[1], v[3]),
                 cadd(v[1], m3), csub(v[1], v[3]), csub(v[1], m3), inv);
}

template <int R, typename T>
__device__ __forceinline__ void butterfly(cplx<T>* v, bool inv) {
  using C = cplx<T>;
  if constexpr (R == 2) {
    dft2(v[0], v[1]);
  } else if constexpr (R == 3) {
    dft3(v[0], v[1], v[2], inv);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3], inv);
  } else if constexpr (R == 5) {
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
    const T s1 = inv ? T(-0.95105651629515357212) : T(0.95105651629515357212);
    const T s2 = inv ? T(-0.58778525229247312917) : T(0.58778525229247312917);
    const C x0 = v[0];
    const C a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const C a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const C r1 = C{x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y};
    const C r2 = C{x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y};
    // i1 = s1 b1 + s2 b2, i2 = s2 b1 - s1 b2; y = r -/+ i * i
    const C i1 = C{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y};
    const C i2 = C{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y};
    v[0] = C{x0.x + a1.x + a2.x, x0.y + a1.y + a2.y};
    v[1] = C{r1.x + i1.y, r1.y - i1.x};
    v[4] = C{r1.x - i1.y, r1.y + i1.x};
    v[2] = C{r2.x + i2.y, r2.y - i2.x};
    v[3] = C{r2.x - i2.y, r2.y + i2.x};
  } else if constexpr (R == 8) {
    // 4-point DFTs of the even and odd inputs, twiddles w8^k, then 2-point
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3, inv);
    dft4(o0, o1, o2, o3, inv);
    radix8_combine(v, e0, e1, e2, e3, o0, o1, o2, o3, inv);
  } else if constexpr (R == 9) {
    // 3-point DFTs of the stride-3 inputs, twiddles w9^(l k), then 3-point
    C y[3][3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      y[l][0] = v[l];
      y[l][1] = v[3 + l];
      y[l][2] = v[6 + l];
      dft3(y[l][0], y[l][1], y[l][2], inv);
    }
    // w9^1, w9^2, w9^4 (forward: exp(-2 pi i e / 9)); the inverse conjugates
    const T c1 = T(0.76604444311897803520), s1v = T(0.64278760968653932632);
    const T c2 = T(0.17364817766693034885), s2v = T(0.98480775301220805936);
    const T c4 = T(-0.93969262078590838405), s4v = T(0.34202014332566873304);
    const T sg = inv ? T(1) : T(-1);
    const C w1 = C{c1, sg * s1v}, w2 = C{c2, sg * s2v}, w4 = C{c4, sg * s4v};
    y[1][1] = cmul(y[1][1], w1);
    y[1][2] = cmul(y[1][2], w2);
    y[2][1] = cmul(y[2][1], w2);
    y[2][2] = cmul(y[2][2], w4);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      C a = y[0][k], b = y[1][k], c = y[2][k];
      dft3(a, b, c, inv);
      v[k] = a;
      v[k + 3] = b;
      v[k + 6] = c;
    }
  }
}

// One Stockham pass of radix R over `batch` sequences of length n = R * nbf:
// butterfly j of sequence b takes inputs j + t * nbf (t < R), twiddled by
// w^(k t twstep) with k = j mod Ls, and writes outputs g Ls R + k + t Ls,
// g = j / Ls.  Inputs come from ld(b, index, t) and outputs go to
// st(b, index, value), so a pass can read or write global memory directly
// (t lets a loader pick per-input data it prepared in registers).
template <typename T, int NT, int R, typename LD, typename ST>
__device__ __forceinline__ void fft_pass_io(LD& ld, ST& st, int batch, FastDiv fls, FastDiv fnbf,
                                            int twstep, const cplx<T>* __restrict__ tw, bool inv) {
  using C = cplx<T>;
  const int nbf = fnbf.d, Ls = fls.d;
  const int total = nbf * batch;
  for (int jj = threadIdx.x; jj < total; jj += NT) {
    const int b = fnbf.div(jj);
    const int j = jj - b * nbf;
    const int g = fls.div(j);
    const int k = j - g * Ls;
    C v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) v[t] = ld(b, j + t * nbf, t);
    if (Ls > 1) {  // the first pass (Ls == 1) has k == 0: no twiddles
#pragma unroll
      for (int t = 1; t < R; ++t) {
        C w = tw[k * t * twstep];
        if (inv) w.y = -w.y;
        v[t] = cmul(v[t], w);
      }
    }
    butterfly<R, T>(v, inv);
    const int base = g * Ls * R + k;
#pragma unroll
    for (int t = 0; t < R; ++t) st(b, base + t * Ls, v[t]);
  }
}

template <typename T, int NT, typename LD, typename ST>
__device__ __forceinline__ void fft_pass_radix(int radix, LD& ld, ST& st, int batch, FastDiv fls,
                                               FastDiv fnbf, int twstep,
                                               const cplx<T>* __restrict__ tw, bool inv) {
  switch (radix) {
    case 8: fft_pass_io<T, NT, 8>(ld, st, batch, fls, fnbf, twstep, tw, inv); break;
    case 9: fft_pass_io<T, NT, 9>(ld, st, batch, fls, fnbf, twstep, tw, inv); break;
    case 4: fft_pass_io<T, NT, 4>(ld, st, batch, fls, fnbf, twstep, tw, inv); break;
    case 2: fft_pass_io<T, NT, 2>(ld, st, batch, fls, fnbf, twstep, tw, inv); break;
    case 3: fft_pass_io<T, NT, 3>(ld, st, batch, fls, fnbf, twstep, tw, inv); break;
    default: fft_pass_io<T, NT, 5>(ld, st, batch, fls, fnbf, twstep, tw, inv); break;
  }
}

// Element e of an LDS transform buffer is stored at lds_swz(e): a bijection
// within each aligned block of 32 elements (bits 0-4 are XORed with bits 3-7)
// that spreads the strided accesses of the Stockham passes over the LDS
// banks.  Buffers hold lds_round(n) elements so that blocks do not straddle
// them.
__device__ __forceinline__ int lds_swz(int e) { return e ^ ((e >> 3) & 7) ^ (((e >> 6) & 3) << 3); }
__host__ __device__ constexpr int lds_round(int n) { return (n + 31) & ~31; }

// Sequence s, element i of an LDS buffer holding sequences `stride` apart.
template <typename T>
struct LdsSeq {
  cplx<T>* p;
  int stride;
  __device__ __forceinline__ cplx<T> operator()(int s, int i, int) const { return p[lds_swz(s * stride + i)]; }
  __device__ __forceinline__ void operator()(int s, int i, cplx<T> v) const { p[lds_swz(s * stride + i)] = v; }
};

// Passes 1 .. npass-1 of descriptor d (npass >= 2), after pass 0 has written
// LDS buffer p0 and a barrier: pass p < npass-1 writes p0 (p even) or p1 (p
// odd), with a barrier after it; the last pass writes through `last`.
template <typename T, int NT, typename ST>
__device__ __forceinline__ void fft_run_tail(const FftDesc& d, ST& last, cplx<T>* p0, cplx<T>* p1,
                                             int stride, int batch, const cplx<T>* __restrict__ tw,
                                             bool inv) {
  const int np = d.npass;
  for (int p = 1; p < np - 1; ++p) {
    LdsSeq<T> i{(p & 1) ? p0 : p1, stride}, o{(p & 1) ? p1 : p0, stride};
    fft_pass_radix<T, NT>(d.radix[p], i, o, batch, d.ls[p], d.nbf[p], d.twstep[p], tw, inv);
    __syncthreads();
  }
  LdsSeq<T> i{((np - 1) & 1) ? p0 : p1, stride};
  fft_pass_radix<T, NT>(d.radix[np - 1], i, last, batch, d.ls[np - 1], d.nbf[np - 1],
                        d.twstep[np - 1], tw, inv);
}

// All passes of descriptor d.  Pass 0 reads through `first`; pass p < npass-1
// writes LDS buffer p0 (p even) or p1 (p odd), with a barrier after it; the
// last pass writes through `last`.  `first` must not read a buffer that pass
// 0 writes, and whatever it reads from LDS must be complete (barrier) before
// the call.
template <typename T, int NT, typename LD, typename ST>
__device__ __forceinline__ void fft_run(const FftDesc& d, LD& first, ST& last, cplx<T>* p0,
                                        cplx<T>* p1, int stride, int batch,
                                        const cplx<T>* __restrict__ tw, bool inv) {
  if (d.npass == 1) {
    fft_pass_radix<T, NT>(d.radix[0], first, last, batch, d.ls[0], d.nbf[0], d.twstep[0], tw, inv);
    return;
  }
  {
    LdsSeq<T> o{p0, stride};
    fft_pass_radix<T, NT>(d.radix[0], first, o, batch, d.ls[0], d.nbf[0], d.twstep[0], tw, inv);
  }
  __syncthreads();
  fft_run_tail<T, NT>(d, last, p0, p1, stride, batch, tw, inv);
}

// As fft_run with the result left in LDS; returns the buffer that holds it
// (p0 or p1) and ends with a barrier.
template <typename T, int NT, typename LD>
__device__ __forceinline__ cplx<T>* fft_run_to_lds(const FftDesc& d, LD& first, cplx<T>* p0,
                                                   cplx<T>* p1, int stride, int batch,
                                                   const cplx<T>* __restrict__ tw, bool inv) {
  cplx<T>* res = ((d.npass - 1) & 1) ? p1 : p0;
  LdsSeq<T> o{res, stride};
  fft_run<T, NT>(d, first, o, p0, p1, stride, batch, tw, inv);
  __syncthreads();
  return res;
}

// Transform `batch` sequences of length d.n held in buffer a (sequence b at
// elements b * stride of it, swizzled), using bbuf as the second buffer;
// returns the buffer that holds the result.  The caller's writes to a must be complete (barrier)
// before the call; the call ends with a barrier.
template <typename T, int NT>
__device__ __forceinline__ cplx<T>* fft_lds(cplx<T>* a, cplx<T>* bbuf, const FftDesc& d, int stride,
                                            int batch, const cplx<T>* __restrict__ tw, bool inv) {
  LdsSeq<T> in{a, stride};
  return fft_run_to_lds<T, NT>(d, in, bbuf, a, stride, batch, tw, inv);
}

// ---------------------------------------------------------------------------
// One-buffer variant for transforms too long for two LDS buffers.  Every
// pass loads the inputs of all its butterflies into registers, waits at a
// barrier, and writes the outputs back into the same buffer, so the whole
// LDS (160 KB per workgroup on gfx950) holds one copy of the data: up to
// kLdsElems<T> elements (10240 complex float64, 20480 complex float32) per
// workgroup, with 1024 threads.  The caller guarantees batch * n <=
// kLdsElems<T>, which bounds the butterflies a thread holds per pass.
// ---------------------------------------------------------------------------
constexpr int kLdsBytes = 160 * 1024;
template <typename T> constexpr int kLdsElems = kLdsBytes / int(sizeof(cplx<T>));
// largest radix the one-buffer plans use (make_fft_desc's max_radix)
template <typename T> constexpr int kLongRadix = sizeof(T) == 8 ? 4 : 8;

template <typename T, int NT, int R, typename LD, typename ST>
__device__ __forceinline__ void fft_pass_1b(LD& ld, ST& st, int batch, FastDiv fls, FastDiv fnbf,
                                            int twstep, const cplx<T>* __restrict__ tw, bool inv) {
  using C = cplx<T>;
  constexpr int MB = (kLdsElems<T> + R * NT - 1) / (R * NT);  // butterflies per thread
  const int nbf = fnbf.d, Ls = fls.d;
  const int total = nbf * batch;
  C v[MB][R];
  int bb[MB], base[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int jj = threadIdx.x + m * NT;
    if (jj < total) {
      const int b = fnbf.div(jj);
      const int j = jj - b * nbf;
      const int g = fls.div(j);
      const int k = j - g * Ls;
#pragma unroll
      for (int t = 0; t < R; ++t) v[m][t] = ld(b, j + t * nbf, t);
      if (Ls > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) {
          C w = tw[k * t * twstep];
          if (inv) w.y = -w.y;
          v[m][t] = cmul(v[m][t], w);
        }
      }
      bb[m] = b;
      base[m] = g * Ls * R + k;
    }
  }
  __syncthreads();  // every input of the pass is read before any output lands
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int jj = threadIdx.x + m * NT;
    if (jj < total) {
      butterfly<R, T>(v[m], inv);
#pragma unroll
      for (int t = 0; t < R; ++t) st(bb[m], base[m] + t * Ls, v[m][t]);
    }
  }
}

template <typename T, int NT, typename LD, typename ST>
__device__ __forceinline__ void fft_pass_radix_1b(int radix, LD& ld, ST& st, int batch, FastDiv fls,
                                                  FastDiv fnbf, int twstep, const cplx<T>* __restrict__ tw,
                                                  bool inv) {
  // only the radices of make_fft_desc(n, kLongRadix<T>) are instantiated,
  // so that the register budget is that of the largest of them
  switch (radix) {
    case 8:
      if constexpr (kLongRadix<T> >= 8) fft_pass_1b<T, NT, 8>(ld, st, batch, fls, fnbf, twstep, tw, inv);
      break;
    case 4: fft_pass_1b<T, NT, 4>(ld, st, batch, fls, fnbf, twstep, tw, inv); break;
    case 2: fft_pass_1b<T, NT, 2>(ld, st, batch, fls, fnbf, twstep, tw, inv); break;
    case 3: fft_pass_1b<T, NT, 3>(ld, st, batch, fls, fnbf, twstep, tw, inv); break;
    default: fft_pass_1b<T, NT, 5>(ld, st, batch, fls, fnbf, twstep, tw, inv); break;
  }
}

// All passes of d in one LDS buffer: pass 0 reads through `first` and writes
// buf; the middle passes transform buf in place; the last pass writes
// through `last`.  A barrier separates consecutive passes.  What `first`
// reads from LDS must be complete (barrier) before the call.
template <typename T, int NT, typename LD, typename ST>
__device__ __forceinline__ void fft_run_1b(const FftDesc& d, LD& first, ST& last, cplx<T>* buf, int stride,
                                           int batch, const cplx<T>* __restrict__ tw, bool inv) {
  LdsSeq<T> io{buf, stride};
  const int np = d.npass;
  for (int p = 0; p < np; ++p) {
    if (p == 0 && np == 1) {
      fft_pass_radix_1b<T, NT>(d.radix[0], first, last, batch, d.ls[0], d.nbf[0], d.twstep[0], tw, inv);
    } else if (p == 0) {
      fft_pass_radix_1b<T, NT>(d.radix[0], first, io, batch, d.ls[0], d.nbf[0], d.twstep[0], tw, inv);
    } else if (p < np - 1) {
      fft_pass_radix_1b<T, NT>(d.radix[p], io, io, batch, d.ls[p], d.nbf[p], d.twstep[p], tw, inv);
    } else {
      fft_pass_radix_1b<T, NT>(d.radix[p], io, last, batch, d.ls[p], d.nbf[p], d.twstep[p], tw, inv);
    }
    if (p < np - 1) __syncthreads();
  }
}

// As fft_run_1b with the result left in buf; ends with a barrier.
template <typename T, int NT, typename LD>
__device__ __forceinline__ cplx<T>* fft_run_to_lds_1b(const FftDesc& d, LD& first, cplx<T>* buf, int stride,
                                                      int batch, const cplx<T>* __restrict__ tw, bool inv) {
  LdsSeq<T> o{buf, stride};
  fft_run_1b<T, NT>(d, first, o, buf, stride, batch, tw, inv);
  __syncthreads();
  return buf;
}

// Transform `batch` sequences held in buf in place; ends with a barrier.
template <typename T, int NT>
__device__ __forceinline__ cplx<T>* fft_lds_1b(cplx<T>* buf, const FftDesc& d, int stride, int batch,
                                               const cplx<T>* __restrict__ tw, bool inv) {
  LdsSeq<T> in{buf, stride};
  return fft_run_to_lds_1b<T, NT>(d, in, buf, stride, batch, tw, inv);
}

// ---------------------------------------------------------------------------
// The same passes for a transform length fixed at compile time: with the
// radix, butterfly count, Ls and twiddle step of every pass known, the
// butterfly and twiddle index arithmetic folds into shifts, masks and
// full-rate 24-bit multiplies, and the sequence stride into constants.
// Three-pass lengths only (512 = 8 * 8 * 8, 576 = 8 * 8 * 9 and
// 648 = 8 * 9 * 9, with the radices in the plans' order).  The
// arithmetic is that of the runtime-descriptor passes; the compiler may fuse
// multiplies and adds differently, so results can differ in the last bits.
// ---------------------------------------------------------------------------
template <int N, int R0, int R1, int R2>
struct Fft3 {
  static_assert(R0 * R1 * R2 == N, "radices must multiply to the length");
  static constexpr int n = N;
  template <int P> static constexpr int radix() { return P == 0 ? R0 : P == 1 ? R1 : R2; }
  template <int P> static constexpr int ls() { return P == 0 ? 1 : P == 1 ? R0 : R0 * R1; }
  template <int P> static constexpr int nbf() { return N / radix<P>(); }
  template <int P> static constexpr int twstep() { return N / (ls<P>() * radix<P>()); }
  // true if this descriptor describes the runtime plan d
  static bool matches(const FftDesc& d) {
    return d.n == N && d.npass == 3 && d.radix[0] == R0 && d.radix[1] == R1 && d.radix[2] == R2;
  }
};
using Fft512 = Fft3<512, 8, 8, 8>;
using Fft576 = Fft3<576, 8, 8, 9>;
using Fft648 = Fft3<648, 8, 9, 9>;
// the compile-time descriptor of a length (SL = 512, 576 or 648)
template <int SL>
using FftOf = std::conditional_t<SL == 512, Fft512, std::conditional_t<SL == 576, Fft576, Fft648>>;

template <typename T, int STRIDE>
struct LdsSeqS {
  cplx<T>* p;
  __device__ __forceinline__ cplx<T> operator()(int s, int i, int) const { return p[lds_swz(s * STRIDE + i)]; }
  __device__ __forceinline__ void operator()(int s, int i, cplx<T> v) const { p[lds_swz(s * STRIDE + i)] = v; }
};

// HALF (pass 0 of a radix-8 first pass only): the sequence is zero from
// half its length on, so inputs t >= 4 of every butterfly are zero and are
// neither loaded nor added.
template <typename T, int NT, typename D, int P, bool HALF = false, typename LD, typename ST>
__device__ __forceinline__ void fft_pass_s(LD& ld, ST& st, int batch, const cplx<T>* __restrict__ tw, bool inv) {
  using C = cplx<T>;
  constexpr int R = D::template radix<P>(), NBF = D::template nbf<P>(), LS = D::template ls<P>(),
                TWS = D::template twstep<P>();
  static_assert(!HALF || (P == 0 && R == 8), "the half-input pass is the radix-8 first pass");
  const int total = NBF * batch;
  for (int jj = threadIdx.x; jj < total; jj += NT) {
    const int b = jj / NBF;
    const int j = jj - b * NBF;
    const int g = j / LS;
    const int k = j - g * LS;
    C v[R];
    if constexpr (HALF) {
#pragma unroll
      for (int t = 0; t < R / 2; ++t) v[t] = ld(b, j + t * NBF, t);
      butterfly8_half<T>(v, inv);
    } else {
#pragma unroll
      for (int t = 0; t < R; ++t) v[t] = ld(b, j + t * NBF, t);
      if constexpr (LS > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) {
          C w = tw[__mul24(k, t * TWS)];  // k < LS, so the 24-bit product is exact
          if (inv) w.y = -w.y;
          v[t] = cmul(v[t], w);
        }
      }
      butterfly<R, T>(v, inv);
    }
    const int base = g * (LS * R) + k;
#pragma unroll
    for (int t = 0; t < R; ++t) st(b, base + t * LS, v[t]);
  }
}

// passes 1 and 2 after pass 0 has written p0 (and a barrier): pass 1 writes
// p1, the last pass writes through `last`
template <typename T, int NT, typename D, typename ST>
__device__ __forceinline__ void fft_run_tail_s(ST& last, cplx<T>* p0, cplx<T>* p1, int batch,
                                               const cplx<T>* __restrict__ tw, bool inv) {
  LdsSeqS<T, D::n> a{p0}, b{p1};
  fft_pass_s<T, NT, D, 1>(a, b, batch, tw, inv);
  __syncthreads();
  fft_pass_s<T, NT, D, 2>(b, last, batch, tw, inv);
}

template <typename T, int NT, typename D, bool HALF0 = false, typename LD, typename ST>
__device__ __forceinline__ void fft_run_s(LD& first, ST& last, cplx<T>* p0, cplx<T>* p1, int batch,
                                          const cplx<T>* __restrict__ tw, bool inv) {
  {
    LdsSeqS<T, D::n> o{p0};
    fft_pass_s<T, NT, D, 0, HALF0>(first, o, batch, tw, inv);
  }
  __syncthreads();
  fft_run_tail_s<T, NT, D>(last, p0, p1, batch, tw, inv);
}

// as fft_run_to_lds: the result (in p0, three passes) ends with a barrier;
// HALF0: the input sequences are zero from half their length on
template <typename T, int NT, typename D, bool HALF0 = false, typename LD>
__device__ __forceinline__ cplx<T>* fft_run_to_lds_s(LD& first, cplx<T>* p0, cplx<T>* p1, int batch,
                                                     const cplx<T>* __restrict__ tw, bool inv) {
  LdsSeqS<T, D::n> o{p0};
  fft_run_s<T, NT, D, HALF0>(first, o, p0, p1, batch, tw, inv);
  __syncthreads();
  return p0;
}

template <typename T, int NT, typename D, bool HALF0 = false>
__device__ __forceinline__ cplx<T>* fft_lds_s(cplx<T>* a, cplx<T>* bbuf, int batch, const cplx<T>* __restrict__ tw,
                                              bool inv) {
  LdsSeqS<T, D::n> in{a};
  return fft_run_to_lds_s<T, NT, D, HALF0>(in, bbuf, a, batch, tw, inv);
}

}  // namespace tvs
