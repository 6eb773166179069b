// Mixed-radix (2, 3, 4, 5) Stockham FFT held entirely in LDS.
//
// A workgroup of NT threads transforms `batch` independent complex
// sequences of length n stored in LDS at buf + b * stride.  Each pass reads
// all of its butterfly inputs into registers, synchronises, and writes the
// outputs to their self-sorting positions (Stockham autosort), so one LDS
// buffer suffices.  Twiddles come from a table tw[m] = exp(-2 pi i m / n)
// kept in global memory (L1/L2 resident).  Forward transforms use the
// exp(-...) convention and are unnormalised; the inverse uses exp(+...).
#pragma once

#include "tvs_internal.hpp"

namespace tvs {

constexpr int kFftThreads = 256;       // workgroup size for short transforms
constexpr int kFftThreadsLong = 1024;  // workgroup size for long transforms

// Elements per thread the register staging can hold for one pass, kept
// small so that several workgroups share a CU (about 100 VGPRs).  The
// 1024-thread float variant holds a little more so that one workgroup can
// transform sequences up to 10240 points.
template <typename T, int NT> struct FftCap { static constexpr int elems = 8; };
template <> struct FftCap<float, 1024> { static constexpr int elems = 10; };

template <int R, typename T>
__device__ __forceinline__ void butterfly(cplx<T>* v, bool inv) {
  using C = cplx<T>;
  if constexpr (R == 2) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    const T s = inv ? T(-0.86602540378443864676) : T(0.86602540378443864676);
    C a = v[0], b = v[1], c = v[2];
    C sum = cadd(b, c);
    C dif = csub(b, c);
    C mid = C{a.x - T(0.5) * sum.x, a.y - T(0.5) * sum.y};
    // -i * s * dif
    C rot = C{s * dif.y, -s * dif.x};
    v[0] = cadd(a, sum);
    v[1] = cadd(mid, rot);
    v[2] = csub(mid, rot);
  } else if constexpr (R == 4) {
    C a = v[0], b = v[1], c = v[2], d = v[3];
    C s0 = cadd(a, c), d0 = csub(a, c);
    C s1 = cadd(b, d), d1 = csub(b, d);
    // forward: y1 = d0 - i d1, y3 = d0 + i d1
    C mi = inv ? C{-d1.y, d1.x} : C{d1.y, -d1.x};  // (-i or +i) * d1
    v[0] = cadd(s0, s1);
    v[2] = csub(s0, s1);
    v[1] = cadd(d0, mi);
    v[3] = csub(d0, mi);
  } else if constexpr (R == 5) {
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
    const T s1 = inv ? T(-0.95105651629515357212) : T(0.95105651629515357212);
    const T s2 = inv ? T(-0.58778525229247312917) : T(0.58778525229247312917);
    C x0 = v[0];
    C a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    C a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    C r1 = C{x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y};
    C r2 = C{x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y};
    // i1 = s1 b1 + s2 b2, i2 = s2 b1 - s1 b2; y = r -/+ i * i
    C i1 = C{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y};
    C i2 = C{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y};
    v[0] = C{x0.x + a1.x + a2.x, x0.y + a1.y + a2.y};
    v[1] = C{r1.x + i1.y, r1.y - i1.x};
    v[4] = C{r1.x - i1.y, r1.y + i1.x};
    v[2] = C{r2.x + i2.y, r2.y - i2.x};
    v[3] = C{r2.x - i2.y, r2.y + i2.x};
  }
}

template <typename T, int NT, int R>
__device__ __forceinline__ void fft_pass(cplx<T>* buf, int stride, int batch, FastDiv fls,
                                         FastDiv fnbf, int twstep, const cplx<T>* __restrict__ tw,
                                         bool inv) {
  using C = cplx<T>;
  constexpr int MAXB = (FftCap<T, NT>::elems + R - 1) / R;
  const int nbf = fnbf.d, Ls = fls.d;
  const int total = nbf * batch;
  C v[MAXB][R];
#pragma unroll
  for (int s = 0; s < MAXB; ++s) {
    const int jj = threadIdx.x + s * NT;
    if (jj < total) {
      const int b = fnbf.div(jj);
      const int j = jj - b * nbf;
      const C* x = buf + b * stride;
      const int k = j - fls.div(j) * Ls;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        C c = x[j + t * nbf];
        if (t > 0) {
          C w = tw[k * t * twstep];
          if (inv) w.y = -w.y;
          c = cmul(c, w);
        }
        v[s][t] = c;
      }
      butterfly<R, T>(v[s], inv);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < MAXB; ++s) {
    const int jj = threadIdx.x + s * NT;
    if (jj < total) {
      const int b = fnbf.div(jj);
      const int j = jj - b * nbf;
      C* y = buf + b * stride;
      const int g = fls.div(j);
      const int k = j - g * Ls;
      const int base = g * Ls * R + k;
#pragma unroll
      for (int t = 0; t < R; ++t) y[base + t * Ls] = v[s][t];
    }
  }
  __syncthreads();
}

// Transform `batch` sequences of length d.n in LDS (sequence b at
// buf + b * stride).  Requires batch * d.n <= NT * FftCap<T, NT>::elems.
template <typename T, int NT>
__device__ void fft_lds(cplx<T>* buf, const FftDesc& d, int stride, int batch,
                        const cplx<T>* __restrict__ tw, bool inv) {
  for (int p = 0; p < d.npass; ++p) {
    const FastDiv ls = d.ls[p], nb = d.nbf[p];
    const int ts = d.twstep[p];
    switch (d.radix[p]) {
      case 4: fft_pass<T, NT, 4>(buf, stride, batch, ls, nb, ts, tw, inv); break;
      case 2: fft_pass<T, NT, 2>(buf, stride, batch, ls, nb, ts, tw, inv); break;
      case 3: fft_pass<T, NT, 3>(buf, stride, batch, ls, nb, ts, tw, inv); break;
      default: fft_pass<T, NT, 5>(buf, stride, batch, ls, nb, ts, tw, inv); break;
    }
  }
}

}  // namespace tvs
