// Image-method Neumann inverse Laplacian on boxes (see green.hpp).
#include "green.hpp"

#include <set>

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace tvs {

// ---------------------------------------------------------------------------
// FFT descriptors and twiddles (host)
// ---------------------------------------------------------------------------
static bool is_smooth(int n) {
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

int smooth_even_at_least(int n) {
  int m = std::max(n, 2);
  if (m & 1) ++m;
  while (!is_smooth(m)) m += 2;
  return m;
}

int green_length(int side) { return smooth_even_at_least(2 * side - 1); }

bool green_side_ok(int side) { return side >= 1 && lds_round(green_length(side)) <= kLdsElems<double>; }

FastDiv make_fastdiv(int d) {
  if (d < 1 || d >= (1 << 16)) throw Error(-1, "divisor out of range");
  FastDiv f{};
  f.d = d;
  f.m = d == 1 ? 0u : unsigned(((1ULL << 32) + d - 1) / d);
  return f;
}

FftDesc make_fft_desc(int n, int max_radix) {
  FftDesc d{};
  d.n = n;
  int m = n, k = 0;
  auto push = [&](int r) {
    if (k >= kMaxPass) throw Error(-1, "FFT length " + std::to_string(n) + " needs too many passes");
    d.radix[k++] = r;
    m /= r;
  };
  if (max_radix >= 8)
    while (m % 8 == 0) push(8);
  while (m % 4 == 0) push(4);
  while (m % 2 == 0) push(2);
  if (max_radix >= 9)
    while (m % 9 == 0) push(9);
  while (m % 3 == 0) push(3);
  while (m % 5 == 0) push(5);
  if (m != 1) throw Error(-1, "FFT length " + std::to_string(n) + " is not 2^a 3^b 5^c");
  d.npass = k;
  int ls = 1;
  for (int p = 0; p < k; ++p) {
    d.ls[p] = make_fastdiv(ls);
    d.nbf[p] = make_fastdiv(n / d.radix[p]);
    d.twstep[p] = n / (ls * d.radix[p]);
    ls *= d.radix[p];
  }
  return d;
}

template <typename T>
static DevBuf make_twiddles(int n, hipStream_t s) {
  std::vector<cplx<T>> h(n);
  const double two_pi = 6.283185307179586476925286766559;
  for (int m = 0; m < n; ++m) {
    const double a = two_pi * double(m) / double(n);
    h[m] = cplx<T>{T(std::cos(a)), T(-std::sin(a))};
  }
  DevBuf d(sizeof(cplx<T>) * n);
  TVS_HIP(hipMemcpyAsync(d.p, h.data(), sizeof(cplx<T>) * n, hipMemcpyHostToDevice, s));
  TVS_HIP(hipStreamSynchronize(s));
  return d;
}

// ---------------------------------------------------------------------------
// Torus kernel table (float64): G = C2^T (W C1) / (4 n2 n1)
// ---------------------------------------------------------------------------

// cos(pi k v / n) with the argument reduced exactly in integers
__global__ void k_cos_table(double* c, int n) {
  const int k = blockIdx.y;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += gridDim.x * blockDim.x) {
    const long long m = (static_cast<long long>(k) * v) % (2LL * n);
    c[static_cast<long long>(k) * (n + 1) + v] = cospi(static_cast<double>(m) / n);
  }
}

// W[k2][k1] = c_k2 c_k1 / mu(k2, k1) with mu the eigenvalue of the periodic
// 5-point Laplacian on the 2n2 x 2n1 torus, 0 for the constant mode, and
// c_k = 1 at k = 0 and k = n, 2 otherwise (the cosine sum folds the torus
// frequencies k and 2n - k together).
__global__ void k_weight_table(double* w, int n2, int n1, double h) {
  const int k2 = blockIdx.y;
  const double s2 = sinpi(static_cast<double>(k2) / (2.0 * n2));
  const double c2 = (k2 == 0 || k2 == n2) ? 1.0 : 2.0;
  for (int k1 = blockIdx.x * blockDim.x + threadIdx.x; k1 <= n1; k1 += gridDim.x * blockDim.x) {
    const double s1 = sinpi(static_cast<double>(k1) / (2.0 * n1));
    const double c1 = (k1 == 0 || k1 == n1) ? 1.0 : 2.0;
    const double lam = 4.0 * (s2 * s2 + s1 * s1) / (h * h);
    w[static_cast<long long>(k2) * (n1 + 1) + k1] = (k2 == 0 && k1 == 0) ? 0.0 : -c2 * c1 / lam;
  }
}

// out[i][j] = scale * sum_k A(i, k) B(k, j), A(i, k) = a[i * ai + k * ak],
// B(k, j) = b[k * ldb + j]; 64 x 64 output tiles, 256 threads, 4 x 4 each.
__global__ __launch_bounds__(256) void k_dgemm(const double* __restrict__ a, long long ai,
                                               long long ak, const double* __restrict__ b,
                                               long long ldb, double* __restrict__ out,
                                               long long ldo, int M, int N, int K, double scale) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int kk = e / 64, ii = e % 64;
      const int gi = i0 + ii, gk = k0 + kk;
      As[kk][ii] = (gi < M && gk < K) ? a[gi * ai + gk * ak] : 0.0;
      const int gj = j0 + ii;
      Bs[kk][ii] = (gk < K && gj < N) ? b[gk * ldb + gj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = As[kk][ty + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = Bs[kk][tx + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fma(av[r], bv[c], acc[r][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gi = i0 + ty + 16 * r, gj = j0 + tx + 16 * c;
      if (gi < M && gj < N) out[gi * ldo + gj] = scale * acc[r][c];
    }
}

GreenTable::GreenTable(int n2_, int n1_, double h_, hipStream_t s) : n2(n2_), n1(n1_), h(h_) {
  const long long a2 = n2 + 1, a1 = n1 + 1;
  DevBuf c1(sizeof(double) * a1 * a1), c2(sizeof(double) * a2 * a2);
  DevBuf w(sizeof(double) * a2 * a1), t(sizeof(double) * a2 * a1);
  g.alloc(sizeof(double) * a2 * a1);
  hipLaunchKernelGGL(k_cos_table, dim3((a1 + 255) / 256, a1), dim3(256), 0, s, c1.as<double>(), n1);
  TVS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_cos_table, dim3((a2 + 255) / 256, a2), dim3(256), 0, s, c2.as<double>(), n2);
  TVS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_weight_table, dim3((a1 + 255) / 256, a2), dim3(256), 0, s, w.as<double>(),
                     n2, n1, h);
  TVS_LAUNCH_CHECK();
  // T[k2][v] = sum_k1 W[k2][k1] C1[k1][v]
  hipLaunchKernelGGL(k_dgemm, dim3((a1 + 63) / 64, (a2 + 63) / 64), dim3(256), 0, s,
                     w.as<double>(), a1, 1LL, c1.as<double>(), a1, t.as<double>(), a1,
                     int(a2), int(a1), int(a1), 1.0);
  TVS_LAUNCH_CHECK();
  // G[u][v] = sum_k2 C2[k2][u] T[k2][v] / (2 n2 * 2 n1)
  hipLaunchKernelGGL(k_dgemm, dim3((a1 + 63) / 64, (a2 + 63) / 64), dim3(256), 0, s,
                     c2.as<double>(), 1LL, a2, t.as<double>(), a1, g.as<double>(), a1, int(a2),
                     int(a1), int(a2), 1.0 / (4.0 * double(n2) * double(n1)));
  TVS_LAUNCH_CHECK();
  TVS_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Window spectra (float64 build)
// ---------------------------------------------------------------------------
struct SlotKey {
  int bi, bj, pi, pj;  // window base offsets; flip phase lengths (-1: none)
  bool operator<(const SlotKey& o) const {
    return std::tie(bi, bj, pi, pj) < std::tie(o.bi, o.bj, o.pi, o.pj);
  }
};

__device__ __forceinline__ double g_lookup(const double* __restrict__ g, int n2, int n1, long long u,
                                           long long v) {
  const long long p2 = 2LL * n2, p1 = 2LL * n1;
  u %= p2; if (u < 0) u += p2; if (u > n2) u = p2 - u;
  v %= p1; if (v < 0) v += p1; if (v > n1) v = p1 - v;
  return g[u * (n1 + 1) + v];
}

// Forward FFT along x of the real windows K(m_i, m_j) = G(bi + d(m_i),
// bj + d(m_j)), d(m) = m below ceil(L/2) and m - L above (the offsets a
// linear convolution of a box with itself needs).  Output row-major
// [slot][m_i][k_j].
template <int NT, bool OB>
__global__ __launch_bounds__(NT) void k_spec_rows(const double* __restrict__ g, int n2, int n1,
                                                  const int4* __restrict__ keys, int Li, int Lj,
                                                  FftDesc fj, const cplx<double>* __restrict__ twj,
                                                  cplx<double>* __restrict__ out, int ppw) {
  extern __shared__ unsigned char smem_raw[];
  cplx<double>* buf = reinterpret_cast<cplx<double>*>(smem_raw);
  const int slot = blockIdx.y;
  const int4 key = keys[slot];
  const int Lh = Lj / 2 + 1;
  const int hi_i = (Li + 1) / 2, hi_j = (Lj + 1) / 2;
  const int q0 = blockIdx.x * ppw;
  for (int e = threadIdx.x; e < ppw * Lj; e += NT) {
    const int qq = e / Lj, c = e - qq * Lj;
    const int ra = 2 * (q0 + qq), rb = ra + 1;
    const long long dj = c < hi_j ? c : c - Lj;
    double va = 0.0, vb = 0.0;
    if (ra < Li) va = g_lookup(g, n2, n1, key.x + (ra < hi_i ? ra : ra - Li), key.y + dj);
    if (rb < Li) vb = g_lookup(g, n2, n1, key.x + (rb < hi_i ? rb : rb - Li), key.y + dj);
    buf[lds_swz(qq * Lj + c)] = cplx<double>{va, vb};
  }
  __syncthreads();
  const cplx<double>* res = OB ? fft_lds_1b<double, NT>(buf, fj, Lj, ppw, twj, false)
                               : fft_lds<double, NT>(buf, buf + lds_round(ppw * Lj), fj, Lj, ppw, twj, false);
  for (int e = threadIdx.x; e < ppw * Lh; e += NT) {
    const int qq = e / Lh, k = e - qq * Lh;
    const int ra = 2 * (q0 + qq), rb = ra + 1;
    const cplx<double> z = res[lds_swz(qq * Lj + k)];
    const cplx<double> zn = res[lds_swz(qq * Lj + (k == 0 ? 0 : Lj - k))];
    const size_t base = static_cast<size_t>(slot) * Li * Lh;
    if (ra < Li) out[base + static_cast<size_t>(ra) * Lh + k] = cplx<double>{0.5 * (z.x + zn.x), 0.5 * (z.y - zn.y)};
    if (rb < Li) out[base + static_cast<size_t>(rb) * Lh + k] = cplx<double>{0.5 * (z.y + zn.y), 0.5 * (zn.x - z.x)};
  }
}

// Forward FFT along y, then the flip phases and the 1/(Li Lj) normalisation
// of the inverse transforms are folded in; output in T, column-major
// [slot][k_j][k_i].
template <typename T, int NT, bool OB>
__global__ __launch_bounds__(NT) void k_spec_cols(const cplx<double>* __restrict__ in,
                                                  const int4* __restrict__ keys, int Li, int Lj,
                                                  FftDesc fi, const cplx<double>* __restrict__ twi,
                                                  const cplx<double>* __restrict__ twj,
                                                  cplx<T>* __restrict__ out, int cpw) {
  extern __shared__ unsigned char smem_raw[];
  cplx<double>* buf = reinterpret_cast<cplx<double>*>(smem_raw);
  const int slot = blockIdx.y;
  const int4 key = keys[slot];
  const int Lh = Lj / 2 + 1;
  const int k0 = blockIdx.x * cpw;
  const size_t base = static_cast<size_t>(slot) * Li * Lh;
  for (int e = threadIdx.x; e < cpw * Li; e += NT) {
    const int r = e / cpw, c = e - r * cpw;
    const int k = k0 + c;
    buf[lds_swz(c * Li + r)] = (k < Lh) ? in[base + static_cast<size_t>(r) * Lh + k] : cplx<double>{0.0, 0.0};
  }
  __syncthreads();
  const cplx<double>* res = OB ? fft_lds_1b<double, NT>(buf, fi, Li, cpw, twi, false)
                               : fft_lds<double, NT>(buf, buf + lds_round(cpw * Li), fi, Li, cpw, twi, false);
  const double scale = 1.0 / (double(Li) * double(Lj));
  for (int e = threadIdx.x; e < cpw * Li; e += NT) {
    const int c = e / Li, r = e - c * Li;
    const int k = k0 + c;
    if (k >= Lh) continue;
    cplx<double> v = res[lds_swz(c * Li + r)];
    v.x *= scale;
    v.y *= scale;
    if (key.z >= 0) v = cmul(v, twi[(static_cast<long long>(r) * key.z) % Li]);
    if (key.w >= 0) v = cmul(v, twj[(static_cast<long long>(k) * key.w) % Lj]);
    out[base + static_cast<size_t>(k) * Li + r] = cplx<T>{T(v.x), T(v.y)};
  }
}

// ---------------------------------------------------------------------------
// Apply kernels.  The half spectra are kept column-major per box,
// S[b][k_j][row], so that the column transforms read contiguous data.
// ---------------------------------------------------------------------------

// LDS of an apply kernel: two transform buffers of batch * n elements, then
// (TWL) the twiddle table of the transform length, which the passes gather
// from at scattered offsets; from LDS those gathers do not queue behind the
// vector L1.
template <typename T, int NT, bool TWL>
__device__ __forceinline__ const cplx<T>* stage_twiddles(cplx<T>* lds, const cplx<T>* __restrict__ tw,
                                                         int n) {
  if constexpr (TWL) {
    for (int i = threadIdx.x; i < n; i += NT) lds[i] = tw[i];
    return lds;
  } else {
    return tw;
  }
}

// Row-pass workgroup -> (row group, box).  With xcd_rows the grid is one-
// dimensional and each XCD (workgroup w runs on XCD w mod 8) takes a
// contiguous range of the units, row group fastest: the few row pairs that
// share a 128-byte chunk of a half-spectrum column then meet in one XCD's L2
// instead of being fetched (and written) once per XCD.  False when idle.
template <typename T>
__device__ __forceinline__ bool row_unit(const GreenDev<T>& d, int& qg, int& b) {
  if (d.xcd_rows) {
    const int units = d.row_groups * d.nbox, per = (units + 7) / 8;
    const int u = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (u >= units) return false;
    qg = u % d.row_groups;
    b = u / d.row_groups;
  } else {
    qg = blockIdx.x;
    b = blockIdx.y;
  }
  return true;
}

// Row transforms of the source: rows 2m and 2m+1 of div u (zero outside the
// box) form the real and imaginary parts of one complex sequence; the half
// spectra of the two rows are separated from the packed result and stored
// column-major.
// Column stride of the half spectra for the compile-time lengths: the box
// rows a length of this size serves (251-256, 271-288, 321-324: the next
// smaller smooth lengths are 500, 540 and 640), rounded up to 32 and padded
// by 16, as the plan computes it; the plan checks it before choosing them.
constexpr int scol_of(int sl) { return sl == 512 ? 272 : sl == 576 ? 304 : 368; }

// SL = 512, 576 or 648: the transform length is fixed at compile time
// (FftOf<SL>), else 0.  OB: one LDS buffer (long transforms, 1024 threads,
// global twiddles).
template <typename T, int NT, bool TWL, int SL, bool OB, bool JB>
__global__ __launch_bounds__(NT) void k_green_rows_fwd(GreenDev<T> d, const T* __restrict__ u,
                                                       Frame uf) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  int qg, b;
  if (!row_unit(d, qg, b)) return;  // whole workgroup idle
  C* Sj = d.S;
  if constexpr (JB) {
    const int j = b / d.nbox_job;
    const JobBufs<T>& jb = d.jobs[j];
    u = jb.z[jb.par ^ d.jflip];
    Sj = jb.S;
    b -= j * d.nbox_job;
  }
  const GreenBox bx = d.boxes[b];
  const int Lj = SL ? SL : d.Lj, Lh = SL ? SL / 2 + 1 : d.Lh, ppw = d.ppw;
  const int q0 = qg * ppw;
  if (2 * q0 >= bx.ni) return;  // whole workgroup idle for this box
  const C* tw = stage_twiddles<T, NT, TWL>(buf + 2 * lds_round(ppw * Lj), d.tw_j, Lj);
  // all NT threads stage the packed rows (the first pass has fewer butterflies
  // than threads, and these loads are the latency-bound part).  With a
  // compile-time length only the first half of each row is staged: a box
  // row has at most L/2 points (L >= 2 nj - 1 and even), and the half-input
  // first pass reads no more.
  constexpr int kHalf = SL ? SL / 2 : 1;
  const int Lst = SL ? kHalf : Lj;
  for (int e = threadIdx.x; e < ppw * Lst; e += NT) {
    const int qq = SL ? e / kHalf : d.fd_Lj.div(e), c = e - qq * Lst;
    const int ra = 2 * (q0 + qq), rb = ra + 1;
    T va = T(0), vb = T(0);
    if (c < bx.nj) {
      if (ra < bx.ni) va = div_at(u, uf, b, bx.i0 + ra, bx.j0 + c, ra, c, d.n2, d.n1, d.inv_h);
      if (rb < bx.ni) vb = div_at(u, uf, b, bx.i0 + rb, bx.j0 + c, rb, c, d.n2, d.n1, d.inv_h);
    }
    buf[lds_swz(qq * Lj + c)] = C{va, vb};
  }
  __syncthreads();
  const C* res;
  if constexpr (SL != 0)
    res = fft_lds_s<T, NT, FftOf<SL>, true>(buf, buf + lds_round(ppw * Lj), ppw, tw, false);
  else if constexpr (OB)
    res = fft_lds_1b<T, NT>(buf, d.fj, Lj, ppw, tw, false);
  else
    res = fft_lds<T, NT>(buf, buf + lds_round(ppw * Lj), d.fj, Lj, ppw, tw, false);
  const int scol = SL ? scol_of(SL) : d.scol;
  C* S = Sj + static_cast<size_t>(b) * scol * Lh;
  for (int e = threadIdx.x; e < ppw * Lh; e += NT) {
    const int k = d.fd_ppw.div(e), qq = e - k * ppw;
    const int ra = 2 * (q0 + qq), rb = ra + 1;
    const C z = res[lds_swz(qq * Lj + k)];
    const C zn = res[lds_swz(qq * Lj + (k == 0 ? 0 : Lj - k))];
    C* col = S + static_cast<size_t>(k) * scol;
    const C va = C{T(0.5) * (z.x + zn.x), T(0.5) * (z.y - zn.y)};
    const C vb = C{T(0.5) * (z.y + zn.y), T(0.5) * (zn.x - z.x)};
    if constexpr (sizeof(T) == 4) {
      // both rows of the pair with one 16-byte store (adjacent in the
      // column; 16-byte aligned: scol and ra even)
      if (rb < bx.ni)
        *reinterpret_cast<float4*>(col + ra) = make_float4(va.x, va.y, vb.x, vb.y);
      else if (ra < bx.ni)
        col[ra] = va;
    } else {
      if (ra < bx.ni) col[ra] = va;
      if (rb < bx.ni) col[rb] = vb;
    }
  }
}

// Phi(ki) from X(ki) = a + i b, X(-ki) = c + i d and the four window spectra:
//   X K00 + conj(X(-ki)) K01 + X(-ki) K10 + conj(X) K11
//     = a P + b Q + c R + d S,
//   P = K00 + K11, Q = i (K00 - K11), R = K01 + K10, S = i (K10 - K01),
// i.e. eight real multiply-adds once P, Q, R, S are formed.
template <typename T>
struct PhiCoef {
  cplx<T> p, q, r, s;
};
template <typename T>
__device__ __forceinline__ PhiCoef<T> phi_coef(cplx<T> k00, cplx<T> k01, cplx<T> k10, cplx<T> k11) {
  return PhiCoef<T>{cplx<T>{k00.x + k11.x, k00.y + k11.y}, cplx<T>{k11.y - k00.y, k00.x - k11.x},
                    cplx<T>{k01.x + k10.x, k01.y + k10.y}, cplx<T>{k01.y - k10.y, k10.x - k01.x}};
}
template <typename T>
__device__ __forceinline__ cplx<T> combine_phi(cplx<T> x, cplx<T> xn, const PhiCoef<T>& k) {
  return cplx<T>{x.x * k.p.x + x.y * k.q.x + xn.x * k.r.x + xn.y * k.s.x,
                 x.x * k.p.y + x.y * k.q.y + xn.x * k.r.y + xn.y * k.s.y};
}

// Column pass with the window spectra of the first inverse pass (radix R,
// one butterfly per thread: column c, index j) loaded up front.
template <typename T, int NT, int R, int SL, typename LD, typename ST>
__device__ __forceinline__ void cols_prefetched(const GreenDev<T>& d, LD& ld_s, ST& st_s,
                                                cplx<T>* bufa, cplx<T>* bufb,
                                                const cplx<T>* const (&sp)[4], int c, int j,
                                                bool act, const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  const int Li = SL ? SL : d.Li, cpw = d.cpw, nbf = SL ? SL / R : d.fi.nbf[0].d;
  // raw values only: combining them here would wait for the loads
  C k[4][R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int o = c * Li + j + t * nbf;
#pragma unroll
    for (int m = 0; m < 4; ++m) k[m][t] = act ? sp[m][o] : C{T(0), T(0)};
  }
  const C* X;
  if constexpr (SL != 0)
    X = fft_run_to_lds_s<T, NT, FftOf<SL>, true>(ld_s, bufa, bufb, cpw, tw, false);  // box rows <= Li / 2
  else
    X = fft_run_to_lds<T, NT>(d.fi, ld_s, bufa, bufb, Li, cpw, tw, false);
  C* Y = (X == bufa) ? bufb : bufa;
  if (act) {
    C v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int ki = j + t * nbf;
      v[t] = combine_phi(X[lds_swz(c * Li + ki)], X[lds_swz(c * Li + (ki == 0 ? 0 : Li - ki))],
                         phi_coef(k[0][t], k[1][t], k[2][t], k[3][t]));
    }
    butterfly<R, T>(v, true);
#pragma unroll
    for (int t = 0; t < R; ++t) Y[lds_swz(c * Li + j * R + t)] = v[t];  // Ls = 1: output j R + t
  }
  __syncthreads();
  if constexpr (SL != 0)
    fft_run_tail_s<T, NT, FftOf<SL>>(st_s, Y, const_cast<C*>(X), cpw, tw, true);
  else
    fft_run_tail<T, NT>(d.fi, st_s, Y, const_cast<C*>(X), Li, cpw, tw, true);
}

// Column transforms, spectral combination and inverse column transforms for
// `cpw` columns of one box.  The forward transform loads the box's ni rows
// of each column (zero beyond), the first inverse pass forms
//   Phi = X K00 + conj(X(-ki)) K01 + X(-ki) K10 + conj(X) K11
// as it loads, and the last inverse pass stores the box's ni rows back.
// Launch order: the box index is the fastest grid dimension, so consecutive
// workgroups (dealt round-robin to the eight XCDs) work on the same column
// tile of neighbouring boxes; boxes of one subdomain column then share an
// XCD and its L2 for the window spectra they have in common.
// (at most 128 VGPRs, so that four 256-thread workgroups fit on a CU)
template <typename T, int NT, bool TWL, int SL, bool OB, bool JB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_green_cols(GreenDev<T> d) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* bufa = reinterpret_cast<C*>(smem_raw);
  int b = blockIdx.x;
  C* Sj = d.S;
  const cplx<T>* specj = d.spec;
  if constexpr (JB) {
    const int j = b / d.nbox_job;
    Sj = d.jobs[j].S;
    specj = d.jobs[j].spec;
    b -= j * d.nbox_job;
  }
  const GreenBox bx = d.boxes[b];
  const int Li = SL ? SL : d.Li, Lh = SL ? SL / 2 + 1 : d.Lh, cpw = d.cpw, scol = SL ? scol_of(SL) : d.scol;
  C* bufb = bufa + lds_round(cpw * Li);
  const int k0 = blockIdx.y * cpw;
  const int ncol = min(cpw, Lh - k0);
  const C* tw = stage_twiddles<T, NT, TWL>(bufa + 2 * lds_round(cpw * Li), d.tw_i, Li);
  C* S = Sj + static_cast<size_t>(b) * scol * Lh + static_cast<size_t>(k0) * scol;
  const size_t slot_sz = static_cast<size_t>(Li) * Lh, col0 = static_cast<size_t>(k0) * Li;
  const C* s00 = specj + static_cast<size_t>(bx.k00) * slot_sz + col0;
  const C* s01 = specj + static_cast<size_t>(bx.k01) * slot_sz + col0;
  const C* s10 = specj + static_cast<size_t>(bx.k10) * slot_sz + col0;
  const C* s11 = specj + static_cast<size_t>(bx.k11) * slot_sz + col0;
  auto ld_s = [&](int c, int r, int) -> C {
    return (c < ncol && r < bx.ni) ? S[c * scol + r] : C{T(0), T(0)};
  };
  auto st_s = [&](int c, int r, C v) {
    if (c < ncol && r < bx.ni) S[c * scol + r] = v;
  };
  if constexpr (OB) {
    // one LDS buffer: forward transform in place; Phi in place, one thread
    // per frequency pair (k, -k), which read each other's X; then the
    // inverse transform in place
    C* X = fft_run_to_lds_1b<T, NT>(d.fi, ld_s, bufa, Li, cpw, tw, false);
    const int half = Li / 2 + 1;
    for (int e = threadIdx.x; e < cpw * half; e += NT) {
      const int c = e / half, k = e - c * half, kn = k == 0 ? 0 : Li - k;
      const int o = c * Li + k, on = c * Li + kn;
      C pk{T(0), T(0)}, pn{T(0), T(0)};
      if (c < ncol) {
        const C x = X[lds_swz(o)], xn = X[lds_swz(on)];
        pk = combine_phi(x, xn, phi_coef(s00[o], s01[o], s10[o], s11[o]));
        pn = combine_phi(xn, x, phi_coef(s00[on], s01[on], s10[on], s11[on]));
      }
      X[lds_swz(o)] = pk;
      if (kn != k) X[lds_swz(on)] = pn;
    }
    __syncthreads();
    LdsSeq<T> io{X, Li};
    fft_run_1b<T, NT>(d.fi, io, st_s, X, Li, cpw, tw, true);
    return;
  } else if constexpr (sizeof(T) == 4 && SL != 0) {
    // One butterfly per thread in the first inverse pass (the plan selects
    // this variant only when cpw * 72 <= NT): its window-spectrum values are
    // loaded before the forward transform, so that their latency overlaps it.
    const cplx<T>* sp[4] = {s00, s01, s10, s11};
    constexpr int nb = FftOf<SL>::template nbf<0>();
    const int c = threadIdx.x / nb, j = threadIdx.x - c * nb;
    const bool act = threadIdx.x < nb * cpw && c < ncol;
    cols_prefetched<T, NT, FftOf<SL>::template radix<0>(), SL>(d, ld_s, st_s, bufa, bufb, sp, c, j, act, tw);
    return;
  } else {
    if constexpr (sizeof(T) == 4) {
      const int r0 = d.fi.radix[0], nbf0 = d.fi.nbf[0].d;
      if (d.fi.npass >= 2 && nbf0 * cpw <= NT) {
        // as above, with the runtime descriptor
        const cplx<T>* sp[4] = {s00, s01, s10, s11};
        const int c = d.fi.nbf[0].div(threadIdx.x), j = threadIdx.x - c * nbf0;
        const bool act = threadIdx.x < nbf0 * cpw && c < ncol;
        switch (r0) {
          case 8: cols_prefetched<T, NT, 8, 0>(d, ld_s, st_s, bufa, bufb, sp, c, j, act, tw); break;
          case 9: cols_prefetched<T, NT, 9, 0>(d, ld_s, st_s, bufa, bufb, sp, c, j, act, tw); break;
          case 4: cols_prefetched<T, NT, 4, 0>(d, ld_s, st_s, bufa, bufb, sp, c, j, act, tw); break;
          case 2: cols_prefetched<T, NT, 2, 0>(d, ld_s, st_s, bufa, bufb, sp, c, j, act, tw); break;
          case 3: cols_prefetched<T, NT, 3, 0>(d, ld_s, st_s, bufa, bufb, sp, c, j, act, tw); break;
          default: cols_prefetched<T, NT, 5, 0>(d, ld_s, st_s, bufa, bufb, sp, c, j, act, tw); break;
        }
        return;
      }
    }
    const C* X = fft_run_to_lds<T, NT>(d.fi, ld_s, bufa, bufb, Li, cpw, tw, false);
    C* Y = (X == bufa) ? bufb : bufa;
    auto ld_phi = [&](int c, int ki, int) -> C {
      if (c >= ncol) return C{T(0), T(0)};
      const int o = c * Li + ki;
      return combine_phi(X[lds_swz(o)], X[lds_swz(c * Li + (ki == 0 ? 0 : Li - ki))],
                         phi_coef(s00[o], s01[o], s10[o], s11[o]));
    };
    fft_run<T, NT>(d.fi, ld_phi, st_s, Y, const_cast<C*>(X), Li, cpw, tw, true);
  }
}

template <typename T, int NT, bool TWL, int SL, bool OB, bool JB>
__global__ __launch_bounds__(NT) void k_green_rows_inv(GreenDev<T> d, T* __restrict__ phi, Frame pf) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  int qg, b;
  if (!row_unit(d, qg, b)) return;  // whole workgroup idle
  const C* Sj = d.S;
  if constexpr (JB) {
    const int j = b / d.nbox_job;
    phi = d.jobs[j].phi;
    Sj = d.jobs[j].S;
    b -= j * d.nbox_job;
  }
  const GreenBox bx = d.boxes[b];
  const int Lj = SL ? SL : d.Lj, Lh = SL ? SL / 2 + 1 : d.Lh, ppw = d.ppw;
  const int q0 = qg * ppw;
  if (2 * q0 >= bx.ni) return;
  const C* tw = stage_twiddles<T, NT, TWL>(buf + 2 * lds_round(ppw * Lj), d.tw_j, Lj);
  const int scol = SL ? scol_of(SL) : d.scol;
  const C* S = Sj + static_cast<size_t>(b) * scol * Lh;
  const int half = Lj / 2;
  auto ld = [&](int qq, int k, int) -> C {
    const int ra = 2 * (q0 + qq), rb = ra + 1;
    const int kk = k <= half ? k : Lj - k;
    const C* col = S + static_cast<size_t>(kk) * scol;
    const C a = ra < bx.ni ? col[ra] : C{T(0), T(0)};
    const C c = rb < bx.ni ? col[rb] : C{T(0), T(0)};
    return k <= half ? C{a.x - c.y, a.y + c.x} : C{a.x + c.y, c.x - a.y};
  };
  T* out = phi + b * pf.box_stride;
  auto st = [&](int qq, int c, C z) {
    const int ra = 2 * (q0 + qq), rb = ra + 1;
    if (ra < bx.ni && c < bx.nj) {
      out[static_cast<long long>(ra) * pf.pitch + c] = z.x;
      if (rb < bx.ni) out[static_cast<long long>(rb) * pf.pitch + c] = z.y;
    }
  };
  if constexpr (!OB) {
    // Stage the packed inputs of the ppw row pairs in the second LDS buffer
    // before the first pass (which then reads LDS): the two rows of a pair
    // are adjacent in a half-spectrum column, so one 16-byte load gives both
    // at frequency kk (and, mirrored, at Lj - kk), and consecutive lanes read
    // consecutive pairs, 128 contiguous bytes per column for 8 pairs, where
    // the first pass would read one element per lane, a column apart.  (The
    // second buffer is first written by the second pass, after a barrier.)
    C* stg = buf + lds_round(ppw * Lj);
    for (int e = threadIdx.x; e < (half + 1) * ppw; e += NT) {
      const int kk = d.fd_ppw.div(e), qq = e - kk * ppw;
      const int ra = 2 * (q0 + qq);
      C a{T(0), T(0)}, c{T(0), T(0)};
      if (ra < bx.ni) {
        // rows ra and ra + 1 (the column holds scol > ni rows, so the second
        // is inside it; past the box it holds no data and is replaced by zero)
        const C* col = S + static_cast<size_t>(kk) * scol + ra;
        if constexpr (sizeof(T) == 4) {
          const float4 v = *reinterpret_cast<const float4*>(col);  // 16-byte aligned: scol and ra even
          a = C{T(v.x), T(v.y)};
          c = C{T(v.z), T(v.w)};
        } else {
          a = col[0];
          c = col[1];
        }
        if (ra + 1 >= bx.ni) c = C{T(0), T(0)};
      }
      stg[lds_swz(qq * Lj + kk)] = C{a.x - c.y, a.y + c.x};
      if (kk != 0 && kk != half) stg[lds_swz(qq * Lj + Lj - kk)] = C{a.x + c.y, c.x - a.y};
    }
    __syncthreads();
    if constexpr (SL != 0) {
      LdsSeqS<T, SL> first{stg};
      fft_run_s<T, NT, FftOf<SL>>(first, st, buf, stg, ppw, tw, true);
    } else {
      LdsSeq<T> first{stg, Lj};
      fft_run<T, NT>(d.fj, first, st, buf, stg, Lj, ppw, tw, true);
    }
  } else {
    fft_run_1b<T, NT>(d.fj, ld, st, buf, Lj, ppw, tw, true);
  }
}

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
template <typename F>
static void allow_lds(F* f, size_t bytes) {
  if (bytes > 65536) TVS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(f),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 static_cast<int>(bytes)));
}

// Workgroup size and batch for transforms of length n: the batch (rows or
// columns per workgroup) sets the granularity of the row/column transpose
// through HBM, so aim for `want` sequences per workgroup (128-byte chunks),
// using 1024 threads when 256 cannot stage them, within `max_lds` bytes.
struct Batch {
  int nt, batch;
  bool ob;  // one LDS buffer (fft_run_1b): 1024 threads, global twiddles
};
// the one-buffer engine: as many sequences as the LDS holds, up to `want`
template <typename T>
static Batch pick_batch_1b(int n, int want) {
  if (lds_round(n) > kLdsElems<T>)
    throw Error(-1, "FFT length " + std::to_string(n) + " exceeds the LDS capacity (" +
                        std::to_string(kLdsElems<T>) + " elements)");
  return Batch{kFftThreadsLong, std::max(1, std::min(want, kLdsElems<T> / lds_round(n))), true};
}
template <typename T>
static Batch pick_batch(int n, int want, size_t max_lds) {
  const size_t elem_bytes = sizeof(cplx<T>);
  constexpr int cs = FftCap<T, kFftThreads>::elems, cl = FftCap<T, kFftThreadsLong>::elems;
  // two buffers of one sequence do not fit, or the thread count cannot cover
  // the passes: the one-buffer engine
  if (n > kFftThreadsLong * cl || 2 * size_t(lds_round(n)) * elem_bytes > size_t(kLdsBytes))
    return pick_batch_1b<T>(n, want);
  const int by_lds = std::max<int>(1, int(max_lds / (2 * size_t(lds_round(n)) * elem_bytes)));
  const int target = std::max(1, std::min(want, by_lds));
  Batch b{};
  b.ob = false;
  if (size_t(target) * n <= size_t(kFftThreads) * cs) {
    b.nt = kFftThreads;
    b.batch = target;
  } else {
    b.nt = kFftThreadsLong;
    b.batch = std::max(1, std::min(target, (kFftThreadsLong * cl) / n));
  }
  if (2 * size_t(lds_round(b.batch * n)) * elem_bytes > 160 * 1024)
    throw Error(-1, "FFT length " + std::to_string(n) + " does not fit in LDS");
  return b;
}

template <typename T>
GreenPlan<T>::GreenPlan(const GreenTable& table, const std::vector<std::array<int, 4>>& boxes,
                        hipStream_t s)
    : n2(table.n2), n1(table.n1), nbox(int(boxes.size())) {
  rows_max = cols_max = 0;
  for (auto& bx : boxes) {
    rows_max = std::max(rows_max, bx[2]);
    cols_max = std::max(cols_max, bx[3]);
  }
  Li = smooth_even_at_least(2 * rows_max - 1);
  Lj = smooth_even_at_least(2 * cols_max - 1);
  const int Lh = Lj / 2 + 1;
  const FftDesc fi = make_fft_desc(Li), fj = make_fft_desc(Lj);

  // slots, deduplicated by window base and flip phase
  std::map<SlotKey, int> slots;
  std::vector<int4> keys;
  auto slot_of = [&](SlotKey k) {
    auto it = slots.find(k);
    if (it != slots.end()) return it->second;
    const int id = int(keys.size());
    slots[k] = id;
    keys.push_back(make_int4(k.bi, k.bj, k.pi, k.pj));
    return id;
  };
  std::vector<GreenBox> hb(nbox);
  for (int b = 0; b < nbox; ++b) {
    const int i0 = boxes[b][0], j0 = boxes[b][1], ni = boxes[b][2], nj = boxes[b][3];
    if (i0 < 0 || j0 < 0 || ni < 1 || nj < 1 || i0 + ni > n2 || j0 + nj > n1)
      throw Error(-1, "Green box outside the grid");
    GreenBox g{i0, j0, ni, nj, 0, 0, 0, 0};
    sum_ni_lh_ += double(ni) * (Lj / 2 + 1);
    sum_box_px_ += double(ni) * nj;
    g.k00 = slot_of({0, 0, -1, -1});
    g.k01 = slot_of({0, 2 * j0 + nj, -1, nj - 1});
    g.k10 = slot_of({2 * i0 + ni, 0, ni - 1, -1});
    g.k11 = slot_of({2 * i0 + ni, 2 * j0 + nj, ni - 1, nj - 1});
    hb[b] = g;
  }
  nslot = keys.size();

  boxes_d_.alloc(sizeof(GreenBox) * nbox);
  TVS_HIP(hipMemcpyAsync(boxes_d_.p, hb.data(), sizeof(GreenBox) * nbox, hipMemcpyHostToDevice, s));
  tw_i_ = make_twiddles<T>(Li, s);
  tw_j_ = make_twiddles<T>(Lj, s);
  spec_.alloc(sizeof(cplx<T>) * nslot * size_t(Li) * Lh);
  // column stride of the half spectra: a multiple of 16 elements (128-byte
  // chunks for float32) that is an odd multiple, so that the columns of a
  // box do not all start on the same memory channel
  const int scol = (rows_max + 31) / 32 * 32 + 16;
  S_.alloc(sizeof(cplx<T>) * size_t(nbox) * scol * Lh);

  // build the window spectra in float64, a chunk of slots at a time
  {
    DevBuf tw_i64 = make_twiddles<double>(Li, s), tw_j64 = make_twiddles<double>(Lj, s);
    DevBuf keys_d(sizeof(int4) * nslot);
    TVS_HIP(hipMemcpyAsync(keys_d.p, keys.data(), sizeof(int4) * nslot, hipMemcpyHostToDevice, s));
    const size_t per_slot = size_t(Li) * Lh;
    const size_t chunk = std::max<size_t>(1, (size_t(512) << 20) / (per_slot * sizeof(cplx<double>)));
    DevBuf tmp(sizeof(cplx<double>) * std::min(chunk, nslot) * per_slot);
    const Batch br = pick_batch<double>(Lj, 8, 80 * 1024);
    const Batch bc = pick_batch<double>(Li, 8, 80 * 1024);
    const size_t lds_r = (br.ob ? 1 : 2) * size_t(lds_round(br.batch * Lj)) * sizeof(cplx<double>);
    const size_t lds_c = (bc.ob ? 1 : 2) * size_t(lds_round(bc.batch * Li)) * sizeof(cplx<double>);
    // the one-buffer engine holds all butterflies of a pass in registers:
    // radices of at most 4 keep that within the register budget for float64
    const FftDesc sfi = bc.ob ? make_fft_desc(Li, kLongRadix<double>) : fi;
    const FftDesc sfj = br.ob ? make_fft_desc(Lj, kLongRadix<double>) : fj;
    auto kr = br.ob ? k_spec_rows<kFftThreadsLong, true>
                    : br.nt == kFftThreads ? k_spec_rows<kFftThreads, false> : k_spec_rows<kFftThreadsLong, false>;
    auto kc = bc.ob ? k_spec_cols<T, kFftThreadsLong, true>
                    : bc.nt == kFftThreads ? k_spec_cols<T, kFftThreads, false> : k_spec_cols<T, kFftThreadsLong, false>;
    allow_lds(kr, lds_r);
    allow_lds(kc, lds_c);
    for (size_t s0 = 0; s0 < nslot; s0 += chunk) {
      const int ns = int(std::min(chunk, nslot - s0));
      hipLaunchKernelGGL(kr, dim3((Li / 2 + br.batch - 1) / br.batch, ns), dim3(br.nt), lds_r, s,
                         table.g.as<double>(), n2, n1, keys_d.as<int4>() + s0, Li, Lj, sfj,
                         tw_j64.as<cplx<double>>(), tmp.as<cplx<double>>(), br.batch);
      TVS_LAUNCH_CHECK();
      hipLaunchKernelGGL(kc, dim3((Lh + bc.batch - 1) / bc.batch, ns), dim3(bc.nt), lds_c, s,
                         tmp.as<cplx<double>>(), keys_d.as<int4>() + s0, Li, Lj, sfi,
                         tw_i64.as<cplx<double>>(), tw_j64.as<cplx<double>>(),
                         spec_.as<cplx<T>>() + s0 * per_slot, bc.batch);
      TVS_LAUNCH_CHECK();
    }
    TVS_HIP(hipStreamSynchronize(s));
  }

  fi_ = fi;
  fj_ = fj;
  dev_.n2 = n2;
  dev_.n1 = n1;
  dev_.Li = Li;
  dev_.Lj = Lj;
  dev_.Lh = Lh;
  dev_.scol = scol;
  dev_.nbox = nbox;
  dev_.nbox_job = nbox;
  dev_.jobs = nullptr;
  dev_.jflip = 0;
  dev_.fd_Li = make_fastdiv(Li);
  dev_.fd_Lj = make_fastdiv(Lj);
  dev_.inv_h = T(1) / T(table.h);
  dev_.boxes = boxes_d_.as<GreenBox>();
  dev_.tw_i = tw_i_.as<cplx<T>>();
  dev_.tw_j = tw_j_.as<cplx<T>>();
  dev_.S = S_.as<cplx<T>>();
  dev_.spec = spec_.as<cplx<T>>();
  // 8 row pairs (16 rows) per workgroup give 128-byte chunks of float32 half
  // spectra in the transposed layout; the column pass, which is bound by
  // its barriers rather than by HBM, keeps 256-thread workgroups
  set_tiles(kDefaultTileRows, (kFftThreads * FftCap<T, kFftThreads>::elems) / Li);
}

// The kernel code path a plan's launches take: the one-buffer engine, the
// workgroup sizes, the twiddle placement, compile-time or runtime transform
// lengths, and (float) whether the column pass loads its window spectra
// ahead.  Workgroup shapes that keep it compute the same values bit for bit;
// another path may round differently (the compiler contracts differently).
template <typename T>
std::array<int, 7> GreenPlan<T>::variant() const {
  int sl = 0;
  for_each_variant([&](auto, auto cf, auto) {
    sl = (reinterpret_cast<const void*>(cf) == reinterpret_cast<const void*>(
                                                   k_green_cols<T, kFftThreads, true, 512, false, false>) ||
          reinterpret_cast<const void*>(cf) == reinterpret_cast<const void*>(
                                                   k_green_cols<T, kFftThreads, true, 576, false, false>) ||
          reinterpret_cast<const void*>(cf) == reinterpret_cast<const void*>(
                                                   k_green_cols<T, kFftThreads, true, 648, false, false>))
             ? 1
             : 0;
  });
  const int pre = sizeof(T) == 4 && !ob_ && dev_.fi.npass >= 2 && dev_.fi.nbf[0].d * dev_.cpw <= nt_cols_;
  return {ob_ ? 1 : 0, nt_rows_, nt_cols_, twl_rows_ ? 1 : 0, twl_cols_ ? 1 : 0, sl, sl ? 1 : pre};
}

template <typename T>
bool GreenPlan<T>::try_tiles(int rows, int cols) {
  const int r0 = tile_rows_, c0 = tile_cols_;
  const std::array<int, 7> v0 = variant();
  set_tiles(rows, cols);
  if (variant() == v0) return true;
  set_tiles(r0, c0);
  return false;
}

template <typename T>
void GreenPlan<T>::set_tiles(int rows, int cols) {
  rows = std::max(1, rows);
  cols = std::max(1, cols);
  Batch br = pick_batch<T>(Lj, rows, 80 * 1024);
  Batch bc = pick_batch<T>(Li, cols, 80 * 1024);
  // a transform too long for two LDS buffers puts all three passes on the
  // one-buffer engine (one kernel variant for long plans)
  ob_ = br.ob || bc.ob;
  if (ob_) {
    br = pick_batch_1b<T>(Lj, br.ob ? br.batch : rows);
    bc = pick_batch_1b<T>(Li, 1);
  }
  tile_rows_ = rows;
  tile_cols_ = cols;
  nt_rows_ = br.nt;
  nt_cols_ = bc.nt;
  dev_.ppw = br.batch;
  dev_.row_groups = ((rows_max + 1) / 2 + br.batch - 1) / br.batch;
  // a workgroup writes (and reads back) 2 ppw rows of every half-spectrum
  // column: below a 128-byte chunk, neighbouring row groups share chunks
  dev_.xcd_rows = 2 * br.batch * int(sizeof(cplx<T>)) < 128 ? 1 : 0;
  dev_.cpw = bc.batch;
  dev_.fd_ppw = make_fastdiv(br.batch);
  dev_.fi = ob_ ? make_fft_desc(Li, kLongRadix<T>) : fi_;
  dev_.fj = ob_ ? make_fft_desc(Lj, kLongRadix<T>) : fj_;
  twl_rows_ = !ob_ && Lj * sizeof(cplx<T>) <= 16 * 1024;
  twl_cols_ = !ob_ && Li * sizeof(cplx<T>) <= 16 * 1024;
  for (bool jobs : {false, true})
    for_each_variant(
        [&](auto rf, auto cf, auto ri) {
          allow_lds(rf, lds_rows());
          allow_lds(ri, lds_rows());
          allow_lds(cf, lds_cols());
        },
        jobs);
}

template <typename T>
size_t GreenPlan<T>::lds_rows() const {
  return ((ob_ ? 1 : 2) * size_t(lds_round(dev_.ppw * Lj)) + (twl_rows_ ? size_t(Lj) : 0)) * sizeof(cplx<T>);
}
template <typename T>
size_t GreenPlan<T>::lds_cols() const {
  return ((ob_ ? 1 : 2) * size_t(lds_round(dev_.cpw * Li)) + (twl_cols_ ? size_t(Li) : 0)) * sizeof(cplx<T>);
}

// Calls f(rows_fwd, cols, rows_inv) with the kernel instantiations this plan
// launches (workgroup size and twiddle placement of each pass).
template <typename T>
template <typename F>
void GreenPlan<T>::for_each_variant(F&& f, bool jobs) const {
  auto pick = [&](auto nt_r, auto nt_c, auto twr, auto twc, auto sl) {
    constexpr int R = decltype(nt_r)::value, Cn = decltype(nt_c)::value, SL = decltype(sl)::value;
    constexpr bool TR = decltype(twr)::value, TC = decltype(twc)::value;
    if (jobs)
      f(k_green_rows_fwd<T, R, TR, SL, false, true>, k_green_cols<T, Cn, TC, SL, false, true>,
        k_green_rows_inv<T, R, TR, SL, false, true>);
    else
      f(k_green_rows_fwd<T, R, TR, SL, false, false>, k_green_cols<T, Cn, TC, SL, false, false>,
        k_green_rows_inv<T, R, TR, SL, false, false>);
  };
  if (ob_) {
    if (jobs)
      f(k_green_rows_fwd<T, kFftThreadsLong, false, 0, true, true>, k_green_cols<T, kFftThreadsLong, false, 0, true, true>,
        k_green_rows_inv<T, kFftThreadsLong, false, 0, true, true>);
    else
      f(k_green_rows_fwd<T, kFftThreadsLong, false, 0, true, false>,
        k_green_cols<T, kFftThreadsLong, false, 0, true, false>,
        k_green_rows_inv<T, kFftThreadsLong, false, 0, true, false>);
    return;
  }
  using S = std::integral_constant<int, kFftThreads>;
  using L = std::integral_constant<int, kFftThreadsLong>;
  using Y = std::true_type;
  using N = std::false_type;
  using G = std::integral_constant<int, 0>;
  const bool rs = nt_rows_ == kFftThreads, cs = nt_cols_ == kFftThreads;
  // square 512-, 576- or 648-point boxes (the 576-point ones come from
  // 256-point subdomain cores) with 1024-thread row and 256-thread column
  // workgroups, twiddles in LDS: the compile-time passes
  if (!rs && cs && twl_rows_ && twl_cols_ && Li == Lj) {
    auto fits = [&](auto desc) {
      using D = decltype(desc);
      return D::matches(dev_.fi) && D::matches(dev_.fj) && dev_.scol == scol_of(D::n) &&
             dev_.cpw * D::template nbf<0>() <= kFftThreads;
    };
    if (Li == 512 && fits(Fft512{})) return pick(L{}, S{}, Y{}, Y{}, std::integral_constant<int, 512>{});
    if (Li == 576 && fits(Fft576{})) return pick(L{}, S{}, Y{}, Y{}, std::integral_constant<int, 576>{});
    if (Li == 648 && fits(Fft648{})) return pick(L{}, S{}, Y{}, Y{}, std::integral_constant<int, 648>{});
  }
  if (rs && cs) {
    if (twl_rows_ && twl_cols_) pick(S{}, S{}, Y{}, Y{}, G{});
    else if (twl_rows_) pick(S{}, S{}, Y{}, N{}, G{});
    else if (twl_cols_) pick(S{}, S{}, N{}, Y{}, G{});
    else pick(S{}, S{}, N{}, N{}, G{});
  } else if (rs) {
    if (twl_rows_ && twl_cols_) pick(S{}, L{}, Y{}, Y{}, G{});
    else if (twl_rows_) pick(S{}, L{}, Y{}, N{}, G{});
    else if (twl_cols_) pick(S{}, L{}, N{}, Y{}, G{});
    else pick(S{}, L{}, N{}, N{}, G{});
  } else if (cs) {
    if (twl_rows_ && twl_cols_) pick(L{}, S{}, Y{}, Y{}, G{});
    else if (twl_rows_) pick(L{}, S{}, Y{}, N{}, G{});
    else if (twl_cols_) pick(L{}, S{}, N{}, Y{}, G{});
    else pick(L{}, S{}, N{}, N{}, G{});
  } else {
    if (twl_rows_ && twl_cols_) pick(L{}, L{}, Y{}, Y{}, G{});
    else if (twl_rows_) pick(L{}, L{}, Y{}, N{}, G{});
    else if (twl_cols_) pick(L{}, L{}, N{}, Y{}, G{});
    else pick(L{}, L{}, N{}, N{}, G{});
  }
}

template <typename T>
size_t GreenPlan<T>::bytes() const {
  return spec_.bytes + S_.bytes + boxes_d_.bytes + tw_i_.bytes + tw_j_.bytes;
}
template <typename T>
size_t GreenPlan<T>::footprint(const std::vector<std::array<int, 4>>& boxes) {
  int rmax = 0, cmax = 0;
  std::set<SlotKey> keys;
  for (auto& bx : boxes) {
    rmax = std::max(rmax, bx[2]);
    cmax = std::max(cmax, bx[3]);
    const int i0 = bx[0], j0 = bx[1], ni = bx[2], nj = bx[3];
    keys.insert({0, 0, -1, -1});
    keys.insert({0, 2 * j0 + nj, -1, nj - 1});
    keys.insert({2 * i0 + ni, 0, ni - 1, -1});
    keys.insert({2 * i0 + ni, 2 * j0 + nj, ni - 1, nj - 1});
  }
  const size_t li = size_t(smooth_even_at_least(2 * rmax - 1));
  const size_t lj = size_t(smooth_even_at_least(2 * cmax - 1)), lh = lj / 2 + 1;
  const size_t scol = size_t((rmax + 31) / 32 * 32 + 16);
  return sizeof(cplx<T>) * (keys.size() * li * lh + boxes.size() * scol * lh + li + lj) +
         sizeof(GreenBox) * boxes.size();
}

// Algorithmic bytes: the row passes read the source field (2 planes) of
// every box and write its half spectrum (rows x (Lj/2+1) complex), or the
// reverse with one output plane; the column pass reads and writes the half
// spectra and reads every distinct window spectrum once.
template <typename T>
double GreenPlan<T>::bytes_rows_fwd() const {
  return sum_box_px_ * 2 * sizeof(T) + sum_ni_lh_ * sizeof(cplx<T>);
}
template <typename T>
double GreenPlan<T>::bytes_cols() const {
  return 2 * sum_ni_lh_ * sizeof(cplx<T>) + double(nslot) * Li * dev_.Lh * sizeof(cplx<T>);
}
template <typename T>
double GreenPlan<T>::bytes_rows_inv() const {
  return sum_ni_lh_ * sizeof(cplx<T>) + sum_box_px_ * sizeof(T);
}

template <typename T>
void GreenPlan<T>::apply_div(const T* u, const Frame& uf, T* phi, const Frame& pf, hipStream_t s,
                             KernelTimer* timer, const char* tag) {
  const int row_groups = dev_.row_groups;
  const dim3 gr = dev_.xcd_rows ? dim3(8 * ((row_groups * nbox + 7) / 8)) : dim3(row_groups, nbox);
  const dim3 gc(nbox, (dev_.Lh + dev_.cpw - 1) / dev_.cpw);
  const size_t lr = lds_rows(), lc = lds_cols();
  const std::string t(tag);
  for_each_variant([&](auto rf, auto cf, auto ri) {
    KernelTimer::time(timer, (t + "_rows_fwd").c_str(), bytes_rows_fwd(), s, [&] {
      hipLaunchKernelGGL(rf, gr, dim3(nt_rows_), lr, s, dev_, u, uf);
      TVS_LAUNCH_CHECK();
    });
    KernelTimer::time(timer, (t + "_cols").c_str(), bytes_cols(), s, [&] {
      hipLaunchKernelGGL(cf, gc, dim3(nt_cols_), lc, s, dev_);
      TVS_LAUNCH_CHECK();
    });
    KernelTimer::time(timer, (t + "_rows_inv").c_str(), bytes_rows_inv(), s, [&] {
      hipLaunchKernelGGL(ri, gr, dim3(nt_rows_), lr, s, dev_, phi, pf);
      TVS_LAUNCH_CHECK();
    });
  });
}

template <typename T>
void GreenPlan<T>::apply_div_jobs(const JobBufs<T>* jobs, int njobs, int flip, const Frame& uf, const Frame& pf,
                                  hipStream_t s, KernelTimer* timer, const char* tag) {
  GreenDev<T> d = dev_;
  d.jobs = jobs;
  d.jflip = flip;
  d.nbox = nbox * njobs;
  const int row_groups = d.row_groups, nb = d.nbox;
  const dim3 gr = d.xcd_rows ? dim3(8 * ((row_groups * nb + 7) / 8)) : dim3(row_groups, nb);
  const dim3 gc(nb, (d.Lh + d.cpw - 1) / d.cpw);
  const size_t lr = lds_rows(), lc = lds_cols();
  const std::string t(tag);
  for_each_variant([&](auto rf, auto cf, auto ri) {
    KernelTimer::time(timer, (t + "_rows_fwd").c_str(), njobs * bytes_rows_fwd(), s, [&] {
      hipLaunchKernelGGL(rf, gr, dim3(nt_rows_), lr, s, d, static_cast<const T*>(nullptr), uf);
      TVS_LAUNCH_CHECK();
    });
    KernelTimer::time(timer, (t + "_cols").c_str(), njobs * bytes_cols(), s, [&] {
      hipLaunchKernelGGL(cf, gc, dim3(nt_cols_), lc, s, d);
      TVS_LAUNCH_CHECK();
    });
    KernelTimer::time(timer, (t + "_rows_inv").c_str(), njobs * bytes_rows_inv(), s, [&] {
      hipLaunchKernelGGL(ri, gr, dim3(nt_rows_), lr, s, d, static_cast<T*>(nullptr), pf);
      TVS_LAUNCH_CHECK();
    });
  }, true);
}

template class GreenPlan<float>;
template class GreenPlan<double>;

}  // namespace tvs
