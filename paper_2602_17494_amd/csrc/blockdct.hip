// LP_m through the block-DCT formula (eq. invLaplLowCapLong): see blockdct.hpp.
#include <algorithm>
#include <cmath>
#include <string>

#include "blockdct.hpp"

namespace tvs {
namespace {

// Orthonormal DCT-II matrix entry C_N[k][n] (eq. form:DCTmat) in float64,
// with the angle k (2n + 1) pi / (2N) reduced exactly modulo 2 pi first.
double dct_entry(int N, int k, int n) {
  const long long num = (static_cast<long long>(k) * (2LL * n + 1)) % (4LL * N);
  const double c = std::cos(M_PI * static_cast<double>(num) / (2.0 * N));
  return (k == 0 ? std::sqrt(1.0 / N) : std::sqrt(2.0 / N)) * (k == 0 ? 1.0 : c);
}

// D[b] = div u on box b (frame data, grid boundary rules) in the box's
// aligned frame: element (r + i0 % 4, q + j0 % 4) holds local (r, q), every
// other element of the ap x bp frame is zero
template <typename T>
__global__ void k_bd_pack(const std::array<int, 4>* __restrict__ boxes, const T* __restrict__ u, Frame uf,
                          int n2, int n1, T inv_h, int ap, int bp, T* __restrict__ D) {
  const int c = blockIdx.x * 64 + threadIdx.x, r = blockIdx.y * 4 + threadIdx.y, b = blockIdx.z;
  if (r >= ap || c >= bp) return;
  const std::array<int, 4> bx = boxes[b];
  const int lr = r - (bx[0] & 3), lq = c - (bx[1] & 3);
  T v = T(0);
  if (lr >= 0 && lq >= 0 && lr < bx[2] && lq < bx[3])
    v = div_at(u, uf, b, bx[0] + lr, bx[1] + lq, lr, lq, n2, n1, inv_h);
  D[(static_cast<size_t>(b) * ap + r) * bp + c] = v;
}

// phi frame of box b = O[b] on the box (read from the aligned frame)
template <typename T>
__global__ void k_bd_unpack(const std::array<int, 4>* __restrict__ boxes, const T* __restrict__ O, int ap, int bp,
                            T* __restrict__ phi, Frame pf) {
  const int c = blockIdx.x * 64 + threadIdx.x, r = blockIdx.y * 4 + threadIdx.y, b = blockIdx.z;
  const std::array<int, 4> bx = boxes[b];
  if (r >= bx[2] || c >= bx[3]) return;
  phi[b * pf.box_stride + static_cast<long long>(r) * pf.pitch + c] =
      O[(static_cast<size_t>(b) * ap + r + (bx[0] & 3)) * bp + c + (bx[1] & 3)];
}

// ---------------------------------------------------------------------------
// The matrix-core step: D = A B + C for a 16 x 16 x 4 block.  Operands: lane
// l holds A[l % 16][l / 16] and B[l / 16][l % 16]; result register r of lane
// l is D[row(l, r)][l % 16].
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  using V = f32x4;
  static __device__ __forceinline__ V step(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <>
struct Mfma<double> {
  using V = f64x4;
  static __device__ __forceinline__ V step(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * r + (l >> 4); }
};

template <typename T>
struct Vec16;  // 16 bytes of T
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

__device__ __forceinline__ int bd_lim(const std::array<int, 4>& bx, int kind, int v) {
  return kind == 1 ? bx[2] : kind == 2 ? bx[3] : v;
}

// four consecutive elements of an LDS row (16-byte aligned)
__device__ __forceinline__ void lds4(const float* p, float (&o)[4]) {
  const auto v = *reinterpret_cast<const Vec16<float>::type*>(p);
  o[0] = v[0];
  o[1] = v[1];
  o[2] = v[2];
  o[3] = v[3];
}
__device__ __forceinline__ void lds4(const double* p, double (&o)[4]) {
  const auto v = reinterpret_cast<const Vec16<double>::type*>(p);
  const auto x = v[0], y = v[1];
  o[0] = x[0];
  o[1] = x[1];
  o[2] = y[0];
  o[3] = y[1];
}

// Z[b] (M x N) = A[b] (M x K) B[b] (K x N) for box b = blockIdx.z, one
// (32 TB) x (32 TB) output tile per workgroup of four waves, each wave
// owning TB x TB blocks of 16 x 16 (the plan launches TB = 2).  K advances in stages of 128 bytes per
// row (32 floats or 16 doubles) through two LDS buffers: the next stage is
// read from global memory (16-byte loads) into registers while the current
// one feeds the matrix cores.  Both tiles are kept with k contiguous (A as
// [m][k], B transposed to [n][k]), and within each 16-wide slice of k the
// lane group g = lane / 16 takes k = 4 g + s in step s, so one 16-byte LDS
// read (two for doubles) gives a lane its operands for four steps; this
// only reorders the terms of the sum over k.  M, N, K and the column
// limits of the operands are multiples of 4, their rows and the allocation
// slack make every 16-byte load lie in the buffer.  mode 0 stores, 1 adds
// to Z, 2 stores lam o (A B).
template <typename T, int TB>
__global__ __launch_bounds__(256) void k_bd_gemm(const std::array<int, 4>* __restrict__ boxes, BdOperand<T> A,
                                                 BdOperand<T> B, T* __restrict__ Z, long long ldz, long long zbs,
                                                 int M, int N, int K, int mode, const T* __restrict__ lam,
                                                 long long ldl) {
  using V = typename Mfma<T>::V;
  using L = typename Vec16<T>::type;
  constexpr int VW = 16 / static_cast<int>(sizeof(T));
  constexpr int TM = 32 * TB;
  constexpr int BK = 128 / static_cast<int>(sizeof(T));
  constexpr int LDK = BK + 4;
  constexpr int KV = BK / VW, NV = TM / VW;
  constexpr int AV = TM * KV / 256, BV = BK * NV / 256;
  static_assert(AV * 256 == TM * KV && BV * 256 == BK * NV, "tile loads must split evenly over 256 threads");
  __shared__ __attribute__((aligned(16))) T sa[2][TM][LDK];
  __shared__ __attribute__((aligned(16))) T sb[2][TM][LDK];
  const int b = blockIdx.z;
  const std::array<int, 4> bx = boxes[b];
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TM;
  const T* pa = A.p + A.off + b * A.bs + bx[0] * A.ro + bx[1] * A.co;
  const T* pb = B.p + B.off + b * B.bs + bx[0] * B.ro + bx[1] * B.co;
  const int ar = min(M, bd_lim(bx, A.rk, A.rv)), ac = min(K, bd_lim(bx, A.ck, A.cv));
  const int br = min(K, bd_lim(bx, B.rk, B.rv)), bc = min(N, bd_lim(bx, B.ck, B.cv));
  const int t = threadIdx.x;
  L ra[AV], rb[BV];
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < AV; ++p) {
      const int e = t + 256 * p;
      const int gm = m0 + e / KV, gk = k0 + (e % KV) * VW;
      ra[p] = (gm < ar && gk < ac) ? *reinterpret_cast<const L*>(pa + static_cast<long long>(gm) * A.ld + gk) : L{};
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int e = t + 256 * p;
      const int gk = k0 + e / NV, gn = n0 + (e % NV) * VW;
      rb[p] = (gk < br && gn < bc) ? *reinterpret_cast<const L*>(pb + static_cast<long long>(gk) * B.ld + gn) : L{};
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int p = 0; p < AV; ++p) {
      const int e = t + 256 * p;
      *reinterpret_cast<L*>(&sa[buf][e / KV][(e % KV) * VW]) = ra[p];
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int e = t + 256 * p;
      const int k = e / NV, n = (e % NV) * VW;
#pragma unroll
      for (int j = 0; j < VW; ++j) sb[buf][n + j][k] = rb[p][j];
    }
  };
  const int lane = t & 63, w = t >> 6, wm = (w >> 1) * 16 * TB, wn = (w & 1) * 16 * TB;
  const int lr = lane & 15, lk = lane >> 4;
  V acc[TB][TB];
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int j = 0; j < TB; ++j) acc[i][j] = V{};
  const int nk = (K + BK - 1) / BK;
  load(0);
  stage(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
    for (int c = 0; c < BK / 16; ++c) {
      T fa[TB][4], fb[TB][4];
#pragma unroll
      for (int i = 0; i < TB; ++i) lds4(&sa[cur][wm + 16 * i + lr][16 * c + 4 * lk], fa[i]);
#pragma unroll
      for (int j = 0; j < TB; ++j) lds4(&sb[cur][wn + 16 * j + lr][16 * c + 4 * lk], fb[j]);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < TB; ++i)
#pragma unroll
          for (int j = 0; j < TB; ++j) acc[i][j] = Mfma<T>::step(fa[i][s], fb[j][s], acc[i][j]);
    }
    if (kt + 1 < nk) stage(cur ^ 1);
    __syncthreads();
  }
  T* z = Z + b * zbs;
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int j = 0; j < TB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + 16 * i + Mfma<T>::row(lane, r), col = n0 + wn + 16 * j + lr;
        if (row >= M || col >= N) continue;
        T v = acc[i][j][r];
        const long long o = static_cast<long long>(row) * ldz + col;
        if (mode == 2) v *= lam[static_cast<long long>(row) * ldl + col];
        if (mode == 1) v += z[o];
        z[o] = v;
      }
}

// Edges of nb near-equal blocks of [0, n), n a multiple of 4, on multiples
// of 4
std::vector<int> block_edges(int n, int nb) {
  std::vector<int> e(nb + 1);
  for (int i = 0; i <= nb; ++i) e[i] = 4 * static_cast<int>(static_cast<long long>(i) * (n / 4) / nb);
  return e;
}

int tiles_of(int x, int tm) { return (x + tm - 1) / tm; }
int round4(int x) { return (x + 3) & ~3; }

}  // namespace

template <typename T>
BlockDctPlan<T>::BlockDctPlan(int n2_, int n1_, double h, const std::vector<std::array<int, 4>>& boxes,
                              hipStream_t s, int force_g2, int force_g1)
    : n2(n2_), n1(n1_), nbox(static_cast<int>(boxes.size())), amax(0), bmax(0), h_(h) {
  if (nbox == 0) throw Error(-1, "internal: block-DCT plan without boxes");
  std::vector<std::array<int, 4>> aligned;
  ap = bp = 0;
  for (const auto& b : boxes) {
    if (b[0] < 0 || b[1] < 0 || b[2] < 1 || b[3] < 1 || b[0] + b[2] > n2 || b[1] + b[3] > n1)
      throw Error(-1, "internal: block-DCT box outside the grid");
    amax = std::max(amax, b[2]);
    bmax = std::max(bmax, b[3]);
    aligned.push_back({b[0] & ~3, b[1] & ~3, b[2] + (b[0] & 3), b[3] + (b[1] & 3)});
    ap = std::max(ap, aligned.back()[2]);
    bp = std::max(bp, aligned.back()[3]);
  }
  ap = round4(ap);
  bp = round4(bp);
  r2 = round4(n2);
  r1 = round4(n1);
  // frequency blocks no larger than the largest box, grouped so that the
  // Y product of one group has about 16384 workgroups of 64 x 64 (whole
  // frequency rows first: the W product's inner dimension is the group's
  // width), with at most 16 blocks per group
  nb2 = (r2 + amax - 1) / amax;
  nb1 = (r1 + bmax - 1) / bmax;
  e2_ = block_edges(r2, nb2);
  e1_ = block_edges(r1, nb1);
  const int fa = (r2 + nb2 - 1) / nb2, fb = (r1 + nb1 - 1) / nb1;
  auto y_wgs = [&](int a, int c) { return static_cast<long long>(nbox) * tiles_of(a * fa, 64) * tiles_of(c * fb, 64); };
  g1 = 1;
  g2 = 1;
  while (g1 < nb1 && (g1 + 1) * g2 <= 16 && y_wgs(g2, g1) < 16384) ++g1;
  if (g1 == nb1)
    while (g2 < nb2 && g1 * (g2 + 1) <= 16 && y_wgs(g2, g1) < 16384) ++g2;
  if (force_g2 > 0 || force_g1 > 0) {
    g2 = force_g2 > 0 ? std::min(force_g2, nb2) : g2;
    g1 = force_g1 > 0 ? std::min(force_g1, nb1) : g1;
  }
  rows_g_ = cols_g_ = 0;
  for (int r = 0; r < nb2; r += g2) rows_g_ = std::max(rows_g_, e2_[std::min(r + g2, nb2)] - e2_[r]);
  for (int c = 0; c < nb1; c += g1) cols_g_ = std::max(cols_g_, e1_[std::min(c + g1, nb1)] - e1_[c]);
  // multiply-adds of the formula on each box's own extents (ni x nj), over
  // the whole frequency grid: U and O n2 ni nj each, Y and W n2 n1 nj each
  macs_ = 0;
  for (const auto& b : boxes) macs_ += 2.0 * n2 * double(b[2]) * b[3] + 2.0 * n2 * double(n1) * b[3];

  // the DCT matrices of both sides and their transposes (shared when the
  // sides agree), r x r with zeros beyond n, plus a zero tail: a 16-byte
  // load of an aligned box frame may run up to ap (bp) elements past a
  // row's data into the next row or the tail, where it meets zeros of the
  // packed input (U) or lands in frame columns that are never unpacked (W)
  auto upload = [&](DevBuf& buf, const std::vector<T>& v) {
    buf.alloc(sizeof(T) * v.size());
    TVS_HIP(hipMemcpyAsync(buf.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
    TVS_HIP(hipStreamSynchronize(s));  // the host table goes out of scope
  };
  const size_t tail = static_cast<size_t>(ap + bp + 64);
  auto dct_tables = [&](int n, int r, DevBuf& c, DevBuf& ct) {
    std::vector<T> m(static_cast<size_t>(r) * r + tail, T(0)), mt(static_cast<size_t>(r) * r + tail, T(0));
    for (int k = 0; k < n; ++k)
      for (int x = 0; x < n; ++x) {
        const T v = T(dct_entry(n, k, x));
        m[static_cast<size_t>(k) * r + x] = v;
        mt[static_cast<size_t>(x) * r + k] = v;
      }
    upload(c, m);
    upload(ct, mt);
  };
  dct_tables(n2, r2, c2_, c2t_);
  if (n1 != n2) dct_tables(n1, r1, c1_, c1t_);
  // sigma_{N,k} = (2/h) sin(k pi / (2N)); Lambda^dagger = -1 / (sigma2^2 + sigma1^2), 0 at (0, 0)
  // and beyond the grid (r2 x r1)
  std::vector<T> lam(static_cast<size_t>(r2) * r1, T(0));
  for (int i = 0; i < n2; ++i) {
    const double si = 2.0 / h * std::sin(M_PI * i / (2.0 * n2));
    for (int j = 0; j < n1; ++j) {
      const double sj = 2.0 / h * std::sin(M_PI * j / (2.0 * n1));
      const double l = si * si + sj * sj;
      lam[static_cast<size_t>(i) * r1 + j] = (i == 0 && j == 0) ? T(0) : T(-1.0 / l);
    }
  }
  upload(lam_, lam);
  boxes_d_.alloc(sizeof(std::array<int, 4>) * nbox);
  aboxes_d_.alloc(sizeof(std::array<int, 4>) * nbox);
  TVS_HIP(hipMemcpyAsync(boxes_d_.p, boxes.data(), sizeof(std::array<int, 4>) * nbox, hipMemcpyHostToDevice, s));
  TVS_HIP(hipMemcpyAsync(aboxes_d_.p, aligned.data(), sizeof(std::array<int, 4>) * nbox, hipMemcpyHostToDevice, s));
  TVS_HIP(hipStreamSynchronize(s));
  const size_t esz = sizeof(T);
  d_.alloc(esz * nbox * size_t(ap) * bp);
  o_.alloc(esz * nbox * size_t(ap) * bp);
  u_.alloc(esz * nbox * size_t(rows_g_) * bp);
  w_.alloc(esz * nbox * size_t(rows_g_) * bp);
  y_.alloc(esz * nbox * size_t(rows_g_) * cols_g_);
}

template <typename T>
size_t BlockDctPlan<T>::bytes() const {
  return boxes_d_.bytes + aboxes_d_.bytes + c2_.bytes + c2t_.bytes + c1_.bytes + c1t_.bytes + lam_.bytes +
         d_.bytes + o_.bytes + u_.bytes + w_.bytes + y_.bytes;
}

template <typename T>
void BlockDctPlan<T>::gemm(const BdOperand<T>& A, const BdOperand<T>& B, T* Z, long long ldz, long long zbs,
                           int m, int n, int k, int mode, const T* lam, long long ldl, hipStream_t s) {
  if ((m | n | k) & 3) throw Error(-1, "internal: block-DCT product extents must be multiples of 4");
  const auto* bx = aboxes_d_.as<std::array<int, 4>>();
  // 64 x 64 tiles: on these shapes (inner dimensions of a few hundred) the
  // 128 x 128 tile ran 1.3 to 1.5 times slower for every grouping tried
  hipLaunchKernelGGL((k_bd_gemm<T, 2>), dim3(tiles_of(n, 64), tiles_of(m, 64), nbox), dim3(256), 0, s, bx, A, B, Z,
                     ldz, zbs, m, n, k, mode, lam, ldl);
  TVS_LAUNCH_CHECK();
}

template <typename T>
void BlockDctPlan<T>::apply_div(const T* u, const Frame& uf, T* phi, const Frame& pf, hipStream_t s,
                                KernelTimer* timer, const char* tag) {
  const auto* bx = boxes_d_.as<std::array<int, 4>>();
  T *D = d_.as<T>(), *U = u_.as<T>(), *Y = y_.as<T>(), *W = w_.as<T>(), *O = o_.as<T>();
  const T *C2 = c2_.as<T>(), *C2T = c2t_.as<T>();
  const T *C1 = n1 == n2 ? C2 : c1_.as<T>(), *C1T = n1 == n2 ? C2T : c1t_.as<T>();
  const long long sbox = static_cast<long long>(ap) * bp, su = static_cast<long long>(rows_g_) * bp,
                  sy = static_cast<long long>(rows_g_) * cols_g_;
  // operand limit kinds: 1 = rows of the aligned box frame, 2 = its columns
  // the timer's work figure for this class is floating-point operations
  // (two per multiply-add of the products), not bytes
  KernelTimer::time(timer, tag, 2.0 * macs_, s, [&] {
    hipLaunchKernelGGL(k_bd_pack<T>, dim3((bp + 63) / 64, (ap + 3) / 4, nbox), dim3(64, 4), 0, s, bx, u, uf, n2, n1,
                       T(1.0 / h_), ap, bp, D);
    TVS_LAUNCH_CHECK();
    for (int rg = 0; rg < nb2; rg += g2) {
      const int i0 = e2_[rg], rows = e2_[std::min(rg + g2, nb2)] - i0;
      // U = [C2]_rows(A) d                  (rows x ap)(ap x bp)
      gemm({C2, static_cast<long long>(i0) * r2, 0, 1, 0, r2, 0, rows, 0, ap},
           {D, 0, sbox, 0, 0, bp, 0, ap, 0, bp}, U, bp, su, rows, bp, ap, 0, nullptr, 0, s);
      for (int cg = 0; cg < nb1; cg += g1) {
        const int j0 = e1_[cg], cols = e1_[std::min(cg + g1, nb1)] - j0;
        // Y = Lambda o (U [C1]_cols(A)^T)  (rows x bp)(bp x cols)
        gemm({U, 0, su, 0, 0, bp, 0, rows, 0, bp}, {C1T, j0, 0, 0, r1, r1, 2, 0, 0, cols}, Y, cols_g_, sy, rows,
             cols, bp, 2, lam_.as<T>() + static_cast<long long>(i0) * r1 + j0, r1, s);
        // W (+)= Y [C1]_cols(B)           (rows x cols)(cols x bp)
        gemm({Y, 0, sy, 0, 0, cols_g_, 0, rows, 0, cols}, {C1, static_cast<long long>(j0) * r1, 0, 0, 1, r1, 0, cols, 0, bp},
             W, bp, su, rows, bp, cols, cg == 0 ? 0 : 1, nullptr, 0, s);
      }
      // O (+)= [C2]_rows(B)^T W            (ap x rows)(rows x bp)
      gemm({C2T, i0, 0, r2, 0, r2, 1, 0, 0, rows}, {W, 0, su, 0, 0, bp, 0, rows, 0, bp}, O, bp, sbox, ap, bp, rows,
           rg == 0 ? 0 : 1, nullptr, 0, s);
    }
    hipLaunchKernelGGL(k_bd_unpack<T>, dim3((bmax + 63) / 64, (amax + 3) / 4, nbox), dim3(64, 4), 0, s, bx, O, ap, bp,
                       phi, pf);
    TVS_LAUNCH_CHECK();
  });
}

template class BlockDctPlan<float>;
template class BlockDctPlan<double>;

}  // namespace tvs
