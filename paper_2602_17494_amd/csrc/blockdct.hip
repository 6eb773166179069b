// LP_m through the block-DCT formula (eq. invLaplLowCapLong): see blockdct.hpp.
#include <cmath>
#include <string>

#include "blockdct.hpp"

namespace tvs {
namespace {

#define TVS_BLAS(expr)                                                                   \
  do {                                                                                   \
    const rocblas_status st_ = (expr);                                                   \
    if (st_ != rocblas_status_success)                                                   \
      throw Error(-3, std::string("rocBLAS: ") + rocblas_status_to_string(st_) + " in " + #expr); \
  } while (0)

// Orthonormal DCT-II matrix entry C_N[k][n] (eq. form:DCTmat) in float64,
// with the angle k (2n + 1) pi / (2N) reduced exactly modulo 2 pi first.
double dct_entry(int N, int k, int n) {
  const long long num = (static_cast<long long>(k) * (2LL * n + 1)) % (4LL * N);
  const double c = std::cos(M_PI * static_cast<double>(num) / (2.0 * N));
  return (k == 0 ? std::sqrt(1.0 / N) : std::sqrt(2.0 / N)) * (k == 0 ? 1.0 : c);
}

// D[b] = div u on box b (frame data, grid boundary rules), zero-padded to
// amax x bmax
template <typename T>
__global__ void k_bd_pack(const std::array<int, 4>* __restrict__ boxes, const T* __restrict__ u, Frame uf,
                          int n2, int n1, T inv_h, int amax, int bmax, T* __restrict__ D) {
  const int c = blockIdx.x * 64 + threadIdx.x, r = blockIdx.y * 4 + threadIdx.y, b = blockIdx.z;
  if (r >= amax || c >= bmax) return;
  const std::array<int, 4> bx = boxes[b];
  T v = T(0);
  if (r < bx[2] && c < bx[3]) v = div_at(u, uf, b, bx[0] + r, bx[1] + c, r, c, n2, n1, inv_h);
  D[(static_cast<size_t>(b) * amax + r) * bmax + c] = v;
}

// X[b] *= Lambda^dagger (elementwise over the n2 x n1 spectrum of box
// b = blockIdx.y)
template <typename T>
__global__ void k_bd_scale(T* __restrict__ X, const T* __restrict__ lam, long long plane) {
  T* x = X + blockIdx.y * plane;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < plane; i += 256LL * gridDim.x) x[i] *= lam[i];
}

// phi frame of box b = P[b] on the box
template <typename T>
__global__ void k_bd_unpack(const std::array<int, 4>* __restrict__ boxes, const T* __restrict__ P, int amax,
                            int bmax, T* __restrict__ phi, Frame pf) {
  const int c = blockIdx.x * 64 + threadIdx.x, r = blockIdx.y * 4 + threadIdx.y, b = blockIdx.z;
  const std::array<int, 4> bx = boxes[b];
  if (r >= bx[2] || c >= bx[3]) return;
  phi[b * pf.box_stride + static_cast<long long>(r) * pf.pitch + c] =
      P[(static_cast<size_t>(b) * amax + r) * bmax + c];
}

// Row-major Z (M x N) = op(A) op(B), batched with strides, through the
// column-major library call on the transposes: Z^T = op(B)^T op(A)^T.
rocblas_status gemm_rm(rocblas_handle h, bool ta, bool tb, int M, int N, int K, const float* A, int lda,
                       rocblas_stride sa, const float* B, int ldb, rocblas_stride sb, float* Z, int ldz,
                       rocblas_stride sz, int batch) {
  const float one = 1.0f, zero = 0.0f;
  return rocblas_sgemm_strided_batched(h, tb ? rocblas_operation_transpose : rocblas_operation_none,
                                       ta ? rocblas_operation_transpose : rocblas_operation_none, N, M, K, &one,
                                       B, ldb, sb, A, lda, sa, &zero, Z, ldz, sz, batch);
}
rocblas_status gemm_rm(rocblas_handle h, bool ta, bool tb, int M, int N, int K, const double* A, int lda,
                       rocblas_stride sa, const double* B, int ldb, rocblas_stride sb, double* Z, int ldz,
                       rocblas_stride sz, int batch) {
  const double one = 1.0, zero = 0.0;
  return rocblas_dgemm_strided_batched(h, tb ? rocblas_operation_transpose : rocblas_operation_none,
                                       ta ? rocblas_operation_transpose : rocblas_operation_none, N, M, K, &one,
                                       B, ldb, sb, A, lda, sa, &zero, Z, ldz, sz, batch);
}

}  // namespace

template <typename T>
BlockDctPlan<T>::BlockDctPlan(int n2_, int n1_, double h, const std::vector<std::array<int, 4>>& boxes,
                              hipStream_t s)
    : n2(n2_), n1(n1_), nbox(static_cast<int>(boxes.size())), amax(0), bmax(0), h_(h) {
  if (nbox == 0) throw Error(-1, "internal: block-DCT plan without boxes");
  for (const auto& b : boxes) {
    if (b[0] < 0 || b[1] < 0 || b[2] < 1 || b[3] < 1 || b[0] + b[2] > n2 || b[1] + b[3] > n1)
      throw Error(-1, "internal: block-DCT box outside the grid");
    amax = std::max(amax, b[2]);
    bmax = std::max(bmax, b[3]);
  }
  // C2[:, A] and C1[:, A] of every box, zero beyond the box (n2 x amax and
  // n1 x bmax, row-major), and Lambda^dagger (n2 x n1)
  std::vector<T> c2(static_cast<size_t>(nbox) * n2 * amax, T(0)), c1(static_cast<size_t>(nbox) * n1 * bmax, T(0));
  for (int b = 0; b < nbox; ++b) {
    const auto& bx = boxes[b];
    for (int k = 0; k < n2; ++k)
      for (int r = 0; r < bx[2]; ++r) c2[(static_cast<size_t>(b) * n2 + k) * amax + r] = T(dct_entry(n2, k, bx[0] + r));
    for (int k = 0; k < n1; ++k)
      for (int q = 0; q < bx[3]; ++q) c1[(static_cast<size_t>(b) * n1 + k) * bmax + q] = T(dct_entry(n1, k, bx[1] + q));
  }
  // sigma_{N,k} = (2/h) sin(k pi / (2N)); Lambda^dagger = -1 / (sigma2^2 + sigma1^2), 0 at (0, 0)
  std::vector<T> lam(static_cast<size_t>(n2) * n1);
  for (int i = 0; i < n2; ++i) {
    const double si = 2.0 / h * std::sin(M_PI * i / (2.0 * n2));
    for (int j = 0; j < n1; ++j) {
      const double sj = 2.0 / h * std::sin(M_PI * j / (2.0 * n1));
      const double l = si * si + sj * sj;
      lam[static_cast<size_t>(i) * n1 + j] = (i == 0 && j == 0) ? T(0) : T(-1.0 / l);
    }
  }
  const size_t esz = sizeof(T);
  boxes_d_.alloc(sizeof(std::array<int, 4>) * nbox);
  c2s_.alloc(esz * c2.size());
  c1s_.alloc(esz * c1.size());
  lam_.alloc(esz * lam.size());
  d_.alloc(esz * nbox * size_t(amax) * bmax);
  u_.alloc(esz * nbox * size_t(n2) * bmax);
  x_.alloc(esz * nbox * size_t(n2) * n1);
  v_.alloc(esz * nbox * size_t(amax) * n1);
  p_.alloc(esz * nbox * size_t(amax) * bmax);
  TVS_HIP(hipMemcpyAsync(boxes_d_.p, boxes.data(), sizeof(std::array<int, 4>) * nbox, hipMemcpyHostToDevice, s));
  TVS_HIP(hipMemcpyAsync(c2s_.p, c2.data(), esz * c2.size(), hipMemcpyHostToDevice, s));
  TVS_HIP(hipMemcpyAsync(c1s_.p, c1.data(), esz * c1.size(), hipMemcpyHostToDevice, s));
  TVS_HIP(hipMemcpyAsync(lam_.p, lam.data(), esz * lam.size(), hipMemcpyHostToDevice, s));
  TVS_HIP(hipStreamSynchronize(s));  // the host tables go out of scope
  TVS_BLAS(rocblas_create_handle(&handle_));
}

template <typename T>
BlockDctPlan<T>::~BlockDctPlan() {
  if (handle_) (void)rocblas_destroy_handle(handle_);
}

template <typename T>
size_t BlockDctPlan<T>::bytes() const {
  return boxes_d_.bytes + c2s_.bytes + c1s_.bytes + lam_.bytes + d_.bytes + u_.bytes + x_.bytes + v_.bytes +
         p_.bytes;
}

template <typename T>
double BlockDctPlan<T>::macs() const {
  // U = C2A D, X = U C1A^T, V = C2A^T X, P = V C1A
  return double(nbox) * (double(n2) * amax * bmax + double(n2) * bmax * n1 + double(amax) * n2 * n1 +
                         double(amax) * n1 * bmax);
}

template <typename T>
void BlockDctPlan<T>::apply_div(const T* u, const Frame& uf, T* phi, const Frame& pf, hipStream_t s,
                                KernelTimer* timer, const char* tag) {
  const auto* bx = boxes_d_.as<std::array<int, 4>>();
  const dim3 blk(64, 4), grd((bmax + 63) / 64, (amax + 3) / 4, nbox);
  T *D = d_.as<T>(), *U = u_.as<T>(), *X = x_.as<T>(), *V = v_.as<T>(), *P = p_.as<T>();
  const T *C2 = c2s_.as<T>(), *C1 = c1s_.as<T>();
  const rocblas_stride sD = rocblas_stride(amax) * bmax, sU = rocblas_stride(n2) * bmax,
                       sX = rocblas_stride(n2) * n1, sV = rocblas_stride(amax) * n1,
                       sC2 = rocblas_stride(n2) * amax, sC1 = rocblas_stride(n1) * bmax;
  // the timer's work figure for this class is floating-point operations
  // (two per multiply-add of the four products), not bytes
  KernelTimer::time(timer, tag, 2.0 * macs(), s, [&] {
    hipLaunchKernelGGL(k_bd_pack<T>, grd, blk, 0, s, bx, u, uf, n2, n1, T(1.0 / h_), amax, bmax, D);
    TVS_LAUNCH_CHECK();
    TVS_BLAS(rocblas_set_stream(handle_, s));
    // U = C2[:,A] D            (n2 x amax)(amax x bmax)
    TVS_BLAS(gemm_rm(handle_, false, false, n2, bmax, amax, C2, amax, sC2, D, bmax, sD, U, bmax, sU, nbox));
    // X = U C1[:,A]^T          (n2 x bmax)(bmax x n1)
    TVS_BLAS(gemm_rm(handle_, false, true, n2, n1, bmax, U, bmax, sU, C1, bmax, sC1, X, n1, sX, nbox));
    const long long plane = (long long)n2 * n1;
    hipLaunchKernelGGL(k_bd_scale<T>, dim3(int(std::min<long long>(1024, (plane + 255) / 256)), nbox), dim3(256), 0,
                       s, X, lam_.as<T>(), plane);
    TVS_LAUNCH_CHECK();
    // V = C2[:,B]^T X          (amax x n2)(n2 x n1)
    TVS_BLAS(gemm_rm(handle_, true, false, amax, n1, n2, C2, amax, sC2, X, n1, sX, V, n1, sV, nbox));
    // P = V C1[:,B]            (amax x n1)(n1 x bmax)
    TVS_BLAS(gemm_rm(handle_, false, false, amax, bmax, n1, V, n1, sV, C1, bmax, sC1, P, bmax, sD, nbox));
    hipLaunchKernelGGL(k_bd_unpack<T>, grd, blk, 0, s, bx, P, amax, bmax, phi, pf);
    TVS_LAUNCH_CHECK();
  });
}

template class BlockDctPlan<float>;
template class BlockDctPlan<double>;

}  // namespace tvs
