// LP_m by the paper's block-DCT formula (eq. invLaplLowCapLong of Section
// 6.2.2): the inverse Laplacian of the whole grid applied to data supported
// on a box A and restricted to a box B, evaluated with the columns of the DCT
// matrices that belong to A and B only,
//   R_B (Delta)^dagger E_A d = C2[:,B]^T (Lambda^dagger o (C2[:,A] d C1[:,A]^T)) C1[:,B],
// where C2 = C_{n2}, C1 = C_{n1} (eq. form:DCTmat) and Lambda^dagger is the
// diagonal of eq. form:DiscInvLaplTild.  The formula's sum over the frequency
// blocks lambda is taken in one piece: every frequency is visited once, which
// is what the sum over a disjoint decomposition of the frequency grid adds up
// to.  The four products per box are dense contractions and run as batched
// GEMMs (rocBLAS) over all boxes at once; this realisation is an alternative
// to the image method of GreenPlan and is selected per context.
#pragma once
#include <array>
#include <vector>

#include <rocblas/rocblas.h>

#include "green.hpp"
#include "tvs_internal.hpp"

namespace tvs {

template <typename T>
class BlockDctPlan {
 public:
  // Boxes are (i0, j0, ni, nj) on the n2 x n1 grid; A = B = the box.
  BlockDctPlan(int n2, int n1, double h, const std::vector<std::array<int, 4>>& boxes, hipStream_t s);
  ~BlockDctPlan();
  BlockDctPlan(const BlockDctPlan&) = delete;
  BlockDctPlan& operator=(const BlockDctPlan&) = delete;
  // phi = R_B (Delta)^dagger E_A div(u) on every box, with the same frames
  // and boundary rules as GreenPlan::apply_div
  void apply_div(const T* u, const Frame& uf, T* phi, const Frame& pf, hipStream_t s,
                 KernelTimer* timer = nullptr, const char* tag = "bdct");
  size_t bytes() const;
  // multiply-adds of one apply (all boxes), for the FLOP roofline
  double macs() const;

  int n2, n1, nbox, amax, bmax;

 private:
  double h_;
  rocblas_handle handle_ = nullptr;
  DevBuf boxes_d_, c2s_, c1s_, lam_, d_, u_, x_, v_, p_;
};

}  // namespace tvs
