// LP_m by the paper's block-DCT formula (eq. invLaplLowCapLong of Section
// 6.2.2): the inverse Laplacian of the whole grid applied to data supported
// on a box A and restricted to a box B, evaluated with the columns of the DCT
// matrices that belong to A and B and, per term, one block of the frequency
// grid:
//   R_B (Delta)^dagger E_A d
//     = sum over lambda of  [C2]_lambda2(B)^T ( Lambda_lambda o ( [C2]_lambda2(A) d [C1]_lambda1(A)^T ) ) [C1]_lambda1(B),
// where C2 = C_{n2}, C1 = C_{n1} (eq. form:DCTmat), [C]_l(A) holds the rows of
// frequency block l and the columns of A, and Lambda_lambda is the block of
// the diagonal of eq. form:DiscInvLaplTild (Lemma lmChainOp splits the product
// over any disjoint rectangular decomposition of the frequency grid, eq.
// def:2DDs; the decomposition of the inverse Laplacian's middle factor has no
// cross terms because that factor is diagonal).  Here A = B = the box, so
// condition conditionAB holds with the box as the only block that carries
// data.
//
// The frequency rows are cut into nb2 = ceil(n2 / amax) blocks and the
// columns into nb1 = ceil(n1 / bmax) blocks of near-equal size (edges on
// multiples of 4), so no block is larger than the largest box.  The sum is
// taken in groups of g2 x g1 blocks (g2 row blocks, g1 column blocks, at
// most 16 blocks per group) so that one launch has enough workgroups to
// fill the chip; per box the workspace is the packed input and output and,
// for one group, U = [C2]_rows(A) d, Y = Lambda o (U [C1]_cols(A)^T) and
// W = sum over the group's columns of Y [C1]_cols(B): a constant times the
// largest block, never the whole frequency grid.
//
// Every product is a dense contraction and runs on the matrix cores through
// one hand-written batched kernel (MFMA 16x16x4, float32 or float64 in and
// out, LDS-staged 64 x 64 tiles, 16-byte global loads),
// launched over all boxes at once.  For those loads every table and
// workspace row is a multiple of 4 elements long and zero beyond the data,
// and each box is handled in a frame that starts at the multiple of 4 at or
// before its first row and column (the packed input carries the offset as
// leading zeros, the unpacking skips it).  The plan is an alternative to the
// image method of GreenPlan and is selected per context.
#pragma once
#include <array>
#include <vector>

#include "green.hpp"
#include "tvs_internal.hpp"

namespace tvs {

// One operand of a batched product: element (i, k) of box b is
//   p[off + b * bs + r0(b) * ro + c0(b) * co + i * ld + k],
// and reads as zero unless i < lim(rk, rv) and k < lim(ck, cv), where a
// limit kind of 0 is the fixed value, 1 the box's row count, 2 its column
// count.  Columns are read 16 bytes at a time, so off, the strides, ld and
// the column limit must be multiples of 4 (the plan uses fixed column
// limits only); a row limit may be any value.
template <typename T>
struct BdOperand {
  const T* p;
  long long off, bs, ro, co, ld;
  int rk, rv, ck, cv;
};

template <typename T>
class BlockDctPlan {
 public:
  // Boxes are (i0, j0, ni, nj) on the n2 x n1 grid; A = B = the box.
  // force_g2, force_g1 > 0 fix the blocks per group (cut to the block
  // counts); 0 chooses them from the launch size.
  BlockDctPlan(int n2, int n1, double h, const std::vector<std::array<int, 4>>& boxes, hipStream_t s,
               int force_g2 = 0, int force_g1 = 0);
  BlockDctPlan(const BlockDctPlan&) = delete;
  BlockDctPlan& operator=(const BlockDctPlan&) = delete;
  // phi = R_B (Delta)^dagger E_A div(u) on every box, with the same frames
  // and boundary rules as GreenPlan::apply_div
  void apply_div(const T* u, const Frame& uf, T* phi, const Frame& pf, hipStream_t s,
                 KernelTimer* timer = nullptr, const char* tag = "bdct");
  size_t bytes() const;
  // multiply-adds of one apply by the formula on the boxes' own extents
  // (all boxes, padding excluded), for the FLOP roofline
  double macs() const { return macs_; }

  int n2, n1, nbox, amax, bmax;
  int nb2, nb1, g2, g1;  // frequency blocks per direction, blocks per group
  int r2, r1;            // n2, n1 rounded up to multiples of 4 (table sizes)
  int ap, bp;            // rows and columns of the aligned box frames

 private:
  // Z[b] (m x n, leading dimension ldz, box stride zbs) = A[b] B[b] with
  // inner dimension k; mode 0 stores, 1 adds to Z, 2 stores lam o (A B)
  // with lam read at lam + i * ldl + j.
  void gemm(const BdOperand<T>& A, const BdOperand<T>& B, T* Z, long long ldz, long long zbs, int m, int n,
            int k, int mode, const T* lam, long long ldl, hipStream_t s);
  double h_;
  double macs_ = 0;
  std::vector<int> e2_, e1_;  // frequency block edges (nb2 + 1, nb1 + 1)
  int rows_g_ = 0, cols_g_ = 0;  // largest group extents
  // boxes as given (packing) and as aligned frames (i0 & ~3, j0 & ~3, rows
  // and columns from there to the box's end)
  DevBuf boxes_d_, aboxes_d_, c2_, c2t_, c1_, c1t_, lam_, d_, u_, y_, w_, o_;
};

}  // namespace tvs
