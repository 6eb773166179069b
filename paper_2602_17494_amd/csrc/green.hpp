// Moore-Penrose inverse of the Neumann Laplacian of a rectangular grid,
// applied to data supported on boxes and read back on the same boxes.
//
// The paper evaluates (Delta)^dagger through the 2-D DCT (eqs.
// form:DiscInvLapl, form:DiscInvLaplTild), and for data supported on a block
// it keeps the full frequency sum in its block formula (eq.
// invLaplLowCapLong).  Here the same operator is realised exactly through
// the image identity: the 5-point Neumann Laplacian of an n2 x n1 grid is
// the periodic Laplacian of the 2n2 x 2n1 torus acting on the half-sample
// even extension, so (Delta)^dagger b at x equals
//     sum_y b(y) [G(x-y) + G(x - R_x y) + G(x - R_y y) + G(x - R_x R_y y)]
// with G the pseudo-inverse kernel of the torus and R_x, R_y the two
// reflections.  For a source box B read on the same box, each of the four
// terms is a linear convolution of the (possibly flipped) box data with a
// window of G; all four are evaluated with one forward and one inverse FFT of
// a smooth length L >= 2 |B| - 1 per axis, combining the four precomputed
// window spectra in the frequency domain.  G itself is tabulated once per
// grid in float64 by two dense contractions (a cosine sum over the torus
// spectrum).
#pragma once

#include <array>
#include <map>
#include <memory>

#include "fft_lds.hpp"

namespace tvs {

// Source = window box of the Green operator, and the four spectrum slots
// (direct, x-reflected, y-reflected, both) used by it.
struct GreenBox {
  int i0, j0, ni, nj;
  int k00, k01, k10, k11;
};

// Layout of a field stored as one frame per box (or one global frame):
// element (plane c, local row r, local column q) of box b is at
// base[b * box_stride + c * plane_stride + r * pitch + q].
struct Frame {
  long long box_stride;
  long long plane_stride;
  int pitch;
};

// div of a 2-plane frame field at local (r, q) of box b, with the boundary
// rules of D^-_x, D^-_y on the whole grid and zeros outside the frame's
// support.
template <typename T>
__device__ __forceinline__ T div_at(const T* __restrict__ u, const Frame& f, int b, int gi, int gj,
                                    int r, int q, int n2, int n1, T inv_h) {
  const T* u1 = u + b * f.box_stride;
  const T* u2 = u1 + f.plane_stride;
  const long long o = static_cast<long long>(r) * f.pitch + q;
  const T a = (gj == n1 - 1) ? T(0) : u1[o];
  const T am = (q > 0) ? u1[o - 1] : T(0);
  const T c = (gi == n2 - 1) ? T(0) : u2[o];
  const T cm = (r > 0) ? u2[o - f.pitch] : T(0);
  return ((a - am) + (c - cm)) * inv_h;
}

// Transform length of a box side (smooth, >= 2 side - 1), and whether a
// plan can hold it: the window spectra are built in float64 in one LDS
// buffer, so L <= 10240 (box sides up to 5120) for both compute types.
int green_length(int side);
bool green_side_ok(int side);
constexpr int kGreenMaxSide = 5120;

// Buffers of one job in a batched launch.  Jobs of one shape (dtype, image
// size, layout) share every geometric descriptor (subdomains, theta tables,
// Green boxes and transform lengths) and differ only in these buffers, so one
// launch covers the subdomains (or Green boxes) of all of them: frame (or
// box) z of the launch is frame z mod nsub of job z / nsub.
//   v[2]   subdomain duals, the two ping-pong states
//   z[2]   Step 1: vecdiv of v in the same two states
//   phi    Step 1: the Green boxes' Delta^dagger div z
//   aux    Step 1: omega frames; Step 2: the b frames
//   S      Step 1: the local plan's half spectra (work buffer)
//   spec   Step 1: the local plan's window spectra
//   par    the state the current sweep's inner iterations started from;
//          a launch for inner iteration nu reads state par ^ (nu & 1)
template <typename T>
struct JobBufs {
  T* v[2];
  T* z[2];
  T* phi;
  const T* aux;
  cplx<T>* S;
  const cplx<T>* spec;
  int par, pad;
};
// A launch's job table: jobs == nullptr for a launch over one problem's own
// buffers (the pointer arguments); otherwise nsub frames per job and the
// state flip of this launch.
template <typename T>
struct JobRef {
  const JobBufs<T>* jobs;
  int nsub, flip;
};

constexpr int kDefaultTileRows = 8;

// Tabulated torus kernel G(u, v), u in [0, n2], v in [0, n1], float64.
struct GreenTable {
  int n2, n1;
  double h;
  DevBuf g;  // (n2 + 1) * (n1 + 1) doubles
  GreenTable(int n2, int n1, double h, hipStream_t s);
};

template <typename T>
struct GreenDev {
  int n2, n1, nbox;  // nbox: boxes of the launch (all jobs')
  int nbox_job;      // boxes of one job's plan
  const JobBufs<T>* jobs;  // batched launch: the jobs' buffers (else nullptr)
  int jflip;         // batched launch: state flip (input frames z[par ^ jflip])
  int row_groups;  // row-pass workgroups per box (2 ppw rows each)
  int xcd_rows;    // 1: row passes use the XCD-contiguous one-dimensional order
  int Li, Lj, Lh;
  int scol;  // column stride of the half spectra S[box][k_j][row]
  int ppw, cpw;
  FastDiv fd_Li, fd_Lj, fd_ppw;
  T inv_h;
  const GreenBox* boxes;
  const cplx<T>* tw_i;
  const cplx<T>* tw_j;
  cplx<T>* S;
  const cplx<T>* spec;
  FftDesc fi, fj;
};

template <typename T>
class GreenPlan {
 public:
  // Boxes are (i0, j0, ni, nj) on the n2 x n1 grid of `table`.
  GreenPlan(const GreenTable& table, const std::vector<std::array<int, 4>>& boxes,
            hipStream_t stream);
  // phi = R_B (Delta)^dagger E_B div(u) on every box B, where u is a 2-plane
  // field (x- and y-component) stored in frame `uf` with zeros outside its
  // support, and div uses the grid's boundary rules (Section 4.1).
  void apply_div(const T* u, const Frame& uf, T* phi, const Frame& pf, hipStream_t stream,
                 KernelTimer* timer = nullptr, const char* tag = "green");
  // The same over njobs jobs of this plan's shape in one launch per pass:
  // job j's input is its z[par ^ flip] frames (layout uf), its output its
  // phi frames (layout pf), with its own half spectra S and window spectra
  // spec (identical geometry, so this plan's descriptors serve all).
  void apply_div_jobs(const JobBufs<T>* jobs, int njobs, int flip, const Frame& uf, const Frame& pf,
                      hipStream_t stream, KernelTimer* timer = nullptr, const char* tag = "green");
  cplx<T>* S_ptr() const { return dev_.S; }
  // Workgroup shape of the passes: about `rows` row pairs per row-pass
  // workgroup and `cols` columns per column-pass workgroup (targets, cut to
  // what the LDS and the thread counts allow).  Every shape computes the
  // same values; only the speed differs.
  void set_tiles(int rows, int cols);
  // set_tiles if the kernels keep their code path (so the results keep their
  // bits); otherwise the shape in force stays and the call returns false
  bool try_tiles(int rows, int cols);
  std::array<int, 7> variant() const;
  int tile_rows() const { return tile_rows_; }
  int tile_cols() const { return tile_cols_; }
  const cplx<T>* spec_ptr() const { return dev_.spec; }
  // algorithmic bytes of one launch of each pass (the minimum HBM traffic
  // it must move: its inputs read once, its outputs written once)
  double bytes_rows_fwd() const, bytes_cols() const, bytes_rows_inv() const;

  int n2, n1, nbox, Li, Lj;
  int rows_max, cols_max;
  size_t nslot = 0;
  size_t bytes() const;
  // bytes() of a plan for these boxes, computed on the host without building it
  static size_t footprint(const std::vector<std::array<int, 4>>& boxes);

 private:
  GreenDev<T> dev_{};
  int nt_rows_ = 0, nt_cols_ = 0;
  bool twl_rows_ = false, twl_cols_ = false;  // twiddle tables staged in LDS
  bool ob_ = false;  // transforms on the one-buffer LDS engine (long lengths)
  int tile_rows_ = 0, tile_cols_ = 0;  // set_tiles targets in force
  FftDesc fi_{}, fj_{};  // descriptors of the transform lengths
  size_t lds_rows() const, lds_cols() const;
  template <typename F> void for_each_variant(F&& f, bool jobs = false) const;
  double sum_ni_lh_ = 0, sum_box_px_ = 0;
  DevBuf boxes_d_, tw_i_, tw_j_, spec_, S_;
};

}  // namespace tvs
