// Stencil, update, combine and reduction kernels of the TV-Stokes dual
// iterations (Sections 4.2 and 6).  Launch helpers are declared here; the
// kernels live in kernels.hip.
#pragma once

#include "green.hpp"

namespace tvs {

// One subdomain as seen by the per-subdomain kernels.  Frames of all
// subdomains share one origin convention: local (r, q) is grid point
// (i0 + r, j0 + q).  s*: the subdomain itself (support of the local dual
// variable v); a*: grown by one row and column (support of z and omega, or of
// the Step-2 data b); b*: grown by two (support of the Green box, Step 1).
struct SubDesc {
  int i0, j0;
  int si, sj;
  int ai, aj;
  int bi, bj;
  int m2, m1;
};

// Grid of a step: n2 x n1 points, mesh size h.
struct Grid {
  int n2, n1;
  double h;
};

// Scalar parameters of one solve, in the compute type.
template <typename T>
struct StepScalars {
  T t;        // dual step size
  T inv_h;    // 1 / h
  T delta;    // TFS weight
  T alpha;    // IRV2 weight
  T ahat;     // Schwarz relaxation
};

// FP64 partial sums: one double per workgroup, summed in a fixed order.
struct Partials {
  double* buf;
  int cap;
};

template <typename T> void launch_fill(T* p, long long n, T v, hipStream_t s);
template <typename T> void launch_tau0(const T* d0, int N2, int N1, T inv_h, T* tau0, hipStream_t s);
template <typename T> void launch_global_vecdiv(const T* p, Grid g, T inv_h, T* z, hipStream_t s);
template <typename T>
void launch_f1(const T* tau0, const T* phi, Grid g, T inv_h, T inv_delta, T* f1, hipStream_t s);
template <typename T>
void launch_residual(const T* f1, const T* z, const T* phi, Grid g, T inv_h, T* r, Partials part,
                     double* out, hipStream_t s);
template <typename T>
void launch_scale(const T* in, long long n, T a, T* out, hipStream_t s);

// Step 1 per-subdomain kernels (4-plane v frames, 2-plane z and omega frames,
// 1-plane phi frames; frame pitch fp, frame rows fr).
// Partition-of-unity factors are tabulated per frame row and column:
// theta_m(i0 + r, j0 + q) = thy[m2 * fr + r] * thx[m1 * fp + q].
struct SubFrames {
  const SubDesc* subs;
  int nsub;
  int fr, fp;                 // frame rows and pitch
  long long plane;            // fr * fp
  AxisLayout ay, ax;          // the partition of unity
  const float* thy_f;         // theta tables in both compute types
  const float* thx_f;
  const double* thy_d;
  const double* thx_d;
  int run;                    // rows per thread of the update kernels (1, 2 or 4)
  int run_div;                // rows per thread of the Step-1 vecdiv kernel
};
template <typename T> __device__ __forceinline__ const T* theta_rows(const SubFrames& sf);
template <> __device__ __forceinline__ const float* theta_rows<float>(const SubFrames& sf) { return sf.thy_f; }
template <> __device__ __forceinline__ const double* theta_rows<double>(const SubFrames& sf) { return sf.thy_d; }
template <typename T> __device__ __forceinline__ const T* theta_cols(const SubFrames& sf);
template <> __device__ __forceinline__ const float* theta_cols<float>(const SubFrames& sf) { return sf.thx_f; }
template <> __device__ __forceinline__ const double* theta_cols<double>(const SubFrames& sf) { return sf.thx_d; }
template <typename T>
void launch_sub_theta_p(const SubFrames& sf, Grid g, const T* p, int planes, T* v, hipStream_t s);
template <typename T>
void launch_sub_vecdiv(const SubFrames& sf, Grid g, T inv_h, const T* v, T* z, hipStream_t s);
// batched over jr's jobs: z[state] = vecdiv v[state], state = par ^ flip
template <typename T>
void launch_sub_vecdiv_jobs(const SubFrames& sf, Grid g, T inv_h, JobRef<T> jr, int njobs, hipStream_t s);
template <typename T>
void launch_sub_omega(const SubFrames& sf, Grid g, T inv_h, const T* r, const T* z, const T* phi,
                      T* omega, hipStream_t s);
template <typename T>
void launch_sub_update1(const SubFrames& sf, Grid g, StepScalars<T> c, const T* v, const T* z,
                        const T* phi, const T* omega, T* v_out, hipStream_t s);
// batched: v[state ^ 1] from v[state], z[state], phi, aux (omega)
template <typename T>
void launch_sub_update1_jobs(const SubFrames& sf, Grid g, StepScalars<T> c, JobRef<T> jr, int njobs,
                             hipStream_t s);
template <typename T>
void launch_combine(const SubFrames& sf, Grid g, int planes, T ahat, const T* v, T* p, hipStream_t s);
template <typename T>
void launch_gap_tfs(const T* tau, const T* p, Grid g, T inv_h, Partials part, double* out,
                    hipStream_t s);

// Step 2
template <typename T>
void launch_bridge_irv2(const T* tau, const T* d0, int N2, int N1, T h, T alpha, T* f2,
                        hipStream_t s);
template <typename T>
void launch_sub2_prologue(const SubFrames& sf, Grid g, T inv_h, const T* p, const T* f2, T* b,
                          hipStream_t s);
template <typename T>
void launch_sub2_update(const SubFrames& sf, Grid g, StepScalars<T> c, const T* v, const T* b,
                        T* v_out, hipStream_t s);
// batched: v[state ^ 1] from v[state] and aux (b)
template <typename T>
void launch_sub2_update_jobs(const SubFrames& sf, Grid g, StepScalars<T> c, JobRef<T> jr, int njobs,
                             hipStream_t s);
template <typename T>
void launch_energy_rof(const T* p, const T* f2, Grid g, T inv_h, Partials part, double* out,
                       hipStream_t s);
template <typename T>
void launch_irv2_image(const T* d0, const T* p, Grid g, T inv_h, T inv_alpha, T* d, hipStream_t s);
template <typename T>
void launch_primal_rof(const T* p, const T* f2, Grid g, T inv_h, T inv_alpha, T* u, hipStream_t s);
template <typename T>
void launch_gap_rof(const T* u, const T* p, Grid g, T inv_h, Partials part, double* out,
                    hipStream_t s);

// IRV1 bridge: xi from tau, f = alpha d0 - div xi, and d = d0 - (div p +
// div xi)/alpha (eqs. eq:defXi2:discrete, ir1dualdis, eq:tau_hat).
template <typename T>
void launch_xi(const T* tau, int N2, int N1, T eps, T* xi, hipStream_t s);
template <typename T>
void launch_irv1_data(const T* d0, const T* xi, Grid g, T inv_h, T alpha, T* f2, hipStream_t s);
template <typename T>
void launch_irv1_image(const T* d0, const T* p, const T* xi, Grid g, T inv_h, T inv_alpha, T* d,
                       hipStream_t s);
// FP64 moments of two n-element arrays: out[0..1] = sum x, sum r; out[2..5] =
// sum (x - mx)^2, sum (r - mr)^2, sum (x - mx)(r - mr), sum (x - r)^2
template <typename T>
void launch_quality_moments(const T* x, const T* r, long long n, Partials part, double* out, hipStream_t s);

}  // namespace tvs
