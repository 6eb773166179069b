// Stencil, update, combine and reduction kernels (see kernels.hpp).
//
// Difference operators follow Section 4.1 on the grid of the step:
//   D^+_x w (j) = (w(j+1) - w(j))/h, and 0 in the last column;
//   D^-_x w (j) = (w(j) - w(j-1))/h inside, w(0)/h in the first column and
//                 -w(N-2)/h in the last one (the value in the last column is
//                 ignored);
// and the same along y.  Per-subdomain data live in frames whose origin is
// the subdomain's first point; everything outside a frame's support is 0.
#include "kernels.hpp"

#include <type_traits>

namespace tvs {

constexpr int kBX = 64, kBY = 4;  // 2-D block shape (one wavefront per row)
constexpr int kRedBlocks = 1024;  // workgroups of the reduction kernels

__device__ __forceinline__ int flat_tid() { return threadIdx.x + threadIdx.y * blockDim.x; }

// Deterministic workgroup sum of a double (fixed shuffle and LDS order);
// the result is valid in thread 0.
__device__ double block_sum(double v) {
  __shared__ double sh[16];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int t = flat_tid();
  const int nw = (blockDim.x * blockDim.y + 63) / 64;
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  double tot = 0.0;
  if (t == 0)
    for (int w = 0; w < nw; ++w) tot += sh[w];
  __syncthreads();
  return tot;
}

__global__ __launch_bounds__(256) void k_final_sum(const double* __restrict__ part, int n,
                                                   double* __restrict__ out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += part[i];
  v = block_sum(v);
  if (threadIdx.x == 0) *out = v;
}

static void finish_sum(Partials part, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, s, part.buf, n, out);
  TVS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// generic
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* p, long long n, T v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
template <typename T> void launch_fill(T* p, long long n, T v, hipStream_t s) {
  if (n <= 0) return;
  if (!p) throw Error(-1, "internal: fill of an unallocated buffer");
  const int blocks = int(std::min<long long>(4096, (n + 255) / 256));
  hipLaunchKernelGGL(k_fill<T>, dim3(blocks), dim3(256), 0, s, p, n, v);
  TVS_LAUNCH_CHECK();
}

template <typename T>
__global__ void k_scale(const T* __restrict__ in, long long n, T a, T* __restrict__ out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = a * in[i];
}
template <typename T> void launch_scale(const T* in, long long n, T a, T* out, hipStream_t s) {
  const int blocks = int(std::min<long long>(4096, (n + 255) / 256));
  hipLaunchKernelGGL(k_scale<T>, dim3(blocks), dim3(256), 0, s, in, n, a, out);
  TVS_LAUNCH_CHECK();
}

static dim3 grid2d(int n2, int n1, int nz = 1) {
  return dim3((n1 + kBX - 1) / kBX, (n2 + kBY - 1) / kBY, nz);
}

// ---------------------------------------------------------------------------
// Step 1, global parts
// ---------------------------------------------------------------------------

// tau_0 = (-D^{neum-}_y d0, D^{neum-}_x d0) on the (N2+1) x (N1+1) grid
// (eq. def:backdiffNeumann and the text after eq. ir2dualdis).
template <typename T>
__global__ void k_tau0(const T* __restrict__ d0, int N2, int N1, T inv_h, T* __restrict__ tau) {
  const int j = blockIdx.x * kBX + threadIdx.x, i = blockIdx.y * kBY + threadIdx.y;
  const int n1 = N1 + 1;
  if (i > N2 || j > N1) return;
  T dx = T(0), dy = T(0);
  if (j >= 1 && j <= N1 - 1) {
    const int ii = i < N2 ? i : N2 - 1;  // the extra row mirrors the last image row
    dx = (d0[(long long)ii * N1 + j] - d0[(long long)ii * N1 + j - 1]) * inv_h;
  }
  if (i >= 1 && i <= N2 - 1) {
    const int jj = j < N1 ? j : N1 - 1;  // the extra column mirrors the last image column
    dy = (d0[(long long)i * N1 + jj] - d0[(long long)(i - 1) * N1 + jj]) * inv_h;
  }
  const long long o = (long long)i * n1 + j;
  const long long plane = (long long)(N2 + 1) * n1;
  tau[o] = -dy;
  tau[plane + o] = dx;
}
template <typename T>
void launch_tau0(const T* d0, int N2, int N1, T inv_h, T* tau0, hipStream_t s) {
  hipLaunchKernelGGL(k_tau0<T>, grid2d(N2 + 1, N1 + 1), dim3(kBX, kBY), 0, s, d0, N2, N1, inv_h, tau0);
  TVS_LAUNCH_CHECK();
}

template <typename T>
__device__ __forceinline__ T dm_at(const T* w, long long o, int idx, int n, long long step) {
  // D^-: (w(idx) unless last) - (w(idx-1) unless first), without 1/h
  const T a = (idx == n - 1) ? T(0) : w[o];
  const T b = (idx > 0) ? w[o - step] : T(0);
  return a - b;
}

// z_k = div p_k, k = 1, 2, on the whole grid (vecdiv, Section 4.1)
template <typename T>
__global__ void k_global_vecdiv(const T* __restrict__ p, Grid g, T inv_h, T* __restrict__ z) {
  const int j = blockIdx.x * kBX + threadIdx.x, i = blockIdx.y * kBY + threadIdx.y;
  if (i >= g.n2 || j >= g.n1) return;
  const long long plane = (long long)g.n2 * g.n1;
  const long long o = (long long)i * g.n1 + j;
  for (int k = 0; k < 2; ++k) {
    const T* px = p + (2 * k) * plane;
    const T* py = p + (2 * k + 1) * plane;
    z[k * plane + o] = (dm_at(px, o, j, g.n1, 1) + dm_at(py, o, i, g.n2, g.n1)) * inv_h;
  }
}
template <typename T> void launch_global_vecdiv(const T* p, Grid g, T inv_h, T* z, hipStream_t s) {
  hipLaunchKernelGGL(k_global_vecdiv<T>, grid2d(g.n2, g.n1), dim3(kBX, kBY), 0, s, p, g, inv_h, z);
  TVS_LAUNCH_CHECK();
}

// (grad phi)_c at (i, j): c = 0 -> D^+_x, c = 1 -> D^+_y
template <typename T>
__device__ __forceinline__ T dp_global(const T* phi, Grid g, int i, int j, int c, T inv_h) {
  const long long o = (long long)i * g.n1 + j;
  if (c == 0) return (j == g.n1 - 1) ? T(0) : (phi[o + 1] - phi[o]) * inv_h;
  return (i == g.n2 - 1) ? T(0) : (phi[o + g.n1] - phi[o]) * inv_h;
}

// f = delta^{-1} P_K tau_0 = (tau_0 - grad phi)/delta with phi = Delta^+ div tau_0
template <typename T>
__global__ void k_f1(const T* tau0, const T* __restrict__ phi, Grid g, T inv_h, T inv_delta,
                     T* f1) {  // tau0 and f1 may alias (each point is read before it is written)
  const int j = blockIdx.x * kBX + threadIdx.x, i = blockIdx.y * kBY + threadIdx.y;
  if (i >= g.n2 || j >= g.n1) return;
  const long long plane = (long long)g.n2 * g.n1;
  const long long o = (long long)i * g.n1 + j;
  for (int c = 0; c < 2; ++c)
    f1[c * plane + o] = (tau0[c * plane + o] - dp_global(phi, g, i, j, c, inv_h)) * inv_delta;
}
template <typename T>
void launch_f1(const T* tau0, const T* phi, Grid g, T inv_h, T inv_delta, T* f1, hipStream_t s) {
  hipLaunchKernelGGL(k_f1<T>, grid2d(g.n2, g.n1), dim3(kBX, kBY), 0, s, tau0, phi, g, inv_h, inv_delta, f1);
  TVS_LAUNCH_CHECK();
}

// r = f - P_K vecdiv p = f - (z - grad phi), and the FP64 energy ||r||^2
template <typename T>
__global__ __launch_bounds__(256) void k_residual(const T* __restrict__ f1, const T* __restrict__ z,
                                                  const T* __restrict__ phi, Grid g, T inv_h,
                                                  T* __restrict__ r, double* __restrict__ part) {
  const long long plane = (long long)g.n2 * g.n1;
  double acc = 0.0;
  for (long long o = blockIdx.x * 256LL + threadIdx.x; o < plane; o += 256LL * gridDim.x) {
    const int i = int(o / g.n1), j = int(o - (long long)i * g.n1);
    for (int c = 0; c < 2; ++c) {
      const T v = f1[c * plane + o] - (z[c * plane + o] - dp_global(phi, g, i, j, c, inv_h));
      r[c * plane + o] = v;
      acc += double(v) * double(v);
    }
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
template <typename T>
void launch_residual(const T* f1, const T* z, const T* phi, Grid g, T inv_h, T* r, Partials part,
                     double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_residual<T>, dim3(kRedBlocks), dim3(256), 0, s, f1, z, phi, g, inv_h, r, part.buf);
  TVS_LAUNCH_CHECK();
  finish_sum(part, kRedBlocks, out, s);
}

// TFS duality gap sum_k sum (|grad tau_k| + grad tau_k . p_k)
template <typename T>
__global__ __launch_bounds__(256) void k_gap_tfs(const T* __restrict__ tau, const T* __restrict__ p,
                                                 Grid g, T inv_h, double* __restrict__ part) {
  const long long plane = (long long)g.n2 * g.n1;
  double acc = 0.0;
  for (long long o = blockIdx.x * 256LL + threadIdx.x; o < plane; o += 256LL * gridDim.x) {
    const int i = int(o / g.n1), j = int(o - (long long)i * g.n1);
    for (int k = 0; k < 2; ++k) {
      const T* t = tau + k * plane;
      const double gx = double(dp_global(t, g, i, j, 0, inv_h));
      const double gy = double(dp_global(t, g, i, j, 1, inv_h));
      const double px = double(p[(2 * k) * plane + o]), py = double(p[(2 * k + 1) * plane + o]);
      acc += sqrt(gx * gx + gy * gy) + gx * px + gy * py;
    }
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
template <typename T>
void launch_gap_tfs(const T* tau, const T* p, Grid g, T inv_h, Partials part, double* out,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_gap_tfs<T>, dim3(kRedBlocks), dim3(256), 0, s, tau, p, g, inv_h, part.buf);
  TVS_LAUNCH_CHECK();
  finish_sum(part, kRedBlocks, out, s);
}

// ---------------------------------------------------------------------------
// Step 1, per subdomain
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T theta_at(const SubFrames& sf, const SubDesc& sd, int gi, int gj) {
  return axis_theta<T>(sf.ay, sd.m2, gi) * axis_theta<T>(sf.ax, sd.m1, gj);
}

// v = theta_m p on the subdomain, 0 elsewhere in the frame
template <typename T>
__global__ void k_sub_theta_p(SubFrames sf, Grid g, const T* __restrict__ p, int planes,
                              T* __restrict__ v) {
  const int q = blockIdx.x * kBX + threadIdx.x, r = blockIdx.y * kBY + threadIdx.y;
  const SubDesc sd = sf.subs[blockIdx.z];
  if (r >= sf.fr || q >= sf.fp) return;
  const long long fo = (long long)blockIdx.z * planes * sf.plane + (long long)r * sf.fp + q;
  const long long gplane = (long long)g.n2 * g.n1;
  const bool in = r < sd.si && q < sd.sj;
  const int gi = sd.i0 + r, gj = sd.j0 + q;
  const T th = in ? theta_at<T>(sf, sd, gi, gj) : T(0);
  const long long go = (long long)gi * g.n1 + gj;
  for (int c = 0; c < planes; ++c) v[fo + c * sf.plane] = in ? th * p[c * gplane + go] : T(0);
}
template <typename T>
void launch_sub_theta_p(const SubFrames& sf, Grid g, const T* p, int planes, T* v, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_theta_p<T>, grid2d(sf.fr, sf.fp, sf.nsub), dim3(kBX, kBY), 0, s, sf, g, p, planes, v);
  TVS_LAUNCH_CHECK();
}

// Element e of an array given by a 32-bit element offset (so the address is a
// scalar base plus a 32-bit vector offset).
template <typename T>
__device__ __forceinline__ T ld32(const T* base, unsigned e) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + e * unsigned(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st32(T* base, unsigned e, T x) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + e * unsigned(sizeof(T))) = x;
}

// Per-subdomain stencil kernels give each thread a run of RY consecutive
// rows of one frame column (a 64-wide wavefront spans one row segment, so
// row quantities are uniform over it).  RY is 1, 2 or 4, chosen per problem
// shape by the tuner (SubFrames::run); every choice computes the same
// values.

// Tiles of kBX columns x kBY * RY rows of the nz frames are numbered rows
// fastest, then columns, then frames.  Workgroups are dealt round-robin to
// the 8 XCDs, so workgroup w takes tile (w mod 8) * per + w / 8 (per = tiles
// per XCD, the grid is 8 * per): each XCD then works through a contiguous
// range of tiles, and tiles that share halo rows run on the same XCD, close
// in time, and find those rows in its L2.
struct RunTiles {
  int ncx, nry, n, ry;
};
static RunTiles run_tiles(int n2, int n1, int nz, int ry) {
  RunTiles t{(n1 + kBX - 1) / kBX, (n2 + kBY * ry - 1) / (kBY * ry), 0, ry};
  t.n = t.ncx * t.nry * nz;
  return t;
}
// calls f(std::integral_constant<int, RY>{}) for the run length of sf
template <typename F>
static void with_run(int run, F&& f) {
  switch (run) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    default: f(std::integral_constant<int, 2>{}); break;
  }
}
static dim3 grid_runs(const RunTiles& t) { return dim3(8 * ((t.n + 7) / 8)); }
// This thread's frame column q, first row r0 (wavefront-uniform) and frame;
// false for the workgroups past the last tile.
__device__ __forceinline__ bool run_tile(const RunTiles& t, int& q, int& r0, int& box) {
  const int per = int(gridDim.x) / 8;
  const int w = blockIdx.x;
  const int tile = (w & 7) * per + (w >> 3);
  if (tile >= t.n) return false;
  const int ry = tile % t.nry, rest = tile / t.nry;
  box = rest / t.ncx;
  q = (rest - box * t.ncx) * kBX + threadIdx.x;
  r0 = __builtin_amdgcn_readfirstlane((ry * kBY + int(threadIdx.y)) * t.ry);
  return true;
}

// z = vecdiv(E_m v) on the grown subdomain.  Only the grown subdomain is
// written: the rest of a z frame is 0 from the start of the solve.  Row runs
// as in the update kernels below, carrying v_xy and v_yy of the row above.
template <typename T, int RY, bool JB>
__global__ __launch_bounds__(kBX* kBY) void k_sub_vecdiv(SubFrames sf, RunTiles rt, Grid g, T inv_h,
                                                        const T* __restrict__ v,
                                                        T* __restrict__ z, JobRef<T> jr) {
  int q, r0, bz;
  if (!run_tile(rt, q, r0, bz)) return;
  if constexpr (JB) {
    const int j = bz / jr.nsub;
    const JobBufs<T>& jb = jr.jobs[j];
    const int st = jb.par ^ jr.flip;
    v = jb.v[st];
    z = jb.z[st];
    bz -= j * jr.nsub;
  }
  const SubDesc sd = sf.subs[bz];
  if (r0 >= sd.ai || q >= sd.aj) return;
  const unsigned fp = sf.fp, pl = unsigned(sf.plane);
  const size_t box = bz;
  const T* v0 = v + box * 4 * pl;
  const T* v1 = v0 + pl;
  const T* v2 = v1 + pl;
  const T* v3 = v2 + pl;
  T* z0 = z + box * 2 * pl;
  T* z1 = z0 + pl;
  const bool lastx = sd.j0 + q == g.n1 - 1;
  const unsigned dl = q > 0 ? 1u : 0u;
  unsigned o = unsigned(r0) * fp + unsigned(q);
  T u1 = r0 > 0 ? ld32(v1, o - fp) : T(0), u3 = r0 > 0 ? ld32(v3, o - fp) : T(0);
  const int rend = min(RY, sd.ai - r0);
  int gi = sd.i0 + r0;
  for (int rr = 0; rr < rend; ++rr, o += fp, ++gi) {
    const bool lasty = gi == g.n2 - 1;
    const T a0 = ld32(v0, o), l0 = ld32(v0, o - dl), a1 = ld32(v1, o);
    const T a2 = ld32(v2, o), l2 = ld32(v2, o - dl), a3 = ld32(v3, o);
    st32(z0, o, (((lastx ? T(0) : a0) - (q > 0 ? l0 : T(0))) + ((lasty ? T(0) : a1) - u1)) * inv_h);
    st32(z1, o, (((lastx ? T(0) : a2) - (q > 0 ? l2 : T(0))) + ((lasty ? T(0) : a3) - u3)) * inv_h);
    u1 = a1;
    u3 = a3;
  }
}
template <typename T>
void launch_sub_vecdiv(const SubFrames& sf, Grid g, T inv_h, const T* v, T* z, hipStream_t s) {
  with_run(sf.run_div, [&](auto ry) {
    const RunTiles rt = run_tiles(sf.fr, sf.fp, sf.nsub, ry);
    hipLaunchKernelGGL((k_sub_vecdiv<T, decltype(ry)::value, false>), grid_runs(rt), dim3(kBX, kBY), 0, s, sf, rt, g,
                       inv_h, v, z, JobRef<T>{nullptr, sf.nsub, 0});
    TVS_LAUNCH_CHECK();
  });
}
template <typename T>
void launch_sub_vecdiv_jobs(const SubFrames& sf, Grid g, T inv_h, JobRef<T> jr, int njobs, hipStream_t s) {
  with_run(sf.run_div, [&](auto ry) {
    const RunTiles rt = run_tiles(sf.fr, sf.fp, sf.nsub * njobs, ry);
    hipLaunchKernelGGL((k_sub_vecdiv<T, decltype(ry)::value, true>), grid_runs(rt), dim3(kBX, kBY), 0, s, sf, rt, g,
                       inv_h, nullptr, nullptr, jr);
    TVS_LAUNCH_CHECK();
  });
}

// (grad phi)_c inside a frame, with the grid's last-row/column rule
template <typename T>
__device__ __forceinline__ T dp_frame(const T* phi, long long lo, int fp, int gi, int gj, Grid g,
                                      int c, T inv_h) {
  if (c == 0) return (gj == g.n1 - 1) ? T(0) : (phi[lo + 1] - phi[lo]) * inv_h;
  return (gi == g.n2 - 1) ? T(0) : (phi[lo + fp] - phi[lo]) * inv_h;
}

// omega_m = R_{m,+} r + LP_m(vecdiv(theta_m p)) = r + z - grad phi on the
// grown subdomain (uses sum_{l != m} theta_l = 1 - theta_m)
template <typename T>
__global__ void k_sub_omega(SubFrames sf, Grid g, T inv_h, const T* __restrict__ r,
                            const T* __restrict__ z, const T* __restrict__ phi, T* __restrict__ omega) {
  const int q = blockIdx.x * kBX + threadIdx.x, rr = blockIdx.y * kBY + threadIdx.y;
  const SubDesc sd = sf.subs[blockIdx.z];
  if (rr >= sf.fr || q >= sf.fp) return;
  const long long lo = (long long)rr * sf.fp + q;
  const T* zb = z + (long long)blockIdx.z * 2 * sf.plane;
  const T* pb = phi + (long long)blockIdx.z * sf.plane;
  T* ob = omega + (long long)blockIdx.z * 2 * sf.plane;
  if (rr < sd.ai && q < sd.aj) {
    const int gi = sd.i0 + rr, gj = sd.j0 + q;
    const long long gplane = (long long)g.n2 * g.n1;
    const long long go = (long long)gi * g.n1 + gj;
    for (int c = 0; c < 2; ++c)
      ob[c * sf.plane + lo] = r[c * gplane + go] + (zb[c * sf.plane + lo] - dp_frame(pb, lo, sf.fp, gi, gj, g, c, inv_h));
  } else {
    ob[lo] = T(0);
    ob[sf.plane + lo] = T(0);
  }
}
template <typename T>
void launch_sub_omega(const SubFrames& sf, Grid g, T inv_h, const T* r, const T* z, const T* phi,
                      T* omega, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_omega<T>, grid2d(sf.fr, sf.fp, sf.nsub), dim3(kBX, kBY), 0, s, sf, g, inv_h, r, z, phi, omega);
  TVS_LAUNCH_CHECK();
}

// theta / (theta + t sqrt(nn)): FP32 uses the hardware square root (about
// 1 ulp) and the hardware reciprocal refined by one Newton step; FP64 the
// correctly rounded operations.
__device__ __forceinline__ float dual_scale(float th, float t, float nn) {
  const float d = th + t * __builtin_amdgcn_sqrtf(nn);
  float r = __builtin_amdgcn_rcpf(d);
  r = fmaf(r, fmaf(-d, r, 1.0f), r);
  return th * r;
}
__device__ __forceinline__ double dual_scale(double th, double t, double nn) {
  return th / (th + t * sqrt(nn));
}

// Inner iteration of Algorithm 5:
//   y = LP_m(z) = z - grad phi,  psi_k = grad(y_k - omega_k) on the subdomain,
//   v_k <- theta (v_k + t psi_k) / (theta + t |psi_k|).
// Each thread walks RY consecutive rows of one column; w_k = y_k - omega_k
// at (r + 1, q), needed for psi at row r, is carried to the next row.  The
// wavefront spans one row segment (kBX == 64), so row quantities are uniform.
// Neighbour offsets are clamped to 0 where the grid ends, which makes the
// corresponding forward difference of phi vanish and keeps every load inside
// the frame; psi components there are set to 0 explicitly.
template <typename T, int RY, bool JB>
__global__ __launch_bounds__(kBX* kBY) void k_sub_update1(SubFrames sf, RunTiles rt, Grid g, StepScalars<T> cs,
                                                         const T* __restrict__ v,
                                                         const T* __restrict__ z,
                                                         const T* __restrict__ phi,
                                                         const T* __restrict__ omega,
                                                         T* __restrict__ v_out, JobRef<T> jr) {
  int q, r0, bz;
  if (!run_tile(rt, q, r0, bz)) return;
  if constexpr (JB) {
    const int j = bz / jr.nsub;
    const JobBufs<T>& jb = jr.jobs[j];
    const int st = jb.par ^ jr.flip;
    v = jb.v[st];
    z = jb.z[st];
    phi = jb.phi;
    omega = jb.aux;
    v_out = jb.v[st ^ 1];
    bz -= j * jr.nsub;
  }
  const SubDesc sd = sf.subs[bz];
  if (r0 >= sd.si || q >= sd.sj) return;
  const unsigned fp = sf.fp, pl = unsigned(sf.plane);
  const size_t box = bz;
  const T* v0 = v + box * 4 * pl;
  const T* v1 = v0 + pl;
  const T* v2 = v1 + pl;
  const T* v3 = v2 + pl;
  T* o0 = v_out + box * 4 * pl;
  T* o1 = o0 + pl;
  T* o2 = o1 + pl;
  T* o3 = o2 + pl;
  const T* z0 = z + box * 2 * pl;
  const T* z1 = z0 + pl;
  const T* m0 = omega + box * 2 * pl;
  const T* m1 = m0 + pl;
  const T* ph = phi + box * pl;
  const T* thy = theta_rows<T>(sf) + sd.m2 * sf.fr;
  const T ih = cs.inv_h, t = cs.t;
  const int gj = sd.j0 + q;
  const bool lastx = gj == g.n1 - 1;                   // psi_x = 0, (grad phi)_x = 0
  const unsigned dx = lastx ? 0u : 1u;                  // (grad phi)_x at column q
  const unsigned de = lastx ? 0u : 1u;                  // right neighbour
  const unsigned dxe = (lastx || gj + 1 == g.n1 - 1) ? 0u : 1u;  // (grad phi)_x there
  const T thx = theta_cols<T>(sf)[sd.m1 * sf.fp + q];
  unsigned o = unsigned(r0) * fp + unsigned(q);
  int gi = sd.i0 + r0;
  T wa0 = ld32(z0, o) - (ld32(ph, o + dx) - ld32(ph, o)) * ih - ld32(m0, o);
  T wa1 = ld32(z1, o) - (ld32(ph, o + (gi == g.n2 - 1 ? 0u : fp)) - ld32(ph, o)) * ih - ld32(m1, o);
  const int rend = min(RY, sd.si - r0);
  for (int rr = 0; rr < rend; ++rr, o += fp, ++gi) {
    const bool lasty = gi == g.n2 - 1;                  // uniform over the wavefront
    const unsigned dy = lasty ? 0u : fp;                // (grad phi)_y in row r; lower neighbour
    const unsigned dys = (lasty || gi + 1 == g.n2 - 1) ? 0u : fp;  // (grad phi)_y in row r + 1
    const unsigned oe = o + de, os = o + dy;
    const T we0 = ld32(z0, oe) - (ld32(ph, oe + dxe) - ld32(ph, oe)) * ih - ld32(m0, oe);
    const T we1 = ld32(z1, oe) - (ld32(ph, oe + dy) - ld32(ph, oe)) * ih - ld32(m1, oe);
    const T wd0 = ld32(z0, os) - (ld32(ph, os + dx) - ld32(ph, os)) * ih - ld32(m0, os);
    const T wd1 = ld32(z1, os) - (ld32(ph, os + dys) - ld32(ph, os)) * ih - ld32(m1, os);
    const T px0 = lastx ? T(0) : (we0 - wa0) * ih;
    const T px1 = lastx ? T(0) : (we1 - wa1) * ih;
    const T py0 = lasty ? T(0) : (wd0 - wa0) * ih;
    const T py1 = lasty ? T(0) : (wd1 - wa1) * ih;
    const T th = thx * thy[r0 + rr];
    const T s0 = dual_scale(th, t, px0 * px0 + py0 * py0);
    const T s1 = dual_scale(th, t, px1 * px1 + py1 * py1);
    st32(o0, o, s0 * (ld32(v0, o) + t * px0));
    st32(o1, o, s0 * (ld32(v1, o) + t * py0));
    st32(o2, o, s1 * (ld32(v2, o) + t * px1));
    st32(o3, o, s1 * (ld32(v3, o) + t * py1));
    wa0 = wd0;
    wa1 = wd1;
  }
}
template <typename T>
void launch_sub_update1(const SubFrames& sf, Grid g, StepScalars<T> c, const T* v, const T* z,
                        const T* phi, const T* omega, T* v_out, hipStream_t s) {
  with_run(sf.run, [&](auto ry) {
    const RunTiles rt = run_tiles(sf.fr, sf.fp, sf.nsub, ry);
    hipLaunchKernelGGL((k_sub_update1<T, decltype(ry)::value, false>), grid_runs(rt), dim3(kBX, kBY), 0, s, sf, rt, g, c,
                       v, z, phi, omega, v_out, JobRef<T>{nullptr, sf.nsub, 0});
    TVS_LAUNCH_CHECK();
  });
}
template <typename T>
void launch_sub_update1_jobs(const SubFrames& sf, Grid g, StepScalars<T> c, JobRef<T> jr, int njobs,
                             hipStream_t s) {
  with_run(sf.run, [&](auto ry) {
    const RunTiles rt = run_tiles(sf.fr, sf.fp, sf.nsub * njobs, ry);
    hipLaunchKernelGGL((k_sub_update1<T, decltype(ry)::value, true>), grid_runs(rt), dim3(kBX, kBY), 0, s, sf, rt, g, c,
                       nullptr, nullptr, nullptr, nullptr, nullptr, jr);
    TVS_LAUNCH_CHECK();
  });
}

// p^{n+1} = (1 - ahat) p^n + ahat sum_m E_m v_m (Algorithm 2).  Along each
// axis a point lies in at most two subdomains: the one owning its core and a
// neighbour whose stripe covers it.
__device__ __forceinline__ int axis_hits(const AxisLayout& a, int x, int lim, int* out) {
  // core index c with cut[c] <= x < cut[c+1]
  int c = int(((long long)(x + 1) * a.m - 1) / a.n);
  if (c >= a.m) c = a.m - 1;
  int k = 0;
  for (int m = c - 1; m <= c + 1; ++m) {
    if (m < 0 || m >= a.m) continue;
    const int e = a.end[m] < lim ? a.end[m] : lim;
    if (x >= a.start[m] && x < e) out[k++] = m;
  }
  return k;
}

template <typename T>
__global__ void k_combine(SubFrames sf, Grid g, int planes, T ahat, const T* __restrict__ v,
                          T* __restrict__ p) {
  const int j = blockIdx.x * kBX + threadIdx.x, i = blockIdx.y * kBY + threadIdx.y;
  if (i >= g.n2 || j >= g.n1) return;
  int hy[3], hx[3];
  const int ny = axis_hits(sf.ay, i, g.n2, hy), nx = axis_hits(sf.ax, j, g.n1, hx);
  const long long gplane = (long long)g.n2 * g.n1;
  const long long go = (long long)i * g.n1 + j;
  for (int c = 0; c < planes; ++c) {
    T acc = T(0);
    for (int a = 0; a < ny; ++a)
      for (int b = 0; b < nx; ++b) {
        const int m = hy[a] * sf.ax.m + hx[b];
        const SubDesc sd = sf.subs[m];
        const long long lo = (long long)(i - sd.i0) * sf.fp + (j - sd.j0);
        acc += v[(long long)m * planes * sf.plane + c * sf.plane + lo];
      }
    p[c * gplane + go] = (T(1) - ahat) * p[c * gplane + go] + ahat * acc;
  }
}
template <typename T>
void launch_combine(const SubFrames& sf, Grid g, int planes, T ahat, const T* v, T* p, hipStream_t s) {
  hipLaunchKernelGGL(k_combine<T>, grid2d(g.n2, g.n1), dim3(kBX, kBY), 0, s, sf, g, planes, ahat, v, p);
  TVS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Step 2
// ---------------------------------------------------------------------------

// IRV2 potential and data: g = h * (row prefix sum of tau_2 on Omega),
// f = alpha (d0 - g).  One workgroup per row; each thread sums a contiguous
// chunk, the chunk totals are scanned in LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_bridge_irv2(const T* __restrict__ tau, const T* __restrict__ d0,
                                                     int N2, int N1, T h, T alpha, T* __restrict__ f2) {
  __shared__ T tot[256];
  const int i = blockIdx.x;
  const int n1t = N1 + 1;
  const T* t2 = tau + (long long)(N2 + 1) * n1t + (long long)i * n1t;
  const int chunk = (N1 + 255) / 256;
  const int a = threadIdx.x * chunk, b = min(N1, a + chunk);
  T s = T(0);
  for (int j = a; j < b; ++j) s += t2[j];
  tot[threadIdx.x] = s;
  __syncthreads();
  // inclusive Hillis-Steele scan of the 256 chunk totals
  for (int off = 1; off < 256; off <<= 1) {
    const T add = threadIdx.x >= off ? tot[threadIdx.x - off] : T(0);
    __syncthreads();
    tot[threadIdx.x] += add;
    __syncthreads();
  }
  T run = threadIdx.x > 0 ? tot[threadIdx.x - 1] : T(0);
  for (int j = a; j < b; ++j) {
    run += t2[j];
    f2[(long long)i * N1 + j] = alpha * (d0[(long long)i * N1 + j] - h * run);
  }
}
template <typename T>
void launch_bridge_irv2(const T* tau, const T* d0, int N2, int N1, T h, T alpha, T* f2, hipStream_t s) {
  hipLaunchKernelGGL(k_bridge_irv2<T>, dim3(N2), dim3(256), 0, s, tau, d0, N2, N1, h, alpha, f2);
  TVS_LAUNCH_CHECK();
}

// b_m = div((1 - theta_m) p) - f on the grown subdomain (Algorithm 3 with
// Lambda = div; only the part near the subdomain is ever read)
template <typename T>
__global__ void k_sub2_prologue(SubFrames sf, Grid g, T inv_h, const T* __restrict__ p,
                                const T* __restrict__ f2, T* __restrict__ bfr) {
  const int q = blockIdx.x * kBX + threadIdx.x, r = blockIdx.y * kBY + threadIdx.y;
  const SubDesc sd = sf.subs[blockIdx.z];
  if (r >= sf.fr || q >= sf.fp) return;
  const long long lo = (long long)r * sf.fp + q;
  T* bb = bfr + (long long)blockIdx.z * sf.plane;
  if (r >= sd.ai || q >= sd.aj) { bb[lo] = T(0); return; }
  const int gi = sd.i0 + r, gj = sd.j0 + q;
  const long long gplane = (long long)g.n2 * g.n1;
  const long long go = (long long)gi * g.n1 + gj;
  auto w = [&](int c, int ii, int jj) {
    const T th = axis_theta<T>(sf.ay, sd.m2, ii) * axis_theta<T>(sf.ax, sd.m1, jj);
    return (T(1) - th) * p[c * gplane + (long long)ii * g.n1 + jj];
  };
  const T a = (gj == g.n1 - 1) ? T(0) : w(0, gi, gj);
  const T am = (gj > 0) ? w(0, gi, gj - 1) : T(0);
  const T c = (gi == g.n2 - 1) ? T(0) : w(1, gi, gj);
  const T cm = (gi > 0) ? w(1, gi - 1, gj) : T(0);
  bb[lo] = ((a - am) + (c - cm)) * inv_h - f2[go];
}
template <typename T>
void launch_sub2_prologue(const SubFrames& sf, Grid g, T inv_h, const T* p, const T* f2, T* b,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_sub2_prologue<T>, grid2d(sf.fr, sf.fp, sf.nsub), dim3(kBX, kBY), 0, s, sf, g, inv_h, p, f2, b);
  TVS_LAUNCH_CHECK();
}

// Inner iteration of Algorithm 3 for the ROF dual: psi = grad(div v + b) on
// the subdomain, v <- theta (v + t psi) / (theta + t |psi|).  Row runs as in
// the Step-1 update: s = div v + b at (r + 1, q) and v there are carried to
// the next row.  Terms of the backward differences that fall outside the
// frame support, or on the grid's last row/column, are selected to 0; their
// loads use clamped offsets inside the frame.
template <typename T, int RY, bool JB>
__global__ __launch_bounds__(kBX* kBY) void k_sub2_update(SubFrames sf, RunTiles rt, Grid g, StepScalars<T> cs,
                                                         const T* __restrict__ v,
                                                         const T* __restrict__ bfr,
                                                         T* __restrict__ v_out, JobRef<T> jr) {
  int q, r0, bz;
  if (!run_tile(rt, q, r0, bz)) return;
  if constexpr (JB) {
    const int j = bz / jr.nsub;
    const JobBufs<T>& jb = jr.jobs[j];
    const int st = jb.par ^ jr.flip;
    v = jb.v[st];
    bfr = jb.aux;
    v_out = jb.v[st ^ 1];
    bz -= j * jr.nsub;
  }
  const SubDesc sd = sf.subs[bz];
  if (r0 >= sd.si || q >= sd.sj) return;
  const unsigned fp = sf.fp, pl = unsigned(sf.plane);
  const size_t box = bz;
  const T* vx = v + box * 2 * pl;
  const T* vy = vx + pl;
  const T* bb = bfr + box * pl;
  T* ox = v_out + box * 2 * pl;
  T* oy = ox + pl;
  const T* thy = theta_rows<T>(sf) + sd.m2 * sf.fr;
  const T ih = cs.inv_h, t = cs.t;
  const int gj = sd.j0 + q;
  const bool lastx = gj == g.n1 - 1;
  const bool lastx1 = lastx || gj + 1 == g.n1 - 1;  // right neighbour on the last column
  const unsigned de = lastx ? 0u : 1u;
  const unsigned dl = q > 0 ? 1u : 0u;             // left neighbour inside the frame
  const T thx = theta_cols<T>(sf)[sd.m1 * sf.fp + q];
  unsigned o = unsigned(r0) * fp + unsigned(q);
  int gi = sd.i0 + r0;
  // s, vx and vy at (r0, q); vy at (r0 - 1, q)
  T xa = ld32(vx, o), ya = ld32(vy, o);
  T yu = r0 > 0 ? ld32(vy, o - fp) : T(0);
  const T xl0 = q > 0 ? ld32(vx, o - dl) : T(0);
  T sa = (((lastx ? T(0) : xa) - xl0) + ((gi == g.n2 - 1 ? T(0) : ya) - yu)) * ih + ld32(bb, o);
  const int rend = min(RY, sd.si - r0);
  for (int rr = 0; rr < rend; ++rr, o += fp, ++gi) {
    const int r = r0 + rr;
    const bool lasty = gi == g.n2 - 1;
    const unsigned dy = lasty ? 0u : fp;
    const unsigned du = r > 0 ? fp : 0u;
    const unsigned oe = o + de, os = o + dy;
    // right neighbour (r, q + 1): vx(r, q+1) - vx(r, q) + vy(r, q+1) - vy(r-1, q+1)
    const T xe = ld32(vx, oe), ye = ld32(vy, oe), yeu = ld32(vy, oe - du);
    const T se = (((lastx1 ? T(0) : xe) - xa) + ((lasty ? T(0) : ye) - (r > 0 ? yeu : T(0)))) * ih +
                 ld32(bb, oe);
    // lower neighbour (r + 1, q): vx(r+1, q) - vx(r+1, q-1) + vy(r+1, q) - vy(r, q)
    const T xs = ld32(vx, os), xsl = ld32(vx, os - dl), ys = ld32(vy, os);
    const bool lasty1 = lasty || gi + 1 == g.n2 - 1;
    const T ss = (((lastx ? T(0) : xs) - (q > 0 ? xsl : T(0))) + ((lasty1 ? T(0) : ys) - ya)) * ih +
                 ld32(bb, os);
    const T px = lastx ? T(0) : (se - sa) * ih;
    const T py = lasty ? T(0) : (ss - sa) * ih;
    const T th = thx * thy[r];
    const T sc = dual_scale(th, t, px * px + py * py);
    st32(ox, o, sc * (xa + t * px));
    st32(oy, o, sc * (ya + t * py));
    sa = ss;
    xa = xs;
    ya = ys;
  }
}
template <typename T>
void launch_sub2_update(const SubFrames& sf, Grid g, StepScalars<T> c, const T* v, const T* b,
                        T* v_out, hipStream_t s) {
  with_run(sf.run, [&](auto ry) {
    const RunTiles rt = run_tiles(sf.fr, sf.fp, sf.nsub, ry);
    hipLaunchKernelGGL((k_sub2_update<T, decltype(ry)::value, false>), grid_runs(rt), dim3(kBX, kBY), 0, s, sf, rt, g, c,
                       v, b, v_out, JobRef<T>{nullptr, sf.nsub, 0});
    TVS_LAUNCH_CHECK();
  });
}
template <typename T>
void launch_sub2_update_jobs(const SubFrames& sf, Grid g, StepScalars<T> c, JobRef<T> jr, int njobs,
                             hipStream_t s) {
  with_run(sf.run, [&](auto ry) {
    const RunTiles rt = run_tiles(sf.fr, sf.fp, sf.nsub * njobs, ry);
    hipLaunchKernelGGL((k_sub2_update<T, decltype(ry)::value, true>), grid_runs(rt), dim3(kBX, kBY), 0, s, sf, rt, g, c,
                       nullptr, nullptr, nullptr, jr);
    TVS_LAUNCH_CHECK();
  });
}

template <typename T>
__device__ __forceinline__ T div_global(const T* p, Grid g, int i, int j, T inv_h) {
  const long long plane = (long long)g.n2 * g.n1;
  const long long o = (long long)i * g.n1 + j;
  return (dm_at(p, o, j, g.n1, 1) + dm_at(p + plane, o, i, g.n2, g.n1)) * inv_h;
}

// ||div p - f||^2 (IRV2 dual energy)
template <typename T>
__global__ __launch_bounds__(256) void k_energy_rof(const T* __restrict__ p, const T* __restrict__ f2,
                                                    Grid g, T inv_h, double* __restrict__ part) {
  const long long plane = (long long)g.n2 * g.n1;
  double acc = 0.0;
  for (long long o = blockIdx.x * 256LL + threadIdx.x; o < plane; o += 256LL * gridDim.x) {
    const int i = int(o / g.n1), j = int(o - (long long)i * g.n1);
    const double v = double(div_global(p, g, i, j, inv_h)) - double(f2[o]);
    acc += v * v;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
template <typename T>
void launch_energy_rof(const T* p, const T* f2, Grid g, T inv_h, Partials part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_rof<T>, dim3(kRedBlocks), dim3(256), 0, s, p, f2, g, inv_h, part.buf);
  TVS_LAUNCH_CHECK();
  finish_sum(part, kRedBlocks, out, s);
}

// Image-quality moments of x against r (Section 5.2): FP64 sums of x and r
// (first pass), then of (x - mean x)^2, (r - mean r)^2, their product and
// (x - r)^2 (second pass, centred on the first pass's means, read from the
// device so that no host round trip separates the passes).
constexpr int kQBlocks = 256;  // workgroups per moment; 4 moments fit 1024 partials

template <typename T>
__global__ __launch_bounds__(256) void k_moments1(const T* __restrict__ x, const T* __restrict__ r, long long n,
                                                  double* __restrict__ part) {
  double sx = 0.0, sr = 0.0;
  for (long long o = blockIdx.x * 256LL + threadIdx.x; o < n; o += 256LL * gridDim.x) {
    sx += double(x[o]);
    sr += double(r[o]);
  }
  sx = block_sum(sx);
  sr = block_sum(sr);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sx;
    part[kQBlocks + blockIdx.x] = sr;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_moments2(const T* __restrict__ x, const T* __restrict__ r, long long n,
                                                  const double* __restrict__ sums, double* __restrict__ part) {
  const double mx = sums[0] / double(n), mr = sums[1] / double(n);
  double vx = 0.0, vr = 0.0, cv = 0.0, se = 0.0;
  for (long long o = blockIdx.x * 256LL + threadIdx.x; o < n; o += 256LL * gridDim.x) {
    const double a = double(x[o]), b = double(r[o]);
    const double da = a - mx, db = b - mr, e = a - b;
    vx += da * da;
    vr += db * db;
    cv += da * db;
    se += e * e;
  }
  vx = block_sum(vx);
  vr = block_sum(vr);
  cv = block_sum(cv);
  se = block_sum(se);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = vx;
    part[kQBlocks + blockIdx.x] = vr;
    part[2 * kQBlocks + blockIdx.x] = cv;
    part[3 * kQBlocks + blockIdx.x] = se;
  }
}

template <typename T>
void launch_quality_moments(const T* x, const T* r, long long n, Partials part, double* out, hipStream_t s) {
  if (part.cap < 4 * kQBlocks) throw Error(-1, "internal: partial-sum buffer too small");
  hipLaunchKernelGGL(k_moments1<T>, dim3(kQBlocks), dim3(256), 0, s, x, r, n, part.buf);
  TVS_LAUNCH_CHECK();
  for (int k = 0; k < 2; ++k) finish_sum(Partials{part.buf + k * kQBlocks, kQBlocks}, kQBlocks, out + k, s);
  hipLaunchKernelGGL(k_moments2<T>, dim3(kQBlocks), dim3(256), 0, s, x, r, n, out, part.buf);
  TVS_LAUNCH_CHECK();
  for (int k = 0; k < 4; ++k) finish_sum(Partials{part.buf + k * kQBlocks, kQBlocks}, kQBlocks, out + 2 + k, s);
}

// d = d0 - div p / alpha
template <typename T>
__global__ void k_irv2_image(const T* __restrict__ d0, const T* __restrict__ p, Grid g, T inv_h,
                             T inv_alpha, T* __restrict__ d) {
  const int j = blockIdx.x * kBX + threadIdx.x, i = blockIdx.y * kBY + threadIdx.y;
  if (i >= g.n2 || j >= g.n1) return;
  const long long o = (long long)i * g.n1 + j;
  d[o] = d0[o] - div_global(p, g, i, j, inv_h) * inv_alpha;
}
template <typename T>
void launch_irv2_image(const T* d0, const T* p, Grid g, T inv_h, T inv_alpha, T* d, hipStream_t s) {
  hipLaunchKernelGGL(k_irv2_image<T>, grid2d(g.n2, g.n1), dim3(kBX, kBY), 0, s, d0, p, g, inv_h, inv_alpha, d);
  TVS_LAUNCH_CHECK();
}

// u = (f - div p) / alpha, the primal of the ROF dual
template <typename T>
__global__ void k_primal_rof(const T* __restrict__ p, const T* __restrict__ f2, Grid g, T inv_h,
                             T inv_alpha, T* __restrict__ u) {
  const int j = blockIdx.x * kBX + threadIdx.x, i = blockIdx.y * kBY + threadIdx.y;
  if (i >= g.n2 || j >= g.n1) return;
  const long long o = (long long)i * g.n1 + j;
  u[o] = (f2[o] - div_global(p, g, i, j, inv_h)) * inv_alpha;
}
template <typename T>
void launch_primal_rof(const T* p, const T* f2, Grid g, T inv_h, T inv_alpha, T* u, hipStream_t s) {
  hipLaunchKernelGGL(k_primal_rof<T>, grid2d(g.n2, g.n1), dim3(kBX, kBY), 0, s, p, f2, g, inv_h, inv_alpha, u);
  TVS_LAUNCH_CHECK();
}

// ROF duality gap sum (|grad u| + grad u . p)
template <typename T>
__global__ __launch_bounds__(256) void k_gap_rof(const T* __restrict__ u, const T* __restrict__ p,
                                                 Grid g, T inv_h, double* __restrict__ part) {
  const long long plane = (long long)g.n2 * g.n1;
  double acc = 0.0;
  for (long long o = blockIdx.x * 256LL + threadIdx.x; o < plane; o += 256LL * gridDim.x) {
    const int i = int(o / g.n1), j = int(o - (long long)i * g.n1);
    const double gx = double(dp_global(u, g, i, j, 0, inv_h));
    const double gy = double(dp_global(u, g, i, j, 1, inv_h));
    acc += sqrt(gx * gx + gy * gy) + gx * double(p[o]) + gy * double(p[plane + o]);
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
template <typename T>
void launch_gap_rof(const T* u, const T* p, Grid g, T inv_h, Partials part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gap_rof<T>, dim3(kRedBlocks), dim3(256), 0, s, u, p, g, inv_h, part.buf);
  TVS_LAUNCH_CHECK();
  finish_sum(part, kRedBlocks, out, s);
}

// IRV1: xi = tau_perp / sqrt(|tau_perp|^2 + eps), tau_perp = R_Omega(tau_2, -tau_1)
template <typename T>
__global__ void k_xi(const T* __restrict__ tau, int N2, int N1, T eps, T* __restrict__ xi) {
  const int j = blockIdx.x * kBX + threadIdx.x, i = blockIdx.y * kBY + threadIdx.y;
  if (i >= N2 || j >= N1) return;
  const long long tp = (long long)(N2 + 1) * (N1 + 1);
  const long long to = (long long)i * (N1 + 1) + j;
  const T a = tau[tp + to], b = -tau[to];
  const T inv = T(1) / sqrt(a * a + b * b + eps);
  const long long o = (long long)i * N1 + j;
  xi[o] = a * inv;
  xi[(long long)N2 * N1 + o] = b * inv;
}
template <typename T> void launch_xi(const T* tau, int N2, int N1, T eps, T* xi, hipStream_t s) {
  hipLaunchKernelGGL(k_xi<T>, grid2d(N2, N1), dim3(kBX, kBY), 0, s, tau, N2, N1, eps, xi);
  TVS_LAUNCH_CHECK();
}
template <typename T>
__global__ void k_irv1_data(const T* __restrict__ d0, const T* __restrict__ xi, Grid g, T inv_h,
                            T alpha, T* __restrict__ f2) {
  const int j = blockIdx.x * kBX + threadIdx.x, i = blockIdx.y * kBY + threadIdx.y;
  if (i >= g.n2 || j >= g.n1) return;
  const long long o = (long long)i * g.n1 + j;
  f2[o] = alpha * d0[o] - div_global(xi, g, i, j, inv_h);
}
template <typename T>
void launch_irv1_data(const T* d0, const T* xi, Grid g, T inv_h, T alpha, T* f2, hipStream_t s) {
  hipLaunchKernelGGL(k_irv1_data<T>, grid2d(g.n2, g.n1), dim3(kBX, kBY), 0, s, d0, xi, g, inv_h, alpha, f2);
  TVS_LAUNCH_CHECK();
}
template <typename T>
__global__ void k_irv1_image(const T* __restrict__ d0, const T* __restrict__ p, const T* __restrict__ xi,
                             Grid g, T inv_h, T inv_alpha, T* __restrict__ d) {
  const int j = blockIdx.x * kBX + threadIdx.x, i = blockIdx.y * kBY + threadIdx.y;
  if (i >= g.n2 || j >= g.n1) return;
  const long long o = (long long)i * g.n1 + j;
  d[o] = d0[o] - (div_global(p, g, i, j, inv_h) + div_global(xi, g, i, j, inv_h)) * inv_alpha;
}
template <typename T>
void launch_irv1_image(const T* d0, const T* p, const T* xi, Grid g, T inv_h, T inv_alpha, T* d,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_irv1_image<T>, grid2d(g.n2, g.n1), dim3(kBX, kBY), 0, s, d0, p, xi, g, inv_h, inv_alpha, d);
  TVS_LAUNCH_CHECK();
}

#define TVS_INST(T)                                                                              \
  template void launch_fill<T>(T*, long long, T, hipStream_t);                                   \
  template void launch_scale<T>(const T*, long long, T, T*, hipStream_t);                       \
  template void launch_tau0<T>(const T*, int, int, T, T*, hipStream_t);                          \
  template void launch_global_vecdiv<T>(const T*, Grid, T, T*, hipStream_t);                    \
  template void launch_f1<T>(const T*, const T*, Grid, T, T, T*, hipStream_t);                  \
  template void launch_residual<T>(const T*, const T*, const T*, Grid, T, T*, Partials, double*, \
                                   hipStream_t);                                                 \
  template void launch_gap_tfs<T>(const T*, const T*, Grid, T, Partials, double*, hipStream_t); \
  template void launch_sub_theta_p<T>(const SubFrames&, Grid, const T*, int, T*, hipStream_t);  \
  template void launch_sub_vecdiv<T>(const SubFrames&, Grid, T, const T*, T*, hipStream_t);     \
  template void launch_sub_vecdiv_jobs<T>(const SubFrames&, Grid, T, JobRef<T>, int, hipStream_t); \
  template void launch_sub_update1_jobs<T>(const SubFrames&, Grid, StepScalars<T>, JobRef<T>, int, hipStream_t); \
  template void launch_sub2_update_jobs<T>(const SubFrames&, Grid, StepScalars<T>, JobRef<T>, int, hipStream_t); \
  template void launch_sub_omega<T>(const SubFrames&, Grid, T, const T*, const T*, const T*, T*, \
                                    hipStream_t);                                                \
  template void launch_sub_update1<T>(const SubFrames&, Grid, StepScalars<T>, const T*,         \
                                      const T*, const T*, const T*, T*, hipStream_t);            \
  template void launch_combine<T>(const SubFrames&, Grid, int, T, const T*, T*, hipStream_t);   \
  template void launch_bridge_irv2<T>(const T*, const T*, int, int, T, T, T*, hipStream_t);     \
  template void launch_sub2_prologue<T>(const SubFrames&, Grid, T, const T*, const T*, T*,      \
                                        hipStream_t);                                            \
  template void launch_sub2_update<T>(const SubFrames&, Grid, StepScalars<T>, const T*,         \
                                      const T*, T*, hipStream_t);                                \
  template void launch_energy_rof<T>(const T*, const T*, Grid, T, Partials, double*,            \
                                     hipStream_t);                                               \
  template void launch_irv2_image<T>(const T*, const T*, Grid, T, T, T*, hipStream_t);          \
  template void launch_quality_moments<T>(const T*, const T*, long long, Partials, double*,      \
                                          hipStream_t);                                          \
  template void launch_primal_rof<T>(const T*, const T*, Grid, T, T, T*, hipStream_t);          \
  template void launch_gap_rof<T>(const T*, const T*, Grid, T, Partials, double*, hipStream_t); \
  template void launch_xi<T>(const T*, int, int, T, T*, hipStream_t);                           \
  template void launch_irv1_data<T>(const T*, const T*, Grid, T, T, T*, hipStream_t);           \
  template void launch_irv1_image<T>(const T*, const T*, const T*, Grid, T, T, T*, hipStream_t);

TVS_INST(float)
TVS_INST(double)

}  // namespace tvs
