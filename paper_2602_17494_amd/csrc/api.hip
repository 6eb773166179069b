// C-ABI entry points of libtvs (include/tvs.h) and the host orchestration of
// Algorithm 2 for both TV-Stokes steps.
#include <chrono>
#include <cstdio>
#include <cstring>
#include <cstdint>
#include <vector>
#include <cmath>
#include <map>
#include <memory>
#include <atomic>
#include <mutex>
#include <string>
#include <tuple>

#include "../../include/tvs.h"
#include "blockdct.hpp"
#include "kernels.hpp"

namespace tvs {

namespace {

thread_local std::string g_last_error;

// ---------------------------------------------------------------------------
// layout (Section 6.1): core cuts floor(k n / M) of the Omega-tilde axis, and
// a stripe of width s shared by neighbours, centred on each cut
// ---------------------------------------------------------------------------
AxisLayout make_axis(int n, int m, int s, const char* name) {
  if (m < 1 || m > kMaxSub)
    throw Error(TVS_EINVAL, std::string("layout: ") + name + " must be in [1, 32]");
  if (s < 0 || (m > 1 && s < 1))
    throw Error(TVS_EINVAL, std::string("layout: overlap along ") + name + " must be >= 1");
  AxisLayout a{};
  a.n = n;
  a.m = m;
  a.s = (m > 1) ? s : 0;
  for (int k = 0; k <= m; ++k) a.cut[k] = int((long long)k * n / m);
  for (int k = 0; k < m; ++k)
    if (a.cut[k + 1] - a.cut[k] < std::max(a.s, 2))
      throw Error(TVS_EINVAL, std::string("layout: a core along ") + name + " is narrower than max(overlap, 2)");
  const int lo = a.s / 2, hi = a.s - a.s / 2;
  for (int k = 0; k < m; ++k) {
    a.start[k] = (k == 0) ? 0 : a.cut[k] - lo;
    a.end[k] = (k == m - 1) ? n : a.cut[k + 1] + hi;
  }
  return a;
}

// frame rows start on 256-byte boundaries (64 float or 32 double columns);
// pad to 64 columns for both
int align_pitch(int fp) { return fp > 64 ? (fp + 63) / 64 * 64 : fp; }

double colouring_alpha_hat(int m2, int m1) {
  if (m1 == 1 && m2 == 1) return 1.0;
  if (m1 == 1 || m2 == 1) return 0.5;
  return 0.25;
}

template <typename T> constexpr tvs_dtype dtype_of();
template <> constexpr tvs_dtype dtype_of<float>() { return TVS_F32; }
template <> constexpr tvs_dtype dtype_of<double>() { return TVS_F64; }

using GridKey = std::tuple<int, int, double>;                       // n2, n1, h
using ShapeKey = std::tuple<int, int, int, double, int, int, int, int>;  // dtype, N2, N1, h, M2, M1, sy, sx

// Workgroup shapes of a problem: the stencil run lengths of Step 1's update
// and vecdiv and of Step 2's update (1, 2 or 4 rows per thread) and the row
// pairs / columns per
// workgroup targets of the Green passes of Step 1's inner iterations
// (0 = not chosen).  Every choice computes the same values.
struct Tiles {
  int run1 = 0, run1d = 0, rows = 0, cols = 0, run2 = 0;
};
// N2, N1, h, M2, M1, sy, sx, LP kind, block groups (rows, columns) of the block-DCT plan
using ProbKey = std::tuple<int, int, double, int, int, int, int, int, int, int>;

struct SubSet {
  AxisLayout ay{}, ax{};
  std::vector<SubDesc> subs;
  DevBuf subs_d, theta_d;
  SubFrames sf{};
  double sub_px = 0;  // sum of subdomain sizes (points)
};

// theta tables of the frames: row r of subdomain row m2 is grid row
// ay.start[m2] + r (0 beyond the subdomain), and likewise for columns
void build_theta_tables(SubSet& ss, hipStream_t s) {
  const int fr = ss.sf.fr, fp = ss.sf.fp, m2 = ss.ay.m, m1 = ss.ax.m;
  const size_t ny = size_t(m2) * fr, nx = size_t(m1) * fp;
  std::vector<double> td(ny + nx);
  std::vector<float> tf(ny + nx);
  for (int a = 0; a < m2; ++a)
    for (int r = 0; r < fr; ++r) {
      td[size_t(a) * fr + r] = axis_theta<double>(ss.ay, a, ss.ay.start[a] + r);
      tf[size_t(a) * fr + r] = axis_theta<float>(ss.ay, a, ss.ay.start[a] + r);
    }
  for (int b = 0; b < m1; ++b)
    for (int q = 0; q < fp; ++q) {
      td[ny + size_t(b) * fp + q] = axis_theta<double>(ss.ax, b, ss.ax.start[b] + q);
      tf[ny + size_t(b) * fp + q] = axis_theta<float>(ss.ax, b, ss.ax.start[b] + q);
    }
  const size_t bd = td.size() * sizeof(double);
  ss.theta_d.alloc(bd + tf.size() * sizeof(float));
  char* base = static_cast<char*>(ss.theta_d.p);
  TVS_HIP(hipMemcpyAsync(base, td.data(), bd, hipMemcpyHostToDevice, s));
  TVS_HIP(hipMemcpyAsync(base + bd, tf.data(), tf.size() * sizeof(float), hipMemcpyHostToDevice, s));
  TVS_HIP(hipStreamSynchronize(s));
  ss.sf.thy_d = reinterpret_cast<const double*>(base);
  ss.sf.thx_d = ss.sf.thy_d + ny;
  ss.sf.thy_f = reinterpret_cast<const float*>(base + bd);
  ss.sf.thx_f = ss.sf.thy_f + ny;
}

// frame shape shared by all subdomains of a set (host side)
void finish_subs(SubSet& ss, int fr, int fp) {
  ss.sf.nsub = int(ss.subs.size());
  ss.sf.fr = fr;
  ss.sf.fp = align_pitch(fp);
  ss.sf.plane = (long long)fr * ss.sf.fp;
  // byte offsets inside one subdomain's four planes are 32-bit in the kernels
  if (4 * 8 * ss.sf.plane >= (1LL << 32)) throw Error(TVS_EINVAL, "layout: subdomain frame too large");
  ss.sf.ay = ss.ay;
  ss.sf.ax = ss.ax;
  ss.sf.run = 2;
  ss.sf.run_div = 2;
}

// the descriptors and theta tables on the device
void upload_subs(SubSet& ss, hipStream_t s) {
  ss.subs_d.alloc(sizeof(SubDesc) * ss.subs.size());
  TVS_HIP(hipMemcpyAsync(ss.subs_d.p, ss.subs.data(), sizeof(SubDesc) * ss.subs.size(),
                         hipMemcpyHostToDevice, s));
  ss.sf.subs = ss.subs_d.as<SubDesc>();
  build_theta_tables(ss, s);
}

// device bytes of upload_subs
size_t subs_device_bytes(const SubSet& ss) {
  const size_t ny = size_t(ss.ay.m) * ss.sf.fr, nx = size_t(ss.ax.m) * ss.sf.fp;
  return sizeof(SubDesc) * ss.subs.size() + (ny + nx) * (sizeof(double) + sizeof(float));
}

// Step 1 subdomains on Omega-tilde: s = the subdomain, a = grown by one
// row/column, b = grown by two (clipped at the grid)
void plan_subs1(SubSet& ss, int n2, int n1) {
  ss.subs.clear();
  ss.sub_px = 0;
  int fr = 0, fp = 0;
  for (int a = 0; a < ss.ay.m; ++a)
    for (int b = 0; b < ss.ax.m; ++b) {
      SubDesc d{};
      d.i0 = ss.ay.start[a];
      d.j0 = ss.ax.start[b];
      d.si = ss.ay.end[a] - d.i0;
      d.sj = ss.ax.end[b] - d.j0;
      d.ai = std::min(d.si + 1, n2 - d.i0);
      d.aj = std::min(d.sj + 1, n1 - d.j0);
      d.bi = std::min(d.si + 2, n2 - d.i0);
      d.bj = std::min(d.sj + 2, n1 - d.j0);
      d.m2 = a;
      d.m1 = b;
      fr = std::max(fr, d.bi);
      fp = std::max(fp, d.bj);
      ss.sub_px += double(d.si) * d.sj;
      ss.subs.push_back(d);
    }
  finish_subs(ss, fr, fp);
}

// Step 2 subdomains: the Step-1 ones cut to Omega; a = grown by one
void plan_subs2(SubSet& ss, int N2, int N1) {
  ss.subs.clear();
  ss.sub_px = 0;
  int fr = 0, fp = 0;
  for (int a = 0; a < ss.ay.m; ++a)
    for (int b = 0; b < ss.ax.m; ++b) {
      SubDesc d{};
      d.i0 = ss.ay.start[a];
      d.j0 = ss.ax.start[b];
      d.si = std::min(ss.ay.end[a], N2) - d.i0;
      d.sj = std::min(ss.ax.end[b], N1) - d.j0;
      if (d.si < 1 || d.sj < 1) throw Error(TVS_EINVAL, "layout: a subdomain misses the image");
      d.ai = std::min(d.si + 1, N2 - d.i0);
      d.aj = std::min(d.sj + 1, N1 - d.j0);
      d.bi = d.ai;
      d.bj = d.aj;
      d.m2 = a;
      d.m1 = b;
      fr = std::max(fr, d.ai);
      fp = std::max(fp, d.aj);
      ss.sub_px += double(d.si) * d.sj;
      ss.subs.push_back(d);
    }
  finish_subs(ss, fr, fp);
}

void build_subs1(SubSet& ss, int n2, int n1, hipStream_t s) {
  plan_subs1(ss, n2, n1);
  upload_subs(ss, s);
}
void build_subs2(SubSet& ss, int N2, int N1, hipStream_t s) {
  plan_subs2(ss, N2, N1);
  upload_subs(ss, s);
}

template <typename T>
struct Step1Problem {
  Grid g{};
  SubSet ss;
  bool plain = false;
  std::unique_ptr<GreenPlan<T>> global, local;
  std::unique_ptr<BlockDctPlan<T>> bdct;    // LP_m by the block-DCT formula instead of `local`
  DevBuf tau0, f1, r, zg, phig, p;         // global arrays on Omega-tilde
  DevBuf va, vb, vt, za, zb, zw, phi, omega;  // per-subdomain frames
  size_t bytes() const {
    size_t b = tau0.bytes + f1.bytes + r.bytes + zg.bytes + phig.bytes + p.bytes + va.bytes +
               vb.bytes + vt.bytes + za.bytes + zb.bytes + zw.bytes + phi.bytes + omega.bytes +
               global->bytes() + ss.subs_d.bytes + ss.theta_d.bytes;
    if (local) b += local->bytes();
    if (bdct) b += bdct->bytes();
    return b;
  }
};

template <typename T>
struct Step2Problem {
  Grid g{};
  SubSet ss;
  DevBuf f2, p, u, xi, va, vb, b;
  size_t bytes() const {
    return f2.bytes + p.bytes + u.bytes + xi.bytes + va.bytes + vb.bytes + b.bytes + ss.subs_d.bytes +
           ss.theta_d.bytes;
  }
};

}  // namespace
}  // namespace tvs

struct tvs_ctx {
  int device = 0;
  std::map<tvs::GridKey, std::unique_ptr<tvs::GreenTable>> tables;
  std::map<tvs::ProbKey, std::unique_ptr<tvs::Step1Problem<float>>> s1f;
  std::map<tvs::ProbKey, std::unique_ptr<tvs::Step1Problem<double>>> s1d;
  std::map<tvs::ProbKey, std::unique_ptr<tvs::Step2Problem<float>>> s2f;
  std::map<tvs::ProbKey, std::unique_ptr<tvs::Step2Problem<double>>> s2d;
  std::map<tvs::GridKey, std::unique_ptr<tvs::GreenPlan<float>>> projf;
  std::map<tvs::GridKey, std::unique_ptr<tvs::GreenPlan<double>>> projd;
  std::map<tvs::GridKey, std::unique_ptr<tvs::DevBuf>> projtmp;
  tvs::KernelTimer timer;
  int lp_kind = TVS_LP_IMAGE;  // realisation of LP_m for the one-shot Step-1 calls
  int bd_g2 = 0, bd_g1 = 0;    // frequency blocks per group of the block-DCT plans (0: automatic)
  tvs::Tiles force;            // tvs_set_tiles: fields > 0 override the tuner
  std::map<tvs::ShapeKey, tvs::Tiles> tuned;  // the tuner's choices per problem shape
  std::vector<double> history;  // energies per sweep of the last one-shot step with statistics
  tvs::DevBuf partials;  // FP64 partial sums
  tvs::DevBuf scal;      // FP64 results (energies per sweep, gap)
  size_t scal_cap = 0;
  // streams a batch call spreads independent jobs over (default priority),
  // with the events that fork them from and join them to the caller's stream
  // the stream a batch call runs its work on (default priority), forked
  // from and joined to the caller's stream, which may be the legacy default
  // stream (not capturable)
  hipStream_t bstream = nullptr;
  hipEvent_t bfork = nullptr, bjoin = nullptr;
  // JobBufs tables of the last batch call, and its sweep bodies recorded as
  // one graph, with the key (job uid, step, ping-pong state, per job) it was
  // recorded for
  tvs::DevBuf jobtab;
  std::vector<unsigned long long> bkey;
  hipGraphExec_t bgraph = nullptr;
  ~tvs_ctx() {
    if (bgraph) (void)hipGraphExecDestroy(bgraph);
    if (bstream) (void)hipStreamDestroy(bstream);
    if (bjoin) (void)hipEventDestroy(bjoin);
    if (bfork) (void)hipEventDestroy(bfork);
  }
};

namespace tvs {
namespace {

template <typename T> auto& s1map(tvs_ctx* c);
template <> auto& s1map<float>(tvs_ctx* c) { return c->s1f; }
template <> auto& s1map<double>(tvs_ctx* c) { return c->s1d; }
template <typename T> auto& s2map(tvs_ctx* c);
template <> auto& s2map<float>(tvs_ctx* c) { return c->s2f; }
template <> auto& s2map<double>(tvs_ctx* c) { return c->s2d; }
template <typename T> auto& projmap(tvs_ctx* c);
template <> auto& projmap<float>(tvs_ctx* c) { return c->projf; }
template <> auto& projmap<double>(tvs_ctx* c) { return c->projd; }

GreenTable& get_table(tvs_ctx* c, int n2, int n1, double h, hipStream_t s) {
  auto key = GridKey{n2, n1, h};
  auto it = c->tables.find(key);
  if (it != c->tables.end()) return *it->second;
  auto t = std::make_unique<GreenTable>(n2, n1, h, s);
  auto& ref = *t;
  c->tables[key] = std::move(t);
  return ref;
}

double* scal(tvs_ctx* c, size_t n) {
  if (c->scal_cap < n) {
    // earlier calls may still be reading the old buffer on some stream
    TVS_HIP(hipDeviceSynchronize());
    const size_t cap = std::max<size_t>(n, 4096);
    c->scal.alloc(sizeof(double) * cap);
    c->scal_cap = cap;
  }
  return c->scal.as<double>();
}

Partials partials(tvs_ctx* c) {
  if (!c->partials.p) c->partials.alloc(sizeof(double) * 1024);
  return Partials{c->partials.as<double>(), 1024};
}

// the inverse Laplacian of a grid of n2 x n1 points (Step 1 runs it on
// Omega-tilde, (N2+1) x (N1+1)) needs transforms of about twice each side
void check_grid_sides(int n2, int n1) {
  if (!green_side_ok(n2) || !green_side_ok(n1))
    throw Error(TVS_EINVAL, "grid of " + std::to_string(n2) + " x " + std::to_string(n1) +
                                " points: sides above " + std::to_string(kGreenMaxSide) +
                                " points are not supported (the transforms of the inverse Laplacian "
                                "would exceed the LDS)");
}

void check_shape(int N2, int N1) {
  if (N2 < 2 || N1 < 2) throw Error(TVS_EINVAL, "image must be at least 2 x 2");
  if ((long long)(N2 + 1) * (N1 + 1) > (1LL << 28)) throw Error(TVS_EINVAL, "image too large");
  check_grid_sides(N2 + 1, N1 + 1);
}

void check_params(const tvs_params* prm, int N2, int N1) {
  if (!prm) throw Error(TVS_EINVAL, "params is NULL");
  check_shape(N2, N1);
  if (!(prm->delta > 0) || !(prm->alpha > 0)) throw Error(TVS_EINVAL, "delta and alpha must be > 0");
  if (!(prm->t > 0) || prm->t > 0.125) throw Error(TVS_EINVAL, "t must lie in (0, 1/8]");
  if (!(prm->h > 0)) throw Error(TVS_EINVAL, "h must be > 0");
  if (prm->variant != TVS_IRV2 && prm->variant != TVS_IRV1) throw Error(TVS_EINVAL, "unknown variant");
  if (prm->variant == TVS_IRV1 && !(prm->eps > 0)) throw Error(TVS_EINVAL, "IRV1 needs eps > 0");
}

void check_iters(const tvs_iters* it) {
  if (!it) throw Error(TVS_EINVAL, "iters is NULL");
  if (it->sweeps < 1 || it->inner < 1) throw Error(TVS_EINVAL, "sweeps and inner must be >= 1");
  if (!(it->tol >= 0)) throw Error(TVS_EINVAL, "tol must be >= 0");
}

double alpha_hat_of(const tvs_layout* l) {
  if (l->alpha_hat <= 0) return colouring_alpha_hat(l->M2, l->M1);
  if (l->alpha_hat > 1) throw Error(TVS_EINVAL, "alpha_hat must lie in (0, 1]");
  return l->alpha_hat;
}

// cache_table = false (jobs): the grid's Green-function table is only needed
// while the plans are built; use the context's if it has one, else build a
// transient one, so that jobs of many grid sizes do not grow the context
template <typename T>
std::unique_ptr<Step1Problem<T>> make_step1(tvs_ctx* c, int N2, int N1, double h, const tvs_layout* l,
                                            hipStream_t s, int lp_kind = TVS_LP_IMAGE, bool cache_table = true) {
  if (!l) throw Error(TVS_EINVAL, "layout is NULL");
  auto P = std::make_unique<Step1Problem<T>>();
  const int n2 = N2 + 1, n1 = N1 + 1;
  P->g = Grid{n2, n1, h};
  P->ss.ay = make_axis(n2, l->M2, l->s_y, "M2");
  P->ss.ax = make_axis(n1, l->M1, l->s_x, "M1");
  build_subs1(P->ss, n2, n1, s);
  P->plain = (l->M2 == 1 && l->M1 == 1);
  std::unique_ptr<GreenTable> own;
  const GreenTable* tp = nullptr;
  if (cache_table) {
    tp = &get_table(c, n2, n1, h, s);
  } else {
    auto it = c->tables.find(GridKey{n2, n1, h});
    if (it != c->tables.end()) {
      tp = it->second.get();
    } else {
      own = std::make_unique<GreenTable>(n2, n1, h, s);
      tp = own.get();
    }
  }
  const GreenTable& tab = *tp;
  P->global = std::make_unique<GreenPlan<T>>(tab, std::vector<std::array<int, 4>>{{0, 0, n2, n1}}, s);
  if (!P->plain) {
    std::vector<std::array<int, 4>> boxes;
    for (auto& d : P->ss.subs) boxes.push_back({d.i0, d.j0, d.bi, d.bj});
    if (lp_kind == TVS_LP_BLOCKDCT)
      P->bdct = std::make_unique<BlockDctPlan<T>>(n2, n1, h, boxes, s, c->bd_g2, c->bd_g1);
    else
      P->local = std::make_unique<GreenPlan<T>>(tab, boxes, s);
  }
  const size_t gp = size_t(n2) * n1 * sizeof(T);
  P->tau0.alloc(2 * gp);
  P->f1.alloc(2 * gp);
  P->r.alloc(2 * gp);
  P->zg.alloc(2 * gp);
  P->phig.alloc(gp);
  P->p.alloc(4 * gp);
  const size_t fpb = size_t(P->ss.sf.plane) * P->ss.sf.nsub * sizeof(T);
  P->va.alloc(4 * fpb);
  P->vb.alloc(4 * fpb);
  P->omega.alloc(2 * fpb);
  if (!P->plain) {
    P->vt.alloc(4 * fpb);
    P->zw.alloc(2 * fpb);
  }
  P->za.alloc(2 * fpb);
  P->zb.alloc(2 * fpb);
  P->phi.alloc(fpb);
  return P;
}

template <typename T>
std::unique_ptr<Step2Problem<T>> make_step2(int N2, int N1, double h, const tvs_layout* l, hipStream_t s) {
  if (!l) throw Error(TVS_EINVAL, "layout is NULL");
  auto P = std::make_unique<Step2Problem<T>>();
  P->g = Grid{N2, N1, h};
  P->ss.ay = make_axis(N2 + 1, l->M2, l->s_y, "M2");
  P->ss.ax = make_axis(N1 + 1, l->M1, l->s_x, "M1");
  build_subs2(P->ss, N2, N1, s);
  const size_t gp = size_t(N2) * N1 * sizeof(T);
  P->f2.alloc(gp);
  P->p.alloc(2 * gp);
  P->u.alloc(gp);
  P->xi.alloc(2 * gp);
  const size_t fpb = size_t(P->ss.sf.plane) * P->ss.sf.nsub * sizeof(T);
  P->va.alloc(2 * fpb);
  P->vb.alloc(2 * fpb);
  P->b.alloc(fpb);
  return P;
}

ShapeKey shape_key(int kind, int N2, int N1, double h, const tvs_layout* l);
template <typename T>
void apply_tiles1(tvs_ctx* c, Step1Problem<T>& P, const ShapeKey& key, hipStream_t s, bool tune = true);
template <typename T>
void apply_tiles2(tvs_ctx* c, Step2Problem<T>& P, const ShapeKey& key, hipStream_t s, bool tune = true);

// problems cached in the context by shape (the one-shot calls)
template <typename T>
Step1Problem<T>& get_step1(tvs_ctx* c, int N2, int N1, double h, const tvs_layout* l, hipStream_t s) {
  if (!l) throw Error(TVS_EINVAL, "layout is NULL");
  const bool bd = c->lp_kind == TVS_LP_BLOCKDCT;
  auto key = ProbKey{N2, N1, h, l->M2, l->M1, l->s_y, l->s_x, c->lp_kind, bd ? c->bd_g2 : 0, bd ? c->bd_g1 : 0};
  auto& mp = s1map<T>(c);
  auto it = mp.find(key);
  Step1Problem<T>& ref = it != mp.end() ? *it->second : *(mp[key] = make_step1<T>(c, N2, N1, h, l, s, c->lp_kind));
  apply_tiles1<T>(c, ref, shape_key(int(dtype_of<T>()) + 2 * c->lp_kind, N2, N1, h, l), s);
  return ref;
}

template <typename T>
Step2Problem<T>& get_step2(tvs_ctx* c, int N2, int N1, double h, const tvs_layout* l, hipStream_t s) {
  if (!l) throw Error(TVS_EINVAL, "layout is NULL");
  auto key = ProbKey{N2, N1, h, l->M2, l->M1, l->s_y, l->s_x, 0, 0, 0};
  auto& mp = s2map<T>(c);
  auto it = mp.find(key);
  Step2Problem<T>& ref = it != mp.end() ? *it->second : *(mp[key] = make_step2<T>(N2, N1, h, l, s));
  apply_tiles2<T>(c, ref, shape_key(int(dtype_of<T>()), N2, N1, h, l), s);
  return ref;
}

Frame global_frame(const Grid& g) { return Frame{0, (long long)g.n2 * g.n1, g.n1}; }
Frame sub_frame(const SubFrames& sf, int planes) { return Frame{planes * sf.plane, sf.plane, sf.fp}; }

// ---------------------------------------------------------------------------
// Tuner: the workgroup shapes of a problem, chosen by timing the candidates
// on the problem's own buffers (zero-filled, before the solve sets them up)
// the first time a problem shape is built in a context.  The choices are
// cached per shape; tvs_set_tiles can force them instead.
// ---------------------------------------------------------------------------
constexpr int kTuneReps = 8;     // launches per measurement
constexpr int kTuneTrials = 3;   // measurements per candidate (the fastest counts)
constexpr float kTuneGain = 0.97f;  // a candidate must beat the current choice by 3 %
template <typename F>
float time_launches(hipStream_t s, int reps, F&& f);
// the fastest of kTuneTrials measurements of kTuneReps launches
template <typename F>
float time_best(hipStream_t s, F&& f) {
  float best = 0;
  for (int k = 0; k < kTuneTrials; ++k) {
    const float ms = time_launches(s, kTuneReps, f);
    if (k == 0 || ms < best) best = ms;
  }
  return best;
}
template <typename F>
float time_launches(hipStream_t s, int reps, F&& f) {
  hipEvent_t a = nullptr, b = nullptr;
  TVS_HIP(hipEventCreate(&a));
  TVS_HIP(hipEventCreate(&b));
  float ms = 0;
  try {
    f();  // warm-up
    TVS_HIP(hipEventRecord(a, s));
    for (int k = 0; k < reps; ++k) f();
    TVS_HIP(hipEventRecord(b, s));
    TVS_HIP(hipEventSynchronize(b));
    TVS_HIP(hipEventElapsedTime(&ms, a, b));
  } catch (...) {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    throw;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

constexpr int kTuneRuns[3] = {1, 2, 4};
constexpr int kTuneRows[4] = {2, 4, 8, 16};
constexpr int kTuneCols[4] = {1, 2, 3, 4};

template <typename T>
Tiles tune_step1(Step1Problem<T>& P, hipStream_t s) {
  Tiles t{};
  SubFrames& sf = P.ss.sf;
  const Grid g = P.g;
  const StepScalars<T> cs{T(0.125), T(1.0 / g.h), T(1), T(1), T(1)};
  const long long fpl = sf.plane * sf.nsub;
  launch_fill<T>(dptr<T>(P.va), 4 * fpl, T(0), s);
  launch_fill<T>(dptr<T>(P.vb), 4 * fpl, T(0), s);
  launch_fill<T>(dptr<T>(P.za), 2 * fpl, T(0), s);
  launch_fill<T>(dptr<T>(P.zb), 2 * fpl, T(0), s);
  launch_fill<T>(dptr<T>(P.phi), fpl, T(0), s);
  launch_fill<T>(dptr<T>(P.omega), 2 * fpl, T(0), s);
  // each stencil kernel from the default run length 2, which a candidate
  // must beat
  auto pick_run = [&](int& field, auto&& launch) {
    field = 2;
    float b = time_best(s, launch);
    int r = 2;
    for (int run : kTuneRuns) {
      if (run == 2) continue;
      field = run;
      const float ms = time_best(s, launch);
      if (ms < kTuneGain * b) {
        b = ms;
        r = run;
      }
    }
    field = r;
    return r;
  };
  t.run1 = pick_run(sf.run, [&] {
    launch_sub_update1<T>(sf, g, cs, dptr<T>(P.va), dptr<T>(P.za), dptr<T>(P.phi), dptr<T>(P.omega),
                          dptr<T>(P.vb), s);
  });
  t.run1d = pick_run(sf.run_div, [&] { launch_sub_vecdiv<T>(sf, g, cs.inv_h, dptr<T>(P.vb), dptr<T>(P.zb), s); });
  float best = 0;
  if (!P.bdct) {
    GreenPlan<T>& gp = P.plain ? *P.global : *P.local;
    const Frame f2p = sub_frame(sf, 2), f1p = sub_frame(sf, 1);
    auto apply = [&] { gp.apply_div(dptr<T>(P.za), f2p, dptr<T>(P.phi), f1p, s); };
    const int cols0 = gp.tile_cols();
    t.rows = gp.tile_rows();
    t.cols = cols0;
    best = time_best(s, apply);
    const int rows0 = t.rows;
    for (int rows : kTuneRows) {
      if (rows == rows0 || !gp.try_tiles(rows, cols0)) continue;
      const float ms = time_best(s, apply);
      if (ms < kTuneGain * best) {
        best = ms;
        t.rows = rows;
      }
      gp.set_tiles(rows0, cols0);
    }
    for (int cols : kTuneCols) {
      if (cols == cols0 || !gp.try_tiles(t.rows, cols)) continue;
      const float ms = time_best(s, apply);
      if (ms < kTuneGain * best) {
        best = ms;
        t.cols = cols;
      }
      gp.set_tiles(t.rows, cols0);
    }
    gp.set_tiles(t.rows, t.cols);
  }
  return t;
}

template <typename T>
int tune_step2(Step2Problem<T>& P, hipStream_t s) {
  SubFrames& sf = P.ss.sf;
  const StepScalars<T> cs{T(0.125), T(1.0 / P.g.h), T(1), T(1), T(1)};
  const long long fpl = sf.plane * sf.nsub;
  launch_fill<T>(dptr<T>(P.va), 2 * fpl, T(0), s);
  launch_fill<T>(dptr<T>(P.b), fpl, T(0), s);
  auto upd = [&] { launch_sub2_update<T>(sf, P.g, cs, dptr<T>(P.va), dptr<T>(P.b), dptr<T>(P.vb), s); };
  int pick = 2;
  sf.run = 2;
  float best = time_best(s, upd);
  for (int run : kTuneRuns) {
    if (run == 2) continue;
    sf.run = run;
    const float ms = time_best(s, upd);
    if (ms < kTuneGain * best) {
      best = ms;
      pick = run;
    }
  }
  sf.run = pick;
  return pick;
}

// kind: the dtype, plus 2 for a Step-1 problem with the block-DCT LP_m
ShapeKey shape_key(int kind, int N2, int N1, double h, const tvs_layout* l) {
  return ShapeKey{kind, N2, N1, h, l->M2, l->M1, l->s_y, l->s_x};
}

// The workgroup shapes of a Step-1 problem: forced, cached for its shape, or
// tuned now (and cached).  With tune = false (jobs) nothing is timed: a shape
// neither forced nor tuned before keeps the plan's defaults, which are tiles
// of the same kernel path, so the results are the same bit for bit.
template <typename T>
void apply_tiles1(tvs_ctx* c, Step1Problem<T>& P, const ShapeKey& key, hipStream_t s, bool tune) {
  const Tiles& f = c->force;
  const bool forced = f.run1 > 0 && f.run1d > 0 && (P.bdct || (f.rows > 0 && f.cols > 0));
  Tiles cached{};
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) cached = it->second;
  if (cached.run1 == 0 && !forced && tune) {
    const Tiles t = tune_step1<T>(P, s);
    Tiles& entry = c->tuned[key];
    entry.run1 = t.run1;
    entry.run1d = t.run1d;
    entry.rows = t.rows;
    entry.cols = t.cols;
    cached = entry;
  }
  if (f.run1 > 0 || cached.run1 > 0) P.ss.sf.run = f.run1 > 0 ? f.run1 : cached.run1;
  if (f.run1d > 0 || cached.run1d > 0) P.ss.sf.run_div = f.run1d > 0 ? f.run1d : cached.run1d;
  if (!P.bdct) {
    GreenPlan<T>& gp = P.plain ? *P.global : *P.local;
    const int rows = f.rows > 0 ? f.rows : cached.rows, cols = f.cols > 0 ? f.cols : cached.cols;
    if (rows > 0 && cols > 0 && (rows != gp.tile_rows() || cols != gp.tile_cols())) gp.try_tiles(rows, cols);
  }
}
template <typename T>
void apply_tiles2(tvs_ctx* c, Step2Problem<T>& P, const ShapeKey& key, hipStream_t s, bool tune) {
  int run2 = 0;
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) run2 = it->second.run2;
  if (run2 == 0 && c->force.run2 <= 0 && tune) run2 = c->tuned[key].run2 = tune_step2<T>(P, s);
  if (c->force.run2 > 0 || run2 > 0) P.ss.sf.run = c->force.run2 > 0 ? c->force.run2 : run2;
}

struct Host64 {
  std::vector<double> v;
};

double residual_of(double e0, double e1, double scale) {
  return std::fabs(std::sqrt(std::max(e0, 0.0)) - std::sqrt(std::max(e1, 0.0))) / scale;
}

double read1(const double* d, hipStream_t s) {
  double h = 0;
  TVS_HIP(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, s));
  TVS_HIP(hipStreamSynchronize(s));
  return h;
}

// ---------------------------------------------------------------------------
// Step 1: Algorithm 2 on Omega-tilde with the inner loop of Algorithm 5, as a
// resumable run: begin() (a1), sweep() (a2-a4: one Schwarz sweep), end() (a5
// and the statistics).  run_step1 chains them; a job calls sweep() once per
// batch sweep.  e holds the FP64 energy of every sweep, then the gap.
// ---------------------------------------------------------------------------
template <typename T>
struct Step1Run {
  Step1Problem<T>* P = nullptr;
  const T* d0 = nullptr;
  int N2 = 0, N1 = 0;
  tvs_params prm{};
  tvs_iters its{};
  StepScalars<T> cs{};
  Partials part{};
  double* e = nullptr;
  KernelTimer* tm = nullptr;
  T *cur = nullptr, *nxt = nullptr, *zcur = nullptr, *znxt = nullptr;
  int n = 0, done = 0;
  bool finished = false;
  std::vector<double>* hist = nullptr;  // receives D(p^0..p^done) when end() computes statistics

  Step1Run(Step1Problem<T>& prob, const T* d0_, int N2_, int N1_, const tvs_params* p, const tvs_layout* l,
           const tvs_iters* it, Partials pt, double* e_, KernelTimer* t)
      : P(&prob), d0(d0_), N2(N2_), N1(N1_), prm(*p), its(*it), part(pt), e(e_), tm(t) {
    const T inv_h = T(1.0 / prm.h);
    cs = StepScalars<T>{T(prm.t), inv_h, T(prm.delta), T(prm.alpha), T(alpha_hat_of(l))};
  }
  // phi = R_B Delta^dagger div u on every Green box (LP_m's inverse Laplacian)
  void local_apply(const T* u, const Frame& uf, T* phi, const Frame& pf, hipStream_t s, const char* tag) {
    if (P->bdct)
      P->bdct->apply_div(u, uf, phi, pf, s, tm, "s1_bdct");
    else
      (P->plain ? *P->global : *P->local).apply_div(u, uf, phi, pf, s, tm, tag);
  }
  double scale() const { return std::sqrt(2.0 * double(P->g.n2) * P->g.n1); }

  void begin(hipStream_t s) {
    const Grid g = P->g;
    const SubFrames& sf = P->ss.sf;
    const long long gpl = (long long)g.n2 * g.n1;
    // a1: tau_0 and f = delta^{-1} P_K tau_0
    launch_tau0<T>(d0, N2, N1, cs.inv_h, dptr<T>(P->tau0), s);
    P->global->apply_div(dptr<T>(P->tau0), global_frame(g), dptr<T>(P->phig), Frame{0, 0, g.n1}, s);
    launch_f1<T>(dptr<T>(P->tau0), dptr<T>(P->phig), g, cs.inv_h, T(1.0 / prm.delta), dptr<T>(P->f1), s);
    launch_fill<T>(dptr<T>(P->p), 4 * gpl, T(0), s);
    launch_fill<T>(dptr<T>(P->va), 4 * sf.plane * sf.nsub, T(0), s);
    launch_fill<T>(dptr<T>(P->vb), 4 * sf.plane * sf.nsub, T(0), s);
    // in the single-domain case omega = f (theta = 1), staged into the frame layout
    if (P->plain) launch_sub_theta_p<T>(sf, g, dptr<T>(P->f1), 2, dptr<T>(P->omega), s);
    cur = dptr<T>(P->va);
    nxt = dptr<T>(P->vb);
    zcur = dptr<T>(P->za);  // vecdiv of cur (0 for v = 0)
    znxt = dptr<T>(P->zb);
    // z frames are written on the grown subdomains only; 0 elsewhere
    launch_fill<T>(zcur, 2 * sf.plane * sf.nsub, T(0), s);
    launch_fill<T>(znxt, 2 * sf.plane * sf.nsub, T(0), s);
    if (!P->plain) launch_fill<T>(dptr<T>(P->zw), 2 * sf.plane * sf.nsub, T(0), s);  // no zw when plain
    n = done = 0;
    finished = false;
  }

  // One sweep; false once the run has no sweep left (count reached, or the
  // stopping residual fell below the tolerance, which reads it back).
  bool sweep(hipStream_t s) {
    if (!head(s)) return false;
    body(s, true);
    return !finished;
  }

  // a2 and the stopping test: the part of a sweep that depends on its index
  // (the FP64 energy lands in e[n]); false when the run stops here.
  bool head(hipStream_t s) {
    if (finished) return false;
    const Grid g = P->g;
    const T inv_h = cs.inv_h;
    // a2: r^n = f - P_K vecdiv p^n (global, once per sweep) and D(p^n)
    launch_global_vecdiv<T>(dptr<T>(P->p), g, inv_h, dptr<T>(P->zg), s);
    P->global->apply_div(dptr<T>(P->zg), global_frame(g), dptr<T>(P->phig), Frame{0, 0, g.n1}, s, tm,
                         "s1_global");
    launch_residual<T>(dptr<T>(P->f1), dptr<T>(P->zg), dptr<T>(P->phig), g, inv_h, dptr<T>(P->r), part, e + n, s);
    if (its.tol > 0 && n >= 1) {
      double hv[2];
      TVS_HIP(hipMemcpyAsync(hv, e + n - 1, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      TVS_HIP(hipStreamSynchronize(s));
      if (residual_of(hv[0], hv[1], scale()) < its.tol) {
        finished = true;
        return false;
      }
    }
    return true;
  }

  // the rest of the sweep (a2's omega prologue, a3, a4): the same launches
  // in every sweep, up to the exchange of the ping-pong buffers, so that a
  // caller may record them once in a graph and replay it; with launch =
  // false only the host-side state advances (the graph did the work).
  void body(hipStream_t s, bool launch) {
    if (launch) {
      prologue(s);
      for (int nu = 0; nu < its.inner; ++nu) {
        inner(s);
        std::swap(cur, nxt);
        std::swap(zcur, znxt);
      }
      combine(s);
    } else {
      for (int nu = 0; nu < its.inner; ++nu) {
        std::swap(cur, nxt);
        std::swap(zcur, znxt);
      }
    }
    ++done;
    ++n;
    if (n >= its.sweeps) finished = true;
  }
  // a2's subdomain part: omega_m = R_{m,+} r^n + LP_m(vecdiv(theta_m p^n))
  void prologue(hipStream_t s) {
    if (P->plain) return;
    const Grid g = P->g;
    const SubFrames& sf = P->ss.sf;
    const T inv_h = cs.inv_h;
    const Frame f2p = sub_frame(sf, 2), f1p = sub_frame(sf, 1);
    launch_sub_theta_p<T>(sf, g, dptr<T>(P->p), 4, dptr<T>(P->vt), s);
    launch_sub_vecdiv<T>(sf, g, inv_h, dptr<T>(P->vt), dptr<T>(P->zw), s);
    local_apply(dptr<T>(P->zw), f2p, dptr<T>(P->phi), f1p, s, "s1_local");
    launch_sub_omega<T>(sf, g, inv_h, dptr<T>(P->r), dptr<T>(P->zw), dptr<T>(P->phi), dptr<T>(P->omega), s);
  }
  // a3: one inner iteration, warm-started from the previous sweep's q_m:
  // phi = Delta^+ div z on the Green box, the update of v, z' = vecdiv v'
  void inner(hipStream_t s) {
    const Grid g = P->g;
    const SubFrames& sf = P->ss.sf;
    const Frame f2p = sub_frame(sf, 2), f1p = sub_frame(sf, 1);
    const double px = P->ss.sub_px, esz = sizeof(T);
    local_apply(zcur, f2p, dptr<T>(P->phi), f1p, s, P->plain ? "s1_plain" : "s1_local");
    KernelTimer::time(tm, "s1_update", 13 * esz * px, s, [&] {
      launch_sub_update1<T>(sf, g, cs, cur, zcur, dptr<T>(P->phi), dptr<T>(P->omega), nxt, s);
    });
    KernelTimer::time(tm, "s1_vecdiv", 6 * esz * px, s,
                      [&] { launch_sub_vecdiv<T>(sf, g, cs.inv_h, nxt, znxt, s); });
  }
  // a4: p^{n+1} = (1 - ahat) p^n + ahat sum_m q_m, with q_m the state the
  // inner iterations ended in (`ahead` iterations after `cur`)
  void combine(hipStream_t s, int ahead = 0) {
    const Grid g = P->g;
    const SubFrames& sf = P->ss.sf;
    const long long gpl = (long long)g.n2 * g.n1;
    const double px = P->ss.sub_px, esz = sizeof(T);
    const T* q = (ahead & 1) ? nxt : cur;
    KernelTimer::time(tm, "s1_combine", 4 * esz * (2.0 * gpl + px), s,
                      [&] { launch_combine<T>(sf, g, 4, cs.ahat, q, dptr<T>(P->p), s); });
  }
  // the Green plan of the inner iterations
  GreenPlan<T>& inner_plan() const { return P->plain ? *P->global : *P->local; }
  // this run's buffers for a batched inner iteration
  JobBufs<T> bufs() const {
    GreenPlan<T>& gp = inner_plan();
    return JobBufs<T>{{dptr<T>(P->va), dptr<T>(P->vb)}, {dptr<T>(P->za), dptr<T>(P->zb)}, dptr<T>(P->phi),
                      dptr<T>(P->omega), gp.S_ptr(), gp.spec_ptr(), parity(), 0};
  }
  // which of the two ping-pong states the next body starts from
  int parity() const { return cur == dptr<T>(P->va) ? 0 : 1; }

  void end(T* tau_out, tvs_stats* st, hipStream_t s) {
    const Grid g = P->g;
    const T inv_h = cs.inv_h;
    const Frame gf = global_frame(g);
    const long long gpl = (long long)g.n2 * g.n1;
    // a5: tau = delta (f - P_K vecdiv p), D(p^S) and the gap
    launch_global_vecdiv<T>(dptr<T>(P->p), g, inv_h, dptr<T>(P->zg), s);
    P->global->apply_div(dptr<T>(P->zg), gf, dptr<T>(P->phig), Frame{0, 0, g.n1}, s);
    launch_residual<T>(dptr<T>(P->f1), dptr<T>(P->zg), dptr<T>(P->phig), g, inv_h, dptr<T>(P->r), part, e + done, s);
    launch_scale<T>(dptr<T>(P->r), 2 * gpl, T(prm.delta), tau_out, s);
    // tau already lies in K; projecting it once more is the identity in exact
    // arithmetic and removes the small divergence left by rounding, which the
    // IRV2 row integral of tau_2 would otherwise accumulate across the image
    P->global->apply_div(tau_out, gf, dptr<T>(P->phig), Frame{0, 0, g.n1}, s, tm, "s1_global");
    launch_f1<T>(tau_out, dptr<T>(P->phig), g, inv_h, T(1), tau_out, s);
    if (st) {
      launch_gap_tfs<T>(tau_out, dptr<T>(P->p), g, inv_h, part, e + its.sweeps + 1, s);
      std::vector<double> hv(size_t(its.sweeps) + 2);
      TVS_HIP(hipMemcpyAsync(hv.data(), e, sizeof(double) * hv.size(), hipMemcpyDeviceToHost, s));
      TVS_HIP(hipStreamSynchronize(s));
      st->sweeps_done = done;
      st->energy = hv[done];
      st->residual = done >= 1 ? residual_of(hv[done - 1], hv[done], scale()) : 0.0;
      st->gap = hv[its.sweeps + 1];
      if (!std::isfinite(st->energy) || !std::isfinite(st->gap))
        throw Error(TVS_ENONFINITE, "step 1: non-finite energy or gap");
      if (hist) hist->assign(hv.begin(), hv.begin() + done + 1);
    }
  }
};

template <typename T>
void run_step1(tvs_ctx* c, const T* d0, int N2, int N1, const tvs_params* prm, const tvs_layout* l,
               const tvs_iters* its, T* tau_out, tvs_stats* st, hipStream_t s) {
  Step1Problem<T>& P = get_step1<T>(c, N2, N1, prm->h, l, s);
  Step1Run<T> run(P, d0, N2, N1, prm, l, its, partials(c), scal(c, size_t(its->sweeps) + 3), &c->timer);
  c->history.clear();
  run.hist = &c->history;
  run.begin(s);
  while (run.sweep(s)) {
  }
  run.end(tau_out, st, s);
}

// ---------------------------------------------------------------------------
// Step 2: Algorithm 2 on Omega with the inner loop of Algorithm 3, resumable
// in the same way: begin() (a6 and the set-up), sweep() (a7-a9), end() (the
// image and the statistics).
// ---------------------------------------------------------------------------
template <typename T>
struct Step2Run {
  Step2Problem<T>* P = nullptr;
  const T* d0 = nullptr;
  int N2 = 0, N1 = 0;
  tvs_params prm{};
  tvs_iters its{};
  StepScalars<T> cs{};
  Partials part{};
  double* e = nullptr;
  KernelTimer* tm = nullptr;
  T *cur = nullptr, *nxt = nullptr;
  int n = 0, done = 0;
  bool finished = false;
  std::vector<double>* hist = nullptr;  // receives D(p^0..p^done) when end() computes statistics

  Step2Run(Step2Problem<T>& prob, const T* d0_, int N2_, int N1_, const tvs_params* p, const tvs_layout* l,
           const tvs_iters* it, Partials pt, double* e_, KernelTimer* t)
      : P(&prob), d0(d0_), N2(N2_), N1(N1_), prm(*p), its(*it), part(pt), e(e_), tm(t) {
    const T inv_h = T(1.0 / prm.h);
    cs = StepScalars<T>{T(prm.t), inv_h, T(prm.delta), T(prm.alpha), T(alpha_hat_of(l))};
  }
  bool irv1() const { return prm.variant == TVS_IRV1; }
  double scale() const { return std::sqrt(double(N2) * N1); }

  void begin(const T* tau, hipStream_t s) {
    const Grid g = P->g;
    const SubFrames& sf = P->ss.sf;
    const long long gpl = (long long)N2 * N1;
    // a6: the bridge from tau to the Step-2 data
    if (irv1()) {
      launch_xi<T>(tau, N2, N1, T(prm.eps), dptr<T>(P->xi), s);
      launch_irv1_data<T>(d0, dptr<T>(P->xi), g, cs.inv_h, T(prm.alpha), dptr<T>(P->f2), s);
    } else {
      launch_bridge_irv2<T>(tau, d0, N2, N1, T(prm.h), T(prm.alpha), dptr<T>(P->f2), s);
    }
    launch_fill<T>(dptr<T>(P->p), 2 * gpl, T(0), s);
    launch_fill<T>(dptr<T>(P->va), 2 * sf.plane * sf.nsub, T(0), s);
    launch_fill<T>(dptr<T>(P->vb), 2 * sf.plane * sf.nsub, T(0), s);
    cur = dptr<T>(P->va);
    nxt = dptr<T>(P->vb);
    n = done = 0;
    finished = false;
  }

  bool sweep(hipStream_t s) {
    if (!head(s)) return false;
    body(s, true);
    return !finished;
  }

  // the energy of p^n (into e[n]) and the stopping test
  bool head(hipStream_t s) {
    if (finished) return false;
    launch_energy_rof<T>(dptr<T>(P->p), dptr<T>(P->f2), P->g, cs.inv_h, part, e + n, s);
    if (its.tol > 0 && n >= 1) {
      double hv[2];
      TVS_HIP(hipMemcpyAsync(hv, e + n - 1, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      TVS_HIP(hipStreamSynchronize(s));
      if (residual_of(hv[0], hv[1], scale()) < its.tol) {
        finished = true;
        return false;
      }
    }
    return true;
  }

  // a7-a9, the same launches in every sweep (see Step1Run::body)
  void body(hipStream_t s, bool launch) {
    if (launch) prologue(s);
    for (int nu = 0; nu < its.inner; ++nu) {
      if (launch) inner(s);
      std::swap(cur, nxt);
    }
    if (launch) combine(s);
    ++done;
    ++n;
    if (n >= its.sweeps) finished = true;
  }
  // a7: b_m = div((1 - theta_m) p^n) - f near the subdomain
  void prologue(hipStream_t s) {
    launch_sub2_prologue<T>(P->ss.sf, P->g, cs.inv_h, dptr<T>(P->p), dptr<T>(P->f2), dptr<T>(P->b), s);
  }
  // a8: one inner iteration
  void inner(hipStream_t s) {
    const double px = P->ss.sub_px, esz = sizeof(T);
    KernelTimer::time(tm, "s2_update", 5 * esz * px, s,
                      [&] { launch_sub2_update<T>(P->ss.sf, P->g, cs, cur, dptr<T>(P->b), nxt, s); });
  }
  // a9: combine (the state `ahead` inner iterations after `cur`)
  void combine(hipStream_t s, int ahead = 0) {
    const long long gpl = (long long)N2 * N1;
    const double px = P->ss.sub_px, esz = sizeof(T);
    const T* q = (ahead & 1) ? nxt : cur;
    KernelTimer::time(tm, "s2_combine", 2 * esz * (2.0 * gpl + px), s,
                      [&] { launch_combine<T>(P->ss.sf, P->g, 2, cs.ahat, q, dptr<T>(P->p), s); });
  }
  JobBufs<T> bufs() const {
    return JobBufs<T>{{dptr<T>(P->va), dptr<T>(P->vb)}, {nullptr, nullptr}, nullptr, dptr<T>(P->b), nullptr,
                      nullptr, parity(), 0};
  }
  int parity() const { return cur == dptr<T>(P->va) ? 0 : 1; }

  void end(T* d_out, tvs_stats* st, hipStream_t s) {
    const Grid g = P->g;
    const T inv_h = cs.inv_h;
    launch_energy_rof<T>(dptr<T>(P->p), dptr<T>(P->f2), g, inv_h, part, e + done, s);
    if (irv1())
      launch_irv1_image<T>(d0, dptr<T>(P->p), dptr<T>(P->xi), g, inv_h, T(1.0 / prm.alpha), d_out, s);
    else
      launch_irv2_image<T>(d0, dptr<T>(P->p), g, inv_h, T(1.0 / prm.alpha), d_out, s);
    if (st) {
      launch_primal_rof<T>(dptr<T>(P->p), dptr<T>(P->f2), g, inv_h, T(1.0 / prm.alpha), dptr<T>(P->u), s);
      launch_gap_rof<T>(dptr<T>(P->u), dptr<T>(P->p), g, inv_h, part, e + its.sweeps + 1, s);
      std::vector<double> hv(size_t(its.sweeps) + 2);
      TVS_HIP(hipMemcpyAsync(hv.data(), e, sizeof(double) * hv.size(), hipMemcpyDeviceToHost, s));
      TVS_HIP(hipStreamSynchronize(s));
      st->sweeps_done = done;
      st->energy = hv[done];
      st->residual = done >= 1 ? residual_of(hv[done - 1], hv[done], scale()) : 0.0;
      st->gap = hv[its.sweeps + 1];
      if (!std::isfinite(st->energy) || !std::isfinite(st->gap))
        throw Error(TVS_ENONFINITE, "step 2: non-finite energy or gap");
      if (hist) hist->assign(hv.begin(), hv.begin() + done + 1);
    }
  }
};

template <typename T>
void run_step2(tvs_ctx* c, const T* d0, const T* tau, int N2, int N1, const tvs_params* prm,
               const tvs_layout* l, const tvs_iters* its, T* d_out, tvs_stats* st, hipStream_t s) {
  Step2Problem<T>& P = get_step2<T>(c, N2, N1, prm->h, l, s);
  Step2Run<T> run(P, d0, N2, N1, prm, l, its, partials(c), scal(c, size_t(its->sweeps) + 3), &c->timer);
  c->history.clear();
  run.hist = &c->history;
  run.begin(tau, s);
  while (run.sweep(s)) {
  }
  run.end(d_out, st, s);
}

template <typename T>
void run_project(tvs_ctx* c, const T* u_in, int n2, int n1, double h, T* u_out, hipStream_t s) {
  GreenTable& tab = get_table(c, n2, n1, h, s);
  auto key = GridKey{n2, n1, h};
  auto& mp = projmap<T>(c);
  if (!mp.count(key))
    mp[key] = std::make_unique<GreenPlan<T>>(tab, std::vector<std::array<int, 4>>{{0, 0, n2, n1}}, s);
  const size_t gp = size_t(n2) * n1 * sizeof(T);
  auto& tmp = c->projtmp[key];
  if (!tmp || tmp->bytes < gp) tmp = std::make_unique<DevBuf>(gp);
  const Grid g{n2, n1, h};
  mp[key]->apply_div(u_in, global_frame(g), tmp->as<T>(), Frame{0, 0, n1}, s);
  // P u = u - grad phi, reusing the f1 kernel with delta = 1
  launch_f1<T>(u_in, tmp->as<T>(), g, T(1.0 / h), T(1), u_out, s);
}

template <typename F>
int guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return TVS_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return TVS_EHIP;
  } catch (...) {
    g_last_error = "unknown error";
    return TVS_EHIP;
  }
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    TVS_HIP(hipGetDevice(&prev));
    if (prev != dev) TVS_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// ---------------------------------------------------------------------------
// Jobs: one image's solve with its own resident state (problems, dual
// variables, d0/tau/d), advanced one Schwarz sweep at a time.  A job runs the
// same launches in the same order as the one-shot calls, so its results are
// bit-identical to theirs.
// ---------------------------------------------------------------------------
template <typename T>
struct JobState {
  DevBuf d0, tau, dout, part, e1, e2;
  std::unique_ptr<Step1Problem<T>> p1;
  std::unique_ptr<Step2Problem<T>> p2;
  std::unique_ptr<Step1Run<T>> r1;
  std::unique_ptr<Step2Run<T>> r2;
  JobState() = default;
  JobState(const JobState&) = delete;
  JobState& operator=(const JobState&) = delete;
  size_t bytes() const {
    return d0.bytes + tau.bytes + dout.bytes + part.bytes + e1.bytes + e2.bytes + p1->bytes() +
           p2->bytes();
  }
};

// bytes of a job's own device state, computed on the host (the same
// allocations as JobState, make_step1 and make_step2)
template <typename T>
size_t job_bytes_estimate(int N2, int N1, const tvs_layout* l, int sweeps) {
  const size_t esz = sizeof(T);
  const int n2 = N2 + 1, n1 = N1 + 1;
  const bool plain = l->M2 == 1 && l->M1 == 1;
  SubSet s1;
  s1.ay = make_axis(n2, l->M2, l->s_y, "M2");
  s1.ax = make_axis(n1, l->M1, l->s_x, "M1");
  plan_subs1(s1, n2, n1);
  size_t b = 13 * size_t(n2) * n1 * esz + size_t(plain ? 15 : 21) * size_t(s1.sf.plane) * s1.sf.nsub * esz +
             subs_device_bytes(s1) + GreenPlan<T>::footprint({{0, 0, n2, n1}});
  if (!plain) {
    std::vector<std::array<int, 4>> boxes;
    for (auto& d : s1.subs) boxes.push_back({d.i0, d.j0, d.bi, d.bj});
    b += GreenPlan<T>::footprint(boxes);
  }
  SubSet s2;
  s2.ay = make_axis(n2, l->M2, l->s_y, "M2");
  s2.ax = make_axis(n1, l->M1, l->s_x, "M1");
  plan_subs2(s2, N2, N1);
  b += 6 * size_t(N2) * N1 * esz + 5 * size_t(s2.sf.plane) * s2.sf.nsub * esz + subs_device_bytes(s2);
  b += (2 * size_t(N2) * N1 + 2 * size_t(n2) * n1) * esz + sizeof(double) * 1024 +
       2 * sizeof(double) * (size_t(sweeps) + 3);
  return b;
}

}  // namespace
}  // namespace tvs

struct tvs_job {
  tvs_ctx* ctx = nullptr;
  unsigned long long uid = 0;  // unique within the process (batch-graph keys)
  tvs_dtype dtype = TVS_F32;
  int N2 = 0, N1 = 0;
  tvs_params prm{};
  tvs_layout lay{};
  tvs_iters its{};
  int step = 1;  // 1, 2, or 3 when finished (or failed)
  int failed = 0;     // the error code that ended the job, 0 if none
  std::string error;  // its message
  tvs_stats st[2]{};
  std::unique_ptr<tvs::JobState<float>> f;
  std::unique_ptr<tvs::JobState<double>> d;
};

using namespace tvs;

namespace {

unsigned long long next_job_uid() {
  static std::atomic<unsigned long long> uid{0};
  return ++uid;
}

template <typename T>
JobState<T>& job_state(tvs_job* j);
template <>
JobState<float>& job_state<float>(tvs_job* j) { return *j->f; }
template <>
JobState<double>& job_state<double>(tvs_job* j) { return *j->d; }

template <typename T>
void job_create(tvs_ctx* c, tvs_job* j, const T* d0, hipStream_t s,
                hipMemcpyKind kind = hipMemcpyDeviceToDevice) {
  auto st = std::make_unique<JobState<T>>();
  const int N2 = j->N2, N1 = j->N1;
  const size_t esz = sizeof(T);
  st->d0.alloc(esz * size_t(N2) * N1);
  st->tau.alloc(2 * esz * size_t(N2 + 1) * (N1 + 1));
  st->dout.alloc(esz * size_t(N2) * N1);
  st->part.alloc(sizeof(double) * 1024);
  st->e1.alloc(sizeof(double) * (size_t(j->its.sweeps) + 3));
  st->e2.alloc(sizeof(double) * (size_t(j->its.sweeps) + 3));
  st->p1 = make_step1<T>(c, N2, N1, j->prm.h, &j->lay, s, TVS_LP_IMAGE, false);
  st->p2 = make_step2<T>(N2, N1, j->prm.h, &j->lay, s);
  const ShapeKey sk = shape_key(int(dtype_of<T>()), N2, N1, j->prm.h, &j->lay);
  // a job uses the shapes forced or tuned before for its problem shape and
  // times none itself: the requests of a server come in many sizes, and each
  // would pay the tuning (0.5 s for a 4096^2 float64 single-domain job)
  apply_tiles1<T>(c, *st->p1, sk, s, false);
  apply_tiles2<T>(c, *st->p2, sk, s, false);
  TVS_HIP(hipMemcpyAsync(st->d0.p, d0, esz * size_t(N2) * N1, kind, s));
  st->r1 = std::make_unique<Step1Run<T>>(*st->p1, st->d0.template as<T>(), N2, N1, &j->prm, &j->lay, &j->its,
                                         Partials{st->part.template as<double>(), 1024}, st->e1.template as<double>(), &c->timer);
  st->r1->begin(s);
  // later calls may come on another stream
  TVS_HIP(hipStreamSynchronize(s));
  if constexpr (sizeof(T) == 4)
    j->f = std::move(st);
  else
    j->d = std::move(st);
}

template <typename T>
void make_run2(tvs_ctx* c, tvs_job* j, JobState<T>& st) {
  st.r2 = std::make_unique<Step2Run<T>>(*st.p2, st.d0.template as<T>(), j->N2, j->N1, &j->prm, &j->lay, &j->its,
                                        Partials{st.part.template as<double>(), 1024},
                                        st.e2.template as<double>(), &c->timer);
}

// The end of a step that has no sweep left (tau and its statistics, then
// the set-up of Step 2; or the image and the statistics of Step 2).
template <typename T>
void job_step_end(tvs_ctx* c, tvs_job* j, hipStream_t s) {
  JobState<T>& st = job_state<T>(j);
  if (j->step == 1) {
    st.r1->end(st.tau.template as<T>(), &j->st[0], s);
    make_run2(c, j, st);
    st.r2->begin(st.tau.template as<T>(), s);
    j->step = 2;
  } else if (j->step == 2) {
    st.r2->end(st.dout.template as<T>(), &j->st[1], s);
    j->step = 3;
  }
}

// The head of the job's current step (the FP64 energy and the stopping
// test); when the stopping test ends the step, its end instead.  True when
// the job's body is to run in this batch call.
template <typename T>
bool job_head(tvs_ctx* c, tvs_job* j, hipStream_t s) {
  JobState<T>& st = job_state<T>(j);
  if (j->step == 1 ? st.r1->head(s) : j->step == 2 ? st.r2->head(s) : false) return true;
  job_step_end<T>(c, j, s);
  return false;
}

// After a body: the end of the step if that was its last sweep.
template <typename T>
void job_after(tvs_ctx* c, tvs_job* j, hipStream_t s) {
  JobState<T>& st = job_state<T>(j);
  if ((j->step == 1 && st.r1->finished) || (j->step == 2 && st.r2->finished)) job_step_end<T>(c, j, s);
}

// Jobs whose sweep bodies run together.  Jobs of one group share the step,
// the dtype, the image shape, the layout, h, t and the inner count, hence
// every geometric descriptor: their inner iterations run as one launch per
// kernel class over all their subdomains (JobBufs tables).
struct BodyGroup {
  int step, dtype;
  std::vector<tvs_job*> jobs;
  size_t table_off = 0;  // byte offset of the group's JobBufs table
};

using GroupKey = std::tuple<int, int, int, int, int, int, int, int, double, double, int>;
GroupKey group_key(const tvs_job* j) {
  return GroupKey{j->step, int(j->dtype), j->N2, j->N1, j->lay.M2, j->lay.M1, j->lay.s_y, j->lay.s_x,
                  j->prm.h, j->prm.t, j->its.inner};
}

template <typename T>
JobBufs<T> job_bufs(tvs_job* j) {
  JobState<T>& st = job_state<T>(j);
  return j->step == 1 ? st.r1->bufs() : st.r2->bufs();
}

// One inner iteration (index nu) of every job of a group, one launch per
// kernel class; `table` is the group's JobBufs array on the device.
template <typename T>
void group_inner(const BodyGroup& G, const JobBufs<T>* table, int nu, KernelTimer* tm, hipStream_t s) {
  const int nj = int(G.jobs.size()), flip = nu & 1;
  JobState<T>& st0 = job_state<T>(G.jobs[0]);
  const double esz = sizeof(T);
  if (G.step == 1) {
    Step1Run<T>& r = *st0.r1;
    const SubFrames& sf = r.P->ss.sf;
    const double px = r.P->ss.sub_px * nj;
    r.inner_plan().apply_div_jobs(table, nj, flip, sub_frame(sf, 2), sub_frame(sf, 1), s, tm,
                                  r.P->plain ? "s1_plain" : "s1_local");
    KernelTimer::time(tm, "s1_update", 13 * esz * px, s, [&] {
      launch_sub_update1_jobs<T>(sf, r.P->g, r.cs, JobRef<T>{table, sf.nsub, flip}, nj, s);
    });
    KernelTimer::time(tm, "s1_vecdiv", 6 * esz * px, s, [&] {
      launch_sub_vecdiv_jobs<T>(sf, r.P->g, r.cs.inv_h, JobRef<T>{table, sf.nsub, flip ^ 1}, nj, s);
    });
  } else {
    Step2Run<T>& r = *st0.r2;
    const SubFrames& sf = r.P->ss.sf;
    KernelTimer::time(tm, "s2_update", 5 * esz * r.P->ss.sub_px * nj, s, [&] {
      launch_sub2_update_jobs<T>(sf, r.P->g, r.cs, JobRef<T>{table, sf.nsub, flip}, nj, s);
    });
  }
}

template <typename T>
void job_prologue(tvs_job* j, hipStream_t s) {
  JobState<T>& st = job_state<T>(j);
  if (j->step == 1) st.r1->prologue(s);
  else st.r2->prologue(s);
}
// the combination, launched before the host state advances: the inner
// iterations ended `inner` ping-pong steps after the current state
template <typename T>
void job_combine(tvs_job* j, hipStream_t s) {
  JobState<T>& st = job_state<T>(j);
  if (j->step == 1) st.r1->combine(s, j->its.inner);
  else st.r2->combine(s, j->its.inner);
}
// the host-side state of a body that ran (ping-pong parity, counters)
template <typename T>
void job_advance(tvs_job* j) {
  JobState<T>& st = job_state<T>(j);
  if (j->step == 1) st.r1->body(nullptr, false);
  else st.r2->body(nullptr, false);
}

// The sweep bodies of all groups: every job's prologue, then the inner
// iterations group by group, nu by nu, then every job's combination.
void launch_bodies(tvs_ctx* c, const std::vector<BodyGroup>& groups, hipStream_t s) {
  KernelTimer* tm = &c->timer;
  int inner = 0;
  for (const BodyGroup& G : groups) {
    inner = std::max(inner, G.jobs[0]->its.inner);
    for (tvs_job* j : G.jobs) {
      if (G.dtype == TVS_F32) job_prologue<float>(j, s);
      else job_prologue<double>(j, s);
    }
  }
  const char* base = static_cast<const char*>(c->jobtab.p);
  for (int nu = 0; nu < inner; ++nu)
    for (const BodyGroup& G : groups) {
      if (nu >= G.jobs[0]->its.inner) continue;
      if (G.dtype == TVS_F32)
        group_inner<float>(G, reinterpret_cast<const JobBufs<float>*>(base + G.table_off), nu, tm, s);
      else
        group_inner<double>(G, reinterpret_cast<const JobBufs<double>*>(base + G.table_off), nu, tm, s);
    }
  for (const BodyGroup& G : groups)
    for (tvs_job* j : G.jobs) {
      if (G.dtype == TVS_F32) job_combine<float>(j, s);
      else job_combine<double>(j, s);
    }
}

// ---- a job's state between sweeps, as one host blob (checkpoint/resume) ----
// Between two sweeps a run is described by its dual variables (the global p
// and the resident subdomain duals of the ping-pong state the next sweep
// starts from, with their vecdiv in Step 1), its FP64 energy history and its
// counters; everything else (tau_0, f, omega, the Step-2 data, the plans) is
// recomputed from d0 and tau by the same kernels, so a restored job continues
// bit for bit as the original would have.
constexpr char kStateMagic[8] = {'T', 'V', 'S', 'J', 'O', 'B', 'S', 'T'};
constexpr uint32_t kStateVersion = 1;
constexpr int kMaxSections = 6;

struct StateHeader {
  char magic[8];
  uint32_t version, header_bytes;
  uint64_t total_bytes;
  int32_t dtype, N2, N1, step, n, done, finished, parity;
  tvs_params prm;
  tvs_layout lay;
  tvs_iters its;
  tvs_stats st[2];
  int32_t nsec, reserved;
  uint64_t sec_bytes[kMaxSections];
};

struct Section {
  void* p;
  size_t bytes;
};

// the device arrays holding a job's state at its current step, in blob order
template <typename T>
std::vector<Section> state_sections(tvs_job* j) {
  JobState<T>& st = job_state<T>(j);
  std::vector<Section> v{{st.d0.p, st.d0.bytes}};
  if (j->step == 1) {
    Step1Run<T>& r = *st.r1;
    v.push_back({r.P->p.p, r.P->p.bytes});
    v.push_back({r.cur, r.P->va.bytes});
    v.push_back({r.zcur, r.P->za.bytes});
    v.push_back({st.e1.p, st.e1.bytes});
  } else if (j->step == 2) {
    Step2Run<T>& r = *st.r2;
    v.push_back({st.tau.p, st.tau.bytes});
    v.push_back({r.P->p.p, r.P->p.bytes});
    v.push_back({r.cur, r.P->va.bytes});
    v.push_back({st.e2.p, st.e2.bytes});
  } else {
    v.push_back({st.tau.p, st.tau.bytes});
    v.push_back({st.dout.p, st.dout.bytes});
  }
  return v;
}

template <typename T>
StateHeader state_header(tvs_job* j, const std::vector<Section>& secs) {
  JobState<T>& st = job_state<T>(j);
  StateHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kStateMagic, sizeof h.magic);
  h.version = kStateVersion;
  h.header_bytes = sizeof(StateHeader);
  h.dtype = j->dtype;
  h.N2 = j->N2;
  h.N1 = j->N1;
  h.step = j->step;
  if (j->step == 1) {
    h.n = st.r1->n;
    h.done = st.r1->done;
    h.finished = st.r1->finished;
    h.parity = st.r1->parity();
  } else {
    h.n = st.r2->n;
    h.done = st.r2->done;
    h.finished = st.r2->finished;
    h.parity = st.r2->parity();
  }
  h.prm = j->prm;
  h.lay = j->lay;
  h.its = j->its;
  h.st[0] = j->st[0];
  h.st[1] = j->st[1];
  h.nsec = int32_t(secs.size());
  h.total_bytes = sizeof(StateHeader);
  for (size_t k = 0; k < secs.size(); ++k) {
    h.sec_bytes[k] = secs[k].bytes;
    h.total_bytes += secs[k].bytes;
  }
  return h;
}

template <typename T>
size_t job_export(tvs_job* j, unsigned char* buf, size_t cap, hipStream_t s) {
  const std::vector<Section> secs = state_sections<T>(j);
  const StateHeader h = state_header<T>(j, secs);
  if (!buf) return h.total_bytes;
  if (cap < h.total_bytes)
    throw Error(TVS_EINVAL, "state buffer of " + std::to_string(cap) + " bytes, " +
                                std::to_string(h.total_bytes) + " needed");
  std::memcpy(buf, &h, sizeof h);
  size_t off = sizeof h;
  for (const Section& sec : secs) {
    TVS_HIP(hipMemcpyAsync(buf + off, sec.p, sec.bytes, hipMemcpyDeviceToHost, s));
    off += sec.bytes;
  }
  TVS_HIP(hipStreamSynchronize(s));
  return h.total_bytes;
}

// restore the state of a job that job_create has just built from the blob's
// d0 (and the blob's shape, parameters, layout and counts)
template <typename T>
void job_restore(tvs_ctx* c, tvs_job* j, const StateHeader& h, const unsigned char* buf, hipStream_t s) {
  JobState<T>& st = job_state<T>(j);
  const int sweeps = j->its.sweeps;
  if (h.n < 0 || h.n > sweeps || h.done < 0 || h.done > sweeps || h.parity < 0 || h.parity > 1)
    throw Error(TVS_EINVAL, "state blob: run counters out of range");
  if (h.nsec != (h.step == 3 ? 3 : 5)) throw Error(TVS_EINVAL, "state blob: wrong number of sections");
  // every section size is checked before any device work, so that a
  // rejected blob leaves nothing queued on the stream
  const std::vector<size_t> want =
      h.step == 1   ? std::vector<size_t>{st.d0.bytes, st.p1->p.bytes, st.p1->va.bytes, st.p1->za.bytes, st.e1.bytes}
      : h.step == 2 ? std::vector<size_t>{st.d0.bytes, st.tau.bytes, st.p2->p.bytes, st.p2->va.bytes, st.e2.bytes}
                    : std::vector<size_t>{st.d0.bytes, st.tau.bytes, st.dout.bytes};
  for (size_t k = 0; k < want.size(); ++k)
    if (want[k] != h.sec_bytes[k])
      throw Error(TVS_EINVAL, "state blob: section " + std::to_string(k) + " has the wrong size");
  j->st[0] = h.st[0];
  j->st[1] = h.st[1];
  if (h.step >= 2) {
    make_run2(c, j, st);
    if (h.step == 2) {
      // the Step-2 data comes from tau; the blob's tau follows d0
      TVS_HIP(hipMemcpyAsync(st.tau.p, buf + sizeof h + h.sec_bytes[0], st.tau.bytes, hipMemcpyHostToDevice, s));
      st.r2->begin(st.tau.template as<T>(), s);
    }
  }
  j->step = h.step;
  if (h.step == 1) {
    Step1Run<T>& r = *st.r1;
    r.n = h.n;
    r.done = h.done;
    r.finished = h.finished != 0;
    if (h.parity != r.parity()) {
      std::swap(r.cur, r.nxt);
      std::swap(r.zcur, r.znxt);
    }
  } else {
    Step2Run<T>& r = *st.r2;
    r.n = h.n;
    r.done = h.done;
    r.finished = h.step == 3 || h.finished != 0;
    if (h.step == 2 && h.parity != r.parity()) std::swap(r.cur, r.nxt);
  }
  const std::vector<Section> secs = state_sections<T>(j);
  size_t off = sizeof h;
  for (const Section& sec : secs) {
    TVS_HIP(hipMemcpyAsync(sec.p, buf + off, sec.bytes, hipMemcpyHostToDevice, s));
    off += sec.bytes;
  }
  // the caller may free the blob on return, and later calls may come on
  // another stream
  TVS_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Allocation-free quality measures: the reduction scratch of
// tvs_quality_noalloc (256 partial sums per moment, 4 moments at a time,
// then the 6 moments) lives in this file-scope device array.  Each device
// holds its own copy; host code must use the address hipGetSymbolAddress
// returns for it with that device current (taken once per device when a
// context is created there), never the array's name.  Every kernel writes
// each slot before it is read, so nothing needs clearing between calls.
// ---------------------------------------------------------------------------
constexpr int kNoAllocPartials = 1024;
constexpr int kNoAllocMoments = 8;
static __device__ __align__(256) double scratch[kNoAllocPartials + kNoAllocMoments];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// with `device` current
void bind_scratch(int device) {
  if (device < 0 || device >= kMaxDevices)
    throw Error(TVS_EINVAL, "device index above " + std::to_string(kMaxDevices - 1));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    throw Error(TVS_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = static_cast<double*>(p);
}

double* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  double* p = (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
  if (!p) throw Error(TVS_EHIP, "no scratch address for this device (no context was created on it)");
  return p;
}

// Section 5.2 with R = 1 (c1 = (0.01 R)^2, c2 = (0.03 R)^2) from the six
// FP64 sums (x, ref, centred squares of x and ref, centred cross term,
// squared difference)
void quality_from_moments(const double (&m)[6], long long n, double* out) {
  for (double v : m)
    if (!std::isfinite(v)) throw Error(TVS_ENONFINITE, "quality: non-finite moment");
  const double c1 = 1e-4, c2 = 9e-4, dn = double(n);
  const double mx = m[0] / dn, mr = m[1] / dn, vx = m[2] / dn, vr = m[3] / dn, cv = m[4] / dn;
  const double mse = m[5] / dn;
  out[0] = mse > 0 ? -10.0 * std::log10(mse) : HUGE_VAL;
  out[1] = (2 * mx * mr + c1) * (2 * cv + c2) / ((mx * mx + mr * mr + c1) * (vx + vr + c2));
  out[2] = mse;
}

}  // namespace

extern "C" {

int tvs_ctx_create(int device, tvs_ctx** out) {
  return guarded([&] {
    if (!out) throw Error(TVS_EINVAL, "out is NULL");
    int n = 0;
    TVS_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) throw Error(TVS_EINVAL, "no such HIP device");
    DeviceGuard dg(device);
    bind_scratch(device);
    auto* c = new tvs_ctx();
    c->device = device;
    *out = c;
  });
}

void tvs_ctx_destroy(tvs_ctx* ctx) {
  if (!ctx) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  delete ctx;
  if (prev >= 0) (void)hipSetDevice(prev);
}

const char* tvs_last_error(void) { return g_last_error.c_str(); }

size_t tvs_ctx_bytes(const tvs_ctx* c) {
  if (!c) return 0;
  size_t b = c->partials.bytes + c->scal.bytes;
  for (auto& kv : c->tables) b += kv.second->g.bytes;
  for (auto& kv : c->s1f) b += kv.second->bytes();
  for (auto& kv : c->s1d) b += kv.second->bytes();
  for (auto& kv : c->s2f) b += kv.second->bytes();
  for (auto& kv : c->s2d) b += kv.second->bytes();
  for (auto& kv : c->projf) b += kv.second->bytes();
  for (auto& kv : c->projd) b += kv.second->bytes();
  for (auto& kv : c->projtmp) b += kv.second->bytes;
  return b;
}

int tvs_step1(tvs_ctx* ctx, const void* d0, int N2, int N1, tvs_dtype dtype,
              const tvs_params* params, const tvs_layout* layout, const tvs_iters* iters,
              void* tau_out, tvs_stats* stats, void* stream) {
  return guarded([&] {
    if (!ctx || !d0 || !tau_out) throw Error(TVS_EINVAL, "NULL argument");
    check_params(params, N2, N1);
    check_iters(iters);
    DeviceGuard dg(ctx->device);
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == TVS_F32)
      run_step1<float>(ctx, static_cast<const float*>(d0), N2, N1, params, layout, iters,
                       static_cast<float*>(tau_out), stats, s);
    else if (dtype == TVS_F64)
      run_step1<double>(ctx, static_cast<const double*>(d0), N2, N1, params, layout, iters,
                        static_cast<double*>(tau_out), stats, s);
    else
      throw Error(TVS_EINVAL, "unknown dtype");
    if (stats)
      stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  });
}

int tvs_step2(tvs_ctx* ctx, const void* d0, const void* tau, int N2, int N1, tvs_dtype dtype,
              const tvs_params* params, const tvs_layout* layout, const tvs_iters* iters,
              void* d_out, tvs_stats* stats, void* stream) {
  return guarded([&] {
    if (!ctx || !d0 || !tau || !d_out) throw Error(TVS_EINVAL, "NULL argument");
    check_params(params, N2, N1);
    check_iters(iters);
    DeviceGuard dg(ctx->device);
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == TVS_F32)
      run_step2<float>(ctx, static_cast<const float*>(d0), static_cast<const float*>(tau), N2, N1,
                       params, layout, iters, static_cast<float*>(d_out), stats, s);
    else if (dtype == TVS_F64)
      run_step2<double>(ctx, static_cast<const double*>(d0), static_cast<const double*>(tau), N2,
                        N1, params, layout, iters, static_cast<double*>(d_out), stats, s);
    else
      throw Error(TVS_EINVAL, "unknown dtype");
    if (stats)
      stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  });
}

int tvs_schwarz_solve(tvs_ctx* ctx, const void* d0, int N2, int N1, tvs_dtype dtype,
                      const tvs_params* params, const tvs_layout* layout, const tvs_iters* iters,
                      void* d_out, void* tau_out, tvs_stats* stats, void* stream) {
  return guarded([&] {
    if (!ctx || !d0 || !d_out) throw Error(TVS_EINVAL, "NULL argument");
    check_params(params, N2, N1);
    check_iters(iters);
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t esz = dtype == TVS_F64 ? sizeof(double) : sizeof(float);
    DevBuf own;
    void* tau = tau_out;
    if (!tau) {
      own.alloc(2 * esz * size_t(N2 + 1) * (N1 + 1));
      tau = own.p;
    }
    auto t0 = std::chrono::steady_clock::now();
    if (dtype == TVS_F32) {
      run_step1<float>(ctx, static_cast<const float*>(d0), N2, N1, params, layout, iters,
                       static_cast<float*>(tau), stats, s);
      auto t1 = std::chrono::steady_clock::now();
      if (stats) stats[0].seconds = std::chrono::duration<double>(t1 - t0).count();
      run_step2<float>(ctx, static_cast<const float*>(d0), static_cast<const float*>(tau), N2, N1,
                       params, layout, iters, static_cast<float*>(d_out), stats ? stats + 1 : nullptr, s);
      if (stats) stats[1].seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
    } else if (dtype == TVS_F64) {
      run_step1<double>(ctx, static_cast<const double*>(d0), N2, N1, params, layout, iters,
                        static_cast<double*>(tau), stats, s);
      auto t1 = std::chrono::steady_clock::now();
      if (stats) stats[0].seconds = std::chrono::duration<double>(t1 - t0).count();
      run_step2<double>(ctx, static_cast<const double*>(d0), static_cast<const double*>(tau), N2,
                        N1, params, layout, iters, static_cast<double*>(d_out), stats ? stats + 1 : nullptr, s);
      if (stats) stats[1].seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
    } else {
      throw Error(TVS_EINVAL, "unknown dtype");
    }
    if (!tau_out) TVS_HIP(hipStreamSynchronize(s));  // before the owned buffer is released
  });
}

int tvs_timing_enable(tvs_ctx* ctx, int enable) {
  return guarded([&] {
    if (!ctx) throw Error(TVS_EINVAL, "NULL context");
    if (enable < 0) throw Error(TVS_EINVAL, "timing: enable must be >= 0");
    ctx->timer.on = enable != 0;
    ctx->timer.every = enable > 0 ? enable : 1;
  });
}

int tvs_timing_reset(tvs_ctx* ctx) {
  return guarded([&] {
    if (!ctx) throw Error(TVS_EINVAL, "NULL context");
    DeviceGuard dg(ctx->device);
    ctx->timer.reset();
  });
}

int tvs_timing_count(tvs_ctx* ctx) {
  if (!ctx) return TVS_EINVAL;
  int n = 0;
  const int rc = guarded([&] {
    DeviceGuard dg(ctx->device);
    ctx->timer.collect();
    n = int(ctx->timer.accs.size());
  });
  return rc == TVS_OK ? n : rc;
}

int tvs_timing_get(tvs_ctx* ctx, int i, char* name, int name_len, long long* launches, double* ms,
                   double* bytes) {
  return guarded([&] {
    if (!ctx || !name || name_len < 1 || !launches || !ms || !bytes) throw Error(TVS_EINVAL, "NULL argument");
    DeviceGuard dg(ctx->device);
    ctx->timer.collect();
    if (i < 0 || i >= int(ctx->timer.accs.size())) throw Error(TVS_EINVAL, "no such timing entry");
    const auto& kv = ctx->timer.accs[size_t(i)];
    std::snprintf(name, size_t(name_len), "%s", kv.first.c_str());
    *launches = kv.second.launches;
    *ms = kv.second.ms;
    *bytes = kv.second.bytes;
  });
}

int tvs_project_div_free(tvs_ctx* ctx, const void* u_in, int n2, int n1, tvs_dtype dtype, double h,
                         void* u_out, void* stream) {
  return guarded([&] {
    if (!ctx || !u_in || !u_out) throw Error(TVS_EINVAL, "NULL argument");
    if (n2 < 2 || n1 < 2) throw Error(TVS_EINVAL, "grid must be at least 2 x 2");
    if ((long long)n2 * n1 > (1LL << 28)) throw Error(TVS_EINVAL, "grid too large");
    check_grid_sides(n2, n1);
    if (!(h > 0)) throw Error(TVS_EINVAL, "h must be > 0");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == TVS_F32)
      run_project<float>(ctx, static_cast<const float*>(u_in), n2, n1, h, static_cast<float*>(u_out), s);
    else if (dtype == TVS_F64)
      run_project<double>(ctx, static_cast<const double*>(u_in), n2, n1, h, static_cast<double*>(u_out), s);
    else
      throw Error(TVS_EINVAL, "unknown dtype");
  });
}

int tvs_energy_history(tvs_ctx* ctx, double* out, int cap, int* n) {
  return guarded([&] {
    if (!ctx || !n) throw Error(TVS_EINVAL, "NULL argument");
    if (cap < 0 || (cap > 0 && !out)) throw Error(TVS_EINVAL, "bad output buffer");
    *n = static_cast<int>(ctx->history.size());
    for (int k = 0; k < std::min(cap, *n); ++k) out[k] = ctx->history[k];
  });
}

int tvs_set_tiles(tvs_ctx* ctx, int run1, int run1d, int rows, int cols, int run2) {
  return guarded([&] {
    if (!ctx) throw Error(TVS_EINVAL, "NULL context");
    auto run_ok = [](int r) { return r == 0 || r == 1 || r == 2 || r == 4; };
    if (!run_ok(run1) || !run_ok(run1d) || !run_ok(run2))
      throw Error(TVS_EINVAL, "tiles: run lengths must be 0, 1, 2 or 4");
    if (rows < 0 || rows > 64 || cols < 0 || cols > 64) throw Error(TVS_EINVAL, "tiles: rows and cols must lie in [0, 64]");
    ctx->force = Tiles{run1, run1d, rows, cols, run2};
  });
}

int tvs_get_tiles(tvs_ctx* ctx, int N2, int N1, tvs_dtype dtype, const tvs_layout* layout, double h, int* out) {
  return guarded([&] {
    if (!ctx || !layout || !out) throw Error(TVS_EINVAL, "NULL argument");
    if (dtype != TVS_F32 && dtype != TVS_F64) throw Error(TVS_EINVAL, "unknown dtype");
    auto it = ctx->tuned.find(shape_key(int(dtype), N2, N1, h, layout));
    const Tiles t = it == ctx->tuned.end() ? Tiles{} : it->second;
    out[0] = t.run1;
    out[1] = t.run1d;
    out[2] = t.rows;
    out[3] = t.cols;
    out[4] = t.run2;
  });
}

int tvs_set_local_projection(tvs_ctx* ctx, int kind) {
  return guarded([&] {
    if (!ctx) throw Error(TVS_EINVAL, "NULL context");
    if (kind != TVS_LP_IMAGE && kind != TVS_LP_BLOCKDCT) throw Error(TVS_EINVAL, "unknown local projection");
    ctx->lp_kind = kind;
  });
}

int tvs_set_block_groups(tvs_ctx* ctx, int g2, int g1) {
  return guarded([&] {
    if (!ctx) throw Error(TVS_EINVAL, "NULL context");
    if (g2 < 0 || g1 < 0 || g2 > 64 || g1 > 64) throw Error(TVS_EINVAL, "block groups must be in [0, 64]");
    ctx->bd_g2 = g2;
    ctx->bd_g1 = g1;
  });
}

int tvs_tangent_field(tvs_ctx* ctx, const void* d, int N2, int N1, tvs_dtype dtype, double h, void* tau_out,
                      void* stream) {
  return guarded([&] {
    if (!ctx || !d || !tau_out) throw Error(TVS_EINVAL, "NULL argument");
    if (N2 < 2 || N1 < 2) throw Error(TVS_EINVAL, "image must be at least 2 x 2");
    if ((long long)(N2 + 1) * (N1 + 1) > (1LL << 28)) throw Error(TVS_EINVAL, "image too large");
    if (!(h > 0)) throw Error(TVS_EINVAL, "h must be > 0");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == TVS_F32)
      launch_tau0<float>(static_cast<const float*>(d), N2, N1, float(1.0 / h), static_cast<float*>(tau_out), s);
    else if (dtype == TVS_F64)
      launch_tau0<double>(static_cast<const double*>(d), N2, N1, 1.0 / h, static_cast<double*>(tau_out), s);
    else
      throw Error(TVS_EINVAL, "unknown dtype");
  });
}

int tvs_quality(tvs_ctx* ctx, const void* x, const void* ref, int n2, int n1, tvs_dtype dtype, double* out,
                void* stream) {
  return guarded([&] {
    if (!ctx || !x || !ref || !out) throw Error(TVS_EINVAL, "NULL argument");
    if (n2 < 1 || n1 < 1) throw Error(TVS_EINVAL, "grid must be at least 1 x 1");
    if ((long long)n2 * n1 > (1LL << 31)) throw Error(TVS_EINVAL, "grid too large");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long long n = (long long)n2 * n1;
    double* dev = scal(ctx, 6);
    if (dtype == TVS_F32)
      launch_quality_moments<float>(static_cast<const float*>(x), static_cast<const float*>(ref), n, partials(ctx),
                                    dev, s);
    else if (dtype == TVS_F64)
      launch_quality_moments<double>(static_cast<const double*>(x), static_cast<const double*>(ref), n,
                                     partials(ctx), dev, s);
    else
      throw Error(TVS_EINVAL, "unknown dtype");
    double m[6];
    TVS_HIP(hipMemcpyAsync(m, dev, sizeof m, hipMemcpyDeviceToHost, s));
    TVS_HIP(hipStreamSynchronize(s));
    quality_from_moments(m, n, out);
  });
}

int tvs_quality_noalloc(tvs_ctx* ctx, const void* x, const void* ref, int n2, int n1, tvs_dtype dtype,
                        double* out, void* stream) {
  return guarded([&] {
    if (!ctx || !x || !ref || !out) throw Error(TVS_EINVAL, "NULL argument");
    if (n2 < 1 || n1 < 1) throw Error(TVS_EINVAL, "grid must be at least 1 x 1");
    if ((long long)n2 * n1 > (1LL << 31)) throw Error(TVS_EINVAL, "grid too large");
    if (dtype != TVS_F32 && dtype != TVS_F64) throw Error(TVS_EINVAL, "unknown dtype");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long long n = (long long)n2 * n1;
    double* base = scratch_of(ctx->device);
    const Partials part{base, kNoAllocPartials};
    double* dev = base + kNoAllocPartials;
    if (dtype == TVS_F32)
      launch_quality_moments<float>(static_cast<const float*>(x), static_cast<const float*>(ref), n, part, dev, s);
    else
      launch_quality_moments<double>(static_cast<const double*>(x), static_cast<const double*>(ref), n, part,
                                     dev, s);
    double m[6];
    TVS_HIP(hipMemcpyAsync(m, dev, sizeof m, hipMemcpyDeviceToHost, s));
    TVS_HIP(hipStreamSynchronize(s));
    quality_from_moments(m, n, out);
  });
}

int tvs_job_footprint(int N2, int N1, tvs_dtype dtype, const tvs_layout* layout, const tvs_iters* iters,
                      size_t* bytes) {
  return guarded([&] {
    if (!layout || !iters || !bytes) throw Error(TVS_EINVAL, "NULL argument");
    check_shape(N2, N1);
    check_iters(iters);
    // the job's own state plus the Green-function table of its grid, which the
    // context holds once per grid size
    const size_t table = sizeof(double) * size_t(N2 + 2) * (N1 + 2);
    if (dtype == TVS_F32)
      *bytes = job_bytes_estimate<float>(N2, N1, layout, iters->sweeps) + table;
    else if (dtype == TVS_F64)
      *bytes = job_bytes_estimate<double>(N2, N1, layout, iters->sweeps) + table;
    else
      throw Error(TVS_EINVAL, "unknown dtype");
  });
}

int tvs_job_create(tvs_ctx* ctx, const void* d0, int N2, int N1, tvs_dtype dtype,
                   const tvs_params* params, const tvs_layout* layout, const tvs_iters* iters,
                   void* stream, tvs_job** out) {
  return guarded([&] {
    if (!ctx || !d0 || !layout || !out) throw Error(TVS_EINVAL, "NULL argument");
    *out = nullptr;
    check_params(params, N2, N1);
    check_iters(iters);
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto j = std::make_unique<tvs_job>();
    j->ctx = ctx;
    j->uid = next_job_uid();
    j->dtype = dtype;
    j->N2 = N2;
    j->N1 = N1;
    j->prm = *params;
    j->lay = *layout;
    j->its = *iters;
    if (dtype == TVS_F32)
      job_create<float>(ctx, j.get(), static_cast<const float*>(d0), s);
    else if (dtype == TVS_F64)
      job_create<double>(ctx, j.get(), static_cast<const double*>(d0), s);
    else
      throw Error(TVS_EINVAL, "unknown dtype");
    *out = j.release();
  });
}

int tvs_batch_sweep(tvs_ctx* ctx, tvs_job* const* jobs, int n, void* stream) {
  return guarded([&] {
    if (!ctx || (n > 0 && !jobs) || n < 0) throw Error(TVS_EINVAL, "bad job list");
    for (int i = 0; i < n; ++i)
      if (!jobs[i] || jobs[i]->ctx != ctx) throw Error(TVS_EINVAL, "job missing or of another context");
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < i; ++k)
        if (jobs[k] == jobs[i]) throw Error(TVS_EINVAL, "a job appears twice in the list");
    if (n == 0) return;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!ctx->bstream) {
      TVS_HIP(hipStreamCreateWithFlags(&ctx->bstream, hipStreamNonBlocking));
      TVS_HIP(hipEventCreateWithFlags(&ctx->bfork, hipEventDisableTiming));
      TVS_HIP(hipEventCreateWithFlags(&ctx->bjoin, hipEventDisableTiming));
    }
    hipStream_t w = ctx->bstream;
    TVS_HIP(hipEventRecord(ctx->bfork, s));
    TVS_HIP(hipStreamWaitEvent(w, ctx->bfork, 0));
    auto join = [&] {
      TVS_HIP(hipEventRecord(ctx->bjoin, w));
      TVS_HIP(hipStreamWaitEvent(s, ctx->bjoin, 0));
    };
    try {
      // 1. heads (and step ends), job by job; a job whose FP64 statistics
      // come out non-finite fails alone: it is marked finished with its
      // error and the other jobs go on
      std::vector<tvs_job*> live;
      for (int i = 0; i < n; ++i) {
        tvs_job* j = jobs[i];
        try {
          const bool go = j->dtype == TVS_F32 ? job_head<float>(ctx, j, w) : job_head<double>(ctx, j, w);
          if (go) live.push_back(j);
        } catch (const Error& e) {
          if (e.code != TVS_ENONFINITE) throw;
          j->failed = e.code;
          j->error = e.what();
          j->step = 3;
        }
      }
      if (!live.empty()) {
        // 2. groups of jobs whose inner iterations run as single launches
        std::vector<BodyGroup> groups;
        std::map<GroupKey, size_t> gidx;
        for (tvs_job* j : live) {
          const GroupKey k = group_key(j);
          auto it = gidx.find(k);
          if (it == gidx.end()) {
            gidx[k] = groups.size();
            groups.push_back(BodyGroup{j->step, int(j->dtype), {j}, 0});
          } else {
            groups[it->second].jobs.push_back(j);
          }
        }
        // their JobBufs tables, uploaded before the bodies run (stream order)
        std::vector<unsigned char> host;
        std::vector<unsigned long long> key;
        for (BodyGroup& G : groups) {
          G.table_off = host.size();
          for (tvs_job* j : G.jobs) {
            const size_t at = host.size();
            host.resize(at + sizeof(JobBufs<double>));
            if (G.dtype == TVS_F32) {
              const JobBufs<float> b = job_bufs<float>(j);
              std::memcpy(host.data() + at, &b, sizeof b);
            } else {
              const JobBufs<double> b = job_bufs<double>(j);
              std::memcpy(host.data() + at, &b, sizeof b);
            }
            key.insert(key.end(), {j->uid, (unsigned long long)j->step,
                                   (unsigned long long)(G.dtype == TVS_F32 ? job_bufs<float>(j).par
                                                                           : job_bufs<double>(j).par)});
          }
          key.push_back(~0ULL);  // group boundary
          host.resize((host.size() + 255) / 256 * 256);
        }
        static_assert(sizeof(JobBufs<float>) == sizeof(JobBufs<double>), "one table layout");
        if (ctx->jobtab.bytes < host.size()) {
          TVS_HIP(hipStreamSynchronize(w));  // earlier launches may still read the old table
          if (ctx->bgraph) {
            (void)hipGraphExecDestroy(ctx->bgraph);
            ctx->bgraph = nullptr;
            ctx->bkey.clear();
          }
          ctx->jobtab.alloc(std::max(host.size(), size_t(1) << 16));
        }
        TVS_HIP(hipMemcpyAsync(ctx->jobtab.p, host.data(), host.size(), hipMemcpyHostToDevice, w));
        // 3. the bodies: replayed from the graph recorded for the same jobs in
        // the same states, or recorded now (eagerly while kernel timing is on)
        if (ctx->timer.on) {
          launch_bodies(ctx, groups, w);
        } else {
          if (!(ctx->bgraph && ctx->bkey == key)) {
            if (ctx->bgraph) {
              (void)hipGraphExecDestroy(ctx->bgraph);
              ctx->bgraph = nullptr;
              ctx->bkey.clear();
            }
            hipGraph_t g = nullptr;
            TVS_HIP(hipStreamBeginCapture(w, hipStreamCaptureModeThreadLocal));
            try {
              launch_bodies(ctx, groups, w);
            } catch (...) {
              (void)hipStreamEndCapture(w, &g);
              if (g) (void)hipGraphDestroy(g);
              throw;
            }
            TVS_HIP(hipStreamEndCapture(w, &g));
            hipGraphExec_t ex = nullptr;
            const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess)
              throw Error(TVS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            ctx->bgraph = ex;
            ctx->bkey = key;
          }
          TVS_HIP(hipGraphLaunch(ctx->bgraph, w));
        }
        for (const BodyGroup& G : groups)
          for (tvs_job* j : G.jobs) {
            if (G.dtype == TVS_F32) job_advance<float>(j);
            else job_advance<double>(j);
          }
        // 4. the ends of the steps whose last sweep this was (each fails
        // alone on non-finite statistics, as above)
        for (tvs_job* j : live) {
          try {
            if (j->dtype == TVS_F32) job_after<float>(ctx, j, w);
            else job_after<double>(ctx, j, w);
          } catch (const Error& e) {
            if (e.code != TVS_ENONFINITE) throw;
            j->failed = e.code;
            j->error = e.what();
            j->step = 3;
          }
        }
      }
    } catch (...) {
      // whatever was enqueued before the failure stays ordered before the
      // caller's later work
      try {
        join();
      } catch (...) {
      }
      throw;
    }
    join();
  });
}

int tvs_job_status(const tvs_job* job, int* step, int* sweeps_done, int* done) {
  return guarded([&] {
    if (!job) throw Error(TVS_EINVAL, "NULL job");
    int sw = 0;
    if (job->dtype == TVS_F32) {
      sw = (job->step == 1 || !job->f->r2) ? job->f->r1->done : job->f->r2->done;
    } else {
      sw = (job->step == 1 || !job->d->r2) ? job->d->r1->done : job->d->r2->done;
    }
    if (step) *step = job->failed ? -1 : job->step;
    if (sweeps_done) *sweeps_done = sw;
    if (done) *done = job->step == 3 ? 1 : 0;
  });
}

int tvs_job_result(tvs_ctx* ctx, tvs_job* job, void* d_out, void* tau_out, tvs_stats* stats,
                   void* stream) {
  return guarded([&] {
    if (!ctx || !job || job->ctx != ctx) throw Error(TVS_EINVAL, "bad job");
    if (job->failed) throw Error(job->failed, job->error);
    if (job->step != 3) throw Error(TVS_EBUSY, "the job has not finished");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t esz = job->dtype == TVS_F64 ? sizeof(double) : sizeof(float);
    const DevBuf& dd = job->dtype == TVS_F64 ? job->d->dout : job->f->dout;
    const DevBuf& tt = job->dtype == TVS_F64 ? job->d->tau : job->f->tau;
    if (d_out)
      TVS_HIP(hipMemcpyAsync(d_out, dd.p, esz * size_t(job->N2) * job->N1, hipMemcpyDeviceToDevice, s));
    if (tau_out)
      TVS_HIP(hipMemcpyAsync(tau_out, tt.p, 2 * esz * size_t(job->N2 + 1) * (job->N1 + 1),
                             hipMemcpyDeviceToDevice, s));
    if (stats) {
      stats[0] = job->st[0];
      stats[1] = job->st[1];
    }
  });
}

int tvs_job_export_state(tvs_ctx* ctx, tvs_job* job, void* buf, size_t cap, size_t* bytes,
                         void* stream) {
  return guarded([&] {
    if (!ctx || !job || job->ctx != ctx) throw Error(TVS_EINVAL, "bad job");
    if (!bytes) throw Error(TVS_EINVAL, "bytes is NULL");
    if (job->failed) throw Error(TVS_EINVAL, "the job has failed: " + job->error);
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto* b = static_cast<unsigned char*>(buf);
    *bytes = job->dtype == TVS_F64 ? job_export<double>(job, b, cap, s) : job_export<float>(job, b, cap, s);
  });
}

int tvs_job_import_state(tvs_ctx* ctx, const void* buf, size_t bytes, void* stream, tvs_job** out) {
  return guarded([&] {
    if (!ctx || !buf || !out) throw Error(TVS_EINVAL, "NULL argument");
    *out = nullptr;
    StateHeader h;
    if (bytes < sizeof h) throw Error(TVS_EINVAL, "state blob shorter than its header");
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, kStateMagic, sizeof h.magic) != 0) throw Error(TVS_EINVAL, "not a job state blob");
    if (h.version != kStateVersion || h.header_bytes != sizeof h)
      throw Error(TVS_EINVAL, "job state blob of another version");
    if (h.total_bytes != bytes) throw Error(TVS_EINVAL, "state blob size does not match its header");
    if (h.dtype != TVS_F32 && h.dtype != TVS_F64) throw Error(TVS_EINVAL, "state blob: unknown dtype");
    if (h.step < 1 || h.step > 3 || h.nsec < 1 || h.nsec > kMaxSections)
      throw Error(TVS_EINVAL, "state blob: bad step or section count");
    uint64_t sum = sizeof h;
    for (int k = 0; k < h.nsec; ++k) sum += h.sec_bytes[k];
    if (sum != h.total_bytes) throw Error(TVS_EINVAL, "state blob: section sizes do not add up");
    check_params(&h.prm, h.N2, h.N1);
    check_iters(&h.its);
    const size_t esz = h.dtype == TVS_F64 ? sizeof(double) : sizeof(float);
    if (h.sec_bytes[0] != esz * size_t(h.N2) * h.N1) throw Error(TVS_EINVAL, "state blob: d0 section size mismatch");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto j = std::make_unique<tvs_job>();
    j->ctx = ctx;
    j->uid = next_job_uid();
    j->dtype = tvs_dtype(h.dtype);
    j->N2 = h.N2;
    j->N1 = h.N1;
    j->prm = h.prm;
    j->lay = h.lay;
    j->its = h.its;
    const auto* b = static_cast<const unsigned char*>(buf);
    if (j->dtype == TVS_F32) {
      job_create<float>(ctx, j.get(), reinterpret_cast<const float*>(b + sizeof h), s, hipMemcpyHostToDevice);
      job_restore<float>(ctx, j.get(), h, b, s);
    } else {
      job_create<double>(ctx, j.get(), reinterpret_cast<const double*>(b + sizeof h), s, hipMemcpyHostToDevice);
      job_restore<double>(ctx, j.get(), h, b, s);
    }
    *out = j.release();
  });
}

size_t tvs_job_bytes(const tvs_job* job) {
  if (!job) return 0;
  return job->dtype == TVS_F64 ? job->d->bytes() : job->f->bytes();
}

int tvs_job_destroy(tvs_job* job) {
  return guarded([&] {
    if (!job) return;
    DeviceGuard dg(job->ctx->device);
    // launches of the job may still be queued on the caller's stream
    TVS_HIP(hipDeviceSynchronize());
    delete job;
  });
}

}  // extern "C"
