// C-ABI entry points of libtvs (include/tvs.h) and the host orchestration of
// Algorithm 2 for both TV-Stokes steps.
#include <chrono>
#include <cstdio>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

#include "../../include/tvs.h"
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
using ProbKey = std::tuple<int, int, double, int, int, int, int>;  // N2, N1, h, M2, M1, sy, sx

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

// Step 1 subdomains on Omega-tilde: s = the subdomain, a = grown by one
// row/column, b = grown by two (clipped at the grid)
void build_subs1(SubSet& ss, int n2, int n1, hipStream_t s) {
  ss.subs.clear();
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
  ss.subs_d.alloc(sizeof(SubDesc) * ss.subs.size());
  TVS_HIP(hipMemcpyAsync(ss.subs_d.p, ss.subs.data(), sizeof(SubDesc) * ss.subs.size(),
                         hipMemcpyHostToDevice, s));
  ss.sf.subs = ss.subs_d.as<SubDesc>();
  ss.sf.nsub = int(ss.subs.size());
  ss.sf.fr = fr;
  ss.sf.fp = align_pitch(fp);
  ss.sf.plane = (long long)fr * ss.sf.fp;
  // byte offsets inside one subdomain's four planes are 32-bit in the kernels
  if (4 * 8 * ss.sf.plane >= (1LL << 32)) throw Error(TVS_EINVAL, "layout: subdomain frame too large");
  ss.sf.ay = ss.ay;
  ss.sf.ax = ss.ax;
  build_theta_tables(ss, s);
}

// Step 2 subdomains: the Step-1 ones cut to Omega; a = grown by one
void build_subs2(SubSet& ss, int N2, int N1, hipStream_t s) {
  ss.subs.clear();
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
  ss.subs_d.alloc(sizeof(SubDesc) * ss.subs.size());
  TVS_HIP(hipMemcpyAsync(ss.subs_d.p, ss.subs.data(), sizeof(SubDesc) * ss.subs.size(),
                         hipMemcpyHostToDevice, s));
  ss.sf.subs = ss.subs_d.as<SubDesc>();
  ss.sf.nsub = int(ss.subs.size());
  ss.sf.fr = fr;
  ss.sf.fp = align_pitch(fp);
  ss.sf.plane = (long long)fr * ss.sf.fp;
  // byte offsets inside one subdomain's four planes are 32-bit in the kernels
  if (4 * 8 * ss.sf.plane >= (1LL << 32)) throw Error(TVS_EINVAL, "layout: subdomain frame too large");
  ss.sf.ay = ss.ay;
  ss.sf.ax = ss.ax;
  build_theta_tables(ss, s);
}

template <typename T>
struct Step1Problem {
  Grid g{};
  SubSet ss;
  bool plain = false;
  std::unique_ptr<GreenPlan<T>> global, local;
  DevBuf tau0, f1, r, zg, phig, p;         // global arrays on Omega-tilde
  DevBuf va, vb, vt, za, zb, zw, phi, omega;  // per-subdomain frames
  size_t bytes() const {
    size_t b = tau0.bytes + f1.bytes + r.bytes + zg.bytes + phig.bytes + p.bytes + va.bytes +
               vb.bytes + vt.bytes + za.bytes + zb.bytes + zw.bytes + phi.bytes + omega.bytes +
               global->bytes();
    if (local) b += local->bytes();
    return b;
  }
};

template <typename T>
struct Step2Problem {
  Grid g{};
  SubSet ss;
  DevBuf f2, p, u, xi, va, vb, b;
  size_t bytes() const {
    return f2.bytes + p.bytes + u.bytes + xi.bytes + va.bytes + vb.bytes + b.bytes;
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
  tvs::DevBuf partials;  // FP64 partial sums
  tvs::DevBuf scal;      // FP64 results (energies per sweep, gap)
  size_t scal_cap = 0;
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

void check_params(const tvs_params* prm, int N2, int N1) {
  if (!prm) throw Error(TVS_EINVAL, "params is NULL");
  if (N2 < 2 || N1 < 2) throw Error(TVS_EINVAL, "image must be at least 2 x 2");
  if ((long long)(N2 + 1) * (N1 + 1) > (1LL << 28)) throw Error(TVS_EINVAL, "image too large");
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

template <typename T>
Step1Problem<T>& get_step1(tvs_ctx* c, int N2, int N1, double h, const tvs_layout* l, hipStream_t s) {
  if (!l) throw Error(TVS_EINVAL, "layout is NULL");
  auto key = ProbKey{N2, N1, h, l->M2, l->M1, l->s_y, l->s_x};
  auto& mp = s1map<T>(c);
  auto it = mp.find(key);
  if (it != mp.end()) return *it->second;
  auto P = std::make_unique<Step1Problem<T>>();
  const int n2 = N2 + 1, n1 = N1 + 1;
  P->g = Grid{n2, n1, h};
  P->ss.ay = make_axis(n2, l->M2, l->s_y, "M2");
  P->ss.ax = make_axis(n1, l->M1, l->s_x, "M1");
  build_subs1(P->ss, n2, n1, s);
  P->plain = (l->M2 == 1 && l->M1 == 1);
  GreenTable& tab = get_table(c, n2, n1, h, s);
  P->global = std::make_unique<GreenPlan<T>>(tab, std::vector<std::array<int, 4>>{{0, 0, n2, n1}}, s);
  if (!P->plain) {
    std::vector<std::array<int, 4>> boxes;
    for (auto& d : P->ss.subs) boxes.push_back({d.i0, d.j0, d.bi, d.bj});
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
  auto& ref = *P;
  mp[key] = std::move(P);
  return ref;
}

template <typename T>
Step2Problem<T>& get_step2(tvs_ctx* c, int N2, int N1, double h, const tvs_layout* l, hipStream_t s) {
  if (!l) throw Error(TVS_EINVAL, "layout is NULL");
  auto key = ProbKey{N2, N1, h, l->M2, l->M1, l->s_y, l->s_x};
  auto& mp = s2map<T>(c);
  auto it = mp.find(key);
  if (it != mp.end()) return *it->second;
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
  auto& ref = *P;
  mp[key] = std::move(P);
  return ref;
}

Frame global_frame(const Grid& g) { return Frame{0, (long long)g.n2 * g.n1, g.n1}; }
Frame sub_frame(const SubFrames& sf, int planes) { return Frame{planes * sf.plane, sf.plane, sf.fp}; }

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
// Step 1: Algorithm 2 on Omega-tilde with the inner loop of Algorithm 5
// ---------------------------------------------------------------------------
template <typename T>
void run_step1(tvs_ctx* c, const T* d0, int N2, int N1, const tvs_params* prm, const tvs_layout* l,
               const tvs_iters* its, T* tau_out, tvs_stats* st, hipStream_t s) {
  Step1Problem<T>& P = get_step1<T>(c, N2, N1, prm->h, l, s);
  const Grid g = P.g;
  const SubFrames& sf = P.ss.sf;
  const T inv_h = T(1.0 / prm->h);
  StepScalars<T> cs{T(prm->t), inv_h, T(prm->delta), T(prm->alpha), T(alpha_hat_of(l))};
  const Frame gf = global_frame(g);
  const Frame f2p = sub_frame(sf, 2), f1p = sub_frame(sf, 1);
  const long long gpl = (long long)g.n2 * g.n1;
  Partials part = partials(c);
  double* e = scal(c, size_t(its->sweeps) + 3);

  // a1: tau_0 and f = delta^{-1} P_K tau_0
  launch_tau0<T>(d0, N2, N1, inv_h, dptr<T>(P.tau0), s);
  P.global->apply_div(dptr<T>(P.tau0), gf, dptr<T>(P.phig), Frame{0, 0, g.n1}, s);
  launch_f1<T>(dptr<T>(P.tau0), dptr<T>(P.phig), g, inv_h, T(1.0 / prm->delta), dptr<T>(P.f1), s);
  launch_fill<T>(dptr<T>(P.p), 4 * gpl, T(0), s);
  launch_fill<T>(dptr<T>(P.va), 4 * sf.plane * sf.nsub, T(0), s);
  launch_fill<T>(dptr<T>(P.vb), 4 * sf.plane * sf.nsub, T(0), s);
  GreenPlan<T>& lp = P.plain ? *P.global : *P.local;
  // in the single-domain case omega = f (theta = 1), staged into the frame layout
  if (P.plain) launch_sub_theta_p<T>(sf, g, dptr<T>(P.f1), 2, dptr<T>(P.omega), s);
  const T* omega = dptr<T>(P.omega);
  T* cur = dptr<T>(P.va);
  T* nxt = dptr<T>(P.vb);
  T* zcur = dptr<T>(P.za);  // vecdiv of cur (0 for v = 0)
  T* znxt = dptr<T>(P.zb);
  // z frames are written on the grown subdomains only; 0 elsewhere
  launch_fill<T>(zcur, 2 * sf.plane * sf.nsub, T(0), s);
  launch_fill<T>(znxt, 2 * sf.plane * sf.nsub, T(0), s);
  if (!P.plain) launch_fill<T>(dptr<T>(P.zw), 2 * sf.plane * sf.nsub, T(0), s);  // no zw when plain
  const double scale = std::sqrt(2.0 * double(gpl));
  KernelTimer* tm = &c->timer;
  const double px = P.ss.sub_px, esz = sizeof(T);
  const char* ltag = P.plain ? "s1_plain" : "s1_local";
  int done = 0;
  for (int n = 0; n < its->sweeps; ++n) {
    // a2: r^n = f - P_K vecdiv p^n (global, once per sweep) and D(p^n)
    launch_global_vecdiv<T>(dptr<T>(P.p), g, inv_h, dptr<T>(P.zg), s);
    P.global->apply_div(dptr<T>(P.zg), gf, dptr<T>(P.phig), Frame{0, 0, g.n1}, s, tm, "s1_global");
    launch_residual<T>(dptr<T>(P.f1), dptr<T>(P.zg), dptr<T>(P.phig), g, inv_h, dptr<T>(P.r), part, e + n, s);
    if (its->tol > 0 && n >= 1) {
      double hv[2];
      TVS_HIP(hipMemcpyAsync(hv, e + n - 1, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      TVS_HIP(hipStreamSynchronize(s));
      if (residual_of(hv[0], hv[1], scale) < its->tol) break;
    }
    if (!P.plain) {
      // omega_m = R_{m,+} r^n + LP_m(vecdiv(theta_m p^n))
      launch_sub_theta_p<T>(sf, g, dptr<T>(P.p), 4, dptr<T>(P.vt), s);
      launch_sub_vecdiv<T>(sf, g, inv_h, dptr<T>(P.vt), dptr<T>(P.zw), s);
      lp.apply_div(dptr<T>(P.zw), f2p, dptr<T>(P.phi), f1p, s, tm, ltag);
      launch_sub_omega<T>(sf, g, inv_h, dptr<T>(P.r), dptr<T>(P.zw), dptr<T>(P.phi), dptr<T>(P.omega), s);
    }
    // a3: inner iterations, warm-started from the previous sweep's q_m:
    // phi = Delta^+ div z on the Green box, the update of v, z' = vecdiv v'
    for (int nu = 0; nu < its->inner; ++nu) {
      lp.apply_div(zcur, f2p, dptr<T>(P.phi), f1p, s, tm, ltag);
      KernelTimer::time(tm, "s1_update", 13 * esz * px, s, [&] {
        launch_sub_update1<T>(sf, g, cs, cur, zcur, dptr<T>(P.phi), omega, nxt, s);
      });
      KernelTimer::time(tm, "s1_vecdiv", 6 * esz * px, s,
                        [&] { launch_sub_vecdiv<T>(sf, g, inv_h, nxt, znxt, s); });
      std::swap(cur, nxt);
      std::swap(zcur, znxt);
    }
    // a4: p^{n+1} = (1 - ahat) p^n + ahat sum_m q_m
    KernelTimer::time(tm, "s1_combine", 4 * esz * (2.0 * gpl + px), s,
                      [&] { launch_combine<T>(sf, g, 4, cs.ahat, cur, dptr<T>(P.p), s); });
    ++done;
  }
  // a5: tau = delta (f - P_K vecdiv p), D(p^S) and the gap
  launch_global_vecdiv<T>(dptr<T>(P.p), g, inv_h, dptr<T>(P.zg), s);
  P.global->apply_div(dptr<T>(P.zg), gf, dptr<T>(P.phig), Frame{0, 0, g.n1}, s);
  launch_residual<T>(dptr<T>(P.f1), dptr<T>(P.zg), dptr<T>(P.phig), g, inv_h, dptr<T>(P.r), part, e + done, s);
  launch_scale<T>(dptr<T>(P.r), 2 * gpl, T(prm->delta), tau_out, s);
  // tau already lies in K; projecting it once more is the identity in exact
  // arithmetic and removes the small divergence left by rounding, which the
  // IRV2 row integral of tau_2 would otherwise accumulate across the image
  P.global->apply_div(tau_out, gf, dptr<T>(P.phig), Frame{0, 0, g.n1}, s, tm, "s1_global");
  launch_f1<T>(tau_out, dptr<T>(P.phig), g, inv_h, T(1), tau_out, s);
  if (st) {
    launch_gap_tfs<T>(tau_out, dptr<T>(P.p), g, inv_h, part, e + its->sweeps + 1, s);
    std::vector<double> hv(size_t(its->sweeps) + 2);
    TVS_HIP(hipMemcpyAsync(hv.data(), e, sizeof(double) * hv.size(), hipMemcpyDeviceToHost, s));
    TVS_HIP(hipStreamSynchronize(s));
    st->sweeps_done = done;
    st->energy = hv[done];
    st->residual = done >= 1 ? residual_of(hv[done - 1], hv[done], scale) : 0.0;
    st->gap = hv[its->sweeps + 1];
    if (!std::isfinite(st->energy) || !std::isfinite(st->gap))
      throw Error(TVS_ENONFINITE, "step 1: non-finite energy or gap");
  }
}

// ---------------------------------------------------------------------------
// Step 2: Algorithm 2 on Omega with the inner loop of Algorithm 3
// ---------------------------------------------------------------------------
template <typename T>
void run_step2(tvs_ctx* c, const T* d0, const T* tau, int N2, int N1, const tvs_params* prm,
               const tvs_layout* l, const tvs_iters* its, T* d_out, tvs_stats* st, hipStream_t s) {
  Step2Problem<T>& P = get_step2<T>(c, N2, N1, prm->h, l, s);
  const Grid g = P.g;
  const SubFrames& sf = P.ss.sf;
  const T inv_h = T(1.0 / prm->h);
  StepScalars<T> cs{T(prm->t), inv_h, T(prm->delta), T(prm->alpha), T(alpha_hat_of(l))};
  const long long gpl = (long long)N2 * N1;
  Partials part = partials(c);
  double* e = scal(c, size_t(its->sweeps) + 3);
  const bool irv1 = prm->variant == TVS_IRV1;

  // a6: the bridge from tau to the Step-2 data
  if (irv1) {
    launch_xi<T>(tau, N2, N1, T(prm->eps), dptr<T>(P.xi), s);
    launch_irv1_data<T>(d0, dptr<T>(P.xi), g, inv_h, T(prm->alpha), dptr<T>(P.f2), s);
  } else {
    launch_bridge_irv2<T>(tau, d0, N2, N1, T(prm->h), T(prm->alpha), dptr<T>(P.f2), s);
  }
  launch_fill<T>(dptr<T>(P.p), 2 * gpl, T(0), s);
  launch_fill<T>(dptr<T>(P.va), 2 * sf.plane * sf.nsub, T(0), s);
  launch_fill<T>(dptr<T>(P.vb), 2 * sf.plane * sf.nsub, T(0), s);
  T* cur = dptr<T>(P.va);
  T* nxt = dptr<T>(P.vb);
  const double scale = std::sqrt(double(gpl));
  KernelTimer* tm = &c->timer;
  const double px = P.ss.sub_px, esz = sizeof(T);
  int done = 0;
  for (int n = 0; n < its->sweeps; ++n) {
    launch_energy_rof<T>(dptr<T>(P.p), dptr<T>(P.f2), g, inv_h, part, e + n, s);
    if (its->tol > 0 && n >= 1) {
      double hv[2];
      TVS_HIP(hipMemcpyAsync(hv, e + n - 1, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      TVS_HIP(hipStreamSynchronize(s));
      if (residual_of(hv[0], hv[1], scale) < its->tol) break;
    }
    // a7: b_m = div((1 - theta_m) p^n) - f near the subdomain
    launch_sub2_prologue<T>(sf, g, inv_h, dptr<T>(P.p), dptr<T>(P.f2), dptr<T>(P.b), s);
    // a8: inner iterations
    for (int nu = 0; nu < its->inner; ++nu) {
      KernelTimer::time(tm, "s2_update", 5 * esz * px, s,
                        [&] { launch_sub2_update<T>(sf, g, cs, cur, dptr<T>(P.b), nxt, s); });
      std::swap(cur, nxt);
    }
    // a9: combine
    KernelTimer::time(tm, "s2_combine", 2 * esz * (2.0 * gpl + px), s,
                      [&] { launch_combine<T>(sf, g, 2, cs.ahat, cur, dptr<T>(P.p), s); });
    ++done;
  }
  launch_energy_rof<T>(dptr<T>(P.p), dptr<T>(P.f2), g, inv_h, part, e + done, s);
  if (irv1)
    launch_irv1_image<T>(d0, dptr<T>(P.p), dptr<T>(P.xi), g, inv_h, T(1.0 / prm->alpha), d_out, s);
  else
    launch_irv2_image<T>(d0, dptr<T>(P.p), g, inv_h, T(1.0 / prm->alpha), d_out, s);
  if (st) {
    launch_primal_rof<T>(dptr<T>(P.p), dptr<T>(P.f2), g, inv_h, T(1.0 / prm->alpha), dptr<T>(P.u), s);
    launch_gap_rof<T>(dptr<T>(P.u), dptr<T>(P.p), g, inv_h, part, e + its->sweeps + 1, s);
    std::vector<double> hv(size_t(its->sweeps) + 2);
    TVS_HIP(hipMemcpyAsync(hv.data(), e, sizeof(double) * hv.size(), hipMemcpyDeviceToHost, s));
    TVS_HIP(hipStreamSynchronize(s));
    st->sweeps_done = done;
    st->energy = hv[done];
    st->residual = done >= 1 ? residual_of(hv[done - 1], hv[done], scale) : 0.0;
    st->gap = hv[its->sweeps + 1];
    if (!std::isfinite(st->energy) || !std::isfinite(st->gap))
      throw Error(TVS_ENONFINITE, "step 2: non-finite energy or gap");
  }
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

}  // namespace
}  // namespace tvs

using namespace tvs;

extern "C" {

int tvs_ctx_create(int device, tvs_ctx** out) {
  return guarded([&] {
    if (!out) throw Error(TVS_EINVAL, "out is NULL");
    int n = 0;
    TVS_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) throw Error(TVS_EINVAL, "no such HIP device");
    DeviceGuard dg(device);
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

}  // extern "C"
