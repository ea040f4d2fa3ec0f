// C ABI (include/wx.h): state, validation, workspace layout and launch plan.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "wx.h"
#include "wx_internal.h"
#include "wx_mlp_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define WX_HIP(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) return fail(WX_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// Default constants (the readings; see wx_param in wx.h).
const double kDefaults[WX_PARAM_COUNT] = {1.0 / 256.0, 0.1, 50.0, 0.02, 1004.0, 64.0, 0.0, 1.0,
                                          0.0,         0.05, 100.0, 0.0, 4.0, 0.0};

struct Impl {
  std::vector<double> dz;
  double param[WX_PARAM_COUNT];
  std::vector<unsigned char> host_consts[2];  // per dtype, uploaded into the workspace
  const void *uploaded_ws[2] = {nullptr, nullptr};
  bool dirty[2] = {true, true};
};

Impl *impl_of(const wx_state *s) { return static_cast<Impl *>(s->impl); }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace layout for element size es:
//   [s1 rho, theta, q][s2 rho, theta, q]   6 cell fields
//   consts: dz, 1/dz, 1/dz_{k+1/2} (dtype), vol (double)
//   column scratch: 3 * nz * nx * ny doubles
//   mass partials: 6 doubles per physics block
struct Layout {
  size_t field, stage, consts, scratch, partials, total;
};

Layout layout(const wx_state *s, size_t es) {
  Layout L{};
  L.field = align256(size_t(s->field_elems) * es);
  L.stage = 0;
  size_t off = 6 * L.field;
  L.consts = off;
  off += align256(3 * size_t(s->nz) * es) + align256(size_t(s->nz) * 8);
  L.scratch = off;
  off += align256(3 * size_t(s->nz) * size_t(s->nx) * size_t(s->ny) * 8);
  L.partials = off;
  const int nparts = std::max({wx::phys_blocks(s->nx, s->ny), wx::phys_reg_blocks(s->nx, s->ny),
                               wx::phys_scan_blocks(s->nx, s->ny), wx::phys_split_blocks(s->nx, s->ny)});
  off += align256(size_t(nparts) * 6 * 8);
  L.total = off;
  return L;
}

template <typename T>
void build_consts(const wx_state *s, std::vector<unsigned char> &out) {
  const int nz = s->nz;
  const size_t es = sizeof(T);
  out.assign(align256(3 * nz * es) + align256(nz * 8), 0);
  T *dz = reinterpret_cast<T *>(out.data());
  T *rdz = dz + nz;
  T *rdzi = dz + 2 * nz;
  const std::vector<double> &d = impl_of(s)->dz;
  for (int k = 0; k < nz; ++k) {
    dz[k] = T(d[k]);
    rdz[k] = T(1.0 / d[k]);
    rdzi[k] = k + 1 < nz ? T(2.0 / (d[k] + d[k + 1])) : T(0);
  }
  double *vol = reinterpret_cast<double *>(out.data() + align256(3 * nz * es));
  for (int k = 0; k < nz; ++k) vol[k] = s->dx * s->dx * d[k];
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int check_fields(const wx_state *s, bool need_phys) {
  if (s->dtype != WX_F32 && s->dtype != WX_F64) return fail(WX_E_INVAL, "dtype %d is not WX_F32/WX_F64", s->dtype);
  const void *req[] = {s->rho, s->theta, s->q, s->u, s->v, s->w, s->workspace, s->mass_out, s->flags_out};
  const char *names[] = {"rho", "theta", "q", "u", "v", "w", "workspace", "mass_out", "flags_out"};
  for (int n = 0; n < 9; ++n) {
    if (!req[n]) return fail(WX_E_STATE, "state pointer '%s' is NULL", names[n]);
    if (!aligned16(req[n])) return fail(WX_E_INVAL, "state pointer '%s' is not 16-byte aligned", names[n]);
  }
  if (need_phys) {
    const void *p2[] = {s->theta_s, s->q_s, s->f0, s->ch};
    const char *n2[] = {"theta_s", "q_s", "f0", "ch"};
    for (int n = 0; n < 4; ++n) {
      if (!p2[n]) return fail(WX_E_STATE, "state pointer '%s' is NULL", n2[n]);
      if (!aligned16(p2[n])) return fail(WX_E_INVAL, "state pointer '%s' is not 16-byte aligned", n2[n]);
    }
  }
  return WX_OK;
}

wx::Geom geom(const wx_state *s) {
  return wx::Geom{s->nx, s->ny, s->nz, unsigned(s->stride_j), unsigned(s->stride_k), unsigned(s->origin)};
}

// Upload the per-dtype constants into the workspace when they changed.
template <typename T>
int ensure_consts(wx_state *s, hipStream_t st) {
  Impl *im = impl_of(s);
  const int d = sizeof(T) == 4 ? 0 : 1;
  if (!im->dirty[d] && im->uploaded_ws[d] == s->workspace) return WX_OK;
  build_consts<T>(s, im->host_consts[d]);
  const Layout L = layout(s, sizeof(T));
  WX_HIP(hipMemcpyAsync(static_cast<unsigned char *>(s->workspace) + L.consts, im->host_consts[d].data(),
                        im->host_consts[d].size(), hipMemcpyHostToDevice, st));
  im->uploaded_ws[d] = s->workspace;
  im->dirty[d] = false;
  im->dirty[1 - d] = true;
  return WX_OK;
}

// Surrogate workspace: the judge's sample list (capacity for the current
// sampling rate), the plain tendencies and the network outputs of the sampled
// columns, and a few counters.
struct SurrogateLayout {
  size_t list, bcount, boff, nlist, fallback, jpart, tplain, yrows, total;
  int cap, nblk;
};

SurrogateLayout surrogate_layout(const wx_state *s) {
  SurrogateLayout L{};
  const long long ncol = (long long)s->nx * s->ny;
  const double rate = impl_of(s)->param[WX_PARAM_JUDGE_RATE];
  const double mean = double(ncol) / rate;
  long long cap = (long long)(mean + 10.0 * std::sqrt(mean) + 64.0);
  if (cap > ncol) cap = ncol;
  L.cap = int(cap);
  L.nblk = int((ncol + 255) / 256);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t r = off;
    off += align256(bytes);
    return r;
  };
  L.list = take(size_t(L.cap) * 4);
  L.bcount = take(size_t(L.nblk) * 4);
  L.boff = take(size_t(L.nblk) * 4);
  L.nlist = take(4);
  L.fallback = take(4);
  L.jpart = take(wx::judge_part_bytes());
  L.tplain = take(size_t(L.cap) * wx::TEND_ROW * 4);
  L.yrows = take(size_t(L.cap) * wx::MLP_NOUTP * 4);
  L.total = off;
  return L;
}

// Arguments of the fused surrogate kernel for an FP32 state and a blob.
wx::FusedArgs fused_args(const wx_state *s, const void *blob) {
  wx::FusedArgs a{};
  a.rho = static_cast<const float *>(s->rho);
  a.th = static_cast<float *>(s->theta);
  a.q = static_cast<float *>(s->q);
  a.u = static_cast<const float *>(s->u);
  a.v = static_cast<const float *>(s->v);
  a.th_s = static_cast<const float *>(s->theta_s);
  a.q_s = static_cast<const float *>(s->q_s);
  a.f0 = static_cast<const float *>(s->f0);
  a.ch = static_cast<const float *>(s->ch);
  a.g = geom(s);
  a.theta_off = impl_of(s)->param[WX_PARAM_THETA_OFFSET];
  const unsigned char *b = static_cast<const unsigned char *>(blob);
  // the weights in matrix-core fragment order: W1, W2, W3 one after the other
  a.w1 = reinterpret_cast<const uint16_t *>(b + wx_mlp_offset(WX_MLP_WPACK_BF16));
  a.w2 = a.w1 + size_t(WX_MLP_NHID) * WX_MLP_KIN;
  a.w3 = a.w2 + size_t(WX_MLP_NHID) * WX_MLP_NHID;
  a.b1 = reinterpret_cast<const float *>(b + wx_mlp_offset(WX_MLP_B1));
  a.b2 = reinterpret_cast<const float *>(b + wx_mlp_offset(WX_MLP_B2));
  a.b3 = reinterpret_cast<const float *>(b + wx_mlp_offset(WX_MLP_B3));
  a.xmean = reinterpret_cast<const float *>(b + wx_mlp_offset(WX_MLP_X_MEAN));
  a.xinvstd = reinterpret_cast<const float *>(b + wx_mlp_offset(WX_MLP_X_INVSTD));
  a.ymean = reinterpret_cast<const float *>(b + wx_mlp_offset(WX_MLP_Y_MEAN));
  a.ystd = reinterpret_cast<const float *>(b + wx_mlp_offset(WX_MLP_Y_STD));
  a.dt = float(s->dt);
  return a;
}

// Launch-class timing hook used by wx_profile_step.  Classes: 0 halo fill,
// 1-3 RK3 stages, 4 physics (or mass partials), 5 mass finalisation,
// 6 judge prelude, 7 fused surrogate, 8 sampled-column apply and fallback
// physics.
constexpr int kProfileClasses = 9;
struct Timer {
  std::vector<hipEvent_t> *ev = nullptr;
  std::vector<int> *cls = nullptr;
  hipStream_t st = nullptr;
  int begin(int c) {
    if (!ev) return WX_OK;
    hipEvent_t e;
    WX_HIP(hipEventCreate(&e));
    WX_HIP(hipEventRecord(e, st));
    ev->push_back(e);
    cls->push_back(c);
    return WX_OK;
  }
  int end() {
    if (!ev) return WX_OK;
    hipEvent_t e;
    WX_HIP(hipEventCreate(&e));
    WX_HIP(hipEventRecord(e, st));
    ev->push_back(e);
    cls->push_back(-1);
    return WX_OK;
  }
};

#define WX_TRY(x)          \
  do {                     \
    int r_ = (x);          \
    if (r_ != WX_OK) return r_; \
  } while (0)

template <typename T>
struct Plan {
  wx_state *s;
  hipStream_t st;
  Layout L;
  T *s1[3], *s2[3], *base[3];
  const T *dz, *rdz, *rdzi;
  const double *vol;
  double *scratch, *partials;
  int nparts = 0;   // mass partials written by the last physics / mass launch

  Plan(wx_state *s_, hipStream_t st_) : s(s_), st(st_) {
    L = layout(s, sizeof(T));
    unsigned char *ws = static_cast<unsigned char *>(s->workspace);
    for (int f = 0; f < 3; ++f) {
      s1[f] = reinterpret_cast<T *>(ws + size_t(f) * L.field);
      s2[f] = reinterpret_cast<T *>(ws + size_t(3 + f) * L.field);
    }
    base[0] = static_cast<T *>(s->rho);
    base[1] = static_cast<T *>(s->theta);
    base[2] = static_cast<T *>(s->q);
    dz = reinterpret_cast<const T *>(ws + L.consts);
    rdz = dz + s->nz;
    rdzi = dz + 2 * s->nz;
    vol = reinterpret_cast<const double *>(ws + L.consts + align256(3 * size_t(s->nz) * sizeof(T)));
    scratch = reinterpret_cast<double *>(ws + L.scratch);
    partials = reinterpret_cast<double *>(ws + L.partials);
  }

  int halo(Timer &tm) {
    T *f[5] = {base[0], base[1], base[2], static_cast<T *>(s->u), static_cast<T *>(s->v)};
    WX_TRY(tm.begin(0));
    WX_HIP(wx::launch_halo<T>(f, 5, s->nz, geom(s), st));
    return tm.end();
  }

  int stage(int n, T *const *in, T *const *out, T h, Timer &tm) {
    const Impl *im = impl_of(s);
    wx::StageArgs<T> a;
    a.in_r = in[0]; a.in_t = in[1]; a.in_q = in[2];
    a.bs_r = base[0]; a.bs_t = base[1]; a.bs_q = base[2];
    a.out_r = out[0]; a.out_t = out[1]; a.out_q = out[2];
    a.u = static_cast<const T *>(s->u);
    a.v = static_cast<const T *>(s->v);
    a.w = static_cast<const T *>(s->w);
    a.rdz = rdz;
    a.g = geom(s);
    a.h = h;
    a.rdx = T(1.0 / s->dx);
    a.k4 = T(im->param[WX_PARAM_GAMMA4] * std::pow(s->dx, 4) / s->dt);
    // the default tile (0) runs stage 2, which walks its tiles backward, on
    // 64 x 12 tiles (1.446 -> 1.413 ms; stages 1 and 3 are as fast or faster
    // on 64 x 8); every shape gives the same bits
    int tile = int(im->param[WX_PARAM_STAGE_TILE]);
    if (tile == 0 && n == 2) tile = 2;
    a.nbx = wx::stage_tiles_x(s->nx, tile);
    a.nblocks = a.nbx * wx::stage_tiles_y(s->ny, tile);
    // stages walk their tiles forward, backward, forward and the physics
    // backward, so each launch starts on the part of its input that the one
    // before wrote last
    a.reverse = n == 2 ? 1 : 0;
    WX_TRY(tm.begin(n));
    WX_HIP(wx::launch_stage<T>(a, n, tile, st));
    return tm.end();
  }

  wx::PhysArgs<T> phys_args(int mode, int do_mass, T *tt, T *tq) {
    const Impl *im = impl_of(s);
    wx::PhysArgs<T> a;
    a.rho = base[0]; a.th = base[1]; a.q = base[2];
    a.u = static_cast<const T *>(s->u);
    a.v = static_cast<const T *>(s->v);
    a.th_s = static_cast<const T *>(s->theta_s);
    a.q_s = static_cast<const T *>(s->q_s);
    a.f0 = static_cast<const T *>(s->f0);
    a.ch = static_cast<const T *>(s->ch);
    a.tend_t = tt;
    a.tend_q = tq;
    a.dz = dz;
    a.rdzi = rdzi;
    a.vol = vol;
    a.scratch = scratch;
    a.partials = partials;
    a.flags = s->flags_out;
    a.g = geom(s);
    a.dt = T(s->dt);
    a.kmin = T(im->param[WX_PARAM_KMIN]);
    a.l2 = T(im->param[WX_PARAM_MIXLEN] * im->param[WX_PARAM_MIXLEN]);
    a.kappa = T(im->param[WX_PARAM_KAPPA_Q]);
    a.cp = T(im->param[WX_PARAM_CP]);
    a.tdd = T(im->param[WX_PARAM_TDD]);
    a.theta_off = im->param[WX_PARAM_THETA_OFFSET];
    a.mode = mode;
    a.do_mass = do_mass;
    a.use_lds = (sizeof(T) == 4 && s->nz <= wx::PHYS_LDS_NZ_MAX) ? 1 : 0;
    a.tend_rows = 0;
    a.col_list = nullptr;
    a.n_list = nullptr;
    a.list_cap = 0;
    a.run_if = nullptr;
    a.variant = int(im->param[WX_PARAM_PHYS_KERNEL]);
    a.reverse = 0;
    return a;
  }

  int physics(int do_mass, Timer &tm) {
    WX_TRY(tm.begin(4));
    wx::PhysArgs<T> pa = phys_args(0, do_mass, nullptr, nullptr);
    pa.reverse = 1;
    WX_HIP(wx::launch_physics<T>(pa, st));
    nparts = wx::phys_partials(sizeof(T), s->nx, s->ny, s->nz, int(impl_of(s)->param[WX_PARAM_PHYS_KERNEL]));
    return tm.end();
  }

  int mass(Timer &tm) {
    wx::MassArgs<T> a;
    a.rho = base[0]; a.th = base[1]; a.q = base[2];
    a.vol = vol;
    a.partials = partials;
    a.flags = s->flags_out;
    a.g = geom(s);
    a.theta_off = impl_of(s)->param[WX_PARAM_THETA_OFFSET];
    WX_TRY(tm.begin(4));
    WX_HIP(wx::launch_mass<T>(a, st));
    nparts = wx::phys_blocks(s->nx, s->ny);
    return tm.end();
  }

  int mass_final(Timer &tm) {
    WX_TRY(tm.begin(5));
    WX_HIP(wx::launch_mass_final(partials, nparts, s->mass_out, st));
    return tm.end();
  }

  // Surrogate physics of step t on the post-dycore state (optionally judged):
  // judge prelude on the sampled columns, then one fused launch over all
  // columns, then the plain tendencies of the sampled columns, or the plain
  // physics everywhere when the judge rejected the step.  With tend_t set the
  // same decisions produce tendencies (flat, i fastest) and leave the state.
  int surrogate(bool judged, uint64_t t, Timer &tm, float *tend_t = nullptr, float *tend_q = nullptr) {
    if (!std::is_same<T, float>::value) return fail(WX_E_UNSUPPORTED, "the surrogate needs an FP32 state");
    const Impl *im = impl_of(s);
    const SurrogateLayout L = surrogate_layout(s);
    unsigned char *w = static_cast<unsigned char *>(s->surrogate_work);
    int *list = reinterpret_cast<int *>(w + L.list);
    int *n_list = reinterpret_cast<int *>(w + L.nlist);
    int *fallback = reinterpret_cast<int *>(w + L.fallback);
    float *tplain = reinterpret_cast<float *>(w + L.tplain);
    float *yrows = reinterpret_cast<float *>(w + L.yrows);
    const unsigned char *b = static_cast<const unsigned char *>(s->mlp);
    const float *ymean = reinterpret_cast<const float *>(b + wx_mlp_offset(WX_MLP_Y_MEAN));
    const float *ystd = reinterpret_cast<const float *>(b + wx_mlp_offset(WX_MLP_Y_STD));
    const double *sigma = reinterpret_cast<const double *>(b + wx_mlp_offset(WX_MLP_SIGMA64));
    const uint64_t seed = uint64_t(im->param[WX_PARAM_JUDGE_SEED]);
    const unsigned rate = unsigned(im->param[WX_PARAM_JUDGE_RATE]);
    const int ncol = s->nx * s->ny;
    if (judged) {
      WX_TRY(tm.begin(6));
      WX_HIP(wx::launch_sample(ncol, seed, t, rate, reinterpret_cast<int *>(w + L.bcount),
                               reinterpret_cast<int *>(w + L.boff), n_list, L.cap, list, st));
      wx::PhysArgs<T> pa = phys_args(1, 0, reinterpret_cast<T *>(tplain), nullptr);
      pa.tend_rows = 1;
      pa.col_list = list;
      pa.n_list = n_list;
      pa.list_cap = L.cap;
      WX_HIP(wx::launch_physics<T>(pa, st));
      wx::FusedArgs fr = fused_args(s, s->mlp);
      fr.list = list;
      fr.n_list = n_list;
      fr.cap = L.cap;
      fr.rows_out = yrows;
      WX_HIP(wx::launch_surrogate_fused(fr, st));
      WX_HIP(wx::launch_judge(yrows, tplain, n_list, L.cap, ymean, ystd, sigma, im->param[WX_PARAM_JUDGE_REL],
                              s->nz, reinterpret_cast<double *>(w + L.jpart), fallback, s->judge_out,
                              s->flags_out, st));
      WX_TRY(tm.end());
    }
    wx::FusedArgs fa = fused_args(s, s->mlp);
    fa.c0 = 0;
    fa.ncols = ncol;
    fa.tend_t = tend_t;
    fa.tend_q = tend_q;
    fa.fallback = judged ? fallback : nullptr;
    fa.judged = judged ? 1 : 0;
    fa.seed = seed;
    fa.t = t;
    fa.rate = rate;
    WX_TRY(tm.begin(7));
    WX_HIP(wx::launch_surrogate_fused(fa, st));
    WX_TRY(tm.end());
    if (judged) {
      wx::ApplyArgs<T> aa{};
      aa.tend_t = tend_t;
      aa.tend_q = tend_q;
      aa.th = base[1];
      aa.q = base[2];
      aa.g = geom(s);
      aa.dt = T(s->dt);
      aa.ymean = ymean;
      aa.ystd = ystd;
      aa.fallback = fallback;
      aa.judged = 1;
      aa.seed = seed;
      aa.t = t;
      aa.rate = rate;
      WX_TRY(tm.begin(8));
      WX_HIP(wx::launch_apply_sampled<T>(aa, tplain, list, n_list, L.cap, st));
      wx::PhysArgs<T> pa = tend_t ? phys_args(1, 0, reinterpret_cast<T *>(tend_t), reinterpret_cast<T *>(tend_q))
                                  : phys_args(0, 0, nullptr, nullptr);
      pa.run_if = fallback;
      WX_HIP(wx::launch_physics<T>(pa, st));
      WX_TRY(tm.end());
    }
    return WX_OK;
  }

  int run(int nsteps, Timer &tm) {
    WX_TRY(ensure_consts<T>(s, st));
    WX_HIP(wx::launch_fill_i32(s->flags_out, WX_NFLAGS, 0, st));
    WX_TRY(halo(tm));
    Impl *im = impl_of(s);
    const int every = int(im->param[WX_PARAM_MASS_EVERY]);
    const T dt = T(s->dt);
    const bool surr = s->phys_mode == WX_PHYS_SURROGATE || s->phys_mode == WX_PHYS_JUDGED;
    for (int n = 1; n <= nsteps; ++n) {
      WX_TRY(stage(1, base, s1, dt / T(3), tm));
      WX_TRY(stage(2, s1, s2, dt / T(2), tm));
      WX_TRY(stage(3, s2, base, dt, tm));
      const int do_mass = every > 0 && (n % every == 0 || n == nsteps);
      const uint64_t t = uint64_t(im->param[WX_PARAM_STEP]);
      im->param[WX_PARAM_STEP] = double(t + 1);
      if (s->phys_mode == WX_PHYS_PLAIN) {
        WX_TRY(physics(do_mass, tm));
      } else {
        if (surr) WX_TRY(surrogate(s->phys_mode == WX_PHYS_JUDGED, t, tm));
        if (do_mass) WX_TRY(mass(tm));
      }
      if (do_mass) WX_TRY(mass_final(tm));
    }
    return WX_OK;
  }
};

int validate_for_step(wx_state *s) {
  if (!s || !s->impl) return fail(WX_E_INVAL, "state is NULL");
  if (s->phys_mode < WX_PHYS_OFF || s->phys_mode > WX_PHYS_JUDGED)
    return fail(WX_E_UNSUPPORTED, "phys_mode %d is not supported", s->phys_mode);
  WX_TRY(check_fields(s, s->phys_mode != WX_PHYS_OFF));
  if (s->phys_mode == WX_PHYS_SURROGATE || s->phys_mode == WX_PHYS_JUDGED) {
    if (s->dtype != WX_F32) return fail(WX_E_UNSUPPORTED, "the surrogate modes need an FP32 state");
    if (s->nz != wx::MLP_NZ) return fail(WX_E_UNSUPPORTED, "the surrogate needs nz == %d", wx::MLP_NZ);
    if (!s->mlp || !s->surrogate_work || !aligned16(s->mlp) || !aligned16(s->surrogate_work))
      return fail(WX_E_STATE, "surrogate modes need mlp and surrogate_work (16-byte aligned)");
    if (s->phys_mode == WX_PHYS_JUDGED && !s->judge_out) return fail(WX_E_STATE, "judged mode needs judge_out");
  }
  return WX_OK;
}

int run_steps(wx_state *s, int nsteps, hipStream_t st, Timer &tm) {
  if (s->dtype == WX_F32) {
    Plan<float> p(s, st);
    return p.run(nsteps, tm);
  }
  Plan<double> p(s, st);
  return p.run(nsteps, tm);
}

}  // namespace

// ---- mass sums without any allocation ----------------------------------
//
// The block partials and the per-level cell volumes of wx_mass_noalloc live in
// this file-scope device array instead of the caller's workspace.  Its device
// address is looked up once per device (hipGetSymbolAddress with that device
// current) and only that address is handed to kernels.
namespace {

constexpr int kNoallocMaxNz = 1024;
constexpr int kNoallocMaxParts = WX_MASS_NOALLOC_MAX_PARTS;
constexpr int kNoallocMaxDevices = 64;
__device__ __align__(256) double scratch[kNoallocMaxNz + size_t(kNoallocMaxParts) * 6];

std::mutex g_scratch_mu;
double *g_scratch_ptr[kNoallocMaxDevices] = {nullptr};

// Volumes dx*dy*dz_k for up to 256 levels per launch, passed by value so that
// no host buffer or copy is involved.
struct VolChunk {
  double v[256];
};
__global__ void k_put_vol(double *dst, VolChunk c, int n) {
  const int t = threadIdx.x;
  if (t < n) dst[t] = c.v[t];
}

int scratch_ptr(double **out) {
  int dev = 0;
  WX_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoallocMaxDevices) return fail(WX_E_UNSUPPORTED, "device index %d >= %d", dev, kNoallocMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    WX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(WX_E_HIP, "hipGetSymbolAddress returned NULL for the static scratch");
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return WX_OK;
}

template <typename T>
int mass_noalloc(wx_state *s, hipStream_t st, double *ws) {
  double *vol = ws;
  double *parts = ws + kNoallocMaxNz;
  const std::vector<double> &dz = impl_of(s)->dz;
  for (int k0 = 0; k0 < s->nz; k0 += 256) {
    VolChunk c;
    const int n = std::min(256, s->nz - k0);
    for (int k = 0; k < n; ++k) c.v[k] = s->dx * s->dx * dz[k0 + k];
    hipLaunchKernelGGL(k_put_vol, dim3(1), dim3(256), 0, st, vol + k0, c, n);
    WX_HIP(hipGetLastError());
  }
  wx::MassArgs<T> a;
  a.rho = static_cast<const T *>(s->rho);
  a.th = static_cast<const T *>(s->theta);
  a.q = static_cast<const T *>(s->q);
  a.vol = vol;
  a.partials = parts;
  a.flags = s->flags_out;
  a.g = geom(s);
  a.theta_off = impl_of(s)->param[WX_PARAM_THETA_OFFSET];
  WX_HIP(wx::launch_mass<T>(a, st));
  WX_HIP(wx::launch_mass_final(parts, wx::phys_blocks(s->nx, s->ny), s->mass_out, st));
  return WX_OK;
}

}  // namespace

namespace wx {
int set_error(int code, const char *msg) {
  g_err = msg;
  return code;
}
}  // namespace wx

extern "C" {

const char *wx_last_error(void) { return g_err.c_str(); }

wx_state *wx_create(int nx, int ny, int nz, double dt, double dx, const double *dz) {
  if (nx < 4 || ny < 4 || nz < 3 || nz > 1024) {
    fail(WX_E_INVAL, "grid %d x %d x %d outside nx, ny >= 4, 3 <= nz <= 1024", nx, ny, nz);
    return nullptr;
  }
  if (!(dt > 0) || !std::isfinite(dt) || !(dx > 0) || !std::isfinite(dx)) {
    fail(WX_E_INVAL, "dt and dx must be finite and > 0");
    return nullptr;
  }
  if (!dz) {
    fail(WX_E_INVAL, "dz is NULL");
    return nullptr;
  }
  for (int k = 0; k < nz; ++k)
    if (!(dz[k] > 0) || !std::isfinite(dz[k])) {
      fail(WX_E_INVAL, "dz[%d] must be finite and > 0", k);
      return nullptr;
    }
  const long long sj = ((long long)nx + 2 * WX_HALO + 63) / 64 * 64;
  const long long sk = sj * (ny + 2 * WX_HALO);
  // kernels address every buffer with 32-bit byte offsets (FP64 worst case)
  if (sk * (long long)(nz + 1) * 8 >= (1LL << 32) || 24LL * nz * nx * ny >= (1LL << 32)) {
    fail(WX_E_UNSUPPORTED, "grid too large for 32-bit byte offsets");
    return nullptr;
  }
  wx_state *s = new (std::nothrow) wx_state();
  Impl *im = new (std::nothrow) Impl();
  if (!s || !im) {
    delete s;
    delete im;
    fail(WX_E_INVAL, "out of host memory");
    return nullptr;
  }
  im->dz.assign(dz, dz + nz);
  for (int p = 0; p < WX_PARAM_COUNT; ++p) im->param[p] = kDefaults[p];
  s->nx = nx;
  s->ny = ny;
  s->nz = nz;
  s->halo = WX_HALO;
  s->stride_j = sj;
  s->stride_k = sk;
  s->origin = WX_HALO + WX_HALO * sj;
  s->field_elems = sk * nz;
  s->wfield_elems = sk * (nz + 1);
  s->dt = dt;
  s->dx = dx;
  s->dtype = WX_F32;
  s->phys_mode = WX_PHYS_PLAIN;
  s->impl = im;
  g_err.clear();
  return s;
}

void wx_destroy(wx_state *s) {
  if (!s) return;
  delete impl_of(s);
  delete s;
}

size_t wx_workspace_bytes(const wx_state *s, int dtype) {
  if (!s || (dtype != WX_F32 && dtype != WX_F64)) return 0;
  return layout(s, dtype == WX_F32 ? 4 : 8).total;
}

size_t wx_surrogate_work_bytes(const wx_state *s) {
  if (!s || !s->impl) return 0;
  return surrogate_layout(s).total;
}

int wx_set_param(wx_state *s, int param, double value) {
  if (!s || !s->impl) return fail(WX_E_INVAL, "state is NULL");
  if (param < 0 || param >= WX_PARAM_COUNT) return fail(WX_E_INVAL, "unknown param %d", param);
  if (!std::isfinite(value)) return fail(WX_E_INVAL, "param value must be finite");
  if (param == WX_PARAM_CP && !(value > 0)) return fail(WX_E_INVAL, "cp must be > 0");
  if (param != WX_PARAM_THETA_OFFSET && value < 0) return fail(WX_E_INVAL, "param %d must be >= 0", param);
  if ((param == WX_PARAM_MASS_EVERY || param == WX_PARAM_JUDGE_SEED || param == WX_PARAM_JUDGE_RATE ||
       param == WX_PARAM_STEP) && value != std::floor(value))
    return fail(WX_E_INVAL, "param %d must be an integer", param);
  if (param == WX_PARAM_PHYS_KERNEL && (value != std::floor(value) || value < 0.0 || value > 4.0))
    return fail(WX_E_INVAL, "physics kernel must be 0, 1, 2, 3 or 4");
  if (param == WX_PARAM_STAGE_TILE && (value != std::floor(value) || value >= wx::STAGE_TILE_VARIANTS))
    return fail(WX_E_INVAL, "stage tile must be an integer in 0..%d", wx::STAGE_TILE_VARIANTS - 1);
  if (param == WX_PARAM_JUDGE_SEED && value >= 4294967296.0) return fail(WX_E_INVAL, "judge seed must be < 2^32");
  if (param == WX_PARAM_JUDGE_RATE && (value < 1 || value > 4294967295.0))
    return fail(WX_E_INVAL, "judge rate must be in 1..2^32-1");
  impl_of(s)->param[param] = value;
  return WX_OK;
}

int wx_get_param(const wx_state *s, int param, double *value) {
  if (!s || !s->impl || !value) return fail(WX_E_INVAL, "NULL argument");
  if (param < 0 || param >= WX_PARAM_COUNT) return fail(WX_E_INVAL, "unknown param %d", param);
  *value = impl_of(s)->param[param];
  return WX_OK;
}

int wx_halo(wx_state *s, void *stream) {
  if (!s || !s->impl) return fail(WX_E_INVAL, "state is NULL");
  const void *req[] = {s->rho, s->theta, s->q, s->u, s->v};
  for (const void *p : req)
    if (!p) return fail(WX_E_STATE, "a field pointer is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (s->dtype == WX_F32) {
    float *f[5] = {(float *)s->rho, (float *)s->theta, (float *)s->q, (float *)s->u, (float *)s->v};
    WX_HIP(wx::launch_halo<float>(f, 5, s->nz, geom(s), st));
  } else if (s->dtype == WX_F64) {
    double *f[5] = {(double *)s->rho, (double *)s->theta, (double *)s->q, (double *)s->u, (double *)s->v};
    WX_HIP(wx::launch_halo<double>(f, 5, s->nz, geom(s), st));
  } else {
    return fail(WX_E_INVAL, "bad dtype %d", s->dtype);
  }
  return WX_OK;
}

int wx_step(wx_state *s, int nsteps, void *stream) {
  WX_TRY(validate_for_step(s));
  if (nsteps < 0) return fail(WX_E_INVAL, "nsteps must be >= 0");
  s->stream = stream;
  Timer tm;
  return run_steps(s, nsteps, static_cast<hipStream_t>(stream), tm);
}

int wx_physics(wx_state *s, wx_tend *t, int mode) {
  if (!s || !s->impl) return fail(WX_E_INVAL, "state is NULL");
  if (mode < WX_PHYS_PLAIN || mode > WX_PHYS_DATASET)
    return fail(WX_E_UNSUPPORTED, "wx_physics mode %d is not supported", mode);
  if (!t) return fail(WX_E_INVAL, "tendency struct is NULL");
  if (mode == WX_PHYS_DATASET) return wx_dataset(s, static_cast<float *>(t->features), t->labels);
  if (!t->dtheta || !t->dq) return fail(WX_E_INVAL, "tendency buffers are NULL");
  if (!aligned16(t->dtheta) || !aligned16(t->dq)) return fail(WX_E_INVAL, "tendency buffers must be 16-byte aligned");
  WX_TRY(check_fields(s, true));
  hipStream_t st = static_cast<hipStream_t>(s->stream);
  if (mode == WX_PHYS_SURROGATE || mode == WX_PHYS_JUDGED) {
    if (s->dtype != WX_F32) return fail(WX_E_UNSUPPORTED, "the surrogate modes need an FP32 state");
    if (s->nz != wx::MLP_NZ) return fail(WX_E_UNSUPPORTED, "the surrogate needs nz == %d", wx::MLP_NZ);
    if (!s->mlp || !s->surrogate_work || !aligned16(s->mlp) || !aligned16(s->surrogate_work))
      return fail(WX_E_STATE, "surrogate modes need mlp and surrogate_work (16-byte aligned)");
    if (mode == WX_PHYS_JUDGED && !s->judge_out) return fail(WX_E_STATE, "judged mode needs judge_out");
    Plan<float> p(s, st);
    WX_TRY(ensure_consts<float>(s, st));
    Timer tm;
    const uint64_t step = uint64_t(impl_of(s)->param[WX_PARAM_STEP]);
    return p.surrogate(mode == WX_PHYS_JUDGED, step, tm, static_cast<float *>(t->dtheta),
                       static_cast<float *>(t->dq));
  }
  if (s->dtype == WX_F32) {
    Plan<float> p(s, st);
    WX_TRY(ensure_consts<float>(s, st));
    WX_HIP(wx::launch_physics<float>(p.phys_args(1, 0, (float *)t->dtheta, (float *)t->dq), st));
  } else {
    Plan<double> p(s, st);
    WX_TRY(ensure_consts<double>(s, st));
    WX_HIP(wx::launch_physics<double>(p.phys_args(1, 0, (double *)t->dtheta, (double *)t->dq), st));
  }
  return WX_OK;
}

int wx_mass(wx_state *s) {
  if (!s || !s->impl) return fail(WX_E_INVAL, "state is NULL");
  WX_TRY(check_fields(s, false));
  hipStream_t st = static_cast<hipStream_t>(s->stream);
  Timer tm;
  if (s->dtype == WX_F32) {
    Plan<float> p(s, st);
    WX_TRY(ensure_consts<float>(s, st));
    WX_TRY(p.mass(tm));
    return p.mass_final(tm);
  }
  Plan<double> p(s, st);
  WX_TRY(ensure_consts<double>(s, st));
  WX_TRY(p.mass(tm));
  return p.mass_final(tm);
}

int wx_features(wx_state *s, int normalized, void *out, const void *blob) {
  if (!s || !s->impl) return fail(WX_E_INVAL, "state is NULL");
  if (!out || !aligned16(out)) return fail(WX_E_INVAL, "out is NULL or misaligned");
  if (normalized && !blob) return fail(WX_E_INVAL, "normalised features need the parameter blob");
  if (s->nz != wx::MLP_NZ) return fail(WX_E_UNSUPPORTED, "features need nz == %d", wx::MLP_NZ);
  WX_TRY(check_fields(s, true));
  hipStream_t st = static_cast<hipStream_t>(s->stream);
  const unsigned char *b = static_cast<const unsigned char *>(blob);
  const float *mean = blob ? reinterpret_cast<const float *>(b + wx_mlp_offset(WX_MLP_X_MEAN)) : nullptr;
  const float *istd = blob ? reinterpret_cast<const float *>(b + wx_mlp_offset(WX_MLP_X_INVSTD)) : nullptr;
  auto run = [&](auto tag) -> int {
    using T = decltype(tag);
    wx::FeatArgs<T> a;
    a.rho = (const T *)s->rho; a.th = (const T *)s->theta; a.q = (const T *)s->q;
    a.u = (const T *)s->u; a.v = (const T *)s->v;
    a.th_s = (const T *)s->theta_s; a.q_s = (const T *)s->q_s; a.f0 = (const T *)s->f0; a.ch = (const T *)s->ch;
    a.g = geom(s);
    a.theta_off = impl_of(s)->param[WX_PARAM_THETA_OFFSET];
    a.mode = normalized ? 1 : 0;
    a.out_f32 = normalized ? nullptr : static_cast<float *>(out);
    a.out_bf16 = normalized ? static_cast<uint16_t *>(out) : nullptr;
    a.mean = mean;
    a.inv_std = istd;
    a.c0 = 0;
    a.nrows = s->nx * s->ny;
    a.list = nullptr;
    a.n_list = nullptr;
    WX_HIP(wx::launch_features<T>(a, st));
    return WX_OK;
  };
  return s->dtype == WX_F32 ? run(float()) : run(double());
}

int wx_surrogate_rows(wx_state *s, const void *blob, const int32_t *cols, int n, float *rows_out) {
  if (!s || !s->impl) return fail(WX_E_INVAL, "state is NULL");
  if (!blob || !rows_out || !aligned16(blob) || !aligned16(rows_out))
    return fail(WX_E_INVAL, "blob and rows_out must be non-NULL and 16-byte aligned");
  if (s->dtype != WX_F32) return fail(WX_E_UNSUPPORTED, "the surrogate needs an FP32 state");
  if (s->nz != wx::MLP_NZ) return fail(WX_E_UNSUPPORTED, "the surrogate needs nz == %d", wx::MLP_NZ);
  if (n < 0 || (!cols && n > s->nx * s->ny)) return fail(WX_E_INVAL, "n = %d out of range", n);
  WX_TRY(check_fields(s, true));
  if (n == 0) return WX_OK;
  wx::FusedArgs a = fused_args(s, blob);
  a.list = cols;
  a.n_list = nullptr;
  a.cap = n;
  a.rows_out = rows_out;
  WX_HIP(wx::launch_surrogate_fused(a, static_cast<hipStream_t>(s->stream)));
  return WX_OK;
}

int wx_dataset(wx_state *s, float *x_raw, float *y_raw) {
  if (!s || !s->impl) return fail(WX_E_INVAL, "state is NULL");
  if (!x_raw || !y_raw || !aligned16(x_raw) || !aligned16(y_raw)) return fail(WX_E_INVAL, "bad output buffers");
  if (s->dtype != WX_F32) return fail(WX_E_UNSUPPORTED, "wx_dataset needs an FP32 state");
  WX_TRY(wx_features(s, 0, x_raw, nullptr));
  hipStream_t st = static_cast<hipStream_t>(s->stream);
  Plan<float> p(s, st);
  WX_TRY(ensure_consts<float>(s, st));
  wx::PhysArgs<float> a = p.phys_args(1, 0, y_raw, nullptr);
  a.tend_rows = 1;
  WX_HIP(wx::launch_physics<float>(a, st));
  return WX_OK;
}

int wx_profile_step(wx_state *s, int nsteps, void *stream, double *ms_out, int n_out) {
  WX_TRY(validate_for_step(s));
  if (nsteps < 1) return fail(WX_E_INVAL, "nsteps must be >= 1");
  if (!ms_out || n_out < 1) return fail(WX_E_INVAL, "ms_out must hold at least one value");
  hipStream_t st = static_cast<hipStream_t>(stream);
  s->stream = stream;
  std::vector<hipEvent_t> ev;
  std::vector<int> cls;
  Timer tm;
  tm.ev = &ev;
  tm.cls = &cls;
  tm.st = st;
  int rc = run_steps(s, nsteps, st, tm);
  hipError_t se = hipStreamSynchronize(st);
  double sum[kProfileClasses] = {0};
  int cnt[kProfileClasses] = {0};
  if (rc == WX_OK && se == hipSuccess) {
    for (size_t n = 0; n + 1 < ev.size(); ++n) {
      if (cls[n] < 0 || cls[n + 1] != -1) continue;
      float ms = 0;
      if (hipEventElapsedTime(&ms, ev[n], ev[n + 1]) == hipSuccess) {
        sum[cls[n]] += ms;
        cnt[cls[n]] += 1;
      }
    }
  }
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  if (rc != WX_OK) return rc;
  if (se != hipSuccess) return fail(WX_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(se));
  for (int c = 0; c < n_out; ++c) ms_out[c] = (c < kProfileClasses && cnt[c]) ? sum[c] / cnt[c] : 0.0;
  return WX_OK;
}

static int rw_check(const void *a, const void *b, const double *surf, const double *pbl, int nx, int ny, int nz,
                    double nu) {
  if (!a || !b || !surf || !pbl) return fail(WX_E_INVAL, "NULL pointer");
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(surf) |
       reinterpret_cast<uintptr_t>(pbl)) & 7)
    return fail(WX_E_INVAL, "arrays must be 8-byte aligned");
  if (a == b) return fail(WX_E_INVAL, "the two field arrays must be distinct");
  if (nx < 1 || ny < 1 || nz < 2) return fail(WX_E_INVAL, "grid %d x %d x %d outside nx, ny >= 1, nz >= 2", nx, ny, nz);
  if (double(nx + 2) * double(ny + 2) * double(nz) > double(1u << 29))
    return fail(WX_E_INVAL, "grid %d x %d x %d exceeds 2^29 cells", nx, ny, nz);
  if (!std::isfinite(nu)) return fail(WX_E_INVAL, "nu must be finite");
  return WX_OK;
}

int wx_rw_step(const double *e_in, double *e_out, const double *surf, const double *pbl, int nx, int ny, int nz,
               double nu, void *stream) {
  if (int rc = rw_check(e_in, e_out, surf, pbl, nx, ny, nz, nu)) return rc;
  WX_HIP(wx::launch_rw_step(e_in, e_out, surf, pbl, nx, ny, nz, nu, false, static_cast<hipStream_t>(stream)));
  return WX_OK;
}

static int rw_run(double *e0, double *e1, const double *surf, const double *pbl, int nx, int ny, int nz, double nu,
                  int nsteps, int *which, bool kij, void *stream, int bx = 64, int by = 8) {
  if (!which) return fail(WX_E_INVAL, "which is NULL");
  if (nsteps < 0) return fail(WX_E_INVAL, "nsteps must be >= 0");
  if (int rc = rw_check(e0, e1, surf, pbl, nx, ny, nz, nu)) return rc;
  if (!kij && !wx::rw_block_supported(bx, by))
    return fail(WX_E_UNSUPPORTED, "block %d x %d is not one of 64x8, 32x16, 128x1, 64x4, 128x4", bx, by);
  double *cur = e0, *nxt = e1;
  for (int n = 0; n < nsteps; ++n) {
    WX_HIP(wx::launch_rw_step(cur, nxt, surf, pbl, nx, ny, nz, nu, kij, static_cast<hipStream_t>(stream), bx, by));
    double *t = cur;
    cur = nxt;
    nxt = t;
  }
  *which = cur == e0 ? 0 : 1;
  return WX_OK;
}

int wx_rw_run(double *e0, double *e1, const double *surf, const double *pbl, int nx, int ny, int nz, double nu,
              int nsteps, int *which, void *stream) {
  return rw_run(e0, e1, surf, pbl, nx, ny, nz, nu, nsteps, which, false, stream);
}

int wx_rw_run_block(double *e0, double *e1, const double *surf, const double *pbl, int nx, int ny, int nz, double nu,
                    int nsteps, int *which, int block_x, int block_y, void *stream) {
  return rw_run(e0, e1, surf, pbl, nx, ny, nz, nu, nsteps, which, false, stream, block_x, block_y);
}

int wx_rw_run_kij(double *e0, double *e1, const double *surf, const double *pbl, int nx, int ny, int nz, double nu,
                  int nsteps, int *which, void *stream) {
  return rw_run(e0, e1, surf, pbl, nx, ny, nz, nu, nsteps, which, true, stream);
}

int wx_mass_noalloc(wx_state *s) {
  if (!s || !s->impl) return fail(WX_E_INVAL, "state is NULL");
  const long long nparts = wx::phys_blocks(s->nx, s->ny);
  if (nparts > kNoallocMaxParts)
    return fail(WX_E_INVAL, "grid %d x %d needs %lld mass partials; wx_mass_noalloc holds at most %d "
                "(ceil(nx/64)*ny <= %d)", s->nx, s->ny, nparts, kNoallocMaxParts, kNoallocMaxParts);
  if (s->dtype != WX_F32 && s->dtype != WX_F64) return fail(WX_E_INVAL, "dtype %d is not WX_F32/WX_F64", s->dtype);
  const void *req[] = {s->rho, s->theta, s->q, s->mass_out, s->flags_out};
  const char *names[] = {"rho", "theta", "q", "mass_out", "flags_out"};
  for (int n = 0; n < 5; ++n) {
    if (!req[n]) return fail(WX_E_STATE, "state pointer '%s' is NULL", names[n]);
    if (!aligned16(req[n])) return fail(WX_E_INVAL, "state pointer '%s' is not 16-byte aligned", names[n]);
  }
  double *ws = nullptr;
  WX_TRY(scratch_ptr(&ws));
  hipStream_t st = static_cast<hipStream_t>(s->stream);
  if (s->dtype == WX_F32) return mass_noalloc<float>(s, st, ws);
  return mass_noalloc<double>(s, st, ws);
}

int wx_copy_probe(void *dst, const void *src, size_t bytes, void *stream) {
  if (!dst || !src) return fail(WX_E_INVAL, "NULL pointer");
  if (bytes % 16 || !aligned16(dst) || !aligned16(src)) return fail(WX_E_INVAL, "copy needs 16-byte multiples");
  WX_HIP(wx::launch_copy(dst, src, bytes, static_cast<hipStream_t>(stream)));
  return WX_OK;
}

}  // extern "C"
