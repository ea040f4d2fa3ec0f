// C ABI of the HEVI fast-mode short steps (include/wx.h, "fast modes"):
// grid description, workspace layout, the per-stage coefficient tables and
// the stage launches with the ping-pong between the caller's fields and the
// workspace copy.
#include <cmath>
#include <cstdio>
#include <vector>

#include "wx.h"
#include "wx_internal.h"

namespace wx {
int set_error(int code, const char *msg);
}

namespace {

int hfail(int code, const char *msg) { return wx::set_error(code, msg); }

#define HX_HIP(call)                                                     \
  do {                                                                   \
    hipError_t e_ = (call);                                              \
    if (e_ != hipSuccess) {                                              \
      char b_[256];                                                      \
      snprintf(b_, sizeof b_, "%s: %s", #call, hipGetErrorString(e_));   \
      return hfail(WX_E_HIP, b_);                                        \
    }                                                                    \
  } while (0)

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace: two coefficient tables (stage lengths tau/2 and tau) and their
// two-sided forms, pi of the first stage, the parked right-hand side of the
// first stage, and a second copy of (u, v, pi) and (w, b) for the ping-pong
// between steps.
struct HeviLayout {
  size_t coef[2], coef2[2], pi1, e1, u, v, pi, w, b, total;
};

HeviLayout hevi_layout(const wx_hevi_grid *g) {
  const size_t es = g->dtype == WX_F32 ? 4 : 8;
  const size_t cell = al256(size_t(g->cell_elems) * es), face = al256(size_t(g->face_elems) * es);
  const size_t ctab = al256(size_t(g->nz) * 8 * es);
  HeviLayout L{};
  size_t off = 0;
  L.coef[0] = off; off += ctab;
  L.coef[1] = off; off += ctab;
  L.coef2[0] = off; off += ctab;
  L.coef2[1] = off; off += ctab;
  L.pi1 = off; off += cell;
  L.e1 = off; off += face;
  L.u = off; off += cell;
  L.v = off; off += cell;
  L.pi = off; off += cell;
  L.w = off; off += face;
  L.b = off; off += face;
  L.total = off;
  return L;
}

// Thomas factors of the constant tridiagonal matrix of a stage of length h,
// in FP64, rounded to T.
template <typename T>
std::vector<wx::HeviCoef<T>> coef_table(const wx_hevi_grid *g, const double *dz, double h) {
  const int nz = g->nz;
  std::vector<wx::HeviCoef<T>> out(nz);
  const double a = h * h * g->c_sound * g->c_sound / 4.0;
  const double diag0 = 1.0 + h * h * g->n_bv * g->n_bv / 4.0;
  double cp = 0.0;
  for (int k = 0; k < nz; ++k) {
    wx::HeviCoef<T> c{};
    c.dz = T(dz[k]);
    c.rdz = T(1.0 / dz[k]);
    if (k > 0) {
      const double dzf = (dz[k - 1] + dz[k]) / 2.0;
      const double lo = a / (dzf * dz[k - 1]);
      const double hi = k + 1 < nz ? a / (dzf * dz[k]) : 0.0;
      // faces 1 .. nz-1; the coupling to the lid face (k = nz) has no unknown
      const double diag = diag0 + lo + a / (dzf * dz[k]);
      const double inv = 1.0 / (diag + lo * cp);
      cp = -hi * inv;
      c.dzf = T(dzf);
      c.rdzf = T(1.0 / dzf);
      c.lo = T(lo);
      c.inv = T(inv);
      c.cp = T(cp);
    }
    out[k] = c;
  }
  return out;
}

// The same system split at face H = nz/2 for a two-sided elimination: faces
// 1 .. H-1 keep the Thomas factors from the ground (lo, inv, cp as above);
// faces H+1 .. nz-1 take factors eliminated from the lid down,
//   inv'_f = 1 / (diag_f + hi_f cp'_{f+1}),  cp'_f = -lo_f inv'_f,
// with hi_f in the lo slot (E'_f = (rhs_f + hi_f E'_{f+1}) inv'_f, then
// wm_f = E'_f - cp'_f wm_{f-1}); face H holds lo_H, hi_H (in pad) and
//   inv = 1 / (diag_H + lo_H cp_{H-1} + hi_H cp'_{H+1}),
// so that wm_H = (rhs_H + lo_H E_{H-1} + hi_H E'_{H+1}) inv.
template <typename T>
std::vector<wx::HeviCoef<T>> coef_table_two_sided(const wx_hevi_grid *g, const double *dz, double h) {
  const int nz = g->nz, H = nz / 2;
  std::vector<wx::HeviCoef<T>> out(nz);
  const double a = h * h * g->c_sound * g->c_sound / 4.0;
  const double diag0 = 1.0 + h * h * g->n_bv * g->n_bv / 4.0;
  std::vector<double> lo(nz, 0.0), hi(nz, 0.0), diag(nz, 0.0), dzf(nz, 0.0);
  for (int k = 1; k < nz; ++k) {
    dzf[k] = (dz[k - 1] + dz[k]) / 2.0;
    lo[k] = a / (dzf[k] * dz[k - 1]);
    hi[k] = k + 1 < nz ? a / (dzf[k] * dz[k]) : 0.0;
    diag[k] = diag0 + lo[k] + a / (dzf[k] * dz[k]);
  }
  std::vector<double> cpf(nz, 0.0), cpr(nz + 1, 0.0), invf(nz, 0.0), invr(nz, 0.0);
  double cp = 0.0;
  for (int k = 1; k < H; ++k) {
    invf[k] = 1.0 / (diag[k] + lo[k] * cp);
    cp = -hi[k] * invf[k];
    cpf[k] = cp;
  }
  double cq = 0.0;
  for (int k = nz - 1; k > H; --k) {
    invr[k] = 1.0 / (diag[k] + hi[k] * cq);
    cq = -lo[k] * invr[k];
    cpr[k] = cq;
  }
  const double inv_mid = 1.0 / (diag[H] + lo[H] * cpf[H - 1] + hi[H] * cpr[H + 1]);
  for (int k = 0; k < nz; ++k) {
    wx::HeviCoef<T> c{};
    c.dz = T(dz[k]);
    c.rdz = T(1.0 / dz[k]);
    if (k > 0) {
      c.dzf = T(dzf[k]);
      c.rdzf = T(1.0 / dzf[k]);
      if (k < H) {
        c.lo = T(lo[k]);
        c.inv = T(invf[k]);
        c.cp = T(cpf[k]);
      } else if (k > H) {
        c.lo = T(hi[k]);
        c.inv = T(invr[k]);
        c.cp = T(cpr[k]);
      } else {
        c.lo = T(lo[k]);
        c.pad = T(hi[k]);
        c.inv = T(inv_mid);
      }
    }
    out[k] = c;
  }
  return out;
}

template <typename T>
int hevi_run(const wx_hevi_grid *g, const double *dz, void *u, void *v, void *w, void *b, void *pi, void *ws,
             int nsteps, hipStream_t st) {
  const HeviLayout L = hevi_layout(g);
  unsigned char *W = static_cast<unsigned char *>(ws);
  const double tau = g->tau;
  for (int s = 0; s < 2; ++s) {
    const std::vector<wx::HeviCoef<T>> tab = coef_table<T>(g, dz, s == 0 ? tau / 2.0 : tau);
    HX_HIP(hipMemcpyAsync(W + L.coef[s], tab.data(), tab.size() * sizeof(tab[0]), hipMemcpyHostToDevice, st));
    // the host table must outlive the copy: wait for it before it goes away
    HX_HIP(hipStreamSynchronize(st));
    if (g->kernel == 2) {
      const std::vector<wx::HeviCoef<T>> t2 = coef_table_two_sided<T>(g, dz, s == 0 ? tau / 2.0 : tau);
      HX_HIP(hipMemcpyAsync(W + L.coef2[s], t2.data(), t2.size() * sizeof(t2[0]), hipMemcpyHostToDevice, st));
      HX_HIP(hipStreamSynchronize(st));
    }
  }
  const wx::Geom geo{g->nx, g->ny, g->nz, unsigned(g->stride_j), unsigned(g->stride_k), unsigned(g->origin)};
  T *mine[5] = {static_cast<T *>(u), static_cast<T *>(v), static_cast<T *>(w), static_cast<T *>(b),
                static_cast<T *>(pi)};
  T *copy[5] = {reinterpret_cast<T *>(W + L.u), reinterpret_cast<T *>(W + L.v), reinterpret_cast<T *>(W + L.w),
                reinterpret_cast<T *>(W + L.b), reinterpret_cast<T *>(W + L.pi)};
  {
    T *f[5] = {mine[0], mine[1], mine[4], mine[4], mine[4]};
    HX_HIP(wx::launch_halo<T>(f, 3, g->nz, geo, st));
  }
  T *const pi1 = reinterpret_cast<T *>(W + L.pi1);
  T *const e1 = reinterpret_cast<T *>(W + L.e1);
  T **cur = mine, **nxt = copy;
  for (int n = 0; n < nsteps; ++n) {
    for (int s = 0; s < 2; ++s) {
      wx::HeviArgs<T> a{};
      a.u = cur[0]; a.v = cur[1]; a.w = cur[2]; a.b = cur[3]; a.pi = cur[4];
      a.pp = s == 0 ? cur[4] : pi1;
      a.coef = reinterpret_cast<const wx::HeviCoef<T> *>(W + L.coef[s]);
      a.coef2 = reinterpret_cast<const wx::HeviCoef<T> *>(W + L.coef2[s]);
      a.g = geo;
      const double h = s == 0 ? tau / 2.0 : tau;
      a.h = T(h);
      a.h2 = T(h / 2.0);
      a.a4 = T(h * h * g->c_sound * g->c_sound / 4.0);
      a.hc2 = T(h * g->c_sound * g->c_sound);
      a.hn2 = T(h * g->n_bv * g->n_bv);
      a.dx = T(g->dx);
      a.rdx = T(1.0 / g->dx);
      if (s == 0) {
        a.pi_o = pi1;
        a.e_o = e1;
      } else {
        a.u_o = nxt[0]; a.v_o = nxt[1]; a.w_o = nxt[2]; a.b_o = nxt[3]; a.pi_o = nxt[4];
        a.e_o = nxt[2];
      }
      HX_HIP(wx::launch_hevi_stage<T>(a, s == 1, g->kernel, st));
    }
    T **t = cur;
    cur = nxt;
    nxt = t;
  }
  if (cur != mine) {
    const size_t es = sizeof(T);
    const size_t bytes[5] = {size_t(g->cell_elems) * es, size_t(g->cell_elems) * es, size_t(g->face_elems) * es,
                             size_t(g->face_elems) * es, size_t(g->cell_elems) * es};
    for (int f = 0; f < 5; ++f) HX_HIP(wx::launch_copy(mine[f], cur[f], bytes[f], st));
  }
  return WX_OK;
}

bool al16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

extern "C" {

int wx_hevi_grid_init(wx_hevi_grid *g, int nx, int ny, int nz, int dtype, double dx, double tau, double c_sound,
                      double n_bv) {
  if (!g) return hfail(WX_E_INVAL, "grid is NULL");
  if (nx < 4 || ny < 4 || nz < 2 || nz > 1024) return hfail(WX_E_INVAL, "grid outside nx, ny >= 4, 2 <= nz <= 1024");
  if (dtype != WX_F32 && dtype != WX_F64) return hfail(WX_E_INVAL, "dtype is not WX_F32/WX_F64");
  if (!(dx > 0) || !std::isfinite(dx) || !(tau > 0) || !std::isfinite(tau) || !(c_sound > 0) ||
      !std::isfinite(c_sound) || !(n_bv >= 0) || !std::isfinite(n_bv))
    return hfail(WX_E_INVAL, "dx, tau, c must be finite and > 0, N finite and >= 0");
  const long long sj = ((long long)nx + 4 + 63) / 64 * 64;
  const long long sk = sj * (ny + 4);
  if (sk * (long long)(nz + 1) * 8 >= (1LL << 32)) return hfail(WX_E_UNSUPPORTED, "grid too large for 32-bit offsets");
  g->nx = nx;
  g->ny = ny;
  g->nz = nz;
  g->dtype = dtype;
  g->stride_j = sj;
  g->stride_k = sk;
  g->origin = 2 + 2 * sj;
  g->cell_elems = sk * nz;
  g->face_elems = sk * (nz + 1);
  g->dx = dx;
  g->tau = tau;
  g->c_sound = c_sound;
  g->n_bv = n_bv;
  g->kernel = 2;
  g->pad = 0;
  return WX_OK;
}

size_t wx_hevi_workspace_bytes(const wx_hevi_grid *g) {
  if (!g || g->nz < 2 || (g->dtype != WX_F32 && g->dtype != WX_F64)) return 0;
  return hevi_layout(g).total;
}

int wx_hevi_run(const wx_hevi_grid *g, const double *dz, void *u, void *v, void *w, void *b, void *pi,
                void *workspace, int nsteps, void *stream) {
  if (!g || g->nz < 2 || g->nx < 4 || g->ny < 4) return hfail(WX_E_INVAL, "grid is NULL or not initialised");
  if (g->dtype != WX_F32 && g->dtype != WX_F64) return hfail(WX_E_INVAL, "dtype is not WX_F32/WX_F64");
  if (!dz) return hfail(WX_E_INVAL, "dz is NULL");
  for (int k = 0; k < g->nz; ++k)
    if (!(dz[k] > 0) || !std::isfinite(dz[k])) return hfail(WX_E_INVAL, "dz must be finite and > 0");
  const void *req[] = {u, v, w, b, pi, workspace};
  for (const void *p : req)
    if (!p || !al16(p)) return hfail(WX_E_INVAL, "field or workspace pointer NULL or not 16-byte aligned");
  if (nsteps < 0) return hfail(WX_E_INVAL, "nsteps must be >= 0");
  if (g->kernel != 0 && g->kernel != 1 && g->kernel != 2) return hfail(WX_E_INVAL, "kernel must be 0, 1 or 2");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (g->dtype == WX_F32) return hevi_run<float>(g, dz, u, v, w, b, pi, workspace, nsteps, st);
  return hevi_run<double>(g, dz, u, v, w, b, pi, workspace, nsteps, st);
}

}  // extern "C"
