// Host side of the C ABI declared in include/sts.h: context management, the
// separable geometry tables, argument checking and the launch sequences of
// RKL2 and BE+PCG.  No arithmetic of the method runs here apart from the
// 1D geometry tables, the RKL2 stage coefficients and the stage count.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "sts_internal.h"

using namespace sts;

sts::Grid sts_ctx::grid() const {
  Grid g;
  g.n0 = n0;
  g.n1 = n1;
  g.n2 = n2;
  g.per0 = bc[0] == STS_BC_PERIODIC;
  g.per1 = bc[2] == STS_BC_PERIODIC;
  g.per2 = bc[4] == STS_BC_PERIODIC;
  g.dir_lo = bc[0] == STS_BC_DIRICHLET;
  g.dir_hi = bc[1] == STS_BC_DIRICHLET;
  g.wg_rev = (debug & STS_DEBUG_WG_REVERSE) ? 1 : 0;
  g.t0 = d_t0;
  g.t1 = d_t1;
  g.t2 = d_t2;
  g.ab_lo = ab_lo;
  g.ab_hi = ab_hi;
  g.db_lo = db_lo;
  g.db_hi = db_hi;
  return g;
}

sts::Coef sts_ctx::coef() const {
  Coef c;
  const long long n = ncell;
  c.w0 = d_w;
  c.w1 = d_w ? d_w + n : nullptr;
  c.w2 = d_w ? d_w + 2 * n : nullptr;
  c.k01 = d_w ? d_w + 3 * n : nullptr;
  c.k02 = d_w ? d_w + 4 * n : nullptr;
  c.k12 = d_w ? d_w + 5 * n : nullptr;
  const long long nb = (long long)n1 * n2;
  c.wb_lo = d_bnd;
  c.wb_hi = d_bnd + nb;
  c.ub_lo = d_bnd + 2 * nb;
  c.ub_hi = d_bnd + 3 * nb;
  c.nu = nu;
  return c;
}

namespace {

#define FAIL(code, msg)     \
  do {                      \
    ctx->err = (msg);       \
    return (code);          \
  } while (0)

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
      return STS_EHIP;                                                            \
    }                                                                             \
  } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

sts_status dalloc(sts_ctx *ctx, void **p, size_t bytes) {
  if (*p) return STS_OK;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    ctx->err = "device allocation of " + std::to_string(bytes) + " bytes failed";
    return STS_ENOMEM;
  }
  return STS_OK;
}

template <class T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

bool finite_increasing(const double *f, int n) {
  for (int m = 0; m <= n; ++m)
    if (!std::isfinite(f[m])) return false;
  for (int m = 0; m < n; ++m)
    if (!(f[m + 1] > f[m])) return false;
  return true;
}

// centre-to-centre distance across the +face of each cell (0 where absent)
std::vector<double> inv_gaps(const double *f, int n, bool periodic) {
  std::vector<double> c(n), ig(n, 0.0);
  for (int m = 0; m < n; ++m) c[m] = 0.5 * (f[m] + f[m + 1]);
  for (int m = 0; m + 1 < n; ++m) ig[m] = 1.0 / (c[m + 1] - c[m]);
  if (periodic) ig[n - 1] = 1.0 / (c[0] + (f[n] - f[0]) - c[n - 1]);
  return ig;
}

// RKL2 stage count: least s >= 2 with s^2 + s - 2 >= 4 dt/dt_E (Eq. rkl2_s)
int stage_count(double ratio) {
  int s = (int)std::ceil((std::sqrt(9.0 + 16.0 * ratio) - 1.0) / 2.0);
  if (s < 2) s = 2;
  while (s - 1 >= 2 && (double)(s - 1) * (s - 1) + (s - 1) - 2.0 >= 4.0 * ratio) --s;
  while ((double)s * s + s - 2.0 < 4.0 * ratio) ++s;
  return s;
}

constexpr int kMaxStages = 1 << 20;
constexpr int kPollEvery = 8;  // PCG iterations enqueued between host polls
constexpr int kRkBuffers = 2;  // RKL2 state buffers besides F0

// Scratch of rkl2_step_noalloc: a file-scope device array, one copy per GPU,
// held until the process ends.  Host code never passes its name to a kernel
// (in host code the name is a host-side stand-in): the device address is
// resolved once per device with hipGetSymbolAddress and used from there on.
constexpr size_t kScratchBytes = (size_t)96 << 20;  // 4,194,304 FP64 cells x components
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];
static hipError_t g_scratch_st[kMaxDevices];
static bool g_scratch_done[kMaxDevices];

// Device address of `scratch` on the current device (resolved at the first
// call on that device); nullptr with err set on failure.
static void *scratch_address(int device, std::string *err) {
  if (device < 0 || device >= kMaxDevices) {
    *err = "device index out of range";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void *ptr = nullptr;
    g_scratch_st[device] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[device] = g_scratch_st[device] == hipSuccess ? ptr : nullptr;
    g_scratch_done[device] = true;
  }
  if (!g_scratch_ptr[device])
    *err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(g_scratch_st[device]);
  return g_scratch_ptr[device];
}

}  // namespace

// ---- per-kernel timing ------------------------------------------------------

namespace sts {

constexpr size_t kProfMaxRecords = (size_t)1 << 20;

static hipEvent_t prof_event(sts_ctx *c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(const sts_ctx *c, const char *name) {
  if (!c || !c->profile || c->prof.size() >= kProfMaxRecords) return;
  sts_ctx *m = const_cast<sts_ctx *>(c);
  a_ = prof_event(m);
  if (!a_ || hipEventRecord(a_, m->stream) != hipSuccess) return;
  c_ = m;
  name_ = name;
}

ProfScope::~ProfScope() {
  if (!c_) return;
  hipEvent_t b = prof_event(c_);
  if (!b || hipEventRecord(b, c_->stream) != hipSuccess) return;
  c_->prof.push_back(ProfRec{name_, a_, b});
}

}  // namespace sts

extern "C" {

sts_status sts_create(sts_ctx **out, int coord, int n0, int n1, int n2, const double *f0,
                      const double *f1, const double *f2, const int bc[6], void *stream) {
  if (!out) return STS_EINVAL;
  *out = nullptr;
  auto *ctx = new sts_ctx();
  auto bad = [&](const char *m) {
    std::fprintf(stderr, "sts_create: %s\n", m);
    delete ctx;
    return STS_EINVAL;
  };
  if (coord != STS_SPHERICAL && coord != STS_CARTESIAN) return bad("unknown coordinate system");
  if (n0 < 1 || n1 < 1 || n2 < 1) return bad("grid dimensions must be >= 1");
  const long long ncell = (long long)n0 * n1 * n2;
  if (ncell > (long long)std::numeric_limits<int>::max() / 2) return bad("grid too large");
  if (!f0 || !f1 || !f2 || !bc) return bad("null face array or bc");
  if (!finite_increasing(f0, n0) || !finite_increasing(f1, n1) || !finite_increasing(f2, n2))
    return bad("face coordinates must be finite and strictly increasing");
  for (int s = 0; s < 6; ++s)
    if (bc[s] != STS_BC_ZEROFLUX && bc[s] != STS_BC_DIRICHLET && bc[s] != STS_BC_PERIODIC)
      return bad("unknown boundary condition");
  const int nn[3] = {n0, n1, n2};
  for (int a = 0; a < 3; ++a) {
    const bool pl = bc[2 * a] == STS_BC_PERIODIC, ph = bc[2 * a + 1] == STS_BC_PERIODIC;
    if (pl != ph) return bad("periodic must be set on both sides of an axis");
    if (pl && nn[a] < 3) return bad("a periodic axis needs at least 3 cells");
    if (a > 0 && (bc[2 * a] == STS_BC_DIRICHLET || bc[2 * a + 1] == STS_BC_DIRICHLET))
      return bad("Dirichlet boundaries are supported on axis 0 only");
  }
  if (coord == STS_SPHERICAL) {
    if (!(f0[0] > 0.0)) return bad("spherical radii must be positive");
    if (!(f1[0] > 0.0) || !(f1[n1] < M_PI)) return bad("colatitudes must lie in (0, pi)");
  }
  ctx->coord = coord;
  ctx->n0 = n0;
  ctx->n1 = n1;
  ctx->n2 = n2;
  ctx->ncell = ncell;
  std::memcpy(ctx->bc, bc, sizeof(ctx->bc));
  ctx->hf[0].assign(f0, f0 + n0 + 1);
  ctx->hf[1].assign(f1, f1 + n1 + 1);
  ctx->hf[2].assign(f2, f2 + n2 + 1);
  ctx->stream = (hipStream_t)stream;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return STS_EHIP;
  }
  ctx->d_scratch = scratch_address(ctx->device, &ctx->scratch_err);
  {
    const char *e = std::getenv("STS_PROFILE");
    ctx->profile = e && *e && std::strcmp(e, "0") != 0;
  }

  // --- separable geometry tables ---
  std::vector<double> t0((size_t)NT0 * n0), t1((size_t)NT1 * n1), t2((size_t)NT2 * n2);
  const bool per0 = bc[0] == STS_BC_PERIODIC, per1 = bc[2] == STS_BC_PERIODIC,
             per2 = bc[4] == STS_BC_PERIODIC;
  const std::vector<double> ig0 = inv_gaps(f0, n0, per0), ig1 = inv_gaps(f1, n1, per1),
                            ig2 = inv_gaps(f2, n2, per2);
  for (int i = 0; i < n0; ++i) {
    const double a = f0[i], b = f0[i + 1], c = 0.5 * (a + b), d = b - a;
    double *T = t0.data();
    if (coord == STS_SPHERICAL) {
      T[T_V0 * n0 + i] = (b * b * b - a * a * a) / 3.0;
      T[T_A00 * n0 + i] = b * b;
      T[T_A10 * n0 + i] = 0.5 * (b * b - a * a);
      T[T_A20 * n0 + i] = 0.5 * (b * b - a * a);
      T[T_IL10 * n0 + i] = 1.0 / c;
      T[T_IL20 * n0 + i] = 1.0 / c;
    } else {
      T[T_V0 * n0 + i] = d;
      T[T_A00 * n0 + i] = 1.0;
      T[T_A10 * n0 + i] = d;
      T[T_A20 * n0 + i] = d;
      T[T_IL10 * n0 + i] = 1.0;
      T[T_IL20 * n0 + i] = 1.0;
    }
    T[T_IL00 * n0 + i] = ig0[i];
    T[T_IV0 * n0 + i] = 1.0 / T[T_V0 * n0 + i];
  }
  for (int j = 0; j < n1; ++j) {
    const double a = f1[j], b = f1[j + 1], c = 0.5 * (a + b), d = b - a;
    double *T = t1.data();
    if (coord == STS_SPHERICAL) {
      T[T_V1 * n1 + j] = std::cos(a) - std::cos(b);
      T[T_A01 * n1 + j] = std::cos(a) - std::cos(b);
      T[T_A11 * n1 + j] = std::sin(b);
      T[T_A21 * n1 + j] = d;
      T[T_IL21 * n1 + j] = 1.0 / std::sin(c);
    } else {
      T[T_V1 * n1 + j] = d;
      T[T_A01 * n1 + j] = d;
      T[T_A11 * n1 + j] = 1.0;
      T[T_A21 * n1 + j] = d;
      T[T_IL21 * n1 + j] = 1.0;
    }
    T[T_IL11 * n1 + j] = ig1[j];
  }
  for (int k = 0; k < n2; ++k) {
    const double d = f2[k + 1] - f2[k];
    double *T = t2.data();
    T[T_V2 * n2 + k] = d;
    T[T_A02 * n2 + k] = d;
    T[T_A12 * n2 + k] = d;
    T[T_A22 * n2 + k] = 1.0;
    T[T_IL22 * n2 + k] = ig2[k];
  }
  if (coord == STS_SPHERICAL) {
    ctx->ab_lo = f0[0] * f0[0];
    ctx->ab_hi = f0[n0] * f0[n0];
  } else {
    ctx->ab_lo = ctx->ab_hi = 1.0;
  }
  ctx->db_lo = 0.5 * (f0[0] + f0[1]) - f0[0];
  ctx->db_hi = f0[n0] - 0.5 * (f0[n0 - 1] + f0[n0]);

  auto cleanup = [&](sts_status st) {
    sts_destroy(ctx);
    return st;
  };
  sts_status st;
  const long long nb = (long long)n1 * n2;
  if ((st = dalloc(ctx, (void **)&ctx->d_t0, t0.size() * 8)) ||
      (st = dalloc(ctx, (void **)&ctx->d_t1, t1.size() * 8)) ||
      (st = dalloc(ctx, (void **)&ctx->d_t2, t2.size() * 8)) ||
      (st = dalloc(ctx, (void **)&ctx->d_bnd, 4 * nb * 8)) ||
      (st = dalloc(ctx, (void **)&ctx->d_flag, 64)) ||
      (st = dalloc(ctx, (void **)&ctx->d_tmp, 64)) ||
      (st = dalloc(ctx, (void **)&ctx->d_sc, sizeof(PcgScalars))))
    return cleanup(st);
  if (hipHostMalloc(&ctx->h_pin, 256, hipHostMallocDefault) != hipSuccess) {
    ctx->h_pin = nullptr;
    return cleanup(STS_ENOMEM);
  }
  if (hipMemcpyAsync(ctx->d_t0, t0.data(), t0.size() * 8, hipMemcpyHostToDevice, ctx->stream) ||
      hipMemcpyAsync(ctx->d_t1, t1.data(), t1.size() * 8, hipMemcpyHostToDevice, ctx->stream) ||
      hipMemcpyAsync(ctx->d_t2, t2.data(), t2.size() * 8, hipMemcpyHostToDevice, ctx->stream))
    return cleanup(STS_EHIP);
  launch_fill(ctx, ctx->d_bnd, 4 * nb, 0.0);
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return cleanup(STS_EHIP);
  *out = ctx;
  return STS_OK;
}

sts_status sts_destroy(sts_ctx *ctx) {
  if (!ctx) return STS_EINVAL;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  dfree(ctx->d_t0);
  dfree(ctx->d_t1);
  dfree(ctx->d_t2);
  dfree(ctx->d_w);
  dfree(ctx->d_wf);
  dfree(ctx->d_rk32);
  dfree(ctx->d_pcg32);
  dfree(ctx->d_sdiag);
  dfree(ctx->d_bnd);
  dfree(ctx->d_rk);
  dfree(ctx->d_pcg);
  dfree(ctx->d_red);
  dfree(ctx->d_sc);
  dfree(ctx->d_ilu);
  for (auto &r : ctx->prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
  dfree(ctx->d_gfac);
  dfree(ctx->d_pct);
  dfree(ctx->d_pcobj);
  dfree(ctx->d_sc0);
  dfree(ctx->d_flag);
  dfree(ctx->d_tmp);
  dfree(ctx->d_rtab);
  dfree(ctx->d_rws);
  if (ctx->h_pin) (void)hipHostFree(ctx->h_pin);
  for (hipEvent_t e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
  return STS_OK;
}

sts_status sts_set_stream(sts_ctx *ctx, void *stream) {
  if (!ctx) return STS_EINVAL;
  ctx->stream = (hipStream_t)stream;
  return STS_OK;
}

const char *sts_last_error(const sts_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

long long sts_num_cells(const sts_ctx *ctx) { return ctx ? ctx->ncell : 0; }

static sts_status refresh_dirichlet_values(sts_ctx *ctx) {
  const long long nb = (long long)ctx->n1 * ctx->n2;
  for (int side = 0; side < 2; ++side)
    if (!ctx->ub_array[side]) launch_fill(ctx, ctx->d_bnd + (2 + side) * nb, nb, ctx->ub_const[side]);
  LAUNCHCHK();
  return STS_OK;
}

sts_status sts_set_debug(sts_ctx *ctx, int flags) {
  if (!ctx) return STS_EINVAL;
  if (flags & ~(STS_DEBUG_WG_REVERSE | STS_DEBUG_SEPARATE_FINALIZE))
    FAIL(STS_EINVAL, "sts_set_debug: unknown flag");
  ctx->debug = flags;
  return STS_OK;
}

sts_status sts_set_profile(sts_ctx *ctx, int on) {
  if (!ctx) return STS_EINVAL;
  ctx->profile = on != 0;
  return STS_OK;
}

sts_status sts_profile_summary(sts_ctx *ctx, char *buf, long long cap, int reset) {
  if (!ctx || !buf || cap < 1) return STS_EINVAL;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  struct Agg {
    long long n = 0;
    double tot = 0.0, mn = 1e300, mx = 0.0;
  };
  std::map<std::string, Agg> agg;
  for (const ProfRec &r : ctx->prof) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    Agg &a = agg[r.name];
    a.n += 1;
    a.tot += ms;
    a.mn = std::min(a.mn, (double)ms);
    a.mx = std::max(a.mx, (double)ms);
  }
  std::vector<std::pair<std::string, Agg>> rows(agg.begin(), agg.end());
  std::sort(rows.begin(), rows.end(),
            [](const auto &x, const auto &y) { return x.second.tot > y.second.tot; });
  std::string out = "calls total_ms avg_us min_us max_us launcher\n";
  char line[256];
  for (const auto &r : rows) {
    std::snprintf(line, sizeof line, "%lld %.4f %.2f %.2f %.2f %s\n", r.second.n, r.second.tot,
                  1e3 * r.second.tot / r.second.n, 1e3 * r.second.mn, 1e3 * r.second.mx,
                  r.first.c_str());
    out += line;
  }
  if ((long long)out.size() + 1 > cap) FAIL(STS_EINVAL, "sts_profile_summary: buffer too small");
  std::memcpy(buf, out.c_str(), out.size() + 1);
  if (reset) {
    for (const ProfRec &r : ctx->prof) {
      ctx->prof_pool.push_back(r.a);
      ctx->prof_pool.push_back(r.b);
    }
    ctx->prof.clear();
  }
  return STS_OK;
}

sts_status sts_set_spitzer(sts_ctx *ctx, const double *T, double kappa0, const double *b0,
                           const double *b1, const double *b2) {
  if (!ctx) return STS_EINVAL;
  if (!T || !b0 || !b1 || !b2) FAIL(STS_EINVAL, "sts_set_spitzer: null field");
  if (!(kappa0 > 0.0) || !std::isfinite(kappa0)) FAIL(STS_EINVAL, "kappa0 must be finite, > 0");
  sts_status st;
  if ((st = dalloc(ctx, (void **)&ctx->d_w, 6 * ctx->ncell * 8)) ||
      (st = dalloc(ctx, (void **)&ctx->d_sdiag, ctx->ncell * 8)))
    return st;
  HIPCHK(hipMemsetAsync(ctx->d_flag, 0, sizeof(int), ctx->stream));
  launch_check_spitzer(ctx, T, b0, b1, b2, ctx->d_flag);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(ctx->h_pin, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (*(int *)ctx->h_pin) FAIL(STS_EINVAL, "sts_set_spitzer: T must be finite and > 0, b finite");
  if ((st = refresh_dirichlet_values(ctx))) return st;
  ctx->op = OP_SPITZER;
  ctx->prec = 0;
  ctx->nu = 0.0;
  launch_spitzer_coef(ctx, T, kappa0, b0, b1, b2);
  LAUNCHCHK();
  launch_sdiag(ctx);
  LAUNCHCHK();
  ctx->dt_euler = -1.0;
  return STS_OK;
}

sts_status sts_set_isotropic(sts_ctx *ctx, double nu) {
  if (!ctx) return STS_EINVAL;
  if (!(nu > 0.0) || !std::isfinite(nu)) FAIL(STS_EINVAL, "nu must be finite and > 0");
  sts_status st;
  if ((st = dalloc(ctx, (void **)&ctx->d_sdiag, ctx->ncell * 8))) return st;
  if ((st = refresh_dirichlet_values(ctx))) return st;
  ctx->op = OP_ISOTROPIC;
  ctx->prec = 0;
  ctx->nu = nu;
  launch_dirichlet_weights(ctx);
  LAUNCHCHK();
  launch_sdiag(ctx);
  LAUNCHCHK();
  ctx->dt_euler = -1.0;
  return STS_OK;
}

sts_status sts_set_spitzer_f32(sts_ctx *ctx, const float *T, double kappa0, const float *b0,
                               const float *b1, const float *b2) {
  if (!ctx) return STS_EINVAL;
  if (!T || !b0 || !b1 || !b2) FAIL(STS_EINVAL, "sts_set_spitzer_f32: null field");
  if (!(kappa0 > 0.0) || !std::isfinite(kappa0)) FAIL(STS_EINVAL, "kappa0 must be finite, > 0");
  sts_status st;
  if ((st = dalloc(ctx, (void **)&ctx->d_w, 6 * ctx->ncell * 8)) ||
      (st = dalloc(ctx, (void **)&ctx->d_wf, 6 * ctx->ncell * 4)) ||
      (st = dalloc(ctx, (void **)&ctx->d_sdiag, ctx->ncell * 8)))
    return st;
  HIPCHK(hipMemsetAsync(ctx->d_flag, 0, sizeof(int), ctx->stream));
  launch_check_spitzer_f32(ctx, T, b0, b1, b2, ctx->d_flag);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(ctx->h_pin, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (*(int *)ctx->h_pin) FAIL(STS_EINVAL, "sts_set_spitzer_f32: T must be finite and > 0");
  if ((st = refresh_dirichlet_values(ctx))) return st;
  ctx->op = OP_SPITZER;
  ctx->prec = 1;
  ctx->nu = 0.0;
  launch_spitzer_coef_f32(ctx, T, kappa0, b0, b1, b2);
  LAUNCHCHK();
  launch_sdiag(ctx);
  LAUNCHCHK();
  ctx->dt_euler = -1.0;
  return STS_OK;
}

sts_status sts_set_isotropic_f32(sts_ctx *ctx, double nu) {
  sts_status st = sts_set_isotropic(ctx, nu);
  if (st) return st;
  ctx->prec = 1;
  return STS_OK;
}

sts_status sts_set_dirichlet(sts_ctx *ctx, int side, const double *values, double value) {
  if (!ctx) return STS_EINVAL;
  if (side != 0 && side != 1) FAIL(STS_EINVAL, "side must be 0 or 1");
  if (!values && !std::isfinite(value)) FAIL(STS_EINVAL, "Dirichlet value must be finite");
  const long long nb = (long long)ctx->n1 * ctx->n2;
  double *dst = ctx->d_bnd + (2 + side) * nb;
  if (values) {
    HIPCHK(hipMemcpyAsync(dst, values, nb * 8, hipMemcpyDeviceToDevice, ctx->stream));
    ctx->ub_array[side] = true;
  } else {
    ctx->ub_const[side] = value;
    ctx->ub_array[side] = false;
    launch_fill(ctx, dst, nb, value);
    LAUNCHCHK();
  }
  return STS_OK;
}

static sts_status ensure_red(sts_ctx *ctx, int need) {
  if (ctx->red_cap >= need) return STS_OK;
  dfree(ctx->d_red);
  ctx->red_cap = 0;
  sts_status st = dalloc(ctx, (void **)&ctx->d_red, (size_t)4 * need * 8);
  if (st) return st;
  ctx->red_cap = need;
  return STS_OK;
}

sts_status sts_dt_euler(sts_ctx *ctx, double *dt_e) {
  if (!ctx || !dt_e) return STS_EINVAL;
  if (ctx->op == OP_NONE) FAIL(STS_EINVAL, "no operator set");
  if (ctx->dt_euler > 0) {
    *dt_e = ctx->dt_euler;
    return STS_OK;
  }
  const int np = gershgorin_parts(ctx);
  sts_status st;
  if ((st = ensure_red(ctx, std::max(np, pcg_parts(ctx))))) return st;
  launch_gershgorin(ctx, ctx->d_red, np);
  LAUNCHCHK();
  std::vector<double> h(np);
  HIPCHK(hipMemcpyAsync(h.data(), ctx->d_red, (size_t)np * 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double m = 0.0;
  for (double v : h) m = std::max(m, v);
  if (!(m > 0.0) || !std::isfinite(m)) FAIL(STS_EINVAL, "operator has no finite nonzero rows");
  ctx->dt_euler = 2.0 / m;
  *dt_e = ctx->dt_euler;
  return STS_OK;
}

sts_status apply_F(sts_ctx *ctx, const double *u, double *Fu, int ncomp) {
  if (!ctx) return STS_EINVAL;
  if (ctx->op == OP_NONE) FAIL(STS_EINVAL, "no operator set");
  if (!u || !Fu || u == Fu) FAIL(STS_EINVAL, "apply_F: null or aliased arrays");
  if (ncomp < 1 || ncomp > 16) FAIL(STS_EINVAL, "apply_F: ncomp must be in [1, 16]");
  if (ctx->prec == 1)
    f32_apply(ctx, ncomp, u, Fu);
  else
    launch_stage(ctx, 0, ncomp, u, nullptr, nullptr, nullptr, Fu, 0, 0, 0, 0);
  LAUNCHCHK();
  return STS_OK;
}

// FP32 form of the super-step: increments delta_k = u_k - u_0 in FP32,
//   delta_1 = mu~_1 dt F0,
//   delta_k = mu_k delta_{k-1} + nu_k delta_{k-2} + mu~_k dt M delta_{k-1}
//             + (mu~_k + gamma~_k) dt F0,
// (F affine: F(u_{k-1}) = F0 + M delta_{k-1}), u^{n+1} = u_0 + delta_s in FP64.
// ws: 3 * ncell * ncomp floats of workspace, or nullptr for the context's own
// (allocated at the first call that needs it).
static sts_status rkl2_step_f32(sts_ctx *ctx, double *u, int ncomp, double dt, int s,
                                float *ws = nullptr) {
  const long long n = ctx->ncell * ncomp;
  if (!ws && ctx->rk32_ncomp < ncomp) {
    dfree(ctx->d_rk32);
    ctx->rk32_ncomp = 0;
    sts_status st = dalloc(ctx, (void **)&ctx->d_rk32, (size_t)3 * n * 4);
    if (st) return st;
    ctx->rk32_ncomp = ncomp;
  }
  float *const W = ws ? ws : ctx->d_rk32;
  float *F0 = W, *Da = W + n, *Db = W + 2 * n;
  const double ss = (double)s * s + s - 2.0;
  auto bk = [](int k) { return k <= 2 ? 1.0 / 3.0 : ((double)k * k + k - 2.0) / (2.0 * k * (k + 1.0)); };
  const double w1 = 4.0 / ss;
  f32_F0(ctx, ncomp, u, F0, Da, (w1 / 3.0) * dt);
  LAUNCHCHK();
  for (int k = 2; k <= s; ++k) {
    const double b = bk(k), b1 = bk(k - 1), b2 = bk(k - 2);
    const double mu = (2.0 * k - 1.0) / k * b / b1;
    const double nu = -(k - 1.0) / k * b / b2;
    const double mut = 4.0 * (2.0 * k - 1.0) / (k * ss) * b / b1;
    const double gt = -(1.0 - b1) * mut;
    const float *dkm1 = ((k - 1) & 1) ? Da : Db;
    // delta_0 = 0: at k = 2 the nu term vanishes (any finite buffer is read)
    const float *dkm2 = (k == 2) ? Da : (((k - 2) & 1) ? Da : Db);
    const double nuk = (k == 2) ? 0.0 : nu;
    const bool last = k == s;
    void *out = last ? (void *)u : (void *)((k & 1) ? Da : Db);
    f32_stage(ctx, last, ncomp, dkm1, dkm2, F0, out, u, mu, nuk, mut * dt, (mut + gt) * dt);
    LAUNCHCHK();
  }
  return STS_OK;
}

// RKL workspace: F0 and the state buffers, ncell * ncomp each
static sts_status rk_workspace(sts_ctx *ctx, int ncomp) {
  const long long n = ctx->ncell * ncomp;
  if (ctx->rk_ncomp < ncomp) {
    dfree(ctx->d_rk);
    ctx->rk_ncomp = 0;
    sts_status st = dalloc(ctx, (void **)&ctx->d_rk, (size_t)(1 + kRkBuffers) * n * 8);
    if (st) return st;
    ctx->rk_ncomp = ncomp;
  }
  return STS_OK;
}

// The conduction operator with kappa taken from each stage value (nullptr:
// the context's stored operator).
struct NlSpitzer {
  double kappa0;
  const double *b0, *b1, *b2;
};

// One super-step of s stages in FP64: scheme 2 = RKL2 (Sec. 3, Fig. "rkl2"),
// scheme 1 = RKL1 (the first-order member of the same family).
// ws: (1 + kRkBuffers) * ncell * ncomp doubles of workspace, or nullptr for the
// context's own (allocated at the first call that needs it).
static sts_status rk_fp64(sts_ctx *ctx, double *u, int ncomp, double dt, int s, int scheme,
                          const NlSpitzer *nl = nullptr, double *ws = nullptr) {
  if (!ws) {
    sts_status st0 = rk_workspace(ctx, ncomp);
    if (st0) return st0;
  }
  const long long n = ctx->ncell * ncomp;
  double *const W = ws ? ws : ctx->d_rk;
  double *F0 = W;
  double *P[kRkBuffers];
  for (int q = 0; q < kRkBuffers; ++q) P[q] = W + (1 + q) * n;
  // stage coefficients (Sec. 3): b_k, mu_k, nu_k, mu~_k, gamma~_k
  const double ss = (double)s * s + s - 2.0;
  auto bk = [](int k) { return k <= 2 ? 1.0 / 3.0 : ((double)k * k + k - 2.0) / (2.0 * k * (k + 1.0)); };
  // RKL1 (scheme 1): mu_k = (2k-1)/k, nu_k = -(k-1)/k, mu~_k = w1 (2k-1)/k,
  // w1 = 2/(s^2+s), no u_0 or F0 terms (mu_k + nu_k = 1, gamma~_k = 0)
  const double w1r1 = 2.0 / ((double)s * s + s);
  auto coef = [&](int k, double out[4]) {
    if (scheme == 1) {
      out[0] = (2.0 * k - 1.0) / k;
      out[1] = -(k - 1.0) / k;
      out[2] = w1r1 * (2.0 * k - 1.0) / k * dt;
      out[3] = 0.0;
      return;
    }
    const double b = bk(k), b1 = bk(k - 1), b2 = bk(k - 2);
    const double mut = 4.0 * (2.0 * k - 1.0) / (k * ss) * b / b1;
    out[0] = (2.0 * k - 1.0) / k * b / b1;  // mu_k
    out[1] = -(k - 1.0) / k * b / b2;       // nu_k
    out[2] = mut * dt;                      // mu~_k dt
    out[3] = -(1.0 - b1) * mut * dt;        // gamma~_k dt
  };
  const double mut1 = scheme == 1 ? w1r1 * dt : (4.0 / ss / 3.0) * dt;
  auto stage = [&](int mode, const double *ukm1, const double *ukm2, double *out,
                   const double c[4]) {
    if (nl)
      launch_stage_nl(ctx, mode, ukm1, ukm2, u, F0, out, c[0], c[1], c[2], c[3], nl->kappa0,
                      nl->b0, nl->b1, nl->b2);
    else
      launch_stage(ctx, mode, ncomp, ukm1, ukm2, u, F0, out, c[0], c[1], c[2], c[3]);
  };
  const double c1st[4] = {0.0, 0.0, mut1, 0.0};
  stage(1, u, nullptr, P[0], c1st);
  LAUNCHCHK();
  if (s == 1) {  // RKL1 with one stage: explicit Euler
    HIPCHK(hipMemcpyAsync(u, P[0], (size_t)n * 8, hipMemcpyDeviceToDevice, ctx->stream));
    return STS_OK;
  }
  LAUNCHCHK();
  // u_{k-1} in prev1, u_{k-2} in prev2 (u_0 = u for k = 2).  A stage reads
  // u_{k-2} only at its own cell, so it may overwrite it; the last stage
  // writes u in place (it reads u_0 only at its own cell).
  const double *prev1 = P[0], *prev2 = u;
  auto free_buf = [&](const double *x, const double *y, const double *z) {
    for (int q = 0; q < kRkBuffers; ++q)
      if (P[q] != x && P[q] != y && P[q] != z) return P[q];
    return (double *)nullptr;
  };
  for (int k = 2; k <= s; ++k) {
    double c1[4];
    coef(k, c1);
    double *out = (k == s) ? u : (prev2 != u ? (double *)prev2 : free_buf(prev1, prev2, nullptr));
    stage(2, prev1, prev2, out, c1);
    LAUNCHCHK();
    prev2 = prev1;
    prev1 = out;
  }
  return STS_OK;
}

// Argument checks and the stage count shared by rkl2_step and
// rkl2_step_noalloc.  With need_cached_dte, s <= 0 requires dt_E to have
// been computed already (its reduction may allocate).
static sts_status rkl2_prepare(sts_ctx *ctx, const char *name, double *u, int ncomp, double dt,
                               int *s, bool need_cached_dte) {
  if (!ctx) return STS_EINVAL;
  const std::string nm(name);
  if (ctx->op == OP_NONE) FAIL(STS_EINVAL, "no operator set");
  if (!u) FAIL(STS_EINVAL, nm + ": null u");
  if (ncomp < 1 || ncomp > 16) FAIL(STS_EINVAL, nm + ": ncomp must be in [1, 16]");
  if (!(dt > 0.0) || !std::isfinite(dt)) FAIL(STS_EINVAL, nm + ": dt must be finite, > 0");
  if (*s <= 0) {
    if (need_cached_dte && !(ctx->dt_euler > 0))
      FAIL(STS_EINVAL, nm + ": s <= 0 needs dt_E, not yet computed for this operator "
                            "(call sts_dt_euler first)");
    double dte;
    sts_status st = sts_dt_euler(ctx, &dte);
    if (st) return st;
    const double ratio = dt / dte;
    if (!(ratio < 0.25 * kMaxStages * (double)kMaxStages)) FAIL(STS_EINVAL, "dt too large");
    *s = stage_count(ratio);
  }
  if (*s < 2 || *s > kMaxStages) FAIL(STS_EINVAL, nm + ": s must be >= 2");
  return STS_OK;
}

sts_status rkl2_step(sts_ctx *ctx, double *u, int ncomp, double dt, int s, int *s_used) {
  sts_status st = rkl2_prepare(ctx, "rkl2_step", u, ncomp, dt, &s, false);
  if (st) return st;
  if (s_used) *s_used = s;
  if (ctx->prec == 1) return rkl2_step_f32(ctx, u, ncomp, dt, s);
  return rk_fp64(ctx, u, ncomp, dt, s, 2);
}

sts_status rkl2_step_noalloc(sts_ctx *ctx, double *u, int ncomp, double dt, int s,
                             int *s_used) {
  sts_status st = rkl2_prepare(ctx, "rkl2_step_noalloc", u, ncomp, dt, &s, true);
  if (st) return st;
  if (!ctx->d_scratch)
    FAIL(STS_EHIP, "rkl2_step_noalloc: the static scratch array has no device address: " +
                       ctx->scratch_err);
  const long long n = ctx->ncell * ncomp;
  const long long need = ctx->prec == 1 ? 3 * n * 4 : (long long)(1 + kRkBuffers) * n * 8;
  if (need > (long long)kScratchBytes)
    FAIL(STS_EINVAL, "rkl2_step_noalloc: needs " + std::to_string(need) +
                         " bytes of scratch, above its " + std::to_string(kScratchBytes) +
                         " (at most " + std::to_string(kScratchBytes / (ctx->prec == 1 ? 12 : 24)) +
                         " cells x components)");
  if (s_used) *s_used = s;
  if (ctx->prec == 1) return rkl2_step_f32(ctx, u, ncomp, dt, s, (float *)ctx->d_scratch);
  return rk_fp64(ctx, u, ncomp, dt, s, 2, nullptr, (double *)ctx->d_scratch);
}


sts_status apply_F_nonlinear(sts_ctx *ctx, const double *u, double *Fu, double kappa0,
                             const double *b0, const double *b1, const double *b2) {
  if (!ctx) return STS_EINVAL;
  if (!u || !Fu || u == Fu) FAIL(STS_EINVAL, "apply_F_nonlinear: null or aliased arrays");
  if (!b0 || !b1 || !b2) FAIL(STS_EINVAL, "apply_F_nonlinear: null b");
  if (!(kappa0 > 0.0) || !std::isfinite(kappa0)) FAIL(STS_EINVAL, "kappa0 must be finite, > 0");
  sts_status st = refresh_dirichlet_values(ctx);
  if (st) return st;
  launch_stage_nl(ctx, 0, u, nullptr, nullptr, nullptr, Fu, 0, 0, 0, 0, kappa0, b0, b1, b2);
  LAUNCHCHK();
  return STS_OK;
}

sts_status rkl2_step_nonlinear(sts_ctx *ctx, double *u, double dt, double kappa0,
                               const double *b0, const double *b1, const double *b2, int s,
                               int *s_used) {
  if (!ctx) return STS_EINVAL;
  if (!u) FAIL(STS_EINVAL, "rkl2_step_nonlinear: null u");
  if (!(dt > 0.0) || !std::isfinite(dt))
    FAIL(STS_EINVAL, "rkl2_step_nonlinear: dt must be finite, > 0");
  if (s > kMaxStages || s == 1) FAIL(STS_EINVAL, "rkl2_step_nonlinear: s must be >= 2");
  // the operator at u^n: input checks, Dirichlet weights, dt_E
  sts_status st = sts_set_spitzer(ctx, u, kappa0, b0, b1, b2);
  if (st) return st;
  if (s <= 0) {
    double dte;
    if ((st = sts_dt_euler(ctx, &dte))) return st;
    const double ratio = dt / dte;
    if (!(ratio < 0.25 * kMaxStages * (double)kMaxStages)) FAIL(STS_EINVAL, "dt too large");
    s = stage_count(ratio);
  }
  if (s_used) *s_used = s;
  const NlSpitzer nl{kappa0, b0, b1, b2};
  return rk_fp64(ctx, u, 1, dt, s, 2, &nl);
}

sts_status rkl_step(sts_ctx *ctx, double *u, int ncomp, double dt, int scheme, int extra,
                    int odd, int nsub, double euler_fraction, double euler_cfl, int *n_apply) {
  if (!ctx) return STS_EINVAL;
  if (ctx->op == OP_NONE) FAIL(STS_EINVAL, "no operator set");
  if (!u) FAIL(STS_EINVAL, "rkl_step: null u");
  if (ncomp < 1 || ncomp > 16) FAIL(STS_EINVAL, "rkl_step: ncomp must be in [1, 16]");
  if (!(dt > 0.0) || !std::isfinite(dt)) FAIL(STS_EINVAL, "rkl_step: dt must be finite, > 0");
  if (scheme != 1 && scheme != 2) FAIL(STS_EINVAL, "rkl_step: scheme must be 1 or 2");
  if (extra < 0 || extra > 1000) FAIL(STS_EINVAL, "rkl_step: extra must be in [0, 1000]");
  if (nsub < 1 || nsub > 10000) FAIL(STS_EINVAL, "rkl_step: nsub must be in [1, 10000]");
  if (!(euler_fraction >= 0.0 && euler_fraction < 1.0))
    FAIL(STS_EINVAL, "rkl_step: euler_fraction must be in [0, 1)");
  if (euler_fraction > 0.0 && !(euler_cfl > 0.0 && euler_cfl <= 1.0))
    FAIL(STS_EINVAL, "rkl_step: euler_cfl must be in (0, 1]");
  if (ctx->prec == 1 && (scheme != 2 || euler_fraction > 0.0))
    FAIL(STS_EINVAL, "rkl_step: the FP32 form supports RKL2 sub-steps only");
  double dte;
  sts_status st = sts_dt_euler(ctx, &dte);
  if (st) return st;
  int napply = 0;
  // explicit Euler sub-steps over euler_fraction * dt, each at most euler_cfl * dt_E
  double rest = dt;
  if (euler_fraction > 0.0) {
    const double span = euler_fraction * dt;
    const double ne = std::ceil(span / (euler_cfl * dte) - 1e-12);
    if (!(ne < 1e7)) FAIL(STS_EINVAL, "rkl_step: too many Euler sub-steps");
    const int n_e = std::max(1, (int)ne);
    const double h = span / n_e;
    if ((st = rk_workspace(ctx, ncomp))) return st;
    const long long n = ctx->ncell * ncomp;
    double *F0 = ctx->d_rk, *tmp = ctx->d_rk + n;
    for (int q = 0; q < n_e; ++q) {
      launch_stage(ctx, 1, ncomp, u, nullptr, u, F0, tmp, 0, 0, h, 0);  // tmp = u + h F(u)
      LAUNCHCHK();
      HIPCHK(hipMemcpyAsync(u, tmp, (size_t)n * 8, hipMemcpyDeviceToDevice, ctx->stream));
    }
    napply += n_e;
    rest = dt - n_e * h;
  }
  if (rest > 0.0) {
    const double ds = rest / nsub, ratio = ds / dte;
    if (!(ratio < 0.25 * kMaxStages * (double)kMaxStages)) FAIL(STS_EINVAL, "dt too large");
    int s;
    if (scheme == 2) {
      s = stage_count(ratio) + extra;
    } else {
      s = std::max(1, (int)std::ceil((std::sqrt(1.0 + 8.0 * ratio) - 1.0) / 2.0));
      while (s > 1 && (double)(s - 1) * s >= 2.0 * ratio) --s;
      while ((double)s * s + s < 2.0 * ratio) ++s;
      s += extra;
    }
    if (odd && s % 2 == 0) ++s;
    if (s > kMaxStages) FAIL(STS_EINVAL, "rkl_step: too many stages");
    for (int q = 0; q < nsub; ++q) {
      st = ctx->prec == 1 ? rkl2_step_f32(ctx, u, ncomp, ds, s) : rk_fp64(ctx, u, ncomp, ds, s, scheme);
      if (st) return st;
    }
    napply += nsub * s;
  }
  if (n_apply) *n_apply = napply;
  return STS_OK;
}

static sts_status pcg_workspace(sts_ctx *ctx, int pc, const int block[3], double **fac) {
  const long long n = ctx->ncell;
  sts_status st;
  if ((st = dalloc(ctx, (void **)&ctx->d_pcg, (size_t)7 * n * 8))) return st;
  int need = pcg_parts(ctx);
  if (pc == STS_PC_BLOCK_ILU0) need = std::max(need, ilu_parts(ctx, block));
  if (pc == STS_PC_FACTOR) {
    need = std::max(need, pc_parts(ctx));
    if (!ctx->d_pct && (st = dalloc(ctx, (void **)&ctx->d_pct, (size_t)n * 8))) return st;
  }
  if ((st = ensure_red(ctx, need))) return st;
  *fac = nullptr;
  if (pc == STS_PC_BLOCK_ILU0) {
    const long long need_f = (long long)ilu_nblocks(ctx, block) * 10 * block[0] * block[1] * block[2];
    if (ctx->ilu_cap < need_f) {
      dfree(ctx->d_ilu);
      ctx->ilu_cap = 0;
      if ((st = dalloc(ctx, (void **)&ctx->d_ilu, (size_t)need_f * 8))) return st;
      ctx->ilu_cap = need_f;
    }
    *fac = ctx->d_ilu;
  }
  return STS_OK;
}

}  // extern "C"

// PCG iterations in batches of kPollEvery.  Each batch's scalars are copied
// behind it into one of two pinned slots and an event is recorded; the host
// waits for batch b's copy only after enqueuing batch b + 1, so the device
// never idles during the host's round trip.  Batches enqueued after
// convergence exit at once (the device also stops at sc->maxit).  On return
// the first slot holds the final scalars.  one(it) enqueues iteration it.
template <class F>
static sts_status pcg_iterate(sts_ctx *ctx, const PcgScalars *sc, int maxit, F &&one) {
  PcgScalars *slot[2] = {(PcgScalars *)ctx->h_pin, (PcgScalars *)((char *)ctx->h_pin + 128)};
  static_assert(sizeof(PcgScalars) <= 128, "two scalar slots in the pinned buffer");
  for (hipEvent_t &e : ctx->ev)
    if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  bool stop = slot[0]->done != 0;  // the caller's copy after the initialisation
  for (int it = 0, batch = 0; !stop && it < maxit; ++batch) {
    const int nb = std::min(kPollEvery, maxit - it);
    for (int q = 0; q < nb; ++q, ++it) one(it);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(slot[batch & 1], sc, sizeof(PcgScalars), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipEventRecord(ctx->ev[batch & 1], ctx->stream));
    if (batch > 0) {
      HIPCHK(hipEventSynchronize(ctx->ev[(batch - 1) & 1]));
      stop = slot[(batch - 1) & 1]->done != 0;
    }
  }
  HIPCHK(hipMemcpyAsync(slot[0], sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return STS_OK;
}

extern "C" {

// FP32 form of BE + Jacobi-PCG: mixed-precision iterative refinement.  The
// outer residual r = b - A x is formed in FP64 (FP32 coefficients widened);
// the correction A e = r is solved by PCG with FP32 vectors and FP64 dot
// products / alpha / beta / norms to a loose relative tolerance; x += e.
// Stops when the FP64 residual meets rtol; *iters counts inner iterations.
constexpr double kInnerTol = 1e-4;
constexpr int kMaxOuter = 30;
static sts_status be_pcg_solve_f32(sts_ctx *ctx, const double *u_n, double *x, double dt,
                                   double rtol, int maxit, int *iters, double *relres) {
  double *fac;
  const int one[3] = {1, 1, 1};
  sts_status st = pcg_workspace(ctx, STS_PC_JACOBI, one, &fac);
  if (st) return st;
  const long long n = ctx->ncell, cap = ctx->red_cap;
  if ((st = dalloc(ctx, (void **)&ctx->d_pcg32, (size_t)7 * n * 4))) return st;
  double *b = ctx->d_pcg, *invd = b + n, *r64 = b + 2 * n;
  float *iv = ctx->d_pcg32, *e = iv + n, *r = iv + 2 * n, *p0 = iv + 3 * n, *p1 = iv + 4 * n,
        *y = iv + 5 * n, *z = iv + 6 * n;
  double *part = ctx->d_red;
  PcgScalars *sc = ctx->d_sc, *h = (PcgScalars *)ctx->h_pin;
  launch_be_rhs(ctx, u_n, dt, b, invd, part + 2 * cap);
  LAUNCHCHK();
  const int np3 = stencil_parts(ctx), np1 = pass_b_parts(ctx);
  int total = 0;
  double rel = 1.0;
  for (int outer = 0; outer < kMaxOuter; ++outer) {
    f32_residual(ctx, b, x, dt, r64, part);
    launch_sum2(ctx, part, np3, ctx->d_tmp);
    LAUNCHCHK();
    double hh[2];
    HIPCHK(hipMemcpyAsync(hh, ctx->d_tmp, 16, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    rel = hh[1] > 0 ? std::sqrt(hh[0] / hh[1]) : 0.0;
    if (!std::isfinite(rel)) FAIL(STS_BREAKDOWN, "FP32 form: non-finite residual");
    if (rel <= rtol || total >= maxit) break;
    f32_inner_init(ctx, r64, invd, r, iv, e, z, part);
    launch_finalize_init_n(ctx, part + cap, np1, part + cap, np1, part, np1, sc, kInnerTol,
                           maxit - total);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(h, sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    float *pold = p0, *pnew = p1;
    // the finalizers run inside the sweeps up to kFuseMaxParts pass-A
    // partials, as in the FP64 Jacobi solve
    double *part_b = part + 2 * cap;
    const bool fuse = fuse_finalizers(ctx, np3);
    st = pcg_iterate(ctx, sc, maxit - total, [&](int it) {
      if (fuse) {
        f32_pass_a(ctx, dt, z, pold, pnew, y, part, sc, it == 0, part_b, np1, it);
        f32_pass_b(ctx, e, pnew, r, y, iv, z, part_b, sc, part, np3);
      } else {
        f32_pass_a(ctx, dt, z, pold, pnew, y, part, sc, it == 0);
        launch_finalize_alpha(ctx, part, np3, sc);
        f32_pass_b(ctx, e, pnew, r, y, iv, z, part_b, sc);
        launch_finalize_beta(ctx, part_b, np1, sc);
      }
      std::swap(pold, pnew);
    });
    if (st) return st;
    if (fuse && maxit - total > 0 && !h->done) {
      launch_finalize_check(ctx, part_b, np1, maxit - total, sc);
      LAUNCHCHK();
      HIPCHK(hipMemcpyAsync(h, sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    if (h->status == -4) FAIL(STS_BREAKDOWN, "FP32 form: inner PCG breakdown");
    total += h->iters;
    f32_add_to(ctx, x, e);
    LAUNCHCHK();
  }
  if (iters) *iters = total;
  if (relres) *relres = rel;
  if (rel <= rtol) return STS_OK;
  ctx->err = "PCG reached maxit";
  return STS_NOT_CONVERGED;
}

sts_status be_pcg_solve(sts_ctx *ctx, const double *u_n, double *x, double dt, int pc,
                        const int block[3], double rtol, int maxit, int *iters, double *relres) {
  if (!ctx) return STS_EINVAL;
  if (ctx->op == OP_NONE) FAIL(STS_EINVAL, "no operator set");
  if (!u_n || !x || u_n == x) FAIL(STS_EINVAL, "be_pcg_solve: null or aliased u_n / x");
  if (!(dt > 0.0) || !std::isfinite(dt)) FAIL(STS_EINVAL, "be_pcg_solve: dt must be finite, > 0");
  if (!(rtol >= 0.0) || !std::isfinite(rtol)) FAIL(STS_EINVAL, "be_pcg_solve: bad rtol");
  if (maxit < 0) FAIL(STS_EINVAL, "be_pcg_solve: maxit must be >= 0");
  if (pc != STS_PC_JACOBI && pc != STS_PC_BLOCK_ILU0 && pc != STS_PC_FACTOR)
    FAIL(STS_EINVAL, "unknown preconditioner");
  if (pc == STS_PC_FACTOR && !ctx->gfac_set)
    FAIL(STS_EINVAL, "STS_PC_FACTOR needs a factor (sts_set_pc_factor or cnn_pc_factor)");
  int blk[3] = {1, 1, 1};
  if (pc == STS_PC_BLOCK_ILU0) {
    if (!block) FAIL(STS_EINVAL, "block ILU0 needs block[3]");
    for (int a = 0; a < 3; ++a) {
      if (block[a] < 1 || block[a] > 8) FAIL(STS_EINVAL, "ILU0 block sizes must be in [1, 8]");
      blk[a] = block[a];
    }
  }
  if (ctx->prec == 1) {
    if (pc != STS_PC_JACOBI) FAIL(STS_EINVAL, "the FP32 form supports the Jacobi preconditioner");
    return be_pcg_solve_f32(ctx, u_n, x, dt, rtol, maxit, iters, relres);
  }
  double *fac;
  sts_status st = pcg_workspace(ctx, pc, blk, &fac);
  if (st) return st;
  const long long n = ctx->ncell, cap = ctx->red_cap;
  double *b = ctx->d_pcg, *invd = b + n, *r = b + 2 * n, *p0 = b + 3 * n, *p1 = b + 4 * n,
         *y = b + 5 * n, *z = b + 6 * n;
  double *part = ctx->d_red;
  PcgScalars *sc = ctx->d_sc;
  const bool ilu = pc == STS_PC_BLOCK_ILU0, fpc = pc == STS_PC_FACTOR;

  launch_be_rhs(ctx, u_n, dt, b, invd, part + 2 * cap);
  LAUNCHCHK();
  launch_residual_init(ctx, b, x, dt, invd, nullptr, r, nullptr, part);
  LAUNCHCHK();
  if (ilu) {
    HIPCHK(hipMemsetAsync(ctx->d_flag, 0, sizeof(int), ctx->stream));
    launch_ilu_factor(ctx, dt, blk, fac, ctx->d_flag);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(ctx->h_pin, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (*(int *)ctx->h_pin) FAIL(STS_BREAKDOWN, "ILU0 breakdown: non-positive pivot");
    launch_ilu_apply_init(ctx, blk, fac, r, z);
    LAUNCHCHK();
  }
  if (fpc) {  // z = G (G^T r)
    launch_pc_gt(ctx, ctx->d_gfac, r, nullptr, ctx->d_pct, nullptr);
    launch_pc_g(ctx, ctx->d_gfac, ctx->d_pct, z, nullptr);
    LAUNCHCHK();
  }
  // every preconditioner keeps z in its own array: pass A forms p = z + beta p
  // from two streamed arrays
  const bool zgiven = ilu || fpc;
  launch_init_p(ctx, r, invd, zgiven ? z : nullptr, p0, part + 2 * cap, zgiven ? nullptr : z);
  LAUNCHCHK();
  launch_finalize_init3(ctx, part + cap, part, part + 2 * cap, sc, rtol, maxit);
  LAUNCHCHK();

  const int nb_parts = ilu ? ilu_parts(ctx, blk) : (fpc ? pc_parts(ctx) : pass_b_parts(ctx));
  PcgScalars *h = (PcgScalars *)ctx->h_pin;
  double *pold = p0, *pnew = p1;
  HIPCHK(hipMemcpyAsync(h, sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  const int np3 = stencil_parts(ctx);
  // Jacobi: two launches per iteration.  Pass B forms alpha from pass A's
  // partials (region 0) and writes its own to regions 2 and 3; the next pass A
  // evaluates the stopping test and beta from those, so no kernel sits
  // between the sweeps (-4 to -5 % per solve, conduction and viscosity).
  // Block ILU0 keeps the separate finalizers (fused, its latency-bound solve
  // sweep measured no faster).  Beyond kFuseMaxParts pass-A partials, and
  // with STS_DEBUG_SEPARATE_FINALIZE, Jacobi takes the four-launch form
  // (single-workgroup finalizers) as well.
  double *part_b = part + 2 * cap;
  const bool fuse = fuse_finalizers(ctx, np3);
  // the factor's second residual array: 1 / A_ii is not used after the start
  double *rcur = r, *ralt = invd;
  st = pcg_iterate(ctx, sc, maxit, [&](int it) {
    if (ilu) {
      launch_pass_a(ctx, dt, z, pold, pnew, y, part, sc, it == 0);
      launch_finalize_alpha(ctx, part, np3, sc);
      launch_pass_b_ilu(ctx, blk, fac, x, pnew, r, y, z, part, sc);
      launch_finalize_beta(ctx, part, nb_parts, sc);
    } else if (fpc) {
      // pass B updates x and r and forms t = G^T r (r ping-pongs between two
      // arrays: the sweep reads its neighbours' old r), with r.z = t.t;
      // z = G t follows.  The finalizers run inside the sweeps as for Jacobi.
      if (fuse) {
        launch_pass_a(ctx, dt, z, pold, pnew, y, part, sc, it == 0, part_b, nb_parts, it);
        launch_pc_xr_gt(ctx, ctx->d_gfac, x, pnew, rcur, ralt, y, ctx->d_pct, part_b, sc, part,
                        np3);
      } else {
        launch_pass_a(ctx, dt, z, pold, pnew, y, part, sc, it == 0);
        launch_finalize_alpha(ctx, part, np3, sc);
        launch_pc_xr_gt(ctx, ctx->d_gfac, x, pnew, rcur, ralt, y, ctx->d_pct, part_b, sc,
                        nullptr, 0);
        launch_finalize_beta(ctx, part_b, nb_parts, sc);
      }
      launch_pc_g(ctx, ctx->d_gfac, ctx->d_pct, z, sc);
      std::swap(rcur, ralt);
    } else if (fuse) {
      launch_pass_a(ctx, dt, z, pold, pnew, y, part, sc, it == 0, part_b, nb_parts, it);
      launch_pass_b_jacobi_fused(ctx, x, pnew, r, y, invd, z, part_b, sc, part, np3);
    } else {
      launch_pass_a(ctx, dt, z, pold, pnew, y, part, sc, it == 0);
      launch_finalize_alpha(ctx, part, np3, sc);
      launch_pass_b_jacobi(ctx, x, pnew, r, y, invd, z, part_b, sc);
      launch_finalize_beta(ctx, part_b, nb_parts, sc);
    }
    std::swap(pold, pnew);
  });
  if (st) return st;
  if (!ilu && fuse && maxit > 0 && !h->done) {
    // every one of the maxit iterations ran; evaluate the last one's end
    launch_finalize_check(ctx, part_b, nb_parts, maxit, sc);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(h, sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  if (iters) *iters = h->iters;
  if (relres) *relres = h->bnorm2 > 0 ? std::sqrt(h->rnorm2 / h->bnorm2) : 0.0;
  if (h->status == -4) FAIL(STS_BREAKDOWN, "PCG breakdown: p.Ap <= 0 or non-finite residual");
  if (h->status == 1) return STS_OK;
  ctx->err = "PCG reached maxit";
  return STS_NOT_CONVERGED;
}

}  // extern "C"

// ---- the factored preconditioner M^-1 = G G^T ------------------------------
// (the sts_* entry points keep the C linkage of their declarations in sts.h)

static sts_status pc_factor_storage(sts_ctx *ctx) {
  if (!ctx->d_gfac) return dalloc(ctx, (void **)&ctx->d_gfac, (size_t)4 * ctx->ncell * 2);
  return STS_OK;
}

sts_status sts_set_pc_factor(sts_ctx *ctx, const float *g) {
  if (!ctx) return STS_EINVAL;
  if (!g) FAIL(STS_EINVAL, "sts_set_pc_factor: null factor");
  sts_status st = pc_factor_storage(ctx);
  if (st) return st;
  HIPCHK(hipMemsetAsync(ctx->d_flag, 0, sizeof(int), ctx->stream));
  launch_pc_check(ctx, g, ctx->d_gfac, ctx->d_flag);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(ctx->h_pin, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (*(int *)ctx->h_pin) {
    ctx->gfac_set = false;
    FAIL(STS_EINVAL, "sts_set_pc_factor: diagonal entries must be finite and > 0, the others "
                     "finite");
  }
  ctx->gfac_set = true;
  return STS_OK;
}

// Network-built factor (cnn_pc_factor): o4 [cells][4] outputs (null: Jacobi).
// Returns STS_BREAKDOWN (factor left unset) if an entry is not finite.
sts_status sts::build_pc_factor(sts_ctx *ctx, double dt, const float *o4) {
  sts_status st = pc_factor_storage(ctx);
  if (st) return st;
  HIPCHK(hipMemsetAsync(ctx->d_flag, 0, sizeof(int), ctx->stream));
  launch_pc_build(ctx, dt, o4, ctx->d_gfac, ctx->d_flag);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(ctx->h_pin, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->gfac_set = *(int *)ctx->h_pin == 0;
  if (!ctx->gfac_set) FAIL(STS_BREAKDOWN, "factor with a non-finite entry");
  return STS_OK;
}

sts_status sts_apply_pc_factor(sts_ctx *ctx, const double *r, double *z) {
  if (!ctx) return STS_EINVAL;
  if (!ctx->gfac_set) FAIL(STS_EINVAL, "sts_apply_pc_factor: no factor set");
  if (!r || !z || r == z) FAIL(STS_EINVAL, "sts_apply_pc_factor: null or aliased arrays");
  sts_status st;
  if (!ctx->d_pct && (st = dalloc(ctx, (void **)&ctx->d_pct, (size_t)ctx->ncell * 8))) return st;
  launch_pc_gt(ctx, ctx->d_gfac, r, nullptr, ctx->d_pct, nullptr);
  launch_pc_g(ctx, ctx->d_gfac, ctx->d_pct, z, nullptr);
  LAUNCHCHK();
  return STS_OK;
}

// Vectors of the objective: w, y, r, q, s, p (scratch of pass A), 6 x ncell.
static sts_status pc_objective_workspace(sts_ctx *ctx) {
  sts_status st;
  if ((st = ensure_red(ctx, std::max(pcg_parts(ctx), pc_parts(ctx))))) return st;
  if (!ctx->d_pcobj && (st = dalloc(ctx, (void **)&ctx->d_pcobj, (size_t)6 * ctx->ncell * 8)))
    return st;
  if (!ctx->d_sc0) {
    if ((st = dalloc(ctx, (void **)&ctx->d_sc0, sizeof(PcgScalars)))) return st;
    HIPCHK(hipMemsetAsync(ctx->d_sc0, 0, sizeof(PcgScalars), ctx->stream));
  }
  return STS_OK;
}

// w = G z, y = A w, r = G^T y - z, q = G r, s = A q, then the gradient
// kernel (dg and / or the network's output gradient dout) and r.r partials.
sts_status sts::pc_objective_sweeps(sts_ctx *ctx, double dt, const double *z, double *dg,
                                    void *dout) {
  sts_status st = pc_objective_workspace(ctx);
  if (st) return st;
  const long long n = ctx->ncell;
  double *w = ctx->d_pcobj, *y = w + n, *r = w + 2 * n, *q = w + 3 * n, *s = w + 4 * n,
         *p = w + 5 * n;
  double *part = ctx->d_red;
  const void *g = ctx->d_gfac;
  launch_pc_g(ctx, g, z, w, nullptr);
  launch_pass_a(ctx, dt, w, nullptr, p, y, part, ctx->d_sc0, 1);
  launch_pc_gt(ctx, g, y, z, r, nullptr);
  launch_pc_g(ctx, g, r, q, nullptr);
  launch_pass_a(ctx, dt, q, nullptr, p, s, part, ctx->d_sc0, 1);
  launch_pc_grad(ctx, dt, g, y, r, s, z, dg, dout, part);
  LAUNCHCHK();
  return STS_OK;
}

sts_status sts_pc_objective(sts_ctx *ctx, double dt, const double *z, double *loss, double *dg) {
  if (!ctx || !loss) return STS_EINVAL;
  if (ctx->op == OP_NONE) FAIL(STS_EINVAL, "no operator set");
  if (ctx->prec != 0) FAIL(STS_EINVAL, "sts_pc_objective: FP64 operators only");
  if (!ctx->gfac_set) FAIL(STS_EINVAL, "sts_pc_objective: no factor set");
  if (!z) FAIL(STS_EINVAL, "sts_pc_objective: null z");
  if (!(dt > 0.0) || !std::isfinite(dt)) FAIL(STS_EINVAL, "dt must be finite, > 0");
  sts_status st = sts::pc_objective_sweeps(ctx, dt, z, dg, nullptr);
  if (st) return st;
  launch_sum2(ctx, ctx->d_red, pc_parts(ctx), ctx->d_tmp);
  LAUNCHCHK();
  double h[2];
  HIPCHK(hipMemcpyAsync(h, ctx->d_tmp, 16, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *loss = h[0] / (double)ctx->ncell;
  return STS_OK;
}

extern "C" {

sts_status sts_be_residual(sts_ctx *ctx, const double *u_n, const double *x, double dt,
                           double *relres) {
  if (!ctx || !relres) return STS_EINVAL;
  if (ctx->op == OP_NONE) FAIL(STS_EINVAL, "no operator set");
  if (!u_n || !x) FAIL(STS_EINVAL, "null array");
  if (!(dt > 0.0) || !std::isfinite(dt)) FAIL(STS_EINVAL, "dt must be finite, > 0");
  double *fac;
  const int one[3] = {1, 1, 1};
  sts_status st = pcg_workspace(ctx, STS_PC_JACOBI, one, &fac);
  if (st) return st;
  const long long n = ctx->ncell, cap = ctx->red_cap;
  double *b = ctx->d_pcg, *invd = b + n;
  launch_be_rhs(ctx, u_n, dt, b, invd, ctx->d_red + 2 * cap);
  launch_true_residual(ctx, b, x, dt, ctx->d_red);
  launch_sum2(ctx, ctx->d_red, stencil_parts(ctx), ctx->d_tmp);
  LAUNCHCHK();
  double h[2];
  HIPCHK(hipMemcpyAsync(h, ctx->d_tmp, 16, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *relres = h[1] > 0 ? std::sqrt(h[0] / h[1]) : 0.0;
  return STS_OK;
}

// ---------------------------------------------------------------------------
// Resistive diffusion of the vector potential on cell edges (Eq. mhd:a).
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

// centres, centre gaps across each face position, and the centres before /
// after each face position of one axis (see k_resist.hip for the layout)
struct AxisGeo {
  int n, m;
  std::vector<double> f, c, d, g, cm, cp;
};

AxisGeo axis_geo(const std::vector<double> &f, bool per) {
  AxisGeo a;
  a.n = (int)f.size() - 1;
  a.m = per ? a.n : a.n + 1;
  a.f = f;
  const double P = f[a.n] - f[0];
  a.c.resize(a.n);
  a.d.resize(a.n);
  for (int q = 0; q < a.n; ++q) {
    a.c[q] = 0.5 * (f[q] + f[q + 1]);
    a.d[q] = f[q + 1] - f[q];
  }
  a.g.assign(a.n + 1, 0.0);
  for (int q = 1; q < a.n; ++q) a.g[q] = a.c[q] - a.c[q - 1];
  if (per) a.g[0] = a.g[a.n] = a.c[0] + P - a.c[a.n - 1];
  a.cm.resize(a.m);
  a.cp.resize(a.m);
  for (int q = 0; q < a.m; ++q) {
    a.cm[q] = q >= 1 ? a.c[q - 1] : (per ? a.c[a.n - 1] - P : f[0]);
    a.cp[q] = q < a.n ? a.c[q] : f[a.n];
  }
  return a;
}

}  // namespace

extern "C" {

sts_status sts_set_resistivity(sts_ctx *ctx, double eta) {
  if (!ctx) return STS_EINVAL;
  if (!(eta > 0.0) || !std::isfinite(eta)) FAIL(STS_EINVAL, "eta must be finite and > 0");
  const bool per[3] = {ctx->bc[0] == STS_BC_PERIODIC, ctx->bc[2] == STS_BC_PERIODIC,
                       ctx->bc[4] == STS_BC_PERIODIC};
  const AxisGeo A = axis_geo(ctx->hf[0], per[0]), B = axis_geo(ctx->hf[1], per[1]),
                C = axis_geo(ctx->hf[2], per[2]);
  const bool sph = ctx->coord == STS_SPHERICAL;
  // 18 tables: (H of r-, t-, p-edges, w of r-, t-, p-faces) x (axis 0, 1, 2)
  std::vector<std::vector<double>> T(18);
  auto fill = [](int n, auto fn) {
    std::vector<double> v(n + 1, 0.0);
    for (int q = 0; q < n; ++q) v[q] = fn(q);
    return v;
  };
  auto half_sq = [](double a, double b) { return 0.5 * (b * b - a * a); };
  if (sph) {
    T[0] = fill(A.n, [&](int i) { return A.c[i] * A.c[i] / A.d[i]; });
    T[1] = fill(B.m, [&](int j) { return std::cos(B.cm[j]) - std::cos(B.cp[j]); });
    T[2] = fill(C.m, [&](int k) { return C.g[k]; });
    T[3] = fill(A.m, [&](int i) { return half_sq(A.cm[i], A.cp[i]) / A.f[i]; });
    T[4] = fill(B.n, [&](int j) { return std::sin(B.c[j]) / B.d[j]; });
    T[5] = fill(C.m, [&](int k) { return C.g[k]; });
    T[6] = fill(A.m, [&](int i) { return half_sq(A.cm[i], A.cp[i]) / A.f[i]; });
    T[7] = fill(B.m, [&](int j) { return (B.cp[j] - B.cm[j]) / std::sin(B.f[j]); });
    T[8] = fill(C.n, [&](int k) { return 1.0 / C.d[k]; });
    T[9] = fill(A.m, [&](int i) { return A.g[i] / (A.f[i] * A.f[i]); });
    T[10] = fill(B.n, [&](int j) { return 1.0 / (std::cos(B.f[j]) - std::cos(B.f[j + 1])); });
    T[11] = fill(C.n, [&](int k) { return 1.0 / C.d[k]; });
    T[12] = fill(A.n, [&](int i) { return A.c[i] / half_sq(A.f[i], A.f[i + 1]); });
    T[13] = fill(B.m, [&](int j) { return B.g[j] / std::sin(B.f[j]); });
    T[14] = fill(C.n, [&](int k) { return 1.0 / C.d[k]; });
    T[15] = fill(A.n, [&](int i) { return A.c[i] / half_sq(A.f[i], A.f[i + 1]); });
    T[16] = fill(B.n, [&](int j) { return std::sin(B.c[j]) / B.d[j]; });
    T[17] = fill(C.m, [&](int k) { return C.g[k]; });
  } else {
    T[0] = fill(A.n, [&](int i) { return 1.0 / A.d[i]; });
    T[1] = fill(B.m, [&](int j) { return B.g[j]; });
    T[2] = fill(C.m, [&](int k) { return C.g[k]; });
    T[3] = fill(A.m, [&](int i) { return A.g[i]; });
    T[4] = fill(B.n, [&](int j) { return 1.0 / B.d[j]; });
    T[5] = fill(C.m, [&](int k) { return C.g[k]; });
    T[6] = fill(A.m, [&](int i) { return A.g[i]; });
    T[7] = fill(B.m, [&](int j) { return B.g[j]; });
    T[8] = fill(C.n, [&](int k) { return 1.0 / C.d[k]; });
    T[9] = fill(A.m, [&](int i) { return A.g[i]; });
    T[10] = fill(B.n, [&](int j) { return 1.0 / B.d[j]; });
    T[11] = fill(C.n, [&](int k) { return 1.0 / C.d[k]; });
    T[12] = fill(A.n, [&](int i) { return 1.0 / A.d[i]; });
    T[13] = fill(B.m, [&](int j) { return B.g[j]; });
    T[14] = fill(C.n, [&](int k) { return 1.0 / C.d[k]; });
    T[15] = fill(A.n, [&](int i) { return 1.0 / A.d[i]; });
    T[16] = fill(B.n, [&](int j) { return 1.0 / B.d[j]; });
    T[17] = fill(C.m, [&](int k) { return C.g[k]; });
  }
  std::vector<double> flat;
  for (int t = 0; t < 18; ++t) {
    ctx->res_off[t] = (int)flat.size();
    flat.insert(flat.end(), T[t].begin(), T[t].end());
  }
  ctx->res_ne[0] = (long long)A.n * B.m * C.m;
  ctx->res_ne[1] = (long long)A.m * B.n * C.m;
  ctx->res_ne[2] = (long long)A.m * B.m * C.n;
  ctx->res_nf[0] = (long long)A.m * B.n * C.n;
  ctx->res_nf[1] = (long long)A.n * B.m * C.n;
  ctx->res_nf[2] = (long long)A.n * B.n * C.m;
  const long long ne = ctx->res_ne[0] + ctx->res_ne[1] + ctx->res_ne[2];
  const long long nf = ctx->res_nf[0] + ctx->res_nf[1] + ctx->res_nf[2];
  dfree(ctx->d_rtab);
  dfree(ctx->d_rws);
  sts_status st;
  if ((st = dalloc(ctx, (void **)&ctx->d_rtab, flat.size() * 8)) ||
      (st = dalloc(ctx, (void **)&ctx->d_rws, (size_t)(2 * nf + 6 * ne) * 8)))
    return st;
  HIPCHK(hipMemcpyAsync(ctx->d_rtab, flat.data(), flat.size() * 8, hipMemcpyHostToDevice,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->res_eta = eta;
  return STS_OK;
}

sts_status sts_resistivity_sizes(const sts_ctx *ctx, long long sizes[3]) {
  if (!ctx || !sizes) return STS_EINVAL;
  const int nn[3] = {ctx->n0, ctx->n1, ctx->n2};
  int m[3];
  for (int a = 0; a < 3; ++a) m[a] = nn[a] + (ctx->bc[2 * a] == STS_BC_PERIODIC ? 0 : 1);
  sizes[0] = (long long)nn[0] * m[1] * m[2];
  sizes[1] = (long long)m[0] * nn[1] * m[2];
  sizes[2] = (long long)m[0] * m[1] * nn[2];
  return STS_OK;
}

sts_status apply_F_resistivity(sts_ctx *ctx, const double *E, double *FE) {
  if (!ctx) return STS_EINVAL;
  if (!(ctx->res_eta > 0.0)) FAIL(STS_EINVAL, "resistivity not set (sts_set_resistivity)");
  if (!E || !FE || E == FE) FAIL(STS_EINVAL, "apply_F_resistivity: null or aliased arrays");
  launch_res_F(ctx, E, FE);
  LAUNCHCHK();
  return STS_OK;
}

sts_status resistivity_dt_euler(sts_ctx *ctx, double *dt_e) {
  if (!ctx || !dt_e) return STS_EINVAL;
  if (!(ctx->res_eta > 0.0)) FAIL(STS_EINVAL, "resistivity not set (sts_set_resistivity)");
  const int np = res_parts(ctx);
  sts_status st;
  if ((st = ensure_red(ctx, np))) return st;
  launch_res_gershgorin(ctx, ctx->d_rws, ctx->d_red);
  LAUNCHCHK();
  std::vector<double> h(np);
  HIPCHK(hipMemcpyAsync(h.data(), ctx->d_red, (size_t)np * 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double m = 0.0;
  for (double v : h) m = std::max(m, v);
  if (!(m > 0.0) || !std::isfinite(m)) FAIL(STS_EINVAL, "no interior edges");
  *dt_e = 2.0 / m;
  return STS_OK;
}

sts_status resistivity_be_pcg_solve(sts_ctx *ctx, const double *E_n, double *E, double dt,
                                    double rtol, int maxit, int *iters, double *relres) {
  if (!ctx) return STS_EINVAL;
  if (!(ctx->res_eta > 0.0)) FAIL(STS_EINVAL, "resistivity not set (sts_set_resistivity)");
  if (!E_n || !E || E_n == E) FAIL(STS_EINVAL, "resistivity_be_pcg_solve: null or aliased arrays");
  if (!(dt > 0.0) || !std::isfinite(dt)) FAIL(STS_EINVAL, "dt must be finite, > 0");
  if (!(rtol >= 0.0) || !std::isfinite(rtol)) FAIL(STS_EINVAL, "bad rtol");
  if (maxit < 0) FAIL(STS_EINVAL, "maxit must be >= 0");
  // partial counts: the two-sweep right-hand side and the 1D sweeps (P), the
  // fused residual and matvec (Pf)
  const int P = res_parts(ctx), Pf = res_parts_fused(ctx);
  sts_status st;
  if ((st = ensure_red(ctx, std::max(std::max(P, Pf), pcg_parts(ctx))))) return st;
  if ((st = dalloc(ctx, (void **)&ctx->d_sc, sizeof(PcgScalars)))) return st;
  const long long ne = ctx->res_ne[0] + ctx->res_ne[1] + ctx->res_ne[2];
  const long long nf = ctx->res_nf[0] + ctx->res_nf[1] + ctx->res_nf[2];
  const long long cap = ctx->red_cap;
  double *Phi = ctx->d_rws, *Wf = Phi + nf, *b = Phi + 2 * nf, *invd = b + ne, *r = b + 2 * ne,
         *p0 = b + 3 * ne, *p1 = b + 4 * ne, *y = b + 5 * ne;
  double *part = ctx->d_red;
  PcgScalars *sc = ctx->d_sc;
  launch_res_rhs(ctx, E_n, dt, E, b, invd, Phi, Wf, part + 2 * cap);
  LAUNCHCHK();
  launch_res_residual(ctx, b, E, dt, r, part + cap);
  LAUNCHCHK();
  launch_init_p_n(ctx, ne, r, invd, p0, part, P);
  LAUNCHCHK();
  launch_finalize_init_n(ctx, part + 2 * cap, P, part + cap, Pf, part, P, sc, rtol, maxit);
  LAUNCHCHK();
  PcgScalars *h = (PcgScalars *)ctx->h_pin;
  double *pold = p0, *pnew = p1;
  HIPCHK(hipMemcpyAsync(h, sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  {
    // alpha, beta and the stopping test inside the sweeps, as in be_pcg_solve:
    // pass B's partials go to regions 2 and 3
    double *part_b = part + 2 * cap;
    const sts_status st = pcg_iterate(ctx, sc, maxit, [&](int it) {
      launch_res_pass_a(ctx, dt, r, invd, pold, pnew, y, part, sc, it == 0, part_b, P, it);
      launch_pass_b_jacobi_n(ctx, ne, E, pnew, r, y, invd, part_b, P, sc, part, Pf);
      std::swap(pold, pnew);
    });
    if (st) return st;
    if (maxit > 0 && !h->done) {
      // every one of the maxit iterations ran; evaluate the last one's end
      launch_finalize_check(ctx, part_b, P, maxit, sc);
      LAUNCHCHK();
      HIPCHK(hipMemcpyAsync(h, sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
    }
  }
  if (iters) *iters = h->iters;
  if (relres) *relres = h->bnorm2 > 0 ? std::sqrt(h->rnorm2 / h->bnorm2) : 0.0;
  if (h->status == -4) FAIL(STS_BREAKDOWN, "PCG breakdown: p.Ap <= 0 or non-finite residual");
  if (h->status == 1) return STS_OK;
  ctx->err = "PCG reached maxit";
  return STS_NOT_CONVERGED;
}

}  // extern "C"
