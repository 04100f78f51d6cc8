// C ABI of the library (declared in include/fvim.h): context management and
// the operator entry points.  Every step of the operator runs in the HIP
// kernels of fft.hip and depth.hip; this file only checks arguments, owns
// the device workspace and sequences the launches on the context stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fvim.h"
#include "common.hpp"
#include "kernels.hpp"
#include "solver.hpp"

using namespace fvim;

namespace {
thread_local std::string g_err;
}

namespace fvim {

int fail(int code, const char* msg) {
  g_err = msg;
  return code;
}

int fail_hip(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return FVIM_EHIP;
}

static bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

template <typename T>
static void* make_twiddles(int n, hipError_t* err) {
  std::vector<cpx<T>> h(n);
  for (int k = 0; k < n; ++k) {
    // exp(-2 pi i k / n), evaluated from the first octant by symmetry so the
    // table is exactly symmetric
    long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)n;
    h[k].x = (T)cosl(a);
    h[k].y = (T)(-sinl(a));
  }
  void* d = nullptr;
  *err = hipMalloc(&d, sizeof(cpx<T>) * n);
  if (*err != hipSuccess) return nullptr;
  *err = hipMemcpy(d, h.data(), sizeof(cpx<T>) * n, hipMemcpyHostToDevice);
  return d;
}

int ctx_reserve(fvim_ctx* c, void** p, size_t* have, size_t need) {
  if (*have >= need) return FVIM_OK;
  if (*p) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
    hipFree(*p);
    *p = nullptr;
    *have = 0;
  }
  hipError_t e = hipMalloc(p, need);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(FVIM_ENOMEM, "device allocation failed for the operator workspace");
  }
  *have = need;
  return FVIM_OK;
}

// Records a pair of events around a launch when the context has timing on.
struct StageTimer {
  fvim_ctx* c;
  int stage = -1;
  hipEvent_t a = nullptr;
  hipStream_t s = nullptr;
  explicit StageTimer(fvim_ctx* cc) : c(cc) {}
  void begin(int stg, hipStream_t on) {
    if (!c->timing) return;
    stage = stg;
    s = on;
    hipEventCreate(&a);
    hipEventRecord(a, s);
  }
  void end() {
    if (!c->timing || stage < 0) return;
    hipEvent_t b;
    hipEventCreate(&b);
    hipEventRecord(b, s);
    c->evs.push_back({stage, a, b});
    stage = -1;
  }
};

static int side_ensure(fvim_ctx* c) {
  if (c->side) return FVIM_OK;
  hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  hipEvent_t* evs[] = {&c->ev_spec, &c->ev_nyq};
  for (hipEvent_t* ev : evs)
    if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  return e == hipSuccess ? FVIM_OK : fail_hip(e, "side stream");
}

// b waits for everything issued on a so far
static hipError_t join(hipEvent_t ev, hipStream_t a, hipStream_t b) {
  hipError_t e = hipEventRecord(ev, a);
  return e == hipSuccess ? hipStreamWaitEvent(b, ev, 0) : e;
}

// Times every valid depth-pass configuration on the live buffers (three
// launches each after one warm-up) and keeps the fastest in the context.
// The choice changes only the order of the depth sums (results agree to
// rounding); it is fixed for the context afterwards, so results are
// reproducible for a given configuration.
template <typename T>
int tune_depth(fvim_ctx* c, const cpx<T>* in, cpx<T>* out, const DepthParams& prm) {
  hipStream_t st = c->stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return fail(FVIM_EHIP, "events");
  float best = 1e30f;
  int best_id = depth_default_config(prm.nz);
  for (int id = 0; id < depth_num_configs(); ++id) {
    if (!depth_config_valid(id, prm.nz)) continue;
    hipError_t e = launch_depth<T>(in, out, prm, id, st);
    hipEventRecord(a, st);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_depth<T>(in, out, prm, id, st);
    hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e != hipSuccess) {
      hipEventDestroy(a);
      hipEventDestroy(b);
      return fail_hip(e, "depth tuning");
    }
    if (ms < best) {
      best = ms;
      best_id = id;
    }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  c->depth_cfg = best_id;
  return FVIM_OK;
}

// u = M[t] + N[C : eps_p] with any subset of outputs (see fvim.h).
template <typename T>
int operator_apply_t(fvim_ctx* c, const double* eps_p, const double* traction, double* strain, double* stress,
                     double* disp, double* surf_u3) {
  const int nx = c->grid.nx, ny = c->grid.ny, nz = c->grid.nz;
  const int kxh = nx / 2 + 1;
  const size_t nmodes = (size_t)kxh * ny;
  DepthParams prm{};
  prm.nx = nx;
  prm.ny = ny;
  prm.nz = nz;
  prm.kxh = kxh;
  prm.lx = c->grid.lx;
  prm.ly = c->grid.ly;
  prm.h = c->grid.lz / (nz - 1);
  prm.mu = c->mu;
  prm.kappa = c->lam / c->mu;
  prm.norm = 1.0 / ((double)nx * (double)ny);
  prm.has_w = eps_p != nullptr;
  prm.has_t = traction != nullptr;
  prm.k0_include = c->k0_policy == FVIM_K0_INCLUDE;
  // in float32 the mean mode is formed in float64 from float64 plane sums
  const bool k0x = sizeof(T) == 4;
  prm.k0_external = k0x ? 1 : 0;
  int np = 0;
  OutSegments seg;
  seg.n = 0;
  prm.off_strain = prm.off_stress = prm.off_disp = prm.off_u3 = -1;
  if (strain) { prm.off_strain = np; seg.first[seg.n] = np; seg.ptr[seg.n++] = strain; np += 6 * nz; }
  if (stress) { prm.off_stress = np; seg.first[seg.n] = np; seg.ptr[seg.n++] = stress; np += 6 * nz; }
  if (disp) { prm.off_disp = np; seg.first[seg.n] = np; seg.ptr[seg.n++] = disp; np += 3 * nz; }
  if (surf_u3) { prm.off_u3 = np; seg.first[seg.n] = np; seg.ptr[seg.n++] = surf_u3; np += 1; }
  prm.np_out = np;
  prm.ld_out = mode_stride<T>(np);
  if (np == 0) return FVIM_OK;
  // input planes: the 6 nz eigenstrain planes, then the 3 traction planes,
  // transformed together (one launch per direction)
  const int np_in = (eps_p ? 6 * nz : 0) + (traction ? 3 : 0);
  prm.np_in = np_in;
  prm.ld_in = mode_stride<T>(np_in);
  prm.off_t = eps_p ? 6 * nz : 0;
  InSegments iseg;
  iseg.n = 0;
  iseg.first[0] = iseg.first[1] = 0;
  iseg.ptr[0] = iseg.ptr[1] = nullptr;
  if (eps_p) { iseg.first[iseg.n] = 0; iseg.ptr[iseg.n++] = eps_p; }
  if (traction) { iseg.first[iseg.n] = prm.off_t; iseg.ptr[iseg.n++] = traction; }
  const size_t planes = (size_t)std::max(prm.ld_out, prm.ld_in);
  const size_t bytes = planes * nmodes * sizeof(cpx<T>);
  int rc = ctx_reserve(c, &c->bufA, &c->bufA_bytes, bytes);
  if (rc) return rc;
  rc = ctx_reserve(c, &c->bufB, &c->bufB_bytes, bytes);
  if (rc) return rc;
  const int wbpp = x_r2c_blocks_per_plane<T>(nx, ny);
  double* wsum = nullptr;
  double* tsum = nullptr;
  double* padd = nullptr;
  if (k0x) {
    const size_t kb = sizeof(double) * ((size_t)(6 * nz + 3) * wbpp + (size_t)np);
    rc = ctx_reserve(c, &c->k0buf, &c->k0buf_bytes, kb);
    if (rc) return rc;
    wsum = (double*)c->k0buf;                      // block sums of every input plane
    tsum = wsum + (size_t)prm.off_t * wbpp;
    padd = wsum + (size_t)(6 * nz + 3) * wbpp;
  }
  void*& mt = sizeof(T) == 8 ? c->mt64 : c->mt32;
  if (!mt) {
    if (hipMalloc(&mt, sizeof(ModeConst<T>) * nmodes) != hipSuccess) {
      mt = nullptr;
      return fail(FVIM_ENOMEM, "device allocation failed for the mode table");
    }
    hipError_t e0 = launch_mode_table<T>((ModeConst<T>*)mt, nx, ny, c->grid.lx, c->grid.ly, prm.h, c->stream);
    if (e0 != hipSuccess) return fail_hip(e0, "mode table");
  }
  prm.mtab = mt;
  const cpx<T>* twx = (const cpx<T>*)(sizeof(T) == 8 ? c->twx64 : c->twx32);
  const cpx<T>* twy = (const cpx<T>*)(sizeof(T) == 8 ? c->twy64 : c->twy32);
  cpx<T>* A = (cpx<T>*)c->bufA;
  cpx<T>* B = (cpx<T>*)c->bufB;
  hipStream_t st = c->stream;
  const bool side = c->use_side != 0;
  if (side && (rc = side_ensure(c))) return rc;
  // the Nyquist-mode depth launch may run on the side stream beside the main
  // one (disjoint modes); measured slower in float64, so off by default
  hipStream_t ss = side ? c->side : st;
  hipError_t e;
  StageTimer tm(c);
  tm.begin(FVIM_STAGE_XFWD, st);
  if ((e = launch_x_r2c<T>(iseg, A, nx, ny, (size_t)np_in, twx, st, wsum)) != hipSuccess)
    return fail_hip(e, "x_r2c");
  tm.end();
  tm.begin(FVIM_STAGE_YFWD, st);
  if ((e = launch_y_fwd<T>(A, B, ny, kxh, np_in, prm.ld_in, twy, st)) != hipSuccess) return fail_hip(e, "y_fwd");
  tm.end();
  if (c->tune_pending) {
    c->tune_pending = 0;
    int rc2 = tune_depth<T>(c, B, A, prm);
    if (rc2) return rc2;
  }
  if (ss != st && (e = join(c->ev_spec, st, ss)) != hipSuccess) return fail_hip(e, "fork");
  tm.begin(FVIM_STAGE_DEPTH, st);
  if ((e = launch_depth<T>(B, A, prm, c->depth_cfg, st, 1)) != hipSuccess) return fail_hip(e, "depth");
  tm.end();
  tm.begin(FVIM_STAGE_DEPTH_NYQ, ss);
  if ((e = launch_depth<T>(B, A, prm, c->depth_cfg, ss, 2)) != hipSuccess)
    return fail_hip(e, "depth (Nyquist modes)");
  tm.end();
  if (ss != st && (e = join(c->ev_nyq, ss, st)) != hipSuccess) return fail_hip(e, "join");
  if (k0x) {
    if ((e = launch_k0_fields(wsum, wbpp, tsum, wbpp, padd, prm, st)) != hipSuccess) return fail_hip(e, "k0");
  }
  tm.begin(FVIM_STAGE_YINV, st);
  if ((e = launch_y_inv<T>(A, B, ny, kxh, np, prm.ld_out, twy, st)) != hipSuccess) return fail_hip(e, "y_inv");
  tm.end();
  tm.begin(FVIM_STAGE_XINV, st);
  if ((e = launch_x_c2r<T>(B, seg, nx, ny, (size_t)np, 1.0, twx, st, padd)) != hipSuccess)
    return fail_hip(e, "x_c2r");
  tm.end();
  return FVIM_OK;
}

static bool misaligned(const void* p) { return p && (reinterpret_cast<uintptr_t>(p) & 15u); }

int operator_apply(fvim_ctx* c, const double* eps_p, const double* traction, double* strain, double* stress,
                   double* disp, double* surf_u3) {
  if (misaligned(eps_p) || misaligned(traction) || misaligned(strain) || misaligned(stress) ||
      misaligned(disp) || misaligned(surf_u3))
    return fail(FVIM_EINVAL, "field pointers must be 16-byte aligned");
  if (c->precision == FVIM_FP32_REFINED && !c->force_fp64)
    return operator_apply_t<float>(c, eps_p, traction, strain, stress, disp, surf_u3);
  return operator_apply_t<double>(c, eps_p, traction, strain, stress, disp, surf_u3);
}

}  // namespace fvim

extern "C" {

const char* fvim_last_error(void) { return g_err.c_str(); }

const char* fvim_version(void) { return "fvim 0.1 gfx950"; }

static int check_grid(const fvim_grid* g) {
  if (!g) return fail(FVIM_EINVAL, "grid is NULL");
  if (!is_pow2(g->nx) || !is_pow2(g->ny) || g->nx < 4 || g->ny < 4 || g->nx > 4096 || g->ny > 4096)
    return fail(FVIM_EINVAL, "nx and ny must be powers of two in [4, 4096]");
  if (g->nz < 2 || g->nz > 512) return fail(FVIM_EINVAL, "nz must be in [2, 512]");
  if (!(g->lx > 0) || !(g->ly > 0) || !(g->lz > 0) || !std::isfinite(g->lx) || !std::isfinite(g->ly) ||
      !std::isfinite(g->lz))
    return fail(FVIM_EINVAL, "cell lengths must be finite and positive");
  return FVIM_OK;
}

int fvim_create(const fvim_grid* grid, const fvim_material* mat, int precision, int k0_policy, void* hip_stream,
                fvim_ctx** out) {
  if (!out) return fail(FVIM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!mat || !(mat->E > 0) || !(mat->nu > -1.0 && mat->nu < 0.5) || !std::isfinite(mat->E) ||
      !(mat->sigma_y0 >= 0) || !(mat->E_h >= 0))
    return fail(FVIM_EINVAL, "material: need E > 0, -1 < nu < 0.5, sigma_y0 >= 0, E_h >= 0");
  if (precision != FVIM_FP64 && precision != FVIM_FP32_REFINED) return fail(FVIM_EINVAL, "unknown precision");
  if (k0_policy != FVIM_K0_INCLUDE && k0_policy != FVIM_K0_EXCLUDE) return fail(FVIM_EINVAL, "unknown k0 policy");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(FVIM_ENODEV, "no HIP device");
  fvim_ctx* c = new fvim_ctx();
  c->grid = *grid;
  c->mat = *mat;
  c->precision = precision;
  c->k0_policy = k0_policy;
  c->stream = (hipStream_t)hip_stream;
  hipGetDevice(&c->device);
  c->mu = mat->E / (2.0 * (1.0 + mat->nu));
  c->lam = mat->E * mat->nu / ((1.0 + mat->nu) * (1.0 - 2.0 * mat->nu));
  hipError_t e = hipSuccess;
  c->twx64 = make_twiddles<double>(grid->nx, &e);
  if (e == hipSuccess) c->twy64 = make_twiddles<double>(grid->ny, &e);
  if (e == hipSuccess) c->twx32 = make_twiddles<float>(grid->nx, &e);
  if (e == hipSuccess) c->twy32 = make_twiddles<float>(grid->ny, &e);
  if (e != hipSuccess) {
    fvim_destroy(c);
    return fail_hip(e, "twiddle tables");
  }
  *out = c;
  return FVIM_OK;
}

void fvim_destroy(fvim_ctx* c) {
  if (!c) return;
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  if (c->side) hipStreamSynchronize(c->side);
  void* ptrs[] = {c->twx64, c->twy64, c->twx32, c->twy32, c->bufA, c->bufB, c->k0buf, c->mt64, c->mt32};
  for (void* p : ptrs)
    if (p) hipFree(p);
  hipEvent_t evs[] = {c->ev_spec, c->ev_nyq};
  for (hipEvent_t ev : evs)
    if (ev) hipEventDestroy(ev);
  if (c->side) hipStreamDestroy(c->side);
  solver_release(c);
  for (auto& ev : c->evs) {
    hipEventDestroy(ev.a);
    hipEventDestroy(ev.b);
  }
  delete c;
}

int fvim_set_option(fvim_ctx* c, int key, int value) {
  if (!c) return fail(FVIM_EINVAL, "ctx is NULL");
  switch (key) {
    case FVIM_OPT_DEPTH_CONFIG:
      if (value != -1 && !depth_config_valid(value, c->grid.nz))
        return fail(FVIM_EINVAL, "depth configuration does not serve this nz");
      c->depth_cfg = value;
      return FVIM_OK;
    case FVIM_OPT_TUNE:
      c->tune_pending = value ? 1 : 0;
      return FVIM_OK;
    case FVIM_OPT_GRAPHS:
      c->use_graphs = value ? 1 : 0;
      return FVIM_OK;
    case FVIM_OPT_SIDE_STREAM:
      c->use_side = value ? 1 : 0;
      return FVIM_OK;
  }
  return fail(FVIM_EINVAL, "unknown option");
}

int fvim_get_option(fvim_ctx* c, int key, int* value) {
  if (!c || !value) return fail(FVIM_EINVAL, "NULL argument");
  switch (key) {
    case FVIM_OPT_DEPTH_CONFIG:
      *value = c->depth_cfg >= 0 ? c->depth_cfg : depth_default_config(c->grid.nz);
      return FVIM_OK;
    case FVIM_OPT_TUNE:
      *value = c->tune_pending;
      return FVIM_OK;
    case FVIM_OPT_GRAPHS:
      *value = c->use_graphs;
      return FVIM_OK;
    case FVIM_OPT_SIDE_STREAM:
      *value = c->use_side;
      return FVIM_OK;
  }
  return fail(FVIM_EINVAL, "unknown option");
}

int fvim_set_timing(fvim_ctx* c, int on) {
  if (!c) return fail(FVIM_EINVAL, "ctx is NULL");
  c->timing = on ? 1 : 0;
  return FVIM_OK;
}

int fvim_stage_times(fvim_ctx* c, double* ms, int* count) {
  if (!c || !ms || !count) return fail(FVIM_EINVAL, "NULL argument");
  for (int k = 0; k < FVIM_NSTAGES; ++k) {
    ms[k] = 0.0;
    count[k] = 0;
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  for (auto& ev : c->evs) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, ev.a, ev.b) == hipSuccess) {
      ms[ev.stage] += t;
      count[ev.stage] += 1;
    }
    hipEventDestroy(ev.a);
    hipEventDestroy(ev.b);
  }
  c->evs.clear();
  return FVIM_OK;
}

int fvim_set_stream(fvim_ctx* c, void* hip_stream) {
  if (!c) return fail(FVIM_EINVAL, "ctx is NULL");
  c->stream = (hipStream_t)hip_stream;
  return FVIM_OK;
}

size_t fvim_footprint_bytes(const fvim_grid* g, int precision, int with_solver_state) {
  if (check_grid(g)) return 0;
  const size_t nmodes = (size_t)(g->nx / 2 + 1) * g->ny;
  // the solvers of the FP32_REFINED mode also apply the float64 operator
  const size_t csz = (precision == FVIM_FP32_REFINED && !with_solver_state) ? 8 : 16;
  const size_t planes = 15 * (size_t)g->nz + 16;   // largest record, padded to 128 B
  size_t b = 2 * planes * nmodes * csz;
  b += nmodes * (sizeof(ModeConst<double>) + (precision == FVIM_FP32_REFINED ? sizeof(ModeConst<float>) : 0));
  const size_t V = (size_t)g->nx * g->ny * g->nz;
  if (with_solver_state) b += solver_footprint(g, V);
  return b;
}

int mindlin_apply(fvim_ctx* c, const double* eps_p, double* strain, double* stress, double* disp, double* surf_u3) {
  if (!c) return fail(FVIM_EINVAL, "ctx is NULL");
  if (!eps_p) return fail(FVIM_EINVAL, "eps_p is NULL");
  return operator_apply(c, eps_p, nullptr, strain, stress, disp, surf_u3);
}

int boussinesq_apply(fvim_ctx* c, const double* traction, double* strain, double* stress, double* disp,
                     double* surf_u3) {
  if (!c) return fail(FVIM_EINVAL, "ctx is NULL");
  if (!traction) return fail(FVIM_EINVAL, "traction is NULL");
  return operator_apply(c, nullptr, traction, strain, stress, disp, surf_u3);
}

int fvim_operator_apply(fvim_ctx* c, const double* eps_p, const double* traction, double* strain, double* stress,
                        double* disp, double* surf_u3) {
  if (!c) return fail(FVIM_EINVAL, "ctx is NULL");
  return operator_apply(c, eps_p, traction, strain, stress, disp, surf_u3);
}

int return_map(fvim_ctx* c, const double* d_eps, const double* sigma_n, const double* ep_n, double* d_eps_p,
               double* d_ep, double* sigma_np1) {
  if (!c) return fail(FVIM_EINVAL, "ctx is NULL");
  if (!d_eps || !sigma_n || !ep_n || !d_eps_p || !d_ep) return fail(FVIM_EINVAL, "NULL field");
  const size_t V = (size_t)c->grid.nx * c->grid.ny * c->grid.nz;
  hipError_t e = launch_return_map(d_eps, sigma_n, ep_n, d_eps_p, d_ep, sigma_np1, V, c->lam, c->mu,
                                   c->mat.sigma_y0, c->mat.E_h, c->stream);
  if (e != hipSuccess) return fail_hip(e, "return_map");
  return FVIM_OK;
}

}  // extern "C"
