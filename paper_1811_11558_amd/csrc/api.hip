// C ABI of the library (declared in include/fvim.h): context management and
// the operator entry points.  Every step of the operator runs in the HIP
// kernels of fft.hip and depth.hip; this file only checks arguments, owns
// the device workspace and sequences the launches on the context stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fvim.h"
#include "common.hpp"
#include "kernels.hpp"
#include "solver.hpp"

using namespace fvim;

namespace {
thread_local std::string g_err;

// Workspace of fvim_operator_apply_noalloc: one region of FVIM_NOALLOC_BYTES
// in every device's memory, held from the library's first use of that device
// until the process ends.  In host code `scratch` only names the symbol; its
// device address (different on every device) comes from
// hipGetSymbolAddress, taken once per device when the first context is
// created there, and is the only thing passed to kernels.
constexpr size_t kNoallocBytes = FVIM_NOALLOC_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mx;
void* g_scratch_addr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
}  // namespace

static __device__ __align__(256) char scratch[kNoallocBytes];

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
    // exp(-2 pi i k / n): cosine and sine of the full angle in long double,
    // rounded once to T
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

std::recursive_mutex& device_lock() {
  static std::recursive_mutex m;
  return m;
}

int ctx_reserve(fvim_ctx* c, void** p, size_t* have, size_t need) {
  if (*have >= need) return FVIM_OK;
  std::lock_guard<std::recursive_mutex> lk(device_lock());
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
  bool on;
  int stage = -1;
  hipEvent_t a = nullptr;
  hipStream_t s = nullptr;
  explicit StageTimer(fvim_ctx* cc, bool enabled = true) : c(cc), on(enabled && cc->timing) {}
  void begin(int stg, hipStream_t st) {
    if (!on) return;
    stage = stg;
    s = st;
    hipEventCreate(&a);
    hipEventRecord(a, s);
  }
  void end() {
    if (!on || stage < 0) return;
    hipEvent_t b;
    hipEventCreate(&b);
    hipEventRecord(b, s);
    c->evs.push_back({stage, a, b});
    stage = -1;
  }
};

static int side_ensure(fvim_ctx* c) {
  if (c->side) return FVIM_OK;
  std::lock_guard<std::recursive_mutex> lk(device_lock());
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

// Times launch(choice) for every candidate choice of a transform of length
// 2^logn (one launch to warm up, then three timed) and returns the fastest in
// *best; lengths without alternatives keep the default.
template <typename F>
static int time_choices(fvim_ctx* c, int logn, F&& launch, FftChoice* best) {
  *best = FftChoice{};
  if (logn < FFT_TUNE_MIN_LOGN || logn > FFT_TUNE_MAX_LOGN) return FVIM_OK;
  hipStream_t st = c->stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return fail(FVIM_EHIP, "events");
  float best_ms = 1e30f;
  hipError_t e = hipSuccess;
  for (int radix = 4; radix <= 8 && e == hipSuccess; radix += 4)
    for (int tile = 0; tile < 3 && e == hipSuccess; ++tile) {
      const FftChoice ch{tile, radix};
      e = launch(ch);
      if (e == hipSuccess) e = hipEventRecord(a, st);
      for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch(ch);
      if (e == hipSuccess) e = hipEventRecord(b, st);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e == hipSuccess && ms < best_ms) {
        best_ms = ms;
        *best = ch;
      }
    }
  hipEventDestroy(a);
  hipEventDestroy(b);
  return e == hipSuccess ? FVIM_OK : fail_hip(e, "transform tuning");
}

// Tuned launch choices kept for the process, keyed by the grid, the planes
// of the application, the precision and the device architecture: a context
// that asks for tuning takes an earlier context's result for the same key
// instead of timing again.
struct TuneKey {
  int nx, ny, nz, np_in, np_out, tsize;
  std::string arch;
  bool operator<(const TuneKey& o) const {
    return std::tie(nx, ny, nz, np_in, np_out, tsize, arch) <
           std::tie(o.nx, o.ny, o.nz, o.np_in, o.np_out, o.tsize, o.arch);
  }
};
struct TuneRec {
  FftChoice ch[4];
  int depth_cfg;
};
static std::mutex g_tune_mx;
static std::map<TuneKey, TuneRec>& tune_records() {
  static std::map<TuneKey, TuneRec> m;
  return m;
}

int fft_pack(const fvim_ctx* c, int prec) {
  int v = 0;
  for (int k = 0; k < 4; ++k) {
    const FftChoice ch = c->fft[prec][k];
    v |= ((ch.tile & 3) | (ch.radix == 8 ? 4 : 0)) << (3 * k);
  }
  return v;
}
int fft_pack_all(const fvim_ctx* c) { return fft_pack(c, 0) | (fft_pack(c, 1) << 12); }

// One operator application on one grid: parameters, buffers, launches.
template <typename T>
struct OpPlan {
  DepthParams prm{};
  OutSegments seg{};
  InSegments iseg{};
  int np = 0, np_in = 0, wbpp = 0, wbmax = 0;
  bool k0x = false;
  bool nt = false;              // launches read their input with streaming loads
  ResidEpilogue ep{};           // residual epilogue of the inverse x transform
  LayerSkip skip{};             // eigenstrain layers known to be zero
  double* wsum = nullptr;
  double* tsum = nullptr;
  double* padd = nullptr;
  cpx<T>* A = nullptr;
  cpx<T>* B = nullptr;
  const cpx<T>* twx = nullptr;
  const cpx<T>* twy = nullptr;
  FftChoice ch[4];              // x_r2c, y_fwd, y_inv, x_c2r
};

template <typename T>
constexpr int prec_index() { return sizeof(T) == 8 ? 0 : 1; }

// Device bytes one application needs: each of the two spectrum buffers
// (spectrum plus the Nyquist sign-replica records), the float64 plane sums
// and mean-mode constants of the float32 path, and the mode table.
struct OpSizes {
  size_t spec = 0, k0 = 0, mt = 0;
};
static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
// One region holding A, B, the float64 sums and the mode table, each on a
// 256-byte boundary.
static size_t scratch_bytes(const OpSizes& s) {
  return 2 * round256(s.spec) + round256(s.k0) + round256(s.mt);
}

// Depth parameters and the output/input plane layout of one application
// u = M[t] + N[C : eps_p] (any subset of outputs, see fvim.h), and the
// workspace it needs.  No device memory is touched.  P.np == 0: nothing
// requested.
template <typename T>
int op_layout(fvim_ctx* c, const double* eps_p, const double* traction, double* strain, double* stress,
              double* disp, double* surf_u3, OpPlan<T>& P, OpSizes& sz) {
  const int nx = c->grid.nx, ny = c->grid.ny, nz = c->grid.nz;
  const int kxh = nx / 2 + 1;
  const size_t nmodes = (size_t)kxh * ny;
  DepthParams& prm = P.prm;
  prm = DepthParams{};
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
  P.k0x = sizeof(T) == 4;
  prm.k0_external = P.k0x ? 1 : 0;
  int np = 0;
  OutSegments& seg = P.seg;
  seg.n = 0;
  prm.off_strain = prm.off_stress = prm.off_disp = prm.off_u3 = -1;
  if (strain) { prm.off_strain = np; seg.first[seg.n] = np; seg.ptr[seg.n++] = strain; np += 6 * nz; }
  if (stress) { prm.off_stress = np; seg.first[seg.n] = np; seg.ptr[seg.n++] = stress; np += 6 * nz; }
  if (disp) { prm.off_disp = np; seg.first[seg.n] = np; seg.ptr[seg.n++] = disp; np += 3 * nz; }
  if (surf_u3) { prm.off_u3 = np; seg.first[seg.n] = np; seg.ptr[seg.n++] = surf_u3; np += 1; }
  P.np = np;
  prm.np_out = np;
  prm.ld_out = mode_stride<T>(np);
  if (np == 0) return FVIM_OK;
  // input planes: the 6 nz eigenstrain planes, then the 3 traction planes,
  // transformed together (one launch per direction)
  const int np_in = (eps_p ? 6 * nz : 0) + (traction ? 3 : 0);
  P.np_in = np_in;
  prm.np_in = np_in;
  prm.ld_in = mode_stride<T>(np_in);
  prm.off_t = eps_p ? 6 * nz : 0;
  InSegments& iseg = P.iseg;
  iseg.n = 0;
  iseg.first[0] = iseg.first[1] = 0;
  iseg.ptr[0] = iseg.ptr[1] = nullptr;
  if (eps_p) { iseg.first[iseg.n] = 0; iseg.ptr[iseg.n++] = eps_p; }
  if (traction) { iseg.first[iseg.n] = prm.off_t; iseg.ptr[iseg.n++] = traction; }
  const size_t planes = (size_t)std::max(prm.ld_out, prm.ld_in);
  // the depth pass writes E to A; the Nyquist sign-replica records follow it
  const size_t nrep = (size_t)depth_replicas(ny, kxh);
  sz.spec = (planes * nmodes + nrep * (size_t)prm.ld_out) * sizeof(cpx<T>);
  for (int k = 0; k < 4; ++k) P.ch[k] = c->fft[prec_index<T>()][k];
  P.wbpp = x_r2c_blocks_per_plane<T>(nx, ny, P.ch[0]);
  // block sums of every input plane for the most blocks any tile choice
  // gives (the tuner runs them all), then the mean-mode constants
  P.wbmax = x_r2c_max_blocks_per_plane<T>(nx, ny);
  sz.k0 = P.k0x ? sizeof(double) * ((size_t)(6 * nz + 3) * P.wbmax + (size_t)np) : 0;
  sz.mt = sizeof(ModeConst<T>) * nmodes;
  // Streaming loads pay off when one launch's output fits the 256 MiB
  // last-level cache, so the next launch can read it from there. Measured
  // on MI355X, operator step off -> on:
  //   256^2 x 64, spectra of 106 and 207 MB: -5.7 % and -4.5 %
  //   128^2 x 64 (52 MB): +2.6 %
  //   410-842 MB spectra: +0.6 % to +4.8 %
  const size_t spec_bytes = planes * nmodes * sizeof(cpx<T>);
  P.nt = c->streaming == 1 ||
         (c->streaming == 2 && spec_bytes > ((size_t)64 << 20) && spec_bytes <= ((size_t)256 << 20));
  prm.nt_in = P.nt ? 1 : 0;
  return FVIM_OK;
}

// Pointers of an application whose workspace is bound: the float64 sums,
// the twiddles, the node table and the Nyquist replica records.
template <typename T>
void op_bind(fvim_ctx* c, OpPlan<T>& P, void* bufA, void* bufB, double* k0buf, const void* mt, bool side) {
  const size_t nmodes = (size_t)P.prm.kxh * P.prm.ny;
  if (P.k0x) {
    P.wsum = k0buf;                                // block sums of every input plane
    P.tsum = P.wsum + (size_t)P.prm.off_t * P.wbpp;
    P.padd = P.wsum + (size_t)(6 * c->grid.nz + 3) * P.wbmax;
  }
  P.prm.mtab = mt;
  P.prm.hz = c->hz;
  P.twx = (const cpx<T>*)(sizeof(T) == 8 ? c->twx64 : c->twx32);
  P.twy = (const cpx<T>*)(sizeof(T) == 8 ? c->twy64 : c->twy32);
  P.A = (cpx<T>*)bufA;
  P.B = (cpx<T>*)bufB;
  // with the side stream the Nyquist modes keep a launch of their own, which
  // can run beside the main one; otherwise their sign replicas join it
  P.prm.rep_out = side ? nullptr : (void*)(P.A + nmodes * (size_t)P.prm.ld_out);
}

// op_layout plus the workspace the context owns (grown on demand) and the
// context's mode table (built on first use).
template <typename T>
int op_plan(fvim_ctx* c, const double* eps_p, const double* traction, double* strain, double* stress,
            double* disp, double* surf_u3, OpPlan<T>& P) {
  OpSizes sz;
  int rc = op_layout<T>(c, eps_p, traction, strain, stress, disp, surf_u3, P, sz);
  if (rc || P.np == 0) return rc;
  if ((rc = ctx_reserve(c, &c->bufA, &c->bufA_bytes, sz.spec))) return rc;
  if ((rc = ctx_reserve(c, &c->bufB, &c->bufB_bytes, sz.spec))) return rc;
  if (P.k0x && (rc = ctx_reserve(c, &c->k0buf, &c->k0buf_bytes, sz.k0))) return rc;
  void*& mt = sizeof(T) == 8 ? c->mt64 : c->mt32;
  if (!mt) {
    std::lock_guard<std::recursive_mutex> lk(device_lock());
    if (hipMalloc(&mt, sz.mt) != hipSuccess) {
      mt = nullptr;
      return fail(FVIM_ENOMEM, "device allocation failed for the mode table");
    }
    hipError_t e0 = launch_mode_table<T>((ModeConst<T>*)mt, c->grid.nx, c->grid.ny, c->grid.lx, c->grid.ly,
                                         P.prm.h, c->stream);
    if (e0 != hipSuccess) return fail_hip(e0, "mode table");
  }
  op_bind<T>(c, P, c->bufA, c->bufB, (double*)c->k0buf, mt, c->use_side != 0);
  return FVIM_OK;
}

// Block count of the forward row transform after a change of its choice:
// the float64 plane sums of the float32 path follow it.
template <typename T>
void op_refresh_sums(fvim_ctx* c, OpPlan<T>& P) {
  P.wbpp = x_r2c_blocks_per_plane<T>(c->grid.nx, c->grid.ny, P.ch[0]);
  if (P.k0x) P.tsum = P.wsum + (size_t)P.prm.off_t * P.wbpp;
}

static int ilog2i(int n) { return 31 - __builtin_clz((unsigned)n); }

// Tuning of the forward transforms on the live input: the row transform's
// choices (its output then recomputed with the fastest), then the column
// transform's on that output.
template <typename T>
int tune_forward(fvim_ctx* c, OpPlan<T>& P) {
  const int nx = c->grid.nx, ny = c->grid.ny, kxh = nx / 2 + 1;
  hipStream_t st = c->stream;
  int rc = time_choices(c, ilog2i(nx), [&](FftChoice ch) {
    return launch_x_r2c<T>(P.iseg, P.A, nx, ny, (size_t)P.np_in, P.twx, st, P.wsum, P.nt, P.skip, ch);
  }, &P.ch[0]);
  if (rc) return rc;
  op_refresh_sums<T>(c, P);
  hipError_t e = launch_x_r2c<T>(P.iseg, P.A, nx, ny, (size_t)P.np_in, P.twx, st, P.wsum, P.nt, P.skip, P.ch[0]);
  if (e != hipSuccess) return fail_hip(e, "x_r2c");
  return time_choices(c, ilog2i(ny), [&](FftChoice ch) {
    return launch_y_fwd<T>(P.A, P.B, ny, kxh, P.np_in, P.prm.ld_in, P.twy, st, P.nt, P.skip, ch);
  }, &P.ch[1]);
}

// Tuning of the inverse transforms on the depth pass's output (the outputs
// are written again by the application's own inverse afterwards).
template <typename T>
int tune_inverse(fvim_ctx* c, OpPlan<T>& P) {
  const int nx = c->grid.nx, ny = c->grid.ny, kxh = nx / 2 + 1;
  hipStream_t st = c->stream;
  hipError_t e;
  if (P.k0x && (e = launch_k0_fields(P.wsum, P.wbpp, P.tsum, P.wbpp, P.padd, P.prm, st)) != hipSuccess)
    return fail_hip(e, "k0");
  int rc = time_choices(c, ilog2i(ny), [&](FftChoice ch) {
    return launch_y_inv<T>(P.A, P.B, ny, kxh, P.np, P.prm.ld_out, P.twy, st, P.nt, ch);
  }, &P.ch[2]);
  if (rc) return rc;
  if ((e = launch_y_inv<T>(P.A, P.B, ny, kxh, P.np, P.prm.ld_out, P.twy, st, P.nt, P.ch[2])) != hipSuccess)
    return fail_hip(e, "y_inv");
  return time_choices(c, ilog2i(nx), [&](FftChoice ch) {
    return launch_x_c2r<T>(P.B, P.seg, nx, ny, (size_t)P.np, 1.0, P.twx, st, P.padd, P.ep, true, ch);
  }, &P.ch[3]);
}

// Forward transforms of the input planes: real fields -> mode-major B.
template <typename T>
int op_forward(fvim_ctx* c, OpPlan<T>& P, hipStream_t st, StageTimer& tm) {
  const int nx = c->grid.nx, ny = c->grid.ny, kxh = nx / 2 + 1;
  hipError_t e;
  tm.begin(FVIM_STAGE_XFWD, st);
  if ((e = launch_x_r2c<T>(P.iseg, P.A, nx, ny, (size_t)P.np_in, P.twx, st, P.wsum, P.nt, P.skip, P.ch[0])) !=
      hipSuccess)
    return fail_hip(e, "x_r2c");
  tm.end();
  tm.begin(FVIM_STAGE_YFWD, st);
  if ((e = launch_y_fwd<T>(P.A, P.B, ny, kxh, P.np_in, P.prm.ld_in, P.twy, st, P.nt, P.skip, P.ch[1])) !=
      hipSuccess)
    return fail_hip(e, "y_fwd");
  tm.end();
  return FVIM_OK;
}

// Mean mode (float32 path) and inverse transforms: mode-major A -> outputs.
template <typename T>
int op_inverse(fvim_ctx* c, OpPlan<T>& P, hipStream_t st, StageTimer& tm) {
  const int nx = c->grid.nx, ny = c->grid.ny, kxh = nx / 2 + 1;
  hipError_t e;
  if (P.k0x && (e = launch_k0_fields(P.wsum, P.wbpp, P.tsum, P.wbpp, P.padd, P.prm, st)) != hipSuccess)
    return fail_hip(e, "k0");
  tm.begin(FVIM_STAGE_YINV, st);
  if ((e = launch_y_inv<T>(P.A, P.B, ny, kxh, P.np, P.prm.ld_out, P.twy, st, P.nt, P.ch[2])) != hipSuccess)
    return fail_hip(e, "y_inv");
  tm.end();
  tm.begin(FVIM_STAGE_XINV, st);
  if ((e = launch_x_c2r<T>(P.B, P.seg, nx, ny, (size_t)P.np, 1.0, P.twx, st, P.padd, P.ep, true, P.ch[3])) !=
      hipSuccess)
    return fail_hip(e, "x_c2r");
  tm.end();
  return FVIM_OK;
}

// u = M[t] + N[C : eps_p] with any subset of outputs (see fvim.h).  With
// scratch set, the workspace and the mode table are carved from that device
// region of scratch_cap bytes instead of the context's (nothing is allocated:
// no tuning, no stage timing, no side stream; the mode table is rebuilt there
// by the same kernel, so results are those of the context's own workspace).
template <typename T>
int operator_apply_t(fvim_ctx* c, const double* eps_p, const double* traction, double* strain, double* stress,
                     double* disp, double* surf_u3, const ResidEpilogue* ep = nullptr,
                     const int* zact = nullptr, char* scratch = nullptr, size_t scratch_cap = 0) {
  OpPlan<T> P;
  int rc;
  if (scratch) {
    OpSizes sz;
    rc = op_layout<T>(c, eps_p, traction, strain, stress, disp, surf_u3, P, sz);
    if (rc || P.np == 0) return rc;
    const size_t need = scratch_bytes(sz);
    if (need > scratch_cap) {
      char msg[200];
      snprintf(msg, sizeof msg, "operator_apply_noalloc: this application needs %zu bytes of workspace, more than "
               "the %zu-byte scratch", need, scratch_cap);
      return fail(FVIM_EINVAL, msg);
    }
    char* a = scratch;
    char* b = a + round256(sz.spec);
    char* k0 = b + round256(sz.spec);
    char* mt = k0 + round256(sz.k0);
    hipError_t e0 = launch_mode_table<T>((ModeConst<T>*)mt, c->grid.nx, c->grid.ny, c->grid.lx, c->grid.ly,
                                         P.prm.h, c->stream);
    if (e0 != hipSuccess) return fail_hip(e0, "mode table");
    op_bind<T>(c, P, a, b, (double*)k0, mt, false);
  } else {
    rc = op_plan<T>(c, eps_p, traction, strain, stress, disp, surf_u3, P);
    if (rc || P.np == 0) return rc;
  }
  if (ep) P.ep = *ep;
  if (zact && eps_p) {
    P.skip = LayerSkip{zact, c->grid.nz, 6 * c->grid.nz};
    P.prm.zact = zact;
  }
  hipStream_t st = c->stream;
  const bool side = c->use_side != 0 && !scratch;
  if (side && (rc = side_ensure(c))) return rc;
  // the Nyquist-mode depth launch may run on the side stream beside the main
  // one (disjoint modes); measured slower in float64, so off by default
  hipStream_t ss = side ? c->side : st;
  hipError_t e;
  StageTimer tm(c, scratch == nullptr);
  // tuning (plain applications only): take the process record for this
  // shape, else time every transform choice and depth layout on this call
  const bool tune = c->tune_pending && !scratch && !ep;
  bool timed = false;
  if (tune) {
    const TuneKey key{c->grid.nx, c->grid.ny, c->grid.nz, P.np_in, P.np, (int)sizeof(T), c->arch};
    TuneRec rec{};
    bool have = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mx);
      auto it = tune_records().find(key);
      if (it != tune_records().end()) {
        rec = it->second;
        have = true;
      }
    }
    if (have) {
      for (int k = 0; k < 4; ++k) P.ch[k] = c->fft[prec_index<T>()][k] = rec.ch[k];
      c->depth_cfg = rec.depth_cfg;
      c->tune_pending = 0;
      op_refresh_sums<T>(c, P);
    } else {
      if ((rc = tune_forward<T>(c, P))) return rc;
      timed = true;
    }
  }
  if ((rc = op_forward<T>(c, P, st, tm))) return rc;
  if (timed) {
    c->tune_pending = 0;
    int rc2 = tune_depth<T>(c, P.B, P.A, P.prm);
    if (rc2) return rc2;
  }
  if (ss != st && (e = join(c->ev_spec, st, ss)) != hipSuccess) return fail_hip(e, "fork");
  tm.begin(FVIM_STAGE_DEPTH, st);
  if ((e = launch_depth<T>(P.B, P.A, P.prm, c->depth_cfg, st, 1)) != hipSuccess) return fail_hip(e, "depth");
  tm.end();
  tm.begin(FVIM_STAGE_DEPTH_NYQ, ss);
  if ((e = launch_depth<T>(P.B, P.A, P.prm, c->depth_cfg, ss, 2)) != hipSuccess)
    return fail_hip(e, "depth (Nyquist modes)");
  tm.end();
  if (ss != st && (e = join(c->ev_nyq, ss, st)) != hipSuccess) return fail_hip(e, "join");
  if (timed) {
    if ((rc = tune_inverse<T>(c, P))) return rc;
    for (int k = 0; k < 4; ++k) c->fft[prec_index<T>()][k] = P.ch[k];
    const TuneKey key{c->grid.nx, c->grid.ny, c->grid.nz, P.np_in, P.np, (int)sizeof(T), c->arch};
    TuneRec rec{};
    for (int k = 0; k < 4; ++k) rec.ch[k] = P.ch[k];
    rec.depth_cfg = c->depth_cfg;
    std::lock_guard<std::mutex> lk(g_tune_mx);
    tune_records()[key] = rec;
  }
  return op_inverse<T>(c, P, st, tm);
}

// Several contexts (grids may differ) on the stream of the first: every
// context's forward transforms, one depth launch per part for up to
// DEPTH_BATCH_MAX contexts at a time, every context's inverse transforms.
template <typename T>
int operator_apply_batch_t(fvim_ctx* const* cs, int n, const double* const* eps, const double* const* tr,
                           double* const* strain, double* const* stress, double* const* disp,
                           double* const* surf_u3) {
  hipStream_t st = cs[0]->stream;
  std::vector<OpPlan<T>> P(n);
  std::vector<hipStream_t> saved(n);
  for (int i = 0; i < n; ++i) saved[i] = cs[i]->stream;
  auto restore = [&](int r) {
    for (int i = 0; i < n; ++i) cs[i]->stream = saved[i];
    return r;
  };
  for (int i = 0; i < n; ++i) cs[i]->stream = st;   // one stream orders the whole batch
  int rc = 0, maxnz = 0;
  for (int i = 0; i < n && !rc; ++i) {
    rc = op_plan<T>(cs[i], eps ? eps[i] : nullptr, tr ? tr[i] : nullptr, strain ? strain[i] : nullptr,
                    stress ? stress[i] : nullptr, disp ? disp[i] : nullptr, surf_u3 ? surf_u3[i] : nullptr, P[i]);
    if (!rc && P[i].np == 0) rc = fail(FVIM_EINVAL, "batch: every context needs an output");
    maxnz = std::max(maxnz, cs[i]->grid.nz);
  }
  if (rc) return restore(rc);
  fvim_ctx* c0 = cs[0];
  if ((rc = ctx_reserve(c0, &c0->dbatch, &c0->dbatch_bytes, sizeof(DepthBatch)))) return restore(rc);
  StageTimer tm(c0);
  // the persistent single-launch form (FVIM_OPT_PERSISTENT): float64, strain
  // only, every grid within the batched transform lengths, one table each
  bool persist = c0->persistent && std::is_same<T, double>::value && !stress && !disp && !surf_u3 &&
                 n <= XFORM_BATCH_MAX && n <= DEPTH_BATCH_MAX;
  for (int i = 0; i < n && persist; ++i)
    persist = ilog2i(cs[i]->grid.nx) <= XFORM_BATCH_MAX_LOGN && ilog2i(cs[i]->grid.ny) <= XFORM_BATCH_MAX_LOGN &&
              !P[i].k0x;
  // Grids whose transform lengths are both at most 2^XFORM_BATCH_MAX_LOGN
  // share one launch per transform stage (up to XFORM_BATCH_MAX grids each,
  // the default choices); longer ones keep launches of their own.
  std::vector<int> bat;
  for (int i = 0; i < n; ++i) {
    if (ilog2i(cs[i]->grid.nx) <= XFORM_BATCH_MAX_LOGN && ilog2i(cs[i]->grid.ny) <= XFORM_BATCH_MAX_LOGN) {
      bat.push_back(i);
      for (int k = 0; k < 4; ++k) P[i].ch[k] = FftChoice{};
      P[i].wbpp = x_r2c_batch_blocks_per_plane<T>(cs[i]->grid.nx, cs[i]->grid.ny);
      if (P[i].k0x) P[i].tsum = P[i].wsum + (size_t)P[i].prm.off_t * P[i].wbpp;
    } else if ((rc = op_forward<T>(cs[i], P[i], st, tm))) {
      return restore(rc);
    }
  }
  // the table of one stage of the batched grids bat[i0 ..], at most
  // XFORM_BATCH_MAX of them
  auto fill_xform = [&](int kind, size_t i0, XformBatch& b) {
      b = XformBatch{};
      b.n = (int)std::min<size_t>(XFORM_BATCH_MAX, bat.size() - i0);
      for (int k = 0; k < b.n; ++k) {
        const int i = bat[i0 + k];
        const OpPlan<T>& p = P[i];
        const int nx = cs[i]->grid.nx, ny = cs[i]->grid.ny;
        b.ny[k] = ny;
        b.kxh[k] = nx / 2 + 1;
        b.logn[k] = ilog2i(kind == 0 || kind == 3 ? nx : ny);
        b.tw[k] = kind == 0 || kind == 3 ? (const void*)p.twx : (const void*)p.twy;
        if (kind == 0) {
          b.NP[k] = p.np_in;
          b.iseg[k] = p.iseg;
          b.out[k] = p.A;
          b.bsum[k] = p.wsum;
        } else if (kind == 1) {
          b.NP[k] = p.np_in;
          b.ldp[k] = p.prm.ld_in;
          b.in[k] = p.A;
          b.out[k] = p.B;
        } else if (kind == 2) {
          b.NP[k] = p.np;
          b.ldp[k] = p.prm.ld_out;
          b.in[k] = p.A;
          b.out[k] = p.B;
        } else {
          b.NP[k] = p.np;
          b.in[k] = p.B;
          b.oseg[k] = p.seg;
          b.padd[k] = p.padd;
          b.nts[k] = 1;
        }
      }
  };
  // one stage of the batched grids, XFORM_BATCH_MAX at a time
  auto xform = [&](int kind, int stage) -> int {
    for (size_t i0 = 0; i0 < bat.size(); i0 += XFORM_BATCH_MAX) {
      XformBatch b;
      fill_xform(kind, i0, b);
      tm.begin(stage, st);
      hipError_t e = launch_xform_batch<T>(kind, b, st);
      tm.end();
      if (e != hipSuccess) return fail_hip(e, "batched transform");
    }
    return FVIM_OK;
  };
  const int cfg = depth_default_config(maxnz);
  const int gpb = depth_groups_per_block(cfg);
  // the depth table of grids i0 .. i0 + DEPTH_BATCH_MAX - 1
  auto fill_depth = [&](int i0, DepthBatch& b) {
    b = DepthBatch{};
    b.n = std::min(DEPTH_BATCH_MAX, n - i0);
    for (int k = 0; k < b.n; ++k) {
      const DepthParams& p = P[i0 + k].prm;
      b.prm[k] = p;
      // the Nyquist sign replicas join the main launch (records after the
      // spectrum in A, reserved by op_plan), whatever the side-stream option
      b.prm[k].rep_out = (void*)(P[i0 + k].A + (size_t)p.kxh * p.ny * p.ld_out);
      depth_derive(b.prm[k]);
      b.in[k] = P[i0 + k].B;
      b.out[k] = P[i0 + k].A;
      b.first_main[k + 1] = b.first_main[k] + (p.kxh * p.ny + depth_replicas(p.ny, p.kxh) + gpb - 1) / gpb;
      b.first_nyq[k + 1] = b.first_nyq[k] + (p.ny + p.kxh - 1);           // one block per Nyquist mode
    }
  };
  if (persist) {
    // every stage in one cooperative launch (falls through to the launches
    // below if this batch does not qualify after all)
    if ((rc = ctx_reserve(c0, &c0->pbatch, &c0->pbatch_bytes, sizeof(OpBatch)))) return restore(rc);
    OpBatch ob;
    for (int k = 0; k < 4; ++k) fill_xform(k, 0, ob.x[k]);
    fill_depth(0, ob.d);
    hipError_t e = launch_operator_persistent<T>(ob, (OpBatch*)c0->pbatch, cfg, false, false, st);
    if (e == hipSuccess) return restore(FVIM_OK);
    if (e != hipErrorNotSupported) return restore(fail_hip(e, "persistent batched operator"));
    (void)hipGetLastError();
  }
  if ((rc = xform(0, FVIM_STAGE_XFWD)) || (rc = xform(1, FVIM_STAGE_YFWD))) return restore(rc);
  for (int i0 = 0; i0 < n; i0 += DEPTH_BATCH_MAX) {
    DepthBatch b;
    fill_depth(i0, b);
    tm.begin(FVIM_STAGE_DEPTH, st);
    hipError_t e = launch_depth_batch<T>(b, (DepthBatch*)c0->dbatch, cfg, st);
    tm.end();
    if (e != hipSuccess) return restore(fail_hip(e, "batched depth pass"));
  }
  for (int i = 0; i < n && !rc; ++i) {
    const bool in_batch = std::find(bat.begin(), bat.end(), i) != bat.end();
    if (!in_batch) {
      rc = op_inverse<T>(cs[i], P[i], st, tm);
    } else if (P[i].k0x) {
      hipError_t e = launch_k0_fields(P[i].wsum, P[i].wbpp, P[i].tsum, P[i].wbpp, P[i].padd, P[i].prm, st);
      if (e != hipSuccess) rc = fail_hip(e, "k0");
    }
  }
  if (rc) return restore(rc);
  if ((rc = xform(2, FVIM_STAGE_YINV)) || (rc = xform(3, FVIM_STAGE_XINV))) return restore(rc);
  return restore(FVIM_OK);
}

static bool misaligned(const void* p) { return p && (reinterpret_cast<uintptr_t>(p) & 15u); }

int operator_apply_resid(fvim_ctx* c, const double* eps_p, const double* traction, const double* x,
                         const double* Fo, double* R, double* part, int* nparts, const int* zact) {
  if (misaligned(eps_p) || misaligned(traction) || misaligned(x) || misaligned(Fo) || misaligned(R))
    return fail(FVIM_EINVAL, "field pointers must be 16-byte aligned");
  const ResidEpilogue ep = {x, Fo, part, c->grid.nz, c->wz};
  const size_t np = (size_t)6 * c->grid.nz;
  if (c->precision == FVIM_FP32_REFINED && !c->force_fp64) {
    *nparts = x_c2r_blocks<float>(c->grid.nx, c->grid.ny, np, c->fft[1][3]);
    return operator_apply_t<float>(c, eps_p, traction, R, nullptr, nullptr, nullptr, &ep, zact);
  }
  *nparts = x_c2r_blocks<double>(c->grid.nx, c->grid.ny, np, c->fft[0][3]);
  return operator_apply_t<double>(c, eps_p, traction, R, nullptr, nullptr, nullptr, &ep, zact);
}

int operator_resid_parts(const fvim_grid& g) {
  const size_t np = (size_t)6 * g.nz;
  return std::max(x_c2r_max_blocks<float>(g.nx, g.ny, np), x_c2r_max_blocks<double>(g.nx, g.ny, np));
}

int operator_reserve(fvim_ctx* c, const double* eps_p, const double* traction, double* strain) {
  OpPlan<double> p64;
  int rc = op_plan<double>(c, eps_p, traction, strain, nullptr, nullptr, nullptr, p64);
  if (rc || c->precision != FVIM_FP32_REFINED) return rc;
  OpPlan<float> p32;
  return op_plan<float>(c, eps_p, traction, strain, nullptr, nullptr, nullptr, p32);
}

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

// Device address of the no-allocation scratch on device dev (current), looked
// up once; a failed lookup is remembered and reported by the entry point.
static void scratch_lookup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mx);
  if (g_scratch_addr[dev] || g_scratch_err[dev] != hipSuccess) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    g_scratch_err[dev] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    (void)hipGetLastError();
    return;
  }
  g_scratch_addr[dev] = p;
}

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
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  fvim_ctx* c = new fvim_ctx();
  c->grid = *grid;
  c->mat = *mat;
  c->precision = precision;
  c->k0_policy = k0_policy;
  c->stream = (hipStream_t)hip_stream;
  hipGetDevice(&c->device);
  scratch_lookup(c->device);
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->arch = prop.gcnArchName;
  }
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
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  if (c->side) hipStreamSynchronize(c->side);
  void* ptrs[] = {c->twx64, c->twy64, c->twx32, c->twy32, c->bufA, c->bufB, c->k0buf, c->mt64, c->mt32, c->dbatch,
                  c->pbatch, c->hz, c->wz};
  for (void* p : ptrs)
    if (p) hipFree(p);
  hipEvent_t evs[] = {c->ev_spec, c->ev_nyq};
  for (hipEvent_t ev : evs)
    if (ev) hipEventDestroy(ev);
  if (c->side) hipStreamDestroy(c->side);
  solver_release(c);
  friction_release(c);
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
    case FVIM_OPT_STREAMING:
      if (value < 0 || value > 2) return fail(FVIM_EINVAL, "streaming: 0, 1 or 2");
      c->streaming = value;
      return FVIM_OK;
    case FVIM_OPT_PERSISTENT:
      c->persistent = value ? 1 : 0;
      return FVIM_OK;
    case FVIM_OPT_FFT_CONFIG: {
      if (value < 0 || value >= (1 << 12)) return fail(FVIM_EINVAL, "fft config: 12 bits");
      const int prec = c->precision == FVIM_FP32_REFINED ? 1 : 0;
      FftChoice ch[4];
      for (int k = 0; k < 4; ++k) {
        const int v = (value >> (3 * k)) & 7;
        ch[k] = FftChoice{v & 3, (v & 4) ? 8 : 4};
        if (ch[k].tile > 2) return fail(FVIM_EINVAL, "fft config: tile 0, 1 or 2");
      }
      for (int k = 0; k < 4; ++k) c->fft[prec][k] = ch[k];
      return FVIM_OK;
    }
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
    case FVIM_OPT_STREAMING:
      *value = c->streaming;
      return FVIM_OK;
    case FVIM_OPT_PERSISTENT:
      *value = c->persistent;
      return FVIM_OK;
    case FVIM_OPT_FFT_CONFIG:
      *value = fft_pack(c, c->precision == FVIM_FP32_REFINED ? 1 : 0);
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

int fvim_set_depth_nodes(fvim_ctx* c, const double* z) {
  if (!c) return fail(FVIM_EINVAL, "ctx is NULL");
  const int nz = c->grid.nz;
  std::vector<double> h;
  if (z) {
    const double lz = c->grid.lz;
    if (!(z[0] == 0.0) || !(std::fabs(z[nz - 1] - lz) <= 1e-12 * lz))
      return fail(FVIM_EINVAL, "depth nodes: need z[0] = 0 and z[nz-1] = lz");
    h.resize(nz - 1);
    for (int e = 0; e + 1 < nz; ++e) {
      h[e] = z[e + 1] - z[e];
      if (!(h[e] > 0.0) || !std::isfinite(h[e])) return fail(FVIM_EINVAL, "depth nodes: need strictly increasing finite z");
    }
  }
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  hipError_t e = c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize();
  if (e != hipSuccess) return fail_hip(e, "depth nodes");
  solver_release(c);             // captured evaluations hold the previous node table
  if (c->hz) {
    hipFree(c->hz);
    c->hz = nullptr;
  }
  if (c->wz) {
    hipFree(c->wz);
    c->wz = nullptr;
  }
  if (!z) return FVIM_OK;
  // trapezoid weights of the nodes in units of the uniform spacing
  const double hu = c->grid.lz / (nz - 1);
  std::vector<double> wz(nz, 0.0);
  for (int i = 0; i + 1 < nz; ++i) {
    wz[i] += 0.5 * h[i] / hu;
    wz[i + 1] += 0.5 * h[i] / hu;
  }
  if (hipMalloc((void**)&c->hz, sizeof(double) * h.size()) != hipSuccess ||
      hipMalloc((void**)&c->wz, sizeof(double) * nz) != hipSuccess) {
    if (c->hz) hipFree(c->hz);
    c->hz = nullptr;
    c->wz = nullptr;
    return fail(FVIM_ENOMEM, "depth nodes: allocation failed");
  }
  e = hipMemcpy(c->hz, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->wz, wz.data(), sizeof(double) * nz, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(c->hz);
    hipFree(c->wz);
    c->hz = nullptr;
    c->wz = nullptr;
    return fail_hip(e, "depth nodes");
  }
  return FVIM_OK;
}

size_t fvim_footprint_bytes(const fvim_grid* g, int precision, int with_solver_state) {
  if (check_grid(g)) return 0;
  const size_t nmodes = (size_t)(g->nx / 2 + 1) * g->ny;
  // the solvers of the FP32_REFINED mode also apply the float64 operator
  const size_t csz = (precision == FVIM_FP32_REFINED && !with_solver_state) ? 8 : 16;
  const size_t planes = 15 * (size_t)g->nz + 16;   // largest record, padded to 128 B
  size_t b = 2 * planes * (nmodes + (size_t)depth_replicas(g->ny, g->nx / 2 + 1)) * csz;
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

int fvim_operator_apply_noalloc(fvim_ctx* c, const double* eps_p, const double* traction, double* strain,
                                double* stress, double* disp, double* surf_u3) {
  if (!c) return fail(FVIM_EINVAL, "ctx is NULL");
  if (misaligned(eps_p) || misaligned(traction) || misaligned(strain) || misaligned(stress) ||
      misaligned(disp) || misaligned(surf_u3))
    return fail(FVIM_EINVAL, "field pointers must be 16-byte aligned");
  if (c->device < 0 || c->device >= kMaxDevices) return fail(FVIM_ENODEV, "operator_apply_noalloc: device index");
  char* base;
  hipError_t se;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mx);
    base = (char*)g_scratch_addr[c->device];
    se = g_scratch_err[c->device];
  }
  if (!base) return fail_hip(se != hipSuccess ? se : hipErrorInvalidSymbol, "operator_apply_noalloc: scratch");
  if (c->precision == FVIM_FP32_REFINED && !c->force_fp64)
    return operator_apply_t<float>(c, eps_p, traction, strain, stress, disp, surf_u3, nullptr, nullptr, base,
                                   kNoallocBytes);
  return operator_apply_t<double>(c, eps_p, traction, strain, stress, disp, surf_u3, nullptr, nullptr, base,
                                  kNoallocBytes);
}

int fvim_operator_apply_batch(fvim_ctx* const* ctxs, int n, const double* const* eps_p,
                              const double* const* traction, double* const* strain, double* const* stress,
                              double* const* disp, double* const* surf_u3) {
  if (!ctxs || n < 1) return fail(FVIM_EINVAL, "batch: need at least one context");
  if (!eps_p && !traction) return fail(FVIM_EINVAL, "batch: no input");
  if (!strain && !stress && !disp && !surf_u3) return fail(FVIM_EINVAL, "batch: no output");
  const fvim_ctx* c0 = ctxs[0];
  for (int i = 0; i < n; ++i) {
    const fvim_ctx* c = ctxs[i];
    if (!c) return fail(FVIM_EINVAL, "batch: NULL context");
    if (c->device != c0->device || c->precision != c0->precision || c->force_fp64 != c0->force_fp64)
      return fail(FVIM_EINVAL, "batch: contexts must share the device and the precision");
    if (c->hz) return fail(FVIM_EINVAL, "batch: contexts with non-uniform depth nodes are not supported");
    const double* ptrs[] = {eps_p ? eps_p[i] : nullptr, traction ? traction[i] : nullptr};
    double* outs[] = {strain ? strain[i] : nullptr, stress ? stress[i] : nullptr, disp ? disp[i] : nullptr,
                      surf_u3 ? surf_u3[i] : nullptr};
    for (const double* p : ptrs)
      if (misaligned(p)) return fail(FVIM_EINVAL, "field pointers must be 16-byte aligned");
    for (double* p : outs)
      if (misaligned(p)) return fail(FVIM_EINVAL, "field pointers must be 16-byte aligned");
    if ((eps_p && !eps_p[i]) || (traction && !traction[i]) || (strain && !strain[i]) || (stress && !stress[i]) ||
        (disp && !disp[i]) || (surf_u3 && !surf_u3[i]))
      return fail(FVIM_EINVAL, "batch: a requested field is NULL for one context");
  }
  if (c0->precision == FVIM_FP32_REFINED && !c0->force_fp64)
    return operator_apply_batch_t<float>(ctxs, n, eps_p, traction, strain, stress, disp, surf_u3);
  return operator_apply_batch_t<double>(ctxs, n, eps_p, traction, strain, stress, disp, surf_u3);
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
