// Tangential (Coulomb, partial-slip) contact under a given normal pressure:
// the friction Sec. 5.1 says the contact step can include.  Normal and
// tangential problems are uncoupled (Goodman's approximation); the
// tangential surface traction q = (q1, q2) minimises the complementary
// energy 1/2 <q, C q> over |q_i| <= mu_f p_i with the total tangential force
// dA sum q = Q prescribed, C the tangential block of the half-space surface
// compliance: per mode, (2 (1 + nu) / (E |k|)) (I - nu n n^T), n = k / |k|,
// k = 0 dropped, n1 n2 averaged to 0 over the sign replicas of a Nyquist
// line.  Its optimality conditions are the stick/slip conditions (one rigid
// shift of the stick zone; slip against the traction where it is on the
// friction limit).
//
// Accelerated projected gradient (FISTA) with gradient restart, step 1 / L,
// L the largest eigenvalue of C.  One iteration, all on the device with no
// host round trip:
//   u = C y            2-plane forward transforms, 2x2 multiplier, inverse
//   v = y - u / L;     q_new = P(v + lam): P the projection onto the disks
//                      |.| <= mu_f p_i, lam (2 values) the root of
//                      dA sum P(v + lam) = Q by Newton steps (block sums of
//                      P and of its 2x2 Jacobian, then one block solves)
//   restart test <y - q_new, q_new - q> > 0, momentum, y and q updated.
// The host reads the change measure dA sum |q_new - q| / (mu_f W) every few
// iterations.  Reductions use a fixed block partition and order.
//
// Coupled form (frictional_contact_solve, coupled = 1): for nu < 1/2 the
// Boussinesq-Cerruti surface response has cross terms, per mode
// u_a = K_a t3 and u3 = sum_a conj(K_a) t_a with K_a = i (1 - 2 nu) n_a /
// (2 mu |k|) (0 at k = 0 and on the Nyquist line of axis a).  The pressure
// then solves the normal problem on h - u3[q] and q the tangential problem
// with the extra displacement u_t[p] (added to C y in the gradient step);
// the two solves alternate, each warm-started from the last, until
// dA sum |dp| / W + dA sum |dq| / (mu_f W) < tol.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"
#include "solver.hpp"

namespace fvim {
namespace {

constexpr int NT = 256;
constexpr int RB = 1024;               // max reduction blocks
constexpr int NEWTON = 2;              // projection Newton steps per iteration (warm-started)
constexpr int CHECK = 8;               // iterations between host checks

// device scalars
enum { F_LAM0 = 0, F_LAM1, F_T, F_BETA, F_CHANGE, F_DOT, F_SUMP, F_STICK, F_CONTACT, F_CP, F_CQ, F_NSC = 16 };

template <int NS>
__device__ __forceinline__ void fblock_sums(double (&v)[NS], double* part) {
  __shared__ double sh[NS][NT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0) sh[k][w] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      double s = 0.0;
      for (int i = 0; i < NT / 64; ++i) s += sh[k][i];
      part[k * RB + blockIdx.x] = s;
    }
  }
}

// total of the nb partials of row k, one block, fixed order
__device__ double ffinal(const double* part, int k, int nb) {
  __shared__ double sh[NT];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += NT) s += part[k * RB + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// totals of the nb partials of rows 0 .. K-1 in one pass: every thread sums
// its strided share of each row, then wave shuffles and one cross-wave step
// (fixed order); the totals are valid in thread 0
template <int K>
__device__ __forceinline__ void ffinal_rows(const double* part, int nb, double (&out)[K]) {
  __shared__ double sh[K][NT / 64];
  double s[K];
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] = 0.0;
  for (int i = threadIdx.x; i < nb; i += NT)
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] += part[k * RB + i];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = s[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0) sh[k][w] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double t = 0.0;
      for (int j = 0; j < NT / 64; ++j) t += sh[k][j];
      out[k] = t;
    }
}

// projection of w onto the disk |.| <= rho: P and its Jacobian (a, b, c) =
// [[a, b], [b, c]]
__device__ __forceinline__ void disk(double w0, double w1, double rho, double& p0, double& p1, double& ja,
                                     double& jb, double& jc) {
  const double r = sqrt(w0 * w0 + w1 * w1);
  if (r <= rho) {
    p0 = w0;
    p1 = w1;
    ja = 1.0;
    jb = 0.0;
    jc = 1.0;
    return;
  }
  const double s = rho / r, a = s / (r * r);
  p0 = s * w0;
  p1 = s * w1;
  ja = s - a * w0 * w0;
  jb = -a * w0 * w1;
  jc = s - a * w1 * w1;
}

// rho = mu_f p; block sums of p (negative pressures, which a contact
// solution does not hold, count as 0)
__global__ __launch_bounds__(NT) void k_f_rho(const double* __restrict__ p, double mu, double* __restrict__ rho,
                                             size_t n, double* part) {
  double v[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    const double pi = fmax(p[i], 0.0);
    rho[i] = mu * pi;
    v[0] += pi;
  }
  fblock_sums<1>(v, part);
}

// q = y = (c0, c1) rho (the full-slip field scaled to the load)
__global__ __launch_bounds__(NT) void k_f_init(const double* __restrict__ rho, double* __restrict__ q,
                                              double* __restrict__ y, size_t n, double c0, double c1) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    const double r = rho[i];
    q[i] = y[i] = c0 * r;
    q[n + i] = y[n + i] = c1 * r;
  }
}

// 2x2 tangential compliance per mode of the mode-major spectrum s[mode][ld]
// (planes 0, 1), with the 1 / (nx ny) of the inverse transform
__global__ __launch_bounds__(NT) void k_f_compliance(cpx<double>* __restrict__ s, int ld, int nx, int ny, double lx,
                                                    double ly, double fac, double nu) {
  const int kxh = nx / 2 + 1;
  const int m = blockIdx.x * NT + threadIdx.x;
  if (m >= kxh * ny) return;
  const int kx = m / ny, ky = m - kx * ny;
  const int k2 = (ky * 2 <= ny) ? ky : ky - ny;
  const double twopi = 6.283185307179586476925286766559;
  const double q1 = twopi * kx / lx, q2 = twopi * k2 / ly;
  const double q = sqrt(q1 * q1 + q2 * q2);
  cpx<double>* r = s + (size_t)m * ld;
  if (m == 0) {
    r[0] = mk(0.0, 0.0);
    r[1] = mk(0.0, 0.0);
    return;
  }
  const double f = fac / q, n1 = q1 / q, n2 = q2 / q;
  const bool nyq = (kx * 2 == nx) || (ky * 2 == ny);
  const double c11 = f * (1.0 - nu * n1 * n1), c22 = f * (1.0 - nu * n2 * n2);
  const double c12 = nyq ? 0.0 : -f * nu * n1 * n2;
  const cpx<double> a = r[0], b = r[1];
  r[0] = mk(c11 * a.x + c12 * b.x, c11 * a.y + c12 * b.y);
  r[1] = mk(c12 * a.x + c22 * b.x, c12 * a.y + c22 * b.y);
}

// displacement of the gradient step: u (C y), plus ue (the pressure's
// tangential displacement) when not NULL
__device__ __forceinline__ double gdisp(const double* __restrict__ u, const double* __restrict__ ue, size_t i) {
  return ue ? u[i] + ue[i] : u[i];
}

// block sums of P(v + lam) and of its Jacobian, v = y - (u + ue) / L
__global__ __launch_bounds__(NT) void k_f_sums(const double* __restrict__ y, const double* __restrict__ u,
                                              const double* __restrict__ ue, double invL,
                                              const double* __restrict__ rho, const double* __restrict__ sc,
                                              size_t n, double* part) {
  const double l0 = sc[F_LAM0], l1 = sc[F_LAM1];
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    const double w0 = y[i] - invL * gdisp(u, ue, i) + l0, w1 = y[n + i] - invL * gdisp(u, ue, n + i) + l1;
    double p0, p1, ja, jb, jc;
    disk(w0, w1, rho[i], p0, p1, ja, jb, jc);
    v[0] += p0;
    v[1] += p1;
    v[2] += ja;
    v[3] += jb;
    v[4] += jc;
  }
  fblock_sums<5>(v, part);
}

// one Newton step on lam: g = sum P - S, J = sum of Jacobians (regularised)
__global__ __launch_bounds__(NT) void k_f_newton(const double* __restrict__ part, int nb, double* sc, double S0,
                                                double S1) {
  double t[5];
  ffinal_rows<5>(part, nb, t);
  if (threadIdx.x == 0) {
    const double g0 = t[0] - S0, g1 = t[1] - S1;
    double a = t[2], b = t[3], c = t[4];
    const double reg = 1e-14 * (a + c + 1.0);
    a += reg;
    c += reg;
    const double det = a * c - b * b;
    if (det > 0.0) {
      sc[F_LAM0] -= (c * g0 - b * g1) / det;
      sc[F_LAM1] -= (a * g1 - b * g0) / det;
    }
  }
}

// q_new = P(v + lam); block sums of |q_new - q| and <y - q_new, q_new - q>
__global__ __launch_bounds__(NT) void k_f_apply(const double* __restrict__ y, const double* __restrict__ u,
                                               const double* __restrict__ ue, double invL,
                                               const double* __restrict__ rho, const double* __restrict__ sc,
                                               const double* __restrict__ q, double* __restrict__ qn, size_t n,
                                               double* part) {
  const double l0 = sc[F_LAM0], l1 = sc[F_LAM1];
  double v[2] = {0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    const double y0 = y[i], y1 = y[n + i];
    const double w0 = y0 - invL * gdisp(u, ue, i) + l0, w1 = y1 - invL * gdisp(u, ue, n + i) + l1;
    double p0, p1, ja, jb, jc;
    disk(w0, w1, rho[i], p0, p1, ja, jb, jc);
    qn[i] = p0;
    qn[n + i] = p1;
    const double d0 = p0 - q[i], d1 = p1 - q[n + i];
    v[0] += fabs(d0) + fabs(d1);
    v[1] += (y0 - p0) * d0 + (y1 - p1) * d1;
  }
  fblock_sums<2>(v, part);
}

// change measure, restart decision and momentum coefficient
__global__ __launch_bounds__(NT) void k_f_momentum(const double* __restrict__ part, int nb, double* sc,
                                                  double* mirror, double cscale) {
  double t2[2];
  ffinal_rows<2>(part, nb, t2);
  if (threadIdx.x == 0) {
    const double ch = t2[0], dot = t2[1];
    const double t = sc[F_T];
    double beta = 0.0, tn = 1.0;
    if (!(dot > 0.0)) {
      tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
      beta = (t - 1.0) / tn;
    }
    sc[F_T] = tn;
    sc[F_BETA] = beta;
    sc[F_CHANGE] = mirror[F_CHANGE] = ch * cscale;
    sc[F_DOT] = dot;
  }
}

// y = q_new + beta (q_new - q); q = q_new
__global__ __launch_bounds__(NT) void k_f_update(double* __restrict__ q, const double* __restrict__ qn,
                                                double* __restrict__ y, const double* __restrict__ sc, size_t n2) {
  const double beta = sc[F_BETA];
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n2; i += (size_t)gridDim.x * NT) {
    const double a = qn[i];
    y[i] = a + beta * (a - q[i]);
    q[i] = a;
  }
}

// block sums of stick points (|q| < rho (1 - 1e-9)) and contact points (rho > 0)
__global__ __launch_bounds__(NT) void k_f_stick(const double* __restrict__ q, const double* __restrict__ rho,
                                               size_t n, double* part) {
  double v[2] = {0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    const double r = rho[i];
    if (r > 0.0) {
      v[1] += 1.0;
      const double a = sqrt(q[i] * q[i] + q[n + i] * q[n + i]);
      if (a < r * (1.0 - 1e-9)) v[0] += 1.0;
    }
  }
  fblock_sums<2>(v, part);
}

// Cerruti cross terms on the mode-major spectrum s[mode][ld] (with the
// 1 / (nx ny) of the inverse transform in fac = 1 / (nx ny)):
// N2T: plane 0 (the pressure) -> planes 0, 1: u_a = K_a p;
// T2N: planes 0, 1 (the tangential traction) -> plane 0: u3 = sum conj(K_a) q_a.
// K_a = i c n_a, c = (1 - 2 nu) / (2 mu |k|); K_1 = 0 on the Nyquist line of
// x, K_2 = 0 on the one of y; mode 0 dropped.
template <bool N2T>
__global__ __launch_bounds__(NT) void k_c_cross(cpx<double>* __restrict__ s, int ld, int nx, int ny, double lx,
                                               double ly, double fac, double nu, double mu) {
  const int kxh = nx / 2 + 1;
  const int m = blockIdx.x * NT + threadIdx.x;
  if (m >= kxh * ny) return;
  const int kx = m / ny, ky = m - kx * ny;
  const int k2 = (ky * 2 <= ny) ? ky : ky - ny;
  const double twopi = 6.283185307179586476925286766559;
  const double q1 = twopi * kx / lx, q2 = twopi * k2 / ly;
  const double q = sqrt(q1 * q1 + q2 * q2);
  cpx<double>* r = s + (size_t)m * ld;
  double c1 = 0.0, c2 = 0.0;      // c n_a, with the Nyquist zeros
  if (m != 0) {
    const double cq = fac * (1.0 - 2.0 * nu) / (2.0 * mu * q * q);
    if (kx * 2 != nx) c1 = cq * q1;
    if (ky * 2 != ny) c2 = cq * q2;
  }
  if (N2T) {
    const cpx<double> a = r[0];                  // i c n_a a
    r[0] = mk(-c1 * a.y, c1 * a.x);
    r[1] = mk(-c2 * a.y, c2 * a.x);
  } else {
    const cpx<double> a = r[0], b = r[1];        // -i (c1 a + c2 b)
    const double zx = c1 * a.x + c2 * b.x, zy = c1 * a.y + c2 * b.y;
    r[0] = mk(zy, -zx);
  }
}

// out = a - b
__global__ __launch_bounds__(NT) void k_c_sub(const double* __restrict__ a, const double* __restrict__ b,
                                             double* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) out[i] = a[i] - b[i];
}

// block sums of |p - p_prev| and |q - q_prev| (both components); t = (q0,
// q1, p) and tp its previous value, [3][n] each
__global__ __launch_bounds__(NT) void k_c_change(const double* __restrict__ t, const double* __restrict__ tp,
                                                size_t n, double* part) {
  double v[2] = {0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    v[0] += fabs(t[2 * n + i] - tp[2 * n + i]);
    v[1] += fabs(t[i] - tp[i]) + fabs(t[n + i] - tp[n + i]);
  }
  fblock_sums<2>(v, part);
}

__global__ __launch_bounds__(NT) void k_f_totals(const double* __restrict__ part, int nb, int k, double* sc,
                                                double* mirror, int slot) {
  double s[3];
  for (int j = 0; j < k; ++j) s[j] = ffinal(part, j, nb);
  if (threadIdx.x == 0)
    for (int j = 0; j < k; ++j) sc[slot + j] = mirror[slot + j] = s[j];
}

int fblocks(size_t n) { return (int)std::min<size_t>((n + NT - 1) / NT, RB); }

}  // namespace

struct FricWork {
  size_t n = 0;
  int ld = 0;
  double* vec = nullptr;          // q, y, u, q_new (2 planes each), rho; then for the
                                  // coupled solve: u_t[p] (2), h - u3[q] (1), previous
                                  // traction (3)
  cpx<double>* specX = nullptr;   // [2][kxh][ny]
  cpx<double>* specM = nullptr;   // [kxh][ny][ld]
  double* part = nullptr;         // [5][RB]
  double* sc = nullptr;           // device scalars
  double* hmap = nullptr;         // mapped host mirror (host view)
  double* dmap = nullptr;         //   (device view)
};

void friction_release(fvim_ctx* c) {
  FricWork* w = c->fric;
  if (!w) return;
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  if (w->vec) hipFree(w->vec);
  if (w->specX) hipFree(w->specX);
  if (w->specM) hipFree(w->specM);
  if (w->part) hipFree(w->part);
  if (w->sc) hipFree(w->sc);
  if (w->hmap) hipHostFree(w->hmap);
  delete w;
  c->fric = nullptr;
}

static int fric_ensure(fvim_ctx* c) {
  if (c->fric) return FVIM_OK;
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  FricWork* w = new FricWork();
  c->fric = w;
  const int nx = c->grid.nx, ny = c->grid.ny, kxh = nx / 2 + 1;
  w->n = (size_t)nx * ny;
  w->ld = mode_stride<double>(2);
  const bool ok = hipMalloc((void**)&w->vec, sizeof(double) * 15 * w->n) == hipSuccess &&
                  hipMalloc((void**)&w->specX, sizeof(cpx<double>) * 2 * kxh * ny) == hipSuccess &&
                  hipMalloc((void**)&w->specM, sizeof(cpx<double>) * (size_t)kxh * ny * w->ld) == hipSuccess &&
                  hipMalloc((void**)&w->part, sizeof(double) * 5 * RB) == hipSuccess &&
                  hipMalloc((void**)&w->sc, sizeof(double) * F_NSC) == hipSuccess &&
                  hipHostMalloc((void**)&w->hmap, sizeof(double) * F_NSC,
                                hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
                  hipHostGetDevicePointer((void**)&w->dmap, w->hmap, 0) == hipSuccess;
  if (!ok) {
    friction_release(c);
    return fail(FVIM_ENOMEM, "tangential contact workspace allocation failed");
  }
  return FVIM_OK;
}

int friction_reserve(fvim_ctx* c) { return fric_ensure(c); }

size_t friction_footprint(const fvim_grid* g) {
  const size_t n = (size_t)g->nx * g->ny, nm = (size_t)(g->nx / 2 + 1) * g->ny;
  return sizeof(double) * (15 * n + 5 * RB + F_NSC) + sizeof(cpx<double>) * nm * (2 + mode_stride<double>(2));
}

// u = C y (2 planes)
static int tangential_compliance(fvim_ctx* c, const double* y, double* u, hipStream_t st) {
  FricWork* w = c->fric;
  const int nx = c->grid.nx, ny = c->grid.ny, kxh = nx / 2 + 1;
  const cpx<double>* twx = (const cpx<double>*)c->twx64;
  const cpx<double>* twy = (const cpx<double>*)c->twy64;
  hipError_t e;
  if ((e = launch_x_r2c<double>(y, w->specX, nx, ny, 2, twx, st)) != hipSuccess) return fail_hip(e, "tangential x");
  if ((e = launch_y_fwd<double>(w->specX, w->specM, ny, kxh, 2, w->ld, twy, st)) != hipSuccess)
    return fail_hip(e, "tangential y");
  const double G = c->mat.E / (2.0 * (1.0 + c->mat.nu));
  const double fac = 1.0 / G / ((double)nx * ny);
  const int nm = kxh * ny;
  hipLaunchKernelGGL(k_f_compliance, dim3((nm + NT - 1) / NT), dim3(NT), 0, st, w->specM, w->ld, nx, ny,
                     c->grid.lx, c->grid.ly, fac, c->mat.nu);
  if ((e = launch_y_inv<double>(w->specM, w->specX, ny, kxh, 2, w->ld, twy, st)) != hipSuccess)
    return fail_hip(e, "tangential y^-1");
  OutSegments seg;
  seg.n = 1;
  seg.first[0] = 0;
  seg.ptr[0] = u;
  if ((e = launch_x_c2r<double>(w->specX, seg, nx, ny, 2, 1.0, twx, st)) != hipSuccess)
    return fail_hip(e, "tangential x^-1");
  return FVIM_OK;
}

// Cerruti cross displacements.  n2t: ut (2 planes) = u_t of the pressure in
// (1 plane); else u3 (1 plane) = u3 of the tangential traction in (2 planes).
static int cerruti_cross(fvim_ctx* c, const double* in, double* out, bool n2t, hipStream_t st) {
  FricWork* w = c->fric;
  const int nx = c->grid.nx, ny = c->grid.ny, kxh = nx / 2 + 1;
  const int pin = n2t ? 1 : 2, pout = n2t ? 2 : 1;
  const cpx<double>* twx = (const cpx<double>*)c->twx64;
  const cpx<double>* twy = (const cpx<double>*)c->twy64;
  hipError_t e;
  if ((e = launch_x_r2c<double>(in, w->specX, nx, ny, pin, twx, st)) != hipSuccess) return fail_hip(e, "cross x");
  if ((e = launch_y_fwd<double>(w->specX, w->specM, ny, kxh, pin, w->ld, twy, st)) != hipSuccess)
    return fail_hip(e, "cross y");
  const double G = c->mat.E / (2.0 * (1.0 + c->mat.nu));
  const double fac = 1.0 / ((double)nx * ny);
  const int nm = kxh * ny;
  if (n2t)
    hipLaunchKernelGGL(k_c_cross<true>, dim3((nm + NT - 1) / NT), dim3(NT), 0, st, w->specM, w->ld, nx, ny,
                       c->grid.lx, c->grid.ly, fac, c->mat.nu, G);
  else
    hipLaunchKernelGGL(k_c_cross<false>, dim3((nm + NT - 1) / NT), dim3(NT), 0, st, w->specM, w->ld, nx, ny,
                       c->grid.lx, c->grid.ly, fac, c->mat.nu, G);
  if ((e = launch_y_inv<double>(w->specM, w->specX, ny, kxh, pout, w->ld, twy, st)) != hipSuccess)
    return fail_hip(e, "cross y^-1");
  OutSegments seg;
  seg.n = 1;
  seg.first[0] = 0;
  seg.ptr[0] = out;
  if ((e = launch_x_c2r<double>(w->specX, seg, nx, ny, pout, 1.0, twx, st)) != hipSuccess)
    return fail_hip(e, "cross x^-1");
  return FVIM_OK;
}

int friction_solve(fvim_ctx* c, const double* p, double mu_f, double Qx, double Qy, double tol, int max_iter,
                   double* q_out, fvim_tangential_info* info, bool warm, const double* ue) {
  if (!(mu_f > 0.0) || !std::isfinite(Qx) || !std::isfinite(Qy) || !(tol > 0.0) || max_iter < 1)
    return fail(FVIM_EINVAL, "tangential_solve: bad arguments");
  int rc = fric_ensure(c);
  if (rc) return rc;
  FricWork* w = c->fric;
  hipStream_t st = c->stream;
  const size_t n = w->n;
  double* q = w->vec;
  double* y = q + 2 * n;
  double* u = y + 2 * n;
  double* qn = u + 2 * n;
  double* rho = qn + 2 * n;
  const int nb = fblocks(n);
  const double dA = c->grid.lx * c->grid.ly / (double)n;
  hipLaunchKernelGGL(k_f_rho, dim3(nb), dim3(NT), 0, st, p, mu_f, rho, n, w->part);
  hipLaunchKernelGGL(k_f_totals, dim3(1), dim3(NT), 0, st, w->part, nb, 1, w->sc, w->dmap, (int)F_SUMP);
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail_hip(e, "tangential_solve");
  const double W = dA * w->hmap[F_SUMP];
  if (!(std::hypot(Qx, Qy) < mu_f * W))
    return fail(FVIM_EINVAL, "tangential_solve: partial slip needs |Q| < mu_f W (full sliding: q = mu_f p Q/|Q|)");
  // largest eigenvalue of C: the lowest wavenumber, along the direction
  // where I - nu n n^T is 1 (the coupling only lowers it)
  const double G = c->mat.E / (2.0 * (1.0 + c->mat.nu));
  const double twopi = 6.283185307179586476925286766559;
  double kmin = INFINITY;
  if (c->grid.nx > 1) kmin = std::min(kmin, twopi / c->grid.lx);
  if (c->grid.ny > 1) kmin = std::min(kmin, twopi / c->grid.ly);
  const double L = 1.0 / (G * kmin);
  const double invL = 1.0 / L;
  const double S0 = Qx / dA, S1 = Qy / dA;
  hipLaunchKernelGGL(k_f_init, dim3(nb), dim3(NT), 0, st, rho, q, y, n, Qx / (mu_f * W), Qy / (mu_f * W));
  double init[F_NSC] = {};
  init[F_T] = 1.0;
  {
    std::lock_guard<std::recursive_mutex> lk(device_lock());     // pageable copy
    e = hipMemcpyAsync(w->sc, init, sizeof(init), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  if (e != hipSuccess) return fail_hip(e, "tangential_solve");
  const double cscale = dA / (mu_f * W);
  if (warm) {
    // start from the projection of the caller's q (the previous solution
    // under a nearby pressure) onto the new constraint set: Newton steps on
    // lam with v = q (step length 0), then q = y = P(q + lam)
    e = hipMemcpyAsync(y, q_out, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail_hip(e, "tangential_solve");
    for (int j = 0; j < 2 * NEWTON + 4; ++j) {
      hipLaunchKernelGGL(k_f_sums, dim3(nb), dim3(NT), 0, st, y, y, (const double*)nullptr, 0.0, rho, w->sc, n,
                         w->part);
      hipLaunchKernelGGL(k_f_newton, dim3(1), dim3(NT), 0, st, w->part, nb, w->sc, S0, S1);
    }
    hipLaunchKernelGGL(k_f_apply, dim3(nb), dim3(NT), 0, st, y, y, (const double*)nullptr, 0.0, rho, w->sc, q,
                       qn, n, w->part);
    e = hipMemcpyAsync(q, qn, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(y, qn, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail_hip(e, "tangential_solve");
  }
  int k = 0;
  double change = INFINITY;
  bool conv = false;
  while (k < max_iter) {
    if ((rc = tangential_compliance(c, y, u, st))) return rc;
    for (int j = 0; j < NEWTON; ++j) {
      hipLaunchKernelGGL(k_f_sums, dim3(nb), dim3(NT), 0, st, y, u, ue, invL, rho, w->sc, n, w->part);
      hipLaunchKernelGGL(k_f_newton, dim3(1), dim3(NT), 0, st, w->part, nb, w->sc, S0, S1);
    }
    hipLaunchKernelGGL(k_f_apply, dim3(nb), dim3(NT), 0, st, y, u, ue, invL, rho, w->sc, q, qn, n, w->part);
    hipLaunchKernelGGL(k_f_momentum, dim3(1), dim3(NT), 0, st, w->part, nb, w->sc, w->dmap, cscale);
    hipLaunchKernelGGL(k_f_update, dim3(fblocks(2 * n)), dim3(NT), 0, st, q, qn, y, w->sc, 2 * n);
    ++k;
    if (k % CHECK == 0 || k == max_iter) {
      if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail_hip(e, "tangential_solve");
      change = w->hmap[F_CHANGE];
      if (!std::isfinite(change)) return fail(FVIM_EINVAL, "tangential_solve: iterate is not finite");
      if (change < tol) {
        conv = true;
        break;
      }
    }
  }
  // outputs: q, stick fraction, the rigid shift L lam of the stick zone
  e = hipMemcpyAsync(q_out, q, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return fail_hip(e, "tangential_solve");
  hipLaunchKernelGGL(k_f_stick, dim3(nb), dim3(NT), 0, st, q, rho, n, w->part);
  hipLaunchKernelGGL(k_f_totals, dim3(1), dim3(NT), 0, st, w->part, nb, 2, w->sc, w->dmap, (int)F_STICK);
  double lam[2];
  {
    std::lock_guard<std::recursive_mutex> lk(device_lock());     // pageable copy
    e = hipMemcpyAsync(lam, w->sc + F_LAM0, sizeof(lam), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  if (e != hipSuccess) return fail_hip(e, "tangential_solve");
  if (info) {
    info->iters = k;
    info->rel_change = change;
    info->stick_fraction = w->hmap[F_CONTACT] > 0 ? w->hmap[F_STICK] / w->hmap[F_CONTACT] : 0.0;
    info->shift[0] = L * lam[0];
    info->shift[1] = L * lam[1];
  }
  if (!conv) return fail(FVIM_ENOCONV, "tangential_solve: iteration limit reached");
  return FVIM_OK;
}

int frictional_solve(fvim_ctx* c, const double* h, double W, double mu_f, double Qx, double Qy, int coupled,
                     double tol, double tol_contact, double tol_f, int max_contact, int max_iter, double* T,
                     bool warm, fvim_frictional_info* info) {
  if (!(mu_f > 0.0) || !(W > 0.0) || !std::isfinite(W) || !std::isfinite(Qx) || !std::isfinite(Qy) ||
      !(tol > 0.0) || !(tol_contact > 0.0) || !(tol_f > 0.0) || max_iter < 1 || max_contact < 1 ||
      (coupled != 0 && coupled != 1))
    return fail(FVIM_EINVAL, "frictional_contact_solve: bad arguments");
  if (!(std::hypot(Qx, Qy) < mu_f * W))
    return fail(FVIM_EINVAL, "frictional_contact_solve: partial slip needs |Q| < mu_f W");
  int rc = fric_ensure(c);
  if (rc) return rc;
  FricWork* w = c->fric;
  hipStream_t st = c->stream;
  const size_t n = w->n;
  const int nb = fblocks(n);
  const double dA = c->grid.lx * c->grid.ly / (double)n;
  double* q = T;
  double* p = T + 2 * n;
  double* ue = w->vec + 9 * n;        // u_t of the pressure [2][n]
  double* he = ue + 2 * n;            // h - u3 of the tangential traction
  double* prev = he + n;              // traction of the previous alternation [3][n]
  hipError_t e;
  int k = 0, cit = 0, tit = 0;
  double change = INFINITY;
  bool conv = !coupled;
  fvim_contact_info ci{};
  fvim_tangential_info fi{};
  const int kmax = coupled ? max_iter : 1;
  for (k = 1; k <= kmax; ++k) {
    const bool haveq = coupled && (k > 1 || warm);      // q holds a traction to start from
    const bool track = coupled && (k > 1 || warm);
    const double* hk = h;
    if (haveq) {
      if ((rc = cerruti_cross(c, q, he, false, st))) return rc;
      hipLaunchKernelGGL(k_c_sub, dim3(nb), dim3(NT), 0, st, h, he, he, n);
      hk = he;
    }
    if (track && (e = hipMemcpyAsync(prev, T, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st)) != hipSuccess)
      return fail_hip(e, "frictional_contact_solve");
    if ((rc = pk_solve(c, hk, W, tol_contact, max_contact, p, nullptr, &ci))) return rc;
    cit += ci.iters;
    if (coupled && (rc = cerruti_cross(c, p, ue, true, st))) return rc;
    rc = friction_solve(c, p, mu_f, Qx, Qy, tol_f, max_contact, q, &fi, coupled ? haveq : warm,
                        coupled ? ue : nullptr);
    if (rc) return rc;
    tit += fi.iters;
    if (track) {
      hipLaunchKernelGGL(k_c_change, dim3(nb), dim3(NT), 0, st, T, prev, n, w->part);
      hipLaunchKernelGGL(k_f_totals, dim3(1), dim3(NT), 0, st, w->part, nb, 2, w->sc, w->dmap, (int)F_CP);
      if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail_hip(e, "frictional_contact_solve");
      change = dA * w->hmap[F_CP] / W + dA * w->hmap[F_CQ] / (mu_f * W);
      if (!std::isfinite(change)) return fail(FVIM_EINVAL, "frictional_contact_solve: iterate is not finite");
      if (change < tol) {
        conv = true;
        break;
      }
    }
  }
  if (k > kmax) k = kmax;
  if (info) {
    info->iters = k;
    info->contact_iters = cit;
    info->tangential_iters = tit;
    info->rel_change = change;
    info->kkt_residual = ci.kkt_residual;
    info->stick_fraction = fi.stick_fraction;
    info->shift[0] = fi.shift[0];
    info->shift[1] = fi.shift[1];
  }
  if (!conv) return fail(FVIM_ENOCONV, "frictional_contact_solve: alternation limit reached");
  return FVIM_OK;
}

int frictional_reserve(fvim_ctx* c) {
  int rc = fric_ensure(c);
  return rc ? rc : solver_reserve(c);
}

}  // namespace fvim

int frictional_contact_solve(fvim_ctx* ctx, const double* h, double W, double mu_f, double Qx, double Qy,
                             int coupled, double tol, int max_iter, int warm, double* traction,
                             fvim_frictional_info* info) {
  if (!ctx || !h || !traction) return fvim::fail(FVIM_EINVAL, "frictional_contact_solve: NULL argument");
  if (info) *info = fvim_frictional_info{};
  // the normal solves to a tenth of the alternation's tolerance (not below
  // 1e-15), the tangential solves to it
  const double tc = std::max(0.1 * tol, 1e-15);
  return fvim::frictional_solve(ctx, h, W, mu_f, Qx, Qy, coupled, tol, tc, tol, 100000, max_iter, traction,
                                warm != 0, info);
}

int tangential_solve(fvim_ctx* ctx, const double* p, double mu_f, double Qx, double Qy, double tol, int max_iter,
                     double* q, fvim_tangential_info* info) {
  if (!ctx || !p || !q) return fvim::fail(FVIM_EINVAL, "tangential_solve: NULL argument");
  return fvim::friction_solve(ctx, p, mu_f, Qx, Qy, tol, max_iter, q, info);
}
