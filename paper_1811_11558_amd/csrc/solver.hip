// Iterative solvers on top of the operators (all arithmetic on the GPU):
//
//  * contact_solve: the Polonsky-Keer projected conjugate gradient for the
//    Kalker dual of frictionless contact under total load (Sec. 5.1).  The
//    compliance u3 = M[p] at z = 0 is 2 / (E* |q|) per mode, applied with
//    the library's FFT kernels on one plane.  Every scalar of the iteration
//    (mean gap on the contact set, CG coefficient, step length, restart flag,
//    load renormalisation, convergence measure) is formed on the device by
//    fixed-order block reductions, so the iteration needs no host round trip;
//    the host reads the convergence measure back every few iterations.
//  * the plasticity fixed point R[d_eps] = 0 (eqn incremental_strain) by
//    DF-SANE (Sec. 4.3) or Picard, residual evaluations = radial return +
//    Mindlin operator + a fused subtraction; the nonmonotone line search
//    decides on the host from one reduced scalar per residual evaluation.
//  * elastoplastic_solve: Algorithm 1 (Sec. 5.2).
// All reductions are deterministic (fixed block partition, fixed order).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "solver.hpp"

namespace fvim {

namespace {
constexpr int NT = 256;
constexpr int RB = 1024;          // max reduction blocks
constexpr int NSCAL = 32;

// device scalar slots
enum {
  S_GBAR = 0, S_G, S_GOLD, S_BETA, S_RBAR, S_TAU, S_DELTA, S_SCALE, S_ERR, S_NIOL, S_SUMP, S_CNT, S_W, S_DA,
  S_DOT0, S_DOT1, S_DOT2, S_KKT, S_TAU0
};

// ---------------------------------------------------------------- reductions
// Block partial sums of NS quantities; block b writes part[k * RB + b].
template <int NS>
__device__ __forceinline__ void block_sums(double (&v)[NS], double* part) {
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

// Sum of nb partials of quantity k, by one block, fixed order.
__device__ double final_sum(const double* part, int k, int nb) {
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

// Block maxima of NS quantities (all >= 0); block b writes part[k * RB + b].
template <int NS>
__device__ __forceinline__ void block_max(double (&v)[NS], double* part) {
  __shared__ double sh[NS][NT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_down(x, o, 64));
    if (lane == 0) sh[k][w] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      double s = 0.0;
      for (int i = 0; i < NT / 64; ++i) s = fmax(s, sh[k][i]);
      part[k * RB + blockIdx.x] = s;
    }
  }
}

// Maximum of nb partials of quantity k (all >= 0), by one block.
__device__ double final_max(const double* part, int k, int nb) {
  __shared__ double sh[NT];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += NT) s = fmax(s, part[k * RB + i]);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

int nblocks(size_t n) {
  size_t b = (n + NT - 1) / NT;
  return (int)std::min<size_t>(b, RB);
}

// ------------------------------------------------------------ PK kernels
// g = u - h; sums over the contact set of g and of 1
__global__ __launch_bounds__(NT) void k_pk_gap(const double* __restrict__ u, const double* __restrict__ h,
                                              const double* __restrict__ p, double* __restrict__ g, size_t n,
                                              double* part) {
  double v[2] = {0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    double gi = u[i] - h[i];
    g[i] = gi;
    if (p[i] > 0.0) {
      v[0] += gi;
      v[1] += 1.0;
    }
  }
  block_sums<2>(v, part);
}

// g -= gbar; sum over the contact set of g^2
__global__ __launch_bounds__(NT) void k_pk_grad(const double* __restrict__ p, double* __restrict__ g, size_t n,
                                               const double* __restrict__ sc, double* part) {
  const double gbar = sc[S_GBAR];
  double v[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    double gi = g[i] - gbar;
    g[i] = gi;
    if (p[i] > 0.0) v[0] += gi * gi;
  }
  block_sums<1>(v, part);
}

// t = g + beta t on the contact set, 0 elsewhere
__global__ __launch_bounds__(NT) void k_pk_dir(const double* __restrict__ p, const double* __restrict__ g,
                                              double* __restrict__ t, size_t n, const double* __restrict__ sc) {
  const double beta = sc[S_BETA];
  // beta = 0 (first iteration, restart) must not read the previous
  // direction: 0 * t would carry a NaN through
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT)
    t[i] = (p[i] > 0.0) ? g[i] + (beta != 0.0 ? beta * t[i] : 0.0) : 0.0;
}

// sums over the contact set of r and 1
__global__ __launch_bounds__(NT) void k_pk_rmean(const double* __restrict__ p, const double* __restrict__ r,
                                                size_t n, double* part) {
  double v[2] = {0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT)
    if (p[i] > 0.0) {
      v[0] += r[i];
      v[1] += 1.0;
    }
  block_sums<2>(v, part);
}

// sums over the contact set of g t and (r - rbar) t
__global__ __launch_bounds__(NT) void k_pk_tau(const double* __restrict__ p, const double* __restrict__ g,
                                              const double* __restrict__ r, const double* __restrict__ t,
                                              size_t n, const double* __restrict__ sc, double* part) {
  const double rbar = sc[S_RBAR];
  double v[2] = {0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT)
    if (p[i] > 0.0) {
      v[0] += g[i] * t[i];
      v[1] += (r[i] - rbar) * t[i];
    }
  block_sums<2>(v, part);
}

// step, projection onto p >= 0, re-admission of the overlap set (points of
// negative gap enter with a pressure proportional to the overlap; when the
// conjugate-gradient step vanishes -- the gap already uniform on the contact
// set, e.g. a set of one point -- with the step of a point load, 1 / M_ii)
__global__ __launch_bounds__(NT) void k_pk_update(double* __restrict__ p, double* __restrict__ pold,
                                                 const double* __restrict__ g, const double* __restrict__ t,
                                                 size_t n, const double* __restrict__ sc, double* part) {
  const double tau = sc[S_TAU];
  const double tre = tau != 0.0 ? tau : sc[S_TAU0];
  double v[2] = {0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    double po = p[i];
    pold[i] = po;
    double pn = po - tau * t[i];
    if (pn < 0.0) pn = 0.0;
    if (pn == 0.0 && g[i] < 0.0) {
      pn = -tre * g[i];
      v[1] += 1.0;
    }
    p[i] = pn;
    v[0] += pn;
  }
  block_sums<2>(v, part);
}

// p *= scale; sum |p - p_old|
__global__ __launch_bounds__(NT) void k_pk_scale(double* __restrict__ p, const double* __restrict__ pold, size_t n,
                                                const double* __restrict__ sc, double* part) {
  const double s = sc[S_SCALE];
  double v[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    double pn = p[i] * s;
    p[i] = pn;
    v[0] += fabs(pn - pold[i]);
  }
  block_sums<1>(v, part);
}

// KKT certificate of a contact solution: with g the gap (u3 - h minus its
// mean on the contact set), the maxima of |g| on the contact set, of -g
// anywhere (a negative gap is an overlap) and of |h|
__global__ __launch_bounds__(NT) void k_pk_kkt(const double* __restrict__ p, const double* __restrict__ g,
                                              const double* __restrict__ h, size_t n, double* part) {
  double v[3] = {0.0, 0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    const double gi = g[i];
    if (p[i] > 0.0) v[0] = fmax(v[0], fabs(gi));
    v[1] = fmax(v[1], -gi);
    v[2] = fmax(v[2], fabs(h[i]));
  }
  block_max<3>(v, part);
}

// One-block finishing steps of the PK iteration: turn partial sums into the
// scalars the next kernel needs.
// Final reductions into the device scalars; the slots the host reads after
// stages 5 and 6 are also written to mirror (mapped host memory), so reading
// them needs no copy.
__global__ __launch_bounds__(NT) void k_pk_final(int stage, const double* part, int nb, double* sc,
                                                double* mirror) {
  if (stage == 0) {            // mean gap on the contact set
    double a = final_sum(part, 0, nb), c = final_sum(part, 1, nb);
    if (threadIdx.x == 0) {
      sc[S_GBAR] = c > 0.0 ? a / c : 0.0;
      sc[S_CNT] = c;
    }
  } else if (stage == 1) {     // CG coefficient
    double G = final_sum(part, 0, nb);
    if (threadIdx.x == 0) {
      double gold = sc[S_GOLD];
      sc[S_BETA] = (gold > 0.0) ? sc[S_DELTA] * G / gold : 0.0;
      sc[S_G] = G;
      sc[S_GOLD] = G;
    }
  } else if (stage == 2) {     // mean of M t on the contact set
    double a = final_sum(part, 0, nb), c = final_sum(part, 1, nb);
    if (threadIdx.x == 0) sc[S_RBAR] = c > 0.0 ? a / c : 0.0;
  } else if (stage == 3) {     // step length
    double a = final_sum(part, 0, nb), b = final_sum(part, 1, nb);
    if (threadIdx.x == 0) sc[S_TAU] = (b != 0.0) ? a / b : 0.0;
  } else if (stage == 4) {     // load renormalisation and restart flag
    double sp = final_sum(part, 0, nb), nol = final_sum(part, 1, nb);
    if (threadIdx.x == 0) {
      sc[S_SUMP] = sp;
      sc[S_SCALE] = sp > 0.0 ? sc[S_W] / (sc[S_DA] * sp) : 1.0;
      sc[S_NIOL] = nol;
      sc[S_DELTA] = nol > 0.0 ? 0.0 : 1.0;
    }
  } else if (stage == 5) {     // convergence measure dA sum |dp| / W
    double d = final_sum(part, 0, nb);
    if (threadIdx.x == 0) {
      const double err = sc[S_DA] * d / sc[S_W];
      sc[S_ERR] = err;
      mirror[S_ERR] = err;
    }
  } else if (stage == 7) {     // KKT certificate max(on, off) / max |h|
    double on = final_max(part, 0, nb), off = final_max(part, 1, nb), hm = final_max(part, 2, nb);
    if (threadIdx.x == 0) sc[S_KKT] = fmax(on, off) / (hm > 0.0 ? hm : 1e-300);
  } else if (stage == 6) {     // generic: sums of up to three quantities
    double a = final_sum(part, 0, nb), b = final_sum(part, 1, nb), c = final_sum(part, 2, nb);
    if (threadIdx.x == 0) {
      sc[S_DOT0] = mirror[S_DOT0] = a;
      sc[S_DOT1] = mirror[S_DOT1] = b;
      sc[S_DOT2] = mirror[S_DOT2] = c;
    }
  }
}

// compliance multiplier per mode, mode-major [kx][ky]: 2 / (E* |q|) / (nx ny), 0 at k = 0
__global__ __launch_bounds__(NT) void k_compliance(cpx<double>* __restrict__ s, int nx, int ny, double lx,
                                                  double ly, double fac) {
  const int kxh = nx / 2 + 1;
  const int m = blockIdx.x * NT + threadIdx.x;
  if (m >= kxh * ny) return;
  const int kx = m / ny, ky = m - kx * ny;
  const int k2 = (ky * 2 <= ny) ? ky : ky - ny;
  const double twopi = 6.283185307179586476925286766559;
  const double q1 = twopi * kx / lx, q2 = twopi * k2 / ly;
  const double q = sqrt(q1 * q1 + q2 * q2);
  const double c = (m == 0) ? 0.0 : fac / q;
  s[m] = mk(s[m].x * c, s[m].y * c);
}

__global__ __launch_bounds__(NT) void k_fill(double* x, size_t n, double v) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) x[i] = v;
}

// sum of x and of |x|
// Adhesive contact (Dugdale cohesive zone): h2 = h + s0 u (u = M[1_C])
__global__ __launch_bounds__(NT) void k_adh_surface(const double* __restrict__ h, const double* __restrict__ u,
                                                   double s0, double* __restrict__ h2, size_t n) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) h2[i] = h[i] + s0 * u[i];
}

// the cohesive set from the gap: C = 1 where gap <= h0; cnt[0] += points
// whose membership changed, cnt[1] += members (one atomic per block)
__global__ __launch_bounds__(NT) void k_adh_set(const double* __restrict__ gap, double h0, double* __restrict__ C,
                                               size_t n, unsigned long long* cnt) {
  __shared__ unsigned int sh[2][NT / 64];
  unsigned int ch = 0, in = 0;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    const double c = gap[i] <= h0 ? 1.0 : 0.0;
    ch += c != C[i];
    in += c != 0.0;
    C[i] = c;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ch += __shfl_down(ch, o, 64);
    in += __shfl_down(in, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = ch;
    sh[1][threadIdx.x >> 6] = in;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long a = 0, b = 0;
    for (int w = 0; w < NT / 64; ++w) {
      a += sh[0][w];
      b += sh[1][w];
    }
    atomicAdd(cnt, a);
    atomicAdd(cnt + 1, b);
  }
}

// total traction p = p_c - s0 C
__global__ __launch_bounds__(NT) void k_adh_total(const double* __restrict__ pc, const double* __restrict__ C,
                                                 double s0, double* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) p[i] = pc[i] - s0 * C[i];
}

__global__ __launch_bounds__(NT) void k_sum_abs(const double* __restrict__ x, size_t n, double* part) {
  double v[2] = {0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    v[0] += x[i];
    v[1] += fabs(x[i]);
  }
  block_sums<2>(v, part);
}

// ----------------------------------------------------- vector kernels
// y = a + s * b
__global__ __launch_bounds__(NT) void k_axpy(double* __restrict__ y, const double* __restrict__ a, double s,
                                            const double* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) y[i] = a[i] + s * b[i];
}

// Weight of element i of a [6][nz][plane] strain field in the scalar
// product: 2 for the shear components (each stands for two tensor entries)
// times the trapezoid weight of its depth node in units of the uniform
// spacing: wz[z] on non-uniform nodes, else 1/2 at the first and last node
// and 1 between.  plane is 2^lp.
__device__ __forceinline__ double field_weight(size_t i, int lp, unsigned nz, const double* wz) {
  const unsigned zc = (unsigned)(i >> lp);      // c * nz + z
  const unsigned z = zc % nz;
  return (zc < 3u * nz ? 1.0 : 2.0) * (wz ? wz[z] : ((z == 0 || z == nz - 1) ? 0.5 : 1.0));
}

// Sums of the pairs part[2 b], part[2 b + 1] (b < nb), in a fixed order, into
// the scalar slots S_DOT0 and S_DOT1 and their host mirror (the weighted
// <F, F> and <Fo, F - Fo> of a residual evaluation).
// zact = 1 + the deepest layer z with flags[z] set (0 if none), written to
// flags[nz] (the layers the operator reads) and flags[nz + 1] (the layers in
// which the next trial return map must store every voxel: d_eps_p is zero
// beyond); the flags are cleared for the next evaluation.
__global__ __launch_bounds__(NT) void k_zact(int* __restrict__ flags, int nz) {
  __shared__ int sh[NT];
  int za = 0;
  for (int z = threadIdx.x; z < nz; z += NT)
    if (flags[z]) {
      za = max(za, z + 1);
      flags[z] = 0;
    }
  sh[threadIdx.x] = za;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    flags[nz] = sh[0];
    flags[nz + 1] = sh[0];
  }
}

__global__ __launch_bounds__(64) void k_set_int(int* p, int v) {
  if (threadIdx.x == 0) p[0] = v;
}

constexpr int NTS = 1024;           // threads of the one block of k_sum_pairs
__global__ __launch_bounds__(NTS) void k_sum_pairs(const double* __restrict__ part, int nb, double* sc,
                                                  double* mirror) {
  __shared__ double sh[2][NTS];
  double a = 0.0, b = 0.0;
#pragma unroll 4
  for (int i = threadIdx.x; i < nb; i += NTS) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int o = NTS / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sc[S_DOT0] = mirror[S_DOT0] = sh[0][0];
    sc[S_DOT1] = mirror[S_DOT1] = sh[1][0];
  }
}

// weighted sums  <a, a>, <a, b>, <b, b>  with a = a1 - a0, b = b1 - b0 (a0/b0 may be NULL)
__global__ __launch_bounds__(NT) void k_wdots(const double* __restrict__ a1, const double* a0,
                                             const double* __restrict__ b1, const double* b0, int lp, unsigned nz,
                                             const double* __restrict__ wz, size_t n, double* part) {
  double v[3] = {0.0, 0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    double a = a1[i] - (a0 ? a0[i] : 0.0);
    double b = b1[i] - (b0 ? b0[i] : 0.0);
    const double wt = field_weight(i, lp, nz, wz);
    v[0] += wt * a * a;
    v[1] += wt * a * b;
    v[2] += wt * b * b;
  }
  block_sums<3>(v, part);
}

// plain sums of squares of (a1 - a0) and of a1 (surfaces)
__global__ __launch_bounds__(NT) void k_sq2(const double* __restrict__ a1, const double* a0, size_t n,
                                           double* part) {
  double v[2] = {0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    double a = a1[i] - (a0 ? a0[i] : 0.0);
    v[0] += a * a;
    v[1] += a1[i] * a1[i];
  }
  block_sums<2>(v, part);
}

// plain sums of a.b, a.a and b.b (surfaces)
__global__ __launch_bounds__(NT) void k_sdot3(const double* __restrict__ a, const double* __restrict__ b, size_t n,
                                             double* part) {
  double v[3] = {0.0, 0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    v[0] += a[i] * b[i];
    v[1] += a[i] * a[i];
    v[2] += b[i] * b[i];
  }
  block_sums<3>(v, part);
}

// ------------------------------------------ Newton-Krylov (Arnoldi) kernels
// Krylov vectors are [6][nz][plane] fields of which only the voxels v < na
// of each component (the layers above the deepest plastic one) take part;
// the basis u_0 .. u_m is stored contiguously, u_i = base + 6 i V, not
// normalised (the host keeps the norms); at most KMAX vectors enter one
// scalar-product or combination launch.
constexpr int KMAX = 32;
struct KCoef {
  double c[KMAX];
};

// Weighted <u_i, x> for i < n; blockIdx.y takes the four vectors from
// 4 blockIdx.y on, x is read once per group of four.  Block b writes
// part[i * RB + b].
__global__ __launch_bounds__(NT) void k_kdot(const double* __restrict__ base, int n, const double* __restrict__ x,
                                            size_t na, size_t V, int lp, unsigned nz, const double* __restrict__ wz,
                                            double* part) {
  const int i0 = blockIdx.y * 4;
  const size_t n6 = 6 * V;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (size_t v = (size_t)blockIdx.x * NT + threadIdx.x; v < na; v += (size_t)gridDim.x * NT) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const size_t i = c * V + v;
      const double xi = x[i] * field_weight(i, lp, nz, wz);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (i0 + k < n) acc[k] += base[(size_t)(i0 + k) * n6 + i] * xi;
    }
  }
  block_sums<4>(acc, part + (size_t)i0 * RB);
}

// y = a x + sum_{i<n} c_i u_i (x may be NULL; y may be x), with the block
// sums of the weighted <y, y> when part is given.
__global__ __launch_bounds__(NT) void k_kcomb(double* y, const double* x, double a, const double* __restrict__ base,
                                             int n, KCoef kc, size_t na, size_t V, int lp, unsigned nz,
                                             const double* __restrict__ wz, double* part) {
  __shared__ double cs[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j)
    if ((int)threadIdx.x == j) cs[j] = kc.c[j];
  __syncthreads();
  const size_t n6 = 6 * V;
  double nn[1] = {0.0};
  for (size_t v = (size_t)blockIdx.x * NT + threadIdx.x; v < na; v += (size_t)gridDim.x * NT) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const size_t i = c * V + v;
      double r = x ? a * x[i] : 0.0;
      for (int j = 0; j < n; ++j) r += cs[j] * base[(size_t)j * n6 + i];
      y[i] = r;
      nn[0] += field_weight(i, lp, nz, wz) * r * r;
    }
  }
  if (part) block_sums<1>(nn, part);
}

// out[k] = sum of the nb partials of row k, one block per row, fixed order.
__global__ __launch_bounds__(NT) void k_kfinal(const double* __restrict__ part, int nb, double* out) {
  const double r = final_sum(part, blockIdx.x, nb);
  if (threadIdx.x == 0) out[blockIdx.x] = r;
}

// ------------------------------------------- Anderson acceleration (outer)
constexpr int AA_MMAX = 6;
constexpr int aa_nsums(int m) { return m * (m + 1) / 2 + m; }

// Gram matrix of the M residual differences dF[j] (stride n) and their
// products with f: sums in the order (0,0) (0,1) .. (M-1,M-1), then <dF_j, f>.
template <int M>
__global__ __launch_bounds__(NT) void k_aa_gram(const double* __restrict__ dF, const double* __restrict__ f,
                                               size_t n, double* part) {
  constexpr int K = aa_nsums(M);
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    double a[M];
#pragma unroll
    for (int j = 0; j < M; ++j) a[j] = dF[(size_t)j * n + i];
    const double fi = f[i];
    int k = 0;
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
      for (int l = j; l < M; ++l) v[k++] += a[j] * a[l];
#pragma unroll
    for (int j = 0; j < M; ++j) v[k++] += a[j] * fi;
  }
  block_sums<K>(v, part);
}

// out[k] = sum over the nb block partials of quantity k, fixed order
__global__ __launch_bounds__(64) void k_aa_final(const double* __restrict__ part, int K, int nb, double* out) {
  const int k = threadIdx.x;
  if (k >= K) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)k * RB + b];
  out[k] = s;
}

struct AACoef {
  double g[AA_MMAX];
};

// x <- x + beta f - sum_j g_j (dX_j + beta dF_j)
__global__ __launch_bounds__(NT) void k_aa_step(double* __restrict__ x, const double* __restrict__ f,
                                               const double* __restrict__ dX, const double* __restrict__ dF,
                                               AACoef c, int m, double beta, size_t n) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    double v = x[i] + beta * f[i];
    for (int j = 0; j < m; ++j) v -= c.g[j] * (dX[(size_t)j * n + i] + beta * dF[(size_t)j * n + i]);
    x[i] = v;
  }
}

}  // namespace

struct SolverWork {
  size_t ns = 0, V = 0;
  int lp = 0;                   // log2(ns)
  double* surf = nullptr;       // 15 surface arrays
  void* specA = nullptr;        // complex kxh*ny
  void* specB = nullptr;
  double* part = nullptr;       // 3 * RB partial sums
  double* sc = nullptr;         // device scalars
  double* hsc = nullptr;        // pinned host copy
  double* hmap = nullptr;       // mapped host memory written by k_pk_final (host view)
  double* dmap = nullptr;       //   (device view)
  double* vol = nullptr;        // volume work arrays (allocated on first plasticity use)
  size_t vol_count = 0;
  double* rpart = nullptr;      // partial-sum pairs of the fused residual evaluation
  int rpart_count = 0;
  int* layers = nullptr;        // [nz] plastic-layer flags of the trial point, zact, zwrite
  // one contact iteration captured as a HIP graph, replayed on a private
  // stream fenced by events against the context stream
  hipStream_t cap = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraph_t pk_graph = nullptr;
  hipGraphExec_t pk_exec = nullptr;
  const double* g_h = nullptr;
  const double* g_p = nullptr;
  // Anderson history of the outer fixed point: dX, dF [AA_MMAX][ns];
  // xprev, fprev, f [ns]; Gram partials and results (device, pinned host)
  double* aa = nullptr;
  double* aa_part = nullptr;
  double* aa_out = nullptr;     // device view of aa_hout (mapped host memory)
  double* aa_hout = nullptr;
  // captured residual evaluations (operator, residual and its reduction),
  // one per combination of the pointers and settings they bake in; replayed
  // on the context stream
  // pointers and settings a captured evaluation bakes in
  static constexpr int NKEY = 13;
  struct ResGraph {
    const void* key[NKEY] = {};
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
  };
  static constexpr int NRG = 8;    // trial or plain point x two buffer parities x two precisions
  ResGraph rg[NRG];
  int rg_next = 0;
  int rg_warm[2] = {0, 0};       // an eager evaluation has sized every buffer (per precision)
  int cap_fail = 0;              // failed captures; from CAP_TRIES on, launch directly
  // Newton-Krylov: basis u_0 .. u_m and the Newton step, [kry_m + 2][6 V];
  // scalar-product partials [KMAX][RB]; their totals (mapped host memory)
  double* kry = nullptr;
  int kry_m = 0;
  double* kry_part = nullptr;
  double* kry_out = nullptr;     // device view
  double* kry_hout = nullptr;    // host view
  // outer Newton-Krylov (coupling = 1): base strain and right-hand side
  // [2][6 V], base traction [3][ns], then surface vectors (x, G(x), F, step,
  // trial, work and the Krylov basis)
  double* cpl = nullptr;
  size_t cpl_count = 0;
  double mdiag = 0.0;           // diagonal of the surface compliance (contact)
  // adhesive contact: cohesive set, repulsive pressure, modified surface,
  // compliance and gap [5][ns]; set counters (device) and their host copy
  double* adh = nullptr;
  unsigned long long* adh_cnt = nullptr;
  unsigned long long* adh_hcnt = nullptr;
};

constexpr int CAP_TRIES = 4;

// The private capture stream and the events that fence it against the
// context stream.
static int cap_ensure(SolverWork* w) {
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  if (!w->cap && hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking) != hipSuccess) {
    w->cap = nullptr;
    return fail(FVIM_EHIP, "graph stream");
  }
  if (!w->ev_in && hipEventCreateWithFlags(&w->ev_in, hipEventDisableTiming) != hipSuccess) {
    w->ev_in = nullptr;
    return fail(FVIM_EHIP, "graph event");
  }
  if (!w->ev_out && hipEventCreateWithFlags(&w->ev_out, hipEventDisableTiming) != hipSuccess) {
    w->ev_out = nullptr;
    return fail(FVIM_EHIP, "graph event");
  }
  return FVIM_OK;
}

// After a capture that failed: drop what it produced and clear the error it
// left, so that the direct launches that replace it report their own status.
static void capture_failed(SolverWork* w, hipGraph_t* g, hipGraphExec_t* ex) {
  if (*ex) hipGraphExecDestroy(*ex);
  if (*g) hipGraphDestroy(*g);
  *ex = nullptr;
  *g = nullptr;
  (void)hipGetLastError();
  ++w->cap_fail;
}

static int sw_ensure(fvim_ctx* c) {
  if (c->sw) return FVIM_OK;
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  SolverWork* w = new SolverWork();
  w->ns = (size_t)c->grid.nx * c->grid.ny;
  w->lp = 0;
  while (((size_t)1 << w->lp) < w->ns) ++w->lp;
  w->V = w->ns * c->grid.nz;
  const size_t nm = (size_t)(c->grid.nx / 2 + 1) * c->grid.ny;
  bool ok = hipMalloc((void**)&w->surf, sizeof(double) * w->ns * 15) == hipSuccess &&
            hipMalloc(&w->specA, sizeof(cpx<double>) * nm) == hipSuccess &&
            hipMalloc(&w->specB, sizeof(cpx<double>) * nm) == hipSuccess &&
            hipMalloc((void**)&w->part, sizeof(double) * 3 * RB) == hipSuccess &&
            hipMalloc((void**)&w->sc, sizeof(double) * NSCAL) == hipSuccess &&
            hipHostMalloc((void**)&w->hsc, sizeof(double) * NSCAL, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&w->hmap, sizeof(double) * NSCAL,
                          hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
            hipHostGetDevicePointer((void**)&w->dmap, w->hmap, 0) == hipSuccess;
  c->sw = w;
  if (!ok) return fail(FVIM_ENOMEM, "solver workspace allocation failed");
  // the final reductions always sum three rows of partials; rows a kernel
  // does not write then read zeros, not whatever the allocation held
  hipError_t e = hipMemsetAsync(w->part, 0, sizeof(double) * 3 * RB, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail_hip(e, "solver workspace");
  return FVIM_OK;
}

int solver_reserve(fvim_ctx* c) { return sw_ensure(c); }

void solver_release(fvim_ctx* c) {
  SolverWork* w = c->sw;
  if (!w) return;
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  if (w->surf) hipFree(w->surf);
  if (w->specA) hipFree(w->specA);
  if (w->specB) hipFree(w->specB);
  if (w->part) hipFree(w->part);
  if (w->sc) hipFree(w->sc);
  if (w->hsc) hipHostFree(w->hsc);
  if (w->hmap) hipHostFree(w->hmap);
  if (w->vol) hipFree(w->vol);
  if (w->rpart) hipFree(w->rpart);
  if (w->layers) hipFree(w->layers);
  if (w->aa) hipFree(w->aa);
  if (w->aa_part) hipFree(w->aa_part);
  if (w->aa_hout) hipHostFree(w->aa_hout);
  if (w->kry) hipFree(w->kry);
  if (w->kry_part) hipFree(w->kry_part);
  if (w->kry_hout) hipHostFree(w->kry_hout);
  if (w->cpl) hipFree(w->cpl);
  if (w->adh) hipFree(w->adh);
  if (w->adh_cnt) hipFree(w->adh_cnt);
  if (w->adh_hcnt) hipHostFree(w->adh_hcnt);
  for (auto& r : w->rg) {
    if (r.ex) hipGraphExecDestroy(r.ex);
    if (r.g) hipGraphDestroy(r.g);
  }
  if (w->pk_exec) hipGraphExecDestroy(w->pk_exec);
  if (w->pk_graph) hipGraphDestroy(w->pk_graph);
  if (w->ev_in) hipEventDestroy(w->ev_in);
  if (w->ev_out) hipEventDestroy(w->ev_out);
  if (w->cap) hipStreamDestroy(w->cap);
  delete w;
  c->sw = nullptr;
}

size_t solver_footprint(const fvim_grid* g, size_t V) {
  const size_t ns = (size_t)g->nx * g->ny;
  const size_t nm = (size_t)(g->nx / 2 + 1) * g->ny;
  // surface arrays (15 + Anderson history 2 AA_MMAX + 3 + adhesion 5), volume work
  // arrays (6 tensors + 1 scalar), residual partial sums, compliance
  // spectra, reduction buffers
  return sizeof(double) * (ns * (23 + 2 * AA_MMAX) + 37 * V + 2 * (size_t)operator_resid_parts(*g)) +
         2 * sizeof(cpx<double>) * nm +
         sizeof(double) * aa_nsums(AA_MMAX) * (RB + 2) + 64 * 1024;
}

// Host copy of device scalars [first, first + n) (synchronises the stream).
// The slots k_pk_final mirrors (S_ERR, S_DOT0..S_DOT2) are taken from the
// mapped mirror once the stream is idle; others are copied.
static int read_scalars_on(fvim_ctx* c, hipStream_t st, int first, int n) {
  SolverWork* w = c->sw;
  const bool mirrored = (first == S_ERR && n == 1) || (first >= S_DOT0 && first + n <= S_DOT2 + 1);
  hipError_t e = hipSuccess;
  if (!mirrored) e = hipMemcpyAsync(w->hsc + first, w->sc + first, sizeof(double) * n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail_hip(e, "scalar readback");
  if (mirrored)
    for (int k = first; k < first + n; ++k) w->hsc[k] = w->hmap[k];
  return FVIM_OK;
}

static int read_scalars(fvim_ctx* c, int first, int n) { return read_scalars_on(c, c->stream, first, n); }

static int set_scalar(fvim_ctx* c, int slot, double v) {
  SolverWork* w = c->sw;
  w->hsc[slot] = v;
  hipError_t e = hipMemcpyAsync(w->sc + slot, w->hsc + slot, sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail_hip(e, "scalar upload");
  return FVIM_OK;
}

// u = M[p] . e3 at z = 0 for a normal surface load p (one plane).
static int compliance(fvim_ctx* c, const double* p, double* u, hipStream_t st) {
  SolverWork* w = c->sw;
  const int nx = c->grid.nx, ny = c->grid.ny, kxh = nx / 2 + 1;
  const cpx<double>* twx = (const cpx<double>*)c->twx64;
  const cpx<double>* twy = (const cpx<double>*)c->twy64;
  cpx<double>* A = (cpx<double>*)w->specA;
  cpx<double>* B = (cpx<double>*)w->specB;
  hipError_t e;
  if ((e = launch_x_r2c<double>(p, A, nx, ny, 1, twx, st)) != hipSuccess) return fail_hip(e, "compliance x");
  if ((e = launch_y_fwd<double>(A, B, ny, kxh, 1, 1, twy, st)) != hipSuccess) return fail_hip(e, "compliance y");
  const double estar = c->mat.E / (1.0 - c->mat.nu * c->mat.nu);
  const double fac = 2.0 / estar / ((double)nx * ny);
  const int nm = kxh * ny;
  hipLaunchKernelGGL(k_compliance, dim3((nm + NT - 1) / NT), dim3(NT), 0, st, B, nx, ny, c->grid.lx, c->grid.ly,
                     fac);
  if ((e = launch_y_inv<double>(B, A, ny, kxh, 1, 1, twy, st)) != hipSuccess) return fail_hip(e, "compliance y^-1");
  OutSegments seg;
  seg.n = 1;
  seg.first[0] = 0;
  seg.ptr[0] = u;
  if ((e = launch_x_c2r<double>(A, seg, nx, ny, 1, 1.0, twx, st)) != hipSuccess)
    return fail_hip(e, "compliance x^-1");
  return FVIM_OK;
}

// One Polonsky-Keer iteration as a fixed sequence of launches on st (no host
// dependency: every scalar lives in device memory), so it can be captured.
static int pk_iteration(fvim_ctx* c, hipStream_t st, const double* h, double* p) {
  SolverWork* w = c->sw;
  const size_t n = w->ns;
  const int nb = nblocks(n);
  const dim3 G(nb), Bk(NT);
  double* u = w->surf;
  double* g = w->surf + n;
  double* t = w->surf + 2 * n;
  double* r = w->surf + 3 * n;
  double* pold = w->surf + 4 * n;
  int rc;
  if ((rc = compliance(c, p, u, st))) return rc;
  hipLaunchKernelGGL(k_pk_gap, G, Bk, 0, st, u, h, p, g, n, w->part);
  hipLaunchKernelGGL(k_pk_final, dim3(1), Bk, 0, st, 0, w->part, nb, w->sc, w->dmap);
  hipLaunchKernelGGL(k_pk_grad, G, Bk, 0, st, p, g, n, w->sc, w->part);
  hipLaunchKernelGGL(k_pk_final, dim3(1), Bk, 0, st, 1, w->part, nb, w->sc, w->dmap);
  hipLaunchKernelGGL(k_pk_dir, G, Bk, 0, st, p, g, t, n, w->sc);
  if ((rc = compliance(c, t, r, st))) return rc;
  hipLaunchKernelGGL(k_pk_rmean, G, Bk, 0, st, p, r, n, w->part);
  hipLaunchKernelGGL(k_pk_final, dim3(1), Bk, 0, st, 2, w->part, nb, w->sc, w->dmap);
  hipLaunchKernelGGL(k_pk_tau, G, Bk, 0, st, p, g, r, t, n, w->sc, w->part);
  hipLaunchKernelGGL(k_pk_final, dim3(1), Bk, 0, st, 3, w->part, nb, w->sc, w->dmap);
  hipLaunchKernelGGL(k_pk_update, G, Bk, 0, st, p, pold, g, t, n, w->sc, w->part);
  hipLaunchKernelGGL(k_pk_final, dim3(1), Bk, 0, st, 4, w->part, nb, w->sc, w->dmap);
  hipLaunchKernelGGL(k_pk_scale, G, Bk, 0, st, p, pold, n, w->sc, w->part);
  hipLaunchKernelGGL(k_pk_final, dim3(1), Bk, 0, st, 5, w->part, nb, w->sc, w->dmap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_hip(e, "contact iteration");
  return FVIM_OK;
}

// Polonsky-Keer on the context stream.  p: in warm start (all zero ->
// uniform), out solution.  gap may be NULL.
int pk_solve(fvim_ctx* c, const double* h, double W, double tol, int max_iter, double* p, double* gap,
             fvim_contact_info* info) {
  int rc = sw_ensure(c);
  if (rc) return rc;
  SolverWork* w = c->sw;
  hipStream_t st = c->stream;
  const size_t n = w->ns;
  const int nb = nblocks(n);
  const dim3 G(nb), Bk(NT);
  double* u = w->surf;
  double* g = w->surf + n;
  double* t = w->surf + 2 * n;
  const double dA = c->grid.lx * c->grid.ly / (double)n;
  // scalars: load, area, restart state, the point-load step 1 / M_ii
  if (!(w->mdiag > 0.0)) {
    // M_ii: the mean over the nx x ny modes of 2 / (E* |q|), mode 0 dropped
    const int nx = c->grid.nx, ny = c->grid.ny;
    const double estar = c->mat.E / (1.0 - c->mat.nu * c->mat.nu);
    const double twopi = 6.283185307179586476925286766559;
    double sum = 0.0;
    for (int ky = 0; ky < ny; ++ky)
      for (int kx = 0; kx < nx; ++kx) {
        if (kx == 0 && ky == 0) continue;
        const int k1 = 2 * kx <= nx ? kx : kx - nx, k2 = 2 * ky <= ny ? ky : ky - ny;
        const double q1 = twopi * k1 / c->grid.lx, q2 = twopi * k2 / c->grid.ly;
        sum += 2.0 / (estar * std::sqrt(q1 * q1 + q2 * q2));
      }
    w->mdiag = sum / ((double)nx * ny);
  }
  w->hsc[S_W] = W;
  w->hsc[S_DA] = dA;
  w->hsc[S_DELTA] = 0.0;
  w->hsc[S_GOLD] = 1.0;
  w->hsc[S_TAU0] = 1.0 / w->mdiag;
  hipError_t e = hipMemcpyAsync(w->sc, w->hsc, sizeof(double) * NSCAL, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail_hip(e, "scalar upload");
  // no previous conjugate direction
  hipLaunchKernelGGL(k_fill, G, Bk, 0, st, t, n, 0.0);
  // initial pressure: warm start renormalised to W, or uniform
  hipLaunchKernelGGL(k_sum_abs, G, Bk, 0, st, p, n, w->part);
  hipLaunchKernelGGL(k_pk_final, dim3(1), Bk, 0, st, 6, w->part, nb, w->sc, w->dmap);
  if ((rc = read_scalars(c, S_DOT0, 2))) return rc;
  const double sp = w->hsc[S_DOT0];
  if (!(sp > 0.0) || !std::isfinite(sp)) {
    hipLaunchKernelGGL(k_fill, G, Bk, 0, st, p, n, W / (n * dA));
  } else {
    if ((rc = set_scalar(c, S_SCALE, W / (dA * sp)))) return rc;
    hipLaunchKernelGGL(k_pk_scale, G, Bk, 0, st, p, p, n, w->sc, w->part);
  }
  int it = 0;
  double err = INFINITY;
  const int check = n <= 4096 ? 1 : 4;        // host convergence check period
  hipStream_t run = st;
  bool graph = c->use_graphs && w->cap_fail < CAP_TRIES;
  if (graph) {
    if ((rc = cap_ensure(w))) return rc;
    if ((e = hipEventRecord(w->ev_in, st)) != hipSuccess) return fail_hip(e, "event");
    if ((e = hipStreamWaitEvent(w->cap, w->ev_in, 0)) != hipSuccess) return fail_hip(e, "event wait");
    run = w->cap;
    if (!w->pk_exec || w->g_h != h || w->g_p != p) {
      if (w->pk_exec) { hipGraphExecDestroy(w->pk_exec); w->pk_exec = nullptr; }
      if (w->pk_graph) { hipGraphDestroy(w->pk_graph); w->pk_graph = nullptr; }
      std::lock_guard<std::recursive_mutex> lk(device_lock());
      if ((e = hipStreamBeginCapture(run, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return fail_hip(e, "graph capture");
      int rc2 = pk_iteration(c, run, h, p);
      e = hipStreamEndCapture(run, &w->pk_graph);
      if (rc2 || e != hipSuccess || !w->pk_graph ||
          hipGraphInstantiate(&w->pk_exec, w->pk_graph, nullptr, nullptr, 0) != hipSuccess) {
        // the capture was invalidated (for instance by a device-wide
        // synchronisation in another thread): nothing it recorded ran, so
        // this solve iterates with direct launches
        capture_failed(w, &w->pk_graph, &w->pk_exec);
        graph = false;
      } else {
        w->g_h = h;
        w->g_p = p;
      }
    }
  }
  for (it = 1; it <= max_iter; ++it) {
    if (graph) {
      if ((e = hipGraphLaunch(w->pk_exec, run)) != hipSuccess) return fail_hip(e, "graph launch");
    } else {
      if ((rc = pk_iteration(c, run, h, p))) return rc;
    }
    if (it % check == 0 || it == max_iter) {
      if ((rc = read_scalars_on(c, run, S_ERR, 1))) return rc;
      err = w->hsc[S_ERR];
      if (!std::isfinite(err)) return fail(FVIM_EINVAL, "contact_solve: non-finite iterate (check h and W)");
      if (err < tol) break;
    }
  }
  if (run != st) {
    if ((e = hipEventRecord(w->ev_out, run)) != hipSuccess) return fail_hip(e, "event");
    if ((e = hipStreamWaitEvent(st, w->ev_out, 0)) != hipSuccess) return fail_hip(e, "event wait");
  }
  const bool conv = err < tol;
  if (it > max_iter) it = max_iter;
  // final gap and certificate
  if ((rc = compliance(c, p, u, st))) return rc;
  hipLaunchKernelGGL(k_pk_gap, G, Bk, 0, st, u, h, p, g, n, w->part);
  hipLaunchKernelGGL(k_pk_final, dim3(1), Bk, 0, st, 0, w->part, nb, w->sc, w->dmap);
  hipLaunchKernelGGL(k_pk_grad, G, Bk, 0, st, p, g, n, w->sc, w->part);
  hipLaunchKernelGGL(k_pk_kkt, G, Bk, 0, st, p, g, h, n, w->part);
  hipLaunchKernelGGL(k_pk_final, dim3(1), Bk, 0, st, 7, w->part, nb, w->sc, w->dmap);
  if (gap) {
    e = hipMemcpyAsync(gap, g, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail_hip(e, "gap copy");
  }
  if ((rc = read_scalars(c, 0, NSCAL))) return rc;
  if (info) {
    info->iters = it;
    info->rel_change = err;
    info->contact_fraction = w->hsc[S_CNT] / (double)n;
    info->mean_gap = w->hsc[S_GBAR];
    info->kkt_residual = w->hsc[S_KKT];
  }
  if (!conv) return fail(FVIM_ENOCONV, "contact_solve: iteration limit reached");
  return FVIM_OK;
}

// --------------------------------------------------------- plasticity
struct PlastBufs {
  double *x, *F, *xt, *Ft, *b, *dep, *dp;
  const double* dT;             // traction increment of the current solve
};

static int vol_ensure(fvim_ctx* c, PlastBufs& pb) {
  SolverWork* w = c->sw;
  const size_t V = w->V;
  const size_t need = 6 * 6 * V + V;
  if (w->vol_count < need) {
    std::lock_guard<std::recursive_mutex> lk(device_lock());
    if (w->vol) {
      hipStreamSynchronize(c->stream);
      hipFree(w->vol);
      w->vol = nullptr;
    }
    if (hipMalloc((void**)&w->vol, sizeof(double) * need) != hipSuccess) {
      w->vol_count = 0;
      return fail(FVIM_ENOMEM, "plasticity workspace allocation failed");
    }
    w->vol_count = need;
    if (w->layers)                                   // a new d_eps_p holds nothing yet
      hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, c->stream, w->layers + c->grid.nz + 1, c->grid.nz);
  }
  const int np2 = operator_resid_parts(c->grid);
  if (w->rpart_count < np2) {
    std::lock_guard<std::recursive_mutex> lk(device_lock());
    if (w->rpart) {
      hipStreamSynchronize(c->stream);
      hipFree(w->rpart);
      w->rpart = nullptr;
    }
    if (hipMalloc((void**)&w->rpart, sizeof(double) * 2 * np2) != hipSuccess) {
      w->rpart_count = 0;
      return fail(FVIM_ENOMEM, "plasticity workspace allocation failed");
    }
    w->rpart_count = np2;
  }
  if (!w->layers) {
    std::lock_guard<std::recursive_mutex> lk(device_lock());
    const size_t bytes = sizeof(int) * ((size_t)c->grid.nz + 2);
    hipError_t e = hipMalloc((void**)&w->layers, bytes);
    if (e == hipSuccess) e = hipMemsetAsync(w->layers, 0, bytes, c->stream);
    if (e == hipSuccess) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, c->stream, w->layers + c->grid.nz + 1,
                                            c->grid.nz);     // d_eps_p holds nothing yet: store every voxel
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      if (w->layers) hipFree(w->layers);
      w->layers = nullptr;
      return fail_hip(e, "plasticity workspace");
    }
  }
  double* q = w->vol;
  pb.x = q;
  pb.F = q + 6 * V;
  pb.xt = q + 12 * V;
  pb.Ft = q + 18 * V;
  pb.b = q + 24 * V;
  pb.dep = q + 30 * V;
  pb.dp = q + 36 * V;
  pb.dT = nullptr;
  return FVIM_OK;
}

// weighted scalar product scale: cell area x depth spacing
static double inner_scale(const fvim_ctx* c) {
  const fvim_grid& g = c->grid;
  return g.lx * g.ly / ((double)g.nx * g.ny) * g.lz / (g.nz - 1);
}

// One residual evaluation after the return map: one operator application
// with both sources (grad_s M[dep] + grad_s M[dT]) whose last transform
// forms F = x - w in place of w, with the block sums of <F, F> and
// <Fo, F - Fo> (Fo may be NULL); then their fixed-order total, on the
// context stream.
static int residual_launches(fvim_ctx* c, PlastBufs& pb, const double* x, double* F, const double* Fo) {
  SolverWork* w = c->sw;
  int nb = 0;
  int rc = operator_apply_resid(c, pb.dep, pb.dT, x, Fo, F, w->rpart, &nb, w->layers + c->grid.nz);
  if (rc) return rc;
  if (nb > w->rpart_count) return fail(FVIM_EINVAL, "residual partial sums: workspace too small");
  hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(NTS), 0, c->stream, w->rpart, nb, w->sc, w->dmap);
  return FVIM_OK;
}

// The launches above as a replayed HIP graph when the context allows it
// (graphs on, no tuning or stage timing pending, buffers already sized by an
// eager evaluation in this precision); else launched directly.
static int residual_enqueue(fvim_ctx* c, PlastBufs& pb, const double* x, double* F, const double* Fo) {
  SolverWork* w = c->sw;
  const int p64 = (c->precision == FVIM_FP64 || c->force_fp64) ? 1 : 0;
  if (!c->use_graphs || w->cap_fail >= CAP_TRIES || c->tune_pending || c->timing || c->use_side)
    return residual_launches(c, pb, x, F, Fo);
  if (!w->rg_warm[p64]) {
    w->rg_warm[p64] = 1;
    return residual_launches(c, pb, x, F, Fo);
  }
  const void* key[SolverWork::NKEY] = {x, F, Fo, pb.dT, w->vol, w->rpart, w->layers, c->bufA, c->bufB, c->k0buf,
                                       (const void*)(intptr_t)(p64 + 2),
                                       (const void*)(intptr_t)(c->depth_cfg + 16 + ((intptr_t)fft_pack_all(c) << 8)),
                                       (const void*)(intptr_t)(c->streaming + 8)};
  for (auto& r : w->rg)
    if (r.ex && std::equal(key, key + SolverWork::NKEY, r.key)) {
      hipError_t e = hipGraphLaunch(r.ex, c->stream);
      return e == hipSuccess ? FVIM_OK : fail_hip(e, "graph launch");
    }
  // capture on the private stream (the context stream is pointed at it)
  int rc = cap_ensure(w);
  if (rc) return rc;
  SolverWork::ResGraph& r = w->rg[w->rg_next];
  w->rg_next = (w->rg_next + 1) % SolverWork::NRG;
  if (r.ex) { hipGraphExecDestroy(r.ex); r.ex = nullptr; }
  if (r.g) { hipGraphDestroy(r.g); r.g = nullptr; }
  hipStream_t saved = c->stream;
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  hipError_t e = hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return fail_hip(e, "graph capture");
  c->stream = w->cap;
  rc = residual_launches(c, pb, x, F, Fo);
  c->stream = saved;
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(w->cap, &g);
  if (rc || e != hipSuccess || !g ||
      hipGraphInstantiate(&r.ex, g, nullptr, nullptr, 0) != hipSuccess) {
    capture_failed(w, &g, &r.ex);       // nothing recorded ran: evaluate directly
    return residual_launches(c, pb, x, F, Fo);
  }
  r.g = g;
  std::copy(key, key + SolverWork::NKEY, r.key);
  e = hipGraphLaunch(r.ex, c->stream);
  return e == hipSuccess ? FVIM_OK : fail_hip(e, "graph launch");
}

// After a return map that stored d_eps_p for every voxel, the field may be
// nonzero in any layer: the next trial return map stores every voxel again.
static void dep_written_everywhere(fvim_ctx* c) {
  SolverWork* w = c->sw;
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, c->stream, w->layers + c->grid.nz + 1, c->grid.nz);
}

// Residual at the trial point xt = x + cf Fo (Fo NULL: at x itself, xt
// ignored) into F: radial return at xt, then the evaluation above.  Returns
// the weighted <F, F> in *f and, with Fo, <Fo, F - Fo> in *d.
static int residual(fvim_ctx* c, const fvim_state* s, PlastBufs& pb, const double* x, const double* Fo, double cf,
                    double* xt, double* F, double* f, double* d = nullptr) {
  SolverWork* w = c->sw;
  hipError_t e = launch_trial_return_map(x, Fo, cf, Fo ? xt : nullptr, s->sigma, s->ep, pb.dep, w->V, c->lam, c->mu,
                                         c->mat.sigma_y0, c->mat.E_h, c->stream, w->layers, w->lp,
                                         w->layers + c->grid.nz + 1);
  if (e != hipSuccess) return fail_hip(e, "return map");
  // the deepest layer with plastic strain: the operator skips the layers below
  hipLaunchKernelGGL(k_zact, dim3(1), dim3(NT), 0, c->stream, w->layers, c->grid.nz);
  int rc = residual_enqueue(c, pb, Fo ? xt : x, F, Fo);
  if (rc) return rc;
  if ((rc = read_scalars(c, S_DOT0, Fo ? 2 : 1))) return rc;
  const double sc = inner_scale(c);
  *f = w->hsc[S_DOT0] * sc;
  if (d) *d = Fo ? w->hsc[S_DOT1] * sc : 0.0;
  if (!std::isfinite(*f)) return fail(FVIM_EINVAL, "plasticity residual is not finite");
  return FVIM_OK;
}

static int wdots(fvim_ctx* c, const double* a1, const double* a0, const double* b1, const double* b0, double out[3]) {
  SolverWork* w = c->sw;
  const size_t n6 = 6 * w->V;
  const int nb = nblocks(n6);
  hipLaunchKernelGGL(k_wdots, dim3(nb), dim3(NT), 0, c->stream, a1, a0, b1, b0, w->lp, (unsigned)c->grid.nz, c->wz,
                     n6, w->part);
  hipLaunchKernelGGL(k_pk_final, dim3(1), dim3(NT), 0, c->stream, 6, w->part, nb, w->sc, w->dmap);
  int rc = read_scalars(c, S_DOT0, 3);
  if (rc) return rc;
  const double sc = inner_scale(c);
  for (int k = 0; k < 3; ++k) out[k] = w->hsc[S_DOT0 + k] * sc;
  return FVIM_OK;
}

static void axpy(fvim_ctx* c, double* y, const double* a, double s, const double* b, size_t n) {
  hipLaunchKernelGGL(k_axpy, dim3(nblocks(n)), dim3(NT), 0, c->stream, y, a, s, b, n);
}

// Restores force_fp64 on scope exit.
struct Fp64Scope {
  fvim_ctx* c;
  int saved;
  Fp64Scope(fvim_ctx* cc, int on) : c(cc), saved(cc->force_fp64) { c->force_fp64 = on; }
  ~Fp64Scope() { c->force_fp64 = saved; }
};

// One DF-SANE / Picard run from the current pb.x to |R| <= tol_abs.
static int fixed_point(fvim_ctx* c, const fvim_state* s, const fvim_ep_opts* o, PlastBufs& pb, double tol_abs,
                       int max_it, int* iters, int* evals, double* fout) {
  double f;
  int rc = residual(c, s, pb, pb.x, nullptr, 0.0, nullptr, pb.F, &f);
  if (rc) return rc;
  int ne = 1, k = 0;
  if (o->solver == 1) {            // Picard: x <- x - R(x)
    while (std::sqrt(f) > tol_abs && k < max_it) {
      if ((rc = residual(c, s, pb, pb.x, pb.F, -1.0, pb.xt, pb.Ft, &f))) return rc;
      std::swap(pb.x, pb.xt);
      std::swap(pb.F, pb.Ft);
      ++ne;
      ++k;
    }
  } else {                         // DF-SANE, parameters of La Cruz et al. (2006)
    const int M = 10;
    const double gamma = 1e-4, smin = 1e-10, smax = 1e10, tmin = 0.1, tmax = 0.5;
    std::vector<double> hist{f};
    const double f0n = std::sqrt(f);
    double sigma = 1.0;
    while (std::sqrt(f) > tol_abs && k < max_it) {
      const double eta = f0n / ((1.0 + k) * (1.0 + k));
      double fbar = 0.0;
      for (size_t i = hist.size() > (size_t)M ? hist.size() - M : 0; i < hist.size(); ++i) fbar = std::max(fbar, hist[i]);
      double ap = 1.0, am = 1.0, fn = 0.0, cs = 0.0, dfy = 0.0;
      int guard = 0;
      while (true) {
        double fp, dp, fm, dm;
        const double cp = -ap * sigma;                     // x + ap d, d = -sigma F
        if ((rc = residual(c, s, pb, pb.x, pb.F, cp, pb.xt, pb.Ft, &fp, &dp))) return rc;
        ++ne;
        if (fp <= fbar + eta - gamma * ap * ap * f) { fn = fp; cs = cp; dfy = dp; break; }
        const double cm = am * sigma;                      // x - am d
        if ((rc = residual(c, s, pb, pb.x, pb.F, cm, pb.xt, pb.Ft, &fm, &dm))) return rc;
        ++ne;
        if (fm <= fbar + eta - gamma * am * am * f) { fn = fm; cs = cm; dfy = dm; break; }
        double at = ap * ap * f / (fp + (2.0 * ap - 1.0) * f);
        ap = std::min(std::max(at, tmin * ap), tmax * ap);
        at = am * am * f / (fm + (2.0 * am - 1.0) * f);
        am = std::min(std::max(at, tmin * am), tmax * am);
        if (++guard > 60) return fail(FVIM_ENOCONV, "DF-SANE line search failed");
      }
      // spectral coefficient from s = xt - x = cs F and y = Ft - F:
      // <s, s> = cs^2 <F, F>, <s, y> = cs <F, Ft - F>
      const double ss = cs * cs * f, sy = cs * dfy;
      if (sy == 0.0) sigma = smax;
      else {
        sigma = ss / sy;
        const double sg = sigma >= 0 ? 1.0 : -1.0;
        sigma = sg * std::min(std::max(std::fabs(sigma), smin), smax);
      }
      std::swap(pb.x, pb.xt);
      std::swap(pb.F, pb.Ft);
      f = fn;
      hist.push_back(f);
      ++k;
    }
  }
  *iters += k;
  *evals += ne;
  *fout = f;
  return FVIM_OK;
}

// ------------------------------------------------------ Newton-Krylov
static int krylov_dim(const fvim_ep_opts* o) { return o->krylov_dim > 0 ? o->krylov_dim : 20; }

// coupling = 2: Algorithm 1 hands over to the outer Newton-Krylov coupling
// once the passes it still needs, extrapolated from the error's rate over
// the last SWITCH_WINDOW passes, exceed SWITCH_LEFT (about what the Newton
// phase costs in passes); checked from pass SWITCH_FIRST on
constexpr int SWITCH_FIRST = 20, SWITCH_WINDOW = 10;
constexpr double SWITCH_LEFT = 100.0;
// outer Newton-Krylov: Krylov steps per Newton step, and its workspace
static int coupling_dim(const fvim_ep_opts* o) { return o->coupling_krylov > 0 ? o->coupling_krylov : 10; }
static size_t coupling_count(size_t V, size_t ns, const fvim_ep_opts* o) {
  return 12 * V + 3 * ns + ns * (size_t)(6 + coupling_dim(o) + 1);
}

size_t krylov_footprint(const fvim_grid* g, const fvim_ep_opts* o) {
  if (!o) return 0;
  const size_t V = (size_t)g->nx * g->ny * g->nz, ns = (size_t)g->nx * g->ny;
  size_t b = 0;
  if (o->solver == 2) b += sizeof(double) * (6 * V * (size_t)(krylov_dim(o) + 2) + (size_t)KMAX * (RB + 1));
  if (o->coupling >= 1) b += sizeof(double) * coupling_count(V, ns, o);
  return b;
}

static int kry_ensure(fvim_ctx* c, int m) {
  SolverWork* w = c->sw;
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  if (!w->kry || w->kry_m < m) {
    if (w->kry) {
      hipStreamSynchronize(c->stream);
      hipFree(w->kry);
      w->kry = nullptr;
      w->kry_m = 0;
    }
    const size_t bytes = sizeof(double) * 6 * w->V * (size_t)(m + 2);
    if (hipMalloc((void**)&w->kry, bytes) != hipSuccess) {
      w->kry = nullptr;
      return fail(FVIM_ENOMEM, "Krylov basis allocation failed");
    }
    // the layers below the plastic ones are never written by the iteration;
    // they are read (and their results ignored) by the residual epilogue
    hipError_t e = hipMemsetAsync(w->kry, 0, bytes, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail_hip(e, "Krylov basis");
    w->kry_m = m;
  }
  if (!w->kry_part && hipMalloc((void**)&w->kry_part, sizeof(double) * KMAX * RB) != hipSuccess) {
    w->kry_part = nullptr;
    return fail(FVIM_ENOMEM, "Krylov workspace allocation failed");
  }
  if (!w->kry_hout) {
    if (hipHostMalloc((void**)&w->kry_hout, sizeof(double) * KMAX, hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void**)&w->kry_out, w->kry_hout, 0) != hipSuccess) {
      if (w->kry_hout) hipHostFree(w->kry_hout);
      w->kry_hout = nullptr;
      return fail(FVIM_ENOMEM, "Krylov workspace allocation failed");
    }
  }
  return FVIM_OK;
}

// out[i] = <u_i, x> (weighted, unscaled) over the na active voxels of each
// component, for the first n basis vectors.
static int kdots(fvim_ctx* c, const double* base, int n, const double* x, size_t na, double* out) {
  SolverWork* w = c->sw;
  const int nb = nblocks(na);
  hipLaunchKernelGGL(k_kdot, dim3(nb, (n + 3) / 4), dim3(NT), 0, c->stream, base, n, x, na, w->V, w->lp,
                     (unsigned)c->grid.nz, c->wz, w->kry_part);
  hipLaunchKernelGGL(k_kfinal, dim3(n), dim3(NT), 0, c->stream, w->kry_part, nb, w->kry_out);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail_hip(e, "Krylov scalar products");
  for (int i = 0; i < n; ++i) out[i] = w->kry_hout[i];
  return FVIM_OK;
}

// y = a x + sum_{i<n} coef_i u_i over the active voxels; with norm2, its
// weighted (unscaled) <y, y>.
static int kcomb(fvim_ctx* c, double* y, const double* x, double a, const double* base, int n, const double* coef,
                 size_t na, double* norm2) {
  SolverWork* w = c->sw;
  const int nb = nblocks(na);
  KCoef kc = {};
  for (int i = 0; i < n; ++i) kc.c[i] = coef[i];
  hipLaunchKernelGGL(k_kcomb, dim3(nb), dim3(NT), 0, c->stream, y, x, a, base, n, kc, na, w->V, w->lp,
                     (unsigned)c->grid.nz, c->wz, norm2 ? w->kry_part : nullptr);
  if (!norm2) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FVIM_OK : fail_hip(e, "Krylov combination");
  }
  hipLaunchKernelGGL(k_kfinal, dim3(1), dim3(NT), 0, c->stream, w->kry_part, nb, w->kry_out);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail_hip(e, "Krylov combination");
  *norm2 = w->kry_hout[0];
  return FVIM_OK;
}

// Fo = x - grad_s N[C : y] (no traction), in the context's operator
// precision; y is read in the layers above *zact only.
static int op_minus(fvim_ctx* c, const double* y, const double* x, double* Fo) {
  SolverWork* w = c->sw;
  int nb = 0;
  int rc = operator_apply_resid(c, y, nullptr, x, nullptr, Fo, w->rpart, &nb, w->layers + c->grid.nz);
  if (rc) return rc;
  if (nb > w->rpart_count) return fail(FVIM_EINVAL, "residual partial sums: workspace too small");
  return FVIM_OK;
}

// Inexact Newton on R[d_eps] = 0 from pb.x to |R| <= tol_abs (Sec. 4.3
// names Newton-Krylov with the consistent tangent as the alternative to
// DF-SANE).  With R = d_eps - grad_s M[dT] - grad_s N[C : d_eps_p(d_eps)],
// the Jacobian is J = I - A T, A = grad_s N[C : .] and T the consistent
// tangent of the radial return at the iterate, which vanishes outside the
// plastic voxels.  J delta = -R is solved on the plastic support: with
// y = T delta it reads (I - T A) y = -T R, and then delta = -R + A y.  The
// Krylov vectors thus live in the layers above the deepest plastic one
// (the operator skips the layers below as sources), and each Arnoldi step
// costs one operator application and one tangent.  GMRES without restart,
// at most m Arnoldi steps (classical Gram-Schmidt, repeated once when it
// cancels more than 30 % of the new vector), to the relative residual eta
// of Eisenstat and Walker (1996), choice 2 (gamma 0.9, exponent 2, their
// safeguard, eta <= 0.5 and not below half the final tolerance over |R|);
// then x + alpha delta, alpha halved until |R| falls by the factor
// 1 - 1e-4 alpha (1 - eta).  Residuals are always float64; the operator
// inside the linear solve and in A y uses the context's precision (float32
// in the FP32_REFINED mode: an inexact Jacobian slows the last steps, it
// does not move the root).  evals counts residuals and operator
// applications of the linear solves.
static int newton_krylov(fvim_ctx* c, const fvim_state* s, const fvim_ep_opts* o, PlastBufs& pb, double tol_abs,
                         int max_it, int* iters, int* evals, double* fout) {
  SolverWork* w = c->sw;
  const size_t V = w->V, n6 = 6 * V;
  const int m = krylov_dim(o);
  if (!w->kry || w->kry_m < m || !w->kry_part || !w->kry_hout)
    return fail(FVIM_EINVAL, "Newton-Krylov workspace not reserved");
  double* U = w->kry;
  double* ystar = U + (size_t)(m + 1) * n6;
  int* hz = reinterpret_cast<int*>(w->hsc + NSCAL - 1);      // pinned host word
  double f;
  int rc;
  {
    Fp64Scope f64(c, 1);
    if ((rc = residual(c, s, pb, pb.x, nullptr, 0.0, nullptr, pb.F, &f))) return rc;
  }
  int ne = 1, k = 0;
  double eta = 0.5, fprev = f;
  std::vector<double> H((size_t)(m + 1) * m), gc(m), gs(m), g(m + 1), sv(m + 1), y(m);
  double d[KMAX], coef[KMAX];
  auto h = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  while (std::sqrt(f) > tol_abs && k < max_it) {
    if (k > 0) {
      const double e2 = 0.9 * f / fprev, sg = 0.9 * eta * eta;
      eta = std::min(0.5, sg > 0.1 ? std::max(e2, sg) : e2);
    }
    eta = std::max(eta, 0.5 * tol_abs / std::sqrt(f));
    // layers with plastic voxels at the iterate (its return map was the last)
    hipError_t e = hipMemcpyAsync(hz, w->layers + c->grid.nz, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail_hip(e, "active layers");
    const size_t na = (size_t)std::min(std::max(*hz, 0), c->grid.nz) * w->ns;
    // u_0 = -T R
    e = launch_plastic_tangent(pb.x, pb.F, nullptr, nullptr, s->sigma, s->ep, U, na, V, c->lam, c->mu,
                               c->mat.sigma_y0, c->mat.E_h, c->stream);
    if (e != hipSuccess) return fail_hip(e, "plastic tangent");
    double b2 = 0.0;
    if (na && (rc = kdots(c, U, 1, U, na, &b2))) return rc;
    const double bn = std::sqrt(b2);
    int kd = 0;
    if (bn > 0.0) {
      std::fill(g.begin(), g.end(), 0.0);
      sv[0] = bn;
      g[0] = bn;
      for (int j = 0; j < m; ++j) {
        double* uj = U + (size_t)j * n6;
        double* un = U + (size_t)(j + 1) * n6;
        // W = (I - T A) u_j = u_j - T (u_j - (u_j - A u_j)), into pb.xt
        if ((rc = op_minus(c, uj, uj, pb.Ft))) return rc;
        e = launch_plastic_tangent(pb.x, uj, pb.Ft, uj, s->sigma, s->ep, pb.xt, na, V, c->lam, c->mu,
                                   c->mat.sigma_y0, c->mat.E_h, c->stream);
        if (e != hipSuccess) return fail_hip(e, "plastic tangent");
        ++ne;
        if ((rc = kdots(c, U, j + 1, pb.xt, na, d))) return rc;
        double hh = 0.0;
        for (int i = 0; i <= j; ++i) {
          h(i, j) = d[i] / (sv[i] * sv[j]);
          coef[i] = -h(i, j) / sv[i];
          hh += h(i, j) * h(i, j);
        }
        double n2;
        if ((rc = kcomb(c, un, pb.xt, 1.0 / sv[j], U, j + 1, coef, na, &n2))) return rc;
        // |W / s_j|^2 = sum h^2 + |u_(j+1)|^2 when the basis is orthonormal
        if (std::sqrt(n2) < 0.7 * std::sqrt(hh + n2)) {
          if ((rc = kdots(c, U, j + 1, un, na, d))) return rc;
          for (int i = 0; i <= j; ++i) {
            h(i, j) += d[i] / sv[i];
            coef[i] = -d[i] / (sv[i] * sv[i]);
          }
          if ((rc = kcomb(c, un, un, 1.0, U, j + 1, coef, na, &n2))) return rc;
        }
        sv[j + 1] = std::sqrt(n2);
        h(j + 1, j) = sv[j + 1];
        for (int i = 0; i < j; ++i) {          // earlier rotations on column j
          const double a = h(i, j), b = h(i + 1, j);
          h(i, j) = gc[i] * a + gs[i] * b;
          h(i + 1, j) = -gs[i] * a + gc[i] * b;
        }
        const double a = h(j, j), b = h(j + 1, j), r = std::hypot(a, b);
        gc[j] = r > 0.0 ? a / r : 1.0;
        gs[j] = r > 0.0 ? b / r : 0.0;
        h(j, j) = r;
        h(j + 1, j) = 0.0;
        g[j + 1] = -gs[j] * g[j];
        g[j] = gc[j] * g[j];
        kd = j + 1;
        if (std::fabs(g[j + 1]) <= eta * bn || !(sv[j + 1] > 1e-13 * std::sqrt(hh + n2))) break;
      }
      for (int i = kd - 1; i >= 0; --i) {       // H y = g, upper triangular
        double t = g[i];
        for (int l = i + 1; l < kd; ++l) t -= h(i, l) * y[l];
        if (h(i, i) == 0.0) return fail(FVIM_ENOCONV, "Newton-Krylov: singular Hessenberg matrix");
        y[i] = t / h(i, i);
      }
      for (int i = 0; i < kd; ++i) coef[i] = y[i] / sv[i];
      if ((rc = kcomb(c, ystar, nullptr, 0.0, U, kd, coef, na, nullptr))) return rc;
    }
    // -delta = R - A y (= R where nothing flows)
    const double* mdel = pb.F;
    if (kd > 0) {
      if ((rc = op_minus(c, ystar, pb.F, U))) return rc;
      ++ne;
      mdel = U;
    }
    double alpha = 1.0, fn;
    for (int guard = 0;; ++guard) {
      {
        Fp64Scope f64(c, 1);
        if ((rc = residual(c, s, pb, pb.x, mdel, -alpha, pb.xt, pb.Ft, &fn))) return rc;
      }
      ++ne;
      if (std::sqrt(fn) <= (1.0 - 1e-4 * alpha * (1.0 - eta)) * std::sqrt(f)) break;
      if (guard >= 30) return fail(FVIM_ENOCONV, "Newton-Krylov line search failed");
      alpha *= 0.5;
    }
    std::swap(pb.x, pb.xt);
    std::swap(pb.F, pb.Ft);
    fprev = f;
    f = fn;
    ++k;
  }
  *iters += k;
  *evals += ne;
  *fout = f;
  return FVIM_OK;
}

// Solves R[d_eps] = 0 for the traction increment dT ([3][ny][nx]); on
// return pb.x holds d_eps, pb.dep / pb.dp the plastic increments.  In the
// FP32_REFINED mode the iteration first runs on the float32 operator down to
// a relative residual of 3e-6 (about its rounding floor) and is then
// continued on the float64 operator to the requested tolerance; the
// right-hand side grad_s M[dT] is always formed in float64.  The iteration
// starts from the elastic trial x = M[dT], or, with warm set, from
// x_prev - M[dT_prev] + M[dT], where x_prev and M[dT_prev] are what pb.x and
// pb.b hold from the previous call: the plastic part of the previous solution
// is kept and only the elastic part follows the new traction.  The residual
// target is tol_rel |M[dT]|.
static int plasticity(fvim_ctx* c, const double* dT, const fvim_state* s, const fvim_ep_opts* o, double tol_rel,
                      bool warm, PlastBufs& pb, int* iters, int* evals, double* res) {
  SolverWork* w = c->sw;
  const size_t n6 = 6 * w->V;
  hipStream_t st = c->stream;
  int rc;
  pb.dT = dT;
  if (warm) axpy(c, pb.x, pb.x, -1.0, pb.b, n6);
  {
    Fp64Scope f64(c, 1);
    rc = operator_apply(c, nullptr, dT, pb.b, nullptr, nullptr, nullptr);
  }
  if (rc) return rc;
  double d3[3];
  if ((rc = wdots(c, pb.b, nullptr, pb.b, nullptr, d3))) return rc;
  const double bn = std::max(std::sqrt(d3[0]), 1e-300);
  const double tol_abs = tol_rel * bn;
  hipError_t e = hipSuccess;
  if (warm) axpy(c, pb.x, pb.x, 1.0, pb.b, n6);
  else e = hipMemcpyAsync(pb.x, pb.b, sizeof(double) * n6, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return fail_hip(e, "copy");
  *iters = 0;
  *evals = 0;
  double f = 0.0;
  const bool mixed = c->precision == FVIM_FP32_REFINED;
  const double tol32 = 3e-6 * bn;
  if (o->solver == 2) {
    if ((rc = newton_krylov(c, s, o, pb, tol_abs, o->max_plastic, iters, evals, &f))) return rc;
  } else {
    // an inexact solve (target above tol_plastic) at or above the float32
    // floor stays in float32; every other solve ends on the float64 operator
    const bool only32 = mixed && tol_rel > o->tol_plastic && tol_abs >= tol32;
    if (mixed && (tol32 > tol_abs || only32)) {
      if ((rc = fixed_point(c, s, o, pb, std::max(tol32, tol_abs), o->max_plastic, iters, evals, &f))) return rc;
    }
    if (!only32) {
      Fp64Scope f64(c, mixed ? 1 : c->force_fp64);
      if ((rc = fixed_point(c, s, o, pb, tol_abs, o->max_plastic, iters, evals, &f))) return rc;
    }
  }
  // plastic increments of the accepted iterate
  e = launch_return_map(pb.x, s->sigma, s->ep, pb.dep, pb.dp, nullptr, w->V, c->lam, c->mu, c->mat.sigma_y0,
                        c->mat.E_h, st);
  if (e != hipSuccess) return fail_hip(e, "return map");
  dep_written_everywhere(c);
  *res = std::sqrt(f);
  if (std::sqrt(f) > tol_abs) return fail(FVIM_ENOCONV, "plasticity: iteration limit reached");
  return FVIM_OK;
}

// |a - b|_2 and |a|_2 of surface arrays (b may be NULL)
static int surf_norms(fvim_ctx* c, const double* a, const double* b, double* dnorm, double* anorm) {
  SolverWork* w = c->sw;
  const int nb = nblocks(w->ns);
  hipLaunchKernelGGL(k_sq2, dim3(nb), dim3(NT), 0, c->stream, a, b, w->ns, w->part);
  hipLaunchKernelGGL(k_pk_final, dim3(1), dim3(NT), 0, c->stream, 6, w->part, nb, w->sc, w->dmap);
  int rc = read_scalars(c, S_DOT0, 2);
  if (rc) return rc;
  *dnorm = std::sqrt(w->hsc[S_DOT0]);
  *anorm = std::sqrt(w->hsc[S_DOT1]);
  return FVIM_OK;
}

static int aa_ensure(fvim_ctx* c) {
  SolverWork* w = c->sw;
  if (w->aa) return FVIM_OK;
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  const int K = aa_nsums(AA_MMAX);
  if (hipMalloc((void**)&w->aa, sizeof(double) * w->ns * (2 * AA_MMAX + 3)) != hipSuccess ||
      hipMalloc((void**)&w->aa_part, sizeof(double) * K * RB) != hipSuccess ||
      hipHostMalloc((void**)&w->aa_hout, sizeof(double) * K, hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess ||
      hipHostGetDevicePointer((void**)&w->aa_out, w->aa_hout, 0) != hipSuccess)
    return fail(FVIM_ENOMEM, "Anderson history allocation failed");
  return FVIM_OK;
}

// Gram sums of the first m residual differences and f, copied to the host.
static int aa_gram(fvim_ctx* c, int m, const double* f) {
  SolverWork* w = c->sw;
  hipStream_t st = c->stream;
  const int nb = nblocks(w->ns);
  const double* dF = w->aa + (size_t)AA_MMAX * w->ns;
#define FVIM_AA_GRAM(M) hipLaunchKernelGGL(k_aa_gram<M>, dim3(nb), dim3(NT), 0, st, dF, f, w->ns, w->aa_part)
  switch (m) {
    case 1: FVIM_AA_GRAM(1); break;
    case 2: FVIM_AA_GRAM(2); break;
    case 3: FVIM_AA_GRAM(3); break;
    case 4: FVIM_AA_GRAM(4); break;
    case 5: FVIM_AA_GRAM(5); break;
    case 6: FVIM_AA_GRAM(6); break;
    default: return fail(FVIM_EINVAL, "Anderson depth out of range");
  }
#undef FVIM_AA_GRAM
  const int K = aa_nsums(m);
  hipLaunchKernelGGL(k_aa_final, dim3(1), dim3(64), 0, st, w->aa_part, K, nb, w->aa_out);
  hipError_t e = hipStreamSynchronize(st);
  return e == hipSuccess ? FVIM_OK : fail_hip(e, "Anderson Gram matrix");
}

// Least-squares weights: (G + 1e-12 max G_jj I) g = r by Cholesky, G_jl =
// <dF_j, dF_l>, r_j = <dF_j, f>.  False when the differences are close to
// linearly dependent (a pivot below 1e-10 of the largest diagonal), in
// which case the caller drops the history.
static bool aa_solve(int m, const double* sums, double* g) {
  double G[AA_MMAX][AA_MMAX], L[AA_MMAX][AA_MMAX] = {}, r[AA_MMAX], y[AA_MMAX];
  int k = 0;
  for (int j = 0; j < m; ++j)
    for (int l = j; l < m; ++l) G[j][l] = G[l][j] = sums[k++];
  for (int j = 0; j < m; ++j) r[j] = sums[k++];
  double dmax = 0.0;
  for (int j = 0; j < m; ++j) dmax = std::max(dmax, G[j][j]);
  if (!(dmax > 0.0) || !std::isfinite(dmax)) return false;
  for (int j = 0; j < m; ++j) G[j][j] += 1e-12 * dmax;
  for (int j = 0; j < m; ++j) {
    double d = G[j][j];
    for (int p = 0; p < j; ++p) d -= L[j][p] * L[j][p];
    if (!(d > 1e-10 * dmax)) return false;
    L[j][j] = std::sqrt(d);
    for (int i = j + 1; i < m; ++i) {
      double t = G[i][j];
      for (int p = 0; p < j; ++p) t -= L[i][p] * L[j][p];
      L[i][j] = t / L[j][j];
    }
  }
  for (int j = 0; j < m; ++j) {
    double t = r[j];
    for (int p = 0; p < j; ++p) t -= L[j][p] * y[p];
    y[j] = t / L[j][j];
  }
  for (int j = m - 1; j >= 0; --j) {
    double t = y[j];
    for (int p = j + 1; p < m; ++p) t -= L[p][j] * g[p];
    g[j] = t / L[j][j];
  }
  return true;
}

// ------------------------------------------------ outer Newton-Krylov
// Algorithm 1's fixed point solved by Newton's method (coupling = 1): with
// G(x) the surface displacement of N[C : d_eps_p] that one pass (contact on
// H0 - x, friction, plasticity) produces, F(x) = G(x) - x = 0 is solved by
// GMRES on (J_G - I) d = -F, the products J_G v formed by forward
// differences of G from the pass at x (Jacobian-free Newton-Krylov, Knoll
// and Keyes 2004), the step halved until |F| decreases.  Every pass solves
// to the full tolerances and starts from the pass at the current x (its
// pressure, traction and strain), so a difference pass starts next to its
// solution.  The stopping test is Algorithm 1's, |G(x) - x| / |H0| <
// tol_outer, and the state is committed from the pass at the final x.

static int cpl_ensure(fvim_ctx* c, const fvim_ep_opts* o) {
  SolverWork* w = c->sw;
  const size_t need = coupling_count(w->V, w->ns, o);
  if (w->cpl_count >= need) return FVIM_OK;
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  if (w->cpl) {
    hipStreamSynchronize(c->stream);
    hipFree(w->cpl);
    w->cpl = nullptr;
  }
  if (hipMalloc((void**)&w->cpl, sizeof(double) * need) != hipSuccess) {
    w->cpl_count = 0;
    return fail(FVIM_ENOMEM, "outer Newton-Krylov workspace allocation failed");
  }
  w->cpl_count = need;
  return FVIM_OK;
}

// a.b, |a|, |b| of surface arrays
static int sdot(fvim_ctx* c, const double* a, const double* b, double out[3]) {
  SolverWork* w = c->sw;
  const int nb = nblocks(w->ns);
  hipLaunchKernelGGL(k_sdot3, dim3(nb), dim3(NT), 0, c->stream, a, b, w->ns, w->part);
  hipLaunchKernelGGL(k_pk_final, dim3(1), dim3(NT), 0, c->stream, 6, w->part, nb, w->sc, w->dmap);
  int rc = read_scalars(c, S_DOT0, 3);
  if (rc) return rc;
  out[0] = w->hsc[S_DOT0];
  out[1] = std::sqrt(w->hsc[S_DOT1]);
  out[2] = std::sqrt(w->hsc[S_DOT2]);
  return FVIM_OK;
}

// Alternations of the coupled normal-tangential contact step (each one a
// normal and a tangential solve); the coupling contracts fast (the cross
// compliance is a fraction (1 - 2 nu) / (2 - 2 nu) of the normal one).
constexpr int CERRUTI_MAX = 200;
// Cohesive-set updates of the adhesive contact step.
constexpr int ADH_MAX = 200;
static int adhesion_solve(fvim_ctx* c, const double* h, double W, double sigma0, double h0, double tol,
                          int max_contact, int max_iter, double* p, double* gap_out, fvim_adhesive_info* info);
static int adh_ensure(fvim_ctx* c);

// The contact step of one outer pass on the surface H under the load Wn:
// the pressure into T[2] (warm-started from what it holds) and, with
// friction, the tangential traction into T[0], T[1]: Goodman's sequence
// (the normal solve, then the tangential one under its pressure) or, with
// o->cerruti, the alternation coupled through the Boussinesq-Cerruti cross
// terms.  warm: T[0], T[1] hold the previous pass's tangential traction.
static int contact_step(fvim_ctx* c, const fvim_ep_opts* o, const double* H, double Wn, double* T, bool warm,
                        double tol_f, fvim_ep_info& inf) {
  const size_t n = c->sw->ns;
  const double Qx = o->q_ratio[0] * o->mu_f * Wn, Qy = o->q_ratio[1] * o->mu_f * Wn;
  int rc;
  if (o->adh_sigma0 > 0) {
    // the total traction of the adhesive contact (no tangential part)
    fvim_adhesive_info ai{};
    hipError_t e = hipMemsetAsync(T, 0, sizeof(double) * 2 * n, c->stream);
    if (e != hipSuccess) return fail_hip(e, "contact step");
    rc = adhesion_solve(c, H, Wn, o->adh_sigma0, o->adh_h0, o->tol_contact, o->max_contact, ADH_MAX, T + 2 * n,
                        nullptr, &ai);
    if (rc) return rc;
    inf.contact_iters += ai.contact_iters;
    inf.kkt = ai.kkt_residual;
    return FVIM_OK;
  }
  if (o->cerruti && o->mu_f > 0 && Wn > 0) {
    // the normal solves to a tenth of the alternation's tolerance (not below
    // 1e-15), as frictional_contact_solve does: solved only to that
    // tolerance, their pressure changes by about it between alternations
    fvim_frictional_info fi{};
    const double tc = std::min(o->tol_contact, std::max(0.1 * tol_f, 1e-15));
    rc = frictional_solve(c, H, Wn, o->mu_f, Qx, Qy, 1, tol_f, tc, tol_f, o->max_contact, CERRUTI_MAX, T, warm, &fi);
    if (rc) return rc;
    inf.contact_iters += fi.contact_iters + fi.tangential_iters;
    inf.kkt = fi.kkt_residual;
    return FVIM_OK;
  }
  double* pcur = T + 2 * n;
  fvim_contact_info ci;
  rc = pk_solve(c, H, Wn, o->tol_contact, o->max_contact, pcur, nullptr, &ci);
  if (rc) return rc;
  inf.contact_iters += ci.iters;
  inf.kkt = ci.kkt_residual;
  if (o->mu_f > 0 && Wn > 0) {
    fvim_tangential_info fi;
    rc = friction_solve(c, pcur, o->mu_f, Qx, Qy, tol_f, o->max_contact, T, &fi, warm);
    if (rc) return rc;
    inf.contact_iters += fi.iters;
  }
  return FVIM_OK;
}

struct PassBufs {
  const double* H0;
  double* H;          // modified surface of the pass
  double* T;          // traction [3][ns] (the pressure is T + 2 ns)
  double* dT;         // traction increment [3][ns]
  double Wn;
};

// One pass of Algorithm 1 at the surface correction x: G(x) into dU.  warm:
// the contact, friction and plasticity iterations start from what the
// buffers hold (else the plasticity starts from the elastic trial).
static int pass_map(fvim_ctx* c, const fvim_state* s, const fvim_ep_opts* o, PlastBufs& pb, PassBufs& q,
                    const double* x, double* dU, bool warm, fvim_ep_info& inf) {
  SolverWork* w = c->sw;
  const size_t n = w->ns;
  axpy(c, q.H, q.H0, -1.0, x, n);                       // H = H0 - x
  int rc = contact_step(c, o, q.H, q.Wn, q.T, warm, std::max(o->tol_contact, 1e-13), inf);
  if (rc) return rc;
  axpy(c, q.dT, q.T, -1.0, s->traction, 3 * n);           // dT = T - T_n
  int it, ne;
  double res;
  rc = plasticity(c, q.dT, s, o, o->tol_plastic, warm, pb, &it, &ne, &res);
  if (rc) return rc;
  inf.plastic_iters += it;
  inf.r_evals += ne;
  inf.plastic_res = res;
  Fp64Scope f64(c, 1);                                  // surface correction in float64
  return operator_apply(c, pb.dep, nullptr, nullptr, nullptr, nullptr, dU);
}

// One load step by outer Newton-Krylov.  On return dU holds G(x) of the
// final pass and pb, T its state (for the commit); inf.outer_iters counts
// Newton steps, inf.outer_err is |G(x) - x| / |H0|.  *conv: converged.
static int outer_newton(fvim_ctx* c, const fvim_state* s, const fvim_ep_opts* o, PlastBufs& pb, PassBufs& q,
                        double hn, const double* x0, double* dU, fvim_ep_info& inf, bool* conv) {
  SolverWork* w = c->sw;
  const size_t n = w->ns, V = w->V, n6 = 6 * V;
  hipStream_t st = c->stream;
  const int m = coupling_dim(o);
  double* bx = w->cpl;                 // base strain and right-hand side of the plasticity solve
  double* bb = bx + n6;
  double* bT = bb + n6;                // base traction [3][n]
  double* x = bT + 3 * n;
  double* Gx = x + n;
  double* F = Gx + n;
  double* d = F + n;
  double* xt = d + n;                  // trial / perturbed point
  double* wv = xt + n;
  double* Vb = wv + n;                 // Krylov basis [m + 1][n]
  hipError_t e;
  auto save_base = [&]() -> int {
    e = hipMemcpyAsync(bx, pb.x, sizeof(double) * n6, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(bb, pb.b, sizeof(double) * n6, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(bT, q.T, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? FVIM_OK : fail_hip(e, "copy");
  };
  auto restore_base = [&]() -> int {
    e = hipMemcpyAsync(pb.x, bx, sizeof(double) * n6, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pb.b, bb, sizeof(double) * n6, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(q.T, bT, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? FVIM_OK : fail_hip(e, "copy");
  };
  // G(x) at x = x0 (warm from the pass that produced x0), else at x = 0
  if (x0) {
    e = hipMemcpyAsync(x, x0, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail_hip(e, "copy");
  } else {
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(NT), 0, st, x, n, 0.0);
  }
  int rc = pass_map(c, s, o, pb, q, x, Gx, x0 != nullptr, inf);
  if (rc) return rc;
  double xn = 0.0;
  if (x0) {
    double xx[3];
    if ((rc = sdot(c, x, x, xx))) return rc;
    xn = xx[1];
  }
  axpy(c, F, Gx, -1.0, x, n);
  double t3[3];
  if ((rc = sdot(c, F, Gx, t3))) return rc;
  double fn = t3[1], gn = t3[2];
  *conv = fn / hn < o->tol_outer;
  int k = 0;
  const double fd_rel = 3e-7;
  // Forcing term eta of the inexact Newton steps (Eisenstat and Walker 1996,
  // their second choice: eta = 0.9 (|F_k| / |F_k-1|)^2, kept at least
  // 0.9 eta_prev^2 when that exceeds 0.1), between 1e-3 (about the accuracy
  // of a forward-difference product) and 0.5, and no smaller than the outer
  // tolerance asks for at the last steps.
  double eta = 0.5, fprev = fn;
  while (!*conv && k < o->max_outer) {
    if (k > 0) {
      const double r = fn / fprev;
      double en = 0.9 * r * r;
      const double sg = 0.9 * eta * eta;
      if (sg > 0.1) en = std::max(en, sg);
      eta = std::min(0.5, std::max(1e-3, en));
    }
    eta = std::min(0.5, std::max(eta, 0.5 * o->tol_outer * hn / fn));
    if ((rc = save_base())) return rc;
    // GMRES on (J_G - I) d = -F from d = 0, classical Gram-Schmidt applied
    // twice, Givens rotations on the host; relative tolerance eta
    std::vector<double> Hh((size_t)(m + 1) * m, 0.0), cs(m, 0.0), sn(m, 0.0), gv(m + 1, 0.0);
    gv[0] = fn;
    // v_0 = -F / |F| (the right-hand side -F = |F| v_0)
    hipLaunchKernelGGL(k_axpy, dim3(nblocks(n)), dim3(NT), 0, st, Vb, F, -1.0 / fn - 1.0, F, n);
    int j = 0;
    const double hs_scale = fd_rel * std::max(xn, gn);
    for (; j < m; ++j) {
      double* vj = Vb + (size_t)j * n;
      double* vn = Vb + (size_t)(j + 1) * n;
      // w = (G(x + h v_j) - G(x)) / h - v_j, |v_j| = 1
      const double hs = hs_scale > 0 ? hs_scale : fd_rel;
      hipLaunchKernelGGL(k_axpy, dim3(nblocks(n)), dim3(NT), 0, st, xt, x, hs, vj, n);
      if ((rc = restore_base())) return rc;
      if ((rc = pass_map(c, s, o, pb, q, xt, wv, true, inf))) return rc;
      hipLaunchKernelGGL(k_axpy, dim3(nblocks(n)), dim3(NT), 0, st, wv, wv, -1.0, Gx, n);   // G - G(x)
      hipLaunchKernelGGL(k_axpy, dim3(nblocks(n)), dim3(NT), 0, st, wv, vj, 1.0 / hs, wv, n); // v + (G - G(x)) / h
      hipLaunchKernelGGL(k_axpy, dim3(nblocks(n)), dim3(NT), 0, st, wv, wv, -2.0, vj, n);     // (G - G(x)) / h - v
      // modified Gram-Schmidt, applied twice
      for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i <= j; ++i) {
          double dd[3];
          if ((rc = sdot(c, wv, Vb + (size_t)i * n, dd))) return rc;
          Hh[(size_t)i * m + j] += dd[0];
          hipLaunchKernelGGL(k_axpy, dim3(nblocks(n)), dim3(NT), 0, st, wv, wv, -dd[0], Vb + (size_t)i * n, n);
        }
      }
      double dd[3];
      if ((rc = sdot(c, wv, wv, dd))) return rc;
      const double hnext = dd[1];
      Hh[(size_t)(j + 1) * m + j] = hnext;
      // Givens rotations on column j
      for (int i = 0; i < j; ++i) {
        const double a = Hh[(size_t)i * m + j], b = Hh[(size_t)(i + 1) * m + j];
        Hh[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
        Hh[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
      }
      const double a = Hh[(size_t)j * m + j], b = Hh[(size_t)(j + 1) * m + j];
      const double r = std::hypot(a, b);
      cs[j] = r > 0 ? a / r : 1.0;
      sn[j] = r > 0 ? b / r : 0.0;
      Hh[(size_t)j * m + j] = r;
      Hh[(size_t)(j + 1) * m + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      const bool done = std::fabs(gv[j + 1]) <= eta * fn || !(hnext > 1e-14 * fn);
      if (!done) hipLaunchKernelGGL(k_axpy, dim3(nblocks(n)), dim3(NT), 0, st, vn, wv, 1.0 / hnext - 1.0, wv, n);
      if (done) {
        ++j;
        break;
      }
    }
    // d = sum y_i v_i with R y = g (back substitution): the least-squares
    // solution of (J_G - I) d = -F over the Krylov space
    std::vector<double> y(j, 0.0);
    for (int i = j - 1; i >= 0; --i) {
      double t = gv[i];
      for (int l = i + 1; l < j; ++l) t -= Hh[(size_t)i * m + l] * y[l];
      y[i] = t / Hh[(size_t)i * m + i];
    }
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(NT), 0, st, d, n, 0.0);
    for (int i = 0; i < j; ++i)
      hipLaunchKernelGGL(k_axpy, dim3(nblocks(n)), dim3(NT), 0, st, d, d, y[i], Vb + (size_t)i * n, n);
    // backtracking on |F|
    double alpha = 1.0, fnew = 0.0;
    for (;;) {
      hipLaunchKernelGGL(k_axpy, dim3(nblocks(n)), dim3(NT), 0, st, xt, x, alpha, d, n);
      if ((rc = restore_base())) return rc;
      if ((rc = pass_map(c, s, o, pb, q, xt, dU, true, inf))) return rc;
      axpy(c, wv, dU, -1.0, xt, n);
      double f3[3];
      if ((rc = sdot(c, wv, dU, f3))) return rc;
      fnew = f3[1];
      if (fnew <= (1.0 - 1e-4 * alpha) * fn || alpha < 1e-3) {
        gn = f3[2];
        break;
      }
      alpha *= 0.5;
    }
    e = hipMemcpyAsync(x, xt, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(Gx, dU, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(F, wv, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail_hip(e, "copy");
    double xx[3];
    if ((rc = sdot(c, x, x, xx))) return rc;
    xn = xx[1];
    fprev = fn;
    fn = fnew;
    ++k;
    *conv = fn / hn < o->tol_outer;
  }
  e = hipMemcpyAsync(dU, Gx, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return fail_hip(e, "copy");
  inf.outer_iters = k;
  inf.outer_err = fn / hn;
  return FVIM_OK;
}

static int adh_ensure(fvim_ctx* c) {
  SolverWork* w = c->sw;
  if (w->adh) return FVIM_OK;
  std::lock_guard<std::recursive_mutex> lk(device_lock());
  if (hipMalloc((void**)&w->adh, sizeof(double) * 5 * w->ns) != hipSuccess ||
      hipMalloc((void**)&w->adh_cnt, 2 * sizeof(unsigned long long)) != hipSuccess ||
      hipHostMalloc((void**)&w->adh_hcnt, 2 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
    if (w->adh) hipFree(w->adh);
    if (w->adh_cnt) hipFree(w->adh_cnt);
    w->adh = nullptr;
    w->adh_cnt = nullptr;
    w->adh_hcnt = nullptr;
    return fail(FVIM_ENOMEM, "adhesive contact workspace allocation failed");
  }
  return FVIM_OK;
}

// Adhesive contact (Dugdale cohesive zone of stress sigma0 and range h0):
// the cohesive set C by fixed point from C = {} -- the frictionless contact
// on h + sigma0 M[1_C] under W + sigma0 dA |C| (Polonsky-Keer, warm-started
// from the previous solve), then C <- {gap <= h0} -- until the set repeats;
// p = p_c - sigma0 1_C.  gap_out may be NULL.
static int adhesion_solve(fvim_ctx* c, const double* h, double W, double sigma0, double h0, double tol,
                          int max_contact, int max_iter, double* p, double* gap_out, fvim_adhesive_info* info) {
  if (!std::isfinite(W) || !(sigma0 >= 0) || !std::isfinite(sigma0) || !(h0 >= 0) || !std::isfinite(h0) ||
      !(tol > 0) || max_iter < 1 || max_contact < 1)
    return fail(FVIM_EINVAL, "adhesive_contact_solve: bad arguments");
  int rc = sw_ensure(c);
  if (rc) return rc;
  if ((rc = adh_ensure(c))) return rc;
  SolverWork* w = c->sw;
  hipStream_t st = c->stream;
  const size_t n = w->ns;
  const int nb = nblocks(n);
  const double dA = c->grid.lx * c->grid.ly / (double)n;
  double* C = w->adh;
  double* pc = C + n;
  double* h2 = pc + n;
  double* u = h2 + n;
  double* gp = u + n;
  hipError_t e = hipMemsetAsync(C, 0, sizeof(double) * 2 * n, st);   // C = {}, p_c = 0 (uniform start)
  if (e != hipSuccess) return fail_hip(e, "adhesive_contact_solve");
  unsigned long long members = 0;
  int k = 0, cit = 0;
  bool conv = false;
  fvim_contact_info ci{};
  for (k = 1; k <= max_iter; ++k) {
    const double* hk = h;
    if (members > 0) {
      if ((rc = compliance(c, C, u, st))) return rc;
      hipLaunchKernelGGL(k_adh_surface, dim3(nb), dim3(NT), 0, st, h, u, sigma0, h2, n);
      hk = h2;
    }
    const double W2 = W + sigma0 * dA * (double)members;
    if (!(W2 > 0)) return fail(FVIM_EINVAL, "adhesive_contact_solve: the repulsive load W + sigma0 dA |C| must be positive");
    if ((rc = pk_solve(c, hk, W2, tol, max_contact, pc, gp, &ci))) return rc;
    cit += ci.iters;
    e = hipMemsetAsync(w->adh_cnt, 0, 2 * sizeof(unsigned long long), st);
    if (e != hipSuccess) return fail_hip(e, "adhesive_contact_solve");
    hipLaunchKernelGGL(k_adh_set, dim3(nb), dim3(NT), 0, st, gp, h0, C, n, w->adh_cnt);
    {
      std::lock_guard<std::recursive_mutex> lk(device_lock());     // pinned copy
      e = hipMemcpyAsync(w->adh_hcnt, w->adh_cnt, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (e != hipSuccess) return fail_hip(e, "adhesive_contact_solve");
    const unsigned long long changed = w->adh_hcnt[0];
    members = w->adh_hcnt[1];
    if (changed == 0) {
      conv = true;
      break;
    }
  }
  if (k > max_iter) k = max_iter;
  hipLaunchKernelGGL(k_adh_total, dim3(nb), dim3(NT), 0, st, pc, C, sigma0, p, n);
  if (gap_out && (e = hipMemcpyAsync(gap_out, gp, sizeof(double) * n, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return fail_hip(e, "adhesive_contact_solve");
  if (info) {
    info->iters = k;
    info->contact_iters = cit;
    info->cohesive_fraction = (double)members / (double)n;
    info->contact_fraction = ci.contact_fraction;
    info->adhesive_force = sigma0 * dA * (double)members;
    info->kkt_residual = ci.kkt_residual;
  }
  if (!conv) return fail(FVIM_ENOCONV, "adhesive_contact_solve: the cohesive set did not settle");
  return FVIM_OK;
}

}  // namespace fvim

using namespace fvim;

extern "C" {

int contact_solve(fvim_ctx* c, const double* h, double W, double tol, int max_iter, double* p, double* gap,
                  fvim_contact_info* info) {
  if (!c || !h || !p) return fail(FVIM_EINVAL, "NULL argument");
  if (!(W > 0) || !std::isfinite(W)) return fail(FVIM_EINVAL, "contact_solve: W must be positive and finite");
  if (!(tol > 0) || max_iter < 1) return fail(FVIM_EINVAL, "contact_solve: need tol > 0 and max_iter >= 1");
  return pk_solve(c, h, W, tol, max_iter, p, gap, info);
}

int adhesive_contact_solve(fvim_ctx* c, const double* h, double W, double sigma0, double h0, double tol,
                           int max_iter, double* p, double* gap, fvim_adhesive_info* info) {
  if (!c || !h || !p) return fail(FVIM_EINVAL, "NULL argument");
  if (info) *info = fvim_adhesive_info{};
  return adhesion_solve(c, h, W, sigma0, h0, tol, 100000, max_iter, p, gap, info);
}

int elastoplastic_solve(fvim_ctx* c, const double* h, const double* W_steps, int n_steps, const fvim_ep_opts* o,
                        fvim_state* s, fvim_ep_info* info) {
  if (!c || !h || !W_steps || !o || !s || !info) return fail(FVIM_EINVAL, "NULL argument");
  if (!s->eps_p || !s->ep || !s->sigma || !s->traction || !s->u3p) return fail(FVIM_EINVAL, "NULL state field");
  if (n_steps < 1 || !(o->relax > 0 && o->relax <= 1) || o->max_outer < 1 || o->anderson_m < 0 ||
      o->coupling < 0 || o->coupling > 2 || o->coupling_krylov < 0 || o->coupling_krylov > 30 ||
      o->anderson_m > AA_MMAX || !(o->inner_rel >= 0) || o->solver < 0 || o->solver > 2 || o->krylov_dim < 0 ||
      o->krylov_dim > KMAX - 2 || !(o->mu_f >= 0) || !std::isfinite(o->mu_f) ||
      (o->mu_f > 0 && !(std::hypot(o->q_ratio[0], o->q_ratio[1]) < 1.0)) || o->cerruti < 0 || o->cerruti > 1 ||
      !(o->adh_sigma0 >= 0) || !std::isfinite(o->adh_sigma0) || !(o->adh_h0 >= 0) || !std::isfinite(o->adh_h0) ||
      (o->adh_sigma0 > 0 && o->mu_f > 0))
    return fail(FVIM_EINVAL, "elastoplastic_solve: bad options");
  int rc = sw_ensure(c);
  if (rc) return rc;
  PlastBufs pb;
  if ((rc = vol_ensure(c, pb))) return rc;
  SolverWork* w = c->sw;
  hipStream_t st = c->stream;
  const size_t n = w->ns, V = w->V;
  // surface work arrays (after the 5 used by the contact solver)
  double* H0 = w->surf + 5 * n;
  double* H = w->surf + 6 * n;
  double* dUp = w->surf + 7 * n;
  double* dU = w->surf + 8 * n;
  double* T = w->surf + 9 * n;        // 3 planes: 9, 10, 11
  double* pcur = T + 2 * n;           // normal component of T
  double* dT = w->surf + 12 * n;      // 3 planes: 12, 13, 14
  const int aam = o->literal_alg1 ? 0 : o->anderson_m;
  if (aam > 0 && (rc = aa_ensure(c))) return rc;
  if (o->solver == 2 && (rc = kry_ensure(c, krylov_dim(o)))) return rc;
  if (o->mu_f > 0 && (rc = friction_reserve(c))) return rc;
  if (o->adh_sigma0 > 0 && (rc = adh_ensure(c))) return rc;
  if (o->coupling >= 1 && (rc = cpl_ensure(c, o))) return rc;
  // every buffer the operator applications of the solve use, sized now: no
  // device memory is freed or allocated while the solve runs
  if ((rc = operator_reserve(c, pb.dep, dT, pb.F))) return rc;
  // Anderson history: differences of the iterates and of the residuals
  double* aX = aam ? w->aa : nullptr;
  double* aF = aam ? w->aa + (size_t)AA_MMAX * n : nullptr;
  double* xprev = aam ? aF + (size_t)AA_MMAX * n : nullptr;
  double* fprev = aam ? xprev + n : nullptr;
  double* fres = aam ? fprev + n : nullptr;
  auto cleanup = [&](int r) {
    hipStreamSynchronize(st);
    return r;
  };
  hipError_t e;
  memset(info, 0, sizeof(fvim_ep_info) * (size_t)n_steps);
  for (int step = 0; step < n_steps; ++step) {
    const double Wn = W_steps[step];
    fvim_ep_info& inf = info[step];
    axpy(c, H0, h, -1.0, s->u3p, n);                      // H0 = h - U3p
    double dn, hn;
    if ((rc = surf_norms(c, H0, nullptr, &dn, &hn))) return cleanup(rc);
    if (hn == 0.0) hn = 1.0;
    e = hipMemcpyAsync(H, H0, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(dUp, 0, sizeof(double) * n, st);
    if (e == hipSuccess) e = hipMemsetAsync(T, 0, sizeof(double) * 2 * n, st);
    // warm start of the pressure: the previous step's normal traction
    if (e == hipSuccess) e = hipMemcpyAsync(pcur, s->traction + 2 * n, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return cleanup(fail_hip(e, "step setup"));
    double err = INFINITY, err_prev = 1.0;
    bool conv = false;
    int k;
    int aa_count = 0, aa_head = 0;
    if (o->coupling == 1) {
      PassBufs q{H0, H, T, dT, Wn};
      rc = outer_newton(c, s, o, pb, q, hn, nullptr, dU, inf, &conv);
      if (rc) return cleanup(rc);
      if (!conv) return cleanup(fail(FVIM_ENOCONV, "outer Newton-Krylov: iteration limit reached"));
    }
    // passes of the alternation (none with coupling = 1)
    const int kmax = o->coupling == 1 ? 0 : o->max_outer;
    std::vector<double> errs;
    bool to_newton = false;
    for (k = 1; k <= kmax; ++k) {
      // inexact inner solves (plasticity, and the tangential contact with
      // friction) while the outer error is large; a pass that may end the
      // step is always solved to the full tolerances
      const bool loose = o->inner_rel > 0 && !(err_prev < o->tol_outer);
      const double tol_f_full = std::max(o->tol_contact, 1e-13);
      double tol_f = tol_f_full;
      if (o->mu_f > 0 && Wn > 0 && loose) tol_f = std::max(tol_f, o->inner_rel * err_prev);
      // the pressure into T[2]; with friction the tangential traction into
      // T[0], T[1] (from the second pass on, T holds the previous pass's)
      rc = contact_step(c, o, H, Wn, T, k > 1, tol_f, inf);
      if (rc) return cleanup(rc);
      axpy(c, dT, T, -1.0, s->traction, 3 * n);           // dT = T - T_n
      double tol_rel = o->tol_plastic;
      if (loose) tol_rel = std::max(tol_rel, o->inner_rel * err_prev);
      const bool exact = tol_rel == o->tol_plastic && tol_f == tol_f_full;
      int it, ne;
      double res;
      rc = plasticity(c, dT, s, o, tol_rel, o->warm_start && k > 1, pb, &it, &ne, &res);
      if (rc) return cleanup(rc);
      inf.plastic_iters += it;
      inf.r_evals += ne;
      inf.plastic_res = res;
      {
        Fp64Scope f64(c, 1);                              // surface correction in float64
        rc = operator_apply(c, pb.dep, nullptr, nullptr, nullptr, nullptr, dU);   // dU3p
      }
      if (rc) return cleanup(rc);
      double an;
      if ((rc = surf_norms(c, dU, dUp, &dn, &an))) return cleanup(rc);
      err = dn / hn;
      err_prev = err;
      conv = err < o->tol_outer && exact;
      inf.outer_err = err;
      inf.outer_iters = k;
      if (o->coupling == 2 && !conv) {
        errs.push_back(err);
        if (k >= SWITCH_FIRST) {
          const double r = err / errs[errs.size() - 1 - SWITCH_WINDOW];
          const double left = r < 1.0 ? SWITCH_WINDOW * std::log(o->tol_outer / err) / std::log(r) : INFINITY;
          to_newton = left > SWITCH_LEFT;
        }
      }
      if (aam > 0) {
        // x = dUp, f = G(x) - x; history update, least squares, step
        axpy(c, fres, dU, -1.0, dUp, n);
        if (k > 1) {
          axpy(c, aX + (size_t)aa_head * n, dUp, -1.0, xprev, n);
          axpy(c, aF + (size_t)aa_head * n, fres, -1.0, fprev, n);
          aa_head = (aa_head + 1) % aam;
          aa_count = std::min(aa_count + 1, aam);
        }
        e = hipMemcpyAsync(xprev, dUp, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(fprev, fres, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return cleanup(fail_hip(e, "copy"));
        if (conv) break;
        AACoef co = {};
        int me = aa_count;
        if (me > 0) {
          if ((rc = aa_gram(c, me, fres))) return cleanup(rc);
          if (!aa_solve(me, w->aa_hout, co.g)) me = aa_count = aa_head = 0;
        }
        hipLaunchKernelGGL(k_aa_step, dim3(nblocks(n)), dim3(NT), 0, st, dUp, fres, aX, aF, co, me, o->relax, n);
        axpy(c, H, H0, -1.0, dUp, n);                     // H = H0 - x_(k+1)
        if (to_newton) break;
        continue;
      }
      // relaxed surface correction, H = H0 - relaxed
      axpy(c, H, dUp, o->relax, dU, n);                  // H <- dUp + relax dU (temporarily)
      axpy(c, H, H, -o->relax, dUp, n);                  //      - relax dUp
      if (o->literal_alg1) {
        e = hipMemcpyAsync(dUp, dU, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return cleanup(fail_hip(e, "copy"));
      } else {
        e = hipMemcpyAsync(dUp, H, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return cleanup(fail_hip(e, "copy"));
      }
      axpy(c, H, H0, -1.0, H, n);                         // H = H0 - relaxed
      if (conv || to_newton) break;
    }
    if (o->coupling != 1) inf.outer_iters = k > kmax ? kmax : k;
    if (to_newton) {
      // the Newton coupling from the alternation's next iterate (dUp),
      // warm from its last pass; outer_iters counts passes and Newton steps
      const int passes = inf.outer_iters;
      PassBufs q{H0, H, T, dT, Wn};
      rc = outer_newton(c, s, o, pb, q, hn, dUp, dU, inf, &conv);
      if (rc) return cleanup(rc);
      inf.outer_iters += passes;
      if (!conv) return cleanup(fail(FVIM_ENOCONV, "outer Newton-Krylov: iteration limit reached"));
    }
    if (!conv) return cleanup(fail(FVIM_ENOCONV, "Algorithm 1: outer iteration limit reached"));
    // state update: eps_p += d_eps_p, ep += d_ep, sigma <- sigma_(n+1), T_n <- T, U3p += dU
    e = launch_return_map(pb.x, s->sigma, s->ep, pb.dep, pb.dp, s->sigma, V, c->lam, c->mu, c->mat.sigma_y0,
                          c->mat.E_h, st);
    if (e != hipSuccess) return cleanup(fail_hip(e, "return map"));
    dep_written_everywhere(c);
    axpy(c, s->eps_p, s->eps_p, 1.0, pb.dep, 6 * V);
    axpy(c, s->ep, s->ep, 1.0, pb.dp, V);
    e = hipMemcpyAsync(s->traction, T, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return cleanup(fail_hip(e, "copy"));
    axpy(c, s->u3p, s->u3p, 1.0, dU, n);
    inf.committed = 1;
  }
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return cleanup(fail_hip(e, "elastoplastic_solve"));
  return cleanup(FVIM_OK);
}

}  // extern "C"
