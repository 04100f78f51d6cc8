// Pointwise float64 kernels: the J2 radial return (Sec. 4.1) and the vector
// algebra of the iterative solvers.  All are HBM-streaming; each thread
// handles consecutive voxels of one component plane so every access is a
// contiguous run.
#include "common.hpp"
#include "kernels.hpp"

namespace fvim {
namespace {

constexpr int NT = 256;

// Backward-Euler radial return for linear isotropic hardening.  The plastic
// multiplier increment is exact for this law: with f = sigma_eq_trial -
// (sy0 + eh ep_n) > 0, the consistency condition
// sigma_eq_trial - 3 mu d_ep = sy0 + eh (ep_n + d_ep) gives
// d_ep = f / (3 mu + eh), and the flow direction is that of dev sigma_trial.
// The strain increment is de + cf F when F is given (a trial point of the
// plasticity iteration), and is then also stored in xt unless xt is NULL;
// d_ep and sigma_(n+1) are written only where dp and sn1 are given.
__global__ __launch_bounds__(NT) void k_return_map(const double* __restrict__ de, const double* __restrict__ F,
                                                  double cf, double* __restrict__ xt, const double* sn,
                                                  const double* __restrict__ epn, double* __restrict__ dep,
                                                  double* __restrict__ dp, double* sn1, size_t V, double lam,
                                                  double mu, double sy0, double eh, int* __restrict__ flags,
                                                  int lp, const int* __restrict__ zwrite) {
  size_t v = (size_t)blockIdx.x * NT + threadIdx.x;
  if (v >= V) return;
  double e[6], s[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    e[c] = de[c * V + v];
    s[c] = sn[c * V + v];
  }
  if (F) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      e[c] += cf * F[c * V + v];
      if (xt) xt[c * V + v] = e[c];
    }
  }
  const double tre = e[0] + e[1] + e[2];
#pragma unroll
  for (int c = 0; c < 6; ++c) s[c] += 2.0 * mu * e[c] + (c < 3 ? lam * tre : 0.0);
  const double m = (s[0] + s[1] + s[2]) * (1.0 / 3.0);
  double d[6] = {s[0] - m, s[1] - m, s[2] - m, s[3], s[4], s[5]};
  const double nn = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + 2.0 * (d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
  const double seq = sqrt(1.5 * nn);
  const double f = seq - (sy0 + eh * epn[v]);
  double dpv = 0.0, fac = 0.0;
  if (f > 0.0) {
    dpv = f / (3.0 * mu + eh);
    fac = 1.5 * dpv / seq;
  }
  if (dp) dp[v] = dpv;
  if (flags && fac != 0.0) flags[v >> lp] = 1;   // d_eps_p = fac dev(sigma_trial) is not zero
  // with zwrite, dep already holds zeros in the layers >= *zwrite: an elastic
  // voxel there needs no store
  if (zwrite && fac == 0.0 && (int)(v >> lp) >= *zwrite) return;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const double x = fac * d[c];
    dep[c * V + v] = x;
    if (sn1) sn1[c * V + v] = s[c] - 2.0 * mu * x;
  }
}

// Consistent tangent T of the radial return above at the strain increment
// de: out = base - T (u1 - u2) (base, u2 may be NULL), for the voxels
// v < na of each component (component stride V).  With d = dev
// sigma_trial, seq = sqrt(3/2)|d|, d_ep = f / (3 mu + eh) and
// d_eps_p = (3 d_ep / (2 seq)) d, a change u of de changes d by
// dd = 2 mu dev(u), seq by (3/2) <d, dd> / seq and d_ep by that over
// (3 mu + eh); the product rule gives the rest.  The trial state is formed
// with the same operations as the return map, so T is nonzero exactly on
// the voxels the return map at de lets flow.
__global__ __launch_bounds__(NT) void k_plastic_tangent(const double* __restrict__ de, const double* u1,
                                                       const double* u2, const double* base,
                                                       const double* __restrict__ sn, const double* __restrict__ epn,
                                                       double* out, size_t na, size_t V, double lam, double mu,
                                                       double sy0, double eh) {
  size_t v = (size_t)blockIdx.x * NT + threadIdx.x;
  if (v >= na) return;
  double e[6], s[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    e[c] = de[c * V + v];
    s[c] = sn[c * V + v];
  }
  const double tre = e[0] + e[1] + e[2];
#pragma unroll
  for (int c = 0; c < 6; ++c) s[c] += 2.0 * mu * e[c] + (c < 3 ? lam * tre : 0.0);
  const double m = (s[0] + s[1] + s[2]) * (1.0 / 3.0);
  const double d[6] = {s[0] - m, s[1] - m, s[2] - m, s[3], s[4], s[5]};
  const double nn = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + 2.0 * (d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
  const double seq = sqrt(1.5 * nn);
  const double f = seq - (sy0 + eh * epn[v]);
  double b[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) b[c] = base ? base[c * V + v] : 0.0;
  if (!(f > 0.0)) {
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c * V + v] = b[c];
    return;
  }
  double dd[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) dd[c] = u1[c * V + v] - (u2 ? u2[c * V + v] : 0.0);
  const double um = (dd[0] + dd[1] + dd[2]) * (1.0 / 3.0);
#pragma unroll
  for (int c = 0; c < 6; ++c) dd[c] = 2.0 * mu * (c < 3 ? dd[c] - um : dd[c]);
  const double dn = d[0] * dd[0] + d[1] * dd[1] + d[2] * dd[2] + 2.0 * (d[3] * dd[3] + d[4] * dd[4] + d[5] * dd[5]);
  const double dseq = 1.5 * dn / seq;
  const double h = 1.0 / (3.0 * mu + eh);
  const double dp = f * h, ddp = dseq * h;
  const double fac = 1.5 * dp / seq;
  const double dfac = 1.5 * (ddp * seq - dp * dseq) / (seq * seq);
#pragma unroll
  for (int c = 0; c < 6; ++c) out[c * V + v] = b[c] - (dfac * d[c] + fac * dd[c]);
}

// Mean-mode fields in float64 (precision FP32_REFINED).  One thread per
// depth node: sums the block partials of the 6 eigenstrain planes of that
// node (and of the 3 traction planes) in a fixed order, forms the laterally
// uniform response (sigma . e3 = -t_mean, eps13 = (w13 - t1)/(2 mu),
// eps23 = (w23 - t2)/(2 mu), eps33 = (w33 - t3)/(lambda + 2 mu), other
// strains 0, displacement 0) and writes one constant per output plane.
__global__ __launch_bounds__(NT) void k_k0_fields(const double* __restrict__ wsum, int wblocks,
                                                 const double* __restrict__ tsum, int tblocks,
                                                 double* __restrict__ out, DepthParams p) {
  const int z = blockIdx.x * NT + threadIdx.x;
  const int nz = p.nz;
  if (z >= nz) return;
  const double inv = p.norm;                      // 1 / (nx ny)
  const double mu = p.mu, lam = p.kappa * p.mu;
  double e[6] = {0, 0, 0, 0, 0, 0};
  double w[6] = {0, 0, 0, 0, 0, 0};
  if (p.has_w) {
    double ep[6];
    for (int c = 0; c < 6; ++c) {
      double s = 0.0;
      const double* b = wsum + ((size_t)c * nz + z) * wblocks;
      for (int k = 0; k < wblocks; ++k) s += b[k];
      ep[c] = s * inv;
    }
    const double tr = ep[0] + ep[1] + ep[2];
    for (int c = 0; c < 6; ++c) w[c] = 2.0 * mu * ep[c] + (c < 3 ? lam * tr : 0.0);
  }
  double t[3] = {0, 0, 0};
  if (p.has_t && p.k0_include) {
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      const double* b = tsum + (size_t)c * tblocks;
      for (int k = 0; k < tblocks; ++k) s += b[k];
      t[c] = s * inv;
    }
  }
  e[4] = (w[4] - t[0]) / (2.0 * mu);
  e[3] = (w[3] - t[1]) / (2.0 * mu);
  e[2] = (w[2] - t[2]) / (lam + 2.0 * mu);
  if (p.off_strain >= 0)
    for (int c = 0; c < 6; ++c) out[p.off_strain + c * nz + z] = e[c];
  if (p.off_stress >= 0) {
    const double tre = e[0] + e[1] + e[2];
    for (int c = 0; c < 6; ++c) out[p.off_stress + c * nz + z] = 2.0 * mu * e[c] + (c < 3 ? lam * tre : 0.0) - w[c];
  }
  if (p.off_disp >= 0)
    for (int c = 0; c < 3; ++c) out[p.off_disp + c * nz + z] = 0.0;
  if (p.off_u3 >= 0 && z == 0) out[p.off_u3] = 0.0;
}

}  // namespace

hipError_t launch_k0_fields(const double* wsum, int wblocks, const double* tsum, int tblocks, double* out,
                            const DepthParams& p, hipStream_t st) {
  hipLaunchKernelGGL(k_k0_fields, dim3((p.nz + NT - 1) / NT), dim3(NT), 0, st, wsum, wblocks, tsum, tblocks, out,
                     p);
  return hipGetLastError();
}

hipError_t launch_return_map(const double* d_eps, const double* sig_n, const double* ep_n, double* d_eps_p,
                             double* d_ep, double* sig_np1, size_t nvox, double lam, double mu, double sy0,
                             double eh, hipStream_t st) {
  unsigned nb = (unsigned)((nvox + NT - 1) / NT);
  hipLaunchKernelGGL(k_return_map, dim3(nb), dim3(NT), 0, st, d_eps, nullptr, 0.0, nullptr, sig_n, ep_n, d_eps_p,
                     d_ep, sig_np1, nvox, lam, mu, sy0, eh, nullptr, 0, nullptr);
  return hipGetLastError();
}

hipError_t launch_trial_return_map(const double* x, const double* F, double cf, double* xt, const double* sig_n,
                                   const double* ep_n, double* d_eps_p, size_t nvox, double lam, double mu,
                                   double sy0, double eh, hipStream_t st, int* layer_flags, int lp,
                                   const int* zwrite) {
  unsigned nb = (unsigned)((nvox + NT - 1) / NT);
  hipLaunchKernelGGL(k_return_map, dim3(nb), dim3(NT), 0, st, x, F, cf, xt, sig_n, ep_n, d_eps_p, nullptr,
                     nullptr, nvox, lam, mu, sy0, eh, layer_flags, lp, zwrite);
  return hipGetLastError();
}

hipError_t launch_plastic_tangent(const double* d_eps, const double* u1, const double* u2, const double* base,
                                  const double* sig_n, const double* ep_n, double* out, size_t na, size_t nvox,
                                  double lam, double mu, double sy0, double eh, hipStream_t st) {
  if (na == 0) return hipSuccess;
  unsigned nb = (unsigned)((na + NT - 1) / NT);
  hipLaunchKernelGGL(k_plastic_tangent, dim3(nb), dim3(NT), 0, st, d_eps, u1, u2, base, sig_n, ep_n, out, na, nvox,
                     lam, mu, sy0, eh);
  return hipGetLastError();
}

}  // namespace fvim
