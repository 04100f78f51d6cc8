// Per-mode depth pass of the Mindlin + Boussinesq operators (gfx950).
//
// For one in-plane mode exp(i q.x) the response of the half-space to the
// P1-interpolated eigenstress w = C : eps_p (Sec. 3.2) and to a surface
// traction t is the decaying solution of a 1D linear system in the depth
// variable Z = |q| z.  In the frame (n = q/|q|, t = e3 x n, e3) it splits
// into an in-plane part (u_n, u_z, tractions sigma_nz, sigma_zz) and an
// antiplane part (u_t, sigma_tz); quantities with an odd number of n indices
// carry a factor i, so all coefficients are real.  Scaled by 1/mu and with
// a = |q| u_n / i, c = |q| u_z, t1 = sigma_nz / (i mu), t2 = sigma_zz / mu,
// kappa = lambda / mu, omega = w / mu:
//   a'  = -c + t1 + omega_nz/i
//   c'  = (kappa a + t2 + omega_zz) / (kappa + 2)
//   t1' = 4 (kappa+1)/(kappa+2) a - kappa/(kappa+2) (t2 + omega_zz) + omega_nn
//   t2' = t1
// and v = |q| u_t, t3 = sigma_tz / mu:  v' = t3 + omega_tz,  t3' = v - omega_nt/i.
// The in-plane matrix has the Jordan form diag(J(-1), J(+1)) with 2x2 blocks
// J(l) = [[l, 1], [0, l]]; the antiplane one has eigenvalues -1, +1.  So the
// solution is carried by two decaying and two growing modal coordinates
// (plus one of each antiplane):
//   * growing ones vanish below the last node and are integrated upward
//     (a backward scan over depth),
//   * the decaying ones start from the surface condition
//     sigma . e3 = -t at z = 0 (total stress; traction-free surface for the
//     eigenstress part, Sec. 2.1) and are integrated downward (a forward scan).
// Over an element of scaled length s = |q| h the exact propagators are
// exp(-s) [[1, +/-s], [0, 1]] and the P1 load enters through four functions
// of s (G0, G0', H0, H0' below), so the per-mode kernel is built on the fly
// and the depth work is O(nz) with no cutoff.  This is mathematically the
// paper's Green's-function sum (Kelvin part, jump term, Boussinesq image),
// organised as recurrences instead of element-pair integrals.
//
// Threads: LPM lanes per mode, P consecutive depth nodes per lane; the
// recurrences run sequentially inside a lane and as Kogge-Stone scans across
// the LPM lanes (log2(LPM) shuffle steps).  Input and output are mode-major,
// so the nz values of one component of one mode are contiguous.
#include "common.hpp"
#include "depth_dev.hpp"
#include "kernels.hpp"

namespace fvim {
namespace {
// NTL: the input spectrum is read with streaming loads (last use); NU:
// non-uniform depth nodes (prm.hz)
template <typename T, int LPM, int P, bool DISP, bool WANTX, bool NYQ, bool NTL, bool NU = false>
__global__ __launch_bounds__(NT) void k_depth(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
                                             DepthParams prm) {
  depth_modes<T, LPM, P, DISP, WANTX, NYQ, NTL, NU>(in, out, prm, blockIdx.x);
}

// Several grids in one launch: block b belongs to the grid c with
// first[c] <= b < first[c + 1] (main or Nyquist block counts); the table is
// in device memory, so its fields are block-uniform loads.
template <typename T, int LPM, int P, bool DISP, bool WANTX, bool NYQ>
__global__ __launch_bounds__(NT) void k_depth_batch(const DepthBatch* __restrict__ b) {
  depth_batch_block<T, LPM, P, DISP, WANTX, NYQ>(b, (int)blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_nyq_average(cpx<T>* __restrict__ out, const cpx<T>* __restrict__ rep,
                                                   int nx, int ny, int kxh, int ld, int np) {
  nyq_average<T>(out, rep, nx, ny, kxh, ld, np, blockIdx.x);
}

// The same over several grids: block b averages Nyquist mode b - first_nyq[c]
// of the grid c with first_nyq[c] <= b < first_nyq[c + 1].
template <typename T>
__global__ __launch_bounds__(NT) void k_nyq_average_batch(const DepthBatch* __restrict__ b) {
  nyq_batch_block<T>(b, (int)blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_mode_table(ModeConst<T>* __restrict__ tab, int nx, int ny, double lx,
                                                  double ly, double h) {
  const int kxh = nx / 2 + 1;
  const int m = blockIdx.x * NT + threadIdx.x;
  if (m >= kxh * ny) return;
  const int kx = m / ny, ky = m - kx * ny;
  const int k2 = (ky * 2 <= ny) ? ky : ky - ny;
  ModeConst<T> c = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
  if (kx != 0 || ky != 0) {
    const double twopi = 6.283185307179586476925286766559;
    const double q1 = twopi * kx / lx, q2 = twopi * k2 / ly;
    const double q = sqrt(q1 * q1 + q2 * q2);
    const double s = q * h;
    double G0, G0p, H0, H0p;
    elem_coeffs(s, G0, G0p, H0, H0p);
    c.s = (T)s;
    c.r = (T)exp(-s);
    c.G0 = (T)G0;
    c.G0p = (T)G0p;
    c.H0 = (T)H0;
    c.H0p = (T)H0p;
    c.iq = (T)(1.0 / q);
  }
  tab[m] = c;
}

template <typename T, int LPM, int P, bool DISP, bool WANTX>
hipError_t launch_two(const cpx<T>* in, cpx<T>* out, const DepthParams& p, hipStream_t st,
                      int part) {
  constexpr int GPB = NT / LPM;
  const int nnyq = p.ny + p.kxh - 1;
  if (part != 2) {
    const int nmodes = p.kxh * p.ny + (p.rep_out ? depth_replicas(p.ny, p.kxh) : 0);
    const unsigned nb = (unsigned)((nmodes + GPB - 1) / GPB);
    // streaming loads only where a load instruction reads whole lines (one
    // node per lane): with P > 1 the lanes read every P-th element and the
    // rest of the line would be fetched again
    bool streamed = false;
    if (p.hz) {
      bool done = false;
      if constexpr (P == 1) {
        if (p.nt_in) {
          hipLaunchKernelGGL((k_depth<T, LPM, P, DISP, WANTX, false, true, true>), dim3(nb), dim3(NT), 0, st, in,
                             out, p);
          done = true;
        }
      }
      if (!done)
        hipLaunchKernelGGL((k_depth<T, LPM, P, DISP, WANTX, false, false, true>), dim3(nb), dim3(NT), 0, st, in,
                           out, p);
      streamed = true;                 // launched
    }
    if constexpr (P == 1) {
      if (p.nt_in && !streamed) {
        hipLaunchKernelGGL((k_depth<T, LPM, P, DISP, WANTX, false, true>), dim3(nb), dim3(NT), 0, st, in, out, p);
        streamed = true;
      }
    }
    if (!streamed)
      hipLaunchKernelGGL((k_depth<T, LPM, P, DISP, WANTX, false, false>), dim3(nb), dim3(NT), 0, st, in, out, p);
  }
  if (part != 1) {
    if (p.rep_out) {
      hipLaunchKernelGGL(k_nyq_average<T>, dim3((unsigned)nnyq), dim3(NT), 0, st, out,
                         static_cast<const cpx<T>*>(p.rep_out), p.nx, p.ny, p.kxh, p.ld_out, p.np_out);
    } else {
      const unsigned nb2 = (unsigned)((nnyq + GPB - 1) / GPB);
      if (p.hz)
        hipLaunchKernelGGL((k_depth<T, LPM, P, DISP, WANTX, true, false, true>), dim3(nb2), dim3(NT), 0, st, in, out,
                           p);
      else
        hipLaunchKernelGGL((k_depth<T, LPM, P, DISP, WANTX, true, false>), dim3(nb2), dim3(NT), 0, st, in, out, p);
    }
  }
  return hipGetLastError();
}

template <typename T, int LPM, int P>
hipError_t launch_cfg(const cpx<T>* in, cpx<T>* out, const DepthParams& p, hipStream_t st,
                      int part) {
  const bool disp = p.off_disp >= 0 || p.off_u3 >= 0;
  const bool wx = p.off_stress >= 0;
  if (disp) return wx ? launch_two<T, LPM, P, true, true>(in, out, p, st, part)
                      : launch_two<T, LPM, P, true, false>(in, out, p, st, part);
  return wx ? launch_two<T, LPM, P, false, true>(in, out, p, st, part)
            : launch_two<T, LPM, P, false, false>(in, out, p, st, part);
}

// (lanes per mode, nodes per lane) configurations; a configuration serves
// nz <= LPM * P.
struct DepthCfg {
  int lpm, p;
};
constexpr DepthCfg kCfgs[] = {{16, 1}, {16, 2}, {32, 1}, {32, 2}, {64, 1}, {64, 2}, {64, 4}, {64, 8}};
constexpr int kNCfg = sizeof(kCfgs) / sizeof(kCfgs[0]);

}  // namespace

int depth_num_configs() { return kNCfg; }

// Whether configuration id serves nz and is not wasteful (at least a quarter
// of the lanes hold a node).
bool depth_config_valid(int id, int nz) {
  if (id < 0 || id >= kNCfg) return false;
  const int cap = kCfgs[id].lpm * kCfgs[id].p;
  return nz <= cap && 4 * nz > cap;
}

// Default without tuning: the fewest nodes per lane that keeps <= 64 lanes.
int depth_default_config(int nz) {
  if (nz <= 16) return 0;
  if (nz <= 32) return 1;
  if (nz <= 64) return 3;
  if (nz <= 128) return 5;
  if (nz <= 256) return 6;
  return 7;
}

template <typename T>
hipError_t launch_mode_table(ModeConst<T>* tab, int nx, int ny, double lx, double ly, double h, hipStream_t st) {
  const int nm = (nx / 2 + 1) * ny;
  hipLaunchKernelGGL(k_mode_table<T>, dim3((unsigned)((nm + NT - 1) / NT)), dim3(NT), 0, st, tab, nx, ny, lx, ly,
                     h);
  return hipGetLastError();
}

void depth_derive(DepthParams& p) {
  const double kap = p.kappa, kp2 = kap + 2.0;
  p.ikp2 = 1.0 / kp2;
  p.kk = (kap + 1.0) / kp2;
  p.i2k4 = 1.0 / (2.0 * kp2);
  p.kapkp2 = kap / kp2;
  p.cfac = kp2 / (2.0 * (kap + 1.0));
  p.ik2 = 1.0 / (2.0 * kap + 2.0);
}

int depth_groups_per_block(int cfg) { return NT / kCfgs[cfg].lpm; }

// main launch (every mode, and the Nyquist sign replicas as modes of their
// own), then one block per Nyquist mode averaging its replicas
template <typename T, int LPM, int P, bool DISP, bool WANTX>
hipError_t launch_batch_two(const DepthBatch* dtab, int nb_main, int nb_nyq, hipStream_t st) {
  if (nb_main > 0)
    hipLaunchKernelGGL((k_depth_batch<T, LPM, P, DISP, WANTX, false>), dim3(nb_main), dim3(NT), 0, st, dtab);
  if (nb_nyq > 0) hipLaunchKernelGGL(k_nyq_average_batch<T>, dim3(nb_nyq), dim3(NT), 0, st, dtab);
  return hipGetLastError();
}

template <typename T, int LPM, int P>
hipError_t launch_batch_cfg(const DepthBatch* dtab, bool disp, bool wx, int nb_main, int nb_nyq, hipStream_t st) {
  if (disp) return wx ? launch_batch_two<T, LPM, P, true, true>(dtab, nb_main, nb_nyq, st)
                      : launch_batch_two<T, LPM, P, true, false>(dtab, nb_main, nb_nyq, st);
  return wx ? launch_batch_two<T, LPM, P, false, true>(dtab, nb_main, nb_nyq, st)
            : launch_batch_two<T, LPM, P, false, false>(dtab, nb_main, nb_nyq, st);
}

template <typename T>
hipError_t launch_depth_batch(const DepthBatch& host, DepthBatch* dtab, int cfg, hipStream_t st) {
  if (host.n < 1 || host.n > DEPTH_BATCH_MAX || cfg < 0 || cfg >= kNCfg) return hipErrorInvalidValue;
  const DepthParams& p0 = host.prm[0];
  const bool disp = p0.off_disp >= 0 || p0.off_u3 >= 0;
  const bool wx = p0.off_stress >= 0;
  for (int c = 0; c < host.n; ++c) {
    const DepthParams& p = host.prm[c];
    if (!p.mtab || !p.rep_out || p.hz || p.nz > kCfgs[cfg].lpm * kCfgs[cfg].p ||
        (p.off_disp >= 0 || p.off_u3 >= 0) != disp || (p.off_stress >= 0) != wx)
      return hipErrorInvalidValue;
  }
  // pageable source: the copy is staged before the call returns
  hipError_t e = hipMemcpyAsync(dtab, &host, sizeof(DepthBatch), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  const int nm = host.first_main[host.n], nq = host.first_nyq[host.n];
  switch (cfg) {
    case 0: return launch_batch_cfg<T, 16, 1>(dtab, disp, wx, nm, nq, st);
    case 1: return launch_batch_cfg<T, 16, 2>(dtab, disp, wx, nm, nq, st);
    case 2: return launch_batch_cfg<T, 32, 1>(dtab, disp, wx, nm, nq, st);
    case 3: return launch_batch_cfg<T, 32, 2>(dtab, disp, wx, nm, nq, st);
    case 4: return launch_batch_cfg<T, 64, 1>(dtab, disp, wx, nm, nq, st);
    case 5: return launch_batch_cfg<T, 64, 2>(dtab, disp, wx, nm, nq, st);
    case 6: return launch_batch_cfg<T, 64, 4>(dtab, disp, wx, nm, nq, st);
    case 7: return launch_batch_cfg<T, 64, 8>(dtab, disp, wx, nm, nq, st);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_depth(const cpx<T>* in, cpx<T>* out, const DepthParams& prm, int cfg, hipStream_t st,
                        int part) {
  if (!prm.mtab) return hipErrorInvalidValue;
  DepthParams p = prm;
  depth_derive(p);
  if (!depth_config_valid(cfg, p.nz)) cfg = depth_default_config(p.nz);
  switch (cfg) {
    case 0: return launch_cfg<T, 16, 1>(in, out, p, st, part);
    case 1: return launch_cfg<T, 16, 2>(in, out, p, st, part);
    case 2: return launch_cfg<T, 32, 1>(in, out, p, st, part);
    case 3: return launch_cfg<T, 32, 2>(in, out, p, st, part);
    case 4: return launch_cfg<T, 64, 1>(in, out, p, st, part);
    case 5: return launch_cfg<T, 64, 2>(in, out, p, st, part);
    case 6: return launch_cfg<T, 64, 4>(in, out, p, st, part);
    case 7: return launch_cfg<T, 64, 8>(in, out, p, st, part);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_depth<double>(const cpx<double>*, cpx<double>*, const DepthParams&, int, hipStream_t,
                                         int);
template hipError_t launch_depth<float>(const cpx<float>*, cpx<float>*, const DepthParams&, int, hipStream_t, int);
template hipError_t launch_mode_table<double>(ModeConst<double>*, int, int, double, double, double, hipStream_t);
template hipError_t launch_depth_batch<double>(const DepthBatch&, DepthBatch*, int, hipStream_t);
template hipError_t launch_depth_batch<float>(const DepthBatch&, DepthBatch*, int, hipStream_t);
template hipError_t launch_mode_table<float>(ModeConst<float>*, int, int, double, double, double, hipStream_t);

}  // namespace fvim
