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
#include "kernels.hpp"

namespace fvim {
namespace {

constexpr int NT = 256;

// Taylor coefficients of the element functions, divided by the power of s
// that multiplies them:
//   G0  = s   int_0^1 (1-t) e^{-st} dt,   G0' = s   int_0^1 t e^{-st} dt,
//   H0  = s^2 int_0^1 t(1-t) e^{-st} dt,  H0' = s^2 int_0^1 t^2 e^{-st} dt.
constexpr double inv_fact(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return 1.0 / f;
}
constexpr double sgn(int k) { return (k & 1) ? -1.0 : 1.0; }
constexpr double ca(int k) { return sgn(k) * inv_fact(k) / ((k + 1.0) * (k + 2.0)); }
constexpr double cb(int k) { return sgn(k) * inv_fact(k) / (k + 2.0); }
constexpr double cc(int k) { return sgn(k) * inv_fact(k) / ((k + 2.0) * (k + 3.0)); }
constexpr double cd(int k) { return sgn(k) * inv_fact(k) / (k + 3.0); }

// Element functions in float64: 26 Taylor terms below s = 2 (the truncation
// is below 2^-53 relative there), closed forms above.
__device__ __forceinline__ void elem_coeffs(double s, double& G0, double& G0p, double& H0, double& H0p) {
  using T = double;
  if (s < T(2)) {
    constexpr int N = 26;
    T a = ca(N - 1), b = cb(N - 1), c = cc(N - 1), d = cd(N - 1);
#pragma unroll
    for (int k = N - 2; k >= 0; --k) {
      a = a * s + ca(k);
      b = b * s + cb(k);
      c = c * s + cc(k);
      d = d * s + cd(k);
    }
    G0 = s * a;
    G0p = s * b;
    H0 = s * s * c;
    H0p = s * s * d;
  } else {
    T e = exp(-s);
    T I0 = T(1) - e;
    T I1 = T(1) - e * (T(1) + s);
    T I2 = T(2) - e * (T(2) + s * (T(2) + s));
    T is = T(1) / s;
    G0 = I0 - I1 * is;
    G0p = I1 * is;
    H0 = I1 - I2 * is;
    H0p = I2 * is;
  }
}

template <typename T, int LPM>
__device__ __forceinline__ cpx<T> sh_down(cpx<T> v, int d) {
  return mk(__shfl_down(v.x, d, LPM), __shfl_down(v.y, d, LPM));
}
template <typename T, int LPM>
__device__ __forceinline__ cpx<T> sh_up(cpx<T> v, int d) {
  return mk(__shfl_up(v.x, d, LPM), __shfl_up(v.y, d, LPM));
}
template <typename T, int LPM>
__device__ __forceinline__ cpx<T> sh_idx(cpx<T> v, int src) {
  return mk(__shfl(v.x, src, LPM), __shfl(v.y, src, LPM));
}

// x^e for 1 <= e <= 31 by squaring
template <typename T>
__device__ __forceinline__ T powi(T x, int e) {
  T p = T(1);
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    if (e & 1) p *= x;
    x *= x;
    e >>= 1;
  }
  return p;
}

// The two scans of the depth pass over a 64-lane group (one wave) on
// uniform nodes, each lane holding P nodes: per lane step the propagator is
// rl = r^P with Jordan shift sl = P s.  Reverse (growing coordinates): the
// suffix Y(l) = sum over j >= l of Rb^(j - l) A_j with Rb = rl [[1, -sl],
// [0, 1]] on (Y2, Y3) and rl on YP; forward (decaying): the prefix
// F(l) = sum over j <= l of Rf^(l - j) a_j with Rf = rl [[1, sl], [0, 1]].
// Kogge-Stone within each row of 16 lanes by DPP moves, then the rows'
// totals combined in order from broadcast lane values (3 sequential steps)
// and carried into every lane with the power of the propagator for its
// distance to the neighbouring row.
template <int D, typename T>
__device__ __forceinline__ void rev_row_step(cpx<T>& Y2, cpx<T>& Y3, cpx<T>& YP, T rk, T ks, int lr) {
  const cpx<T> o2 = dpp_move<DPP_ROW_DOWN + D>(Y2), o3 = dpp_move<DPP_ROW_DOWN + D>(Y3);
  const cpx<T> op = dpp_move<DPP_ROW_DOWN + D>(YP);
  const T wk = (lr + D < 16) ? rk : T(0);
  Y2 = add(Y2, scl(axpy(o2, -ks, o3), wk));
  Y3 = add(Y3, scl(o3, wk));
  YP = add(YP, scl(op, wk));
}
template <int D, typename T>
__device__ __forceinline__ void fwd_row_step(cpx<T>& F0, cpx<T>& F1, cpx<T>& FM, T rk, T ks, int lr) {
  const cpx<T> o0 = dpp_move<DPP_ROW_UP + D>(F0), o1 = dpp_move<DPP_ROW_UP + D>(F1);
  const cpx<T> om = dpp_move<DPP_ROW_UP + D>(FM);
  const T wk = (lr >= D) ? rk : T(0);
  F0 = add(F0, scl(axpy(o0, ks, o1), wk));
  F1 = add(F1, scl(o1, wk));
  FM = add(FM, scl(om, wk));
}

template <typename T>
__device__ __forceinline__ void reverse_scan64(cpx<T>& Y2, cpx<T>& Y3, cpx<T>& YP, T rl, T sl, int l) {
  const int lr = l & 15, row = l >> 4;
  T rk = rl, ks = sl;
  rev_row_step<1>(Y2, Y3, YP, rk, ks, lr);
  rk *= rk; ks += ks;
  rev_row_step<2>(Y2, Y3, YP, rk, ks, lr);
  rk *= rk; ks += ks;
  rev_row_step<4>(Y2, Y3, YP, rk, ks, lr);
  rk *= rk; ks += ks;
  rev_row_step<8>(Y2, Y3, YP, rk, ks, lr);
  rk *= rk; ks += ks;                       // rl^16, 16 sl: one row
  // complete suffixes at the starts of rows 3, 2, 1
  cpx<T> t2 = lane_value(Y2, 48), t3 = lane_value(Y3, 48), tp = lane_value(YP, 48);
  cpx<T> c2 = t2, c3 = t3, cp = tp;        // carry for row 2
  t2 = add(lane_value(Y2, 32), scl(axpy(t2, -ks, t3), rk));
  t3 = add(lane_value(Y3, 32), scl(t3, rk));
  tp = add(lane_value(YP, 32), scl(tp, rk));
  if (row == 1) { c2 = t2; c3 = t3; cp = tp; }
  t2 = add(lane_value(Y2, 16), scl(axpy(t2, -ks, t3), rk));
  t3 = add(lane_value(Y3, 16), scl(t3, rk));
  tp = add(lane_value(YP, 16), scl(tp, rk));
  if (row == 0) { c2 = t2; c3 = t3; cp = tp; }
  if (row < 3) {
    const int dist = 16 - lr;
    const T wk = powi(rl, dist), kd = (T)dist * sl;
    Y2 = add(Y2, scl(axpy(c2, -kd, c3), wk));
    Y3 = add(Y3, scl(c3, wk));
    YP = add(YP, scl(cp, wk));
  }
}

template <typename T>
__device__ __forceinline__ void forward_scan64(cpx<T>& F0, cpx<T>& F1, cpx<T>& FM, T rl, T sl, int l) {
  const int lr = l & 15, row = l >> 4;
  T rk = rl, ks = sl;
  fwd_row_step<1>(F0, F1, FM, rk, ks, lr);
  rk *= rk; ks += ks;
  fwd_row_step<2>(F0, F1, FM, rk, ks, lr);
  rk *= rk; ks += ks;
  fwd_row_step<4>(F0, F1, FM, rk, ks, lr);
  rk *= rk; ks += ks;
  fwd_row_step<8>(F0, F1, FM, rk, ks, lr);
  rk *= rk; ks += ks;
  // complete prefixes at the ends of rows 0, 1, 2
  cpx<T> t0 = lane_value(F0, 15), t1 = lane_value(F1, 15), tm = lane_value(FM, 15);
  cpx<T> c0 = t0, c1 = t1, cm = tm;        // carry for row 1
  t0 = add(lane_value(F0, 31), scl(axpy(t0, ks, t1), rk));
  t1 = add(lane_value(F1, 31), scl(t1, rk));
  tm = add(lane_value(FM, 31), scl(tm, rk));
  if (row == 2) { c0 = t0; c1 = t1; cm = tm; }
  t0 = add(lane_value(F0, 47), scl(axpy(t0, ks, t1), rk));
  t1 = add(lane_value(F1, 47), scl(t1, rk));
  tm = add(lane_value(FM, 47), scl(tm, rk));
  if (row == 3) { c0 = t0; c1 = t1; cm = tm; }
  if (row > 0) {
    const int dist = lr + 1;
    const T wk = powi(rl, dist), kd = (T)dist * sl;
    F0 = add(F0, scl(axpy(c0, kd, c1), wk));
    F1 = add(F1, scl(c1, wk));
    FM = add(FM, scl(cm, wk));
  }
}

// Modal loads of one node from the rotated eigenstress/mu (in-plane part
// (f0, f1) decaying, (f2, f3) growing; antiplane fm decaying, fp growing).
template <typename T>
struct Loads {
  cpx<T> f0, f1, f2, f3, fm, fp;
};

// Ratios of kappa = lambda / mu used per node (computed once on the host).
template <typename T>
struct MatC {
  T kap, ikp2, kk, i2k4, kapkp2;
};

template <typename T>
__device__ __forceinline__ Loads<T> modal_loads(const cpx<T> o[5], const MatC<T>& m) {
  // o = (omega_nn, omega_zz, omega_nz / i, omega_nt / i, omega_tz)
  const T kk = m.kk, i2k4 = m.i2k4;
  cpx<T> ec = scl(o[1], m.ikp2);
  cpx<T> et1 = sub(o[0], scl(o[1], m.kapkp2));
  Loads<T> L;
  L.f0 = sub(scl(ec, -kk), scl(et1, i2k4));
  L.f1 = axpy(sub(scl(o[2], -kk), scl(ec, kk)), T(0.5) * kk, et1);
  L.f2 = axpy(scl(ec, kk), i2k4, et1);
  L.f3 = axpy(sub(scl(o[2], kk), scl(ec, kk)), T(0.5) * kk, et1);
  L.fm = scl(add(o[4], o[3]), T(0.5));
  L.fp = scl(sub(o[4], o[3]), T(0.5));
  return L;
}

template <typename T>
__device__ __forceinline__ void put(cpx<T>* __restrict__ dst, cpx<T> v, bool first) {
  if (!first) v = add(v, *dst);
  *dst = v;
}

// NYQ = false: every mode except the Nyquist ones (kx = nx/2 or ky = ny/2),
// one evaluation each.  NYQ = true: only the Nyquist modes, each the average
// of its 2 or 4 sign replicas (indexed by group: first the kx = nx/2 column,
// then the ky = ny/2 row without its kx = nx/2 entry).
// Block `block` of the pass over one grid (prm): GPB = NT / LPM lane groups,
// one mode each.
// NU: non-uniform depth nodes (prm.hz): every element has its own scaled
// length s_e = |q| h_e, propagator exp(-s_e) [[1, +/-s_e], [0, 1]] and
// element functions; since these propagators commute and compose by adding
// the s_e, the scans carry each lane's (product of exp(-s_e), sum of s_e)
// instead of powers of one per-mode constant.
template <typename T, int LPM, int P, bool DISP, bool WANTX, bool NYQ, bool NTL = false, bool NU = false>
__device__ __forceinline__ void depth_modes(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
                                            const DepthParams& prm, int block) {
  constexpr int GPB = NT / LPM;
  // one wave per mode on uniform nodes: the scans and lane moves use DPP
  constexpr bool DPPS = LPM == 64 && !NU;
  const int g = threadIdx.x / LPM;
  const int l = threadIdx.x - g * LPM;
  const int gid = block * GPB + g;
  int kx, ky;
  // vrep >= 0: this group evaluates sign replica vrep of a Nyquist mode,
  // unweighted, into replica record vslot of prm.rep_out.  Replica records:
  // 2 j, 2 j + 1 for Nyquist mode j (the kx = nx/2 column first, then the
  // ky = ny/2 row), then replicas 2 and 3 of the corner
  int vrep = -1, vslot = 0;
  if (NYQ) {
    if (gid >= prm.ny + prm.kxh - 1) return;
    if (gid < prm.ny) { kx = prm.nx / 2; ky = gid; }
    else { kx = gid - prm.ny; ky = prm.ny / 2; }
  } else {
    const int nmain = prm.kxh * prm.ny;
    if (gid >= nmain) {
      vslot = gid - nmain;
      const int mn = prm.ny + prm.kxh - 1;
      if (!prm.rep_out || vslot >= 2 * mn + 2) return;   // the whole lane group leaves together
      int j;
      if (vslot < 2 * mn) { j = vslot >> 1; vrep = vslot & 1; }
      else { j = prm.ny / 2; vrep = 2 + (vslot - 2 * mn); }
      if (j < prm.ny) { kx = prm.nx / 2; ky = j; }
      else { kx = j - prm.ny; ky = prm.ny / 2; }
    } else {
      kx = gid / prm.ny;
      ky = gid - kx * prm.ny;
      if (kx * 2 == prm.nx || ky * 2 == prm.ny) return;
    }
  }
  const int mode = kx * prm.ny + ky;
  const int nz = prm.nz;
  const cpx<T>* __restrict__ src = in + (size_t)mode * prm.ld_in;
  cpx<T>* __restrict__ dst = vrep >= 0 ? static_cast<cpx<T>*>(prm.rep_out) + (size_t)vslot * prm.ld_out
                                       : out + (size_t)mode * prm.ld_out;
  const T nrm = (T)prm.norm;
  const T kap = (T)prm.kappa;
  const T mu = (T)prm.mu;
  const int i0 = l * P;
  const bool wantS = prm.off_strain >= 0;
  // eigenstrain layers z >= za are zero (their spectra were not written)
  const int za = prm.zact ? min(*prm.zact, nz) : nz;
  const bool has_w = prm.has_w != 0;
  constexpr bool wantX = WANTX;

  cpx<T> tr[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) tr[c] = prm.has_t ? scl(src[prm.off_t + c], nrm / mu) : zero<T>();

  // strain e (original frame, 6 comps) of node i -> outputs (stress needs eps_p again)
  auto emit = [&](int i, const cpx<T> e[6], bool first, T wgt) {
    if (wantS) {
#pragma unroll
      for (int c = 0; c < 6; ++c) put(dst + prm.off_strain + (size_t)c * nz + i, scl(e[c], wgt), first);
    }
    if (wantX) {
      cpx<T> ep[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) ep[c] = (has_w && i < za) ? scl(src[(size_t)c * nz + i], nrm) : zero<T>();
      cpx<T> tre = add(add(e[0], e[1]), e[2]);
      cpx<T> trp = add(add(ep[0], ep[1]), ep[2]);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        cpx<T> sc = scl(sub(e[c], ep[c]), T(2) * mu);
        if (c < 3) sc = axpy(sc, kap * mu, sub(tre, trp));
        put(dst + prm.off_stress + (size_t)c * nz + i, scl(sc, wgt), first);
      }
    }
  };

  if (!NYQ && kx == 0 && ky == 0) {
    // laterally uniform mode: sigma . e3 = -t everywhere, no in-plane strain
    const T tk = prm.k0_include ? T(1) : T(0);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int i = i0 + p;
      if (i >= nz) continue;
      cpx<T> ep[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) ep[c] = (has_w && i < za) ? src[(size_t)c * nz + i] : zero<T>();
      cpx<T> trp = add(add(ep[0], ep[1]), ep[2]);
      cpx<T> w33 = scl(axpy(scl(trp, kap), T(2), ep[2]), nrm);     // w33 / mu
      cpx<T> e[6] = {zero<T>(), zero<T>(), zero<T>(), zero<T>(), zero<T>(), zero<T>()};
      e[4] = sub(scl(ep[4], nrm), scl(tr[0], T(0.5) * tk));        // e13
      e[3] = sub(scl(ep[3], nrm), scl(tr[1], T(0.5) * tk));        // e23
      e[2] = scl(sub(w33, scl(tr[2], tk)), (T)prm.ikp2);             // e33
      if (prm.k0_external) {          // the caller adds this mode in float64
        if (wantS) {
#pragma unroll
          for (int c = 0; c < 6; ++c) dst[prm.off_strain + (size_t)c * nz + i] = zero<T>();
        }
        if (wantX) {
#pragma unroll
          for (int c = 0; c < 6; ++c) dst[prm.off_stress + (size_t)c * nz + i] = zero<T>();
        }
      } else {
        emit(i, e, true, T(1));
      }
      if (DISP) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
          if (prm.off_disp >= 0) dst[prm.off_disp + (size_t)c * nz + i] = zero<T>();
        if (prm.off_u3 >= 0 && i == 0) dst[prm.off_u3] = zero<T>();
      }
    }
    return;
  }

  const int nyqx = (NYQ || vrep >= 0) && (kx * 2 == prm.nx);
  const int nyqy = (NYQ || vrep >= 0) && (ky * 2 == prm.ny);
  const int nrep = NYQ ? (nyqx ? 2 : 1) * (nyqy ? 2 : 1) : 1;
  const int rep0 = vrep >= 0 ? vrep : 0;
  const int k1 = kx;
  const int k2 = (ky * 2 <= prm.ny) ? ky : ky - prm.ny;
  const T wrep = nrep == 1 ? T(1) : (nrep == 2 ? T(0.5) : T(0.25));
  const T cfac = (T)prm.cfac;
  const T ik2 = (T)prm.ik2;
  const MatC<T> mc = {kap, (T)prm.ikp2, (T)prm.kk, (T)prm.i2k4, (T)prm.kapkp2};
  // |q| and everything built from it are the same for every sign replica
  const ModeConst<T> K = static_cast<const ModeConst<T>*>(prm.mtab)[mode];
  const double twopi = 6.283185307179586476925286766559;
  const T iq = K.iq;
  const T q1a = (T)(twopi * k1 / prm.lx);
  const T q2a = (T)(twopi * k2 / prm.ly);
  const T s = K.s, r = K.r;
  T rP = r;
#pragma unroll
  for (int k = 1; k < P; ++k) rP *= r;
  const T G0 = K.G0, G0p = K.G0p, H0 = K.H0, H0p = K.H0p;
  // NU: per element e = i0 + p (nodes e, e + 1; length 0 past the last
  // node) and the lane's totals
  T se[NU ? P : 1], re[NU ? P : 1], eg0[NU ? P : 1], eg0p[NU ? P : 1], eh0[NU ? P : 1], eh0p[NU ? P : 1];
  T SL = T(0), RL = T(1);
  if constexpr (NU) {
    const double q1d = twopi * k1 / prm.lx, q2d = twopi * k2 / prm.ly;
    const double qd = sqrt(q1d * q1d + q2d * q2d);
    double S = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int e = i0 + p;
      const double sd = (e + 1 < nz) ? qd * prm.hz[e] : 0.0;
      double a, b, c, d;
      elem_coeffs(sd, a, b, c, d);
      se[p] = (T)sd;
      re[p] = (T)exp(-sd);
      eg0[p] = (T)a;
      eg0p[p] = (T)b;
      eh0[p] = (T)c;
      eh0p[p] = (T)d;
      S += sd;
    }
    SL = (T)S;
    RL = (T)exp(-S);
  }

  for (int rep = rep0; rep < rep0 + nrep; ++rep) {
    int bits = rep;
    T s1 = T(1), s2 = T(1);
    if (nyqx) { s1 = (bits & 1) ? T(-1) : T(1); bits >>= 1; }
    if (nyqy) { s2 = (bits & 1) ? T(-1) : T(1); }
    const T n1 = s1 * q1a * iq, n2 = s2 * q2a * iq;

    // ---- load, rotate, scale: o = (w_nn, w_zz, w_nz/i, w_nt/i, w_tz) / mu ----
    cpx<T> o[P][5];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int i = i0 + p;
      cpx<T> ep[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) ep[c] = (has_w && i < za) ? ld_in<NTL>(src + (size_t)c * nz + i) : zero<T>();
      cpx<T> trp = add(add(ep[0], ep[1]), ep[2]);
      cpx<T> exx = add(add(scl(ep[0], n1 * n1), scl(ep[5], T(2) * n1 * n2)), scl(ep[1], n2 * n2));
      cpx<T> exe = add(add(scl(ep[0], -n1 * n2), scl(ep[5], n1 * n1 - n2 * n2)), scl(ep[1], n1 * n2));
      cpx<T> exz = add(scl(ep[4], n1), scl(ep[3], n2));
      cpx<T> eez = sub(scl(ep[3], n1), scl(ep[4], n2));
      o[p][0] = scl(axpy(scl(trp, kap), T(2), exx), nrm);
      o[p][1] = scl(axpy(scl(trp, kap), T(2), ep[2]), nrm);
      o[p][2] = scl(mul_mi(exz), T(2) * nrm);
      o[p][3] = scl(mul_mi(exe), T(2) * nrm);
      o[p][4] = scl(eez, T(2) * nrm);
    }
    // rotated loads of the next lane's first node (zero past the last node)
    cpx<T> on[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      if constexpr (DPPS) on[c] = dpp_move<DPP_WAVE_DOWN1>(o[0][c]);
      else on[c] = sh_down<T, LPM>(o[0][c], 1);
    }

    // ---- backward (growing) recurrence inside the lane, zero carry ----
    cpx<T> M2[P], M3[P], MP[P];
    {
      cpx<T> x2 = zero<T>(), x3 = zero<T>(), xp = zero<T>();
      Loads<T> Ln = modal_loads<T>(on, mc);
#pragma unroll
      for (int p = P - 1; p >= 0; --p) {
        const int e = i0 + p;                    // element e joins nodes e, e+1
        Loads<T> L = modal_loads<T>(o[p], mc);
        cpx<T> b2 = zero<T>(), b3 = zero<T>(), bp = zero<T>();
        const T g0 = NU ? eg0[NU ? p : 0] : G0, g0p = NU ? eg0p[NU ? p : 0] : G0p;
        const T h0 = NU ? eh0[NU ? p : 0] : H0, h0p = NU ? eh0p[NU ? p : 0] : H0p;
        const T se_ = NU ? se[NU ? p : 0] : s, re_ = NU ? re[NU ? p : 0] : r;
        if (e + 1 < nz) {
          b3 = add(scl(L.f3, g0), scl(Ln.f3, g0p));
          b2 = sub(add(scl(L.f2, g0), scl(Ln.f2, g0p)), add(scl(L.f3, h0), scl(Ln.f3, h0p)));
          bp = add(scl(L.fp, g0), scl(Ln.fp, g0p));
        }
        x2 = sub(scl(axpy(x2, -se_, x3), re_), b2);
        x3 = sub(scl(x3, re_), b3);
        xp = sub(scl(xp, re_), bp);
        M2[p] = x2;
        M3[p] = x3;
        MP[p] = xp;
        Ln = L;
      }
    }
    // ---- reverse scan across lanes: Y_l = A_l + Rb^P Y_(l+1) ----
    cpx<T> Y2 = M2[0], Y3 = M3[0], YP = MP[0];
    if constexpr (DPPS) {
      reverse_scan64<T>(Y2, Y3, YP, rP, (T)P * s, l);
    } else {
      T rk = NU ? RL : rP, ks = NU ? SL : (T)P * s;
#pragma unroll
      for (int d = 1; d < LPM; d <<= 1) {
        cpx<T> o2 = sh_down<T, LPM>(Y2, d), o3 = sh_down<T, LPM>(Y3, d), op = sh_down<T, LPM>(YP, d);
        const T wk = (l + d < LPM) ? rk : T(0);    // no partner below the last lane
        Y2 = add(Y2, scl(axpy(o2, -ks, o3), wk));
        Y3 = add(Y3, scl(o3, wk));
        YP = add(YP, scl(op, wk));
        if constexpr (NU) {                        // lanes l .. l + 2d - 1
          const T prk = __shfl_down(rk, d, LPM), pks = __shfl_down(ks, d, LPM);
          rk = rk * prk;
          ks = ks + pks;
        } else {
          rk = rk * rk;
          ks = ks + ks;
        }
      }
    }
    {
      cpx<T> C2, C3, CP;
      if constexpr (DPPS) {
        C2 = dpp_move<DPP_WAVE_DOWN1>(Y2);
        C3 = dpp_move<DPP_WAVE_DOWN1>(Y3);
        CP = dpp_move<DPP_WAVE_DOWN1>(YP);
      } else {
        C2 = sh_down<T, LPM>(Y2, 1);
        C3 = sh_down<T, LPM>(Y3, 1);
        CP = sh_down<T, LPM>(YP, 1);
      }
      if (l == LPM - 1) { C2 = zero<T>(); C3 = zero<T>(); CP = zero<T>(); }
      T rk = NU ? re[NU ? P - 1 : 0] : r, ks = NU ? se[NU ? P - 1 : 0] : s;   // Rb^(P-p) on the carry
#pragma unroll
      for (int p = P - 1; p >= 0; --p) {
        M2[p] = add(M2[p], scl(axpy(C2, -ks, C3), rk));
        M3[p] = add(M3[p], scl(C3, rk));
        MP[p] = add(MP[p], scl(CP, rk));
        if constexpr (NU) {
          if (p > 0) {
            rk = rk * re[p - 1];
            ks = ks + se[p - 1];
          }
        } else {
          rk = rk * r;
          ks = ks + s;
        }
      }
    }
    // ---- surface condition: sigma . e3 = -t at z = 0 ----
    cpx<T> bc0, bc1, bcm;
    {
      cpx<T> g20, g30, gp0;
      if constexpr (DPPS) {
        g20 = lane_value(M2[0], 0);
        g30 = lane_value(M3[0], 0);
        gp0 = lane_value(MP[0], 0);
      } else {
        g20 = sh_idx<T, LPM>(M2[0], 0);
        g30 = sh_idx<T, LPM>(M3[0], 0);
        gp0 = sh_idx<T, LPM>(MP[0], 0);
      }
      cpx<T> Txi = add(scl(tr[0], n1), scl(tr[1], n2));
      cpx<T> t1bc = mul_i(Txi);                          // -(T_n / i) = i T_n
      cpx<T> t2bc = scl(tr[2], T(-1));
      cpx<T> t3bc = sub(scl(tr[0], n2), scl(tr[1], n1)); // -T_t
      bc0 = sub(t2bc, g20);
      bc1 = sub(sub(add(t1bc, bc0), g20), g30);
      bcm = sub(gp0, t3bc);
    }
    // ---- forward (decaying) recurrence inside the lane, zero carry ----
    cpx<T> Z0[P], Z1[P], ZM[P];
    cpx<T> F0, F1, FM;
    {
      cpx<T> z0 = zero<T>(), z1 = zero<T>(), zm = zero<T>();
#pragma unroll
      for (int p = 0; p < P; ++p) {
        Z0[p] = z0;
        Z1[p] = z1;
        ZM[p] = zm;
        const int e = i0 + p;
        cpx<T> a0 = zero<T>(), a1 = zero<T>(), am = zero<T>();
        const T g0 = NU ? eg0[NU ? p : 0] : G0, g0p = NU ? eg0p[NU ? p : 0] : G0p;
        const T h0 = NU ? eh0[NU ? p : 0] : H0, h0p = NU ? eh0p[NU ? p : 0] : H0p;
        const T se_ = NU ? se[NU ? p : 0] : s, re_ = NU ? re[NU ? p : 0] : r;
        if (e + 1 < nz) {
          Loads<T> L = modal_loads<T>(o[p], mc);
          Loads<T> Ln = modal_loads<T>(p + 1 < P ? o[(p + 1) % P] : on, mc);
          a1 = add(scl(L.f1, g0p), scl(Ln.f1, g0));
          a0 = add(add(scl(L.f0, g0p), scl(Ln.f0, g0)), add(scl(L.f1, h0p), scl(Ln.f1, h0)));
          am = add(scl(L.fm, g0p), scl(Ln.fm, g0));
        }
        z0 = add(scl(axpy(z0, se_, z1), re_), a0);
        z1 = add(scl(z1, re_), a1);
        zm = add(scl(zm, re_), am);
      }
      F0 = z0;
      F1 = z1;
      FM = zm;
    }
    // ---- forward scan across lanes with the surface value on lane 0 ----
    if (l == 0) {
      const T ps = NU ? SL : (T)P * s, rl = NU ? RL : rP;
      F0 = add(F0, scl(axpy(bc0, ps, bc1), rl));
      F1 = add(F1, scl(bc1, rl));
      FM = add(FM, scl(bcm, rl));
    }
    if constexpr (DPPS) {
      forward_scan64<T>(F0, F1, FM, rP, (T)P * s, l);
    } else {
      T rk = NU ? RL : rP, ks = NU ? SL : (T)P * s;
#pragma unroll
      for (int d = 1; d < LPM; d <<= 1) {
        cpx<T> o0 = sh_up<T, LPM>(F0, d), o1 = sh_up<T, LPM>(F1, d), om = sh_up<T, LPM>(FM, d);
        const T wk = (l >= d) ? rk : T(0);         // no partner above the first lane
        F0 = add(F0, scl(axpy(o0, ks, o1), wk));
        F1 = add(F1, scl(o1, wk));
        FM = add(FM, scl(om, wk));
        if constexpr (NU) {                        // lanes l - 2d + 1 .. l
          const T prk = __shfl_up(rk, d, LPM), pks = __shfl_up(ks, d, LPM);
          rk = rk * prk;
          ks = ks + pks;
        } else {
          rk = rk * rk;
          ks = ks + ks;
        }
      }
    }
    cpx<T> D0, D1, DM;
    if constexpr (DPPS) {
      D0 = dpp_move<DPP_WAVE_UP1>(F0);
      D1 = dpp_move<DPP_WAVE_UP1>(F1);
      DM = dpp_move<DPP_WAVE_UP1>(FM);
    } else {
      D0 = sh_up<T, LPM>(F0, 1);
      D1 = sh_up<T, LPM>(F1, 1);
      DM = sh_up<T, LPM>(FM, 1);
    }
    if (l == 0) { D0 = bc0; D1 = bc1; DM = bcm; }

    // ---- nodal fields, strains, outputs ----
    {
      T rk = T(1), ks = T(0);
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const int i = i0 + p;
        cpx<T> m0 = add(Z0[p], scl(axpy(D0, ks, D1), rk));
        cpx<T> m1 = add(Z1[p], scl(D1, rk));
        cpx<T> mm = add(ZM[p], scl(DM, rk));
        if constexpr (NU) {
          rk = rk * re[NU ? p : 0];
          ks = ks + se[NU ? p : 0];
        } else {
          rk = rk * r;
          ks = ks + s;
        }
        if (i >= nz) continue;
        cpx<T> m2 = M2[p], m3 = M3[p], mpp = MP[p];
        cpx<T> a = add(sub(scl(add(m0, m2), T(0.5)), scl(m1, cfac)), scl(m3, cfac));
        cpx<T> t1 = add(add(sub(m1, m0), m2), m3);
        cpx<T> t2 = add(m0, m2);
        cpx<T> v = add(mpp, mm);
        cpx<T> t3 = sub(mpp, mm);
        cpx<T> exx = scl(a, T(-1));
        cpx<T> ezz = scl(add(add(scl(a, kap), t2), o[p][1]), (T)prm.ikp2);
        cpx<T> exz = mul_i(scl(add(t1, o[p][2]), T(0.5)));
        cpx<T> eez = scl(add(t3, o[p][4]), T(0.5));
        cpx<T> exe = mul_i(scl(v, T(0.5)));
        cpx<T> e[6];
        e[0] = sub(scl(exx, n1 * n1), scl(exe, T(2) * n1 * n2));
        e[1] = add(scl(exx, n2 * n2), scl(exe, T(2) * n1 * n2));
        e[2] = ezz;
        e[3] = add(scl(exz, n2), scl(eez, n1));
        e[4] = sub(scl(exz, n1), scl(eez, n2));
        e[5] = add(scl(exx, n1 * n2), scl(exe, n1 * n1 - n2 * n2));
        emit(i, e, rep == rep0, wrep);
        if (DISP) {
          cpx<T> c = sub(sub(scl(sub(m2, m0), T(0.5)), scl(m1, ik2)), scl(m3, ik2));
          cpx<T> U = mul_i(scl(a, iq));
          cpx<T> V = scl(v, iq);
          cpx<T> W = scl(c, iq);
          if (prm.off_disp >= 0) {
            put(dst + prm.off_disp + i, scl(sub(scl(U, n1), scl(V, n2)), wrep), rep == rep0);
            put(dst + prm.off_disp + (size_t)nz + i, scl(add(scl(U, n2), scl(V, n1)), wrep), rep == rep0);
            put(dst + prm.off_disp + (size_t)2 * nz + i, scl(W, wrep), rep == rep0);
          }
          if (prm.off_u3 >= 0 && i == 0) put(dst + prm.off_u3, scl(W, wrep), rep == rep0);
        }
      }
    }
  }
}

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
  const int* first = NYQ ? b->first_nyq : b->first_main;
  int c = 0;
  while (c + 1 < b->n && (int)blockIdx.x >= first[c + 1]) ++c;
  depth_modes<T, LPM, P, DISP, WANTX, NYQ>(static_cast<const cpx<T>*>(b->in[c]), static_cast<cpx<T>*>(b->out[c]),
                                           b->prm[c], (int)blockIdx.x - first[c]);
}

// Nyquist mode j <- the weighted sum of its sign replicas, in the order and
// with the weights (1/2, or 1/4 at the corner) of the replica loop of the
// NYQ kernel; one block per mode.
template <typename T>
__device__ __forceinline__ void nyq_average(cpx<T>* __restrict__ out, const cpx<T>* __restrict__ rep, int nx,
                                            int ny, int kxh, int ld, int np, int j) {
  const int mn = ny + kxh - 1;
  int kx, ky;
  if (j < ny) { kx = nx / 2; ky = j; }
  else { kx = j - ny; ky = ny / 2; }
  const bool corner = kx * 2 == nx && ky * 2 == ny;
  const T w = corner ? T(0.25) : T(0.5);
  const cpx<T>* r0 = rep + (size_t)(2 * j) * ld;
  const cpx<T>* r1 = r0 + ld;
  const cpx<T>* r2 = rep + (size_t)(2 * mn) * ld;
  const cpx<T>* r3 = r2 + ld;
  cpx<T>* dst = out + (size_t)(kx * ny + ky) * ld;
  for (int c = threadIdx.x; c < np; c += NT) {
    cpx<T> v = add(scl(r1[c], w), scl(r0[c], w));
    if (corner) {
      v = add(scl(r2[c], w), v);
      v = add(scl(r3[c], w), v);
    }
    dst[c] = v;
  }
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
  int c = 0;
  while (c + 1 < b->n && (int)blockIdx.x >= b->first_nyq[c + 1]) ++c;
  const DepthParams& p = b->prm[c];
  nyq_average<T>(static_cast<cpx<T>*>(b->out[c]), static_cast<const cpx<T>*>(p.rep_out), p.nx, p.ny, p.kxh,
                 p.ld_out, p.np_out, (int)blockIdx.x - b->first_nyq[c]);
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
