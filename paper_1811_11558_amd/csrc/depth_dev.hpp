// Device code of the per-mode depth pass (the bodies the depth kernels and
// the persistent batched operator run).  Included by depth.hip and
// persist.hip; everything is in an anonymous namespace (one copy per
// translation unit).
#pragma once
#include "common.hpp"
#include "kernels.hpp"

namespace fvim {
namespace {


#ifndef FVIM_NT_DEFINED
#define FVIM_NT_DEFINED
constexpr int NT = 256;   // threads per block of every kernel here
#endif

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

// One block of a batched depth launch (main modes or, NYQ, the Nyquist
// averages) over the grids of the table b: block blk belongs to the grid c
// with first[c] <= blk < first[c + 1].
template <typename T, int LPM, int P, bool DISP, bool WANTX, bool NYQ>
__device__ __forceinline__ void depth_batch_block(const DepthBatch* __restrict__ b, int blk) {
  const int* first = NYQ ? b->first_nyq : b->first_main;
  int c = 0;
  while (c + 1 < b->n && blk >= first[c + 1]) ++c;
  depth_modes<T, LPM, P, DISP, WANTX, NYQ>(static_cast<const cpx<T>*>(b->in[c]), static_cast<cpx<T>*>(b->out[c]),
                                           b->prm[c], blk - first[c]);
}

template <typename T>
__device__ __forceinline__ void nyq_batch_block(const DepthBatch* __restrict__ b, int blk) {
  int c = 0;
  while (c + 1 < b->n && blk >= b->first_nyq[c + 1]) ++c;
  const DepthParams& p = b->prm[c];
  nyq_average<T>(static_cast<cpx<T>*>(b->out[c]), static_cast<const cpx<T>*>(p.rep_out), p.nx, p.ny, p.kxh,
                 p.ld_out, p.np_out, blk - b->first_nyq[c]);
}

}  // namespace
}  // namespace fvim
