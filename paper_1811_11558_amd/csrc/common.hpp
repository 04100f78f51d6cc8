// Shared device/host helpers of the fvim HIP library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fvim {

template <typename T>
struct cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T a, T b) {
  cpx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
// Loads that mark the line as streaming (non-temporal): for data a kernel
// reads for the last time, so that it does not displace what the next kernel
// will read (the previous kernel's output) from the caches.
template <typename T>
struct nt_vec;
template <>
struct nt_vec<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <>
struct nt_vec<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <typename T>
__device__ __forceinline__ cpx<T> ld_nt(const cpx<T>* p) {
  typedef typename nt_vec<T>::type V;
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  cpx<T> r;
  r.x = v.x;
  r.y = v.y;
  return r;
}
// a load that streams when NT is set
template <bool NT, typename T>
__device__ __forceinline__ cpx<T> ld_in(const cpx<T>* p) {
  if constexpr (NT) return ld_nt(p);
  else return *p;
}
template <bool NT>
__device__ __forceinline__ double2 ld_in(const double2* p) {
  if constexpr (NT) {
    const cpx<double> v = ld_nt(reinterpret_cast<const cpx<double>*>(p));
    return make_double2(v.x, v.y);
  } else {
    return *p;
  }
}
template <typename T>
__device__ __forceinline__ cpx<T> add(cpx<T> a, cpx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> sub(cpx<T> a, cpx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> mul(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cpx<T> mulc(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cpx<T> scl(cpx<T> a, T s) { return mk(a.x * s, a.y * s); }
// a + s * b  (s real)
template <typename T>
__device__ __forceinline__ cpx<T> axpy(cpx<T> a, T s, cpx<T> b) { return mk(a.x + s * b.x, a.y + s * b.y); }
// i * a
template <typename T>
__device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return mk(-a.y, a.x); }
// -i * a
template <typename T>
__device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) { return mk(a.y, -a.x); }
template <typename T>
__device__ __forceinline__ cpx<T> zero() { return mk(T(0), T(0)); }

// Launch helpers defined in the individual translation units.  All take the
// stream explicitly and return hipError_t of the launch.
struct FftPlan1D {
  int n;                 // transform length (power of two)
  void* tw;              // device twiddle table exp(-2 pi i k / n), k < n
};

// Lane moves that stay in the vector unit (DPP, no LDS round trip): within
// rows of 16 lanes, lane i takes lane i + d (DOWN) or i - d (UP) of its row,
// 0 when that lane is outside the row; WAVE_DOWN1 / WAVE_UP1 move by one
// lane across the whole wave (0 past either end); SWAP1 exchanges the
// values of lanes 2j and 2j + 1.  readlane broadcasts one lane's value.
// Doubles move as two 32-bit halves.
enum : int {
  DPP_ROW_DOWN = 0x100,
  DPP_ROW_UP = 0x110,
  DPP_WAVE_DOWN1 = 0x130,
  DPP_WAVE_UP1 = 0x138,
  DPP_SWAP1 = 0xB1          // quad_perm (1, 0, 3, 2)
};

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL, typename T>
__device__ __forceinline__ cpx<T> dpp_move(cpx<T> v) {
  return mk(dpp_move<CTRL>(v.x), dpp_move<CTRL>(v.y));
}
__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ float lane_value(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
template <typename T>
__device__ __forceinline__ cpx<T> lane_value(cpx<T> v, int lane) {
  return mk(lane_value(v.x, lane), lane_value(v.y, lane));
}

}  // namespace fvim
