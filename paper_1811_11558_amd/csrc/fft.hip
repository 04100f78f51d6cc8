// In-plane transforms of the layered fields (the DFT of Sec. 3.1, eqn dft),
// written for gfx950: every kernel stages a batch of 1D transforms through
// LDS and runs a self-sorting (Stockham) radix-4 FFT with one radix-2 stage
// when log2(n) is odd.  Global memory is touched once on the way in and once
// on the way out, with the layouts chosen so both sides are contiguous runs:
//
//   real field        [P][ny][nx]          (P planes = components x layers)
//   x-spectrum   X    [P][nx/2+1][ny]      written by x_r2c, read by y_fwd
//   mode-major   S    [nx/2+1][ny][P]      written by y_fwd, read by the
//                                          depth pass (all planes of one
//                                          mode are contiguous)
//
// and the mirror images for the inverse.  Real transforms of length nx are
// done two rows at a time as one complex transform (z = a + i b).
// Forward transforms are unnormalised; the depth pass applies 1/(nx ny).
#include "common.hpp"
#include "kernels.hpp"

namespace fvim {

namespace {

constexpr int NT = 256;   // threads per block of every FFT kernel

template <typename T, bool INV>
__device__ __forceinline__ cpx<T> twid(const cpx<T>* __restrict__ tw, int idx) {
  cpx<T> w = tw[idx];
  if (INV) w.y = -w.y;
  return w;
}

// B transforms of length n held at buf[b * ld + k]; ELEMS >= B * n bounds
// the per-thread register staging.  Must be called by all NT threads.
template <typename T, bool INV, int ELEMS>
__device__ void lds_fft(cpx<T>* buf, int n, int ld, int B, const cpx<T>* __restrict__ tw) {
  const int tid = threadIdx.x;
  int ns = 1;
  int lg = 31 - __clz(n);
  if (lg & 1) {                       // radix-2 stage, trivial twiddles
    constexpr int MB = (ELEMS / 2 + NT - 1) / NT;
    const int half = n >> 1;
    const int nb = B * half;
    cpx<T> v0[MB], v1[MB];
#pragma unroll
    for (int u = 0; u < MB; ++u) {
      int j = tid + u * NT;
      if (j < nb) {
        int b = j / half, jj = j - b * half;
        v0[u] = buf[b * ld + jj];
        v1[u] = buf[b * ld + jj + half];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MB; ++u) {
      int j = tid + u * NT;
      if (j < nb) {
        int b = j / half, jj = j - b * half;
        buf[b * ld + 2 * jj] = add(v0[u], v1[u]);
        buf[b * ld + 2 * jj + 1] = sub(v0[u], v1[u]);
      }
    }
    __syncthreads();
    ns = 2;
  }
  constexpr int MB4 = (ELEMS / 4 + NT - 1) / NT;
  const int quarter = n >> 2;
  const int nb4 = B * quarter;
  while (ns < n) {
    cpx<T> v[MB4][4];
    const int tstep = n / (4 * ns);
#pragma unroll
    for (int u = 0; u < MB4; ++u) {
      int j = tid + u * NT;
      if (j < nb4) {
        int b = j / quarter, jj = j - b * quarter;
        const cpx<T>* src = buf + b * ld + jj;
        v[u][0] = src[0];
        v[u][1] = src[quarter];
        v[u][2] = src[2 * quarter];
        v[u][3] = src[3 * quarter];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MB4; ++u) {
      int j = tid + u * NT;
      if (j < nb4) {
        int b = j / quarter, jj = j - b * quarter;
        int k = jj % ns;
        cpx<T> a0 = v[u][0];
        cpx<T> a1 = v[u][1], a2 = v[u][2], a3 = v[u][3];
        if (k != 0) {
          a1 = mul(a1, twid<T, INV>(tw, k * tstep));
          a2 = mul(a2, twid<T, INV>(tw, 2 * k * tstep));
          a3 = mul(a3, twid<T, INV>(tw, 3 * k * tstep));
        }
        cpx<T> s02 = add(a0, a2), d02 = sub(a0, a2);
        cpx<T> s13 = add(a1, a3), d13 = sub(a1, a3);
        // forward: y1 = d02 - i d13, y3 = d02 + i d13 (conjugate for inverse)
        cpx<T> id13 = INV ? mul_i(d13) : mul_mi(d13);
        int o = b * ld + (jj / ns) * ns * 4 + k;
        buf[o] = add(s02, s13);
        buf[o + ns] = add(d02, id13);
        buf[o + 2 * ns] = sub(s02, s13);
        buf[o + 3 * ns] = sub(d02, id13);
      }
    }
    __syncthreads();
    ns *= 4;
  }
}

// Rows of nx reals -> half spectra.  Block = R consecutive rows of one
// plane (R even, R | ny).  Output X[(plane * kxh + k) * ny + y].
template <typename T, int ELEMS>
__global__ __launch_bounds__(NT) void k_x_r2c(const double* __restrict__ in, cpx<T>* __restrict__ out,
                                             int nx, int ny, int R, const cpx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  const int ld = nx;
  const size_t row0 = (size_t)blockIdx.x * R;
  const size_t plane = row0 / ny;
  const int y0 = (int)(row0 - plane * ny);
  const int kxh = nx / 2 + 1;
  const int tot = R * nx;
  for (int i = threadIdx.x; i < tot; i += NT) {
    int r = i / nx, x = i - r * nx;
    T v = (T)in[(row0 + r) * nx + x];
    cpx<T>& d = buf[(r >> 1) * ld + x];
    if (r & 1) d.y = v; else d.x = v;
  }
  __syncthreads();
  lds_fft<T, false, ELEMS>(buf, nx, ld, R / 2, tw);
  const int tot2 = kxh * R;
  for (int i = threadIdx.x; i < tot2; i += NT) {
    int yl = i % R, k = i / R;
    int p = yl >> 1;
    cpx<T> Z = buf[p * ld + k];
    cpx<T> Zc = buf[p * ld + ((nx - k) & (nx - 1))];
    cpx<T> X;
    if ((yl & 1) == 0) X = mk(T(0.5) * (Z.x + Zc.x), T(0.5) * (Z.y - Zc.y));
    else X = mk(T(0.5) * (Z.y + Zc.y), T(0.5) * (Zc.x - Z.x));
    out[(plane * kxh + k) * ny + y0 + yl] = X;
  }
}

// Forward column transform: X[p][kx][y] -> S[kx][ky][p]; block = B planes of one kx.
template <typename T, int ELEMS>
__global__ __launch_bounds__(NT) void k_y_fwd(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
                                             int ny, int kxh, int NP, int B, int ld,
                                             const cpx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  const int npb = (NP + B - 1) / B;
  const int kx = blockIdx.x / npb;
  const int p0 = (blockIdx.x - kx * npb) * B;
  const int tot = B * ny;
  for (int i = threadIdx.x; i < tot; i += NT) {
    int b = i / ny, y = i - b * ny;
    int p = p0 + b;
    buf[b * ld + y] = (p < NP) ? in[((size_t)p * kxh + kx) * ny + y] : zero<T>();
  }
  __syncthreads();
  lds_fft<T, false, ELEMS>(buf, ny, ld, B, tw);
  for (int i = threadIdx.x; i < tot; i += NT) {
    int b = i % B, ky = i / B;
    int p = p0 + b;
    if (p < NP) out[((size_t)kx * ny + ky) * NP + p] = buf[b * ld + ky];
  }
}

// Inverse column transform: S[kx][ky][p] -> X[p][kx][y].
template <typename T, int ELEMS>
__global__ __launch_bounds__(NT) void k_y_inv(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
                                             int ny, int kxh, int NP, int B, int ld,
                                             const cpx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  const int npb = (NP + B - 1) / B;
  const int kx = blockIdx.x / npb;
  const int p0 = (blockIdx.x - kx * npb) * B;
  const int tot = B * ny;
  for (int i = threadIdx.x; i < tot; i += NT) {
    int b = i % B, ky = i / B;
    int p = p0 + b;
    buf[b * ld + ky] = (p < NP) ? in[((size_t)kx * ny + ky) * NP + p] : zero<T>();
  }
  __syncthreads();
  lds_fft<T, true, ELEMS>(buf, ny, ld, B, tw);
  for (int i = threadIdx.x; i < tot; i += NT) {
    int b = i / ny, y = i - b * ny;
    int p = p0 + b;
    if (p < NP) out[((size_t)p * kxh + kx) * ny + y] = buf[b * ld + y];
  }
}

// Half spectra -> rows of nx reals, two rows per complex transform.  Plane p
// of the input goes to the output segment that contains it.
template <typename T, int ELEMS>
__global__ __launch_bounds__(NT) void k_x_c2r(const cpx<T>* __restrict__ in, OutSegments seg,
                                             int nx, int ny, int R, double scale,
                                             const cpx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  const int ld = nx;
  const size_t row0 = (size_t)blockIdx.x * R;
  const int plane = (int)(row0 / ny);
  const int y0 = (int)(row0 - (size_t)plane * ny);
  const int kxh = nx / 2 + 1;
  const int hp = R / 2;
  const int tot = kxh * hp;
  const int nyq = nx / 2;
  for (int i = threadIdx.x; i < tot; i += NT) {
    int pr = i % hp, k = i / hp;
    size_t a = ((size_t)plane * kxh + k) * ny + y0 + 2 * pr;
    cpx<T> X0 = in[a], X1 = in[a + 1];
    if (k == 0 || k == nyq) {
      buf[pr * ld + k] = mk(X0.x, X1.x);
    } else {
      buf[pr * ld + k] = mk(X0.x - X1.y, X0.y + X1.x);
      buf[pr * ld + nx - k] = mk(X0.x + X1.y, X1.x - X0.y);
    }
  }
  __syncthreads();
  lds_fft<T, true, ELEMS>(buf, nx, ld, hp, tw);
  int s = 0;
  while (s + 1 < seg.n && plane >= seg.first[s + 1]) ++s;
  double* dst = seg.ptr[s];
  const size_t lp = (size_t)(plane - seg.first[s]);
  const int tot2 = R * nx;
  for (int i = threadIdx.x; i < tot2; i += NT) {
    int r = i / nx, x = i - r * nx;
    cpx<T> v = buf[(r >> 1) * ld + x];
    T val = (r & 1) ? v.y : v.x;
    dst[(lp * ny + y0 + r) * nx + x] = (double)val * scale;
  }
}

template <typename T>
constexpr int elems_for() { return sizeof(T) == 8 ? 4096 : 8192; }

constexpr size_t LDS_BUDGET = 65536;   // bytes of LDS per block

// Rows per block of the x kernels: R/2 unpadded sequences of length nx in
// the budget, R a power of two dividing ny.
int rows_per_block(int nx, int ny, int elems) {
  int r = (2 * elems) / nx;
  if (r > ny) r = ny;
  if (r < 2) r = 2;
  return r;
}

// Columns per block of the y kernels: B sequences of length ny with a
// one-element pad per sequence within the budget.
int cols_per_block(int ny, int elems, size_t csize) {
  int b = (int)(LDS_BUDGET / ((size_t)(ny + 1) * csize));
  if (b > elems / ny) b = elems / ny;
  if (b < 1) b = 1;
  return b;
}

// Leading dimension of the y tiles: padded by one element unless that would
// exceed the budget (single column of the longest transform).
int col_ld(int ny, int B, size_t csize) {
  return ((size_t)B * (ny + 1) * csize <= LDS_BUDGET) ? ny + 1 : ny;
}

}  // namespace

template <typename T>
hipError_t launch_x_r2c(const double* in, cpx<T>* out, int nx, int ny, size_t nplanes,
                        const cpx<T>* tw, hipStream_t st) {
  constexpr int EL = elems_for<T>();
  int R = rows_per_block(nx, ny, EL);
  size_t rows = nplanes * (size_t)ny;
  size_t lds = (size_t)(R / 2) * nx * sizeof(cpx<T>);
  hipLaunchKernelGGL((k_x_r2c<T, EL>), dim3((unsigned)(rows / R)), dim3(NT), lds, st, in, out, nx, ny,
                     R, tw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_y_fwd(const cpx<T>* in, cpx<T>* out, int ny, int kxh, int NP, const cpx<T>* tw,
                        hipStream_t st) {
  constexpr int EL = elems_for<T>();
  int B = cols_per_block(ny, EL, sizeof(cpx<T>));
  if (B > NP) B = NP;
  int npb = (NP + B - 1) / B;
  const int ld = col_ld(ny, B, sizeof(cpx<T>));
  size_t lds = (size_t)B * ld * sizeof(cpx<T>);
  hipLaunchKernelGGL((k_y_fwd<T, EL>), dim3((unsigned)(kxh * npb)), dim3(NT), lds, st, in, out, ny, kxh,
                     NP, B, ld, tw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_y_inv(const cpx<T>* in, cpx<T>* out, int ny, int kxh, int NP, const cpx<T>* tw,
                        hipStream_t st) {
  constexpr int EL = elems_for<T>();
  int B = cols_per_block(ny, EL, sizeof(cpx<T>));
  if (B > NP) B = NP;
  int npb = (NP + B - 1) / B;
  const int ld = col_ld(ny, B, sizeof(cpx<T>));
  size_t lds = (size_t)B * ld * sizeof(cpx<T>);
  hipLaunchKernelGGL((k_y_inv<T, EL>), dim3((unsigned)(kxh * npb)), dim3(NT), lds, st, in, out, ny, kxh,
                     NP, B, ld, tw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_x_c2r(const cpx<T>* in, const OutSegments& seg, int nx, int ny, size_t nplanes,
                        double scale, const cpx<T>* tw, hipStream_t st) {
  constexpr int EL = elems_for<T>();
  int R = rows_per_block(nx, ny, EL);
  size_t rows = nplanes * (size_t)ny;
  size_t lds = (size_t)(R / 2) * nx * sizeof(cpx<T>);
  hipLaunchKernelGGL((k_x_c2r<T, EL>), dim3((unsigned)(rows / R)), dim3(NT), lds, st, in, seg, nx, ny, R,
                     scale, tw);
  return hipGetLastError();
}

template hipError_t launch_x_r2c<double>(const double*, cpx<double>*, int, int, size_t, const cpx<double>*,
                                         hipStream_t);
template hipError_t launch_x_r2c<float>(const double*, cpx<float>*, int, int, size_t, const cpx<float>*,
                                        hipStream_t);
template hipError_t launch_y_fwd<double>(const cpx<double>*, cpx<double>*, int, int, int, const cpx<double>*,
                                         hipStream_t);
template hipError_t launch_y_fwd<float>(const cpx<float>*, cpx<float>*, int, int, int, const cpx<float>*,
                                        hipStream_t);
template hipError_t launch_y_inv<double>(const cpx<double>*, cpx<double>*, int, int, int, const cpx<double>*,
                                         hipStream_t);
template hipError_t launch_y_inv<float>(const cpx<float>*, cpx<float>*, int, int, int, const cpx<float>*,
                                        hipStream_t);
template hipError_t launch_x_c2r<double>(const cpx<double>*, const OutSegments&, int, int, size_t, double,
                                         const cpx<double>*, hipStream_t);
template hipError_t launch_x_c2r<float>(const cpx<float>*, const OutSegments&, int, int, size_t, double,
                                        const cpx<float>*, hipStream_t);

}  // namespace fvim
