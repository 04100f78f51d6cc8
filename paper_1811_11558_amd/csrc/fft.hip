// In-plane transforms of the layered fields (the DFT of Sec. 3.1, eqn dft),
// written for gfx950: every kernel stages a batch of 1D transforms through
// LDS and runs a self-sorting (Stockham) FFT of radix 4 (one radix-2 stage
// when log2(n) is odd) or radix 8 (one radix-2 or radix-4 stage first).
// Global memory is touched once on the way in and once on the way out, with
// the layouts chosen so both sides are contiguous runs:
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
//
// The LDS tile (half, default or twice the default) and the radix are
// choices of each launch (FftChoice), timed by the context's tuner for
// lengths 2^5 .. 2^10; other lengths use the default.  Kernels over several
// grids (XformBatch) run the default choice of each grid's length.
#include <algorithm>

#include "common.hpp"
#include "fft_dev.hpp"
#include "kernels.hpp"

namespace fvim {

namespace {
// ---------------------------------------------------- single-grid kernels
template <typename T, int LOGN, int TILE>
__host__ __device__ constexpr int r2c_lds_elems() {
  return r2c_seq<T>(1 << LOGN, TILE) * ((1 << LOGN) + 1);
}
template <typename T, int LOGN, int TILE>
__host__ __device__ constexpr int c2r_lds_elems() {
  return c2r_seq<T>(1 << LOGN, TILE) * ((1 << LOGN) + 1);
}
template <typename T, int LOGN, int TILE>
__host__ __device__ constexpr int col_lds_elems() {
  return col_batch<T>(1 << LOGN, TILE) * ((1 << LOGN) + 1);
}

template <typename T, int LOGN, bool NTL, int TILE, int RADIX>
__global__ __launch_bounds__(NT) void k_x_r2c(InSegments seg, cpx<T>* __restrict__ out, int ny, int R,
                                             const cpx<T>* __restrict__ tw, double* __restrict__ bsum,
                                             LayerSkip skip) {
  __shared__ cpx<T> buf[r2c_lds_elems<T, LOGN, TILE>()];
  __shared__ double red[NT / 64];
  x_r2c_body<T, LOGN, NTL, TILE, RADIX>(buf, red, blockIdx.x, seg, out, ny, R, tw, bsum, skip);
}

template <typename T, int LOGN, bool NTL, int TILE, int RADIX>
__global__ __launch_bounds__(NT) void k_y_fwd(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, int kxh,
                                             int NP, int ldp, const cpx<T>* __restrict__ tw, LayerSkip skip) {
  __shared__ cpx<T> buf[col_lds_elems<T, LOGN, TILE>()];
  y_fwd_body<T, LOGN, NTL, TILE, RADIX>(buf, xcd_block(), in, out, kxh, NP, ldp, tw, skip);
}

template <typename T, int LOGN, bool NTL, int TILE, int RADIX>
__global__ __launch_bounds__(NT) void k_y_inv(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, int kxh,
                                             int NP, int ldp, const cpx<T>* __restrict__ tw) {
  __shared__ cpx<T> buf[col_lds_elems<T, LOGN, TILE>()];
  y_inv_body<T, LOGN, NTL, TILE, RADIX>(buf, xcd_block(), in, out, kxh, NP, ldp, tw);
}

template <typename T, int LOGN, int TILE, int RADIX>
__global__ __launch_bounds__(NT) void k_x_c2r(const cpx<T>* __restrict__ in, OutSegments seg, int ny, int R,
                                             double scale, const cpx<T>* __restrict__ tw,
                                             const double* __restrict__ padd, ResidEpilogue ep, int nts) {
  __shared__ cpx<T> buf[c2r_lds_elems<T, LOGN, TILE>()];
  __shared__ double red[NT / 64];
  // the last planes first: the inverse column transform wrote them last
  x_c2r_body<T, LOGN, TILE, RADIX>(buf, red, (int)(gridDim.x - 1 - blockIdx.x), in, seg, ny, R, scale, tw, padd, ep,
                                   nts != 0);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_x_r2c_batch(XformBatch b) {
  __shared__ double red[NT / 64];
  x_r2c_batch_block<T>(b, (int)blockIdx.x, red);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_y_fwd_batch(XformBatch b) {
  y_fwd_batch_block<T>(b, xcd_block());
}

template <typename T>
__global__ __launch_bounds__(NT) void k_y_inv_batch(XformBatch b) {
  y_inv_batch_block<T>(b, xcd_block());
}

template <typename T>
__global__ __launch_bounds__(NT) void k_x_c2r_batch(XformBatch b) {
  __shared__ double red[NT / 64];
  x_c2r_batch_block<T>(b, (int)blockIdx.x, red);
}

// -------------------------------------------------------------- launches
// R of a row kernel launch: 2 SEQ rows, or the whole plane when it is shorter
int rows_per_block(int seq, int ny) { return 2 * seq < ny ? 2 * seq : ny; }

int ilog2(int n) { return 31 - __builtin_clz((unsigned)n); }

bool fft_tunable(int logn) { return logn >= FFT_TUNE_MIN_LOGN && logn <= FFT_TUNE_MAX_LOGN; }

// Runtime tile -> compile-time tile of a row kernel's SEQ (or a column
// kernel's B) for a length 2^L.
template <typename T, int L>
int r2c_seq_rt(int tile) {
  return tile == 0 ? r2c_seq<T>(1 << L, 0) : (tile == 2 ? r2c_seq<T>(1 << L, 2) : r2c_seq<T>(1 << L, 1));
}
template <typename T, int L>
int c2r_seq_rt(int tile) {
  return tile == 0 ? c2r_seq<T>(1 << L, 0) : (tile == 2 ? c2r_seq<T>(1 << L, 2) : c2r_seq<T>(1 << L, 1));
}

#define FVIM_LOGN_SWITCH(logn, CALL) \
  switch (logn) {                    \
    case 2: CALL(2); break;          \
    case 3: CALL(3); break;          \
    case 4: CALL(4); break;          \
    case 5: CALL(5); break;          \
    case 6: CALL(6); break;          \
    case 7: CALL(7); break;          \
    case 8: CALL(8); break;          \
    case 9: CALL(9); break;          \
    case 10: CALL(10); break;        \
    case 11: CALL(11); break;        \
    case 12: CALL(12); break;        \
    default: return hipErrorInvalidValue; \
  }

// Calls GO<TILE, RADIX>() of the launcher struct for the effective choice:
// the six (tile, radix) variants exist for tunable lengths only.
template <int L, typename F>
hipError_t with_choice(FftChoice ch, F& f) {
  if constexpr (L >= FFT_TUNE_MIN_LOGN && L <= FFT_TUNE_MAX_LOGN) {
    if (ch.radix == 8) {
      if (ch.tile == 0) return f.template go<L, 0, 8>();
      if (ch.tile == 2) return f.template go<L, 2, 8>();
      return f.template go<L, 1, 8>();
    }
    if (ch.tile == 0) return f.template go<L, 0, 4>();
    if (ch.tile == 2) return f.template go<L, 2, 4>();
  }
  return f.template go<L, 1, 4>();
}

template <typename T>
struct R2CLaunch {
  const InSegments& seg;
  cpx<T>* out;
  int ny;
  size_t nplanes;
  const cpx<T>* tw;
  hipStream_t st;
  double* bsum;
  bool stream_in;
  const LayerSkip& skip;
  template <int L, int TILE, int RADIX>
  hipError_t go() {
    const int R = rows_per_block(r2c_seq<T>(1 << L, TILE), ny);
    const dim3 grid((unsigned)(nplanes * (size_t)ny / R));
    if (stream_in)
      hipLaunchKernelGGL((k_x_r2c<T, L, true, TILE, RADIX>), grid, dim3(NT), 0, st, seg, out, ny, R, tw, bsum, skip);
    else
      hipLaunchKernelGGL((k_x_r2c<T, L, false, TILE, RADIX>), grid, dim3(NT), 0, st, seg, out, ny, R, tw, bsum, skip);
    return hipGetLastError();
  }
};

template <typename T, bool FWD>
struct ColLaunch {
  const cpx<T>* in;
  cpx<T>* out;
  int kxh, NP, ldp;
  const cpx<T>* tw;
  hipStream_t st;
  bool stream_in;
  const LayerSkip& skip;
  template <int L, int TILE, int RADIX>
  hipError_t go() {
    constexpr int B = col_batch<T>(1 << L, TILE);
    const dim3 grid((unsigned)(kxh * ((NP + B - 1) / B)));
    if (FWD) {
      if (stream_in)
        hipLaunchKernelGGL((k_y_fwd<T, L, true, TILE, RADIX>), grid, dim3(NT), 0, st, in, out, kxh, NP, ldp, tw, skip);
      else
        hipLaunchKernelGGL((k_y_fwd<T, L, false, TILE, RADIX>), grid, dim3(NT), 0, st, in, out, kxh, NP, ldp, tw,
                           skip);
    } else {
      if (stream_in)
        hipLaunchKernelGGL((k_y_inv<T, L, true, TILE, RADIX>), grid, dim3(NT), 0, st, in, out, kxh, NP, ldp, tw);
      else
        hipLaunchKernelGGL((k_y_inv<T, L, false, TILE, RADIX>), grid, dim3(NT), 0, st, in, out, kxh, NP, ldp, tw);
    }
    return hipGetLastError();
  }
};

template <typename T>
struct C2RLaunch {
  const cpx<T>* in;
  const OutSegments& seg;
  int ny;
  size_t nplanes;
  double scale;
  const cpx<T>* tw;
  hipStream_t st;
  const double* padd;
  const ResidEpilogue& ep;
  bool stream_out;
  template <int L, int TILE, int RADIX>
  hipError_t go() {
    const int R = rows_per_block(c2r_seq<T>(1 << L, TILE), ny);
    const dim3 grid((unsigned)(nplanes * (size_t)ny / R));
    hipLaunchKernelGGL((k_x_c2r<T, L, TILE, RADIX>), grid, dim3(NT), 0, st, in, seg, ny, R, scale, tw, padd, ep,
                       stream_out ? 1 : 0);
    return hipGetLastError();
  }
};

template <typename T, bool R2C>
struct SeqOf {
  template <int L, int TILE, int RADIX>
  hipError_t go() {
    seq = R2C ? r2c_seq<T>(1 << L, TILE) : c2r_seq<T>(1 << L, TILE);
    return hipSuccess;
  }
  int seq = 0;
};

template <typename T, bool R2C>
int row_seq_of(int nx, FftChoice ch) {
  SeqOf<T, R2C> f;
  auto run = [&]() -> hipError_t {
#define CALL(L) return with_choice<L>(ch, f)
    FVIM_LOGN_SWITCH(ilog2(nx), CALL)
#undef CALL
    return hipErrorInvalidValue;
  };
  run();
  return f.seq;
}

}  // namespace

FftChoice fft_effective(int logn, FftChoice ch) {
  if (!fft_tunable(logn) || (ch.radix != 4 && ch.radix != 8) || ch.tile < 0 || ch.tile > 2) return FftChoice{};
  return ch;
}

template <typename T>
int x_r2c_blocks_per_plane(int nx, int ny, FftChoice ch) {
  return ny / rows_per_block(row_seq_of<T, true>(nx, fft_effective(ilog2(nx), ch)), ny);
}

template <typename T>
int x_r2c_max_blocks_per_plane(int nx, int ny) {
  int m = 0;
  for (int t = 0; t < 3; ++t) m = std::max(m, x_r2c_blocks_per_plane<T>(nx, ny, FftChoice{t, 4}));
  return m;
}

template <typename T>
hipError_t launch_x_r2c(const InSegments& seg, cpx<T>* out, int nx, int ny, size_t nplanes, const cpx<T>* tw,
                        hipStream_t st, double* bsum, bool stream_in, const LayerSkip& skip, FftChoice ch) {
  if (seg.n < 1 || seg.n > 2 || seg.first[0] != 0) return hipErrorInvalidValue;
  R2CLaunch<T> f{seg, out, ny, nplanes, tw, st, bsum, stream_in, skip};
  ch = fft_effective(ilog2(nx), ch);
#define CALL(L) return with_choice<L>(ch, f)
  FVIM_LOGN_SWITCH(ilog2(nx), CALL)
#undef CALL
}

template <typename T>
hipError_t launch_x_r2c(const double* in, cpx<T>* out, int nx, int ny, size_t nplanes, const cpx<T>* tw,
                        hipStream_t st, double* bsum, bool stream_in) {
  InSegments seg;
  seg.n = 1;
  seg.first[0] = seg.first[1] = 0;
  seg.ptr[0] = seg.ptr[1] = in;
  return launch_x_r2c<T>(seg, out, nx, ny, nplanes, tw, st, bsum, stream_in, LayerSkip{}, FftChoice{});
}

template <typename T>
hipError_t launch_y_fwd(const cpx<T>* in, cpx<T>* out, int ny, int kxh, int NP, int ldp, const cpx<T>* tw,
                        hipStream_t st, bool stream_in, const LayerSkip& skip, FftChoice ch) {
  if (ldp < NP) return hipErrorInvalidValue;
  ColLaunch<T, true> f{in, out, kxh, NP, ldp, tw, st, stream_in, skip};
  ch = fft_effective(ilog2(ny), ch);
#define CALL(L) return with_choice<L>(ch, f)
  FVIM_LOGN_SWITCH(ilog2(ny), CALL)
#undef CALL
}

template <typename T>
hipError_t launch_y_inv(const cpx<T>* in, cpx<T>* out, int ny, int kxh, int NP, int ldp, const cpx<T>* tw,
                        hipStream_t st, bool stream_in, FftChoice ch) {
  if (ldp < NP) return hipErrorInvalidValue;
  const LayerSkip none{};
  ColLaunch<T, false> f{in, out, kxh, NP, ldp, tw, st, stream_in, none};
  ch = fft_effective(ilog2(ny), ch);
#define CALL(L) return with_choice<L>(ch, f)
  FVIM_LOGN_SWITCH(ilog2(ny), CALL)
#undef CALL
}

template <typename T>
hipError_t launch_x_c2r(const cpx<T>* in, const OutSegments& seg, int nx, int ny, size_t nplanes,
                        double scale, const cpx<T>* tw, hipStream_t st, const double* padd,
                        const ResidEpilogue& ep, bool stream_out, FftChoice ch) {
  // the epilogue reads its fields at the output's own offsets: one segment
  // holding the 6 nz strain planes from plane 0
  if (ep.x && (seg.n != 1 || seg.first[0] != 0 || !ep.part || ep.nz < 1 || nplanes != (size_t)6 * ep.nz))
    return hipErrorInvalidValue;
  C2RLaunch<T> f{in, seg, ny, nplanes, scale, tw, st, padd, ep, stream_out};
  ch = fft_effective(ilog2(nx), ch);
#define CALL(L) return with_choice<L>(ch, f)
  FVIM_LOGN_SWITCH(ilog2(nx), CALL)
#undef CALL
}

template <typename T>
int x_c2r_blocks(int nx, int ny, size_t nplanes, FftChoice ch) {
  return (int)(nplanes * (size_t)ny / rows_per_block(row_seq_of<T, false>(nx, fft_effective(ilog2(nx), ch)), ny));
}

template <typename T>
int x_c2r_max_blocks(int nx, int ny, size_t nplanes) {
  int m = 0;
  for (int t = 0; t < 3; ++t) m = std::max(m, x_c2r_blocks<T>(nx, ny, nplanes, FftChoice{t, 4}));
  return m;
}

// ------------------------------------------------- launches over grids
namespace {

// block count and LDS bytes of one grid's part of a batched launch (the
// default tile), and its rows per block (row kernels)
template <typename T>
struct BatchGeom {
  int blocks = 0, R = 0;
  size_t lds = 0;
};

template <typename T>
BatchGeom<T> geom_r2c(int logn, int ny, int nplanes) {
  BatchGeom<T> g;
  const int n = 1 << logn;
  const int seq = r2c_seq<T>(n, 1);
  g.R = rows_per_block(seq, ny);
  g.blocks = nplanes * ny / g.R;
  g.lds = (size_t)seq * (n + 1) * sizeof(cpx<T>);
  return g;
}
template <typename T>
BatchGeom<T> geom_c2r(int logn, int ny, int nplanes) {
  BatchGeom<T> g;
  const int n = 1 << logn;
  const int seq = c2r_seq<T>(n, 1);
  g.R = rows_per_block(seq, ny);
  g.blocks = nplanes * ny / g.R;
  g.lds = (size_t)seq * (n + 1) * sizeof(cpx<T>);
  return g;
}
template <typename T>
BatchGeom<T> geom_col(int logn, int kxh, int NP) {
  BatchGeom<T> g;
  const int n = 1 << logn;
  const int B = col_batch<T>(n, 1);
  g.blocks = kxh * ((NP + B - 1) / B);
  g.lds = (size_t)B * (n + 1) * sizeof(cpx<T>);
  return g;
}

}  // namespace

// kind: 0 x_r2c, 1 y_fwd, 2 y_inv, 3 x_c2r.  The host fills every grid's
// fields but first[]; logn is the transform length of the kernel (nx for
// the row kernels, ny for the column kernels), nplanes[c] its plane count.
template <typename T>
size_t xform_batch_prepare(int kind, XformBatch& b) {
  if (b.n < 1 || b.n > XFORM_BATCH_MAX || kind < 0 || kind > 3) return 0;
  size_t lds = 0;
  b.first[0] = 0;
  for (int c = 0; c < b.n; ++c) {
    if (b.logn[c] < 2 || b.logn[c] > XFORM_BATCH_MAX_LOGN) return 0;
    BatchGeom<T> g = kind == 0 ? geom_r2c<T>(b.logn[c], b.ny[c], b.NP[c])
                     : kind == 3 ? geom_c2r<T>(b.logn[c], b.ny[c], b.NP[c])
                                 : geom_col<T>(b.logn[c], b.kxh[c], b.NP[c]);
    b.R[c] = g.R;
    b.first[c + 1] = b.first[c] + g.blocks;
    lds = std::max(lds, g.lds);
  }
  return lds;
}

template <typename T>
hipError_t launch_xform_batch(int kind, XformBatch& b, hipStream_t st) {
  if (b.n < 1 || b.n > XFORM_BATCH_MAX) return hipErrorInvalidValue;
  size_t lds = 0;
  b.first[0] = 0;
  for (int c = 0; c < b.n; ++c) {
    if (b.logn[c] < 2 || b.logn[c] > XFORM_BATCH_MAX_LOGN) return hipErrorInvalidValue;
    BatchGeom<T> g = kind == 0 ? geom_r2c<T>(b.logn[c], b.ny[c], b.NP[c])
                     : kind == 3 ? geom_c2r<T>(b.logn[c], b.ny[c], b.NP[c])
                                 : geom_col<T>(b.logn[c], b.kxh[c], b.NP[c]);
    b.R[c] = g.R;
    b.first[c + 1] = b.first[c] + g.blocks;
    lds = std::max(lds, g.lds);
  }
  const dim3 grid((unsigned)b.first[b.n]);
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_x_r2c_batch<T>, grid, dim3(NT), lds, st, b); break;
    case 1: hipLaunchKernelGGL(k_y_fwd_batch<T>, grid, dim3(NT), lds, st, b); break;
    case 2: hipLaunchKernelGGL(k_y_inv_batch<T>, grid, dim3(NT), lds, st, b); break;
    case 3: hipLaunchKernelGGL(k_x_c2r_batch<T>, grid, dim3(NT), lds, st, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// blocks per plane of the batched x_r2c (the float32 mean-mode sums)
template <typename T>
int x_r2c_batch_blocks_per_plane(int nx, int ny) {
  return ny / rows_per_block(r2c_seq<T>(nx, 1), ny);
}

#define FVIM_INST(T)                                                                                            \
  template int x_r2c_blocks_per_plane<T>(int, int, FftChoice);                                                  \
  template int x_r2c_max_blocks_per_plane<T>(int, int);                                                         \
  template int x_r2c_batch_blocks_per_plane<T>(int, int);                                                       \
  template hipError_t launch_x_r2c<T>(const InSegments&, cpx<T>*, int, int, size_t, const cpx<T>*, hipStream_t, \
                                      double*, bool, const LayerSkip&, FftChoice);                              \
  template hipError_t launch_x_r2c<T>(const double*, cpx<T>*, int, int, size_t, const cpx<T>*, hipStream_t,     \
                                      double*, bool);                                                           \
  template hipError_t launch_y_fwd<T>(const cpx<T>*, cpx<T>*, int, int, int, int, const cpx<T>*, hipStream_t,   \
                                      bool, const LayerSkip&, FftChoice);                                       \
  template hipError_t launch_y_inv<T>(const cpx<T>*, cpx<T>*, int, int, int, int, const cpx<T>*, hipStream_t,   \
                                      bool, FftChoice);                                                         \
  template hipError_t launch_x_c2r<T>(const cpx<T>*, const OutSegments&, int, int, size_t, double,              \
                                      const cpx<T>*, hipStream_t, const double*, const ResidEpilogue&, bool,    \
                                      FftChoice);                                                               \
  template int x_c2r_blocks<T>(int, int, size_t, FftChoice);                                                    \
  template int x_c2r_max_blocks<T>(int, int, size_t);                                                           \
  template hipError_t launch_xform_batch<T>(int, XformBatch&, hipStream_t);                                      \
  template size_t xform_batch_prepare<T>(int, XformBatch&);
FVIM_INST(double)
FVIM_INST(float)
#undef FVIM_INST

}  // namespace fvim
