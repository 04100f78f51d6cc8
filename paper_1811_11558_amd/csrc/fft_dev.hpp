// Device code of the in-plane transforms (constants, LDS Stockham stages and
// the row/column bodies, single-grid and batched).  Included by fft.hip and
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

template <typename T, bool INV>
__device__ __forceinline__ cpx<T> twid(const cpx<T>* __restrict__ tw, int idx) {
  cpx<T> w = tw[idx];
  if (INV) w.y = -w.y;
  return w;
}

// Complex elements of one block's LDS tile in the row kernels.  TILE picks
// half (0), the default (1) or twice (2) the default, which was chosen per
// kernel and precision by measurement on 256^2 x 64: a smaller tile lets
// more blocks share a CU (the forward transform gains: 16 KiB in float64),
// a larger one gives the inverse transform's strided reads longer runs
// (32 KiB in float64; 16 KiB in float32).  The tuner times the three.
__host__ __device__ constexpr int tile_scale(int base, int tile) {
  return tile == 0 ? base / 2 : (tile == 2 ? base * 2 : base);
}
template <typename T>
__host__ __device__ constexpr int r2c_tile_elems(int tile) { return tile_scale(sizeof(T) == 8 ? 1024 : 2048, tile); }
template <typename T>
__host__ __device__ constexpr int c2r_tile_elems(int tile) { return tile_scale(2048, tile); }
// Row pairs per block of a row kernel (R = 2 SEQ rows of length n).  The
// X[p][kx][y] side is touched in runs of R elements of one kx, so SEQ is the
// tile's share but at least what gives runs of ROW_RUN bytes, as far as the
// 160 KiB of LDS a block may use and a tile of 8192 elements (the loads of a
// whole tile are staged in registers) allow.  (At nx = 1024 in float64 a 16 KiB
// tile alone gives 2-row blocks, 32-byte runs and 1.5 TB/s.)
constexpr int ROW_RUN = 128;
__host__ __device__ constexpr int row_seq(int n, int csize, int tile) {
  int seq = tile / n;
  if (seq < 1) seq = 1;
  const int minseq = ROW_RUN / (2 * csize);
  if (seq < minseq) seq = minseq;
  while (seq > 1 && (seq * (n + 1) * csize > 160 * 1024 || seq * n > 8192)) seq /= 2;
  return seq;
}
template <typename T>
__host__ __device__ constexpr int r2c_seq(int n, int tile) {
  return row_seq(n, (int)sizeof(cpx<T>), r2c_tile_elems<T>(tile));
}
template <typename T>
__host__ __device__ constexpr int c2r_seq(int n, int tile) {
  return row_seq(n, (int)sizeof(cpx<T>), c2r_tile_elems<T>(tile));
}
// Columns (planes) per block of the column (y) kernels.  The mode-major side
// S[kx][ky][p] is touched in runs of B consecutive planes, so B is the tile's
// share (32 KiB by default; half or twice with TILE 0 or 2) unless that makes
// runs shorter than 64 bytes (ny >= 1024 in float64, >= 1024 in float32), in
// which case the tile grows up to the 160 KiB of LDS a block may use (powers
// of two).  Measured: 32-byte runs ran at 1.5 TB/s, 64-byte runs at 4.4 TB/s,
// and 64 KiB tiles with 256-byte runs were slower than 32 KiB ones at
// ny = 256.
__host__ __device__ constexpr int col_batch_bytes(int n, int csize, int tile) {
  int b = (tile_scale(32768, tile) / csize) / n;
  if (b < 1) b = 1;
  const int minb = 64 / csize;
  int maxb = 1;
  while (2 * maxb * (n + 1) * csize <= 160 * 1024) maxb *= 2;
  if (b < minb) b = minb < maxb ? minb : maxb;
  if (b > maxb) b = maxb;
  return b;
}
template <typename T>
__host__ __device__ constexpr int col_batch(int n, int tile) { return col_batch_bytes(n, (int)sizeof(cpx<T>), tile); }

__host__ __device__ constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// Radix-R butterfly (R = 2, 4, 8) of the DFT with kernel exp(-2 pi i / R)
// (its conjugate for INV), in place on a[0 .. R).
template <typename T, int R, bool INV>
__device__ __forceinline__ void butterfly(cpx<T>* a) {
  if constexpr (R == 2) {
    const cpx<T> a0 = a[0], a1 = a[1];
    a[0] = add(a0, a1);
    a[1] = sub(a0, a1);
  } else if constexpr (R == 4) {
    const cpx<T> s02 = add(a[0], a[2]), d02 = sub(a[0], a[2]);
    const cpx<T> s13 = add(a[1], a[3]), d13 = sub(a[1], a[3]);
    // forward: y1 = d02 - i d13, y3 = d02 + i d13 (conjugate for inverse)
    const cpx<T> id13 = INV ? mul_i(d13) : mul_mi(d13);
    a[0] = add(s02, s13);
    a[1] = add(d02, id13);
    a[2] = sub(s02, s13);
    a[3] = sub(d02, id13);
  } else {
    static_assert(R == 8, "radix 2, 4 or 8");
    // two length-4 transforms (even and odd inputs), then the odd ones
    // turned by w^p, w = exp(-+ 2 pi i / 8), and combined
    cpx<T> e[4] = {a[0], a[2], a[4], a[6]};
    cpx<T> o[4] = {a[1], a[3], a[5], a[7]};
    butterfly<T, 4, INV>(e);
    butterfly<T, 4, INV>(o);
    const T c = T(0.70710678118654752440084436210485);
    cpx<T> t1, t3;
    if (INV) {
      t1 = mk((o[1].x - o[1].y) * c, (o[1].x + o[1].y) * c);      // (1 + i)/sqrt2
      t3 = mk(-(o[3].x + o[3].y) * c, (o[3].x - o[3].y) * c);     // (-1 + i)/sqrt2
    } else {
      t1 = mk((o[1].x + o[1].y) * c, (o[1].y - o[1].x) * c);      // (1 - i)/sqrt2
      t3 = mk((o[3].y - o[3].x) * c, -(o[3].x + o[3].y) * c);     // (-1 - i)/sqrt2
    }
    const cpx<T> t2 = INV ? mul_i(o[2]) : mul_mi(o[2]);
    a[0] = add(e[0], o[0]);
    a[4] = sub(e[0], o[0]);
    a[1] = add(e[1], t1);
    a[5] = sub(e[1], t1);
    a[2] = add(e[2], t2);
    a[6] = sub(e[2], t2);
    a[3] = add(e[3], t3);
    a[7] = sub(e[3], t3);
  }
}

// One self-sorting (Stockham) radix-R stage of NB transforms of length
// N = 2^LOGN held at buf[b * ld + k] (NB <= NBMAX), for sub-transforms of
// length ns = 2^LS: butterfly j of a transform takes elements j + m N/R,
// turned by w^(m k N/(R ns)) with k = j mod ns, and writes them to
// (j / ns) ns R + k + m ns.  Called by all NT threads.
template <typename T, int LOGN, int NBMAX, bool INV, int R, int LS>
__device__ __forceinline__ void stockham_stage(cpx<T>* buf, int ld, int NB, const cpx<T>* __restrict__ tw) {
  constexpr int N = 1 << LOGN;
  constexpr int LR = ilog2c(R);
  constexpr int M = N / R;
  constexpr int ns = 1 << LS;
  constexpr int tstep = M >> LS;
  constexpr int MB = (NBMAX * M + NT - 1) / NT;
  const int tid = threadIdx.x;
  const int nb = NB * M;
  cpx<T> v[MB][R];
#pragma unroll
  for (int u = 0; u < MB; ++u) {
    const int j = tid + u * NT;
    if (j < nb) {
      const int b = j >> (LOGN - LR), jj = j & (M - 1);
      const cpx<T>* src = buf + b * ld + jj;
#pragma unroll
      for (int m = 0; m < R; ++m) v[u][m] = src[m * M];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < MB; ++u) {
    const int j = tid + u * NT;
    if (j < nb) {
      const int b = j >> (LOGN - LR), jj = j & (M - 1);
      const int k = jj & (ns - 1);
      if constexpr (LS > 0) {
#pragma unroll
        for (int m = 1; m < R; ++m) v[u][m] = mul(v[u][m], twid<T, INV>(tw, m * k * tstep));
      }
      butterfly<T, R, INV>(v[u]);
      const int o = b * ld + ((jj >> LS) << (LS + LR)) + k;
#pragma unroll
      for (int m = 0; m < R; ++m) buf[o + m * ns] = v[u][m];
    }
  }
  __syncthreads();
}

template <typename T, int LOGN, int NBMAX, bool INV, int R, int LS>
__device__ __forceinline__ void stockham_from(cpx<T>* buf, int ld, int NB, const cpx<T>* __restrict__ tw) {
  if constexpr (LS < LOGN) {
    stockham_stage<T, LOGN, NBMAX, INV, R, LS>(buf, ld, NB, tw);
    stockham_from<T, LOGN, NBMAX, INV, R, LS + ilog2c(R)>(buf, ld, NB, tw);
  }
}

// NB transforms of length N = 2^LOGN held at buf[b * ld + k] (NB <= NBMAX),
// Stockham autosort.  RADIX 4: one radix-2 stage first when LOGN is odd,
// then radix-4 stages; RADIX 8: one radix-2 or radix-4 stage first when
// LOGN mod 3 is 1 or 2, then radix-8 stages.  All index arithmetic is shifts
// and masks.  Called by all NT threads.
template <typename T, int LOGN, int NBMAX, bool INV, int RADIX>
__device__ __forceinline__ void lds_fft(cpx<T>* buf, int ld, int NB, const cpx<T>* __restrict__ tw) {
  if constexpr (RADIX == 4) {
    if constexpr (LOGN & 1) {
      stockham_stage<T, LOGN, NBMAX, INV, 2, 0>(buf, ld, NB, tw);
      stockham_from<T, LOGN, NBMAX, INV, 4, 1>(buf, ld, NB, tw);
    } else {
      stockham_from<T, LOGN, NBMAX, INV, 4, 0>(buf, ld, NB, tw);
    }
  } else {
    static_assert(RADIX == 8, "radix 4 or 8");
    if constexpr (LOGN % 3 == 1) {
      stockham_stage<T, LOGN, NBMAX, INV, 2, 0>(buf, ld, NB, tw);
      stockham_from<T, LOGN, NBMAX, INV, 8, 1>(buf, ld, NB, tw);
    } else if constexpr (LOGN % 3 == 2) {
      stockham_stage<T, LOGN, NBMAX, INV, 4, 0>(buf, ld, NB, tw);
      stockham_from<T, LOGN, NBMAX, INV, 8, 2>(buf, ld, NB, tw);
    } else {
      stockham_from<T, LOGN, NBMAX, INV, 8, 0>(buf, ld, NB, tw);
    }
  }
}

// Sum of v over the block (fixed order: waves by shuffles, then the waves in
// turn); red: NT / 64 doubles of LDS.  Every thread gets the total.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// ------------------------------------------------------------------ bodies
// Each transform is a device body over one block's tile (logical block lb of
// one grid) using the LDS tile buf (and red, NT/64 doubles), shared by the
// single-grid kernels and by the kernels that serve several grids in one
// launch.

// Rows of nx = 2^LOGN reals -> half spectra.  Block = R consecutive rows of
// one plane (R even, R | ny), two rows per complex sequence.  Output
// X[(plane * kxh + k) * ny + y].
// If bsum is not NULL, block lb also writes the float64 sum of its R rows to
// bsum[lb] (the plane means of the mean mode are then formed in float64).
template <typename T, int LOGN, bool NTL, int TILE, int RADIX>
__device__ __forceinline__ void x_r2c_body(cpx<T>* buf, double* red, int lb, const InSegments& seg,
                                           cpx<T>* __restrict__ out, int ny, int R,
                                           const cpx<T>* __restrict__ tw, double* __restrict__ bsum,
                                           const LayerSkip& skip) {
  constexpr int N = 1 << LOGN;
  constexpr int SEQ = r2c_seq<T>(N, TILE);
  constexpr int ld = N + 1;
  constexpr int kxh = N / 2 + 1;
  const size_t row0 = (size_t)lb * R;
  const size_t plane = row0 / ny;
  const int y0 = (int)(row0 - plane * ny);
  // a layer without plastic strain: its rows sum to zero, nothing to transform
  if (skip.zact && (int)plane < skip.nw && (int)(plane % skip.nz) >= *skip.zact) {
    if (bsum && threadIdx.x == 0) bsum[lb] = 0.0;
    return;
  }
  const int sg = (seg.n > 1 && (int)plane >= seg.first[1]) ? 1 : 0;
  const double* in = seg.ptr[sg] + ((plane - seg.first[sg]) * ny + y0) * (size_t)N;
  // 16-byte loads: two consecutive x of one row
  constexpr int MV = (2 * SEQ * N / 2 + NT - 1) / NT;
  const int tot = R * N / 2;
  const double2* src = reinterpret_cast<const double2*>(in);
  double2 v[MV];
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    int i = threadIdx.x + u * NT;
    if (i < tot) v[u] = ld_in<NTL>(src + i);
  }
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    int i = threadIdx.x + u * NT;
    if (i < tot) {
      int r = (2 * i) >> LOGN, x = (2 * i) & (N - 1);
      cpx<T>* d = buf + (r >> 1) * ld + x;
      if (r & 1) { d[0].y = (T)v[u].x; d[1].y = (T)v[u].y; }
      else { d[0].x = (T)v[u].x; d[1].x = (T)v[u].y; }
    }
  }
  if (bsum) {
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < MV; ++u) {
      int i = threadIdx.x + u * NT;
      if (i < tot) acc += v[u].x + v[u].y;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) bsum[lb] = acc;
  }
  __syncthreads();
  lds_fft<T, LOGN, SEQ, false, RADIX>(buf, ld, R / 2, tw);
  const int tot2 = kxh * R;
  for (int i = threadIdx.x; i < tot2; i += NT) {
    int k = i / R, yl = i - k * R;
    int p = yl >> 1;
    cpx<T> Z = buf[p * ld + k];
    cpx<T> Zc = buf[p * ld + ((N - k) & (N - 1))];
    cpx<T> X;
    if ((yl & 1) == 0) X = mk(T(0.5) * (Z.x + Zc.x), T(0.5) * (Z.y - Zc.y));
    else X = mk(T(0.5) * (Z.y + Zc.y), T(0.5) * (Zc.x - Z.x));
    out[(plane * kxh + k) * ny + y0 + yl] = X;
  }
}

// Logical block index such that the blocks dispatched to one XCD (physical
// blocks b, b + 8, b + 16, ...) take consecutive logical indices.
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, n = gridDim.x;
  const int x = b & 7, slot = b >> 3, per = n >> 3, rem = n & 7;
  return x * per + (x < rem ? x : rem) + slot;
}

// Forward column transform: X[p][kx][y] -> S[kx][ky][p]; block = up to B
// planes of one kx (B = tile / ny).  Tile rows past the last plane are filled
// with copies of it (never stored), so every load is unconditional: with
// conditional loads the staging array was not kept in registers and went
// through scratch memory, doubling the kernel's memory traffic.
template <typename T, int LOGN, bool NTL, int TILE, int RADIX>
__device__ __forceinline__ void y_fwd_body(cpx<T>* buf, int lb, const cpx<T>* __restrict__ in,
                                           cpx<T>* __restrict__ out, int kxh, int NP, int ldp,
                                           const cpx<T>* __restrict__ tw, const LayerSkip& skip) {
  constexpr int N = 1 << LOGN;
  constexpr int B = col_batch<T>(N, TILE);
  static_assert((B * N) % NT == 0, "tile must be a multiple of the block");
  constexpr int ld = N + 1;
  const int npb = (NP + B - 1) / B;
  const int kx = lb / npb;
  const int p0 = (lb - kx * npb) * B;
  const int nb = min(B, NP - p0);
  if (skip.zact) {                     // every plane of the group in a layer without plastic strain
    const int za = *skip.zact;
    bool live = false;
    for (int b = 0; b < nb; ++b) {
      const int p = p0 + b;
      live = live || p >= skip.nw || p % skip.nz < za;
    }
    if (!live) return;
  }
  constexpr int MV = B * N / NT;
  cpx<T> v[MV];
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    const int i = threadIdx.x + u * NT;
    const int b = i >> LOGN, y = i & (N - 1);
    const int bc = b < nb ? b : nb - 1;
    v[u] = ld_in<NTL>(in + ((size_t)(p0 + bc) * kxh + kx) * N + y);
  }
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    const int i = threadIdx.x + u * NT;
    buf[(i >> LOGN) * ld + (i & (N - 1))] = v[u];
  }
  __syncthreads();
  lds_fft<T, LOGN, B, false, RADIX>(buf, ld, nb, tw);
  // consecutive lanes take consecutive planes of one ky: runs of nb elements
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    const int i = threadIdx.x + u * NT;
    const int ky = i / B, b = i - ky * B;
    if (b < nb) out[((size_t)kx * N + ky) * ldp + p0 + b] = buf[b * ld + ky];
  }
}

// Inverse column transform: S[kx][ky][p] -> X[p][kx][y].
template <typename T, int LOGN, bool NTL, int TILE, int RADIX>
__device__ __forceinline__ void y_inv_body(cpx<T>* buf, int lb, const cpx<T>* __restrict__ in,
                                           cpx<T>* __restrict__ out, int kxh, int NP, int ldp,
                                           const cpx<T>* __restrict__ tw) {
  constexpr int N = 1 << LOGN;
  constexpr int B = col_batch<T>(N, TILE);
  static_assert((B * N) % NT == 0, "tile must be a multiple of the block");
  constexpr int ld = N + 1;
  const int npb = (NP + B - 1) / B;
  // blocks run plane group by plane group (kx fastest), so the inverse row
  // transform, which runs its blocks from the last plane back, finds the
  // planes written last still in the last-level cache
  const int kx = lb % kxh;
  const int p0 = (lb / kxh) * B;
  const int nb = min(B, NP - p0);
  constexpr int MV = B * N / NT;
  // consecutive lanes read consecutive planes of one ky (runs of nb
  // elements); lanes past the last plane repeat it into unused tile rows
  cpx<T> v[MV];
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    const int i = threadIdx.x + u * NT;
    const int ky = i / B, b = i - ky * B;
    const int bc = b < nb ? b : nb - 1;
    v[u] = ld_in<NTL>(in + ((size_t)kx * N + ky) * ldp + p0 + bc);
  }
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    const int i = threadIdx.x + u * NT;
    const int ky = i / B, b = i - ky * B;
    buf[b * ld + ky] = v[u];
  }
  __syncthreads();
  lds_fft<T, LOGN, B, true, RADIX>(buf, ld, nb, tw);
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    int i = threadIdx.x + u * NT;
    int b = i >> LOGN, y = i & (N - 1);
    if (b < nb) out[((size_t)(p0 + b) * kxh + kx) * N + y] = buf[b * ld + y];
  }
}

// Half spectra -> rows of nx = 2^LOGN reals, two rows per complex transform.
// Plane p of the input goes to the output segment that contains it.
// If padd is not NULL, padd[plane] (float64) is added to every output value
// of that plane (the mean mode computed in float64).  nts: the outputs
// (without the epilogue) are stored as streaming writes.
template <typename T, int LOGN, int TILE, int RADIX>
__device__ __forceinline__ void x_c2r_body(cpx<T>* buf, double* red, int lb, const cpx<T>* __restrict__ in,
                                           const OutSegments& seg, int ny, int R, double scale,
                                           const cpx<T>* __restrict__ tw, const double* __restrict__ padd,
                                           const ResidEpilogue& ep, bool nts) {
  constexpr int N = 1 << LOGN;
  constexpr int SEQ = c2r_seq<T>(N, TILE);
  constexpr int ld = N + 1;
  constexpr int kxh = N / 2 + 1;
  constexpr int nyq = N / 2;
  const int hp = R / 2;                  // a power of two (R = ny or 2 SEQ)
  const int lr = __builtin_ctz(R);
  // one element per lane, consecutive lanes on consecutive rows y of one kx
  // (runs of R elements); slots past the end repeat the last row pair, which
  // writes the same values again.  The rows 2 pr, 2 pr + 1 of a pair sit in
  // lanes 2 j, 2 j + 1 and are exchanged by a DPP lane swap.
  const int totr = kxh * R;
  const bool odd = threadIdx.x & 1;
  const int last = totr - (odd ? 1 : 2);
  constexpr int MV = (kxh * 2 * SEQ + NT - 1) / NT;
  const size_t row0 = (size_t)lb * R;
  const int plane = (int)(row0 / ny);
  const int y0 = (int)(row0 - (size_t)plane * ny);
  cpx<T> v[MV];
  {
    const cpx<T>* src = in + (size_t)plane * kxh * ny + y0;
#pragma unroll
    for (int u = 0; u < MV; ++u) {
      const int i = min((int)threadIdx.x + u * NT, last);
      const int k = i >> lr, y = i & (R - 1);
      v[u] = src[(size_t)k * ny + y];
    }
  }
  {
#pragma unroll
    for (int u = 0; u < MV; ++u) {
      const int i = min((int)threadIdx.x + u * NT, last);
      const int k = i >> lr, pr = (i & (R - 1)) >> 1;
      const cpx<T> o = dpp_move<DPP_SWAP1>(v[u]);
      const cpx<T> X0 = odd ? o : v[u], X1 = odd ? v[u] : o;
      if (k == 0 || k == nyq) {
        if (!odd) buf[pr * ld + k] = mk(X0.x, X1.x);
      } else if (!odd) {
        buf[pr * ld + k] = mk(X0.x - X1.y, X0.y + X1.x);
      } else {
        buf[pr * ld + N - k] = mk(X0.x + X1.y, X1.x - X0.y);
      }
    }
    __syncthreads();
    lds_fft<T, LOGN, SEQ, true, RADIX>(buf, ld, hp, tw);
    int s = 0;
    while (s + 1 < seg.n && plane >= seg.first[s + 1]) ++s;
    double* dst = seg.ptr[s] + ((size_t)(plane - seg.first[s]) * ny + y0) * N;
    const double add = padd ? padd[plane] : 0.0;
    typedef double v2d __attribute__((ext_vector_type(2)));
    if (!ep.x) {
      // Each thread stores one x pair of a row pair: the real parts of the
      // two LDS elements it reads go to row 2 pr, their imaginary parts to
      // row 2 pr + 1.  The operator's outputs are not read again by the
      // operator, so they are stored as streaming (non-temporal) writes,
      // which do not displace the spectrum buffers from the last-level
      // cache; the contact solver's compliance, read at once by the next
      // kernel, keeps ordinary stores.
      const int tot4 = hp * (N / 2);
      for (int i = threadIdx.x; i < tot4; i += NT) {
        const int pr = (2 * i) >> LOGN, x = (2 * i) & (N - 1);
        const cpx<T>* b = buf + pr * ld + x;
        const cpx<T> b0 = b[0], b1 = b[1];
        v2d o0, o1;
        o0.x = (double)b0.x * scale + add;
        o0.y = (double)b1.x * scale + add;
        o1.x = (double)b0.y * scale + add;
        o1.y = (double)b1.y * scale + add;
        v2d* q0 = reinterpret_cast<v2d*>(dst) + (size_t)(2 * pr) * (N / 2) + (x >> 1);
        v2d* q1 = q0 + (N / 2);
        if (nts) {
          __builtin_nontemporal_store(o0, q0);
          __builtin_nontemporal_store(o1, q1);
        } else {
          *q0 = o0;
          *q1 = o1;
        }
      }
    } else {
      // residual epilogue (the residual is the first and only segment)
      const int tot2 = R * N / 2;
      double2* d2 = reinterpret_cast<double2*>(dst);
      const size_t off = ((size_t)plane * ny + y0) * N;
      const double2* x2 = reinterpret_cast<const double2*>(ep.x + off);
      const double2* f2 = ep.Fo ? reinterpret_cast<const double2*>(ep.Fo + off) : nullptr;
      double s0 = 0.0, s1 = 0.0;
      for (int i = threadIdx.x; i < tot2; i += NT) {
        int r = (2 * i) >> LOGN, x = (2 * i) & (N - 1);
        const cpx<T>* b = buf + (r >> 1) * ld + x;
        double2 o;
        if (r & 1) { o.x = (double)b[0].y * scale + add; o.y = (double)b[1].y * scale + add; }
        else { o.x = (double)b[0].x * scale + add; o.y = (double)b[1].x * scale + add; }
        const double2 xv = x2[i];
        const double2 rr = make_double2(xv.x - o.x, xv.y - o.y);
        d2[i] = rr;
        s0 += rr.x * rr.x + rr.y * rr.y;
        if (f2) {
          const double2 f = f2[i];
          s1 += f.x * (rr.x - f.x) + f.y * (rr.y - f.y);
        }
      }
      const double a = block_sum(s0, red);
      const double c = block_sum(s1, red);
      if (threadIdx.x == 0) {
        const int cp = plane / ep.nz, z = plane - cp * ep.nz;
        const double wt = (cp < 3 ? 1.0 : 2.0) * (ep.wz ? ep.wz[z] : ((z == 0 || z == ep.nz - 1) ? 0.5 : 1.0));
        ep.part[2 * lb] = wt * a;
        ep.part[2 * lb + 1] = wt * c;
      }
    }
  }
}

// --------------------------------------------- kernels over several grids
// One launch serves the grids of an XformBatch (transform lengths up to
// 2^XFORM_BATCH_MAX_LOGN, default tile and radix 4): block b belongs to grid
// c with first[c] <= b < first[c + 1] and runs that grid's body with the
// block index b - first[c]; the tile lives in dynamic LDS sized by the host
// for the largest grid.  A grid's results are those of its own launch.
extern __shared__ double2 fvim_dyn_lds[];

__device__ __forceinline__ int batch_grid(const XformBatch& b, int blk) {
  int c = 0;
  while (c + 1 < b.n && blk >= b.first[c + 1]) ++c;
  return c;
}

#define FVIM_BATCH_LOGN_SWITCH(logn, CALL) \
  switch (logn) {                          \
    case 2: CALL(2); break;                \
    case 3: CALL(3); break;                \
    case 4: CALL(4); break;                \
    case 5: CALL(5); break;                \
    case 6: CALL(6); break;                \
    case 7: CALL(7); break;                \
    case 8: CALL(8); break;                \
    case 9: CALL(9); break;                \
  }

// One block of each batched transform (block blk of the launch over the
// table b); the kernels below and the persistent batched operator run them.
template <typename T>
__device__ __forceinline__ void x_r2c_batch_block(const XformBatch& b, int blk, double* red) {
  const int c = batch_grid(b, blk);
  const int lb = blk - b.first[c];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(fvim_dyn_lds);
  cpx<T>* out = static_cast<cpx<T>*>(b.out[c]);
  const cpx<T>* tw = static_cast<const cpx<T>*>(b.tw[c]);
#define CALL(L) x_r2c_body<T, L, false, 1, 4>(buf, red, lb, b.iseg[c], out, b.ny[c], b.R[c], tw, b.bsum[c], LayerSkip{})
  FVIM_BATCH_LOGN_SWITCH(b.logn[c], CALL)
#undef CALL
}

template <typename T>
__device__ __forceinline__ void y_fwd_batch_block(const XformBatch& b, int blk) {
  const int c = batch_grid(b, blk);
  const int lb = blk - b.first[c];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(fvim_dyn_lds);
  const cpx<T>* in = static_cast<const cpx<T>*>(b.in[c]);
  cpx<T>* out = static_cast<cpx<T>*>(b.out[c]);
  const cpx<T>* tw = static_cast<const cpx<T>*>(b.tw[c]);
#define CALL(L) y_fwd_body<T, L, false, 1, 4>(buf, lb, in, out, b.kxh[c], b.NP[c], b.ldp[c], tw, LayerSkip{})
  FVIM_BATCH_LOGN_SWITCH(b.logn[c], CALL)
#undef CALL
}

template <typename T>
__device__ __forceinline__ void y_inv_batch_block(const XformBatch& b, int blk) {
  const int c = batch_grid(b, blk);
  const int lb = blk - b.first[c];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(fvim_dyn_lds);
  const cpx<T>* in = static_cast<const cpx<T>*>(b.in[c]);
  cpx<T>* out = static_cast<cpx<T>*>(b.out[c]);
  const cpx<T>* tw = static_cast<const cpx<T>*>(b.tw[c]);
#define CALL(L) y_inv_body<T, L, false, 1, 4>(buf, lb, in, out, b.kxh[c], b.NP[c], b.ldp[c], tw)
  FVIM_BATCH_LOGN_SWITCH(b.logn[c], CALL)
#undef CALL
}

template <typename T>
__device__ __forceinline__ void x_c2r_batch_block(const XformBatch& b, int blk, double* red) {
  const int c = batch_grid(b, blk);
  const int lb = blk - b.first[c];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(fvim_dyn_lds);
  const cpx<T>* in = static_cast<const cpx<T>*>(b.in[c]);
  const cpx<T>* tw = static_cast<const cpx<T>*>(b.tw[c]);
#define CALL(L) \
  x_c2r_body<T, L, 1, 4>(buf, red, lb, in, b.oseg[c], b.ny[c], b.R[c], 1.0, tw, b.padd[c], ResidEpilogue{}, \
                         b.nts[c] != 0)
  FVIM_BATCH_LOGN_SWITCH(b.logn[c], CALL)
#undef CALL
}

}  // namespace
}  // namespace fvim
